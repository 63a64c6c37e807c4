"""Pins of the CNN oracle (no GPU) against what the definition and the mathematics fix.

A transposed tap order or a wrong padding fails the brute-force convolution; a swapped concatenation order, a
wrong pooling or upsampling, or a misplaced layer fails the independent numpy evaluation of the whole network;
a wrong gradient fails the finite-difference check; a wrong Adam moment or bias correction fails its closed
form; a shifted prolongation grid fails exactness on trilinear functions.
"""
import numpy as np
import pytest
import torch

from oracle import cnn


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    out = []
    for ci, co, taps, _ in cnn.LAYERS:
        a = np.sqrt(6.0 / (ci * taps)) * scale
        out.append(rng.uniform(-a, a, co * ci * taps))
        out.append(rng.uniform(-0.1, 0.1, co))
    return np.concatenate(out)


def test_param_count_matches_layer_table():
    assert cnn.num_params() == sum(co * ci * t + co for ci, co, t, _ in cnn.LAYERS)
    # by hand: 880 + 6928 + 13856 + 27680 + 55360 + 3 * 110656 + 221248 + 82976 + 20752 + 34
    assert cnn.num_params() == 761682


def test_conv_matches_bruteforce_loops():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 4, 4))
    W = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    ref = cnn.conv3d_bruteforce(x, W, b)
    got = torch.nn.functional.conv3d(torch.as_tensor(x)[None], torch.as_tensor(W), torch.as_tensor(b), padding=1)[0]
    assert np.abs(got.numpy() - ref).max() < 1e-12


def _np_conv(x, W, b, relu):
    """Zero-padded cross-correlation by shifted slices (independent of torch's conv3d)."""
    co, ci, k = W.shape[0], W.shape[1], W.shape[-1]
    S = x.shape[1]
    r = k // 2
    xp = np.pad(x, ((0, 0), (r, r), (r, r), (r, r)))
    y = np.zeros((co, S, S, S)) + b[:, None, None, None]
    for dz in range(k):
        for dy in range(k):
            for dx in range(k):
                sh = xp[:, dz:dz + S, dy:dy + S, dx:dx + S]
                y += np.tensordot(W[:, :, dz, dy, dx], sh, axes=(1, 0))
    return np.maximum(y, 0) if relu else y


def _np_network(params, x):
    layers, off = [], 0
    for ci, co, taps, relu in cnn.LAYERS:
        k = 3 if taps == 27 else 1
        W = params[off:off + co * ci * taps].reshape(co, ci, k, k, k)
        off += co * ci * taps
        layers.append((W, params[off:off + co], relu))
        off += co
    c = lambda i, t: _np_conv(t, *layers[i])
    pool = lambda t: t.reshape(t.shape[0], t.shape[1] // 2, 2, t.shape[2] // 2, 2, t.shape[3] // 2, 2).mean(axis=(2, 4, 6))
    up = lambda t: t.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)
    s1 = c(1, c(0, x))
    s2 = c(3, c(2, pool(s1)))
    s3 = c(5, c(4, pool(s2)))
    bt = c(7, c(6, pool(s3)))
    d3 = c(8, np.concatenate([up(bt), s3]))
    d2 = c(9, np.concatenate([up(d3), s2]))
    d1 = c(10, np.concatenate([up(d2), s1]))
    return c(11, d1)


def test_network_matches_independent_numpy_evaluation():
    S = 8
    p = _params(2)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 2, S ** 3))
    ref = _np_network(p, x[0].reshape(2, S, S, S)).reshape(1, 2, -1)
    got = cnn.forward(p, x)
    assert np.abs(got - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())


def test_gradient_matches_finite_differences():
    S = 8
    p = _params(4)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, 2, S ** 3))
    t = rng.standard_normal((2, 2, S ** 3))
    loss, g = cnn.loss_and_grad(p, x, t)
    ref_loss = np.mean((cnn.forward(p, x) - t) ** 2)
    assert abs(loss - ref_loss) < 1e-12 * ref_loss
    # a few entries of every layer (weights and biases), central differences
    idx, off = [], 0
    for ci, co, taps, _ in cnn.LAYERS:
        nw = co * ci * taps
        idx += list(rng.integers(off, off + nw, 2)) + [off + nw + int(rng.integers(0, co))]
        off += nw + co
    eps = 1e-7     # small enough that no ReLU kink is crossed, large against FP64 round-off of an O(1) loss
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (np.mean((cnn.forward(pp, x) - t) ** 2) - np.mean((cnn.forward(pm, x) - t) ** 2)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g).max()), (i, fd, g[i])


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments equal g and g^2, so every step moves by lr g/(|g|+eps)."""
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    lr = 1e-2
    for step in range(1, 6):
        w_new, m, v = cnn.adam_step(w, g, m, v, step, lr)
        assert np.allclose(w - w_new, lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        w = w_new


@pytest.mark.parametrize("nc,nf", [(8, 8), (8, 17), (16, 33)])
def test_prolong_exact_for_trilinear_fields(nc, nf):
    def f(z, y, x):
        return (0.3 + 2 * x) * (1 - 0.5 * y) * (0.7 + z) + 1j * (1 + x) * (2 - y) * (0.5 + 0.2 * z)
    pc = (np.arange(nc) + 1) / (nc + 1)
    Z, Y, X = np.meshgrid(pc, pc, pc, indexing="ij")
    u = f(Z, Y, X)
    coarse = np.stack([u.real, u.imag]).reshape(2, -1)
    got = cnn.prolong(coarse, nc, nf, scale=2.0).reshape(nf, nf, nf)
    pf = (np.arange(nf) + 1) / (nf + 1)
    inside = (pf >= pc[0] - 1e-14) & (pf <= pc[-1] + 1e-14)
    Zf, Yf, Xf = np.meshgrid(pf[inside], pf[inside], pf[inside], indexing="ij")
    assert np.abs(got[np.ix_(inside, inside, inside)] - 2.0 * f(Zf, Yf, Xf)).max() < 1e-12
    if nf == nc:
        assert np.abs(got - 2.0 * u).max() < 1e-13
    else:   # nodes outside the coarse range interpolate toward zero
        assert abs(got[0, 0, 0]) < abs(2.0 * u[0, 0, 0])


@pytest.mark.parametrize("S,nf", [(8, 17), (8, 26), (16, 16)])
def test_features_inject_on_nested_grids(S, nf):
    """When nf+1 = r (S+1) the network node i is solver node r(i+1)-1: plain injection."""
    rng = np.random.default_rng(nf)
    P = nf + 4
    k2 = 900.0 * (1 + 0.3 * rng.random((P, P, P)))
    f = rng.standard_normal((P, P, P)) + 1j * rng.standard_normal((P, P, P))
    x = cnn.features(k2, f, 2, nf, S, 30.0, 2.0, 0.5).reshape(2, S, S, S)
    r = (nf + 1) // (S + 1)
    idx = 2 + r * (np.arange(S) + 1) - 1
    sub = np.ix_(idx, idx, idx)
    assert np.abs(x[0] - 2.0 * (k2[sub] / 900.0 - 1)).max() < 1e-12
    assert np.abs(x[1] - 0.5 * f[sub].real).max() < 1e-12


def test_features_exact_for_trilinear_fields():
    S, nf = 16, 40
    P = nf + 4
    t = (np.arange(P) - 1) / (nf + 1)          # coordinates of the halo array's nodes
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    k2 = 900.0 * (1 + 0.1 * (1 + X) * (2 - Y) * (1 + 0.5 * Z))
    f = (0.5 + X) * (1 + 2 * Y) * (3 - Z) + 0j
    x = cnn.features(k2, f, 2, nf, S, 30.0, 1.0, 1.0).reshape(2, S, S, S)
    s = (np.arange(S) + 1) / (S + 1)
    z, y, xx = np.meshgrid(s, s, s, indexing="ij")
    assert np.abs(x[0] - 0.1 * (1 + xx) * (2 - y) * (1 + 0.5 * z)).max() < 1e-12
    assert np.abs(x[1] - (0.5 + xx) * (1 + 2 * y) * (3 - z)).max() < 1e-11


@pytest.mark.parametrize("nc,nf", [(8, 17), (6, 20), (5, 5)])
def test_prolong_ghost_rule_equals_kronecker_of_1d_interpolation(nc, nf):
    """The 3-D prolongation with ghost factor gamma equals P (x) P (x) P applied to the coarse field, where the
    1-D matrix P interpolates linearly between nodes (i+1)/(nc+1) and folds the ghost nodes -1 and nc onto
    their neighbours with weight gamma (Sec. 2.3, eq. D_bc)."""
    gam = (2 + 1j * 60 / (nc + 1)) / (2 - 1j * 60 / (nc + 1))
    P = np.zeros((nf, nc), dtype=complex)
    for I in range(nf):
        x = (I + 1) / (nf + 1) * (nc + 1) - 1          # coarse index coordinate
        i0 = int(np.floor(x))
        w = x - i0
        for i, wt in ((i0, 1 - w), (i0 + 1, w)):
            if i < 0:
                P[I, 0] += wt * gam
            elif i >= nc:
                P[I, nc - 1] += wt * gam
            else:
                P[I, i] += wt
    rng = np.random.default_rng(nc + nf)
    u = rng.standard_normal((nc, nc, nc)) + 1j * rng.standard_normal((nc, nc, nc))
    ref = np.einsum("ai,bj,ck,ijk->abc", P, P, P, u).reshape(-1)
    got = cnn.prolong(np.stack([u.real.reshape(-1), u.imag.reshape(-1)]), nc, nf, scale=1.0, gamma=gam)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("nc,nf", [(10, 21), (9, 30), (7, 7)])
def test_prolong_cubic_reproduces_quadratics_and_identity(nc, nf):
    """Keys' cubic convolution (a = -1/2) reproduces quadratic polynomials wherever its four coarse nodes are
    inside the grid, and is the identity when nf = nc."""
    def f(z, y, x):
        return (1 + x - 2 * x * x) * (0.5 + y * y) * (2 - z + z * z) + 1j * (x * x + y - z)
    pc = (np.arange(nc) + 1) / (nc + 1)
    Z, Y, X = np.meshgrid(pc, pc, pc, indexing="ij")
    u = f(Z, Y, X)
    got = cnn.prolong_cubic(np.stack([u.real.reshape(-1), u.imag.reshape(-1)]), nc, nf, gamma=0.3 + 0.4j)
    got = got.reshape(nf, nf, nf)
    if nf == nc:
        assert np.abs(got - u).max() < 1e-12
        return
    pf = (np.arange(nf) + 1) / (nf + 1)
    inside = (pf >= pc[1]) & (pf <= pc[-2])                 # all four stencil nodes are real nodes
    Zf, Yf, Xf = np.meshgrid(pf[inside], pf[inside], pf[inside], indexing="ij")
    assert np.abs(got[np.ix_(inside, inside, inside)] - f(Zf, Yf, Xf)).max() < 1e-12


def test_prolong_cubic_ghost_folding_in_one_dimension():
    """On a field constant in y and z the ghost factors of those axes appear only near their faces; a fine
    node between the first coarse node and the boundary mixes gamma^2, gamma and the nodes 0, 1."""
    nc, nf, gam = 4, 9, 0.5 - 0.25j
    u = np.zeros((nc, nc, nc), dtype=complex)
    u[1:3, 1:3, :] = np.arange(1, nc + 1)                   # x-profile 1..4 on the inner y, z nodes
    got = cnn.prolong_cubic(np.stack([u.real.reshape(-1), u.imag.reshape(-1)]), nc, nf, gamma=gam).reshape(nf, nf, nf)
    # fine x-node 0: coarse coordinate x = 1*5/10 - 1 = -0.5, i0 = -1, t = 0.5; nodes -2, -1, 0, 1
    t, a = 0.5, -0.5
    w = [a * t ** 3 - 2 * a * t * t + a * t, (a + 2) * t ** 3 - (a + 3) * t * t + 1,
         -(a + 2) * t ** 3 + (2 * a + 3) * t * t - a * t, -a * t ** 3 + a * t * t]
    expect_x = w[0] * gam ** 2 * 1 + w[1] * gam * 1 + w[2] * 1 + w[3] * 2
    # fine y = z = node 4: coarse coordinate 5*5/10 - 1 = 1.5, nodes 0..3 with profile 0,1,1,0
    wy = w                                                   # same t = 0.5
    yz = wy[1] + wy[2]
    assert abs(got[4, 4, 0] - yz * yz * expect_x) < 1e-12
