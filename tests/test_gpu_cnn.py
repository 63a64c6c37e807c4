"""GPU parity of the warm-start CNN kernels (forward, gradients, Adam, features, prolongation) with the CPU
FP64 oracle, through the C ABI.

Tolerances: FP32 MFMA operands give errors of FP32 accumulation over K <= 3456 terms per output (normwise
below 1e-5 of the output and of the whole gradient). Per layer the FP32 gradient bound is 1e-3: a ReLU whose
pre-activation lies within FP32 rounding of zero switches, and plain FP32 evaluation of the same network on the
CPU (torch) differs from FP64 by 2.5e-4 in the first layer of the 16^3 case for exactly that reason. BF16 operands round every
activation and weight to 8 mantissa bits, about 0.4 % per rounding; the first layer's gradient ends a chain of
23 such steps (12 forward, 11 data-gradient) and also sees ReLU patterns that flip near zero, so the bounds are
3 % for outputs, 10 % per layer and 5 % for the whole gradient, with its direction within 0.5 % (cosine).
"""
import numpy as np
import pytest
import torch

from oracle import cnn as ocnn

pytestmark = pytest.mark.gpu


def H():
    import paper_2602_07711_amd as H
    return H


def _params(seed):
    rng = np.random.default_rng(seed)
    out = []
    for ci, co, taps, _ in ocnn.LAYERS:
        a = np.sqrt(6.0 / (ci * taps))
        out.append(rng.uniform(-a, a, co * ci * taps))
        out.append(rng.uniform(-0.1, 0.1, co))
    return np.concatenate(out).astype(np.float32)


def _inputs(seed, B, S):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, 2, S ** 3)).astype(np.float32)
    t = rng.standard_normal((B, 2, S ** 3)).astype(np.float32)
    return x, t


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _layer_slices():
    out, off = [], 0
    for ci, co, taps, _ in ocnn.LAYERS:
        out.append(slice(off, off + co * ci * taps))
        off += co * ci * taps
        out.append(slice(off, off + co))
        off += co
    return out


@pytest.mark.parametrize("bf16", [False, True], ids=["fp32", "bf16"])
@pytest.mark.parametrize("S,B", [(8, 1), (16, 2), (24, 3)])
def test_forward_parity(S, B, bf16):
    print(f"cnn forward S={S} B={B} bf16={bf16}", flush=True)
    net = H().Cnn(S, max_batch=B, bf16=bf16, seed=1)
    p = _params(7)
    net.set_params(torch.from_numpy(p))
    assert np.array_equal(net.params().numpy(), p)
    x, _ = _inputs(8, B, S)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = ocnn.forward(p, x)
    err = _rel(y, ref)
    assert err < (3e-2 if bf16 else 1e-5), err
    if not bf16:
        assert np.abs(y - ref).max() < 1e-4 * np.abs(ref).max()
    net.close()


@pytest.mark.parametrize("bf16", [False, True], ids=["fp32", "bf16"])
@pytest.mark.parametrize("S,B", [(8, 2), (16, 2), (24, 1)])
def test_gradient_parity(S, B, bf16):
    print(f"cnn gradient S={S} B={B} bf16={bf16}", flush=True)
    net = H().Cnn(S, max_batch=B, bf16=bf16, seed=2)
    p = _params(9)
    net.set_params(torch.from_numpy(p))
    x, t = _inputs(10, B, S)
    loss = net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = net.grads().numpy()
    ref_loss, ref_g = ocnn.loss_and_grad(p, x, t)
    assert abs(loss - ref_loss) <= (2e-2 if bf16 else 1e-6) * ref_loss
    for sl in _layer_slices():
        err = _rel(g[sl], ref_g[sl])
        assert err < (1e-1 if bf16 else 1e-3), (sl, err)
    assert _rel(g, ref_g) < (5e-2 if bf16 else 1e-4)
    cos = float(np.dot(g, ref_g) / (np.linalg.norm(g) * np.linalg.norm(ref_g)))
    assert cos > (0.995 if bf16 else 1 - 1e-9), cos
    net.close()


def test_full_size_parity_bf16():
    """The training configuration: 64^3 volumes, BF16 operands; forward on a batch of two and the gradient."""
    S, B = 64, 2
    print(f"cnn full size S={S} B={B}", flush=True)
    net = H().Cnn(S, max_batch=B, bf16=True, seed=3)
    p = _params(11)
    net.set_params(torch.from_numpy(p))
    x, t = _inputs(12, B, S)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    y = net.forward(xd).cpu().numpy()
    assert _rel(y, ocnn.forward(p, x)) < 3e-2
    net.loss_grad(xd[:1].contiguous(), td[:1].contiguous())
    g = net.grads().numpy()
    _, ref_g = ocnn.loss_and_grad(p, x[:1], t[:1])
    for sl in _layer_slices():
        assert _rel(g[sl], ref_g[sl]) < 1e-1, sl
    assert _rel(g, ref_g) < 5e-2
    net.close()


def test_adam_matches_closed_form_update():
    S, B = 8, 1
    net = H().Cnn(S, max_batch=B, bf16=False, seed=4)
    p = _params(13)
    net.set_params(torch.from_numpy(p))
    x, t = _inputs(14, B, S)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    w = p.astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for step in (1, 2, 3):
        net.loss_grad(xd, td)
        g = net.grads().numpy().astype(np.float64)
        net.adam_step(1e-3)
        w, m, v = ocnn.adam_step(w, g, m, v, step, 1e-3)
        got = net.params().numpy()
        assert np.abs(got - w).max() < 1e-6, step


def test_training_reduces_loss():
    S, B = 16, 2
    net = H().Cnn(S, max_batch=B, bf16=True, seed=5)
    rng = np.random.default_rng(15)
    x = rng.standard_normal((B, 2, S ** 3)).astype(np.float32)
    t = (0.5 * x[:, ::-1] + 0.1).astype(np.float32)         # a learnable map of the input
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(np.ascontiguousarray(t)).cuda()
    first = net.train_step(xd, td, 1e-3)
    for _ in range(60):
        last = net.train_step(xd, td, 1e-3)
    assert last < 0.5 * first, (first, last)
    net.close()


def test_saved_network_reloads_bitwise(tmp_path):
    """A trained warm-start network written by WarmStart.save and read back by WarmStart.load holds the same
    parameters and predicts the same output, bit for bit (the checkpoint is the parameter vector and the
    scaling metadata; the optimiser state is not part of it)."""
    from paper_2602_07711_amd import warmstart as W
    S, B = 16, 2
    net = H().Cnn(S, max_batch=B, bf16=True, seed=8)
    rng = np.random.default_rng(18)
    x = rng.standard_normal((B, 2, S ** 3)).astype(np.float32)
    t = (0.5 * x[:, ::-1] - 0.2).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(np.ascontiguousarray(t)).cuda()
    for _ in range(5):
        net.train_step(xd, td, 1e-3, want_loss=False)
    ws = W.WarmStart(net, 33.0, 2.5, cubic=False)
    path = str(tmp_path / "ws.npz")
    ws.save(path)
    ws2 = W.WarmStart.load(path, max_batch=B)
    assert (ws2.k0, ws2.t_scale, ws2.cubic, ws2.net.size, ws2.net.bf16) == (33.0, 2.5, False, S, True)
    assert np.array_equal(ws2.net.params().numpy(), net.params().numpy())
    y1 = net.forward(xd).cpu().numpy()
    y2 = ws2.net.forward(xd).cpu().numpy()
    assert np.array_equal(y1, y2)
    net.close()
    ws2.net.close()


@pytest.mark.parametrize("cubic", [False, True], ids=["linear", "cubic"])
@pytest.mark.parametrize("gamma", [0.0, (2 + 0.9j) / (2 - 0.9j)], ids=["zero", "abc"])
@pytest.mark.parametrize("nc,nf", [(8, 8), (8, 17), (16, 33), (13, 41), (64, 128)])
def test_prolong_parity(nc, nf, gamma, cubic):
    net = H().Cnn(8, max_batch=1, bf16=True, seed=6)
    rng = np.random.default_rng(nc * 100 + nf)
    c = rng.standard_normal((2, nc ** 3)).astype(np.float32)
    fine = net.prolong(torch.from_numpy(c).cuda(), nf, scale=0.37, gamma=gamma, cubic=cubic).cpu().numpy()
    ref = (ocnn.prolong_cubic if cubic else ocnn.prolong)(c, nc, nf, scale=0.37, gamma=gamma)
    assert np.abs(fine - ref).max() < 1e-12 * np.abs(ref).max()
    net.close()


@pytest.mark.parametrize("S,nf", [(8, 8), (8, 17), (16, 33), (8, 26), (64, 128), (16, 21)])
def test_features_parity(S, nf):
    net = H().Cnn(S, max_batch=1, bf16=True, seed=7)
    rng = np.random.default_rng(nf)
    P = nf + 4
    k0 = 30.0
    k2 = (k0 * k0 * (1 + 0.3 * rng.random((P, P, P)))).astype(np.float64)
    f = rng.standard_normal((P, P, P)) + 1j * rng.standard_normal((P, P, P))
    x = net.features(torch.from_numpy(k2).cuda(), torch.from_numpy(f).cuda(), k0, c_scale=2.0, f_scale=0.5)
    ref = ocnn.features(k2, f, 2, nf, S, k0, 2.0, 0.5)
    assert np.abs(x.cpu().numpy().reshape(2, -1) - ref).max() < 1e-5
    net.close()


def test_rejects_bad_sizes():
    Hm = H()
    with pytest.raises(Hm.HelmError):
        Hm.Cnn(12, max_batch=1)
    net = Hm.Cnn(16, max_batch=1)
    k2 = torch.zeros(12 ** 3, dtype=torch.float64, device="cuda")      # nf = 8 < 16
    f = torch.zeros(12 ** 3, dtype=torch.complex128, device="cuda")
    with pytest.raises(Hm.HelmError):
        net.features(k2, f, 10.0)
    net.close()
