"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test fails on a plausible mistake in the oracle: a dropped term or wrong coefficient in A or F shows in
the truncation or convergence order, a wrong gamma/zeta/grid placement shows in the paper's printed Table 2
errors, a transposed eigenvector matrix shows in the EigT-vs-sparse-LU check, and so on.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg as spla

import synth
from oracle import krylov as kr
from oracle import operators as op
from oracle import precond as pc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------------------------------- 1D pieces

def test_gamma_satisfies_two_point_closure():
    """U_0 = gamma U_1 solves (U_1 - U_0)/h + i k0 (U_1 + U_0)/2 = 0 (Sec. 2.3); |gamma| = 1 for real k0."""
    for k0, h in ((20.0, 1 / 33), (120.0, 1 / 257), (60.0, 0.01)):
        g = op.gamma_abc(k0, h)
        u1 = 0.7 - 0.2j
        u0 = g * u1
        assert abs((u1 - u0) / h + 1j * k0 * (u1 + u0) / 2) < 1e-12 * abs(u1) / h
        assert abs(abs(g) - 1.0) < 1e-15 and g.imag > 0


def test_dirichlet_eigenpairs_closed_form():
    """gamma = 0: eigenvalues 2 cos(pi h i), orthonormal eigenvectors sqrt(2h) sin(pi h i l) (Sec. 3.1 eq. LMB_egv)."""
    n = 17
    d, V, Vi = pc.eig1d(n, 0.0)
    S = pc.dst_matrix(n)
    lam = 2 * np.cos(np.pi * np.arange(1, n + 1) / (n + 1))
    assert np.allclose(np.sort(d.real), np.sort(lam), atol=1e-13) and abs(d.imag).max() < 1e-13
    # each computed eigenvector is a multiple of one sine vector
    C = np.abs(S.T @ (V / np.linalg.norm(V, axis=0)))
    assert np.allclose(np.sort(C.max(axis=0)), 1.0, atol=1e-12)
    assert np.allclose(S @ S.T, np.eye(n), atol=1e-13)


def test_thomas_matches_dense_solve():
    rng = np.random.default_rng(5)
    nz, ny, nx = 9, 3, 4
    b = rng.standard_normal((ny, nx)) * 0.3 - 2.0 + 1j * rng.uniform(0.05, 0.5, (ny, nx))
    gz = 0.8 + 0.6j
    r = rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))
    u = pc.thomas(b, gz, r)
    for j in range(ny):
        for i in range(nx):
            T = np.diag(np.full(nz, b[j, i])) + np.diag(np.ones(nz - 1), 1) + np.diag(np.ones(nz - 1), -1)
            T[0, 0] += gz
            T[-1, -1] += gz
            assert np.allclose(u[:, j, i], np.linalg.solve(T, r[:, j, i]), rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------------------------------- operator A

@pytest.mark.parametrize("cplx", [False, True], ids=["real_k2", "complex_k2"])
@pytest.mark.parametrize("order", [2, 4, 6])
def test_kron_route_equals_stencil_route(order, cplx):
    rng = np.random.default_rng(order)
    shape = (5, 6, 7)
    h3 = (0.1, 0.1, 0.1) if order == 6 else (0.1, 0.13, 0.07)
    k2h = 30 + 10 * rng.random(tuple(s + 4 for s in shape))
    if cplx:
        k2h = k2h + 1j * (3 + 2 * rng.random(k2h.shape))
    k2i = k2h[2:-2, 2:-2, 2:-2]
    g = (0.3 + 0.8j, 0.5 + 0.2j, -0.4 + 0.9j)
    fields = op.derived_fields(k2h, h3[0]) if order == 6 else None
    A1 = op.A_kron(order, k2i, h3, g, fields)
    A2 = op.A_stencil(order, k2i, h3, g, fields)
    assert abs(A1 - A2).max() <= 1e-14 * abs(A1).max()
    assert np.diff(A1.indptr).max() == {2: 7, 4: 19, 6: 27}[order]


@pytest.mark.parametrize("bc", ["abc", "dirichlet"])
@pytest.mark.parametrize("cplx", [False, True], ids=["real_k2", "complex_k2"])
@pytest.mark.parametrize("order", [2, 4, 6])
def test_sampled_matvec_equals_kron_rows(order, cplx, bc):
    """The row-sampled operator used for full-size checks equals A_kron @ x on every node of a ragged box: every
    face, edge and corner class, a distinct gamma per axis (so a ghost factor taken from the wrong axis shows),
    non-uniform h for orders 2/4 and complex k^2 (Sec. 2.2 eq. scheme4, Sec. 2.3 eq. scheme6 and eq. D_bc)."""
    rng = np.random.default_rng(100 * order + 10 * cplx + (bc == "abc"))
    shape = (14, 13, 9)                                   # (Nz, Ny, Nx)
    h3 = (0.07, 0.07, 0.07) if order == 6 else (0.07, 0.09, 0.05)
    k2h = 40 + 25 * rng.random(tuple(s + 4 for s in shape))
    if cplx:
        k2h = k2h + 1j * (2 + 3 * rng.random(k2h.shape))
    gs = (0.3 + 0.8j, 0.5 + 0.2j, -0.4 + 0.9j) if bc == "abc" else (0.0, 0.0, 0.0)
    fields = op.derived_fields(k2h, h3[0]) if order == 6 else None
    A = op.A_kron(order, k2h[2:-2, 2:-2, 2:-2], h3, gs, fields)
    n = int(np.prod(shape))
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y_ref = A @ x
    nodes = rng.permutation(n)                            # every node, in an arbitrary order
    y = op.sampled_matvec(order, k2h, h3, gs, x, nodes)
    assert np.linalg.norm(y - y_ref[nodes]) <= 1e-14 * np.linalg.norm(y_ref)


@pytest.mark.parametrize("bc", ["abc", "dirichlet"])
def test_sampled_M_equals_matrix_rows(bc):
    """The row-sampled preconditioner operator equals M_matrix @ z on every node of a ragged box, with a distinct
    gamma and h per axis (M = Delta + k0^2 I with the ghost-eliminated closure, Sec. 4)."""
    rng = np.random.default_rng(11 + (bc == "abc"))
    shape = (14, 13, 9)
    h3 = (0.07, 0.09, 0.05)
    k0 = 17.0
    gs = (0.3 + 0.8j, 0.5 + 0.2j, -0.4 + 0.9j) if bc == "abc" else (0.0, 0.0, 0.0)
    M = pc.M_matrix(shape, h3, k0, gs)
    n = int(np.prod(shape))
    z = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y_ref = M @ z
    nodes = rng.permutation(n)
    y = pc.sampled_M(shape, h3, k0, gs, z, nodes)
    assert np.linalg.norm(y - y_ref[nodes]) <= 1e-14 * np.linalg.norm(y_ref)


def test_problem_keeps_complex_k2():
    """Second order, A = Delta_h + diag(k^2): adding i k_i to k^2 must add exactly i diag(k_i) to the assembled
    matrix (and leave F = f unchanged)."""
    rng = np.random.default_rng(4)
    n, h, k0 = 6, 1.0 / 7, 9.0
    kr_ = 60 + 20 * rng.random((n + 4,) * 3)
    ki = 3 + rng.random((n + 4,) * 3)
    f = rng.standard_normal((n + 4,) * 3) + 0j
    A0, F0 = op.problem(2, kr_, f, h, k0)
    A1, F1 = op.problem(2, kr_ + 1j * ki, f, h, k0)
    D = (A1 - A0).toarray()
    assert np.allclose(D, np.diag(1j * ki[2:-2, 2:-2, 2:-2].ravel()), rtol=0, atol=1e-12)
    assert np.array_equal(F0, F1)


def _smooth_case(n, cplx=False):
    """u = exp(i k.x)(1 + 0.3 x y) with k = (2.1, -1.3, 1.7); k^2 = 30 (1 + 0.5 sin 2x cos(3y + z)), plus, for an
    attenuating medium, 6i (1 + 0.5 cos(x + 2y)), on the halo grid."""
    c = synth.halo_coords(n)
    z, y, x = c[:, None, None], c[None, :, None], c[None, None, :]
    kv = np.array([2.1, -1.3, 1.7])
    E = np.exp(1j * (kv[0] * x + kv[1] * y + kv[2] * z))
    u = E * (1 + 0.3 * x * y)
    lapu = E * (-(kv @ kv) * (1 + 0.3 * x * y) + 2j * 0.3 * (kv[0] * y + kv[1] * x))
    k2 = 30.0 * (1 + 0.5 * np.sin(2 * x) * np.cos(3 * y + z))
    if cplx:
        k2 = k2 + 6j * (1 + 0.5 * np.cos(x + 2 * y)) + 0 * z
    return u, k2, lapu + k2 * u


def _truncation(order, n, cplx=False):
    h = 1.0 / (n + 1)
    u, k2, f = _smooth_case(n, cplx)
    fields = op.derived_fields(k2, h) if order == 6 else None
    coefs = op.stencil_coefficients(order, (h, h, h), k2[1:-1, 1:-1, 1:-1], fields)
    Au = op.apply_unfolded(coefs, u[1:-1, 1:-1, 1:-1])
    F = op.rhs(order, f, (h, h, h), k2[2:-2, 2:-2, 2:-2], fields)
    return np.abs(Au - F).max()


@pytest.mark.parametrize("cplx", [False, True], ids=["real_k2", "complex_k2"])
@pytest.mark.parametrize("order,slope", [(2, 1.85), (4, 3.75), (6, 5.6)])
def test_truncation_order(order, slope, cplx):
    """Local truncation error of A u - F on smooth u and variable k^2 falls as h^order (Sec. 2.2, 2.3); with a
    complex k^2 too (a dropped imaginary part of any k^2 term would leave an O(1) error)."""
    e1, e2 = _truncation(order, 16, cplx), _truncation(order, 32, cplx)
    assert np.log2(e1 / e2) > slope


def _exact_ghost_error(order, n):
    """Global error with exact ghost data: A_D U = F - (ghost terms), A_D the gamma = 0 fold."""
    h = 1.0 / (n + 1)
    u, k2, f = _smooth_case(n)
    fields = op.derived_fields(k2, h) if order == 6 else None
    k2i = k2[2:-2, 2:-2, 2:-2]
    A_D = op.A_stencil(order, k2i, (h, h, h), (0.0, 0.0, 0.0), fields)
    coefs = op.stencil_coefficients(order, (h, h, h), k2[1:-1, 1:-1, 1:-1], fields)
    ghost = u[1:-1, 1:-1, 1:-1].copy()
    ghost[1:-1, 1:-1, 1:-1] = 0.0
    F = op.rhs(order, f, (h, h, h), k2i, fields) - op.apply_unfolded(coefs, ghost)
    U = spla.splu(A_D.tocsc()).solve(F.ravel())
    ui = u[2:-2, 2:-2, 2:-2].ravel()
    return np.linalg.norm(U - ui) / np.linalg.norm(ui)


@pytest.mark.parametrize("order,slope", [(4, 3.6), (6, 5.5)])
def test_global_order_with_exact_ghosts(order, slope):
    e1, e2 = _exact_ghost_error(order, 8), _exact_ghost_error(order, 16)
    assert np.log2(e1 / e2) > slope


def test_derived_fields_fourth_order():
    def err(n):
        h = 1.0 / (n + 1)
        c = synth.halo_coords(n)
        z, y, x = c[:, None, None], c[None, :, None], c[None, None, :]
        k2 = np.sin(2 * x) * np.cos(3 * y + z) + x * x * y
        kx, ky, kz, lap = op.derived_fields(k2, h)
        I = (slice(2, -2),) * 3
        ex = (2 * np.cos(2 * x) * np.cos(3 * y + z) + 2 * x * y)[I]
        ez = (-np.sin(2 * x) * np.sin(3 * y + z) + 0 * y)[I]
        el = (-4 * np.sin(2 * x) * np.cos(3 * y + z) - 10 * np.sin(2 * x) * np.cos(3 * y + z) + 2 * y)[I]
        return max(abs(kx - ex).max(), abs(kz - ez).max(), abs(lap - el).max())
    assert np.log2(err(16) / err(32)) > 3.7


def test_abc_manufactured_solution_second_order():
    """With the first-order two-point absorbing closure the global error is O(h^2) whatever the interior order
    (Sec. 6): phi(x)phi(y)phi(z) of Sec. 5.1 with a, b on the boundary planes solves the continuous problem."""
    def err(order, n):
        k0 = 6.0
        h = 1.0 / n
        xs = (np.arange(-2, n + 2) + 0.5) * h   # staggered nodes, boundary at 0 and 1
        z, y, x = xs[:, None, None], xs[None, :, None], xs[None, None, :]
        ph = lambda t: np.exp(1j * k0 * t) + np.exp(-1j * k0 * (t - 1)) - 2
        p2 = lambda t: -k0 * k0 * (np.exp(1j * k0 * t) + np.exp(-1j * k0 * (t - 1)))
        u = ph(x) * ph(y) * ph(z)
        f = p2(x) * ph(y) * ph(z) + ph(x) * p2(y) * ph(z) + ph(x) * ph(y) * p2(z) + k0 * k0 * u
        k2 = np.full(u.shape, k0 * k0)
        A, F = op.problem(order, k2, f, h, k0)
        U = spla.splu(A.tocsc()).solve(F)
        ui = u[2:-2, 2:-2, 2:-2].ravel()
        return np.linalg.norm(U - ui) / np.linalg.norm(ui)
    for order in (4, 6):
        assert 1.7 < np.log2(err(order, 8) / err(order, 16)) < 2.6


# ------------------------------------------------------------------------------------------- the paper's Table 2

def _test_problem_direct(n):
    k0 = np.sqrt(439.2)
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    X, Y, Z = x[None, None, :], x[None, :, None], x[:, None, None]
    ph = lambda t: np.exp(1j * k0 * t) + np.exp(-1j * k0 * (t - 1.0)) - 2
    p2 = lambda t: -k0 * k0 * (np.exp(1j * k0 * t) + np.exp(-1j * k0 * (t - 1.0)))
    u = ph(X) * ph(Y) * ph(Z)
    f = p2(X) * ph(Y) * ph(Z) + ph(X) * p2(Y) * ph(Z) + ph(X) * ph(Y) * p2(Z) + k0 * k0 * u
    g = op.gamma_abc(k0, h)
    U = pc.EigT((n, n, n), (h, h, h), k0, (g, g, g)).solve(f.ravel()).reshape(u.shape)
    return np.abs(U - u).max(), np.linalg.norm(U - u) / np.linalg.norm(u)


def test_paper_table2_direct_second_order_errors():
    """EigT2 as a direct solver of the 2nd-order system reproduces the errors printed in Table 2."""
    with open(os.path.join(GOLDEN, "table2_direct_2nd_order.json")) as fh:
        g = json.load(fh)
    for n, mx_p, l2_p in g["rows"]:
        mx, l2 = _test_problem_direct(n)
        assert abs(mx - mx_p) <= 0.006 * mx_p, (n, mx, mx_p)          # printed to 3 digits
        assert abs(l2 - l2_p) <= 0.05 * l2_p, (n, l2, l2_p)           # printed to 2 digits


def test_paper_table6_scattering_iterations_100():
    """The single-inclusion scattering problem of Sec. 5.1 (complex k^2 in a sphere, staggered 100^3 grid,
    sixth order): GMRES(50) with the EigT preconditioner reaches rel-res 1e-8 in the number of iterations that
    Table 6 prints for EigT2 (12)."""
    with open(os.path.join(GOLDEN, "table6_scattering.json")) as fh:
        row = {r[0]: r for r in json.load(fh)["rows"]}[100]
    n = 100
    w = synth.single_inclusion_problem(n)
    A, F = op.problem(6, w["k2"], w["f"], w["h"], w["k0"])
    g = op.gamma_abc(w["k0"], w["h"])
    e = pc.EigT((n, n, n), (w["h"],) * 3, w["k0"], (g, g, g))
    x, info = kr.gmres(lambda v: A @ v, e.solve, F, m=50, rtol=1e-8)
    assert np.linalg.norm(F - A @ x) <= 1.0001e-8 * np.linalg.norm(F)
    assert info["iters"] == row[2]


# ------------------------------------------------------------------------------------------- preconditioners

def _prec_case(n=10, k0=20.0):
    h = 1.0 / (n + 1)
    g = op.gamma_abc(k0, h)
    shape = (n, n + 1, n + 2)
    h3 = (h, h, h)
    rng = np.random.default_rng(7)
    y = rng.standard_normal(np.prod(shape)) + 1j * rng.standard_normal(np.prod(shape))
    return shape, h3, k0, (g, g, g), y


def test_eigt_inverts_M():
    shape, h3, k0, gs, y = _prec_case()
    M = pc.M_matrix(shape, h3, k0, gs)
    z = pc.EigT(shape, h3, k0, gs).solve(y)
    assert np.linalg.norm(M @ z - y) <= 1e-12 * np.linalg.norm(y)
    zs = spla.splu(M.tocsc()).solve(y)
    assert np.linalg.norm(z - zs) <= 1e-12 * np.linalg.norm(zs)


def test_eigt_non_uniform_h():
    n = 8
    shape, h3 = (n, n, n), (0.1, 0.08, 0.12)
    gs = tuple(op.gamma_abc(15.0, h) for h in h3)
    rng = np.random.default_rng(3)
    y = rng.standard_normal(n ** 3) + 0j
    M = pc.M_matrix(shape, h3, 15.0, gs)
    z = pc.EigT(shape, h3, 15.0, gs).solve(y)
    assert np.linalg.norm(M @ z - y) <= 1e-12 * np.linalg.norm(y)


def test_pfft_equals_eigt_and_sparse_transforms():
    shape, h3, k0, gs, y = _prec_case()
    e = pc.EigT(shape, h3, k0, gs)
    z = e.solve(y)
    zp = pc.PFFT(shape, h3, k0, gs).solve(y)
    assert np.linalg.norm(zp - z) <= 1e-11 * np.linalg.norm(z)
    rng = np.random.default_rng(9)
    ring = np.zeros(shape, bool)
    ring[:, :, [0, -1]] = True
    ring[:, [0, -1], :] = True
    Yr = np.where(ring, rng.standard_normal(shape), 0.0).astype(complex)
    assert abs(pc.sparse_forward(e, Yr) - e.forward(Yr)).max() < 1e-13
    Wb = rng.standard_normal(shape) + 0j
    assert abs(pc.restricted_inverse(e, Wb) - np.where(ring, e.inverse(Wb), 0)).max() < 1e-13


def test_dirichlet_eigt_is_the_sine_solver():
    """gamma = 0 in x and y turns EigT into the sine-transform solver of A_p^F (Sec. 4.2)."""
    shape, h3, k0, gs, y = _prec_case()
    gz = gs[2]
    e = pc.EigT(shape, h3, k0, (0.0, 0.0, gz))
    p = pc.PFFT(shape, h3, k0, (0.0, 0.0, gz))
    ys = h3[2] ** 2 * y.reshape(shape)
    assert np.linalg.norm(e.solve(y) - p.solve_F(ys).ravel()) <= 1e-12 * np.linalg.norm(y)


def test_eigt_with_dirichlet_closures_inverts_fft2_matrix():
    shape, h3, k0, _, y = _prec_case()
    z = pc.EigT(shape, h3, k0, (0.0, 0.0, 0.0)).solve(y)
    zs = spla.splu(pc.M_dirichlet(shape, h3, k0).tocsc()).solve(y)
    assert np.linalg.norm(z - zs) <= 1e-11 * np.linalg.norm(zs)


@pytest.mark.parametrize("order", [4, 6])
def test_fft46_matrix_sine_modes_closed_form(order):
    """FFT4 / FFT6's matrices (compact scheme, constant k0, gamma = 0) have the product sine modes as eigenvectors;
    with t_a = (2 cos(pi p_a h_a) - 2)/h_a^2 the eigenvalue is the scheme's symbol:
      order 4: sum t_a + sum_{a<b} (h_a^2 + h_b^2)/12 t_a t_b + k0^2 (1 + sum h_a^2/12 t_a);
      order 6: (1 + h^2 k0^2/30) sum t_a + h^4/30 t_x t_y t_z + k0^2 + h^2/6 (1 + h^2 k0^2/15) sum_{a<b} t_a t_b
               - h^2 k0^4/20."""
    nz, ny, nx = (5, 7, 6) if order == 4 else (6, 6, 6)
    h3 = (1.0 / (nx + 1), 1.0 / (ny + 1), 1.0 / (nz + 1))
    k0 = 9.0
    M = pc.M_dirichlet_compact((nz, ny, nx), h3, k0, order)
    x = np.arange(1, nx + 1) * h3[0]
    y = np.arange(1, ny + 1) * h3[1]
    z = np.arange(1, nz + 1) * h3[2]
    for p, q, r in [(1, 1, 1), (6, 2, 3), (3, 5, 5), (2, 6, 1)]:
        u = (np.sin(np.pi * r * z)[:, None, None] * np.sin(np.pi * q * y)[None, :, None]
             * np.sin(np.pi * p * x)[None, None, :]).ravel()
        t = [(2 * np.cos(np.pi * m * hh) - 2) / hh ** 2 for m, hh in zip((p, q, r), h3)]
        pairs = [(0, 1), (0, 2), (1, 2)]
        if order == 4:
            lam = (sum(t) + sum((h3[a] ** 2 + h3[b] ** 2) / 12 * t[a] * t[b] for a, b in pairs)
                   + k0 ** 2 * (1 + sum(h3[a] ** 2 / 12 * t[a] for a in range(3))))
        else:
            h2, k2 = h3[0] ** 2, k0 ** 2
            lam = ((1 + h2 * k2 / 30) * sum(t) + h2 * h2 / 30 * t[0] * t[1] * t[2] + k2
                   + h2 / 6 * (1 + h2 * k2 / 15) * sum(t[a] * t[b] for a, b in pairs) - h2 * k2 * k2 / 20)
        assert np.linalg.norm(M @ u - lam * u) <= 1e-12 * abs(lam) * np.linalg.norm(u)


def test_fft2_matrix_sine_modes_closed_form():
    """FFT2's matrix (gamma = 0 on every axis) has the product sine modes sin(pi p x) sin(pi q y) sin(pi r z) as
    eigenvectors with eigenvalue sum_a (2 cos(pi p_a h_a) - 2) / h_a^2 + k0^2 (h_a = 1/(N_a + 1)); checked for
    several modes on a box with three different N, and against the absorbing M (which differs on the faces)."""
    nz, ny, nx = 5, 7, 6
    h3 = (1.0 / (nx + 1), 1.0 / (ny + 1), 1.0 / (nz + 1))
    k0 = 9.0
    M = pc.M_dirichlet((nz, ny, nx), h3, k0)
    x = np.arange(1, nx + 1) * h3[0]
    y = np.arange(1, ny + 1) * h3[1]
    z = np.arange(1, nz + 1) * h3[2]
    for p, q, r in [(1, 1, 1), (6, 2, 3), (3, 7, 5), (2, 5, 1)]:
        u = (np.sin(np.pi * r * z)[:, None, None] * np.sin(np.pi * q * y)[None, :, None]
             * np.sin(np.pi * p * x)[None, None, :]).ravel()
        lam = sum((2 * np.cos(np.pi * m * hh) - 2) / hh ** 2 for m, hh in zip((p, q, r), h3)) + k0 * k0
        assert np.linalg.norm(M @ u - lam * u) <= 1e-12 * abs(lam) * np.linalg.norm(u)
    g = tuple(op.gamma_abc(k0, hh) for hh in h3)
    D = (pc.M_matrix((nz, ny, nx), h3, k0, g) - M).tocoo()
    face = lambda k: np.unravel_index(k, (nz, ny, nx))
    for r_, c_ in zip(D.row, D.col):
        assert r_ == c_
        l, j, i = face(r_)
        assert l in (0, nz - 1) or j in (0, ny - 1) or i in (0, nx - 1)


def test_eigt_collocated_zeta2_inverts_its_matrix():
    """EigT with zeta = 2 (the collocated three-point closure, gamma = 2 i k0 h) equals the sparse LU solve of the
    collocated second-order matrix, on a box with three different N and h."""
    shape = (9, 11, 13)
    h3 = (1.0 / 12, 1.0 / 10, 1.0 / 8)
    k0 = 7.0
    gs = tuple(2j * k0 * hh for hh in h3)
    rng = np.random.default_rng(12)
    y = rng.standard_normal(np.prod(shape)) + 1j * rng.standard_normal(np.prod(shape))
    M = pc.M_collocated(shape, h3, k0, gs)
    z = pc.EigT(shape, h3, k0, gs, zeta=2.0).solve(y)
    zs = spla.splu(M.tocsc()).solve(y)
    assert np.linalg.norm(z - zs) <= 1e-11 * np.linalg.norm(zs)
    assert np.linalg.norm(M @ z - y) <= 1e-11 * np.linalg.norm(y)


def test_pfft_collocated_zeta2_equals_eigt_and_inverts_its_matrix():
    """PFFT with zeta = 2: the correction E = A_p^F - A_p reaches two layers per face, and the result must still be
    the exact solve: equal to EigT(zeta = 2) and to the sparse LU of the collocated matrix (odd and even axes)."""
    for shape in [(9, 11, 13), (8, 6, 10)]:
        h3 = (1.0 / (shape[2] - 1), 1.0 / (shape[1] - 1), 1.0 / (shape[0] - 1))
        k0 = 7.0
        gs = tuple(2j * k0 * hh for hh in h3)
        rng = np.random.default_rng(13)
        y = rng.standard_normal(np.prod(shape)) + 1j * rng.standard_normal(np.prod(shape))
        zp = pc.PFFT(shape, h3, k0, gs, zeta=2.0).solve(y)
        ze = pc.EigT(shape, h3, k0, gs, zeta=2.0).solve(y)
        M = pc.M_collocated(shape, h3, k0, gs)
        assert np.linalg.norm(zp - ze) <= 1e-11 * np.linalg.norm(ze)
        assert np.linalg.norm(M @ zp - y) <= 1e-11 * np.linalg.norm(y)
        # one layer per face (dropping the zeta - 1 term's inner layer) is not the solve: the pin sees the second layer
        p1 = pc.PFFT(shape, h3, k0, gs, zeta=2.0)
        Ys = p1.hz2 * y.reshape(shape)
        theta = p1.solve_F(Ys)
        W = p1.eig.inverse(pc.thomas(p1.eig.bbar, p1.gz, p1.eig.forward(p1.E_apply(theta)), 2.0))
        ring = np.zeros(shape, bool)
        ring[:, :, [0, -1]] = True
        ring[:, [0, -1], :] = True
        bad = p1.solve_F(Ys + p1.E_apply(theta + np.where(ring, W, 0.0))).ravel()
        assert np.linalg.norm(bad - ze) > 1e-3 * np.linalg.norm(ze)


def _collocated_test_error(n):
    """The Sec. 5.1 test problem on the collocated grid x_j = j h, j = 0..N-1, h = 1/(N-1) (boundary nodes are
    unknowns): the second-order system with the three-point closure solved by EigT(zeta = 2)."""
    k0 = np.sqrt(439.2)
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    X, Y, Z = x[None, None, :], x[None, :, None], x[:, None, None]
    ph = lambda t: np.exp(1j * k0 * t) + np.exp(-1j * k0 * (t - 1.0)) - 2
    p2 = lambda t: -k0 * k0 * (np.exp(1j * k0 * t) + np.exp(-1j * k0 * (t - 1.0)))
    u = ph(X) * ph(Y) * ph(Z)
    f = p2(X) * ph(Y) * ph(Z) + ph(X) * p2(Y) * ph(Z) + ph(X) * ph(Y) * p2(Z) + k0 * k0 * u
    g = 2j * k0 * h
    U = pc.EigT((n, n, n), (h, h, h), k0, (g, g, g), zeta=2.0).solve(f.ravel()).reshape(u.shape)
    return np.linalg.norm(U - u) / np.linalg.norm(u)


def test_collocated_closure_second_order():
    """The three-point closure (central difference of u_n + i k0 u = 0 at the boundary node) makes the collocated
    second-order solution converge at O(h^2) to the analytic test solution, which satisfies that condition."""
    e1, e2 = _collocated_test_error(33), _collocated_test_error(65)
    assert 1.8 < np.log2(e1 / e2) < 2.3


# ------------------------------------------------------------------------------------------- GMRES

def _small_problem(order=6, n=14, k0=None):
    k0 = k0 or 0.47 * (n + 1)
    h = 1.0 / (n + 1)
    k2 = synth.inclusions_k2(n, k0)
    f = synth.gaussian_source(n)
    A, F = op.problem(order, k2, f, h, k0)
    g = op.gamma_abc(k0, h)
    e = pc.EigT((n, n, n), (h, h, h), k0, (g, g, g))
    return A, F, e


@pytest.mark.parametrize("order", [4, 6])
def test_gmres_matches_sparse_lu(order):
    A, F, e = _small_problem(order)
    xs = spla.splu(A.tocsc()).solve(F)
    for flexible, m in ((False, 50), (True, 50), (False, 4)):
        x, info = kr.gmres(lambda v: A @ v, e.solve, F, m=m, rtol=1e-10, flexible=flexible)
        assert info["converged"]
        assert np.linalg.norm(F - A @ x) <= 1e-10 * np.linalg.norm(F) * 1.0001
        assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
        h = np.array(info["hist"])
        if m == 50:
            assert np.all(np.diff(h) <= 1e-12)      # residual is monotone within one cycle
            assert info["iters"] <= 15


def test_gmres_second_order_constant_k_one_iteration():
    """order 2 with k^2 = k0^2 makes A equal to M, so preconditioned GMRES converges in one step."""
    n, k0 = 12, 6.0
    h = 1.0 / (n + 1)
    A, F = op.problem(2, np.full((n + 4,) * 3, k0 * k0), synth.gaussian_source(n), h, k0)
    g = op.gamma_abc(k0, h)
    e = pc.EigT((n, n, n), (h, h, h), k0, (g, g, g))
    x, info = kr.gmres(lambda v: A @ v, e.solve, F, m=10, rtol=1e-12)
    assert info["iters"] == 1 and info["relres"] < 1e-12


def test_gmres_zero_rhs_and_iteration_cap():
    A, F, e = _small_problem(6, n=8, k0=4.0)
    x, info = kr.gmres(lambda v: A @ v, e.solve, 0 * F, m=10)
    assert info["iters"] == 0 and not np.any(x)
    x, info = kr.gmres(lambda v: A @ v, e.solve, F, m=10, rtol=1e-14, maxit=2)
    assert info["iters"] == 2 and not info["converged"]


def test_constant_k_spectrum_clusters_near_one():
    """Constant k: A6 and M share the eigenvectors V_z (x) V_y (x) V_x, and the eigenvalues of A M^{-1}
    stay in a bounded cluster around 1 (1 + O((k h)^2) for the smooth modes, the 3D analogue of Sec. 3.1
    eq. 1DEGV; the highest-frequency modes differ by O(1) between the compact and 7-point symbols)."""
    n, k0 = 6, 3.0
    h = 1.0 / (n + 1)
    A, _ = op.problem(6, np.full((n + 4,) * 3, k0 * k0), synth.gaussian_source(n), h, k0)
    g = op.gamma_abc(k0, h)
    M = pc.M_matrix((n, n, n), (h, h, h), k0, (g, g, g))
    lam = scipy.linalg.eigvals(A.toarray() @ np.linalg.inv(M.toarray()))
    assert abs(lam - 1).max() < 0.6 and abs(lam - 1).min() < 0.05 and lam.real.min() > 0.4
    _, V, Vi = pc.eig1d(n, g)
    W = np.kron(V, np.kron(V, V))
    D = np.kron(Vi, np.kron(Vi, Vi)) @ A.toarray() @ W
    assert abs(D - np.diag(np.diag(D))).max() < 1e-9 * abs(D).max()
