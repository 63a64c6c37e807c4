"""Oracle: the compact 4th/6th-order Helmholtz operator A, its right-hand side F and the derived k^2 fields.

TEST INFRASTRUCTURE ONLY (see the package docstring). complex128 / float64 throughout.

Arrays are indexed [z, y, x] (x fastest), so a flattened vector has index i + Nx*(j + Ny*l): the slice
ordering of Sec. 4.1 (block-tridiagonal form, eq. VecPre_system).

Two independent routes assemble A:
  * `A_kron`: the matrix form. Every difference operator is the 1D matrix with the ghost nodes eliminated
    by U_0 = gamma U_1, U_{N+1} = gamma U_N (Sec. 2.3, eq. D_bc), lifted by Kronecker products; the scheme
    is then written term by term (Sec. 2.2 eq. scheme4, Sec. 2.3 eq. scheme6).
  * `stencil_coefficients` + `fold_matrix`: the 27 per-offset coefficients of the unfolded stencil,
    collected by neighbour class, and then folded onto in-domain nodes with one factor gamma per clamped
    axis. `apply_unfolded` applies the same coefficients with exact ghost values (used for truncation tests).

Readings of the paper used here (silent or ambiguous passages):
  R1 (grid): nodes x_i = i h, h = 1/(N+1), ghosts at 0 and 1, boundary half a cell outside the first node.
  R2 (eq. scheme6, "(delta^2..)(1 + k^2 h^2/30) U"): the factor multiplies the grid function, i.e.
      Delta (U + h^2/30 K U), and likewise P (U + h^2/15 K U).
  R3 ("nabla^4 f" in eq. scheme6): the sum of pure fourth derivatives f_xxxx + f_yyyy + f_zzzz.
  R4 ("(nabla^2(k^2) - k^4)_{ijl}" in Delta_h(k^2 U)): multiplies U_{ijl}.
  R5 (delta_x(1 + h^2/6(delta_y^2 + delta_z^2 + k^2))U): k^2 acts on the grid function inside delta_x.
  R6 (ghosts): the ghost rule applies to every grid function a difference touches (U, KU, T_y U, ...).
  R7 (derived fields): grad k^2 and lap k^2 at the nodes come from 4th-order central differences of k^2
      sampled on a two-cell halo.
  R8 (RHS): f is data sampled on the halo (no ghost elimination); the continuous derivatives of f in
      eq. scheme4/scheme6 are replaced by central differences accurate enough for the scheme's order.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------------------------------------------
# 1D building blocks
# ----------------------------------------------------------------------------------------------------------

def gamma_abc(k0: float, h: float) -> complex:
    """Ghost factor of the two-point absorbing closure: gamma = (2 + i k0 h)/(2 - i k0 h) (Sec. 2.3, eq. D_bc)."""
    return (2.0 + 1j * k0 * h) / (2.0 - 1j * k0 * h)


def lambda_bar(n: int, gamma: complex, zeta: complex = 1.0) -> sp.csr_matrix:
    """The N x N tridiagonal block Lambda-bar: zero diagonal, unit off-diagonals, corners gamma and zeta
    (Sec. 4.1, eq. lambda_mat_definition)."""
    main = np.zeros(n, np.complex128)
    main[0] += gamma
    main[-1] += gamma
    up = np.ones(n - 1, np.complex128)
    lo = np.ones(n - 1, np.complex128)
    up[0] = zeta
    lo[-1] = zeta
    return sp.diags([lo, main, up], [-1, 0, 1], format="csr")


def d2_1d(n: int, h: float, gamma: complex) -> sp.csr_matrix:
    """delta^2 (Sec. 2.1) with the ghosts eliminated (eq. D_bc): T = (Lambda-bar - 2I)/h^2."""
    return ((lambda_bar(n, gamma) - 2.0 * sp.identity(n, np.complex128, format="csr")) / (h * h)).tocsr()


def d1_1d(n: int, h: float, gamma: complex) -> sp.csr_matrix:
    """delta (Sec. 2.1), (u_{i+1} - u_{i-1})/(2h), with the same ghost rule: row 1 reads (u_2 - gamma u_1)/(2h),
    row N reads (gamma u_N - u_{N-1})/(2h)."""
    main = np.zeros(n, np.complex128)
    main[0] = -gamma
    main[-1] = gamma
    return (sp.diags([-np.ones(n - 1), main, np.ones(n - 1)], [-1, 0, 1], format="csr") / (2.0 * h)).tocsr()


def _lift(shape, op1d, axis):
    """Lift a 1D operator acting along `axis` (0=x, 1=y, 2=z) to the 3D grid of `shape` = (Nz, Ny, Nx)."""
    nz, ny, nx = shape
    ix, iy, iz = (sp.identity(k, np.complex128, format="csr") for k in (nx, ny, nz))
    if axis == 0:
        return sp.kron(iz, sp.kron(iy, op1d)).tocsr()
    if axis == 1:
        return sp.kron(iz, sp.kron(op1d, ix)).tocsr()
    return sp.kron(op1d, sp.kron(iy, ix)).tocsr()


def lifted_ops(shape, h3, gammas):
    """(T_x, T_y, T_z) and (C_x, C_y, C_z) on the 3D grid; h3 = (hx, hy, hz), gammas = (gx, gy, gz)."""
    nz, ny, nx = shape
    ns = (nx, ny, nz)
    T = [_lift(shape, d2_1d(ns[a], h3[a], gammas[a]), a) for a in range(3)]
    C = [_lift(shape, d1_1d(ns[a], h3[a], gammas[a]), a) for a in range(3)]
    return T, C


# ----------------------------------------------------------------------------------------------------------
# Derived fields of k^2 (reading R7) and finite differences on halo-padded arrays
# ----------------------------------------------------------------------------------------------------------

def _interior(a: np.ndarray, halo: int, dz: int = 0, dy: int = 0, dx: int = 0) -> np.ndarray:
    """The interior block of a halo-padded array, shifted by (dz, dy, dx)."""
    nz, ny, nx = (s - 2 * halo for s in a.shape)
    return a[halo + dz:halo + dz + nz, halo + dy:halo + dy + ny, halo + dx:halo + dx + nx]


def _axis_shift(a, halo, axis, s):
    d = [0, 0, 0]
    d[2 - axis] = s  # axis 0 = x is the last array index
    return _interior(a, halo, *d)


def derived_fields(k2_halo: np.ndarray, h: float):
    """grad k^2 and lap k^2 at the interior nodes from 5-point 4th-order central differences (reading R7).

    k2_halo has a two-cell halo. Returns (kx, ky, kz, lap), each of interior shape.
    """
    g = []
    lap = np.zeros_like(_interior(k2_halo, 2))
    for ax in range(3):
        p1, m1 = _axis_shift(k2_halo, 2, ax, 1), _axis_shift(k2_halo, 2, ax, -1)
        p2, m2 = _axis_shift(k2_halo, 2, ax, 2), _axis_shift(k2_halo, 2, ax, -2)
        c = _interior(k2_halo, 2)
        g.append((-p2 + 8.0 * p1 - 8.0 * m1 + m2) / (12.0 * h))
        lap = lap + (-p2 + 16.0 * p1 - 30.0 * c + 16.0 * m1 - m2) / (12.0 * h * h)
    return g[0], g[1], g[2], lap


# ----------------------------------------------------------------------------------------------------------
# Route 1: matrix (Kronecker) form
# ----------------------------------------------------------------------------------------------------------

def A_kron(order: int, k2_int: np.ndarray, h3, gammas, fields=None) -> sp.csr_matrix:
    """The operator A by the matrix form of the scheme.

    order 2: Delta + K (the 7-point second-order operator with variable k^2).
    order 4: Sec. 2.2 eq. scheme4,
        Delta + sum_{nu<mu} (h_nu^2 + h_mu^2)/12 T_nu T_mu + (I + sum_nu h_nu^2/12 T_nu) K.
    order 6: Sec. 2.3 eq. scheme6 with Delta_h(k^2 U) expanded (readings R2-R6), uniform h:
        Delta (I + h^2/30 K) + h^4/30 T_x T_y T_z + K + h^2/6 P (I + h^2/15 K)
        + h^2/20 [ (L - K^2) + 2 sum_nu K_nu C_nu (I + h^2/6 (Delta - T_nu) + h^2/6 K) ],
        P = T_x T_y + T_x T_z + T_y T_z, K_nu = diag(d k^2/d nu), L = diag(lap k^2).
    The k^2 f and f_nu terms of Delta_h(k^2 U) belong to the right-hand side (see `rhs`).
    """
    shape = k2_int.shape
    T, C = lifted_ops(shape, h3, gammas)
    n = k2_int.size
    eye = sp.identity(n, np.complex128, format="csr")
    K = sp.diags(k2_int.ravel().astype(np.complex128), format="csr")
    Lap = T[0] + T[1] + T[2]
    if order == 2:
        return (Lap + K).tocsr()
    if order == 4:
        hx, hy, hz = (float(v) for v in h3)
        A = (Lap + (hx * hx + hy * hy) / 12.0 * (T[0] @ T[1]) + (hx * hx + hz * hz) / 12.0 * (T[0] @ T[2])
             + (hy * hy + hz * hz) / 12.0 * (T[1] @ T[2])
             + (eye + hx * hx / 12.0 * T[0] + hy * hy / 12.0 * T[1] + hz * hz / 12.0 * T[2]) @ K)
        return A.tocsr()
    if order == 6:
        h = float(h3[0])
        assert abs(h3[1] - h) < 1e-15 * h and abs(h3[2] - h) < 1e-15 * h, "6th order needs uniform h"
        kx, ky, kz, lap = fields
        Kn = [sp.diags(f.ravel().astype(np.complex128), format="csr") for f in (kx, ky, kz)]
        L = sp.diags(lap.ravel().astype(np.complex128), format="csr")
        P = T[0] @ T[1] + T[0] @ T[2] + T[1] @ T[2]
        h2 = h * h
        A = (Lap @ (eye + h2 / 30.0 * K) + h2 * h2 / 30.0 * (T[0] @ T[1] @ T[2]) + K
             + h2 / 6.0 * P @ (eye + h2 / 15.0 * K))
        inner = L - K @ K
        for nu in range(3):
            G = eye + h2 / 6.0 * (Lap - T[nu]) + h2 / 6.0 * K
            inner = inner + 2.0 * Kn[nu] @ C[nu] @ G
        A = A + h2 / 20.0 * inner
        return A.tocsr()
    raise ValueError(order)


# ----------------------------------------------------------------------------------------------------------
# Route 2: per-offset stencil coefficients (unfolded), folding, and the exact-ghost apply
# ----------------------------------------------------------------------------------------------------------

OFFSETS = [o for o in itertools.product((-1, 0, 1), repeat=3)]  # (dx, dy, dz)


def _offset_coefficient(order, h3, o, kc, ko, fields):
    """The unfolded coefficient of neighbour offset o = (dx, dy, dz) (see `stencil_coefficients`); kc is k^2 at
    the node, ko k^2 at the neighbour, fields = (kx, ky, kz, lap) at the node (order 6). Works elementwise on
    arrays of any shape. Returns None for offsets outside the stencil."""
    nzs = [a for a in range(3) if o[a] != 0]
    hs = [float(v) for v in h3]
    if order == 2:
        if len(nzs) == 0:
            return -sum(2.0 / (x * x) for x in hs) + kc
        if len(nzs) == 1:
            return np.full(np.shape(kc), 1.0 / hs[nzs[0]] ** 2)
        return None
    if order == 4:
        if len(nzs) == 0:
            return (-sum(2.0 / (x * x) for x in hs)
                    + sum((hs[a] ** 2 + hs[b] ** 2) / (3.0 * hs[a] ** 2 * hs[b] ** 2)
                          for a, b in ((0, 1), (0, 2), (1, 2)))
                    + 0.5 * kc)
        if len(nzs) == 1:
            a = nzs[0]
            return (1.0 / hs[a] ** 2
                    - sum((hs[a] ** 2 + hs[b] ** 2) / (6.0 * hs[a] ** 2 * hs[b] ** 2) for b in range(3) if b != a)
                    + ko / 12.0)
        if len(nzs) == 2:
            a, b = nzs
            return np.full(np.shape(kc), (hs[a] ** 2 + hs[b] ** 2) / (12.0 * hs[a] ** 2 * hs[b] ** 2))
        return None
    if order == 6:
        h = hs[0]
        h2 = h * h
        grads = fields[:3]
        lap = fields[3]
        if len(nzs) == 0:
            return -64.0 / (15.0 * h2) + 14.0 / 15.0 * kc + h2 / 20.0 * (lap - kc * kc)
        if len(nzs) == 1:
            a = nzs[0]
            return 14.0 / (30.0 * h2) - ko / 90.0 + o[a] * h * grads[a] * (2.0 + h2 * ko) / 120.0
        if len(nzs) == 2:
            a, b = nzs
            return 3.0 / (30.0 * h2) + ko / 90.0 + h * (o[a] * grads[a] + o[b] * grads[b]) / 120.0
        return np.full(np.shape(kc), 1.0 / (30.0 * h2))
    raise ValueError(order)


def stencil_coefficients(order: int, h3, k2_ext: np.ndarray, fields=None):
    """Coefficient arrays c_o (interior shape) of the unfolded stencil, (A U)_p = sum_o c_o(p) U_{p+o}.

    k2_ext is k^2 on the interior plus one ghost layer; it supplies k^2 at the neighbour in the products
    K U that the scheme differences. Collecting the terms of eq. scheme4 / scheme6 by neighbour class gives:

    order 4 (general h): centre -sum 2/h_nu^2 + sum_{nu<mu} (h_nu^2+h_mu^2)/(3 h_nu^2 h_mu^2) + k_0^2/2;
        face nu: 1/h_nu^2 - sum_{mu != nu} (h_nu^2+h_mu^2)/(6 h_nu^2 h_mu^2) + k_o^2/12;
        edge (nu, mu): (h_nu^2 + h_mu^2)/(12 h_nu^2 h_mu^2); corner 0.
    order 6 (uniform h, readings R2-R6): centre -64/(15h^2) + 14/15 k^2 + h^2/20 (lap k^2 - k^4);
        face +-nu: 14/(30h^2) - k_o^2/90 +- h (k^2)_nu (2 + h^2 k_o^2)/120;
        edge (s_nu nu, s_mu mu): 3/(30h^2) + k_o^2/90 + h (s_nu (k^2)_nu + s_mu (k^2)_mu)/120;
        corner 1/(30h^2).
    """
    nz, ny, nx = (s - 2 for s in k2_ext.shape)
    kc = k2_ext[1:-1, 1:-1, 1:-1]
    coefs = {}
    for o in OFFSETS:
        dx, dy, dz = o
        ko = k2_ext[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
        c = _offset_coefficient(order, h3, o, kc, ko, fields)
        if c is not None:
            coefs[o] = np.asarray(c, np.complex128)
    return coefs


def sampled_matvec(order: int, k2_halo: np.ndarray, h3, gammas, x: np.ndarray, nodes: np.ndarray) -> np.ndarray:
    """(A x)_p for the flat node indices `nodes` only, by the per-offset route (the same coefficients and ghost
    folding as `A_stencil`), so that full-size grids can be checked row by row. k2_halo has a two-cell halo
    (order 2/4 read only its interior); x is the flat vector."""
    nz, ny, nx = (s - 4 for s in k2_halo.shape)
    k2i = k2_halo[2:-2, 2:-2, 2:-2]
    nodes = np.asarray(nodes, np.int64)
    I = nodes % nx
    J = (nodes // nx) % ny
    L = nodes // (nx * ny)
    kc = k2i[L, J, I]
    fields = None
    if order == 6:
        h = float(h3[0])
        g = []
        lap = np.zeros(len(nodes))
        for ax, (di, dj, dl) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
            at = lambda s: k2_halo[L + 2 + s * dl, J + 2 + s * dj, I + 2 + s * di]
            g.append((-at(2) + 8.0 * at(1) - 8.0 * at(-1) + at(-2)) / (12.0 * h))
            lap = lap + (-at(2) + 16.0 * at(1) - 30.0 * at(0) + 16.0 * at(-1) - at(-2)) / (12.0 * h * h)
        fields = (g[0], g[1], g[2], lap)
    dims = (nx, ny, nz)
    out = np.zeros(len(nodes), np.complex128)
    for o in OFFSETS:
        q = [I + o[0], J + o[1], L + o[2]]
        fac = np.ones(len(nodes), np.complex128)
        for a in range(3):
            outside = (q[a] < 0) | (q[a] > dims[a] - 1)
            fac = np.where(outside, fac * gammas[a], fac)
            q[a] = np.clip(q[a], 0, dims[a] - 1)
        ko = k2i[q[2], q[1], q[0]]
        c = _offset_coefficient(order, h3, o, kc, ko, fields)
        if c is None:
            continue
        out += c * fac * x[q[0] + nx * (q[1] + ny * q[2])]
    return out


def apply_unfolded(coefs, u_pad: np.ndarray) -> np.ndarray:
    """sum_o c_o U_{p+o} with U given on the interior plus one ghost layer (exact ghost data)."""
    nz, ny, nx = (s - 2 for s in u_pad.shape)
    out = np.zeros((nz, ny, nx), np.complex128)
    for (dx, dy, dz), c in coefs.items():
        out += c * u_pad[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
    return out


def fold_matrix(coefs, shape, gammas) -> sp.csr_matrix:
    """Assemble the sparse A from unfolded coefficients: a neighbour outside the grid along an axis is
    replaced by the boundary node on that axis times gamma of that axis (eq. D_bc, reading R6)."""
    nz, ny, nx = shape
    ii = np.arange(nz * ny * nx).reshape(shape)
    L, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rows, cols, vals = [], [], []
    dims = (nx, ny, nz)
    for (dx, dy, dz), c in coefs.items():
        fac = np.ones(shape, np.complex128)
        tgt = []
        for ax, (base, d) in enumerate(((I, dx), (J, dy), (L, dz))):
            q = base + d
            lo = q < 0
            hi = q > dims[ax] - 1
            fac = np.where(lo | hi, fac * gammas[ax], fac)
            tgt.append(np.clip(q, 0, dims[ax] - 1))
        col = tgt[0] + nx * (tgt[1] + ny * tgt[2])
        rows.append(ii.ravel())
        cols.append(col.ravel())
        vals.append((c * fac).ravel())
    n = nz * ny * nx
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return A.tocsr()


def A_stencil(order: int, k2_int: np.ndarray, h3, gammas, fields=None) -> sp.csr_matrix:
    """Route 2 for the absorbing (or Dirichlet, gamma = 0) problem: the ghost k^2 in K U is the clamped
    interior value, as the ghost rule applied to the grid function K U requires (reading R6)."""
    k2_ext = np.pad(k2_int, 1, mode="edge")
    return fold_matrix(stencil_coefficients(order, h3, k2_ext, fields), k2_int.shape, gammas)


# ----------------------------------------------------------------------------------------------------------
# Right-hand side F = R_h f
# ----------------------------------------------------------------------------------------------------------

def rhs(order: int, f_halo: np.ndarray, h3, k2_int=None, fields=None) -> np.ndarray:
    """The modified right-hand side, f given on a two-cell halo (reading R8).

    order 2: F = f.
    order 4: F = (1 + sum_nu h_nu^2/12 delta_nu^2) f = f^(IV) (Sec. 2.2, eq. scheme4).
    order 6: f^(VI) of eq. scheme6 minus the f-terms of h^2/20 Delta_h(k^2 U) (Sec. 2.3):
        F = f + h^2/12 Lap_h f - h^4/240 sum delta_nu^4 f + h^4/90 P_h f - h^2/20 k^2 f
            + h^4/60 sum_nu (k^2)_nu delta_nu f,
      where h^2/12 Lap_h f - h^4/240 sum delta^4 f = h^2/12 lap f + h^4/360 sum f_(4 nu) + O(h^6).
    Returns the interior array (Nz, Ny, Nx) complex128.
    """
    f = f_halo.astype(np.complex128)
    c = _interior(f, 2)
    if order == 2:
        return c.copy()
    hs = [float(v) for v in h3]
    d2 = []
    for ax in range(3):
        d2.append((_axis_shift(f, 2, ax, 1) - 2.0 * c + _axis_shift(f, 2, ax, -1)) / hs[ax] ** 2)
    if order == 4:
        return c + sum(hs[a] ** 2 / 12.0 * d2[a] for a in range(3))
    if order == 6:
        h = hs[0]
        h2 = h * h
        kx, ky, kz, _ = fields
        grads = (kx, ky, kz)
        out = c + h2 / 12.0 * (d2[0] + d2[1] + d2[2])
        for ax in range(3):
            d4 = (_axis_shift(f, 2, ax, 2) - 4.0 * _axis_shift(f, 2, ax, 1) + 6.0 * c
                  - 4.0 * _axis_shift(f, 2, ax, -1) + _axis_shift(f, 2, ax, -2)) / h2 ** 2
            out = out - h2 * h2 / 240.0 * d4
            d1 = (_axis_shift(f, 2, ax, 1) - _axis_shift(f, 2, ax, -1)) / (2.0 * h)
            out = out + h2 * h2 / 60.0 * grads[ax] * d1
        # P_h f = sum over axis pairs of delta_a^2 delta_b^2 f (uses the edge neighbours)
        for a, b in ((0, 1), (0, 2), (1, 2)):
            acc = np.zeros_like(c)
            for sa in (-1, 0, 1):
                for sb in (-1, 0, 1):
                    wa = -2.0 if sa == 0 else 1.0
                    wb = -2.0 if sb == 0 else 1.0
                    d = [0, 0, 0]
                    d[2 - a] += sa
                    d[2 - b] += sb
                    acc = acc + wa * wb * _interior(f, 2, *d)
            out = out + h2 * h2 / 90.0 * acc / h2 ** 2
        out = out - h2 / 20.0 * k2_int * c
        return out
    raise ValueError(order)


# ----------------------------------------------------------------------------------------------------------
# Convenience: the whole discrete problem
# ----------------------------------------------------------------------------------------------------------

def problem(order: int, k2_halo: np.ndarray, f_halo: np.ndarray, h: float, k0: float, bc: str = "abc",
            route: str = "kron"):
    """Assemble (A, F) for k^2 and f sampled on a two-cell halo, uniform h, gamma from k0 (bc="abc") or
    gamma = 0 (bc="dirichlet"). k^2 may be complex (an attenuating medium, as in the scattering test of
    Sec. 5.1); the scheme is the same."""
    k2_int = _interior(k2_halo, 2)
    k2_int = k2_int.astype(np.complex128 if np.iscomplexobj(k2_int) else np.float64)
    g = gamma_abc(k0, h) if bc == "abc" else 0.0
    gammas = (g, g, g)
    h3 = (h, h, h)
    fields = derived_fields(k2_halo, h) if order == 6 else None
    if route == "kron":
        A = A_kron(order, k2_int, h3, gammas, fields)
    else:
        A = A_stencil(order, k2_int, h3, gammas, fields)
    F = rhs(order, f_halo, h3, k2_int, fields).ravel()
    return A, F
