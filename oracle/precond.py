"""Oracle: the second-order preconditioner M = A_p / h_z^2 and its direct solvers EigT and PFFT.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A_p (Sec. 4.1) = I_z (x) (a_y Lb_y (x) I_x + a_x I_y (x) Lb_x) + (Lb_z + K_z - 2(a_x + a_y + 1) I_z) (x) I_xy,
a_nu = h_z^2 / h_nu^2, K_z = h_z^2 k0^2 I (constant background k0, Sec. 4). Dividing by h_z^2 gives
M = Delta + k0^2 I with the same ghost-eliminated T_nu as the high-order operator, so M is close to A in
scale (reading: the library solves M z = y, i.e. A_p z = h_z^2 y).

Readings: the diagonal of the decoupled z-systems is a_x d_x,i + a_y d_y,j + h_z^2 k0^2 - 2(a_x + a_y + 1)
(eq. DIAGprec; the unscaled d_x,i + d_y,j printed under eq. Indep_precond_system agrees when a = 1);
zeta = 1 (staggered two-point closure) on every axis; zeta = 2 (the three-point closure of collocated grids, the
boundary nodes being unknowns, gamma = 2 i k0 h) for EigT as a direct solver (M_collocated).
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.sparse as sp

from .operators import lambda_bar, d2_1d, _lift


def M_matrix(shape, h3, k0: float, gammas) -> sp.csr_matrix:
    """M = T_x + T_y + T_z + k0^2 I, the 7-point operator with the ghost-eliminated absorbing closure."""
    nz, ny, nx = shape
    ns = (nx, ny, nz)
    M = sum(_lift(shape, d2_1d(ns[a], h3[a], gammas[a]), a) for a in range(3))
    return (M + k0 * k0 * sp.identity(nx * ny * nz, np.complex128)).tocsr()


def M_collocated(shape, h3, k0: float, gammas, zeta: complex = 2.0) -> sp.csr_matrix:
    """The second-order operator with the three-point closure of collocated grids (Sec. 4.1: Lambda-bar with
    corners gamma and zeta = 2, the boundary nodes being unknowns): sum_a (Lambda-bar_a - 2I)/h_a^2 + k0^2 I."""
    nz, ny, nx = shape
    ns = (nx, ny, nz)
    M = sum(_lift(shape, ((lambda_bar(ns[a], gammas[a], zeta) - 2.0 * sp.identity(ns[a], np.complex128))
                          / (h3[a] * h3[a])).tocsr(), a) for a in range(3))
    return (M + k0 * k0 * sp.identity(nx * ny * nz, np.complex128)).tocsr()


def M_dirichlet(shape, h3, k0: float) -> sp.csr_matrix:
    """The comparison preconditioner FFT2 (Sec. 5.1; the FFT-type approach recalled at the start of Sec. 4): the
    same 7-point operator with the constant k0 but zero Dirichlet values on all six faces, i.e. M with gamma = 0
    on every axis. Its inverse applied to y is the sparse LU solve of this matrix."""
    return M_matrix(shape, h3, k0, (0.0, 0.0, 0.0))


def M_dirichlet_compact(shape, h3, k0: float, order: int) -> sp.csr_matrix:
    """The comparison preconditioners FFT4 / FFT6 (Sec. 5.1): the fourth- / sixth-order compact operator of
    eq. scheme4 / scheme6 with the constant background k0 (so every derivative of k^2 vanishes) and zero Dirichlet
    values on all six faces (gamma = 0). Its inverse applied to y is the sparse LU solve of this matrix."""
    from .operators import A_kron
    nz, ny, nx = shape
    k2 = np.full(shape, k0 * k0)
    fields = None
    if order == 6:
        z = np.zeros(shape)
        fields = (z, z, z, z)
    return A_kron(order, k2, h3, (0.0, 0.0, 0.0), fields)


def eig1d(n: int, gamma: complex, zeta: complex = 1.0):
    """Step 1 of eq. EIG_SOLVER: D, V, V^{-1} of Lambda-bar (numpy eig and inv). Returns (d, V, Vinv)."""
    Lb = lambda_bar(n, gamma, zeta).toarray()
    d, V = np.linalg.eig(Lb)
    return d, V, np.linalg.inv(V)


def thomas(bbar: np.ndarray, gz: complex, r: np.ndarray, zeta: complex = 1.0) -> np.ndarray:
    """Solve, for every line (j, i) at once, the z-systems of eq. Indep_precond_system:
        (gz + b) u_1 + zeta u_2 = r_1,  u_{l-1} + b u_l + u_{l+1} = r_l,  zeta u_{N-1} + (gz + b) u_N = r_N.
    bbar has shape (Ny, Nx); r has shape (Nz, Ny, Nx). Plain Thomas elimination without pivoting on the
    tridiagonal with sub-diagonal a_l, diagonal d_l and super-diagonal c_l."""
    nz = r.shape[0]
    cp = np.empty_like(r)
    dp = np.empty_like(r)
    for l in range(nz):
        d = bbar + (gz if (l == 0 or l == nz - 1) else 0.0)
        c = zeta if l == 0 else 1.0                     # super-diagonal of row l
        a = zeta if l == nz - 1 else 1.0                # sub-diagonal of row l
        if l == 0:
            p = d
            dp[0] = r[0] / p
        else:
            p = d - a * cp[l - 1]
            dp[l] = (r[l] - a * dp[l - 1]) / p
        cp[l] = c / p
    u = np.empty_like(r)
    u[-1] = dp[-1]
    for l in range(nz - 2, -1, -1):
        u[l] = dp[l] - cp[l] * u[l + 1]
    return u


class EigT:
    """The EigT direct solver of M z = y (Sec. 4.1, eq. EIG_SOLVER)."""

    def __init__(self, shape, h3, k0: float, gammas, zeta: complex = 1.0):
        self.shape = shape
        nz, ny, nx = shape
        hx, hy, hz = h3
        self.ax, self.ay = hz * hz / (hx * hx), hz * hz / (hy * hy)
        self.hz2 = hz * hz
        self.gz = gammas[2]
        self.zeta = zeta
        self.dx, self.Vx, self.Vxi = eig1d(nx, gammas[0], zeta)       # Step 1
        self.dy, self.Vy, self.Vyi = eig1d(ny, gammas[1], zeta)
        self.bbar = (self.ax * self.dx[None, :] + self.ay * self.dy[:, None] + hz * hz * k0 * k0
                     - 2.0 * (self.ax + self.ay + 1.0))

    def forward(self, Y):
        """Step 2: Ybar_l = (V_y^{-1} (x) V_x^{-1}) Y_l for every slice l."""
        return self.Vyi @ Y @ self.Vxi.T

    def inverse(self, Ub):
        """Step 4: U_l = (V_y (x) V_x) Ubar_l."""
        return self.Vy @ Ub @ self.Vx.T

    def solve(self, y: np.ndarray) -> np.ndarray:
        Y = y.reshape(self.shape)
        Yb = self.forward(Y)
        Ub = thomas(self.bbar, self.gz, self.hz2 * Yb, self.zeta)  # Step 3 (A_p z = h_z^2 y)
        return self.inverse(Ub).ravel()


def dst_matrix(n: int) -> np.ndarray:
    """Orthonormal eigenvectors of the Dirichlet Lambda (Sec. 3.1, eq. LMB_egv): sqrt(2h) sin(pi h i l)."""
    h = 1.0 / (n + 1)
    i = np.arange(1, n + 1)
    return np.sqrt(2.0 * h) * np.sin(np.pi * h * np.outer(i, i))


class PFFT:
    """The PFFT direct solver of M z = y (Sec. 4.2, eq. PFFT_SOLVER).

    Step 1: Theta = (A_p^F)^{-1} Y with a 2D sine transform per slice (scipy DST-I) and z-solves.
    Step 2: A_p W = (A_p^F - A_p) Theta; the right-hand side lives on the faces i in {1, N_x} and
            j in {1, N_y} of every slice, and only W on those faces is used afterwards.
    Step 3: U = (A_p^F)^{-1} [Y + (A_p^F - A_p)(Theta + W)].
    A_p^F uses the Dirichlet Lambda in x and y and the absorbing Lambda-bar in z (eq. TFprec).
    With zeta != 1 (the collocated closure) Lambda - Lambda-bar has rows 1 and N only, but each reaches two
    layers: gamma on the face node and zeta - 1 on its inner neighbour (eq. lambda_mat_definition), so W is kept
    on two layers per face.
    """

    def __init__(self, shape, h3, k0: float, gammas, zeta: complex = 1.0):
        self.shape = shape
        nz, ny, nx = shape
        hx, hy, hz = h3
        self.ax, self.ay = hz * hz / (hx * hx), hz * hz / (hy * hy)
        self.hz2 = hz * hz
        self.gx, self.gy, self.gz = gammas
        lam_x = 2.0 * np.cos(np.pi * np.arange(1, nx + 1) / (nx + 1))
        lam_y = 2.0 * np.cos(np.pi * np.arange(1, ny + 1) / (ny + 1))
        self.bF = (self.ax * lam_x[None, :] + self.ay * lam_y[:, None] + hz * hz * k0 * k0
                   - 2.0 * (self.ax + self.ay + 1.0)).astype(np.complex128)
        self.zeta = zeta
        self.eig = EigT(shape, h3, k0, gammas, zeta)

    @staticmethod
    def _dst2(Y):
        # orthonormal DST-I along x and y of every slice; it is its own inverse
        return scipy.fft.dstn(Y, type=1, axes=(1, 2), norm="ortho")

    def solve_F(self, Ys):
        """(A_p^F)^{-1} Ys for an h_z^2-scaled right-hand side."""
        return self._dst2(thomas(self.bF, self.gz, self._dst2(Ys), self.zeta))

    def E_apply(self, X):
        """(A_p^F - A_p) X = a_x (Lambda - Lambda-bar)_x X + a_y (Lambda - Lambda-bar)_y X: on the face row 1,
        -a (gamma X_1 + (zeta - 1) X_2), and the mirror on row N (eq. PFFT_SOLVER, the vectors Theta^x_l,
        Theta^y_l)."""
        out = np.zeros_like(X)
        z1 = self.zeta - 1.0
        out[:, :, 0] -= self.ax * (self.gx * X[:, :, 0] + z1 * X[:, :, 1])
        out[:, :, -1] -= self.ax * (self.gx * X[:, :, -1] + z1 * X[:, :, -2])
        out[:, 0, :] -= self.ay * (self.gy * X[:, 0, :] + z1 * X[:, 1, :])
        out[:, -1, :] -= self.ay * (self.gy * X[:, -1, :] + z1 * X[:, -2, :])
        return out

    def solve(self, y: np.ndarray) -> np.ndarray:
        Ys = self.hz2 * y.reshape(self.shape)
        theta = self.solve_F(Ys)                                        # Step 1
        rhs_w = self.E_apply(theta)
        W = self.eig.inverse(thomas(self.eig.bbar, self.gz, self.eig.forward(rhs_w), self.zeta))  # Step 2
        ring = np.zeros(self.shape, bool)
        layers = [0, -1] if self.zeta == 1.0 else [0, 1, -2, -1]
        ring[:, :, layers] = True
        ring[:, layers, :] = True
        W = np.where(ring, W, 0.0)                                      # only W where E reads it is kept
        U = self.solve_F(Ys + self.E_apply(theta + W))                  # Step 3
        return U.ravel()


def sparse_forward(eig: EigT, Yr: np.ndarray) -> np.ndarray:
    """Forward transform of a slice stack supported on the faces i in {1,N_x}, j in {1,N_y} (Sec. 4.2,
    Step 1 and Step 2*): S_m = V_x^{-1} Y_m for the rows m in {1, N_y}, then the two boundary columns of
    V_x^{-1} times the interior part of the x-faces. Same result as `eig.forward` on such input."""
    nz, ny, nx = Yr.shape
    out = np.zeros_like(Yr)
    Vxi, Vyi = eig.Vxi, eig.Vyi
    for m in (0, ny - 1):                     # rows on the y-faces: full x-transform, then spread over j
        S = Yr[:, m, :] @ Vxi.T               # (nz, nx)
        out += Vyi[None, :, m, None] * S[:, None, :]
    inner = Yr[:, 1:ny - 1, :]                # interior rows carry data only at i = 1, N_x
    for nu in (0, nx - 1):
        t = inner[:, :, nu] @ Vyi[:, 1:ny - 1].T   # (nz, ny): sum over m = 2..N_y-1 of v^{-1}_{y,j,m} Y_{nu,m}
        out += t[:, :, None] * Vxi[None, None, :, nu]
    return out


def restricted_inverse(eig: EigT, Wb: np.ndarray) -> np.ndarray:
    """Inverse transform evaluated on the faces only (Sec. 4.2, eq. PFFT_INV). Returns a full-size array that is
    zero away from the faces i in {1, N_x}, j in {1, N_y}."""
    nz, ny, nx = Wb.shape
    out = np.zeros_like(Wb)
    Vx, Vy = eig.Vx, eig.Vy
    for j in (0, ny - 1):                                  # Step 1: rows j = 1, N_y in full
        out[:, j, :] = np.einsum("m,lmk->lk", Vy[j, :], Wb) @ Vx.T
    s = np.einsum("im,ljm->lji", Vx[[0, nx - 1], :], Wb)   # Step 2: s_{i,j} for i = 1, N_x
    for a, i in enumerate((0, nx - 1)):                     # Step 3: W_{i,j} for j = 2..N_y-1
        out[:, 1:ny - 1, i] = s[:, :, a] @ Vy[1:ny - 1, :].T
    return out


def sampled_M(shape, h3, k0: float, gammas, z: np.ndarray, nodes: np.ndarray) -> np.ndarray:
    """(M z)_p for the flat node indices `nodes` only: the 7-point rows of Delta + k0^2 I with the ghost rule
    U_0 = gamma U_1 per axis, for checking a preconditioner output on full-size grids row by row."""
    nz, ny, nx = shape
    nodes = np.asarray(nodes, np.int64)
    P = [nodes % nx, (nodes // nx) % ny, nodes // (nx * ny)]
    dims = (nx, ny, nz)
    zc = z[nodes]
    out = k0 * k0 * zc
    for a in range(3):
        for s in (-1, 1):
            q = [P[0].copy(), P[1].copy(), P[2].copy()]
            q[a] = q[a] + s
            outside = (q[a] < 0) | (q[a] > dims[a] - 1)
            q[a] = np.clip(q[a], 0, dims[a] - 1)
            val = z[q[0] + nx * (q[1] + ny * q[2])]
            val = np.where(outside, gammas[a] * val, val)
            out = out + (val - zc) / (h3[a] * h3[a])
    return out
