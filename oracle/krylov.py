"""Oracle: restarted right-preconditioned GMRES(m) and flexible GMRES(m), complex128.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper solves A A_p^{-1} Y = F, A_p U = Y with right-preconditioned restarted GMRES (Sec. 3.1, eq.
Preconditioned_System; Sec. 4; Sec. 5: MATLAB gmres, restart 20), citing Saad's book for the method. Written
here from that method's definition: modified Gram-Schmidt Arnoldi on A M^{-1}, Givens rotations on the
Hessenberg matrix, and at the end of a cycle x = x0 + M^{-1} V_k y_k (flexible: x = x0 + Z_k y_k with the
stored Z_j = M^{-1} v_j).

Stopping rule (reading): stop when the residual norm is <= rtol * ||F||. With x0 = 0 this is the paper's
rel-res ||A U - F|| / ||A U^0 - F|| (Sec. 5.1); with a warm start it keeps the same absolute target, so a good
initial guess is not penalised. At the end of every cycle the true residual decides whether to restart.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def _givens(a: complex, b: complex):
    """(c, s, r) with [[c, s], [-conj(s), c]] [a, b]^T = [r, 0]^T, c real."""
    if b == 0:
        return 1.0, 0.0 + 0.0j, a
    if a == 0:
        return 0.0, 1.0 + 0.0j, b
    t = np.hypot(abs(a), abs(b))
    ph = a / abs(a)
    return abs(a) / t, ph * np.conj(b) / t, ph * t


def gmres(A, M, b, x0=None, m=30, rtol=1e-8, maxit=10000, flexible=False):
    """Solve A x = b. A(v), M(v) are callables (M applies the preconditioner inverse). Returns (x, info)."""
    b = np.asarray(b, np.complex128)
    n = b.size
    x = np.zeros(n, np.complex128) if x0 is None else np.array(x0, np.complex128)
    bnorm = np.linalg.norm(b)
    info = dict(iters=0, restarts=0, hist=[], converged=False, breakdown=False)
    if bnorm == 0.0:
        info.update(converged=True, relres=0.0)
        return np.zeros(n, np.complex128), info
    its = 0
    while True:
        r = b - A(x)
        beta = np.linalg.norm(r)
        info["hist"].append(beta / bnorm)
        if beta <= rtol * bnorm:
            info["converged"] = True
            break
        if its >= maxit:
            break
        V = np.zeros((m + 1, n), np.complex128)
        Z = np.zeros((m, n), np.complex128) if flexible else None
        H = np.zeros((m + 1, m), np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, np.complex128)
        g = np.zeros(m + 1, np.complex128)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            z = M(V[j])
            if flexible:
                Z[j] = z
            w = A(z)
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            for i in range(j):                           # previous rotations on the new column
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            hj1 = H[j + 1, j]
            cs[j], sn[j], H[j, j] = _givens(H[j, j], hj1)
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            info["hist"].append(abs(g[j + 1]) / bnorm)
            if hj1 == 0.0:
                info["breakdown"] = True
                break
            if abs(g[j + 1]) <= rtol * bnorm or its >= maxit:
                break
            V[j + 1] = w / hj1
        y = scipy.linalg.solve_triangular(H[:k, :k], g[:k])
        if flexible:
            x = x + Z[:k].T @ y
        else:
            x = x + M(V[:k].T @ y)
        info["restarts"] += 1
    info["iters"] = its
    info["relres"] = np.linalg.norm(b - A(x)) / bnorm
    return x, info
