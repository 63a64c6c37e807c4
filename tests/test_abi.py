"""The C-ABI library: it loads, exports every symbol include/helm.h declares, and its host-only logic
(argument validation before any device call, the host 1D eigensolver) is right. No GPU needed."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import operators as op

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "helm.h")


def _lib():
    from paper_2602_07711_amd import helm
    if not os.path.exists(helm.LIB_PATH):
        pytest.skip("libhelm.so not built")
    return helm


def test_exports_every_declared_symbol():
    helm = _lib()
    src = open(HEADER).read()
    names = sorted(set(re.findall(r"\b(helm_[a-z0-9_]+)\s*\(", src)))
    assert {"helm_setup", "helm_matvec", "helm_precond_apply", "helm_gmres_solve", "helm_rhs"} <= set(names)
    L = ctypes.CDLL(helm.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.parametrize("n,k0", [(5, 3.0), (32, 20.0), (128, 60.0), (256, 120.0)])
def test_host_eigensolver(n, k0):
    helm = _lib()
    h = 1.0 / (n + 1)
    g = op.gamma_abc(k0, h)
    d, V, Vi = helm.helm_eig1d(n, g)
    L = op.lambda_bar(n, g).toarray()
    assert abs(L @ V - V * d).max() < 1e-13
    assert abs(Vi @ V - np.eye(n)).max() < 1e-12
    ref = np.sort_complex(np.linalg.eigvals(L))
    assert abs(np.sort_complex(d) - ref).max() < 1e-12


@pytest.mark.parametrize("n,k0", [(5, 3.0), (33, 20.0), (128, 60.0), (256, 120.0)])
def test_host_eigensolver_collocated_zeta2(n, k0):
    """Lambda-bar of the collocated closure (gamma = 2 i k0 h, zeta = 2 in the corner off-diagonals) is not
    symmetric; the host eigensolver must still give Lambda-bar V = V diag(d), V^{-1} V = I and numpy's eigenvalues."""
    helm = _lib()
    h = 1.0 / (n - 1)
    g = 2j * k0 * h
    d, V, Vi = helm.helm_eig1d(n, g, 2.0)
    L = op.lambda_bar(n, g, 2.0).toarray()
    assert abs(L @ V - V * d).max() < 1e-12
    assert abs(Vi @ V - np.eye(n)).max() < 1e-11
    ref = np.sort_complex(np.linalg.eigvals(L))
    assert abs(np.sort_complex(d) - ref).max() < 1e-11


@pytest.mark.parametrize("n", [2, 3, 4, 7, 40, 41])
@pytest.mark.parametrize("zeta", [1.0, 2.0])
def test_host_eigensolver_small_and_centrosymmetric(n, zeta):
    """Smallest axes (blocks of one or two modes) and the structure the preconditioner relies on: Lambda-bar has the
    same closure at both ends, so the first ceil(n/2) eigenvectors are symmetric about the middle of the axis and the
    rest skew; rows of V^{-1} likewise."""
    helm = _lib()
    k0 = 5.0
    g = op.gamma_abc(k0, 1.0 / (n + 1)) if zeta == 1.0 else 2j * k0 / (n - 1)
    d, V, Vi = helm.helm_eig1d(n, g, zeta)
    L = op.lambda_bar(n, g, zeta).toarray()
    assert abs(L @ V - V * d).max() < 1e-12
    assert abs(Vi @ V - np.eye(n)).max() < 1e-11
    ev = np.linalg.eigvals(L)
    assert max(np.abs(ev - x).min() for x in d) < 1e-11
    ms = n - n // 2
    assert abs(V[:, :ms] - V[::-1, :ms]).max() < 1e-13
    assert abs(V[:, ms:] + V[::-1, ms:]).max() < 1e-13
    assert abs(Vi[:ms] - Vi[:ms, ::-1]).max() < 1e-13
    assert abs(Vi[ms:] + Vi[ms:, ::-1]).max() < 1e-13


def test_host_eigensolver_dirichlet_closed_form():
    helm = _lib()
    n = 17
    d, V, Vi = helm.helm_eig1d(n, 0j)
    lam = 2 * np.cos(np.pi * np.arange(1, n + 1) / (n + 1))
    assert abs(np.sort(d.real) - np.sort(lam)).max() < 1e-13


def test_setup_validation_returns_einval_without_device():
    helm = _lib()
    L = helm.lib()
    ptr = ctypes.c_void_p()
    hh = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
    bad = [
        (helm.helm_grid(2, 8, 8), hh, 4, 0),                                   # dimension < 3
        (helm.helm_grid(8, 8, 8), (ctypes.c_double * 3)(0.1, 0.2, 0.1), 6, 2),  # order 6 with unequal h
        (helm.helm_grid(8, 8, 8), hh, 5, 2),                                   # bad order
        (helm.helm_grid(8, 8, 8), hh, 6, 0),                                   # order 6 without halo
        (helm.helm_grid(8, 8, 8), (ctypes.c_double * 3)(0.1, -0.1, 0.1), 4, 0),  # negative h
    ]
    for grid, h, order, halo in bad:
        st = L.helm_setup(ctypes.byref(ptr), grid, h, ctypes.c_void_p(1), halo, order, helm.helm_bc(0, 10.0), None)
        assert st == helm.HELM_EINVAL, (order, halo)
        assert L.helm_last_setup_error()
    st = L.helm_setup(ctypes.byref(ptr), helm.helm_grid(8, 8, 8), hh, None, 0, 4, helm.helm_bc(0, 10.0), None)
    assert st == helm.HELM_EINVAL
    st = L.helm_setup(ctypes.byref(ptr), helm.helm_grid(8, 8, 8), hh, ctypes.c_void_p(1), 0, 4,
                      helm.helm_bc(0, float("nan")), None)
    assert st == helm.HELM_EINVAL
