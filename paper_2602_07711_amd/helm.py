"""ctypes binding of libhelm (include/helm.h). Argument marshalling only: every step runs in the HIP library.

Tensors are torch tensors on the GPU (complex128 vectors of n = Nx*Ny*Nz entries, x fastest; float64 k^2 and
complex128 f on the interior plus a two-cell halo). The binding checks device, dtype, contiguity and size,
then passes raw device pointers and torch's current HIP stream.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_longlong, c_void_p

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhelm.so")

HELM_OK, HELM_EINVAL, HELM_ENOMEM, HELM_EDEVICE, HELM_ENOCONV, HELM_EBREAKDOWN, HELM_ENUMERIC, HELM_EUNSUPPORTED = range(8)
STATUS_NAMES = ["HELM_OK", "HELM_EINVAL", "HELM_ENOMEM", "HELM_EDEVICE", "HELM_ENOCONV", "HELM_EBREAKDOWN",
                "HELM_ENUMERIC", "HELM_EUNSUPPORTED"]
BC_ABC2, BC_DIRICHLET, BC_ABC3 = 0, 1, 2
PREC_EIGT, PREC_PFFT, PREC_NONE, PREC_FFT2, PREC_FFT4, PREC_FFT6 = 0, 1, 2, 3, 4, 5
_PREC = {"eigt": PREC_EIGT, "pfft": PREC_PFFT, "none": PREC_NONE, "fft2": PREC_FFT2, "fft4": PREC_FFT4,
         "fft6": PREC_FFT6}
_BC = {"abc": BC_ABC2, "dirichlet": BC_DIRICHLET, "abc3": BC_ABC3}


class HelmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}: {msg}")


class helm_grid(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("nz", c_int)]


class helm_bc(ctypes.Structure):
    _fields_ = [("kind", c_int), ("k0", c_double)]


class helm_solve_opts(ctypes.Structure):
    _fields_ = [("m", c_int), ("maxit", c_int), ("rtol", c_double), ("flexible", c_int), ("prec_fp32", c_int),
                ("prec", c_int), ("x0_given", c_int), ("resid_hist", POINTER(c_double)), ("hist_len", c_int)]


class helm_solve_info(ctypes.Structure):
    _fields_ = [("iters", c_int), ("restarts", c_int), ("converged", c_int), ("hist_used", c_int),
                ("reorths", c_int), ("relres_est", c_double), ("relres_true", c_double), ("t_ms", c_double * 6)]


_lib = None


def lib():
    """Load libhelm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2602_07711_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.helm_setup.argtypes = [POINTER(c_void_p), helm_grid, POINTER(c_double), c_void_p, c_int, c_int, helm_bc, c_void_p]
    L.helm_setup.restype = c_int
    L.helm_setup_complex.argtypes = [POINTER(c_void_p), helm_grid, POINTER(c_double), c_void_p, c_int, c_int, helm_bc,
                                     c_void_p]
    L.helm_setup_complex.restype = c_int
    L.helm_rhs.argtypes = [c_void_p, c_void_p, c_void_p]
    L.helm_rhs.restype = c_int
    L.helm_matvec.argtypes = [c_void_p, c_void_p, c_void_p]
    L.helm_matvec.restype = c_int
    L.helm_precond_apply.argtypes = [c_void_p, c_void_p, c_void_p, c_int, c_int]
    L.helm_precond_apply.restype = c_int
    L.helm_precond_apply_noalloc.argtypes = [c_void_p, c_void_p, c_void_p]
    L.helm_precond_apply_noalloc.restype = c_int
    L.helm_gmres_solve.argtypes = [c_void_p, c_void_p, c_void_p, POINTER(helm_solve_opts), POINTER(helm_solve_info)]
    L.helm_gmres_solve.restype = c_int
    L.helm_size.argtypes = [c_void_p]
    L.helm_size.restype = c_longlong
    L.helm_last_error.argtypes = [c_void_p]
    L.helm_last_error.restype = ctypes.c_char_p
    L.helm_last_setup_error.argtypes = []
    L.helm_last_setup_error.restype = ctypes.c_char_p
    L.helm_destroy.argtypes = [c_void_p]
    L.helm_destroy.restype = None
    L.helm_eig1d.argtypes = [c_int, c_double, c_double, c_void_p, c_void_p, c_void_p]
    L.helm_eig1d.restype = c_int
    L.helm_eig1d_zeta.argtypes = [c_int, c_double, c_double, c_double, c_void_p, c_void_p, c_void_p]
    L.helm_eig1d_zeta.restype = c_int
    L.helm_profile_enable.argtypes = [c_void_p, c_int]
    L.helm_profile_enable.restype = c_int
    L.helm_profile_read.argtypes = [c_void_p, c_int, POINTER(c_double), POINTER(c_longlong), POINTER(c_double)]
    L.helm_profile_read.restype = c_int
    L.helm_profile_name.argtypes = [c_int]
    L.helm_profile_name.restype = ctypes.c_char_p
    L.helm_autotune.argtypes = [c_void_p, c_int, POINTER(c_int), POINTER(c_double)]
    L.helm_autotune.restype = c_int
    L.helm_gemm_config.argtypes = [c_void_p, c_int, c_int]
    L.helm_gemm_config.restype = c_int
    L.helm_batch_create.argtypes = [POINTER(c_void_p), POINTER(c_void_p), c_int, c_int, c_int]
    L.helm_batch_create.restype = c_int
    L.helm_batch_solve.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), c_int, c_double, c_int, c_int,
                                   POINTER(helm_solve_info)]
    L.helm_batch_solve.restype = c_int
    L.helm_batch_destroy.argtypes = [c_void_p]
    L.helm_batch_destroy.restype = None
    L.helm_batch_last_error.argtypes = [c_void_p]
    L.helm_batch_last_error.restype = ctypes.c_char_p
    L.helm_scale_guess.argtypes = [c_void_p, c_void_p, c_void_p, POINTER(c_double), POINTER(c_double)]
    L.helm_scale_guess.restype = c_int
    L.helm_cnn_create.argtypes = [POINTER(c_void_p), c_int, c_int, c_int, ctypes.c_ulonglong, c_void_p]
    L.helm_cnn_create.restype = c_int
    L.helm_cnn_num_params.argtypes = [c_void_p]
    L.helm_cnn_num_params.restype = c_longlong
    for name in ("helm_cnn_get_params", "helm_cnn_set_params", "helm_cnn_get_grads"):
        getattr(L, name).argtypes = [c_void_p, c_void_p]
        getattr(L, name).restype = c_int
    L.helm_cnn_forward.argtypes = [c_void_p, c_void_p, c_void_p, c_int]
    L.helm_cnn_forward.restype = c_int
    L.helm_cnn_loss_grad.argtypes = [c_void_p, c_void_p, c_void_p, c_int, POINTER(c_double)]
    L.helm_cnn_loss_grad.restype = c_int
    L.helm_cnn_adam_step.argtypes = [c_void_p, c_double]
    L.helm_cnn_adam_step.restype = c_int
    L.helm_cnn_train_step.argtypes = [c_void_p, c_void_p, c_void_p, c_int, c_double, POINTER(c_double)]
    L.helm_cnn_train_step.restype = c_int
    L.helm_cnn_prolong.argtypes = [c_void_p, c_void_p, c_int, c_double, c_double, c_double, c_int, c_void_p,
                                   c_int]
    L.helm_cnn_prolong.restype = c_int
    L.helm_cnn_features.argtypes = [c_void_p, c_void_p, c_void_p, c_int, c_int, c_double, c_double, c_double,
                                    c_void_p]
    L.helm_cnn_features.restype = c_int
    L.helm_cnn_last_error.argtypes = [c_void_p]
    L.helm_cnn_last_error.restype = ctypes.c_char_p
    L.helm_cnn_destroy.argtypes = [c_void_p]
    L.helm_cnn_destroy.restype = None
    _lib = L
    return L


def _stream_ptr():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(t: torch.Tensor, dtype, numel: int, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


class Context:
    """Owns a helm_ctx*. Created by helm_setup, freed by helm_destroy (or when garbage-collected)."""

    def __init__(self, ptr: c_void_p, shape, h, order, bc, k0, device):
        self.ptr = ptr
        self.shape = tuple(shape)     # (nz, ny, nx)
        self.n = shape[0] * shape[1] * shape[2]
        self.h = tuple(h)
        self.order = order
        self.bc = bc
        self.k0 = k0
        self.device = device

    def error(self) -> str:
        return lib().helm_last_error(self.ptr).decode()

    def check(self, status: int):
        if status != HELM_OK:
            raise HelmError(status, self.error())

    def __del__(self):
        try:
            if self.ptr:
                lib().helm_destroy(self.ptr)
                self.ptr = None
        except Exception:
            pass


def helm_setup(k2: torch.Tensor, h, order: int, bc: str = "abc", k0: float = 0.0, shape=None) -> Context:
    """Create a context from k^2 (float64, or complex128 for an attenuating medium, on the GPU). k2 has shape
    (Nz+4, Ny+4, Nx+4) (two-cell halo) or, for order 2/4 only, (Nz, Ny, Nx); `shape` = (Nz, Ny, Nx) can be given
    to disambiguate."""
    if (not isinstance(k2, torch.Tensor) or not k2.is_cuda or k2.dtype not in (torch.float64, torch.complex128)
            or not k2.is_contiguous()):
        raise ValueError("k2 must be a contiguous float64 or complex128 GPU tensor")
    if k2.dim() != 3:
        raise ValueError("k2 must be 3-D (z, y, x)")
    if shape is None:
        halo = 2 if order == 6 else 2
        shape = tuple(s - 4 for s in k2.shape) if halo else tuple(k2.shape)
    nz, ny, nx = shape
    if tuple(k2.shape) == (nz + 4, ny + 4, nx + 4):
        halo = 2
    elif tuple(k2.shape) == (nz, ny, nx):
        halo = 0
    else:
        raise ValueError(f"k2 shape {tuple(k2.shape)} does not match grid {shape} with halo 0 or 2")
    hh = (c_double * 3)(*(float(v) for v in (h if hasattr(h, "__len__") else (h, h, h))))
    ptr = c_void_p()
    fn = lib().helm_setup_complex if k2.dtype == torch.complex128 else lib().helm_setup
    st = fn(byref(ptr), helm_grid(nx, ny, nz), hh, c_void_p(k2.data_ptr()), halo, int(order),
            helm_bc(_BC[bc], float(k0)), _stream_ptr())
    if st != HELM_OK:
        raise HelmError(st, lib().helm_last_setup_error().decode())
    return Context(ptr, shape, tuple(hh), order, bc, k0, k2.device)


def helm_rhs(ctx: Context, f: torch.Tensor, F: torch.Tensor | None = None) -> torch.Tensor:
    nz, ny, nx = ctx.shape
    _check(f, torch.complex128, (nz + 4) * (ny + 4) * (nx + 4), "f")
    if F is None:
        F = torch.empty(ctx.n, dtype=torch.complex128, device=f.device)
    _check(F, torch.complex128, ctx.n, "F")
    ctx.check(lib().helm_rhs(ctx.ptr, c_void_p(f.data_ptr()), c_void_p(F.data_ptr())))
    return F


def helm_matvec(ctx: Context, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
    _check(x, torch.complex128, ctx.n, "x")
    if y is None:
        y = torch.empty_like(x)
    _check(y, torch.complex128, ctx.n, "y")
    ctx.check(lib().helm_matvec(ctx.ptr, c_void_p(x.data_ptr()), c_void_p(y.data_ptr())))
    return y


def helm_precond_apply(ctx: Context, y: torch.Tensor, z: torch.Tensor | None = None, kind: str = "eigt",
                       fp32: bool = False) -> torch.Tensor:
    _check(y, torch.complex128, ctx.n, "y")
    if z is None:
        z = torch.empty_like(y)
    _check(z, torch.complex128, ctx.n, "z")
    ctx.check(lib().helm_precond_apply(ctx.ptr, c_void_p(y.data_ptr()), c_void_p(z.data_ptr()), _PREC[kind],
                                       int(bool(fp32))))
    return z


def helm_precond_apply_noalloc(ctx: Context, y: torch.Tensor, z: torch.Tensor) -> torch.Tensor:
    """z = M^{-1} y by the FP32 EigT preconditioner with the library's static staging array (no device allocation
    inside the call; n <= 2^21). z must be given."""
    _check(y, torch.complex128, ctx.n, "y")
    _check(z, torch.complex128, ctx.n, "z")
    ctx.check(lib().helm_precond_apply_noalloc(ctx.ptr, c_void_p(y.data_ptr()), c_void_p(z.data_ptr())))
    return z


def helm_scale_guess(ctx: Context, F: torch.Tensor, x: torch.Tensor) -> complex:
    """x <- alpha x with alpha minimising ||F - alpha A x|| (in place); returns alpha."""
    _check(F, torch.complex128, ctx.n, "F")
    _check(x, torch.complex128, ctx.n, "x")
    ar, ai = c_double(), c_double()
    ctx.check(lib().helm_scale_guess(ctx.ptr, c_void_p(F.data_ptr()), c_void_p(x.data_ptr()), byref(ar), byref(ai)))
    return complex(ar.value, ai.value)


def helm_gmres_solve(ctx: Context, F: torch.Tensor, x: torch.Tensor | None = None, m: int = 50, maxit: int = 1000,
                     rtol: float = 1e-8, flexible: bool = False, prec: str = "eigt", prec_fp32: bool = False,
                     hist_len: int = 4096, raise_on_noconv: bool = True, x0_given: bool | None = None):
    """Solve A x = F. `x` (optional) is the output buffer; it is also the initial guess unless x0_given is
    False (default: x0_given = x is not None); x0_given = 2 (flexible only) takes it as the first search direction
    instead (include/helm.h). Returns (x, info) with info a dict (iters, restarts, converged,
    relres_est, relres_true, t_ms = {matvec, precond, arnoldi, update, host, total}, hist)."""
    _check(F, torch.complex128, ctx.n, "F")
    if x0_given is None:
        x0_given = x is not None
    if x is None:
        x = torch.empty_like(F)
    _check(x, torch.complex128, ctx.n, "x")
    hist = (c_double * max(1, hist_len))()
    opts = helm_solve_opts(int(m), int(maxit), float(rtol), int(bool(flexible)), int(bool(prec_fp32)), _PREC[prec],
                           int(x0_given), ctypes.cast(hist, POINTER(c_double)), int(hist_len))
    info = helm_solve_info()
    st = lib().helm_gmres_solve(ctx.ptr, c_void_p(F.data_ptr()), c_void_p(x.data_ptr()), byref(opts), byref(info))
    out = dict(iters=info.iters, restarts=info.restarts, converged=bool(info.converged), reorths=info.reorths,
               relres_est=info.relres_est,
               relres_true=info.relres_true, status=STATUS_NAMES[st],
               t_ms=dict(zip(("matvec", "precond", "arnoldi", "update", "host", "total"), list(info.t_ms))),
               hist=[hist[i] for i in range(info.hist_used)])
    if st != HELM_OK and not (st == HELM_ENOCONV and not raise_on_noconv):
        raise HelmError(st, ctx.error())
    return x, out


KERNEL_CLASSES = 11


def helm_profile_enable(ctx: Context, on: bool = True):
    """Start (and reset) or stop per-kernel device timing on the context stream."""
    ctx.check(lib().helm_profile_enable(ctx.ptr, int(bool(on))))


def helm_profile_read(ctx: Context) -> dict:
    """{class name: {"ms": total device ms, "launches": count, "work": algorithmic bytes or flops}}."""
    out = {}
    for k in range(KERNEL_CLASSES):
        ms, n, w = c_double(), c_longlong(), c_double()
        ctx.check(lib().helm_profile_read(ctx.ptr, k, byref(ms), byref(n), byref(w)))
        if n.value:
            out[lib().helm_profile_name(k).decode()] = dict(ms=ms.value, launches=n.value, work=w.value)
    return out


GEMM_CONFIGS = [(64, 64, 16), (64, 64, 32), (128, 64, 16), (64, 128, 16)]
GEMM_KINDS = ["x64", "y64", "x32", "y32"]


def helm_autotune(ctx: Context, reps: int = 5) -> dict:
    """Time every tile configuration of the four EigT transforms (forward and inverse separately) on this context
    and keep the fastest. Returns {kind: {"chosen": (BM, BN, BK), "ms": [per-config average ms or None],
    "chosen_inverse": ..., "ms_inverse": [...]}}."""
    chosen = (c_int * 8)()
    ms = (c_double * 32)(*([-1.0] * 32))
    ctx.check(lib().helm_autotune(ctx.ptr, int(reps), chosen, ms))
    out = {}
    for k, name in enumerate(GEMM_KINDS):
        f = [ms[4 * k + c] for c in range(4)]
        i = [ms[16 + 4 * k + c] for c in range(4)]
        out[name] = dict(chosen=GEMM_CONFIGS[chosen[k]], ms=[v if v >= 0 else None for v in f],
                         chosen_inverse=GEMM_CONFIGS[chosen[4 + k]], ms_inverse=[v if v >= 0 else None for v in i])
    return out


def helm_gemm_config(ctx: Context, kind: str, cfg: int):
    ctx.check(lib().helm_gemm_config(ctx.ptr, GEMM_KINDS.index(kind), int(cfg)))


class Batch:
    """Owns a helm_batch*: P FGMRES(m) solves (shared or distinct contexts) advanced together."""

    def __init__(self, ptr, ctxs, m, fp32):
        self.ptr = ptr
        self.ctxs = list(ctxs)   # keeps the contexts alive
        self.m = m
        self.fp32 = fp32

    def error(self) -> str:
        return lib().helm_batch_last_error(self.ptr).decode()

    def __del__(self):
        try:
            if self.ptr:
                lib().helm_batch_destroy(self.ptr)
                self.ptr = None
        except Exception:
            pass


def helm_batch_create(ctxs, m: int = 30, prec_fp32: bool = True) -> Batch:
    arr = (c_void_p * len(ctxs))(*(c.ptr for c in ctxs))
    ptr = c_void_p()
    st = lib().helm_batch_create(byref(ptr), arr, len(ctxs), int(m), int(bool(prec_fp32)))
    if st != HELM_OK:
        raise HelmError(st, lib().helm_batch_last_error(None).decode())
    return Batch(ptr, ctxs, m, prec_fp32)


def helm_batch_solve(batch: Batch, Fs, xs=None, x0_given: bool = False, rtol: float = 1e-8, maxit: int = 1000,
                     use_graph: bool = True, raise_on_noconv: bool = True):
    """Solve every problem of the batch; Fs/xs are lists of complex128 GPU vectors (xs allocated if None).
    Returns (xs, infos) with one info dict per problem."""
    P = len(batch.ctxs)
    if len(Fs) != P:
        raise ValueError("one right-hand side per problem")
    if xs is None:
        xs = [torch.empty_like(F) for F in Fs]
        x0_given = False
    for c, F, x in zip(batch.ctxs, Fs, xs):
        _check(F, torch.complex128, c.n, "F")
        _check(x, torch.complex128, c.n, "x")
    Fa = (c_void_p * P)(*(F.data_ptr() for F in Fs))
    xa = (c_void_p * P)(*(x.data_ptr() for x in xs))
    infos = (helm_solve_info * P)()
    st = lib().helm_batch_solve(batch.ptr, Fa, xa, int(bool(x0_given)), float(rtol), int(maxit), int(bool(use_graph)),
                                infos)
    out = [dict(iters=i.iters, restarts=i.restarts, converged=bool(i.converged), relres_est=i.relres_est,
                relres_true=i.relres_true, cancellations=i.reorths) for i in infos]
    if st != HELM_OK and not (st == HELM_ENOCONV and not raise_on_noconv):
        raise HelmError(st, batch.error())
    return xs, out


def helm_batch_destroy(batch: Batch):
    if batch.ptr:
        lib().helm_batch_destroy(batch.ptr)
        batch.ptr = None


def helm_destroy(ctx: Context):
    if ctx.ptr:
        lib().helm_destroy(ctx.ptr)
        ctx.ptr = None


def helm_eig1d(n: int, gamma: complex, zeta: float = 1.0):
    """Host 1D eigen-decomposition of Lambda-bar (no GPU). Returns numpy (d, V, Vinv)."""
    import numpy as np
    d = np.zeros(n, np.complex128)
    V = np.zeros((n, n), np.complex128)
    Vi = np.zeros((n, n), np.complex128)
    st = lib().helm_eig1d_zeta(int(n), float(gamma.real), float(gamma.imag), float(zeta), c_void_p(d.ctypes.data),
                               c_void_p(V.ctypes.data), c_void_p(Vi.ctypes.data))
    if st != HELM_OK:
        raise HelmError(st, "helm_eig1d failed")
    return d, V, Vi


# ------------------------------------------------------------------------------------------ learned warm start
class Cnn:
    """Owns a helm_cnn* (the warm-start encoder-decoder network of include/helm.h). All its work is ordered on
    the stream that was current at creation."""

    def __init__(self, size: int, max_batch: int = 1, bf16: bool = True, seed: int = 0):
        L = lib()
        self.size = int(size)
        self.max_batch = int(max_batch)
        self.bf16 = bool(bf16)
        self.stream = torch.cuda.current_stream()
        p = c_void_p()
        st = L.helm_cnn_create(byref(p), self.size, self.max_batch, int(self.bf16), ctypes.c_ulonglong(seed),
                               c_void_p(self.stream.cuda_stream))
        if st != HELM_OK:
            raise HelmError(st, L.helm_cnn_last_error(None).decode())
        self.ptr = p
        self.num_params = int(L.helm_cnn_num_params(p))

    def _raise(self, st):
        if st != HELM_OK:
            raise HelmError(st, lib().helm_cnn_last_error(self.ptr).decode())

    def _batch(self, x: torch.Tensor, name: str) -> int:
        V = self.size ** 3
        if x.dim() != 3 or x.shape[1:] != (2, V):
            raise ValueError(f"{name} must have shape [B, 2, {V}], got {tuple(x.shape)}")
        B = x.shape[0]
        if not 1 <= B <= self.max_batch:
            raise ValueError(f"batch {B} outside 1..{self.max_batch}")
        _check(x, torch.float32, B * 2 * V, name)
        return B

    def params(self) -> torch.Tensor:
        out = torch.empty(self.num_params, dtype=torch.float32)
        self._raise(lib().helm_cnn_get_params(self.ptr, c_void_p(out.data_ptr())))
        return out

    def set_params(self, w: torch.Tensor):
        w = w.detach().to(torch.float32).contiguous().cpu()
        if w.numel() != self.num_params:
            raise ValueError(f"expected {self.num_params} parameters, got {w.numel()}")
        self._raise(lib().helm_cnn_set_params(self.ptr, c_void_p(w.data_ptr())))

    def grads(self) -> torch.Tensor:
        out = torch.empty(self.num_params, dtype=torch.float32)
        self._raise(lib().helm_cnn_get_grads(self.ptr, c_void_p(out.data_ptr())))
        return out

    def forward(self, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
        B = self._batch(x, "x")
        if y is None:
            y = torch.empty_like(x)
        self._batch(y, "y")
        self._raise(lib().helm_cnn_forward(self.ptr, c_void_p(x.data_ptr()), c_void_p(y.data_ptr()), B))
        return y

    def loss_grad(self, x: torch.Tensor, t: torch.Tensor) -> float:
        B = self._batch(x, "x")
        if self._batch(t, "t") != B:
            raise ValueError("x and t batch sizes differ")
        loss = c_double()
        self._raise(lib().helm_cnn_loss_grad(self.ptr, c_void_p(x.data_ptr()), c_void_p(t.data_ptr()), B,
                                             byref(loss)))
        return loss.value

    def adam_step(self, lr: float):
        self._raise(lib().helm_cnn_adam_step(self.ptr, float(lr)))

    def train_step(self, x: torch.Tensor, t: torch.Tensor, lr: float, want_loss: bool = True) -> float | None:
        B = self._batch(x, "x")
        if self._batch(t, "t") != B:
            raise ValueError("x and t batch sizes differ")
        loss = c_double()
        self._raise(lib().helm_cnn_train_step(self.ptr, c_void_p(x.data_ptr()), c_void_p(t.data_ptr()), B,
                                              float(lr), byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def prolong(self, coarse: torch.Tensor, nf: int, scale: float = 1.0, gamma: complex = 0.0,
                fine: torch.Tensor | None = None, cubic: bool = False):
        """Trilinear (or cubic) prolongation of a [2, nc^3] prediction to a complex128 vector of nf^3 entries;
        `gamma` is the coarse grid's ghost factor (0: zero extension)."""
        nc = round((coarse.numel() / 2) ** (1 / 3))
        if 2 * nc ** 3 != coarse.numel():
            raise ValueError("coarse must hold 2 * nc^3 values")
        _check(coarse, torch.float32, 2 * nc ** 3, "coarse")
        if fine is None:
            fine = torch.empty(nf ** 3, dtype=torch.complex128, device=coarse.device)
        _check(fine, torch.complex128, nf ** 3, "fine")
        g = complex(gamma)
        self._raise(lib().helm_cnn_prolong(self.ptr, c_void_p(coarse.data_ptr()), nc, float(scale), g.real, g.imag,
                                           int(bool(cubic)), c_void_p(fine.data_ptr()), nf))
        return fine

    def features(self, k2_halo: torch.Tensor, f_halo: torch.Tensor, k0: float, c_scale: float = 1.0,
                 f_scale: float = 1.0, halo: int = 2, out: torch.Tensor | None = None) -> torch.Tensor:
        """Network input [1, 2, S^3] from the solver's k^2 (float64) and f (complex128) arrays with halo."""
        P = round(k2_halo.numel() ** (1 / 3))
        if P ** 3 != k2_halo.numel():
            raise ValueError("k2_halo must be a cube")
        _check(k2_halo, torch.float64, P ** 3, "k2_halo")
        _check(f_halo, torch.complex128, P ** 3, "f_halo")
        if out is None:
            out = torch.empty(1, 2, self.size ** 3, dtype=torch.float32, device=k2_halo.device)
        _check(out, torch.float32, 2 * self.size ** 3, "out")
        self._raise(lib().helm_cnn_features(self.ptr, c_void_p(k2_halo.data_ptr()), c_void_p(f_halo.data_ptr()),
                                            halo, P - 2 * halo, float(k0), float(c_scale), float(f_scale),
                                            c_void_p(out.data_ptr())))
        return out

    def close(self):
        if getattr(self, "ptr", None):
            lib().helm_cnn_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
