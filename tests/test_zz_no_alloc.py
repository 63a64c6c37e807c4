"""The entry point that allocates nothing (helm_precond_apply_noalloc) against helm_precond_apply's FP32 EigT
preconditioner, through the C ABI: two calls in a row, the second on a smaller problem, then a rejected size.

The two entry points run the same kernels in the same order on the same inputs, so their outputs must agree to
rounding; the bar is TOL32 (the FP32 preconditioner's parity bound against the oracle), and each output is also
checked against the oracle's EigT to that bound.
"""
import numpy as np
import pytest

from oracle import operators as op
from oracle import precond as pc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL32 = 1e-5
MAX_N = 1 << 21


def H():
    import paper_2602_07711_amd as mod
    mod.lib()
    return mod


def _case(shape, seed):
    nz, ny, nx = shape
    h3 = (1.0 / (nx + 1), 1.0 / (ny + 1), 1.0 / (nz + 1))
    k0 = 0.45 / h3[0]
    k2 = np.full((nz + 4, ny + 4, nx + 4), k0 * k0)
    rng = np.random.default_rng(seed)
    y = rng.standard_normal(nx * ny * nz) + 1j * rng.standard_normal(nx * ny * nz)
    return h3, k0, k2, y


def _run(h, shape, seed):
    h3, k0, k2, y = _case(shape, seed)
    nz, ny, nx = shape
    print(f"noalloc case shape={shape} seed={seed}", flush=True)
    ctx = h.helm_setup(torch.from_numpy(k2).cuda(), h3, 4, k0=k0, shape=shape)
    yd = torch.from_numpy(y).cuda()
    z_ref = h.helm_precond_apply(ctx, yd, fp32=True)
    z_na = torch.full_like(yd, float("nan"))
    h.helm_precond_apply_noalloc(ctx, yd, z_na)
    torch.cuda.synchronize()
    zr, zn = z_ref.cpu().numpy(), z_na.cpu().numpy()
    d = np.linalg.norm(zn - zr) / np.linalg.norm(zr)
    gs = tuple(op.gamma_abc(k0, hh) for hh in h3)
    zo = pc.EigT(shape, h3, k0, gs).solve(y)
    e = np.linalg.norm(zn - zo) / np.linalg.norm(zo)
    print(f"  noalloc vs helm_precond_apply {d:.2e} (bitwise {np.array_equal(zn, zr)}), vs oracle EigT {e:.2e}",
          flush=True)
    assert np.all(np.isfinite(zn))
    assert d <= TOL32 and e <= TOL32
    return ctx


def test_noalloc_matches_precond_apply_two_calls():
    h = H()
    big = (128, 128, 128)                  # exactly the maximum size
    small = (12, 20, 70)                   # ragged tiles, smaller than the first call
    assert np.prod(big) == MAX_N
    _run(h, big, 1)
    _run(h, small, 2)


def test_noalloc_rejects_sizes_above_its_maximum():
    h = H()
    shape = (128, 128, 129)
    h3, k0, k2, _ = _case(shape, 3)
    ctx = h.helm_setup(torch.from_numpy(k2).cuda(), h3, 4, k0=k0, shape=shape)
    y = torch.zeros(int(np.prod(shape)), dtype=torch.complex128, device="cuda")
    z = torch.zeros_like(y)
    with pytest.raises(RuntimeError, match="exceeds its maximum"):
        h.helm_precond_apply_noalloc(ctx, y, z)
