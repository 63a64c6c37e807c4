"""Per-kernel device timing (helm_profile_enable / helm_profile_read) on the context stream.

The library times its launches with HIP events, and consecutive timed launches share one event (the end of one
launch is the start of the next). These tests check that the launch counts and the algorithmic work of each class
follow the solve's structure, that the class totals fit inside the solve's own duration, and that work the caller
enqueues on the same stream between two library calls is not counted as library kernel time.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def H():
    import paper_2602_07711_amd as mod
    mod.lib()   # fails loudly if the HIP library is missing
    return mod


def _context(n=64):
    h = H()
    w = synth.workload("inclusions", n=n)
    ctx = h.helm_setup(torch.from_numpy(w["k2"]).cuda(), w["h"], w["order"], k0=w["k0"])
    F = h.helm_rhs(ctx, torch.from_numpy(w["f"]).cuda())
    return h, ctx, F


def test_profile_counts_work_and_totals_follow_the_solve():
    h, ctx, F = _context()
    x = torch.empty_like(F)
    form = dict(m=50, rtol=1e-8, flexible=True, prec_fp32=True, x0_given=False)
    h.helm_gmres_solve(ctx, F, x, **form)              # warm-up (lazy set-up, first launches)
    torch.cuda.synchronize()
    h.helm_profile_enable(ctx, True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    _, info = h.helm_gmres_solve(ctx, F, x, **form)
    e1.record()
    torch.cuda.synchronize()
    r = h.helm_profile_read(ctx)
    h.helm_profile_enable(ctx, False)
    wall = e0.elapsed_time(e1)
    its = info["iters"]
    assert info["converged"] and its > 0
    # one FP32 EigT application per Arnoldi step: x and y transforms forward and inverse around one z-solve
    assert r["tridiag32"]["launches"] == its
    assert r["gemm_x32"]["launches"] == 2 * its
    assert r["gemm_y32"]["launches"] == 2 * its
    # one matvec per step, plus restart residuals and the final true residual
    assert its <= r["matvec"]["launches"] <= its + info["restarts"] + 2
    assert r["dots"]["launches"] >= its and r["lincomb"]["launches"] >= its
    # every transform launch carries the same algorithmic work (the folded flop count of the 64^3 grid)
    n = 64
    folded = 8.0 * ((n + 1) // 2) ** 2 + 8.0 * (n // 2) ** 2    # real flops per line of the two half products
    per_launch = r["gemm_x32"]["work"] / r["gemm_x32"]["launches"]
    assert per_launch == pytest.approx(folded * n * n, rel=1e-12)
    total = sum(v["ms"] for v in r.values())
    assert all(v["ms"] > 0 for v in r.values())
    assert total <= 1.05 * wall + 0.05, (total, wall)


def test_profile_excludes_caller_work_between_library_calls():
    h, ctx, F = _context()
    y = torch.empty_like(F)
    a = torch.randn(4096, 4096, device="cuda")
    h.helm_matvec(ctx, F, y)
    _ = a @ a
    torch.cuda.synchronize()
    # alone: two matvecs on an idle stream
    h.helm_profile_enable(ctx, True)
    h.helm_matvec(ctx, F, y)
    h.helm_matvec(ctx, F, y)
    alone = h.helm_profile_read(ctx)["matvec"]
    h.helm_profile_enable(ctx, False)
    assert alone["launches"] == 2
    # busy: the caller's matrix products before and between the two matvecs keep the stream busy, so the first
    # matvec's end event is still pending when the second call is made
    h.helm_profile_enable(ctx, True)
    for _ in range(10):
        b = a @ a
    h.helm_matvec(ctx, F, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b = a @ a
    e1.record()
    h.helm_matvec(ctx, F, y)
    busy = h.helm_profile_read(ctx)["matvec"]
    h.helm_profile_enable(ctx, False)
    torch.cuda.synchronize()
    caller = e0.elapsed_time(e1)
    assert busy["launches"] == 2
    assert caller > 5.0, caller                        # the caller's work is long against a 64^3 matvec
    assert busy["ms"] < 0.2 * caller, (busy["ms"], caller)
    assert busy["ms"] < 3.0 * alone["ms"] + 0.05, (busy["ms"], alone["ms"])
    del b
