"""Batched solves (many right-hand sides on one medium, and uneven independent problems) against the oracle:
every problem of a batch must reach the same solution as its own sparse LU solve (relative L2 <= 1e-8 at
rtol 1e-10), and the graph-replayed cycle must give bitwise the same result as direct launches."""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import operators as op

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def H():
    import paper_2602_07711_amd as mod
    mod.lib()
    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("fp32", [True, False])
def test_batch_multi_rhs_plane_waves(fp32):
    """Four incident plane waves scattered by one inclusion medium (the scattering source -(k^2 - k0^2) e^{ik0 d.x})."""
    h = H()
    n = 18
    k0 = 0.47 * (n + 1)
    hh = 1.0 / (n + 1)
    k2 = synth.inclusions_k2(n, k0)
    dirs = synth.unit_directions(4, seed=4)
    fs = synth.plane_wave_sources(k2, k0, dirs)
    ctx = h.helm_setup(dev(k2), hh, 6, k0=k0)
    Fs = [h.helm_rhs(ctx, dev(f)) for f in fs]
    batch = h.helm_batch_create([ctx] * len(Fs), m=30, prec_fp32=fp32)
    xs, infos = h.helm_batch_solve(batch, Fs, rtol=1e-10)
    A, _ = op.problem(6, k2, fs[0], hh, k0)
    lu = spla.splu(A.tocsc())
    for f, F, x, info in zip(fs, Fs, xs, infos):
        Fr = op.rhs(6, f, (hh,) * 3, k2[2:-2, 2:-2, 2:-2], op.derived_fields(k2, hh)).ravel()
        xr = lu.solve(Fr)
        rel = np.linalg.norm(host(x) - xr) / np.linalg.norm(xr)
        # the same method one problem at a time: the batch may differ only in the rounding order
        _, single = h.helm_gmres_solve(ctx, F, m=30, rtol=1e-10, flexible=True, prec_fp32=fp32)
        print("multi-rhs", fp32, info, single["iters"], rel)
        assert info["converged"] and rel <= 1e-8
        assert abs(info["iters"] - single["iters"]) <= 1


def test_batch_uneven_problems_graph_and_direct():
    h = H()
    probs = []
    for n, seed in ((14, 400), (17, 401), (21, 402)):
        k0 = 0.45 * (n + 1)
        hh = 1.0 / (n + 1)
        k2 = synth.inclusions_k2(n, k0, seed=seed)
        f = synth.gaussian_source(n)
        probs.append((n, k0, hh, k2, f))
    ctxs = [h.helm_setup(dev(k2), hh, 6, k0=k0) for n, k0, hh, k2, f in probs]
    Fs = [h.helm_rhs(c, dev(p[4])) for c, p in zip(ctxs, probs)]
    batch = h.helm_batch_create(ctxs, m=20, prec_fp32=True)
    xg, ig = h.helm_batch_solve(batch, Fs, rtol=1e-10, use_graph=True)
    xd, idr = h.helm_batch_solve(batch, Fs, rtol=1e-10, use_graph=False)
    xg2, _ = h.helm_batch_solve(batch, Fs, rtol=1e-10, use_graph=True)   # replay of the captured graph
    for (n, k0, hh, k2, f), a, b, c, info in zip(probs, xg, xd, xg2, ig):
        A, Fr = op.problem(6, k2, f, hh, k0)
        xr = spla.splu(A.tocsc()).solve(Fr)
        rel = np.linalg.norm(host(a) - xr) / np.linalg.norm(xr)
        print("uneven", n, info, rel)
        assert info["converged"] and rel <= 1e-8
        assert np.array_equal(host(a), host(b)) and np.array_equal(host(a), host(c))


def test_batch_restarts_and_iteration_cap():
    h = H()
    n = 16
    k0 = 0.47 * (n + 1)
    hh = 1.0 / (n + 1)
    k2 = synth.inclusions_k2(n, k0)
    f = synth.gaussian_source(n)
    ctx = h.helm_setup(dev(k2), hh, 6, k0=k0)
    F = h.helm_rhs(ctx, dev(f))
    batch = h.helm_batch_create([ctx, ctx], m=4, prec_fp32=False)     # restart every 4 steps
    xs, infos = h.helm_batch_solve(batch, [F, F.clone()], rtol=1e-10)
    A, Fr = op.problem(6, k2, f, hh, k0)
    xr = spla.splu(A.tocsc()).solve(Fr)
    for x, info in zip(xs, infos):
        assert info["converged"] and info["restarts"] >= 2
        assert np.linalg.norm(host(x) - xr) <= 1e-8 * np.linalg.norm(xr)
    xs, infos = h.helm_batch_solve(batch, [F, F.clone()], rtol=1e-14, maxit=3, raise_on_noconv=False)
    assert all(i["iters"] == 3 and not i["converged"] for i in infos)


@pytest.mark.parametrize("fp32", [True, False])
def test_split_direction_tiles_single_and_batch(fp32, tmp_path, monkeypatch):
    """Forward and inverse transforms with different tile configurations (forced through the tune cache): the
    single-problem preconditioner keeps its parity with the oracle, and a batch, whose grouped launches take a tile
    count per role from those choices, reaches the sparse LU solution. The box is ragged (the halves of every axis
    span more than one tile of the forward shapes)."""
    from oracle import precond as pc
    h = H()
    nx, ny, nz = 70, 20, 12
    shape = (nz, ny, nx)
    hh = 1.0 / (nx + 1)
    k0 = 0.45 * (nx + 1)
    rng = np.random.default_rng(5)
    k2 = k0 * k0 * (1.0 + 0.2 * rng.random((nz + 4, ny + 4, nx + 4)))
    # tune-cache keys: transform kind, direction (0 forward, 1 inverse), axis length, lines, slices
    fwd = {0: 3, 1: 2, 2: 3, 3: 2}       # (64,128,16) on x, (128,64,16) on y
    inv = {0: 1, 1: 1, 2: 1, 3: 1}       # (64,64,32)
    lines = []
    for kind in range(4):
        n_ax, rows, batch = (nx, ny * nz, 1) if kind % 2 == 0 else (ny, nx, nz)
        lines.append(f"v5 {kind} 0 {n_ax} {rows} {batch} {fwd[kind]}")
        lines.append(f"v5 {kind} 1 {n_ax} {rows} {batch} {inv[kind]}")
    cache = tmp_path / "tune.txt"
    cache.write_text("\n".join(lines) + "\n")
    monkeypatch.setenv("HELM_TUNE_CACHE", str(cache))
    ctx = h.helm_setup(dev(k2), hh, 4, k0=k0, shape=shape)
    res = h.helm_autotune(ctx, reps=1)
    from paper_2602_07711_amd import helm as hm
    cfgs = hm.GEMM_CONFIGS
    for kind, name in enumerate(hm.GEMM_KINDS):
        assert tuple(res[name]["chosen"]) == tuple(cfgs[fwd[kind]])
        assert tuple(res[name]["chosen_inverse"]) == tuple(cfgs[inv[kind]])
    # single-problem preconditioner
    y = rng.standard_normal(nx * ny * nz) + 1j * rng.standard_normal(nx * ny * nz)
    gs = tuple(op.gamma_abc(k0, hh) for _ in range(3))
    zr = pc.EigT(shape, (hh, hh, hh), k0, gs).solve(y)
    z = host(h.helm_precond_apply(ctx, dev(y), fp32=fp32))
    assert np.linalg.norm(z - zr) <= (1e-5 if fp32 else 1e-11) * np.linalg.norm(zr)
    # a batch of two right-hand sides on this context
    fs = [rng.standard_normal((nz + 4, ny + 4, nx + 4)) + 0j for _ in range(2)]
    Fs = [h.helm_rhs(ctx, dev(f)) for f in fs]
    batch = h.helm_batch_create([ctx, ctx], m=30, prec_fp32=fp32)
    xs, infos = h.helm_batch_solve(batch, Fs, rtol=1e-10)
    A, _ = op.problem(4, k2, fs[0], hh, k0)
    lu = spla.splu(A.tocsc())
    for f, x, info in zip(fs, xs, infos):
        xr = lu.solve(op.rhs(4, f, (hh, hh, hh), k2[2:-2, 2:-2, 2:-2]).ravel())
        rel = np.linalg.norm(host(x) - xr) / np.linalg.norm(xr)
        print("split tiles batch", fp32, info, rel)
        assert info["converged"] and rel <= 1e-8


@pytest.mark.parametrize("fp32", [True, False])
def test_second_gram_schmidt_pass_single_and_batch(fp32):
    """The second Gram-Schmidt pass (taken only on severe cancellation by default) forced on every step whose
    orthogonalised vector keeps less than half of its squared norm (HELM_CGS_REORTH = 0.5, the DGKS criterion): the
    single-problem and the batched solvers then take second passes, and both must reach the default runs'
    solutions with the same iteration counts."""
    h = H()
    n = 18
    k0 = 0.47 * (n + 1)
    hh = 1.0 / (n + 1)
    k2 = synth.inclusions_k2(n, k0)
    fs = synth.plane_wave_sources(k2, k0, synth.unit_directions(3, seed=4))
    ctx = h.helm_setup(dev(k2), hh, 6, k0=k0)
    Fs = [h.helm_rhs(ctx, dev(f)) for f in fs]
    kw = dict(m=30, rtol=1e-10, flexible=True, prec_fp32=fp32)
    base = [h.helm_gmres_solve(ctx, F, **kw) for F in Fs]
    batch = h.helm_batch_create([ctx] * len(Fs), m=30, prec_fp32=fp32)
    xb, ib = h.helm_batch_solve(batch, Fs, rtol=1e-10)
    os.environ["HELM_CGS_REORTH"] = "0.5"
    try:
        forced = [h.helm_gmres_solve(ctx, F, **kw) for F in Fs]
        xbf, ibf = h.helm_batch_solve(batch, Fs, rtol=1e-10)
    finally:
        del os.environ["HELM_CGS_REORTH"]
    for (x0, i0), (x1, i1), a, ia, b, iff in zip(base, forced, xb, ib, xbf, ibf):
        r_single = float(torch.linalg.vector_norm(x1 - x0) / torch.linalg.vector_norm(x0))
        r_batch = float(torch.linalg.vector_norm(b - a) / torch.linalg.vector_norm(a))
        print("forced second pass", fp32, i0["iters"], i1["iters"], i1["reorths"], ia["iters"], iff["iters"],
              iff["cancellations"], r_single, r_batch)
        assert i1["reorths"] > 0 and iff["cancellations"] > 0
        assert i1["converged"] and iff["converged"]
        assert abs(i1["iters"] - i0["iters"]) <= 1 and abs(iff["iters"] - ia["iters"]) <= 1
        assert r_single <= 1e-9 and r_batch <= 1e-9
