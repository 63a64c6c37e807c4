#!/usr/bin/env python3
"""Benchmark of the compact-Helmholtz EigT-(F)GMRES solve on one MI355X.

Workload (the 256^3 filtered-noise medium): 6th-order compact 27-point scheme, N = 256 per axis, h = 1/257,
k0 = 120 (k0 h = 0.467), k^2 = k0^2 (1 + 0.2 w) with w seeded uniform noise filtered by a Gaussian of width
8 cells and normalised to max|w| = 1, Gaussian point source (sigma = 2h) at the centre, two-point absorbing
closure on all faces. Every input is synthetic and seeded.

One step = one complete solve to ||F - A x|| <= 1e-8 ||F|| from x = 0 with inputs resident in HBM:
  * headline form: FGMRES(50) in FP64 with the EigT preconditioner in complex FP32 on MFMA;
  * reference form: plain right-preconditioned GMRES(50) with the EigT preconditioner in FP64;
  * the PFFT preconditioner (second path) in the same two forms;
  * optionally (--forms), the Dirichlet comparison preconditioner FFT2 in both forms, capped at 1000 iterations.
value = unknowns x iterations / s of the headline form; ms_per_step = its time-to-solution.

Prints one JSON line. Per-kernel device times come from HIP events recorded on the solve's stream over the
timed region (helm_profile_*); the roofline entry is the kernel class with the largest share of device time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

PEAK = {"hbm_GBps": 8000.0, "fp64_TFLOPs": 78.6, "fp32_TFLOPs": 157.3}
# kernel class -> (bound, unit, peak) ; work is bytes (hbm) or flops (mfma)
KCLASS = {
    "matvec": ("hbm", "GB/s", PEAK["hbm_GBps"]),
    "gemm_x64": ("mfma", "TFLOP/s", PEAK["fp64_TFLOPs"]),
    "gemm_y64": ("mfma", "TFLOP/s", PEAK["fp64_TFLOPs"]),
    "gemm_x32": ("mfma", "TFLOP/s", PEAK["fp32_TFLOPs"]),
    "gemm_y32": ("mfma", "TFLOP/s", PEAK["fp32_TFLOPs"]),
    "tridiag64": ("hbm", "GB/s", PEAK["hbm_GBps"]),
    "tridiag32": ("hbm", "GB/s", PEAK["hbm_GBps"]),
    "dots": ("hbm", "GB/s", PEAK["hbm_GBps"]),
    "lincomb": ("hbm", "GB/s", PEAK["hbm_GBps"]),
    "sine": ("mfma", "TFLOP/s", None),      # peak by the form's precision (see kernel_table)
    "ring": ("hbm", "GB/s", PEAK["hbm_GBps"]),
}


# HBM traffic per dispatch measured by rocprofv3 (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy) for the
# headline form; kernel class -> kernel name in that summary. Classes whose launches use several kernel
# variants (the GEMMs) have no single row and report no traffic.
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "noise256_fp32_eigt_fgmres_hbm_traffic.md")
TRAFFIC_KERNEL = {"lincomb": ("k_lincomb_cgs", "k_lincomb<z64>", "k_lincomb<z32>"), "dots": ("k_dots",),
                  "matvec": ("k_matvec<6, true, z32, false>",), "tridiag32": ("k_tridiag_chunk<float, z32>",)}


def measured_traffic(kclass: str):
    """Bytes per dispatch (read + write) of the kernel class from the committed counter summary: the average over
    the dispatches of the class's kernels (weighted by their dispatch counts), or None."""
    names = TRAFFIC_KERNEL.get(kclass)
    if names is None or not os.path.exists(TRAFFIC_FILE):
        return None
    tot, cnt = 0.0, 0
    for line in open(TRAFFIC_FILE):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 4 and cells[0].strip("`") in names:
            tot += int(cells[1]) * (float(cells[2]) + float(cells[3])) * 2 ** 20
            cnt += int(cells[1])
    return tot / cnt if cnt else None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_table(prof, fp32=False):
    out = {}
    for name, v in prof.items():
        bound, unit, peak = KCLASS[name]
        if peak is None:
            peak = PEAK["fp32_TFLOPs"] if fp32 else PEAK["fp64_TFLOPs"]
        avg_ms = v["ms"] / v["launches"]
        rate = v["work"] / (v["ms"] * 1e-3)
        achieved = rate / (1e9 if unit == "GB/s" else 1e12)
        out[name] = dict(bound=bound, launches=v["launches"], total_ms=round(v["ms"], 4), avg_ms=round(avg_ms, 5),
                         work_per_launch=v["work"] / v["launches"], achieved=round(achieved, 3), unit=unit,
                         peak=peak, frac=round(achieved / peak, 4))
    return out


def cpu_baseline(n_cpu: int = 256, iters: int = 8):
    """The oracle (numpy/scipy complex128, per-offset CSR assembly, its EigT and its GMRES(50)) on the benchmark
    workload itself (256^3 filtered noise, 6th order, k0 = 120), timed on the host over a bounded sample: the
    first `iters` GMRES iterations. Assembly and eigen set-up (about 90 s and 40 GB at 256^3) are timed
    separately and excluded from the rate."""
    import threadpoolctl

    import synth
    from oracle import krylov as kr
    from oracle import operators as op
    from oracle import precond as pc
    w = synth.workload("noise", n_cpu)
    k0, h = w["k0"] * (n_cpu + 1) / 257.0, 1.0 / (n_cpu + 1)
    k2 = w["k2"] if n_cpu == 256 else synth.filtered_noise_k2(n_cpu, k0)
    t0 = time.perf_counter()
    A, F = op.problem(6, k2, w["f"], h, k0, route="stencil")
    g = op.gamma_abc(k0, h)
    e = pc.EigT((n_cpu,) * 3, (h,) * 3, k0, (g, g, g))
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    x, info = kr.gmres(lambda v: A @ v, e.solve, F, m=50, rtol=1e-8, maxit=iters)
    t_solve = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()] or [1])
    rate = n_cpu ** 3 * info["iters"] / t_solve
    return dict(value=rate, unit="unknowns*iterations/s", cores=int(threads), kind="oracle",
                sample=(f"the first {info['iters']} iterations of the oracle's FP64 EigT-GMRES(50) on the {n_cpu}^3 "
                        f"filtered-noise workload (6th order, k0 = {k0:.2f}), {t_solve:.2f} s including the final "
                        f"true-residual matvec; per-offset CSR assembly + eigen set-up {t_setup:.2f} s excluded"),
                time_s=round(t_solve, 3), iters=info["iters"], setup_s=round(t_setup, 2))


def bench_batched(H, torch, dev, args):
    """The batched workloads, FP32-EigT FGMRES(30) at rtol 1e-8, one batched solve against the same problems
    solved one after another:
      * multi-RHS: 64 plane waves (seeded directions) scattered by the 128^3 four-inclusion medium (k0 = 60),
        f_m = -(k^2 - k0^2) exp(i k0 d_m . x);
      * uneven: 16 independent problems, N_p = 64..160, k0_p ~ U[30, 90] (seed 40), four-inclusion media
        (seeds 400 + p), Gaussian source."""
    import synth
    out = {}
    m, rtol = 30, 1e-8

    def run(name, ctxs, Fs):
        batch = H.helm_batch_create(ctxs, m=m, prec_fp32=True)
        xs = [torch.empty_like(F) for F in Fs]
        H.helm_batch_solve(batch, Fs, xs, rtol=rtol)                     # warm-up (captures the cycle graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, infos = H.helm_batch_solve(batch, Fs, xs, rtol=rtol)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        del batch
        torch.cuda.empty_cache()
        x1 = torch.empty_like(Fs[0])
        seq_iters = []
        H.helm_gmres_solve(ctxs[0], Fs[0], x1, m=m, rtol=rtol, flexible=True, prec_fp32=True, x0_given=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c, F in zip(ctxs, Fs):
            if x1.numel() != F.numel():
                x1 = torch.empty_like(F)
            _, inf = H.helm_gmres_solve(c, F, x1, m=m, rtol=rtol, flexible=True, prec_fp32=True, x0_given=False)
            seq_iters.append(inf["iters"])
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        work = sum(c.n * i["iters"] for c, i in zip(ctxs, infos))
        res = dict(problems=len(ctxs), batch_ms=round(1e3 * tb, 2), sequential_ms=round(1e3 * ts, 2),
                   speedup=round(ts / tb, 3), unknowns_iters_per_s=work / tb,
                   iters=[i["iters"] for i in infos], sequential_iters=seq_iters,
                   all_converged=all(i["converged"] for i in infos),
                   max_relres=max(i["relres_true"] for i in infos))
        log(f"batched {name}: {res['batch_ms']} ms batched vs {res['sequential_ms']} ms sequential "
            f"({res['speedup']}x), {res['unknowns_iters_per_s']:.3e} unknowns*it/s")
        return res

    w = synth.workload("inclusions")
    k2 = torch.from_numpy(w["k2"]).to(dev)
    ctx = H.helm_setup(k2, w["h"], 6, k0=w["k0"])
    if not args.no_autotune:
        H.helm_autotune(ctx, reps=3)
    dirs = synth.unit_directions(64, seed=4)
    Fs = []
    for d in dirs:
        f = synth.plane_wave_sources(w["k2"], w["k0"], d[None, :])[0]
        Fs.append(H.helm_rhs(ctx, torch.from_numpy(f).to(dev)))
    out["multi_rhs_64x128"] = run("64 RHS x 128^3", [ctx] * len(Fs), Fs)
    del Fs
    torch.cuda.empty_cache()
    ctxs, Fs = [], []
    for p, (n, k0) in enumerate(synth.uneven_problem_set()):
        k2p = synth.inclusions_k2(n, k0, seed=400 + p)
        c = H.helm_setup(torch.from_numpy(k2p).to(dev), 1.0 / (n + 1), 6, k0=k0)
        ctxs.append(c)
        Fs.append(H.helm_rhs(c, torch.from_numpy(synth.gaussian_source(n)).to(dev)))
    if not args.no_autotune:
        H.helm_autotune(ctxs[0], reps=3)
    out["uneven_16"] = run("16 uneven 64^3..160^3", ctxs, Fs)
    return out


def bench_learned(H, torch, args):
    """Learned warm start: 64^3 four-inclusion problems (k0 = 60, source width 0.03, inclusion and source
    centres seeded per problem) solved by FP32-EigT FGMRES generate the training set (targets unit-RMS per
    sample), the CNN trains on the GPU with the library's BF16 kernels, and held-out 128^3 problems (seeds
    100000, ...) are solved to rtol 1e-8 from zero and from the prolonged, residual-scaled prediction (2000
    training solves, 20 epochs and 16 evaluation problems by default; --ws-samples / --ws-epochs / --ws-eval
    shorten it)."""
    from paper_2602_07711_amd import warmstart as W
    S = 64
    ws, rep = W.fit(size=S, samples=args.ws_samples, epochs=args.ws_epochs, batch=4, lr=1e-3, k0=60.0,
                    log=None)
    fwd, train = W.cnn_flops(S)
    step_ms = 1e3 * rep["train_s"] / max(1, rep["train_steps"])
    control = W.WarmStart(H.Cnn(S, 1, bf16=True, seed=999), 60.0, ws.t_scale)
    ev = W.evaluate(ws, 128, range(W.EVAL_SEED0, W.EVAL_SEED0 + args.ws_eval), control=control)
    m = ev["mean"]
    out = dict(train=dict(samples=rep["samples"], epochs=rep["epochs"], steps=rep["train_steps"], batch=4,
                          gen_s=rep["gen_s"], train_s=rep["train_s"], ms_per_step=round(step_ms, 3),
                          tflops=round(4 * train / (step_ms * 1e-3) / 1e12, 2), loss_first=rep["loss_first"],
                          loss_last=rep["loss_last"]),
               infer_ms=round(m["infer_ms"], 3), forward_gflop=round(fwd / 1e9, 2),
               eval_problems=args.ws_eval, iters_zero=m["zero_iters"], iters_warm=m["warm_iters"],
               iters_warm_trilinear=m.get("warm_linear_iters"), iters_untrained=m["control_iters"],
               e0_warm=round(m["warm_e0"], 4), e0_untrained=round(m["control_e0"], 4),
               r0_warm=round(m["warm_r0"], 4), iters_warm_residual_amplitude=m["other_amp_iters"],
               e0_warm_residual_amplitude=round(m["other_amp_e0"], 4),
               iters_warm_direction=m["dir_iters"], ms_fp32_learned_direction=round(m["dir_ms"], 3),
               ms_fp32_zero=round(m["zero_ms"], 3), ms_fp32_learned=round(m["warm_ms"], 3),
               ms_fp64_zero=round(m["fp64_ms"], 3))
    log(f"learned warm start: {out['iters_warm']} vs {out['iters_zero']} iterations (untrained "
        f"{out['iters_untrained']}), e0 {out['e0_warm']}, {out['ms_fp32_learned']} ms vs {out['ms_fp32_zero']} ms "
        f"(FP64 plain {out['ms_fp64_zero']} ms); training {out['train']['ms_per_step']} ms/step "
        f"({out['train']['tflops']} TFLOP/s)")
    return out


def bench_direct_sweep(H, torch, dev, sizes):
    """The paper's Table 2 workload: the preconditioner as a direct solver of the second-order system of the
    Sec. 5.1 test problem (u = phi(x) phi(y) phi(z), k0^2 = 439.2, staggered nodes, two-point absorbing closure).
    Per grid: setup time, the direct-solve time of EigT (FP64/FP32) and PFFT (FP64/FP32) on the solve
    stream (mean of 3 after one untimed call), and max-err / L2-err of the FP64 EigT solution against u; then the
    same for EigT and PFFT with the collocated three-point closure (EigT3, PFFT3) on the nodes j/(N-1)."""
    import math
    k0 = math.sqrt(439.2)
    rows = []
    for n in sizes:
        x = ((torch.arange(n, dtype=torch.float64, device=dev) + 0.5) / n).to(torch.complex128)
        e1, e2 = torch.exp(1j * k0 * x), torch.exp(-1j * k0 * (x - 1.0))
        ph, p2 = e1 + e2 - 2, -k0 * k0 * (e1 + e2)
        u = ph[:, None, None] * ph[None, :, None] * ph[None, None, :]
        f = p2[:, None, None] * ph[None, :, None] * ph[None, None, :]
        f += ph[:, None, None] * p2[None, :, None] * ph[None, None, :]
        f += ph[:, None, None] * ph[None, :, None] * p2[None, None, :]
        f += k0 * k0 * u
        k2 = torch.full((n, n, n), k0 * k0, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = H.helm_setup(k2, 1.0 / n, 2, "abc", k0, shape=(n, n, n))
        torch.cuda.synchronize()
        row = dict(n=n, setup_s=round(time.perf_counter() - t0, 3))
        del k2
        fv = f.reshape(-1)
        z = torch.empty_like(fv)
        for kind in ["eigt", "pfft"]:
            for fp32 in (False, True):
                H.helm_precond_apply(ctx, fv, z, kind=kind, fp32=fp32)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(3):
                    H.helm_precond_apply(ctx, fv, z, kind=kind, fp32=fp32)
                torch.cuda.synchronize()
                row[f"{kind}_{'fp32' if fp32 else 'fp64'}_ms"] = round((time.perf_counter() - t0) / 3 * 1e3, 3)
                if kind == "eigt" and not fp32:
                    d = z.view(n, n, n) - u
                    row["max_err"] = float(d.abs().max())
                    row["l2_err"] = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(u))
                    del d
        # the collocated three-point closure (EigT3): the same test problem on the nodes j/(N-1), j = 0..N-1
        xc = (torch.arange(n, dtype=torch.float64, device=dev) / (n - 1)).to(torch.complex128)
        e1, e2 = torch.exp(1j * k0 * xc), torch.exp(-1j * k0 * (xc - 1.0))
        ph, p2 = e1 + e2 - 2, -k0 * k0 * (e1 + e2)
        u.copy_(ph[:, None, None] * ph[None, :, None] * ph[None, None, :])
        f.copy_(p2[:, None, None] * ph[None, :, None] * ph[None, None, :])
        f += ph[:, None, None] * p2[None, :, None] * ph[None, None, :]
        f += ph[:, None, None] * ph[None, :, None] * p2[None, None, :]
        f += k0 * k0 * u
        H.helm_destroy(ctx)
        k2 = torch.full((n, n, n), k0 * k0, dtype=torch.float64, device=dev)
        ctx = H.helm_setup(k2, 1.0 / (n - 1), 2, "abc3", k0, shape=(n, n, n))
        del k2
        for kind in ["eigt", "pfft"]:
            for fp32 in (False, True):
                H.helm_precond_apply(ctx, fv, z, kind=kind, fp32=fp32)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(3):
                    H.helm_precond_apply(ctx, fv, z, kind=kind, fp32=fp32)
                torch.cuda.synchronize()
                row[f"{kind}3_{'fp32' if fp32 else 'fp64'}_ms"] = round((time.perf_counter() - t0) / 3 * 1e3, 3)
                if not fp32:
                    d = z.view(n, n, n) - u
                    row[f"{kind}3_max_err"] = float(d.abs().max())
                    row[f"{kind}3_l2_err"] = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(u))
                    del d
        log(f"direct solve {n}^3: {row}")
        rows.append(row)
        H.helm_destroy(ctx)
        del u, f, fv, z
        torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="grid points per axis (256 is the benchmark workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="fp32_eigt_fgmres,fp64_eigt_gmres,fp32_pfft_fgmres,fp64_pfft_gmres")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched workloads")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-warm-start leg")
    ap.add_argument("--ws-samples", type=int, default=2000, help="training solves of the learned leg")
    ap.add_argument("--ws-epochs", type=int, default=20, help="training epochs of the learned leg")
    ap.add_argument("--ws-eval", type=int, default=16, help="held-out 128^3 problems of the learned leg")
    ap.add_argument("--direct-sweep", default=None,
                    help="comma-separated grid sizes: also time the preconditioner as a direct solver of the paper's "
                         "second-order test problem (Table 2 workload), e.g. 100,127,200,255,400,511,600,767,800")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run three plain 256 MiB device-to-device copies (reference dispatches for scaling "
                         "hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): this solver has no multi-GPU path; "
              "the z-slab decomposition is a design note, not code.", file=sys.stderr)
        sys.exit(2)
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import torch

    import paper_2602_07711_amd as H
    import synth

    n = args.n
    log(f"generating the {n}^3 filtered-noise medium")
    w = synth.workload("noise", n=n)
    hh, k0 = w["h"], w["k0"]
    if n != 256:
        k0 = 120.0 * (n + 1) / 257.0
        w = dict(w, k0=k0, k2=synth.filtered_noise_k2(n, k0))
    dev = torch.device("cuda:0")
    k2 = torch.from_numpy(w["k2"]).to(dev)
    f = torch.from_numpy(w["f"]).to(dev)
    t0 = time.perf_counter()
    ctx = H.helm_setup(k2, hh, 6, k0=k0)
    F = H.helm_rhs(ctx, f)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    log(f"setup {t_setup:.3f} s")
    tune = None
    if not args.no_autotune:
        tune = H.helm_autotune(ctx, reps=5)
        log("autotuned transform tiles (forward / inverse): "
            + ", ".join(f"{k}={v['chosen']}/{v['chosen_inverse']}" for k, v in tune.items()))
    del k2, f
    x = torch.empty_like(F)
    unknowns = n ** 3
    if args.copy_calib:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)   # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    forms_def = {
        "fp32_eigt_fgmres": dict(m=50, flexible=True, prec_fp32=True, prec="eigt"),
        "fp64_eigt_gmres": dict(m=50, flexible=False, prec_fp32=False, prec="eigt"),
        "fp64_eigt_fgmres": dict(m=50, flexible=True, prec_fp32=False, prec="eigt"),
        "fp32_pfft_fgmres": dict(m=50, flexible=True, prec_fp32=True, prec="pfft"),
        "fp64_pfft_gmres": dict(m=50, flexible=False, prec_fp32=False, prec="pfft"),
        # the Dirichlet comparison preconditioner FFT2 (not in the default set)
        "fp32_fft2_fgmres": dict(m=50, flexible=True, prec_fp32=True, prec="fft2", maxit=1000, raise_on_noconv=False),
        "fp64_fft2_gmres": dict(m=50, flexible=False, prec_fp32=False, prec="fft2", maxit=1000,
                                raise_on_noconv=False),
    }
    forms = {}
    for name in args.forms.split(","):
        kw = forms_def[name]
        for _ in range(args.warmup):
            H.helm_gmres_solve(ctx, F, x, rtol=1e-8, x0_given=False, **kw)
        torch.cuda.synchronize()
        H.helm_profile_enable(ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for _ in range(args.steps):
            _, info = H.helm_gmres_solve(ctx, F, x, rtol=1e-8, x0_given=False, **kw)
            infos.append(info)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = H.helm_profile_read(ctx)
        H.helm_profile_enable(ctx, False)
        iters = sum(i["iters"] for i in infos)
        forms[name] = dict(ms_per_solve=round(1e3 * dt / args.steps, 3), iters=infos[-1]["iters"],
                           reorths=infos[-1]["reorths"],
                           unknowns_iters_per_s=unknowns * iters / dt, relres_true=infos[-1]["relres_true"],
                           converged=all(i["converged"] for i in infos),
                           phase_ms=dict((k, round(v, 3)) for k, v in infos[-1]["t_ms"].items()),
                           kernels=kernel_table(prof, fp32=kw["prec_fp32"]))
        log(f"{name}: {forms[name]['ms_per_solve']} ms/solve, {forms[name]['iters']} iterations, "
            f"{forms[name]['unknowns_iters_per_s']:.3e} unknowns*it/s")
    head = "fp32_eigt_fgmres" if "fp32_eigt_fgmres" in forms else next(iter(forms))
    hf = forms[head]
    dom = max(hf["kernels"].items(), key=lambda kv: kv[1]["total_ms"])
    dname, dk = dom
    traffic = measured_traffic(dname) if (head == "fp32_eigt_fgmres" and n == 256) else None
    roofline = dict(kernel=dname, bound=dk["bound"], achieved=dk["achieved"], peak=dk["peak"], unit=dk["unit"],
                    frac=dk["frac"], traffic=traffic,
                    algorithmic_bytes_per_launch=dk["work_per_launch"] if dk["bound"] == "hbm" else None,
                    note="achieved = algorithmic work per launch / average launch time (HIP events on the solve "
                         "stream over the timed region); traffic = HBM bytes per launch from rocprofv3 FETCH_SIZE "
                         "and WRITE_SIZE (scaled by a plain copy) in profiles/noise256_fp32_eigt_fgmres_hbm_traffic.md")
    batched = None
    if not args.no_batched:
        del x
        torch.cuda.empty_cache()
        batched = bench_batched(H, torch, dev, args)
    learned = None
    if not args.no_learned:
        torch.cuda.empty_cache()
        learned = bench_learned(H, torch, args)
    direct = None
    if args.direct_sweep:
        torch.cuda.empty_cache()
        direct = bench_direct_sweep(H, torch, dev, [int(v) for v in args.direct_sweep.split(",")])
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline()
        log(f"cpu oracle {cpu['value']:.3e} unknowns*it/s on {cpu['cores']} threads")
    speedup = None
    if "fp64_eigt_gmres" in forms and head != "fp64_eigt_gmres":
        speedup = forms["fp64_eigt_gmres"]["ms_per_solve"] / hf["ms_per_solve"]
    line = {
        "metric": "time-to-solution & unknowns·iters/s at 256^3, rtol 1e-8: FP32/learned vs FP64 EigT",
        "value": hf["unknowns_iters_per_s"],
        "unit": "unknowns*iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hf["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 outer, f32 preconditioner" if head == "fp32_eigt_fgmres" else "f64",
        "data": "synthetic",
        "config": {"workload": (f"filtered-noise medium {n}^3: 6th-order compact 27-point Helmholtz, k0={k0:g} "
                                f"(k0 h = {k0 * hh:.3f}), 0.2 x Gaussian-filtered (8 cells) seeded noise, "
                                "Gaussian point source, two-point absorbing closure; FGMRES(50) + EigT "
                                "complex-FP32 preconditioner, rtol 1e-8, x0 = 0"),
                   "n": n, "order": 6, "restart": 50, "rtol": 1e-8, "form": head},
        "time_to_solution_ms": hf["ms_per_solve"],
        "speedup_vs_fp64_eigt": round(speedup, 3) if speedup else None,
        "setup_s": round(t_setup, 3),
        "forms": forms,
        "gemm_autotune": tune,
        "batched": batched,
        "learned_warm_start": learned,
        "direct_sweep": direct,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
