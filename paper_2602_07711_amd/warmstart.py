"""Learned warm start for the compact-Helmholtz FGMRES: data generation with the solver, GPU training of the
encoder-decoder CNN (helm_cnn_* in include/helm.h), and inference as the initial guess x0.

The paper's runs start from U^0 = 0 (Sec. 4); here a network predicts U^0 from (contrast, source) on a coarse
S^3 grid, the prediction is prolonged trilinearly to the solver's grid, and FGMRES runs from it to the same
tolerance relative to ||F||. Every arithmetic step runs in libhelm's kernels: the features, the network, the
prolongation and the solve; this module orders the calls and reshapes training data.

Training data: `count` seeded problems of the four-inclusion family on S^3 (inclusion centres and the source
centre, U[0.3, 0.7]^3, seeded per sample; k0; a unit-peak Gaussian source of fixed physical width), solved by
FP32-EigT FGMRES. Each target is normalised per sample by its source's L2 norm (the solution is linear in the
source, so the factor is known at inference and undone exactly), times one constant of the training set that gives
the targets unit RMS. Optionally (amplitude="residual") the prolonged prediction is instead scaled by the complex
factor that minimises ||F - alpha A x0|| (helm_scale_guess), which guarantees ||F - A x0|| <= ||F||; the residual
weights the prediction's high-frequency error by 1/h^2, so that factor is biased towards 0 and the source-norm
amplitude is the default.

Usage (GPU):  python -m paper_2602_07711_amd.warmstart --samples 2000 --size 64 --epochs 20 --eval-n 128
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

from . import helm as H

C_SCALE = 1.0 / 0.3      # contrast amplitude of the inclusion family -> O(1) input
EVAL_SEED0 = 100_000     # held-out evaluation problems: seeds 100000, 100001, ... (training uses 0 .. count-1)
F_SCALE = 1.0            # sources are unit-peak Gaussians


def _problem(n, seed, k0, sigma):
    import synth
    return synth.warmstart_problem(n, seed, k0=k0, sigma=sigma)


def _solve(prob, rtol, m=30, x0=None, fp32=True):
    dev = torch.device("cuda")
    k2 = torch.from_numpy(prob["k2"]).to(dev)
    f = torch.from_numpy(prob["f"]).to(dev)
    ctx = H.helm_setup(k2, prob["h"], prob["order"], "abc", prob["k0"])
    F = H.helm_rhs(ctx, f)
    x, info = H.helm_gmres_solve(ctx, F, x0, m=m, rtol=rtol, flexible=fp32, prec_fp32=fp32,
                                 x0_given=x0 is not None)
    return ctx, k2, f, F, x, info


def source_norm(f_halo: np.ndarray) -> float:
    """Continuum L2 norm sqrt(h^3 sum |f|^2) of a source over the interior nodes of its (n+4)^3 halo array
    (h = 1/(n+1)); grids of different n give the same value up to O(h^2) for a smooth source."""
    n = f_halo.shape[0] - 4
    fi = f_halo[2:-2, 2:-2, 2:-2]
    return float(math.sqrt(np.vdot(fi, fi).real / (n + 1) ** 3))


def generate(net: H.Cnn, count: int, seed0: int = 0, k0: float = 60.0, sigma: float = 0.03, rtol: float = 1e-7,
             log=None):
    """Solve `count` problems on the network's S^3 grid. Returns (X [count,2,S^3], U [count,2,S^3]) float32 on
    the GPU (U: Re, Im of each solution divided by its source's L2 norm) and the summed solver iterations."""
    S = net.size
    V = S ** 3
    X = torch.empty(count, 2, V, dtype=torch.float32, device="cuda")
    U = torch.empty(count, 2, V, dtype=torch.float32, device="cuda")
    iters = 0
    t0 = time.time()
    for i in range(count):
        prob = _problem(S, seed0 + i, k0, sigma)
        ctx, k2, f, F, x, info = _solve(prob, rtol)
        iters += info["iters"]
        net.features(k2.reshape(-1), f.reshape(-1), k0, C_SCALE, F_SCALE, out=X[i:i + 1])
        U[i] = (torch.view_as_real(x).t() / source_norm(prob["f"])).to(torch.float32)   # layout [Re..., Im...]
        H.helm_destroy(ctx)
        if log and (i + 1) % max(1, count // 10) == 0:
            log(f"generated {i + 1}/{count} ({time.time() - t0:.1f} s, {iters / (i + 1):.1f} it/solve)")
    return X, U, iters


def train(net: H.Cnn, X, T, epochs: int, batch: int, lr: float, seed: int = 0, log=None):
    """Adam with cosine decay from lr to lr/100 over all steps; shuffled mini-batches (seeded). Returns the
    mean loss of each epoch."""
    n = X.shape[0]
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    rng = np.random.default_rng(seed)
    xb = torch.empty(batch, *X.shape[1:], dtype=torch.float32, device="cuda")
    tb = torch.empty_like(xb)
    hist = []
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        acc = 0.0
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            torch.index_select(X, 0, idx, out=xb)
            torch.index_select(T, 0, idx, out=tb)
            a = lr * (0.01 + 0.99 * 0.5 * (1 + math.cos(math.pi * step / max(1, total))))
            acc += net.train_step(xb, tb, a)
            step += 1
        hist.append(acc / max(1, steps_per_epoch))
        if log:
            log(f"epoch {ep + 1}/{epochs} loss {hist[-1]:.4e}")
    return hist


# (ci, co, taps, level) of the twelve convolutions, as in the network of include/helm.h
_CONVS = [(2, 16, 27, 0), (16, 16, 27, 0), (16, 32, 27, 1), (32, 32, 27, 1), (32, 64, 27, 2), (64, 64, 27, 2),
          (64, 64, 27, 3), (64, 64, 27, 3), (128, 64, 27, 2), (96, 32, 27, 1), (48, 16, 27, 0), (16, 2, 1, 0)]


def cnn_flops(size: int):
    """Algorithmic multiply-add flops (2 per MAC) of the convolutions per sample: (forward, training step =
    forward + weight gradient + data gradient of every layer but the first)."""
    fwd = sum(2 * ci * co * t * (size >> lv) ** 3 for ci, co, t, lv in _CONVS)
    dgrad = fwd - 2 * 2 * 16 * 27 * size ** 3
    return fwd, 2 * fwd + dgrad


class WarmStart:
    """A trained network; produces x0 for a solver problem. t_scale: the training set's target scale (targets =
    t_scale * u / source_norm(f)). amplitude: "source" (undo that normalisation) or "residual" (helm_scale_guess)."""

    def __init__(self, net: H.Cnn, k0: float, t_scale: float, cubic: bool = True, amplitude: str = "source"):
        if amplitude not in ("source", "residual"):
            raise ValueError("amplitude must be 'source' or 'residual'")
        self.net = net
        self.k0 = float(k0)
        self.t_scale = float(t_scale)
        self.cubic = bool(cubic)
        self.amplitude = amplitude
        self._x = torch.empty(1, 2, net.size ** 3, dtype=torch.float32, device="cuda")
        self._y = torch.empty_like(self._x)

    def initial_guess(self, ctx: H.Context, F: torch.Tensor, k2_halo: torch.Tensor, f_halo: torch.Tensor, nf: int,
                      f_norm: float, out=None) -> torch.Tensor:
        """Features -> network -> prolongation to nf^3 (complex128, cubic or trilinear) -> amplitude. f_norm is
        source_norm of the problem's source. Beyond the boundary nodes the coarse field follows the absorbing
        closure's ghost rule on the network grid, gamma = (2 + i k0 h_c)/(2 - i k0 h_c)."""
        self.net.features(k2_halo.reshape(-1), f_halo.reshape(-1), self.k0, C_SCALE, F_SCALE, out=self._x)
        self.net.forward(self._x, self._y)
        kh = self.k0 / (self.net.size + 1)
        gamma = (2 + 1j * kh) / (2 - 1j * kh)
        x0 = self.net.prolong(self._y[0], nf, scale=f_norm / self.t_scale, gamma=gamma, fine=out, cubic=self.cubic)
        if self.amplitude == "residual":
            H.helm_scale_guess(ctx, F, x0)
        return x0

    def save(self, path: str):
        meta = dict(size=self.net.size, bf16=self.net.bf16, k0=self.k0, t_scale=self.t_scale, c_scale=C_SCALE,
                    f_scale=F_SCALE, cubic=self.cubic)
        np.savez(path, params=self.net.params().numpy(), meta=np.frombuffer(json.dumps(meta).encode(), np.uint8))

    @staticmethod
    def load(path: str, max_batch: int = 1) -> "WarmStart":
        z = np.load(path, allow_pickle=False)
        meta = json.loads(z["meta"].tobytes().decode())
        net = H.Cnn(meta["size"], max_batch=max_batch, bf16=meta["bf16"])
        net.set_params(torch.from_numpy(z["params"]))
        return WarmStart(net, meta["k0"], meta["t_scale"], meta.get("cubic", True))


def fit(size: int, samples: int, epochs: int, batch: int = 4, lr: float = 1e-3, k0: float = 60.0,
        sigma: float = 0.03, seed0: int = 0, bf16: bool = True, log=None):
    """Generate data on the GPU with the solver, train, and return (WarmStart, report dict)."""
    net = H.Cnn(size, max_batch=batch, bf16=bf16, seed=seed0 + 12345)
    t0 = time.time()
    X, U, iters = generate(net, samples, seed0, k0, sigma, log=log)
    torch.cuda.synchronize()
    t_gen = time.time() - t0
    t_scale = 1.0 / float(torch.sqrt(torch.mean(U.double() ** 2)))
    T = U.mul_(t_scale)
    t0 = time.time()
    hist = train(net, X, T, epochs, batch, lr, seed=seed0, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    report = dict(samples=samples, size=size, epochs=epochs, batch=batch, lr=lr, bf16=bf16,
                  gen_s=round(t_gen, 2), gen_iters_per_solve=iters / max(1, samples), train_s=round(t_train, 2),
                  train_steps=epochs * (samples // batch), loss_first=hist[0], loss_last=hist[-1], t_scale=t_scale)
    del X, T
    return WarmStart(net, k0, t_scale), report


def evaluate(ws: WarmStart, nf: int, seeds, sigma: float = 0.03, rtol: float = 1e-8, m: int = 50,
             control: WarmStart | None = None, fp64_plain: bool = True):
    """Solve each held-out problem on nf^3 from zero and from the learned x0 (and from an untrained control
    network's x0, the trilinear prolongation, the residual-scaled amplitude and the prediction taken as the first
    FGMRES search direction instead of the initial iterate as variants). Reports iterations,
    time-to-solution (inference included), the guesses' relative errors e0 and residuals r0 (against the
    converged zero-start solution and ||F||) and the agreement of the solutions."""
    rows = []
    dev = torch.device("cuda")
    for sd in seeds:
        prob = _problem(nf, sd, ws.k0, sigma)
        k2 = torch.from_numpy(prob["k2"]).to(dev)
        f = torch.from_numpy(prob["f"]).to(dev)
        fn = source_norm(prob["f"])
        ctx = H.helm_setup(k2, prob["h"], prob["order"], "abc", prob["k0"])
        F = H.helm_rhs(ctx, f)
        nF = torch.linalg.vector_norm(F)
        row = dict(seed=sd)

        def timed(fn_):
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = fn_()
            torch.cuda.synchronize()
            return out, (time.perf_counter() - t) * 1e3

        # warm-up of every path once (first-call allocations), then timed runs
        H.helm_gmres_solve(ctx, F, None, m=m, rtol=rtol, flexible=True, prec_fp32=True)
        ws.initial_guess(ctx, F, k2, f, nf, fn)
        (x_zero, i_zero), t_zero = timed(lambda: H.helm_gmres_solve(ctx, F, None, m=m, rtol=rtol, flexible=True,
                                                                    prec_fp32=True))
        nx = torch.linalg.vector_norm(x_zero)
        x0 = torch.empty_like(F)

        def warm(w):
            w.initial_guess(ctx, F, k2, f, nf, fn, out=x0)
            return H.helm_gmres_solve(ctx, F, x0, m=m, rtol=rtol, flexible=True, prec_fp32=True, x0_given=True)

        def quality():
            r0 = F - H.helm_matvec(ctx, x0)
            return (float(torch.linalg.vector_norm(x0 - x_zero) / nx), float(torch.linalg.vector_norm(r0) / nF))

        def direction(w):
            w.initial_guess(ctx, F, k2, f, nf, fn, out=x0)
            return H.helm_gmres_solve(ctx, F, x0, m=m, rtol=rtol, flexible=True, prec_fp32=True, x0_given=2)

        (x_warm, i_warm), t_warm = timed(lambda: warm(ws))
        (x_dir, i_dir), t_dir = timed(lambda: direction(ws))
        row.update(dir_iters=i_dir["iters"], dir_ms=t_dir,
                   dir_rel_diff=float(torch.linalg.vector_norm(x_dir - x_zero) / nx))
        rel_diff = float(torch.linalg.vector_norm(x_warm - x_zero) / nx)
        _, t_inf = timed(lambda: ws.initial_guess(ctx, F, k2, f, nf, fn, out=x0))     # x0 is the guess again
        e0, r0 = quality()
        row.update(zero_iters=i_zero["iters"], warm_iters=i_warm["iters"], zero_ms=t_zero, warm_ms=t_warm,
                   infer_ms=t_inf, warm_e0=e0, warm_r0=r0, warm_relres=i_warm["relres_true"], rel_diff=rel_diff)
        if control is not None:
            control.initial_guess(ctx, F, k2, f, nf, fn, out=x0)
            e0, r0 = quality()
            (_, i_c), t_c = timed(lambda: warm(control))
            row.update(control_e0=e0, control_r0=r0, control_iters=i_c["iters"], control_ms=t_c)
        if ws.cubic:
            ws.cubic = False
            (_, i_l), t_l = timed(lambda: warm(ws))
            ws.cubic = True
            row.update(warm_linear_iters=i_l["iters"], warm_linear_ms=t_l)
        amp = ws.amplitude
        ws.amplitude = "residual" if amp == "source" else "source"
        ws.initial_guess(ctx, F, k2, f, nf, fn, out=x0)
        e0, r0 = quality()
        (_, i_a), t_a = timed(lambda: warm(ws))
        ws.amplitude = amp
        row.update(other_amp_e0=e0, other_amp_r0=r0, other_amp_iters=i_a["iters"], other_amp_ms=t_a)
        if fp64_plain:
            H.helm_gmres_solve(ctx, F, None, m=m, rtol=rtol)
            (_, i_64), t_64 = timed(lambda: H.helm_gmres_solve(ctx, F, None, m=m, rtol=rtol))
            row.update(fp64_iters=i_64["iters"], fp64_ms=t_64)
        H.helm_destroy(ctx)
        rows.append(row)
    keys = [k for k in rows[0] if k != "seed"]
    mean = {k: float(np.mean([r[k] for r in rows])) for k in keys}
    return dict(rows=rows, mean=mean)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--samples", type=int, default=2000)
    ap.add_argument("--size", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--k0", type=float, default=60.0)
    ap.add_argument("--fp32", action="store_true", help="FP32 MFMA operands instead of BF16")
    ap.add_argument("--eval-n", type=int, default=128)
    ap.add_argument("--eval-count", type=int, default=16)
    ap.add_argument("--save", default=None)
    ap.add_argument("--json", default=None)
    a = ap.parse_args()
    log = lambda s: print(s, flush=True)
    ws, rep = fit(a.size, a.samples, a.epochs, a.batch, a.lr, a.k0, bf16=not a.fp32, log=log)
    log(json.dumps(rep))
    if a.save:
        ws.save(a.save)
    control = WarmStart(H.Cnn(a.size, 1, bf16=not a.fp32, seed=999), a.k0, ws.t_scale)
    ev = evaluate(ws, a.eval_n, range(EVAL_SEED0, EVAL_SEED0 + a.eval_count), control=control)
    out = dict(train=rep, eval=ev)
    log(json.dumps(ev["mean"]))
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
