"""The learned warm start end to end on the GPU: solver-generated data, training with the library's own
forward/backward/Adam kernels, and what the trained network gains over the method without it.

Small configuration so the test runs in seconds: 400 training problems on 32^3 (k0 = 30, so k0 h = 0.91 as on
64^3 with k0 = 60; inclusion and source centres seeded per problem), evaluation on held-out 64^3 media. Targets
are unit-RMS per sample and the prolonged prediction is scaled by the residual-minimising amplitude. What the
network gains is measured directly: the relative error of its scaled prediction against the converged solution
must fall well below that of an untrained network of the same architecture put through the same scaling (whose
best multiple of its output still misses the field almost entirely), and the initial residual below ||F||
(the scaling guarantees <= ||F||). EigT-preconditioned FGMRES reduces the residual by a factor 3-5 per iteration here, so a guess
accurate to 5-10 % is worth at most about one iteration: the test bounds the iteration change by one on average
(the full-size iteration and time effect at 128^3 is measured by the benchmark). No gain over the zero guess is
achieved or asserted: at 128^3 the trained network saves 0.3 iterations and its 0.6 ms of inference make the solve
slower, and the prediction as an extra search direction saves none (every variant's measured ceiling is recorded with
the network's design). The solver decides the answer: every run converges to rtol 1e-8 relative to ||F||, so the warm-started and zero-started
solutions agree to that level whatever the network predicts.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_learned_warm_start_gains_over_untrained_and_zero_guess():
    from paper_2602_07711_amd import helm as H
    from paper_2602_07711_amd import warmstart as W
    print("warm start: fit 32^3", flush=True)
    ws, rep = W.fit(size=32, samples=400, epochs=8, batch=4, lr=2e-3, k0=30.0, sigma=0.06, seed0=0)
    print(rep, flush=True)
    assert rep["loss_last"] < 0.1 * rep["loss_first"]
    control = W.WarmStart(H.Cnn(32, 1, bf16=True, seed=999), 30.0, ws.t_scale)
    print("warm start: evaluate 64^3", flush=True)
    ev = W.evaluate(ws, 64, range(W.EVAL_SEED0, W.EVAL_SEED0 + 4), sigma=0.06, control=control, fp64_plain=False)
    for r in ev["rows"]:
        print({k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}, flush=True)
        assert r["warm_relres"] <= 1e-8 * 1.0001
        assert r["rel_diff"] < 1e-6
        assert r["warm_e0"] < 0.25 * r["control_e0"]
        assert r["warm_r0"] < 1.0
        assert r["other_amp_r0"] <= 1.0 + 1e-12      # the residual-minimising amplitude never raises ||r0||
    m = ev["mean"]
    print(m, flush=True)
    assert m["warm_e0"] < 0.15
    assert m["control_e0"] > 0.7
    assert abs(m["warm_iters"] - m["zero_iters"]) <= 1.0, m
