"""The iteration comparison of the paper's Tables 3 and 4 on the GPU: the Sec. 5.1 test problem (u = phi(x) phi(y)
phi(z), k0^2 = 439.2, staggered N^3 grid, the two-point absorbing closure) with the fourth- and sixth-order compact
schemes, preconditioned by EigT (GMRES(50)) and by the Dirichlet FFT2 and FFT4 / FFT6 (GMRES(100), cap 100).

The paper's runs use collocated grids with high-order three-point closures it does not specify, so its errors are
not comparable (the staggered closure makes ours second order) and its counts are a reference, printed next to ours.
What is checked is what the paper concludes from them: EigT needs a handful of iterations and the count does not
grow with N (it falls to 3); the Dirichlet preconditioners need many times more, and more as N grows; raising their
order helps only marginally.
"""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table34_iterations.json")
SIZES = [50, 64, 100, 127, 200, 255, 400]


@pytest.mark.parametrize("order", [4, 6])
def test_tables34_iteration_comparison(order):
    import paper_2602_07711_amd as H
    H.lib()
    with open(GOLDEN) as fh:
        paper = {r[0]: r for r in json.load(fh)[f"order{order}"]}
    dev = torch.device("cuda")
    rows = []
    for n in SIZES:
        w = synth.paper_test_problem(n)
        ctx = H.helm_setup(torch.from_numpy(w["k2"]).to(dev), w["h"], order, k0=w["k0"])
        F = H.helm_rhs(ctx, torch.from_numpy(w["f"]).to(dev))
        del w
        x = torch.empty_like(F)
        it = {}
        for name, kw in [("eigt", dict(prec="eigt", m=50, maxit=200)), ("fft2", dict(prec="fft2", m=100, maxit=100)),
                         ("ffth", dict(prec=f"fft{order}", m=100, maxit=100))]:
            _, info = H.helm_gmres_solve(ctx, F, x, rtol=1e-8, x0_given=False, raise_on_noconv=False, **kw)
            assert info["converged"], (n, name, info["iters"], info["relres_true"])
            it[name] = info["iters"]
        p = paper.get(n) or paper.get(n - 1)
        print(f"order {order} N={n}: EigT {it['eigt']} (paper EigT3 {p[1]}), FFT2 {it['fft2']} ({p[3]}), "
              f"FFT{order} {it['ffth']} ({p[4]})", flush=True)
        rows.append((n, it))
        H.helm_destroy(ctx)
        del F, x
        torch.cuda.empty_cache()
    eig = [r[1]["eigt"] for r in rows]
    assert max(eig) <= 8 and eig[-1] == 3
    assert all(b <= a for a, b in zip(eig, eig[1:]))                       # non-increasing in N
    for n, it in rows:
        if n >= 100:
            assert it["fft2"] >= 8 * it["eigt"] and it["ffth"] >= 8 * it["eigt"]
            assert it["ffth"] >= 0.85 * it["fft2"]                         # the higher order helps only marginally
    fft = [r[1]["fft2"] for r in rows]
    assert fft[-1] > 2 * fft[0]                                             # the Dirichlet count grows with N


def test_table5_wavenumber_sweep():
    """The paper's Table 5: the test problem with k0 = k in {10, 20, 50, 100} on 100^3 ... 511^3, sixth order, the
    absorbing-closure preconditioner (EigT and PFFT, which must take the same number of iterations).
    Checked: every count at most the printed one (the preconditioner here carries exactly the operator's closure),
    counts non-increasing in N for every k and non-decreasing in k for every N."""
    import paper_2602_07711_amd as H
    H.lib()
    with open(os.path.join(os.path.dirname(__file__), "golden", "table5_wavenumbers.json")) as fh:
        g = json.load(fh)
    ks = g["k"]
    dev = torch.device("cuda")
    got = {}
    for row in g["rows"]:
        n = row[0]
        for k, n0 in zip(ks, row[1:]):
            w = synth.paper_test_problem(n, k0sq=float(k * k))
            ctx = H.helm_setup(torch.from_numpy(w["k2"]).to(dev), w["h"], 6, k0=w["k0"])
            F = H.helm_rhs(ctx, torch.from_numpy(w["f"]).to(dev))
            del w
            x = torch.empty_like(F)
            its = []
            for prec in ["eigt", "pfft"]:
                _, info = H.helm_gmres_solve(ctx, F, x, m=50, maxit=300, rtol=1e-8, x0_given=False, prec=prec)
                its.append(info["iters"])
            print(f"table5 N={n} k={k}: {its} (paper {n0})", flush=True)
            assert len(set(its)) == 1 and its[0] <= n0
            got[(n, k)] = its[0]
            H.helm_destroy(ctx)
            del F, x
            torch.cuda.empty_cache()
    ns = [r[0] for r in g["rows"]]
    for k in ks:
        assert all(got[(b, k)] <= got[(a, k)] for a, b in zip(ns, ns[1:]))
    for n in ns:
        assert all(got[(n, b)] >= got[(n, a)] for a, b in zip(ks, ks[1:]))
