"""The paper's Table 6 on the GPU: the single-inclusion scattering problem of Sec. 5.1 (k^2 = 1050 + 2.26i in a
sphere of radius 0.1 at (0.5, 0.5, 0.7), k0^2 = 439.2, f = -(k^2 - k0^2) exp(i k0 z), staggered N^3 grid,
sixth-order scheme, two-point absorbing closure) solved by GMRES(50) with the EigT and the PFFT preconditioners
(every grid, 100^3 ... 511^3) to rel-res 1e-8. The iteration counts must be the ones
Table 6 prints for EigT2 / PFFT2 (+-1: the paper does not say how its sixth-order derivatives of k^2 treat the
jump at the sphere; here the sphere is sampled at the nodes and differenced like any medium). The FP32-EigT
FGMRES form is held to the same count +-2. Memory at 511^3: about 130 GB of device memory.

The FFT6 column (the sixth-order compact operator with constant k0 and Dirichlet closures as the preconditioner,
GMRES without restart, capped at 100 iterations as in the paper) is checked for N <= 400: the printed counts
(68, 72, 84, 93) within 3 iterations, and no convergence within the cap at 400^3.
"""
import json
import os

import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table6_scattering.json")


def _rows():
    with open(GOLDEN) as fh:
        return sorted(json.load(fh)["rows"])


@pytest.mark.parametrize("row", _rows(), ids=lambda r: f"N{r[0]}")
def test_table6_iterations(row):
    import paper_2602_07711_amd as H
    H.lib()
    n, n0_eig, n0_pfft = row[0], row[2], row[4]
    print(f"table6 N={n}", flush=True)
    w = synth.single_inclusion_problem(n)
    dev = torch.device("cuda")
    ctx = H.helm_setup(torch.from_numpy(w["k2"]).to(dev), w["h"], 6, k0=w["k0"])
    F = H.helm_rhs(ctx, torch.from_numpy(w["f"]).to(dev))
    del w
    x = torch.empty_like(F)
    forms = [("eigt", dict(prec="eigt"), n0_eig, 1), ("eigt_fp32", dict(prec="eigt", flexible=True, prec_fp32=True),
                                                     n0_eig, 2)]
    forms.append(("pfft", dict(prec="pfft"), n0_pfft, 1))
    for name, kw, n0, tol in forms:
        _, info = H.helm_gmres_solve(ctx, F, x, m=50, rtol=1e-8, x0_given=False, **kw)
        print(f"  {name}: {info['iters']} iterations (Table 6: {n0}), rel-res {info['relres_true']:.2e}, "
              f"{info['t_ms']['total']:.1f} ms", flush=True)
        assert info["converged"] and info["relres_true"] <= 1e-8
        assert abs(info["iters"] - n0) <= tol
    H.helm_destroy(ctx)
    del F, x
    torch.cuda.empty_cache()


@pytest.mark.parametrize("row", [r for r in _rows() if r[0] <= 400], ids=lambda r: f"N{r[0]}")
def test_table6_fft6_iterations(row):
    import paper_2602_07711_amd as H
    H.lib()
    n, n0 = row[0], row[6]
    print(f"table6 FFT6 N={n}", flush=True)
    w = synth.single_inclusion_problem(n)
    dev = torch.device("cuda")
    ctx = H.helm_setup(torch.from_numpy(w["k2"]).to(dev), w["h"], 6, k0=w["k0"])
    F = H.helm_rhs(ctx, torch.from_numpy(w["f"]).to(dev))
    del w
    x = torch.empty_like(F)
    _, info = H.helm_gmres_solve(ctx, F, x, m=100, maxit=100, rtol=1e-8, x0_given=False, prec="fft6",
                                 raise_on_noconv=False)
    print(f"  fft6: {info['iters']} iterations (Table 6: {n0}), rel-res {info['relres_true']:.2e}, "
          f"{info['t_ms']['total']:.1f} ms", flush=True)
    if n0 >= 100:
        assert not info["converged"] and info["iters"] == 100
    else:
        assert info["converged"] and info["relres_true"] <= 1e-8
        assert abs(info["iters"] - n0) <= 3
    H.helm_destroy(ctx)
    del F, x
    torch.cuda.empty_cache()
