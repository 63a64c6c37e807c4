"""Seeded media and sources on the unit cube.

Grid convention: N unknowns per axis at x_i = i*h, h = 1/(N+1), i = 1..N. The ghost nodes x_0 = 0 and
x_{N+1} = 1 sit one cell outside, so the absorbing boundary lies half a cell from the first and last node (the
staggered two-point placement of Sec. 2.3). Every field here is sampled on the interior plus a two-cell halo,
i.e. on i = -1..N+2, which gives arrays of shape (N+4, N+4, N+4) in (z, y, x) order, x fastest.

All generators use numpy's PCG64 (`default_rng(seed)`) in float64.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

HALO = 2


def halo_coords(n: int) -> np.ndarray:
    """Node coordinates i*h for i = -1..N+2 (length N+4), h = 1/(N+1)."""
    h = 1.0 / (n + 1)
    return (np.arange(n + 2 * HALO) - (HALO - 1)) * h


def _mesh(n: int):
    c = halo_coords(n)
    z = c[:, None, None]
    y = c[None, :, None]
    x = c[None, None, :]
    return x, y, z


def gaussian_source(n: int, sigma_cells: float = 2.0, center=(0.5, 0.5, 0.5)) -> np.ndarray:
    """f = exp(-|x-c|^2 / (2 sigma^2)), sigma = sigma_cells*h, complex128 on the halo grid."""
    h = 1.0 / (n + 1)
    s = sigma_cells * h
    x, y, z = _mesh(n)
    r2 = (x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2
    return np.exp(-r2 / (2 * s * s)).astype(np.complex128)


def inclusions_k2(n: int, k0: float, amp: float = 0.3, n_inc: int = 4, width: float = 0.1,
                  seed: int = 2, lo: float = 0.2, hi: float = 0.8) -> np.ndarray:
    """k^2 = k0^2 (1 + amp * sum_m exp(-|x-c_m|^2/(2 width^2))), c_m ~ U[lo,hi]^3 (seeded)."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(lo, hi, size=(n_inc, 3))
    x, y, z = _mesh(n)
    bump = np.zeros((n + 4,) * 3)
    for c in centers:
        bump += np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * width * width))
    return k0 * k0 * (1.0 + amp * bump)


def filtered_noise_k2(n: int, k0: float, amp: float = 0.2, sigma_cells: float = 8.0, seed: int = 3,
                      pad: int = 32) -> np.ndarray:
    """k^2 = k0^2 (1 + amp * w), w = Gaussian-filtered U(-1,1) noise normalised to max|w| = 1 inside.

    The noise lives on the halo grid padded by `pad` cells per side, is filtered by a separable Gaussian of
    width sigma_cells (truncated at 4 sigma), then cropped to the (N+4)^3 halo box.
    """
    rng = np.random.default_rng(seed)
    m = n + 2 * HALO + 2 * pad
    w = rng.uniform(-1.0, 1.0, size=(m, m, m))
    for ax in range(3):
        w = ndimage.gaussian_filter1d(w, sigma=sigma_cells, axis=ax, truncate=4.0, mode="constant")
    w = w[pad:pad + n + 4, pad:pad + n + 4, pad:pad + n + 4]
    inner = w[HALO:-HALO, HALO:-HALO, HALO:-HALO]
    w = w / np.abs(inner).max()
    return k0 * k0 * (1.0 + amp * w)


def unit_directions(count: int, seed: int = 4) -> np.ndarray:
    """count directions d = g/|g|, g ~ N(0, I_3)."""
    g = np.random.default_rng(seed).standard_normal((count, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def plane_wave_sources(k2: np.ndarray, k0: float, dirs: np.ndarray) -> np.ndarray:
    """Scattering sources f_m = -(k^2 - k0^2) exp(i k0 d_m . x) for each incident direction (Sec. 5.1.4).

    Returns shape (len(dirs), N+4, N+4, N+4) complex128 on the halo grid.
    """
    n = k2.shape[0] - 2 * HALO
    x, y, z = _mesh(n)
    out = np.empty((len(dirs),) + k2.shape, np.complex128)
    contrast = -(k2 - k0 * k0)
    for m, d in enumerate(dirs):
        out[m] = contrast * np.exp(1j * k0 * (d[0] * x + d[1] * y + d[2] * z))
    return out


def uneven_problem_set(count: int = 16, n_lo: int = 64, n_hi: int = 160, k_lo: float = 30.0,
                       k_hi: float = 90.0, seed: int = 40):
    """Sizes N_p = round(n_lo + (n_hi-n_lo) p/(count-1)) and wavenumbers k0_p ~ U[k_lo, k_hi]."""
    ks = np.random.default_rng(seed).uniform(k_lo, k_hi, size=count)
    ns = [int(round(n_lo + (n_hi - n_lo) * p / (count - 1))) for p in range(count)]
    return list(zip(ns, ks.tolist()))


def warmstart_problem(n: int, seed: int, k0: float = 60.0, sigma: float = 0.03, center=None):
    """Learned-warm-start sample: the four-inclusion medium (centres seeded by `seed`, amplitude 0.3, width 0.1)
    with a unit-peak Gaussian source of fixed physical width `sigma` whose centre is drawn from U[0.3, 0.7]^3 by a
    second stream of the same seed (or given), 6th order. The width does not scale with h, so grids of different
    N discretise the same continuous problem."""
    if center is None:
        center = np.random.default_rng((seed, 77)).uniform(0.3, 0.7, size=3)
    return dict(n=n, h=1.0 / (n + 1), order=6, k0=k0, k2=inclusions_k2(n, k0, seed=seed),
                f=gaussian_source(n, sigma_cells=sigma * (n + 1), center=tuple(center)), center=tuple(center))


def staggered_coords(n: int) -> np.ndarray:
    """Staggered node coordinates (j + 1/2) h, h = 1/N, for j = -2..N+1 (length N+4): the grid of the
    scattering experiment of Sec. 5.1 (the boundary lies half a cell outside the first and last nodes)."""
    return (np.arange(n + 4) - 2 + 0.5) / n


def single_inclusion_problem(n: int, k2_in: complex = 1050 + 2.26j, k0sq: float = 439.2,
                             center=(0.5, 0.5, 0.7), radius: float = 0.1):
    """The single-inclusion scattering problem of Sec. 5.1 on the staggered N^3 grid (h = 1/N): k^2 = k2_in
    inside the sphere |x - c| <= r, k0^2 outside (sampled at the nodes, no smoothing), and the scattered-field
    source f = -(k^2 - k0^2) exp(i k0 z) of the incident plane wave exp(i k0 z). Returns dict(n, h, k0, k2, f)
    with complex128 k2 and f on the halo grid."""
    c = staggered_coords(n)
    z, y, x = c[:, None, None], c[None, :, None], c[None, None, :]
    inside = (x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2 <= radius * radius
    k2 = np.where(inside, complex(k2_in), complex(k0sq)).astype(np.complex128)
    k0 = float(np.sqrt(k0sq))
    f = (-(k2 - k0sq) * np.exp(1j * k0 * z)).astype(np.complex128)
    return dict(n=n, h=1.0 / n, k0=k0, k2=k2, f=f)


def paper_test_problem(n: int, k0sq: float = 439.2):
    """The 3D test problem of Sec. 5.1 on the staggered N^3 grid (h = 1/N): u = phi(x) phi(y) phi(z) with
    phi(t) = exp(i k0 t) + exp(-i k0 (t - 1)) - 2 (it satisfies the absorbing condition on every face),
    f = Delta u + k0^2 u in closed form, constant k^2 = k0^2. Returns dict(n, h, k0, k2, f, u) on the halo grid
    (u also on the halo grid)."""
    k0 = float(np.sqrt(k0sq))
    c = staggered_coords(n)
    e1, e2 = np.exp(1j * k0 * c), np.exp(-1j * k0 * (c - 1.0))
    ph, p2 = e1 + e2 - 2.0, -k0sq * (e1 + e2)
    Z, Y, X = (slice(None), None, None), (None, slice(None), None), (None, None, slice(None))
    u = ph[Z] * ph[Y] * ph[X]
    f = p2[Z] * ph[Y] * ph[X] + ph[Z] * p2[Y] * ph[X] + ph[Z] * ph[Y] * p2[X] + k0sq * u
    return dict(n=n, h=1.0 / n, k0=k0, k2=np.full(u.shape, k0sq), f=f.astype(np.complex128),
                u=u.astype(np.complex128))


def workload(name: str, n: int | None = None):
    """The named synthetic workloads. Returns dict(n, h, order, k0, k2 (halo), f (halo), m, ...).

    * "gauss32":     N=32, 4th order, constant k=20, Gaussian source, restart 30.
    * "inclusions":  N=128 (default), 6th order, k0=60, four Gaussian inclusions (seed 2), restart 50.
    * "noise":       N=256 (default), 6th order, k0=120, 0.2 x filtered noise (seed 3), restart 50.
    """
    if name == "gauss32":
        n = n or 32
        k0 = 20.0
        k2 = np.full((n + 4,) * 3, k0 * k0)
        return dict(n=n, h=1.0 / (n + 1), order=4, k0=k0, k2=k2, f=gaussian_source(n), m=30)
    if name == "inclusions":
        n = n or 128
        k0 = 60.0
        return dict(n=n, h=1.0 / (n + 1), order=6, k0=k0, k2=inclusions_k2(n, k0), f=gaussian_source(n), m=50)
    if name == "noise":
        n = n or 256
        k0 = 120.0
        return dict(n=n, h=1.0 / (n + 1), order=6, k0=k0, k2=filtered_noise_k2(n, k0), f=gaussian_source(n),
                    m=50)
    raise KeyError(name)
