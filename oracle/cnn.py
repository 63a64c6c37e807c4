"""CPU FP64 oracle of the warm-start encoder-decoder CNN (torch CPU ops with autograd).

TEST INFRASTRUCTURE ONLY (see the package docstring). The network is not part of the paper: it is the learned
initial-guess extension of its GMRES (the paper's runs start from U^0 = 0, Sec. 4), defined here from its
description:
  * 4 levels with 16/32/64/64 channels on S, S/2, S/4, S/8 grids; two 3x3x3 convolutions (bias, ReLU) per
    encoder level, 2x average pooling between levels;
  * decoder: nearest 2x upsampling, concatenation [upsampled | skip], one 3x3x3 convolution (bias, ReLU) per
    level, then a linear 1x1x1 head to 2 channels (Re u, Im u);
  * zero-padded cross-correlation, tap index 9 (dz+1) + 3 (dy+1) + (dx+1), volumes [z][y][x];
  * parameters: one flat array, per layer W[co][ci][tap] then b[co];
  * training: mean-squared error, Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
The library routines used as steps are torch's conv3d, avg_pool3d, nearest interpolation and autograd.
Pins (tests/test_oracle_cnn_pins.py): conv3d against a brute-force loop, the whole network against an
independent numpy evaluation (shifted slices, reshaped means, repeats), the gradient against central finite
differences, Adam against its closed form for a constant gradient, prolongation and feature sampling exact on
trilinear fields and nested grids.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as Fn

# (ci, co, taps, relu) of the twelve convolutions in execution order
LAYERS = [
    (2, 16, 27, True), (16, 16, 27, True),
    (16, 32, 27, True), (32, 32, 27, True),
    (32, 64, 27, True), (64, 64, 27, True),
    (64, 64, 27, True), (64, 64, 27, True),
    (128, 64, 27, True), (96, 32, 27, True), (48, 16, 27, True),
    (16, 2, 1, False),
]


def num_params() -> int:
    return sum(co * ci * t + co for ci, co, t, _ in LAYERS)


def unpack(params) -> list:
    """Split the flat parameter array into (W [co, ci, k, k, k], b [co]) float64 tensors."""
    p = torch.as_tensor(np.asarray(params, dtype=np.float64))
    out, off = [], 0
    for ci, co, taps, _ in LAYERS:
        k = 3 if taps == 27 else 1
        W = p[off:off + co * ci * taps].reshape(co, ci, k, k, k)
        off += co * ci * taps
        b = p[off:off + co]
        off += co
        out.append((W, b))
    assert off == p.numel()
    return out


def _conv(x, W, b, relu):
    y = Fn.conv3d(x, W, b, padding=W.shape[-1] // 2)
    return torch.relu(y) if relu else y


def forward_layers(layers, x):
    """x: [B, 2, S, S, S] float64 tensor -> [B, 2, S, S, S]."""
    L = layers
    c = lambda i, t: _conv(t, L[i][0], L[i][1], LAYERS[i][3])
    s1 = c(1, c(0, x))
    s2 = c(3, c(2, Fn.avg_pool3d(s1, 2)))
    s3 = c(5, c(4, Fn.avg_pool3d(s2, 2)))
    bott = c(7, c(6, Fn.avg_pool3d(s3, 2)))
    up = lambda t: Fn.interpolate(t, scale_factor=2, mode="nearest")
    d3 = c(8, torch.cat([up(bott), s3], dim=1))
    d2 = c(9, torch.cat([up(d3), s2], dim=1))
    d1 = c(10, torch.cat([up(d2), s1], dim=1))
    return c(11, d1)


def forward(params, x) -> np.ndarray:
    """Inference: params flat, x [B, 2, S^3] (any float) -> y [B, 2, S^3] float64."""
    x = np.asarray(x, dtype=np.float64)
    B, _, V = x.shape
    S = round(V ** (1 / 3))
    with torch.no_grad():
        y = forward_layers(unpack(params), torch.as_tensor(x).reshape(B, 2, S, S, S))
    return y.reshape(B, 2, V).numpy()


def loss_and_grad(params, x, t):
    """Mean-squared error over all outputs and its gradient with respect to the flat parameters."""
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    B, _, V = x.shape
    S = round(V ** (1 / 3))
    p = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    layers, off = [], 0
    for ci, co, taps, _ in LAYERS:
        k = 3 if taps == 27 else 1
        W = p[off:off + co * ci * taps].reshape(co, ci, k, k, k)
        off += co * ci * taps
        b = p[off:off + co]
        off += co
        layers.append((W, b))
    y = forward_layers(layers, torch.as_tensor(x).reshape(B, 2, S, S, S))
    loss = ((y.reshape(B, 2, V) - torch.as_tensor(t)) ** 2).mean()
    loss.backward()
    return float(loss.detach()), p.grad.numpy().copy()


def adam_step(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update (Kingma and Ba, 2015); returns new (w, m, v). step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def conv3d_bruteforce(x, W, b):
    """Zero-padded 3x3x3 cross-correlation by explicit loops: x [ci, S, S, S], W [co, ci, 3, 3, 3]."""
    ci_n, S = x.shape[0], x.shape[1]
    co_n = W.shape[0]
    y = np.zeros((co_n, S, S, S))
    for co in range(co_n):
        for z in range(S):
            for yy in range(S):
                for xx in range(S):
                    s = b[co]
                    for ci in range(ci_n):
                        for dz in (-1, 0, 1):
                            for dy in (-1, 0, 1):
                                for dx in (-1, 0, 1):
                                    zz, y2, x2 = z + dz, yy + dy, xx + dx
                                    if 0 <= zz < S and 0 <= y2 < S and 0 <= x2 < S:
                                        s += W[co, ci, dz + 1, dy + 1, dx + 1] * x[ci, zz, y2, x2]
                    y[co, z, yy, xx] = s
    return y


def prolong(coarse, nc: int, nf: int, scale: float = 1.0, gamma: complex = 0.0) -> np.ndarray:
    """Trilinear interpolation of channels (Re, Im) on coarse nodes (i+1)/(nc+1), i = 0..nc-1, to fine nodes
    (I+1)/(nf+1); beyond the outermost coarse nodes the field is extended by the coarse ghost rule of Sec. 2.3
    (eq. D_bc), U(-1) = gamma U(0), U(nc) = gamma U(nc-1) on each axis (gamma = 0: zero extension).
    Returns complex128 [nf^3] times scale."""
    c = np.asarray(coarse, dtype=np.float64).reshape(2, nc, nc, nc)
    up = np.zeros((nc + 2, nc + 2, nc + 2), dtype=complex)      # ghost ring at coarse indices -1 and nc
    up[1:-1, 1:-1, 1:-1] = c[0] + 1j * c[1]
    for ax in range(3):                                          # one gamma per axis crossed (corners: gamma^k)
        lo, first, hi, last = ([slice(None)] * 3 for _ in range(4))
        lo[ax], first[ax], hi[ax], last[ax] = 0, 1, nc + 1, nc
        up[tuple(lo)] = gamma * up[tuple(first)]
        up[tuple(hi)] = gamma * up[tuple(last)]
    pos = (np.arange(nf) + 1) * (nc + 1) / (nf + 1) - 1.0        # coarse index coordinate of each fine node
    i0 = np.floor(pos).astype(int)
    fr = pos - i0
    out = np.zeros((nf, nf, nf), dtype=complex)
    for dz in (0, 1):
        wz = fr if dz else 1 - fr
        for dy in (0, 1):
            wy = fr if dy else 1 - fr
            for dx in (0, 1):
                wx = fr if dx else 1 - fr
                sel = np.ix_(np.minimum(i0 + dz + 1, nc + 1), np.minimum(i0 + dy + 1, nc + 1),
                             np.minimum(i0 + dx + 1, nc + 1))
                out += wz[:, None, None] * wy[None, :, None] * wx[None, None, :] * up[sel]
    return scale * out.reshape(-1)


def prolong_cubic(coarse, nc: int, nf: int, scale: float = 1.0, gamma: complex = 0.0) -> np.ndarray:
    """Keys' cubic convolution (a = -1/2) from the coarse nodes (i+1)/(nc+1) to the fine nodes (I+1)/(nf+1), as
    the Kronecker product of three 1-D interpolation matrices; coarse indices -m and nc-1+m (m = 1, 2) are ghost
    values gamma^m times the boundary node (the closure of Sec. 2.3, eq. D_bc, applied m times)."""
    a = -0.5
    P = np.zeros((nf, nc), dtype=complex)
    for I in range(nf):
        x = (I + 1) * (nc + 1) / (nf + 1) - 1.0
        i0 = int(np.floor(x))
        t = x - i0
        kern = [a * t ** 3 - 2 * a * t ** 2 + a * t, (a + 2) * t ** 3 - (a + 3) * t ** 2 + 1,
                -(a + 2) * t ** 3 + (2 * a + 3) * t ** 2 - a * t, -a * t ** 3 + a * t ** 2]
        for k, wk in enumerate(kern):
            i = i0 - 1 + k
            if i < 0:
                P[I, 0] += wk * gamma ** (-i)
            elif i >= nc:
                P[I, nc - 1] += wk * gamma ** (i - nc + 1)
            else:
                P[I, i] += wk
    c = np.asarray(coarse, dtype=np.float64).reshape(2, nc, nc, nc)
    u = c[0] + 1j * c[1]
    u = np.tensordot(P, u, axes=(1, 0))                              # z
    u = np.tensordot(P, u, axes=(1, 1)).transpose(1, 0, 2)           # y
    u = np.tensordot(P, u, axes=(1, 2)).transpose(1, 2, 0)           # x
    return scale * u.reshape(-1)


def features(k2_halo, f_halo, halo: int, nf: int, S: int, k0: float, c_scale: float, f_scale: float) -> np.ndarray:
    """Network input [2, S^3]: k^2 and Re f interpolated trilinearly from the solver nodes (I+1)/(nf+1) to the
    network nodes (i+1)/(S+1); channel 0 = c_scale (k^2/k0^2 - 1), channel 1 = f_scale Re f."""
    P = nf + 2 * halo
    k2 = np.asarray(k2_halo, dtype=np.float64).reshape(P, P, P)
    fr = np.asarray(f_halo).reshape(P, P, P).real.astype(np.float64)
    pos = (np.arange(S) + 1) * (nf + 1) / (S + 1) - 1.0 + halo     # index into the halo array
    i0 = np.floor(pos).astype(int)
    w = pos - i0
    out = np.zeros((2, S, S, S))
    for dz in (0, 1):
        wz = w if dz else 1 - w
        for dy in (0, 1):
            wy = w if dy else 1 - w
            for dx in (0, 1):
                wx = w if dx else 1 - w
                ww = wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
                sel = np.ix_(np.minimum(i0 + dz, P - 1), np.minimum(i0 + dy, P - 1), np.minimum(i0 + dx, P - 1))
                out[0] += ww * k2[sel]
                out[1] += ww * fr[sel]
    out[0] = c_scale * (out[0] / (k0 * k0) - 1.0)
    out[1] = f_scale * out[1]
    return out.reshape(2, -1)
