"""Dyadic multiresolution pyramid of the DD subdivision, FP64.  Test infrastructure.

Section 2.4, eq. (6): the trial solution u^N = sum_k c_k phi_k with
c_k = u(x_k) on the nested meshes G^{j0} (coarsest) .. G^J (finest).  A point
first appearing on G^l carries the detail d = u - P(u|G^{l-1}), P being the
DD prediction from the coarser mesh; details that are small are dropped
(|u - u^N| < eps filter).

Periodic square, N = 2^J nodes per side, f[y][x] row-major.  Level l has
stride s = 2^(J-l) in finest-grid index units.  Readings where the paper is
silent (periodic domain, coarsest level, tensor-product 2-D rule, threshold
scaling, adjacent zone) are the ones listed in the design notes.

Packed layout (one entry per finest node): the 2^j0 x 2^j0 coarse values at
offset 0, then for l = j0+1..J the three bands of level l, each
2^(l-1) x 2^(l-1) row-major [b][a], at offsets 4^(l-1) (X: x odd, y even at
level l), 2*4^(l-1) (Y: x even, y odd) and 3*4^(l-1) (XY: both odd).
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np

from .dd import canonical_pairs


def coarsest_level(p: int) -> int:
    return int(math.ceil(math.log2(2 * p)))


def _weights(p: int):
    return [(float(w), lo, hi) for w, (lo, hi) in canonical_pairs(p)]


def pred_mid(c: np.ndarray, axis: int, p: int) -> np.ndarray:
    """DD prediction halfway between coarse nodes a and a+1 along `axis`
    (periodic): s = w0*(c[a]+c[a+1]); s = s + w1*(c[a-1]+c[a+2]); ..., each
    operation rounded once (numpy never fuses multiply-add)."""
    s = None
    for w, lo, hi in _weights(p):
        t = w * (np.roll(c, -lo, axis) + np.roll(c, -hi, axis))
        s = t if s is None else s + t
    return s


def _band_slices(J: int, l: int):
    s = 1 << (J - l)
    return ((slice(0, None, 2 * s), slice(s, None, 2 * s)),      # X
            (slice(s, None, 2 * s), slice(0, None, 2 * s)),      # Y
            (slice(s, None, 2 * s), slice(s, None, 2 * s)))      # XY


def _preds(c: np.ndarray, p: int):
    pY = pred_mid(c, 0, p)
    return pred_mid(c, 1, p), pY, pred_mid(pY, 1, p)


def packed_to_fine(J: int, j0: int) -> np.ndarray:
    """fine index y*N + x of every packed position."""
    N = 1 << J
    out = np.empty(N * N, dtype=np.int64)
    n0, s0 = 1 << j0, 1 << (J - j0)
    b, a = np.meshgrid(np.arange(n0), np.arange(n0), indexing="ij")
    out[: n0 * n0] = (b * s0 * N + a * s0).ravel()
    for l in range(j0 + 1, J + 1):
        n, s = 1 << (l - 1), 1 << (J - l)
        b, a = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        base = n * n
        out[base:2 * base] = ((2 * b * s) * N + (2 * a + 1) * s).ravel()
        out[2 * base:3 * base] = (((2 * b + 1) * s) * N + 2 * a * s).ravel()
        out[3 * base:4 * base] = (((2 * b + 1) * s) * N + (2 * a + 1) * s).ravel()
    return out


def level_of_packed(J: int, j0: int) -> np.ndarray:
    N = 1 << J
    lev = np.empty(N * N, dtype=np.int64)
    lev[: 1 << (2 * j0)] = j0
    for l in range(j0 + 1, J + 1):
        lev[1 << (2 * (l - 1)): 1 << (2 * l)] = l
    return lev


def pack(fine: np.ndarray, J: int, j0: int) -> np.ndarray:
    return fine.ravel()[packed_to_fine(J, j0)]


def unpack(packed: np.ndarray, J: int, j0: int) -> np.ndarray:
    N = 1 << J
    out = np.empty(N * N, dtype=packed.dtype)
    out[packed_to_fine(J, j0)] = packed
    return out.reshape(N, N)


def forward(u: np.ndarray, J: int, p: int) -> np.ndarray:
    """Packed pyramid: coarse samples, then the details of every level.  All
    levels are independent because the coarse values are samples of u."""
    j0 = coarsest_level(p)
    N = 1 << J
    assert u.shape == (N, N)
    out = np.empty(N * N, dtype=np.float64)
    s0 = 1 << (J - j0)
    out[: 1 << (2 * j0)] = u[::s0, ::s0].ravel()
    for l in range(j0 + 1, J + 1):
        s, n = 1 << (J - l), 1 << (l - 1)
        c = u[::2 * s, ::2 * s]
        for k, (sl, pr) in enumerate(zip(_band_slices(J, l), _preds(c, p))):
            out[(k + 1) * n * n:(k + 2) * n * n] = (u[sl] - pr).ravel()
    return out


def inverse(packed: np.ndarray, J: int, p: int) -> np.ndarray:
    """Coarse-to-fine reconstruction u = d + P(u|G^{l-1})."""
    j0 = coarsest_level(p)
    N = 1 << J
    u = np.empty((N, N), dtype=np.float64)
    n0, s0 = 1 << j0, 1 << (J - j0)
    u[::s0, ::s0] = packed[: n0 * n0].reshape(n0, n0)
    for l in range(j0 + 1, J + 1):
        s, n = 1 << (J - l), 1 << (l - 1)
        c = u[::2 * s, ::2 * s].copy()
        for k, (sl, pr) in enumerate(zip(_band_slices(J, l), _preds(c, p))):
            u[sl] = packed[(k + 1) * n * n:(k + 2) * n * n].reshape(n, n) + pr
    return u


def active_dense(index_fine: np.ndarray, J: int) -> np.ndarray:
    N = 1 << J
    a = np.zeros(N * N, dtype=bool)
    a[index_fine] = True
    return a.reshape(N, N)


def prolong(values: np.ndarray, index_fine: np.ndarray, J: int, p: int) -> np.ndarray:
    """Nodal inverse transform Pi (eq. (6) with c_k = u(x_k)): active nodes keep
    their value; an inactive node of level l takes the DD prediction from the
    already final level-(l-1) values.  The coarsest mesh is always active."""
    j0 = coarsest_level(p)
    N = 1 << J
    act = active_dense(index_fine, J)
    s0 = 1 << (J - j0)
    assert act[::s0, ::s0].all(), "coarsest mesh must be active"
    u = np.zeros(N * N, dtype=np.float64)
    u[index_fine] = values
    u = u.reshape(N, N)
    for l in range(j0 + 1, J + 1):
        s = 1 << (J - l)
        c = u[::2 * s, ::2 * s].copy()
        for sl, pr in zip(_band_slices(J, l), _preds(c, p)):
            u[sl] = np.where(act[sl], u[sl], pr)
    return u


def threshold(packed: np.ndarray, u: np.ndarray, eps: float, J: int, p: int,
              adjacent_zone: bool = True) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Active set M = G^{j0} + S + AZ(S), S = {non-coarse nodes with
    |d| >= tau}, tau = eps * max|u| over the finest grid.  The adjacent zone of
    a significant node of level l adds every node of G^{min(l+1,J)} within
    periodic Chebyshev distance 2^(J-l) (finest index units).

    Returns (mask in packed layout (uint8), index_packed, index_fine); both
    index lists ascend in packed order."""
    j0 = coarsest_level(p)
    N = 1 << J
    tau = eps * float(np.max(np.abs(u)))
    ptf = packed_to_fine(J, j0)
    lev = level_of_packed(J, j0)
    n0 = 1 << (2 * j0)
    sig = np.zeros(N * N, dtype=bool)
    sig[n0:] = np.abs(packed[n0:]) >= tau
    keep = np.zeros((N, N), dtype=bool)
    s0 = 1 << (J - j0)
    keep[::s0, ::s0] = True
    fy, fx = ptf[sig] // N, ptf[sig] % N
    keep[fy, fx] = True
    if adjacent_zone:
        ls = lev[sig]
        for l in range(j0 + 1, J + 1):
            sel = ls == l
            if not sel.any():
                continue
            y, x = fy[sel], fx[sel]
            dist = 1 << (J - l)
            step = dist // 2 if l < J else 1
            r = dist // step
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    keep[(y + dy * step) % N, (x + dx * step) % N] = True
    mask = keep.ravel()[ptf].astype(np.uint8)
    index_packed = np.flatnonzero(mask).astype(np.int64)
    return mask, index_packed, ptf[index_packed]


def significance_tau(u: np.ndarray, eps: float) -> float:
    return eps * float(np.max(np.abs(u)))
