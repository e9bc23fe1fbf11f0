"""Vortex-centre tracking (test infrastructure).

Section 3.2 measures the interaction by the separation b(t) of the vortex
centres against the convective time t* = t / t_c, t_c = 2 pi b0^2 / Gamma,
from the rotation of the corresponding point-vortex pair (Gamma read as the
circulation of one vortex of the pair).  The paper does not say how a centre
is located; the reading used here (S19):

* each node belongs to the nearest of the previous centres (periodic
  distance; ties to the lower index);
* a centre is the previous centre plus the mean periodic displacement of its
  nodes weighted by the positive part of the vorticity, max(w, 0);
* a vortex whose region holds no positive vorticity keeps its centre.

One application is one update; tracking a run applies it after every step
(the centres move far less than their spacing per step).
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np


def periodic_delta(a: np.ndarray, c: float, length: float) -> np.ndarray:
    """a - c wrapped into [-length/2, length/2)."""
    return (a - c + 0.5 * length) % length - 0.5 * length


def update_centres(omega: np.ndarray, centres: Sequence[Tuple[float, float]],
                   length: float = 2.0 * math.pi) -> List[Tuple[float, float]]:
    N = omega.shape[0]
    h = length / N
    x = np.arange(N) * h
    X, Y = np.meshgrid(x, x)                    # f[y][x]
    d2 = []
    for cx, cy in centres:
        dx, dy = periodic_delta(X, cx, length), periodic_delta(Y, cy, length)
        d2.append(dx * dx + dy * dy)
    owner = np.argmin(np.stack(d2), axis=0)     # ties: lowest index
    w = np.maximum(omega, 0.0)
    out = []
    for k, (cx, cy) in enumerate(centres):
        sel = owner == k
        wt = float(w[sel].sum())
        if wt <= 0.0:
            out.append((cx, cy))
            continue
        mx = float((w[sel] * periodic_delta(X[sel], cx, length)).sum()) / wt
        my = float((w[sel] * periodic_delta(Y[sel], cy, length)).sum()) / wt
        out.append(((cx + mx) % length, (cy + my) % length))
    return out


def separation(c1: Tuple[float, float], c2: Tuple[float, float], length: float = 2.0 * math.pi) -> float:
    dx = periodic_delta(np.array(c2[0]), c1[0], length)
    dy = periodic_delta(np.array(c2[1]), c1[1], length)
    return float(math.hypot(dx, dy))


def convective_time(b0: float, gamma: float) -> float:
    return 2.0 * math.pi * b0 * b0 / gamma
