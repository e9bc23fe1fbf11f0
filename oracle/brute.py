"""Pure-Python loop twins of the oracle for tiny grids.  Test infrastructure.

Each function re-derives its result from the definition with explicit loops
(and, where possible, different arithmetic) so that the vectorised oracle can
be pinned against it: a wrong index, roll direction, band or sign in one of
them shows up as a disagreement.
"""
from __future__ import annotations

import math
from typing import List

import numpy as np

from .dd import d1_coeffs, d2_coeffs


def lagrange_at_half(p: int) -> List[float]:
    """Weights of the degree-(2p-1) interpolant at 1/2 through nodes -p+1..p,
    evaluated in floating point by the product formula."""
    nodes = list(range(-p + 1, p + 1))
    out = []
    for k in nodes:
        v = 1.0
        for j in nodes:
            if j != k:
                v *= (0.5 - j) / (k - j)
        out.append(v)
    return out


def forward_brute(u: np.ndarray, J: int, p: int, j0: int) -> np.ndarray:
    """Details by explicit 1-D / tensor 2-D Lagrange interpolation, returned on
    the finest grid (d[y][x]; coarse nodes hold u)."""
    N = 1 << J
    L = lagrange_at_half(p)
    offs = list(range(-p + 1, p + 1))
    d = u.copy()
    for y in range(N):
        for x in range(N):
            lev = j0
            for l in range(J, j0, -1):
                s = 1 << (J - l)
                if (x % s == 0 and y % s == 0) and ((x // s) % 2 == 1 or (y // s) % 2 == 1):
                    lev = l
                    break
            if lev == j0:
                continue
            s = 1 << (J - lev)
            ox, oy = (x // s) % 2 == 1, (y // s) % 2 == 1
            pred = 0.0
            if ox and not oy:
                a0 = x - s
                for w, o in zip(L, offs):
                    pred += w * u[y, (a0 + 2 * s * o) % N]
            elif oy and not ox:
                b0 = y - s
                for w, o in zip(L, offs):
                    pred += w * u[(b0 + 2 * s * o) % N, x]
            else:
                a0, b0 = x - s, y - s
                for wy, oy_ in zip(L, offs):
                    for wx, ox_ in zip(L, offs):
                        pred += wy * wx * u[(b0 + 2 * s * oy_) % N, (a0 + 2 * s * ox_) % N]
            d[y, x] = u[y, x] - pred
    return d


def level_of_node(x: int, y: int, J: int, j0: int) -> int:
    for l in range(j0, J + 1):
        s = 1 << (J - l)
        if x % s == 0 and y % s == 0:
            return l
    raise AssertionError


def active_set_brute(dfine: np.ndarray, u: np.ndarray, eps: float, J: int, j0: int,
                     adjacent_zone: bool = True) -> np.ndarray:
    """Dense boolean active set straight from the definition."""
    N = 1 << J
    tau = eps * max(abs(float(v)) for v in u.ravel())
    lev = [[level_of_node(x, y, J, j0) for x in range(N)] for y in range(N)]
    sig = [(x, y, lev[y][x]) for y in range(N) for x in range(N)
           if lev[y][x] > j0 and abs(dfine[y, x]) >= tau]
    act = np.zeros((N, N), dtype=bool)
    for y in range(N):
        for x in range(N):
            if lev[y][x] == j0:
                act[y, x] = True
    for (x, y, l) in sig:
        act[y, x] = True
    if adjacent_zone:
        for py in range(N):
            for px in range(N):
                if act[py, px]:
                    continue
                for (x, y, l) in sig:
                    if lev[py][px] > min(l + 1, J):
                        continue
                    dx = min((px - x) % N, (x - px) % N)
                    dy = min((py - y) % N, (y - py) % N)
                    if max(dx, dy) <= (1 << (J - l)):
                        act[py, px] = True
                        break
    return act


def d1_matrix(N: int, h: float, p: int, axis: int) -> np.ndarray:
    a = [float(c) for c in d1_coeffs(p)]
    M = np.zeros((N * N, N * N))
    for y in range(N):
        for x in range(N):
            r = y * N + x
            for n, an in enumerate(a, start=1):
                if axis == 1:
                    M[r, y * N + (x + n) % N] += an / h
                    M[r, y * N + (x - n) % N] -= an / h
                else:
                    M[r, ((y + n) % N) * N + x] += an / h
                    M[r, ((y - n) % N) * N + x] -= an / h
    return M


def lap_matrix(N: int, h: float, p: int) -> np.ndarray:
    c = [float(v) for v in d2_coeffs(p)]
    M = np.zeros((N * N, N * N))
    for y in range(N):
        for x in range(N):
            r = y * N + x
            M[r, r] += 2.0 * c[0] / (h * h)
            for n in range(1, p + 1):
                for q in (y * N + (x + n) % N, y * N + (x - n) % N,
                          ((y + n) % N) * N + x, ((y - n) % N) * N + x):
                    M[r, q] += c[n] / (h * h)
    return M


def rhs_matrix_twin(omega: np.ndarray, h: float, p: int, nu0: float, cs: float,
                    mu: float = 0.0):
    """F and the frozen-viscosity Jacobian as explicit matrices (mode 2)."""
    N = omega.shape[0]
    Dx, Dy, L = d1_matrix(N, h, p, 1), d1_matrix(N, h, p, 0), lap_matrix(N, h, p)
    n = N * N
    # Poisson: minimum-norm solution of L psi = -w (zero mean)
    Linv = np.linalg.pinv(L)
    w = omega.ravel()
    psi = -Linv @ w
    u, v = Dy @ psi, -(Dx @ psi)
    s11, s22, s12 = Dx @ u, Dy @ v, 0.5 * (Dy @ u + Dx @ v)
    S = np.sqrt(2.0 * (s11 ** 2 + s22 ** 2 + 2 * s12 ** 2))
    nu = nu0 + (cs * h) ** 2 * S
    F = -(Dx @ (u * w) + Dy @ (v * w)) + 0.5 * (L @ (nu * w) + nu * (L @ w) - w * (L @ nu)) - mu * w
    # Jacobian with nu frozen
    Pu, Pv = Dy @ (-Linv), -(Dx @ (-Linv))       # d u / d w, d v / d w
    Jm = -(Dx @ (np.diag(w) @ Pu + np.diag(u)) + Dy @ (np.diag(w) @ Pv + np.diag(v)))
    Jm += 0.5 * (L @ np.diag(nu) + np.diag(nu) @ L - np.diag(L @ nu)) - mu * np.eye(n)
    return F.reshape(N, N), Jm
