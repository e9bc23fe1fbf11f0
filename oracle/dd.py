"""Exact Deslauriers-Dubuc (DD) coefficients as rationals.  Test infrastructure.

Section 2.4: the DD subdivision of order 2p inserts a node halfway between two
coarse nodes and gives it the value at 1/2 of the degree-(2p-1) polynomial
through the 2p nearest coarse values.  Its limit function phi is even, has
support [-(2p-1), 2p-1] and reproduces polynomials of degree <= 2p-1.

Section 2.5: the collocation first derivative at node x_k is
sum_j c_j phi_j'(x_k), i.e. a centred filter with the weights phi'(n).  They
are obtained here exactly from the refinement equation.  The second
derivative uses the (2p+1)-point Lagrange rule instead of phi'' (documented
reading: the 4-point phi has no phi'' filter and the 6-point one converges
only at fourth order).
"""
from __future__ import annotations

from fractions import Fraction as Fr
from typing import Dict, List, Tuple

import numpy as np


def midpoint_weights(p: int) -> Dict[int, Fr]:
    """Lagrange weights at x = 1/2 for the coarse nodes at offsets -p+1 .. p."""
    offs = list(range(-p + 1, p + 1))
    w = {}
    for o in offs:
        v = Fr(1)
        for q in offs:
            if q != o:
                v *= (Fr(1, 2) - q) / Fr(o - q)
        w[o] = v
    return w


def canonical_pairs(p: int) -> List[Tuple[Fr, Tuple[int, int]]]:
    """Symmetric node pairs, nearest first: [(weight, (lo, hi))] with lo = -i,
    hi = i + 1.  The prediction is evaluated as
    s = w_0*(c_0 + c_1); s = s + w_1*(c_-1 + c_2); ...  (one rounding per op)."""
    w = midpoint_weights(p)
    out = []
    for i in range(p):
        assert w[-i] == w[i + 1]
        out.append((w[-i], (-i, i + 1)))
    return out


def refinement_mask(p: int) -> Dict[int, Fr]:
    """h_k = phi(k/2): phi(x) = sum_k h_k phi(2x - k)."""
    w = midpoint_weights(p)
    h = {0: Fr(1)}
    for i in range(p):
        h[2 * i + 1] = w[-i]
        h[-(2 * i + 1)] = w[-i]
    return h


def _nullspace(A: List[List[Fr]]) -> List[List[Fr]]:
    """Exact null space of a rational matrix by reduced row echelon form."""
    rows = [r[:] for r in A]
    nr, nc = len(rows), len(rows[0])
    piv_cols = []
    r = 0
    for c in range(nc):
        piv = next((i for i in range(r, nr) if rows[i][c] != 0), None)
        if piv is None:
            continue
        rows[r], rows[piv] = rows[piv], rows[r]
        pv = rows[r][c]
        rows[r] = [x / pv for x in rows[r]]
        for i in range(nr):
            if i != r and rows[i][c] != 0:
                f = rows[i][c]
                rows[i] = [a - f * b for a, b in zip(rows[i], rows[r])]
        piv_cols.append(c)
        r += 1
        if r == nr:
            break
    free = [c for c in range(nc) if c not in piv_cols]
    basis = []
    for fc in free:
        v = [Fr(0)] * nc
        v[fc] = Fr(1)
        for i, pc in enumerate(piv_cols):
            v[pc] = -rows[i][fc]
        basis.append(v)
    return basis


def phi_prime_at_integers(p: int) -> Dict[int, Fr]:
    """phi'(n) for |n| <= 2p-1 from phi'(x) = 2 sum_k h_k phi'(2x - k) at the
    integers (eigenvector of [2 h_{2n-m}] for eigenvalue 1), normalised by the
    reproduction of x: sum_n n phi'(n) = -1."""
    h = refinement_mask(p)
    R = 2 * p - 1
    idx = list(range(-R, R + 1))
    A = [[2 * h.get(2 * n - m, Fr(0)) - (1 if n == m else 0) for m in idx] for n in idx]
    ns = _nullspace(A)
    if len(ns) != 1:
        raise ValueError(f"derivative eigenproblem for p={p} is degenerate ({len(ns)})")
    d = ns[0]
    s = sum(n * d[i] for i, n in enumerate(idx))
    d = [x * Fr(-1) / s for x in d]
    return dict(zip(idx, d))


def d1_coeffs(p: int) -> List[Fr]:
    """a_n, n = 1..2p-2, of (D1 f)[k] = (1/h) sum_n a_n (f[k+n] - f[k-n]);
    a_n = -phi'(n) (Section 2.5)."""
    pp = phi_prime_at_integers(p)
    assert pp[2 * p - 1] == 0
    return [-pp[n] for n in range(1, 2 * p - 1)]


def _poly_mul(a: List[Fr], b: List[Fr]) -> List[Fr]:
    out = [Fr(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def d2_coeffs(p: int) -> List[Fr]:
    """c_0..c_p of the (2p+1)-point Lagrange second derivative at node 0:
    (D2 f)[k] = (1/h^2) (c_0 f[k] + sum_n c_n (f[k+n] + f[k-n]))."""
    nodes = list(range(-p, p + 1))
    c = {}
    for k in nodes:
        poly = [Fr(1)]
        for j in nodes:
            if j != k:
                poly = _poly_mul(poly, [Fr(-j, k - j), Fr(1, k - j)])
        c[k] = 2 * poly[2]
    assert all(c[k] == c[-k] for k in nodes)
    return [c[n] for n in range(0, p + 1)]


def cascade_phi(p: int, levels: int) -> Tuple[np.ndarray, np.ndarray]:
    """Brute-force phi on the dyadic points of [-K, K] by running the DD
    subdivision `levels` times from a unit impulse at 0 (Section 2.4)."""
    K = 4 * p
    vals = np.zeros(2 * K + 1)
    vals[K] = 1.0
    wts = [(float(w), lo, hi) for w, (lo, hi) in canonical_pairs(p)]
    for _ in range(levels):
        n = vals.size
        pad = np.concatenate([np.zeros(p), vals, np.zeros(p)])
        mids = np.zeros(n - 1)
        for w, lo, hi in wts:
            mids += w * (pad[p + lo: p + lo + n - 1] + pad[p + hi: p + hi + n - 1])
        new = np.empty(2 * n - 1)
        new[0::2] = vals
        new[1::2] = mids
        vals = new
    x = np.linspace(-K, K, vals.size)
    return x, vals
