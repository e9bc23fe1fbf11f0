"""Level-adapted evaluation of the residual and of the Jacobian-vector
product, FP64.  Test infrastructure.

Section 2.1 places the method beside the adaptive wavelet collocation method,
which takes the derivatives at an active node with a finite-difference
stencil on the grid of the level that resolves the node's neighbourhood,
using the values of the interpolant at stencil points that are not active
(ghost points).  The dense evaluation (ops.py) instead applies the finest
stencils to Pi(omega) at every node.  Readings (where the paper gives no
rule):

* Local level.  An active node y of level l resolves the nodes within its
  first-derivative reach at its own level, periodic Chebyshev distance
  R 2^(J-l) with R = 2p - 2 (the half-width of the D1 filter).  The local
  level lambda(x) of an active node x is the finest level of an active node
  that resolves it; x resolves itself, so lambda(x) >= level(x), and x is a
  node of G^lambda(x).
* Outer derivatives at the local level.  With s = 2^(J - lambda(x)) the node
  spacing of that level (in finest nodes), the flux divergence and the three
  Laplacians of the conservative diffusion at x use the stencils of D1 and L
  with spacing s h, on values of the dense fields at the stencil points:
  w~ = Pi(omega) (the ghost values), the velocity and the eddy viscosity of
  the dense evaluation (the streamfunction Poisson solve stays the spectral
  one of ops.py, and nu_e its finest-level strain formula).
* Where every node is active (eps = 0), lambda = J everywhere and the
  evaluation is the dense one.

The Jacobian-vector product is the derivative of this residual at frozen
eddy viscosity, with v~ = Pi(v) and the velocity of the spectral solve of v~.
"""
from __future__ import annotations

from typing import Dict

import numpy as np
import scipy.ndimage

from . import mra, ops
from .dd import d1_coeffs, d2_coeffs


def node_level(J: int, p: int) -> np.ndarray:
    """Level of every finest node [N][N]: the coarsest l >= j0 with the node on G^l."""
    j0 = mra.coarsest_level(p)
    N = 1 << J
    lev = np.full((N, N), J, dtype=np.int64)
    for l in range(J - 1, j0 - 1, -1):
        s = 1 << (J - l)
        lev[::s, ::s] = l
    return lev


def local_level(index_fine: np.ndarray, J: int, p: int) -> np.ndarray:
    """lambda of every active node, in index_fine order: the finest level l of
    an active node of level l within periodic Chebyshev distance
    (2p - 2) 2^(J - l) (a maximum filter of the level-l active nodes over that
    box, wrapped)."""
    N = 1 << J
    R = 2 * p - 2
    act = mra.active_dense(index_fine, J)
    lev = node_level(J, p)
    lam = np.full((N, N), -1, dtype=np.int64)
    for l in range(mra.coarsest_level(p), J + 1):
        src = act & (lev == l)
        if not src.any():
            continue
        r = R << (J - l)
        if 2 * r + 1 >= N:
            reach = np.ones((N, N), dtype=bool)
        else:
            reach = scipy.ndimage.maximum_filter(src, size=2 * r + 1, mode="wrap")
        lam[reach] = l            # levels ascend: the finest one that reaches a node stays
    return lam.ravel()[index_fine]


def _d1_at(f: np.ndarray, axis: int, s: int, h: float, p: int) -> np.ndarray:
    """(D1 f) with node spacing s at every node (periodic)."""
    out = np.zeros_like(f)
    for n, a in enumerate(d1_coeffs(p), start=1):
        out += float(a) * (np.roll(f, -n * s, axis) - np.roll(f, n * s, axis))
    return out / (s * h)


def _lap_at(f: np.ndarray, s: int, h: float, p: int) -> np.ndarray:
    c = d2_coeffs(p)
    out = 2.0 * float(c[0]) * f
    for n in range(1, p + 1):
        out = out + float(c[n]) * ((np.roll(f, -n * s, 1) + np.roll(f, n * s, 1)) +
                                   (np.roll(f, -n * s, 0) + np.roll(f, n * s, 0)))
    return out / ((s * h) * (s * h))


def _diffusion_at(nu, w, s, h, p):
    return 0.5 * (_lap_at(nu * w, s, h, p) + nu * _lap_at(w, s, h, p) - w * _lap_at(nu, s, h, p))


def rhs(wt: np.ndarray, base: Dict[str, np.ndarray], index_fine: np.ndarray, lam: np.ndarray, h: float,
        p: int, fl: ops.Flow) -> np.ndarray:
    """F at the active nodes (index_fine order), outer derivatives at each
    node's local level lam.  base: ops.base_fields of wt (dense u, v, nu_e)."""
    J = int(round(np.log2(wt.shape[0])))
    out = np.empty(index_fine.size)
    u, v, nu = base["u"], base["v"], base["nu"]
    for l in np.unique(lam):
        s = 1 << (J - int(l))
        sel = lam == l
        f = -(_d1_at(u * wt, 1, s, h, p) + _d1_at(v * wt, 0, s, h, p)) + _diffusion_at(nu, wt, s, h, p) - fl.mu * wt
        if not fl.advect:
            f = _diffusion_at(nu, wt, s, h, p) - fl.mu * wt
        out[sel] = f.ravel()[index_fine[sel]]
    return out


def jvp(vt: np.ndarray, base: Dict[str, np.ndarray], index_fine: np.ndarray, lam: np.ndarray, h: float,
        p: int, fl: ops.Flow) -> np.ndarray:
    """J v at the active nodes at frozen nu_e, outer derivatives at the local level."""
    J = int(round(np.log2(vt.shape[0])))
    psv = ops.poisson(vt, h, p)
    uv, vv = ops.velocities(psv, h, p)
    w, u, v, nu = base["omega"], base["u"], base["v"], base["nu"]
    out = np.empty(index_fine.size)
    for l in np.unique(lam):
        s = 1 << (J - int(l))
        sel = lam == l
        f = _diffusion_at(nu, vt, s, h, p) - fl.mu * vt
        if fl.advect:
            f = f - (_d1_at(uv * w + u * vt, 1, s, h, p) + _d1_at(vv * w + v * vt, 0, s, h, p))
        out[sel] = f.ravel()[index_fine[sel]]
    return out
