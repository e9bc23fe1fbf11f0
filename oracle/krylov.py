"""Krylov-projected exponential time step with regrid, FP64.  Test infrastructure.

The paper integrates in time by projecting the discrete system onto a Krylov
subspace (abstract; Section 2.1), without naming the scheme.  The reading
used here is the exponential Rosenbrock-Euler step

    omega_M <- omega_M + dt * phi_1(dt A) F_M,     phi_1(z) = (e^z - 1)/z,

with A = R J Pi the Jacobian (eddy viscosity frozen; or, with exact=True, the
exact Jacobian that also linearises the viscosity) restricted to the active
nodes, approximated in the Arnoldi basis of K_m(A, F_M):
phi_1(dt A) F_M ~= beta V_m phi_1(dt H_m) e_1.  phi_1(dt H_m) e_1 is the last
column of expm([[dt H_m, e_1], [0, 0]]) (scipy's expm is the library step).
Arnoldi uses modified Gram-Schmidt; a happy breakdown
h_{j+1,j} <= 1e-13 ||A v_j|| ends the basis early; beta = 0 skips the update.
After the update the state is regridded in FP64: Pi on the old active set,
forward transform, threshold, and the new active values are the Pi field
sampled at the new active set.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional

import numpy as np
import scipy.linalg

from . import mra, ops

BREAKDOWN = 1e-13


def phi1_e1(Hdt: np.ndarray) -> np.ndarray:
    k = Hdt.shape[0]
    aug = np.zeros((k + 1, k + 1))
    aug[:k, :k] = Hdt
    aug[0, k] = 1.0
    return scipy.linalg.expm(aug)[:k, k]


@dataclasses.dataclass
class Grid:
    J: int
    p: int
    eps: float
    length: float = 2.0 * np.pi
    adjacent_zone: bool = True

    @property
    def N(self):
        return 1 << self.J

    @property
    def h(self):
        return self.length / self.N

    @property
    def j0(self):
        return mra.coarsest_level(self.p)


def regrid(dense: np.ndarray, g: Grid):
    """Forward transform + threshold of a dense field: (mask, index_packed,
    index_fine, active values)."""
    pk = mra.forward(dense, g.J, g.p)
    mask, ip, fi = mra.threshold(pk, dense, g.eps, g.J, g.p, g.adjacent_zone)
    return mask, ip, fi, dense.ravel()[fi].copy()


class Operator:
    """F and A = R J Pi at a fixed active set; J at frozen eddy viscosity, or
    the exact Jacobian (exact=True).  adapted=True: the level-adapted
    evaluation of adapted.py (outer derivatives at each active node's local
    level; frozen-viscosity Jacobian only)."""

    def __init__(self, g: Grid, fl: ops.Flow, index_fine: np.ndarray, exact: bool = False,
                 adapted: bool = False):
        assert not (exact and adapted)
        self.g, self.fl, self.fi, self.exact, self.adapted = g, fl, index_fine, exact, adapted
        if adapted:
            from . import adapted as ad
            self.lam = ad.local_level(index_fine, g.J, g.p)

    def dense(self, vals):
        return mra.prolong(vals, self.fi, self.g.J, self.g.p)

    def F(self, omega_M):
        w = self.dense(omega_M)
        self.base = ops.base_fields(w, self.g.h, self.g.p, self.fl)
        if self.adapted:
            from . import adapted as ad
            return ad.rhs(w, self.base, self.fi, self.lam, self.g.h, self.g.p, self.fl)
        return ops.rhs(w, self.g.h, self.g.p, self.fl, self.base).ravel()[self.fi]

    def Av(self, v):
        vt = self.dense(v)
        if self.adapted:
            from . import adapted as ad
            return ad.jvp(vt, self.base, self.fi, self.lam, self.g.h, self.g.p, self.fl)
        f = ops.jvp_exact if self.exact else ops.jvp
        return f(vt, self.base, self.g.h, self.g.p, self.fl).ravel()[self.fi]


def arnoldi_mgs(Av, v0: np.ndarray, m: int):
    """Returns (V [(m_eff+1) x n], H [(m_eff+1) x m_eff], m_eff, beta)."""
    beta = float(np.linalg.norm(v0))
    n = v0.size
    V = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    if beta == 0.0:
        return V[:1], H[:1, :0], 0, 0.0
    V[0] = v0 / beta
    m_eff = m
    for j in range(m):
        w = Av(V[j])
        nAv = float(np.linalg.norm(w))
        for i in range(j + 1):
            H[i, j] = float(np.dot(V[i], w))
            w = w - H[i, j] * V[i]
        H[j + 1, j] = float(np.linalg.norm(w))
        if H[j + 1, j] <= BREAKDOWN * nAv:
            m_eff = j + 1
            break
        V[j + 1] = w / H[j + 1, j]
    return V[:m_eff + 1], H[:m_eff + 1, :m_eff], m_eff, beta


@dataclasses.dataclass
class State:
    omega_M: np.ndarray
    mask: np.ndarray
    index_packed: np.ndarray
    index_fine: np.ndarray
    t: float = 0.0
    steps: int = 0
    last_m_eff: int = 0
    last_beta: float = 0.0


def init_state(omega0: np.ndarray, g: Grid) -> State:
    mask, ip, fi, vals = regrid(omega0, g)
    return State(vals, mask, ip, fi)


def step(st: State, g: Grid, fl: ops.Flow, m: int, dt: float, do_regrid: bool = True,
         exact: bool = False, adapted: bool = False) -> State:
    op = Operator(g, fl, st.index_fine, exact, adapted)
    F = op.F(st.omega_M)
    V, H, m_eff, beta = arnoldi_mgs(op.Av, F, m)
    om = st.omega_M.copy()
    if beta != 0.0 and m_eff > 0:
        y = phi1_e1(dt * H[:m_eff, :m_eff])
        om = om + dt * beta * (V[:m_eff].T @ y)
    if not do_regrid:
        return State(om, st.mask, st.index_packed, st.index_fine, st.t + dt, st.steps + 1, m_eff, beta)
    dense = mra.prolong(om, st.index_fine, g.J, g.p)
    mask, ip, fi, vals = regrid(dense, g)
    return State(vals, mask, ip, fi, st.t + dt, st.steps + 1, m_eff, beta)


def diagnostics(omega: np.ndarray, g: Grid) -> Dict[str, float]:
    """Gamma = h^2 sum w; E = h^2/2 sum(u^2+v^2); Z = h^2/2 sum w^2;
    P = h^2/2 sum |grad w|^2; max|w| (Sections 3.3, 3.4)."""
    h, p = g.h, g.p
    psi = ops.poisson(omega, h, p)
    u, v = ops.velocities(psi, h, p)
    gx, gy = ops.d1(omega, 1, h, p), ops.d1(omega, 0, h, p)
    h2 = h * h
    return dict(gamma=h2 * float(omega.sum()),
                energy=0.5 * h2 * float((u * u + v * v).sum()),
                enstrophy=0.5 * h2 * float((omega * omega).sum()),
                palinstrophy=0.5 * h2 * float((gx * gx + gy * gy).sum()),
                max_abs=float(np.abs(omega).max()))


def run(omega0: np.ndarray, g: Grid, fl: ops.Flow, m: int, dt: float, nsteps: int,
        st: Optional[State] = None, exact: bool = False) -> State:
    st = st if st is not None else init_state(omega0, g)
    for _ in range(nsteps):
        st = step(st, g, fl, m, dt, exact=exact)
    return st
