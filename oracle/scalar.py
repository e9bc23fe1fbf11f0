"""Passive-scalar transport (water vapor mixing ratio), FP64.  Test
infrastructure: only tests, the smoke check and the benchmark's CPU baseline
use this module.

Section 3.6 solves the vapor equation (eq. (3)) with the same initial
condition for every vortex run and with only a diffusion term on its right
hand side, i.e. the advection-diffusion equation

    dr/dt = -div(u r) + diffusion(kappa, r)

for the mixing ratio r, transported by the vortex flow.  Readings (the paper
names neither the diffusivity nor the coupling of the time steps):

* the flux form and the symmetric conservative diffusion of the vorticity
  residual are used, so that sum(r) is kept to round-off on the dense grid;
* kappa is the eddy viscosity nu_e of the flow (unit turbulent Schmidt
  number) or a constant;
* the scalar's own adaptive grid (threshold, adjacent zone, regrid) and the
  exponential Rosenbrock-Euler step are those of the vorticity; the operator
  is linear in r, so the step is exp(dt L) r up to the Krylov error;
* coupling is first-order splitting: the scalar step from t_n to t_n + dt uses
  the velocity and nu_e of the vorticity at t_n (the base fields of the
  vorticity step that starts at t_n).

Condensation (Section 2.6, the moving vapor interface): the loss of vapor is
the variational derivative of the functional int 1/2 r^2 (r - 1)^2 +
D_v |grad r|^2.  Read as the gradient flow of that functional (the sign that
makes a vapor patch shrink, as the section's experiment describes; the
printed sign would make the flow ill posed), it adds

    - c f'(r),   f(r) = 1/2 r^2 (r - 1)^2,   f'(r) = r (r - 1) (2 r - 1),

to the right-hand side at every active node (c = 1 in the section's
parameterization, 0 when off), and 2 D_v Laplacian(r), which is the
diffusion above with the constant kappa = 2 D_v.  The step linearises the
reaction at the state of the step's start: its Jacobian adds
-c f''(r_n) v with f''(r) = 6 r^2 - 6 r + 1.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional

import numpy as np

from . import krylov, mra, ops


@dataclasses.dataclass
class ScalarFlow:
    kappa0: float = 0.0          # constant diffusivity (eddy = False)
    eddy: bool = True            # kappa = nu_e of the flow
    cond: float = 0.0            # condensation rate c (0: passive transport only)


def cond_fp(r: np.ndarray) -> np.ndarray:
    """f'(r) for f(r) = 1/2 r^2 (r - 1)^2."""
    return r * (r - 1.0) * (2.0 * r - 1.0)


def cond_fpp(r: np.ndarray) -> np.ndarray:
    """f''(r) = 6 r^2 - 6 r + 1."""
    return 6.0 * r * r - 6.0 * r + 1.0


def operator_dense(r: np.ndarray, u: np.ndarray, v: np.ndarray, kappa: np.ndarray, h: float, p: int):
    """L r = -[D1_x(u r) + D1_y(v r)] + 1/2 [L(kappa r) + kappa L r - r L kappa]
    at every finest node."""
    return ops.advection(u, v, r, h, p) + ops.diffusion(kappa, r, h, p)


def kappa_field(base: Dict[str, np.ndarray], sf: ScalarFlow) -> np.ndarray:
    return base["nu"] if sf.eddy else np.full_like(base["u"], sf.kappa0)


class ScalarOperator:
    """F(r) = L Pi(r) - c f'(r) and A v = L Pi(v) - c f''(r_n) v at the active
    nodes of the scalar (r_n: the active values at the step's start)."""

    def __init__(self, g: krylov.Grid, index_fine: np.ndarray, u: np.ndarray, v: np.ndarray,
                 kappa: np.ndarray, r_base: Optional[np.ndarray] = None, cond: float = 0.0):
        self.g, self.fi, self.u, self.v, self.kappa = g, index_fine, u, v, kappa
        self.r_base, self.cond = r_base, cond

    def linear(self, vals: np.ndarray) -> np.ndarray:
        dense = mra.prolong(vals, self.fi, self.g.J, self.g.p)
        return operator_dense(dense, self.u, self.v, self.kappa, self.g.h, self.g.p).ravel()[self.fi]

    def Av(self, vals: np.ndarray) -> np.ndarray:
        out = self.linear(vals)
        if self.cond != 0.0:
            out = out - self.cond * cond_fpp(self.r_base) * vals
        return out

    def F(self, vals: np.ndarray) -> np.ndarray:
        out = self.linear(vals)
        if self.cond != 0.0:
            out = out - self.cond * cond_fp(vals)
        return out


def step(st: krylov.State, g: krylov.Grid, u: np.ndarray, v: np.ndarray, kappa: np.ndarray, m: int,
         dt: float, do_regrid: bool = True, cond: float = 0.0) -> krylov.State:
    """One exponential step of the scalar with the velocity and diffusivity
    held fixed (and the condensation linearised at the step's start), then
    the FP64 regrid of the scalar's own active set."""
    op = ScalarOperator(g, st.index_fine, u, v, kappa, st.omega_M, cond)
    F = op.F(st.omega_M)
    V, H, m_eff, beta = krylov.arnoldi_mgs(op.Av, F, m)
    r = st.omega_M.copy()
    if beta != 0.0 and m_eff > 0:
        y = krylov.phi1_e1(dt * H[:m_eff, :m_eff])
        r = r + dt * beta * (V[:m_eff].T @ y)
    if not do_regrid:
        return krylov.State(r, st.mask, st.index_packed, st.index_fine, st.t + dt, st.steps + 1, m_eff, beta)
    dense = mra.prolong(r, st.index_fine, g.J, g.p)
    mask, ip, fi, vals = krylov.regrid(dense, g)
    return krylov.State(vals, mask, ip, fi, st.t + dt, st.steps + 1, m_eff, beta)


def coupled_step(vs: krylov.State, ss: krylov.State, gv: krylov.Grid, gs: krylov.Grid, fl: ops.Flow,
                 sf: ScalarFlow, m: int, ms: int, dt: float):
    """Vorticity step, then the scalar step with the vorticity's base fields
    at the start of the step (first-order splitting)."""
    w = mra.prolong(vs.omega_M, vs.index_fine, gv.J, gv.p)
    base = ops.base_fields(w, gv.h, gv.p, fl)
    vs2 = krylov.step(vs, gv, fl, m, dt)
    ss2 = step(ss, gs, base["u"], base["v"], kappa_field(base, sf), ms, dt, cond=sf.cond)
    return vs2, ss2


def run(omega0: np.ndarray, r0: np.ndarray, gv: krylov.Grid, gs: krylov.Grid, fl: ops.Flow, sf: ScalarFlow,
        m: int, ms: int, dt: float, nsteps: int):
    vs, ss = krylov.init_state(omega0, gv), krylov.init_state(r0, gs)
    for _ in range(nsteps):
        vs, ss = coupled_step(vs, ss, gv, gs, fl, sf, m, ms, dt)
    return vs, ss


def mass(r_dense: np.ndarray, h: float) -> float:
    return h * h * float(r_dense.sum())
