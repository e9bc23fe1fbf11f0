"""Implicit theta-scheme step solved by Newton-Krylov (GMRES), FP64.  Test
infrastructure: only tests, the smoke check and the benchmark's CPU baseline
use this module.

Section 2.1 places the method among Newton-Krylov solvers of the discrete
collocation system without fixing a time scheme.  This module is the implicit
alternative to the exponential step of `krylov.py` (readings, S20):

* the theta-scheme on the active nodes of the step's start,
      G(w) = w - w_n - dt [theta F(w) + (1 - theta) F(w_n)] = 0,
  theta = 1/2 is Crank-Nicolson, theta = 1 backward Euler, theta = 0 the
  explicit Euler step;
* Newton from w_0 = w_n, a fixed number K of iterations,
      (I - theta dt J(w_k)) d = -G(w_k),   w_{k+1} = w_k + d,
  with J = R J Pi at eddy viscosity frozen at w_k (the same Jacobian as the
  exponential step; exact when the Smagorinsky term is off, an inexact Newton
  otherwise), or the exact Jacobian (exact=True: Newton proper);
* each linear system by one cycle of GMRES(m) from a zero guess: Arnoldi
  (modified Gram-Schmidt) on A = I - theta dt J from r = -G, the happy
  breakdown rule of `krylov.py` (h_{j+1,j} <= 1e-13 ||A v_j||), and the
  minimiser of ||beta e_1 - H y|| (numpy's least squares);
* then the FP64 regrid of `krylov.py`.
"""
from __future__ import annotations

import numpy as np

from . import krylov, mra, ops


def gmres(Av, b: np.ndarray, m: int):
    """One GMRES(m) cycle from x0 = 0: returns (x, k) with x in K_k(A, b)
    minimising ||b - A x||, k the Arnoldi dimension reached."""
    V, H, k, beta = krylov.arnoldi_mgs(Av, b, m)
    if beta == 0.0 or k == 0:
        return np.zeros_like(b), 0
    rhs = np.zeros(k + 1)
    rhs[0] = beta
    y = np.linalg.lstsq(H[:k + 1, :k], rhs, rcond=None)[0]
    return V[:k].T @ y, k


def theta_step(st: krylov.State, g: krylov.Grid, fl: ops.Flow, m: int, dt: float, theta: float,
               newton_iters: int, do_regrid: bool = True, exact: bool = False) -> krylov.State:
    op = krylov.Operator(g, fl, st.index_fine, exact)
    wn = st.omega_M.copy()
    Fn = op.F(wn)                          # also sets the frozen fields at w_0
    w, F = wn.copy(), Fn
    k_last = 0
    for it in range(newton_iters):
        if it > 0:
            F = op.F(w)                    # residual and frozen fields at w_k
        r = (wn - w) + dt * (theta * F + (1.0 - theta) * Fn)      # -G(w_k)
        d, k_last = gmres(lambda v: v - theta * dt * op.Av(v), r, m)
        w = w + d
    if not do_regrid:
        return krylov.State(w, st.mask, st.index_packed, st.index_fine, st.t + dt, st.steps + 1, k_last, 0.0)
    dense = mra.prolong(w, st.index_fine, g.J, g.p)
    mask, ip, fi, vals = krylov.regrid(dense, g)
    return krylov.State(vals, mask, ip, fi, st.t + dt, st.steps + 1, k_last, 0.0)


def residual(st: krylov.State, w: np.ndarray, g: krylov.Grid, fl: ops.Flow, dt: float, theta: float) -> np.ndarray:
    """G(w) of the theta-scheme on the active set of `st` (for checks)."""
    op = krylov.Operator(g, fl, st.index_fine)
    Fn = op.F(st.omega_M)
    return w - st.omega_M - dt * (theta * op.F(w) + (1.0 - theta) * Fn)


def run(omega0: np.ndarray, g: krylov.Grid, fl: ops.Flow, m: int, dt: float, theta: float, newton_iters: int,
        nsteps: int) -> krylov.State:
    st = krylov.init_state(omega0, g)
    for _ in range(nsteps):
        st = theta_step(st, g, fl, m, dt, theta, newton_iters)
    return st
