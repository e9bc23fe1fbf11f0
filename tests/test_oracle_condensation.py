"""The oracle's vapor condensation (Section 2.6: the gradient flow of
int 1/2 r^2 (r - 1)^2 + D_v |grad r|^2) pinned to what the mathematics fixes:
the stationary uniform states, the closed-form solution of the uniform
field's reaction ODE (with the second order of the exponential
Rosenbrock-Euler step), and the Jacobian of the reaction term against
central differences of the residual."""
import math

import numpy as np
import pytest

from oracle import krylov as ok, scalar as osc

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _op(g, st, cond, kappa=2e-3, seed=0, calm=True):
    N = g.N
    rng = np.random.default_rng(seed)
    u = np.zeros((N, N)) if calm else rng.standard_normal((N, N))
    v = np.zeros((N, N)) if calm else rng.standard_normal((N, N))
    return osc.ScalarOperator(g, st.index_fine, u, v, np.full((N, N), kappa), st.omega_M, cond)


@pytest.mark.parametrize("level", [0.0, 0.5, 1.0])
def test_uniform_fixed_points(level):
    """f'(0) = f'(1/2) = f'(1) = 0 exactly, and a uniform field has no
    diffusion (to the rounding of the Laplacian's weights)."""
    g = ok.Grid(J=4, p=2, eps=1e-3)
    st = ok.init_state(np.full((g.N, g.N), level), g)
    assert np.abs(osc.cond_fp(st.omega_M)).max() == 0.0
    F = _op(g, st, 1.0).F(st.omega_M)
    assert np.abs(F).max() <= 1e-15


def closed_form(r0, c, t):
    """dr/dt = -c r (r - 1)(2r - 1): r (r - 1) / (2r - 1)^2 = K exp(-c t), so
    r = 1/2 -+ 1/2 / sqrt(1 - 4 K exp(-c t)) (the branch of r0)."""
    K = r0 * (r0 - 1.0) / (2.0 * r0 - 1.0) ** 2
    q = K * math.exp(-c * t)
    s = 0.5 / math.sqrt(1.0 - 4.0 * q)
    return 0.5 - s if r0 < 0.5 else 0.5 + s


@pytest.mark.parametrize("r0", [0.3, 0.8])
def test_uniform_field_follows_closed_form_at_second_order(r0):
    g = ok.Grid(J=4, p=2, eps=1e-3)
    N = g.N
    zero = np.zeros((N, N))
    kappa = np.full((N, N), 2e-3)
    T, c = 1.0, 1.5
    errs = []
    for n in (5, 10, 20):
        st = ok.init_state(np.full((N, N), r0), g)
        for _ in range(n):
            st = osc.step(st, g, zero, zero, kappa, 6, T / n, cond=c)
        got = st.omega_M
        assert np.ptp(got) == 0.0                      # stays uniform
        errs.append(abs(got[0] - closed_form(r0, c, T)))
    order = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(order) >= 1.8, (errs, order)
    assert errs[-1] <= 1e-4


def test_jacobian_matches_central_differences():
    """A v = L v - c f''(r) v against (F(r + d v) - F(r - d v)) / (2 d): the
    reaction's derivative and sign, on an all-active random field."""
    g = ok.Grid(J=4, p=2, eps=0.0)
    rng = np.random.default_rng(3)
    r = 0.5 + 0.4 * np.sin(np.add.outer(np.arange(g.N), 2 * np.arange(g.N)) * 2 * math.pi / g.N)
    st = ok.init_state(r, g)
    op = _op(g, st, 1.3, calm=False)
    v = rng.standard_normal(st.omega_M.size)
    d = 1e-5
    fd = (op.F(st.omega_M + d * v) - op.F(st.omega_M - d * v)) / (2 * d)
    Av = op.Av(v)
    assert np.abs(fd - Av).max() <= 1e-6 * np.abs(Av).max()
    # the reaction part alone is the diagonal -c f''(r)
    op0 = _op(g, st, 1.3, kappa=0.0)
    lin = op0.linear(v)
    assert np.allclose(op0.Av(v) - lin, -1.3 * (6 * st.omega_M ** 2 - 6 * st.omega_M + 1) * v, rtol=0, atol=1e-12)
