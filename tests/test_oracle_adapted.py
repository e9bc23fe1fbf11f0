"""Pins of the oracle's level-adapted evaluation (oracle/adapted.py): the
local level against a brute-force scan, the residual against a node-by-node
loop twin, the dense evaluation recovered when every node is active, the
Jacobian-vector product as the exact derivative of the residual at frozen
viscosity, the order 2p of the outer stencils on a manufactured flow at the
local spacing, and the distance to the dense evaluation falling with the
threshold (O(eps))."""
import math

import numpy as np
import pytest

from oracle import adapted as ad, krylov as ok, mra as om, ops as oo
from oracle.dd import d1_coeffs, d2_coeffs
import workloads as W


def _field(N, seed=0, noise=0.0):
    vs = [W.Vortex(1.0, 0.4, 2.6, 3.1), W.Vortex(0.8, 0.3, 3.9, 3.3)]
    f = W.vorticity_field(N, vs)
    return f + noise * W.random_field(N, seed) if noise else f


def _active(u, J, p, eps):
    pk = om.forward(u, J, p)
    mask, ip, fi = om.threshold(pk, u, eps, J, p)
    return fi


def _level(x, y, J, j0):
    t = x | y
    if t == 0:
        return j0
    tz = (t & -t).bit_length() - 1
    return max(j0, J - tz)


@pytest.mark.parametrize("p,J,eps", [(2, 5, 3e-3), (3, 5, 3e-3), (2, 6, 1e-2)])
def test_local_level_brute_force(p, J, eps):
    N = 1 << J
    fi = _active(_field(N, 1, 1e-3), J, p, eps)
    j0 = om.coarsest_level(p)
    R = 2 * p - 2
    pts = [(int(k) % N, int(k) // N) for k in fi]
    lev = [_level(x, y, J, j0) for x, y in pts]
    want = []
    for (x, y) in pts:
        best = -1
        for (x2, y2), l2 in zip(pts, lev):
            dx = min((x - x2) % N, (x2 - x) % N)
            dy = min((y - y2) % N, (y2 - y) % N)
            if max(dx, dy) <= R * (1 << (J - l2)):
                best = max(best, l2)
        want.append(best)
    got = ad.local_level(fi, J, p)
    assert np.array_equal(got, np.array(want))
    assert all(g >= l for g, l in zip(got, lev))


def _loop_rhs(wt, base, fi, lam, h, p, fl):
    """Node by node: the flux divergence and the conservative diffusion with
    stencils of spacing s = 2^(J - lambda), explicit sums over the offsets."""
    N = wt.shape[0]
    J = N.bit_length() - 1
    a = [float(c) for c in d1_coeffs(p)]
    c = [float(x) for x in d2_coeffs(p)]
    u, v, nu = base["u"], base["v"], base["nu"]
    out = []
    for k, l in zip(fi, lam):
        x, y = int(k) % N, int(k) // N
        s = 1 << (J - int(l))
        H = s * h
        g = lambda f, dx, dy: f[(y + dy) % N, (x + dx) % N]
        fx = sum(a[n - 1] * (g(u, n * s, 0) * g(wt, n * s, 0) - g(u, -n * s, 0) * g(wt, -n * s, 0))
                 for n in range(1, 2 * p - 1)) / H
        fy = sum(a[n - 1] * (g(v, 0, n * s) * g(wt, 0, n * s) - g(v, 0, -n * s) * g(wt, 0, -n * s))
                 for n in range(1, 2 * p - 1)) / H

        def lap(f):
            t = 2 * c[0] * g(f, 0, 0)
            for n in range(1, p + 1):
                t += c[n] * (g(f, n * s, 0) + g(f, -n * s, 0) + g(f, 0, n * s) + g(f, 0, -n * s))
            return t / (H * H)
        nw = nu * wt
        dif = 0.5 * (lap(nw) + g(nu, 0, 0) * lap(wt) - g(wt, 0, 0) * lap(nu))
        out.append(-(fx + fy) + dif - fl.mu * g(wt, 0, 0))
    return np.array(out)


@pytest.mark.parametrize("p,J,eps", [(2, 4, 0.1), (2, 5, 0.03), (3, 5, 0.1)])
def test_rhs_loop_twin(p, J, eps):
    N = 1 << J
    h = 2 * math.pi / N
    u = _field(N, 2, 1e-2)
    fi = _active(u, J, p, eps)
    wt = om.prolong(u.ravel()[fi], fi, J, p)
    fl = oo.Flow(nu0=2e-3, cs=0.5, mu=0.05)
    base = oo.base_fields(wt, h, p, fl)
    lam = ad.local_level(fi, J, p)
    assert len(set(lam.tolist())) > 1                       # several local levels in play
    F = ad.rhs(wt, base, fi, lam, h, p, fl)
    ref = _loop_rhs(wt, base, fi, lam, h, p, fl)
    assert np.abs(F - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("p", [2, 3])
def test_all_active_is_the_dense_evaluation(p):
    J = 6
    N = 1 << J
    h = 2 * math.pi / N
    u = _field(N, 3, 1e-2)
    fi = _active(u, J, p, 0.0)
    assert fi.size == N * N
    lam = ad.local_level(fi, J, p)
    assert (lam == J).all()
    fl = oo.Flow(nu0=1e-3, cs=0.17)
    wt = om.prolong(u.ravel()[fi], fi, J, p)
    base = oo.base_fields(wt, h, p, fl)
    F = ad.rhs(wt, base, fi, lam, h, p, fl)
    Fd = oo.rhs(wt, h, p, fl, base).ravel()[fi]
    assert np.abs(F - Fd).max() <= 1e-13 * np.abs(Fd).max()
    v = W.random_field(N, 5, smooth=1).ravel()[fi]
    vt = om.prolong(v, fi, J, p)
    Jv = ad.jvp(vt, base, fi, lam, h, p, fl)
    Jd = oo.jvp(vt, base, h, p, fl).ravel()[fi]
    assert np.abs(Jv - Jd).max() <= 1e-13 * np.abs(Jd).max()


@pytest.mark.parametrize("p", [2, 3])
def test_jvp_is_the_derivative_at_frozen_viscosity(p):
    """At frozen nu_e the residual is quadratic in w~, so the central
    difference of the adapted residual equals the adapted product for any
    step."""
    J = 6
    N = 1 << J
    h = 2 * math.pi / N
    u = _field(N, 4, 1e-2)
    fi = _active(u, J, p, 3e-3)
    fl = oo.Flow(nu0=1e-3, cs=0.3)
    wt = om.prolong(u.ravel()[fi], fi, J, p)
    base = oo.base_fields(wt, h, p, fl)
    lam = ad.local_level(fi, J, p)
    v = W.random_field(N, 6, smooth=2).ravel()[fi]
    vt = om.prolong(v, fi, J, p)

    def F(w):
        b = oo.base_fields(w, h, p, fl)
        b["nu"] = base["nu"]                      # viscosity frozen at the base state
        return ad.rhs(w, b, fi, lam, h, p, fl)

    d = 0.37
    cd = (F(wt + d * vt) - F(wt - d * vt)) / (2 * d)
    Jv = ad.jvp(vt, base, fi, lam, h, p, fl)
    assert np.abs(cd - Jv).max() <= 1e-10 * np.abs(Jv).max()


@pytest.mark.parametrize("p", [2, 3])
def test_order_of_the_outer_stencils_at_the_local_level(p):
    """Only the nodes of G^l active (no finer ones): every node's local level
    is l, and on a manufactured flow (uniform velocity U, constant viscosity)
    the adapted residual converges to -U d/dx w + nu lap w at order 2p in the
    local spacing."""
    J = 8
    N = 1 << J
    h = 2 * math.pi / N
    xs = np.arange(N) * h
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    w = np.sin(X) * np.cos(2 * Y) + 0.5 * np.cos(3 * X + Y)
    exact = -(0.7 * (np.cos(X) * np.cos(2 * Y) - 1.5 * np.sin(3 * X + Y))) \
        + 0.02 * (-5 * np.sin(X) * np.cos(2 * Y) - 5.0 * np.cos(3 * X + Y))
    fl = oo.Flow(nu0=0.02, smag_mode=0)
    base = {"omega": w, "u": np.full_like(w, 0.7), "v": np.zeros_like(w), "nu": np.full_like(w, 0.02)}
    errs = []
    for l in (4, 5, 6):
        s = 1 << (J - l)
        ys, xs_ = np.meshgrid(np.arange(0, N, s), np.arange(0, N, s), indexing="ij")
        fi = np.sort((ys * N + xs_).ravel())
        lam = ad.local_level(fi, J, p)
        assert (lam == l).all()
        F = ad.rhs(w, base, fi, lam, h, p, fl)
        errs.append(np.abs(F - exact.ravel()[fi]).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(o - 2 * p) < 0.4 for o in orders), orders


@pytest.mark.parametrize("p", [2, 3])
def test_distance_to_the_dense_evaluation_is_order_eps(p):
    J = 7
    N = 1 << J
    h = 2 * math.pi / N
    u = _field(N)
    fl = oo.Flow(nu0=1e-3, cs=0.17)
    dist = []
    for eps in (1e-2, 1e-3, 1e-4):
        fi = _active(u, J, p, eps)
        wt = om.prolong(u.ravel()[fi], fi, J, p)
        base = oo.base_fields(wt, h, p, fl)
        Fd = oo.rhs(wt, h, p, fl, base).ravel()[fi]
        Fa = ad.rhs(wt, base, fi, ad.local_level(fi, J, p), h, p, fl)
        d = np.abs(Fa - Fd).max() / np.abs(Fd).max()
        assert d <= eps, (eps, d)
        dist.append(d)
    assert dist[0] > dist[1] > dist[2]


def test_adapted_step_all_active_equals_dense_step():
    pb = W.plain_pair(J=5)
    g = ok.Grid(J=pb.J, p=pb.p, eps=0.0)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    st = ok.init_state(W.initial_field(pb), g)
    a = ok.step(st, g, fl, 8, pb.dt, adapted=True)
    b = ok.step(st, g, fl, 8, pb.dt)
    assert np.abs(a.omega_M - b.omega_M).max() <= 1e-13 * np.abs(b.omega_M).max()
