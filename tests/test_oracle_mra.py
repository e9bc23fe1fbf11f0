"""Pins of the oracle's multiresolution pyramid (Section 2.4, eq. (6)):
polynomial annihilation, round trip, brute-force loop twins, translation
invariance, layout bijection, active-set invariants and the prolongation
identities."""
import numpy as np
import pytest

from oracle import brute, mra
from workloads import random_field, vorticity_field, Vortex


@pytest.mark.parametrize("p", [2, 3])
def test_pack_unpack_bijection(p):
    J, j0 = 5, mra.coarsest_level(p)
    ptf = mra.packed_to_fine(J, j0)
    assert np.array_equal(np.sort(ptf), np.arange(1 << (2 * J)))
    f = random_field(1 << J, 1)
    assert np.array_equal(mra.unpack(mra.pack(f, J, j0), J, j0), f)


@pytest.mark.parametrize("p", [2, 3])
def test_forward_annihilates_tensor_polynomials(p):
    # x^a y^b with a, b <= 2p-1 on integer nodes: every detail whose stencil
    # does not cross the periodic seam is exactly zero.
    # centred integer coordinates keep every intermediate below 2^53
    J = {2: 6, 3: 5}[p]
    N = 1 << J
    j0 = mra.coarsest_level(p)
    x = np.arange(N, dtype=np.float64) - N // 2
    X, Y = np.meshgrid(x, x)
    ptf = mra.packed_to_fine(J, j0)
    lev = mra.level_of_packed(J, j0)
    fy, fx = ptf // N, ptf % N
    reach = (2 * p - 1) * (1 << (J - lev))       # stencil half-width in fine units
    inner = (fx - reach >= 0) & (fx + reach < N) & (fy - reach >= 0) & (fy + reach < N)
    inner[: 1 << (2 * j0)] = False
    for a in range(2 * p):
        for b in range(2 * p):
            d = mra.forward(X ** a * Y ** b, J, p)
            assert np.all(d[inner] == 0.0), (a, b)
    assert inner.sum() > 0
    d = mra.forward(X ** (2 * p), J, p)
    assert np.abs(d[inner]).max() > 0


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("J", [6, 9])
def test_round_trip(p, J):
    u = random_field(1 << J, 7 + J)
    back = mra.inverse(mra.forward(u, J, p), J, p)
    lam = {2: 5 / 4, 3: 89 / 64}[p]
    bound = 4 * lam ** (2 * (J - mra.coarsest_level(p))) * np.finfo(float).eps * np.abs(u).max()
    assert np.abs(back - u).max() <= bound


@pytest.mark.parametrize("p", [2, 3])
def test_forward_matches_brute_force_lagrange(p):
    J = 4
    N = 1 << J
    j0 = mra.coarsest_level(p)
    u = random_field(N, 3)
    ref = brute.forward_brute(u, J, p, j0)
    got = mra.unpack(mra.forward(u, J, p), J, j0)
    assert np.abs(got - ref).max() < 1e-13


@pytest.mark.parametrize("p", [2, 3])
def test_translation_commutes(p):
    J = 6
    j0 = mra.coarsest_level(p)
    s = 1 << (J - j0)
    u = random_field(1 << J, 11)
    d = mra.unpack(mra.forward(u, J, p), J, j0)
    d2 = mra.unpack(mra.forward(np.roll(u, (s, 2 * s), (0, 1)), J, p), J, j0)
    assert np.array_equal(np.roll(d, (s, 2 * s), (0, 1)), d2)


def _vortex_field(N):
    return vorticity_field(N, [Vortex(1.0, 0.5, 2.6, 3.1), Vortex(0.7, 0.4, 3.9, 3.3)])


@pytest.mark.parametrize("p,J,eps", [(2, 4, 1e-2), (2, 5, 3e-3), (3, 4, 1e-2), (3, 5, 1e-3)])
def test_active_set_matches_brute_force(p, J, eps):
    N = 1 << J
    j0 = mra.coarsest_level(p)
    u = _vortex_field(N) + 1e-3 * random_field(N, 5)
    pk = mra.forward(u, J, p)
    mask, ip, fi = mra.threshold(pk, u, eps, J, p)
    ref = brute.active_set_brute(mra.unpack(pk, J, j0), u, eps, J, j0)
    assert np.array_equal(mra.active_dense(fi, J), ref)
    assert np.array_equal(ip, np.flatnonzero(mask))
    assert np.all(np.diff(ip) > 0)


@pytest.mark.parametrize("p", [2, 3])
def test_active_set_invariants(p):
    J = 6
    N = 1 << J
    j0 = mra.coarsest_level(p)
    u = _vortex_field(N)
    pk = mra.forward(u, J, p)
    sets = []
    for eps in (1e-1, 1e-2, 1e-3, 1e-4):
        mask, ip, fi = mra.threshold(pk, u, eps, J, p)
        assert mask[: 1 << (2 * j0)].all()                        # coarsest mesh kept
        sets.append(set(ip.tolist()))
    for a, b in zip(sets, sets[1:]):
        assert a <= b                                             # monotone in eps
    mask, ip, fi = mra.threshold(pk, u, 0.0, J, p)
    assert mask.all()


@pytest.mark.parametrize("p", [2, 3])
def test_prolong_identities(p):
    J = 6
    N = 1 << J
    j0 = mra.coarsest_level(p)
    u = _vortex_field(N) + 1e-3 * random_field(N, 2)
    # all active: Pi(R u) = u exactly
    all_fi = mra.packed_to_fine(J, j0)
    assert np.array_equal(mra.prolong(u.ravel()[all_fi], all_fi, J, p), u)
    pk = mra.forward(u, J, p)
    mask, ip, fi = mra.threshold(pk, u, 1e-3, J, p)
    v = random_field(N, 9).ravel()[fi]
    # R Pi v = v exactly
    assert np.array_equal(mra.prolong(v, fi, J, p).ravel()[fi], v)
    # Pi is characterised by: equal to v on M and zero details off M (the
    # details of an inactive node are pred - pred, exactly zero); and its
    # inverse transform with those details gives it back to round-off.
    w = mra.prolong(u.ravel()[fi], fi, J, p)
    dw = mra.forward(w, J, p)
    assert np.all(dw[mask == 0] == 0.0)
    assert np.array_equal(w.ravel()[fi], u.ravel()[fi])
    assert np.abs(mra.inverse(dw, J, p) - w).max() <= 1e-13 * np.abs(u).max()
    # a non-closed mask: Pi differs from simply zeroing u's own inactive details
    pz = pk.copy()
    pz[mask == 0] = 0.0
    assert np.abs(mra.inverse(pz, J, p) - w).max() < 1e-2 * np.abs(u).max()
