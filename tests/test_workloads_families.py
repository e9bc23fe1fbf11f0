"""The unequal-strength (Section 3.3) and unequal-size (Section 3.4)
initial-condition families: each vortex's circulation, peak vorticity,
core-edge speed ratio, radius and spacing, measured on the sampled field."""
import math

import numpy as np
import pytest

import workloads as W


def one_vortex(pb, k, N=512):
    return W.vorticity_field(N, [pb.vortices[k]], pb.length)


@pytest.mark.parametrize("ratio", W.E6_U2_OVER_U1)
def test_unequal_strength_pair(ratio):
    pb = W.unequal_strength_pair(ratio)
    h = pb.length / 512
    w1, w2 = one_vortex(pb, 0), one_vortex(pb, 1)
    g1, g2 = h * h * w1.sum(), h * h * w2.sum()
    assert abs(g1 - 1.0) < 1e-12 and abs(g2 - ratio) < 1e-12
    # equal core size: the peak vorticities and the core-edge speeds
    # Gamma / (2 pi a) are both in the ratio U2/U1
    assert pb.vortices[0].r0 == pb.vortices[1].r0
    assert abs(w2.max() / w1.max() - ratio) < 1e-12
    assert abs(pb.vortices[1].gamma / pb.vortices[0].gamma - ratio) < 1e-15
    assert abs((pb.vortices[1].cx - pb.vortices[0].cx) / pb.vortices[0].r0 - 4.5) < 1e-12
    assert pb.re == 37440.0 and abs(pb.nu0 - 1.0 / (2 * math.pi * 37440.0)) < 1e-18


def test_unequal_strength_speeds_are_the_papers():
    u2 = np.array(W.E6_U2_OVER_U1) * 46.8
    assert np.allclose(u2, [46.8, 37.5, 32.8, 28.1, 23.4], rtol=0, atol=1e-12)


@pytest.mark.parametrize("ratio", W.E7_R2_OVER_R1)
def test_unequal_size_pair(ratio):
    pb = W.unequal_size_pair(ratio)
    h = pb.length / 512
    w1, w2 = one_vortex(pb, 0), one_vortex(pb, 1)
    assert abs(h * h * w2.sum() - ratio ** 2) < 1e-12
    # equal peak vorticity Gamma / (pi a^2) (the sampled maxima are off-node
    # by less than h, so compare the analytic peaks and the samples loosely)
    p1 = pb.vortices[0].gamma / (math.pi * pb.vortices[0].r0 ** 2)
    p2 = pb.vortices[1].gamma / (math.pi * pb.vortices[1].r0 ** 2)
    assert abs(p2 / p1 - 1.0) < 1e-14
    assert abs(w2.max() / w1.max() - 1.0) < 0.05
    assert abs(pb.vortices[1].r0 / pb.vortices[0].r0 - ratio) < 1e-15


def test_ensemble_generator_follows_its_distribution():
    probs = W.ensemble(256)
    assert len(probs) == 256 and {pb.J for pb in probs} == {7, 8, 9, 10}
    for pb in probs:
        b = pb.vortices[1].cx - pb.vortices[0].cx
        assert 0.8 <= b <= 2.0 and 2000.0 <= pb.re <= 37440.0 and 1e-5 <= pb.eps <= 1e-3
        assert pb.p == 2 and pb.m == 20 and pb.steps == 200
    assert [pb.name for pb in W.ensemble(256)] == [pb.name for pb in probs]            # seeded


def test_serving_requests_follow_their_distribution():
    timed = W.serving_requests(300, rate=50.0)
    t = np.array([a for a, _ in timed])
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 50.0) < 10.0                 # Poisson arrivals at about 50/s
    for _, pb in timed:
        assert 6 <= pb.J <= 11 and 200 <= pb.steps <= 2000 and 1e3 <= pb.re <= 4e4
        assert 1 <= len(pb.vortices) <= 3 and pb.vortices[0].gamma == 1.0
        assert pb.dt == min(0.01, 2 * math.pi / pb.N)
        rmax = max(v.r0 for v in pb.vortices)
        for i, a in enumerate(pb.vortices):
            assert math.hypot(a.cx - math.pi, a.cy - math.pi) <= 1.5 + 1e-12
            for q in pb.vortices[i + 1:]:
                assert math.hypot(a.cx - q.cx, a.cy - q.cy) >= 2.5 * rmax
