"""Pins of the vortex-centre tracking (Section 3.2: b(t)/b(0) against
t* = t / t_c): symmetric Gaussians give their exact centres, tracking commutes
with whole-node translations, separations wrap periodically."""
import math

import numpy as np

from oracle import track
import workloads as W

L = 2 * math.pi


def test_single_gaussian_centre_is_recovered_from_an_offset_guess():
    N = 64
    h = L / N
    c = (20 * h, 37 * h)                      # on a node: the sampled field is symmetric about it
    w = W.vorticity_field(N, [W.Vortex(1.0, 0.3, *c)])
    (cx, cy), = track.update_centres(w, [(c[0] + 0.2, c[1] - 0.15)])
    assert abs(cx - c[0]) < 1e-13 and abs(cy - c[1]) < 1e-13


def test_separated_pair_centres_and_separation():
    N = 128
    h = L / N
    c1, c2 = (40 * h, 64 * h), (88 * h, 64 * h)          # b = 48 h ~ 2.36, radii 0.2
    w = W.vorticity_field(N, [W.Vortex(1.0, 0.2, *c1), W.Vortex(0.7, 0.2, *c2)])
    got = track.update_centres(w, [(c1[0] + 0.05, c1[1] + 0.05), (c2[0] - 0.05, c2[1])])
    assert np.allclose(got, [c1, c2], atol=1e-12)
    assert abs(track.separation(*got) - 48 * h) < 1e-12


def test_translation_by_whole_nodes_commutes():
    N = 64
    h = L / N
    w = W.vorticity_field(N, [W.Vortex(1.0, 0.3, 2.9, 3.2), W.Vortex(0.8, 0.25, 3.9, 3.0)])
    guess = [(2.8, 3.1), (4.0, 3.1)]
    a = track.update_centres(w, guess)
    sx, sy = 5, -7
    b = track.update_centres(np.roll(np.roll(w, sy, axis=0), sx, axis=1),
                             [((x + sx * h) % L, (y + sy * h) % L) for x, y in guess])
    for (ax, ay), (bx, by) in zip(a, b):
        assert abs(track.periodic_delta(np.array(bx), (ax + sx * h) % L, L)) < 1e-12
        assert abs(track.periodic_delta(np.array(by), (ay + sy * h) % L, L)) < 1e-12


def test_separation_wraps_and_convective_time():
    assert abs(track.separation((0.1, 1.0), (L - 0.1, 1.0)) - 0.2) < 1e-14
    assert abs(track.convective_time(2.0, 1.0) - 8 * math.pi) < 1e-14
