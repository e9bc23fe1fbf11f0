"""Seeded synthetic inputs for the vortex-interaction workloads.

This module is shared by the CPU oracle and by the GPU path.  It only draws
parameters and samples initial vorticity fields; it holds none of the
method's arithmetic (no transform, derivative, Poisson solve or time step).

Every field is FP64, sampled at the nodes x_i = i*h, y_j = j*h of the periodic
square [0, length)^2 with h = length / N, stored row-major as f[y][x].

Initial condition (Section 3.1): the complex potential
w = i*Gamma/(2*pi*r) * (1 - exp(-r^2/a^2)) has the vorticity
omega = Gamma/(pi*a^2) * exp(-r^2/a^2), a Gaussian of circulation Gamma and
radius a.  Distances are plain (not periodised); the periodic mismatch of the
configurations below is below FP64 round-off.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclasses.dataclass(frozen=True)
class Vortex:
    gamma: float          # circulation
    r0: float             # Gaussian radius a
    cx: float
    cy: float


@dataclasses.dataclass
class Problem:
    """One solve: grid, flow and integrator numbers plus the initial vortices."""
    name: str
    J: int                       # finest grid N = 2**J per side
    p: int                       # DD order 2p (p=2: 4-point, p=3: 6-point)
    eps: float                   # threshold
    re: float                    # Reynolds number (mapped to nu0 by nu0_from_re)
    cs: float                    # Smagorinsky constant
    m: int                       # Krylov dimension
    dt: float
    steps: int
    vortices: Tuple[Vortex, ...]
    noise_amp: float = 0.0       # i.i.d. U[-amp, amp] added per node
    noise_seed: int = 0
    length: float = TWO_PI
    smag_mode: int = 2           # 0 off, 1 a-priori s0, 2 local |S|
    s0: float = 0.0
    mu: float = 0.0              # optional linear friction (off)
    adjacent_zone: int = 1

    @property
    def N(self) -> int:
        return 1 << self.J

    @property
    def j0(self) -> int:
        return coarsest_level(self.p)

    @property
    def nu0(self) -> float:
        return nu0_from_re(self.re, self.vortices)


def coarsest_level(p: int) -> int:
    """Smallest periodic level that holds the 2p-point stencil without repeats."""
    return int(math.ceil(math.log2(2 * p)))


def nu0_from_re(re: float, vortices: Sequence[Vortex]) -> float:
    """Re = U R / nu with U the core-edge speed Gamma/(2 pi a) and R = a
    (Section 3.2.5), so nu0 = Gamma_1 / (2 pi Re) with Gamma_1 the strongest
    vortex's circulation."""
    g1 = max(abs(v.gamma) for v in vortices)
    return g1 / (TWO_PI * re)


def vorticity_field(N: int, vortices: Sequence[Vortex], length: float = TWO_PI,
                    noise_amp: float = 0.0, noise_seed: int = 0) -> np.ndarray:
    """Gaussian vortices (Section 3.1) sampled at the nodes, FP64 [N][N]."""
    h = length / N
    x = np.arange(N, dtype=np.float64) * h
    X, Y = np.meshgrid(x, x, indexing="xy")     # X[y][x] = x_i, Y[y][x] = y_j
    w = np.zeros((N, N), dtype=np.float64)
    for v in vortices:
        r2 = (X - v.cx) ** 2 + (Y - v.cy) ** 2
        w += v.gamma / (math.pi * v.r0 ** 2) * np.exp(-r2 / v.r0 ** 2)
    if noise_amp > 0.0:
        rng = np.random.default_rng(noise_seed)
        w += rng.uniform(-noise_amp, noise_amp, size=(N, N))
    return w


def initial_field(pb: Problem) -> np.ndarray:
    return vorticity_field(pb.N, pb.vortices, pb.length, pb.noise_amp, pb.noise_seed)


def vapor_field(N: int, sharpness: float = 8.0, length: float = TWO_PI) -> np.ndarray:
    """Initial vapor mixing ratio of the passive-scalar experiment (Section
    3.6): moist (1) in one half of the domain, dry (0) in the other.  The step is the periodic, smooth
    1/2 (1 + tanh(-A sin(2 pi y / length))) with A = sharpness, so that both
    interfaces (y = 0 and y = length/2) are resolved by the grid."""
    y = (np.arange(N) * (length / N))[:, None]
    r = 0.5 * (1.0 + np.tanh(-sharpness * np.sin(TWO_PI * y / length)))
    return np.repeat(r, N, axis=1)


# Vapor condensation (Section 2.6's moving interface): the section gives the
# functional and a shrinking circular patch but no sizes, so the recipe is
# dimensionless: a patch of radius R0 = 1 centred in the periodic square,
# D_v = 1e-3 (interface width 2 sqrt(2 D_v) ~ 0.09, seven 512^2 nodes), times
# t = 40 and 80 as in the section's figure.
COND_DV = 1e-3


def vapor_patch(N: int, R0: float = 1.0, D_v: float = COND_DV, length: float = TWO_PI) -> np.ndarray:
    """Circular vapor patch: 1 inside a circle of radius R0 at the centre of
    the periodic square, 0 outside, joined by the profile
    1/2 (1 - tanh(d / (2 sqrt(2 D_v)))) of the signed distance d to the circle
    (the planar front of the condensation flow with kappa = 2 D_v)."""
    x = np.arange(N) * (length / N) - length / 2
    d = np.hypot(x[None, :], x[:, None]) - R0
    return 0.5 * (1.0 - np.tanh(d / (2.0 * np.sqrt(2.0 * D_v))))


def random_field(N: int, seed: int, smooth: int = 0) -> np.ndarray:
    """Seeded N(0,1) field, optionally box-smoothed `smooth` times (periodic)."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((N, N))
    for _ in range(smooth):
        f = (f + np.roll(f, 1, 0) + np.roll(f, -1, 0) + np.roll(f, 1, 1) + np.roll(f, -1, 1)) / 5.0
    return f


# ---------------------------------------------------------------- configurations

def plain_pair(J: int = 6) -> Problem:
    """Two equal Gaussian vortices, r0 = 0.3, centres (pi -/+ 0.6, pi); 4-point
    DD, threshold 1e-3, Re = 5000, Cs = 0.17, m = 20, dt = 0.01, 100 steps."""
    c = math.pi
    vs = (Vortex(1.0, 0.3, c - 0.6, c), Vortex(1.0, 0.3, c + 0.6, c))
    return Problem("pair64_fp64", J=J, p=2, eps=1e-3, re=5000.0, cs=0.17, m=20, dt=0.01,
                   steps=100, vortices=vs)


def fujiwhara_pair(seed: int, J: int = 9) -> Problem:
    """Fujiwhara pair at Re = 5000 on 512^2: equal radii r0 ~ U[0.2, 0.4] and
    separation b ~ U[1.0, 1.6] drawn from `seed`; 4-point DD, threshold 1e-4,
    m = 20, dt = 0.01, 2000 steps."""
    rng = np.random.default_rng(seed)
    r0 = float(rng.uniform(0.2, 0.4))
    b = float(rng.uniform(1.0, 1.6))
    c = math.pi
    vs = (Vortex(1.0, r0, c - b / 2, c), Vortex(1.0, r0, c + b / 2, c))
    return Problem(f"fujiwhara512_s{seed}", J=J, p=2, eps=1e-4, re=5000.0, cs=0.17, m=20,
                   dt=0.01, steps=2000, vortices=vs)


# Section 3.3's unequal-strength runs: U1 = 46.8 m/s against U2, equal core
# size, b = 450 km at R = 100 km (b/R = 4.5), Re = 37440 from U1.
E6_U2_OVER_U1 = (1.0, 37.5 / 46.8, 32.8 / 46.8, 28.1 / 46.8, 23.4 / 46.8)
# Section 3.4's cyclone and convection-induced vortex: equal peak vorticity,
# R2/R1 in {0.9, 0.7, 0.5}.
E7_R2_OVER_R1 = (0.9, 0.7, 0.5)


def unequal_strength_pair(u2_over_u1: float, J: int = 9, r0: float = 0.3) -> Problem:
    """Two Gaussians of equal radius r0 whose core-edge speeds Gamma/(2 pi r0)
    are in the ratio u2_over_u1 (so Gamma2 = u2_over_u1 * Gamma1, Gamma1 = 1),
    separation b = 4.5 r0 along x; 4-point DD, threshold 1e-4, Re = 37440,
    m = 20, dt = 0.01."""
    c, b = math.pi, 4.5 * r0
    vs = (Vortex(1.0, r0, c - b / 2, c), Vortex(float(u2_over_u1), r0, c + b / 2, c))
    return Problem(f"unequal_u{u2_over_u1:.3f}", J=J, p=2, eps=1e-4, re=37440.0, cs=0.17, m=20, dt=0.01,
                   steps=2000, vortices=vs)


def unequal_size_pair(r2_over_r1: float, J: int = 9, r1: float = 0.3) -> Problem:
    """A Gaussian of radius r1 (Gamma1 = 1) and one of radius r2 = r2_over_r1 * r1
    with the same peak vorticity Gamma/(pi r^2), so Gamma2 = r2_over_r1^2;
    separation b = 4.5 r1 between the centres (the paper gives none for these
    runs: the unequal-strength spacing is reused); other numbers as
    unequal_strength_pair."""
    c, b = math.pi, 4.5 * r1
    r2 = r2_over_r1 * r1
    vs = (Vortex(1.0, r1, c - b / 2, c), Vortex(float(r2_over_r1) ** 2, r2, c + b / 2, c))
    return Problem(f"unequal_r{r2_over_r1:.2f}", J=J, p=2, eps=1e-4, re=37440.0, cs=0.17, m=20, dt=0.01,
                   steps=2000, vortices=vs)


def three_vortex(J: int = 11) -> Problem:
    """Three Gaussians shaped like the unequal-strength Re = 37440 runs
    (Gamma ratios 1.6 and 2.7, radius ratios 1.25 and 1.7, b/R = 4.5) plus
    seeded white noise of amplitude 1e-3; 6-point DD, threshold 1e-4, m = 30,
    dt = 0.002, 5000 steps."""
    c = math.pi
    vs = (Vortex(1.0, 0.3, c - 0.675, c),
          Vortex(1.0 / 1.6, 0.24, c + 0.675, c),
          Vortex(1.0 / 2.7, 0.3 / 1.7, c, c + 1.35))
    return Problem("three2048", J=J, p=3, eps=1e-4, re=37440.0, cs=0.17, m=30, dt=0.002,
                   steps=5000, vortices=vs, noise_amp=1e-3, noise_seed=37440)


def ensemble(n: int = 256, seed: int = 2026, steps: int = 200) -> List[Problem]:
    """Batched ensemble of two-vortex solves: N ~ U{128..1024}, b ~ U[0.8, 2.0],
    Re ~ U[2000, 37440], threshold 10^U[-5,-3]; r0 = 0.3, 4-point DD, m = 20."""
    rng = np.random.default_rng(seed)
    out = []
    c = math.pi
    for i in range(n):
        J = int(rng.integers(7, 11))
        b = float(rng.uniform(0.8, 2.0))
        re = float(rng.uniform(2000.0, 37440.0))
        eps = float(10.0 ** rng.uniform(-5.0, -3.0))
        vs = (Vortex(1.0, 0.3, c - b / 2, c), Vortex(1.0, 0.3, c + b / 2, c))
        out.append(Problem(f"ens{i}", J=J, p=2, eps=eps, re=re, cs=0.17, m=20, dt=0.01,
                           steps=steps, vortices=vs))
    return out


def serving_requests(n: int = 1000, seed: int = 50, rate: float = 50.0,
                     J_range: Tuple[int, int] = (6, 11),
                     steps_range: Tuple[int, int] = (200, 2000)) -> List[Tuple[float, Problem]]:
    """Poisson arrivals of 1-3 vortex solves: (arrival time [s], problem)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    c = math.pi
    for i in range(n):
        t += float(rng.exponential(1.0 / rate))
        nv = int(rng.integers(1, 4))
        rs = [float(rng.uniform(0.2, 0.4)) for _ in range(nv)]
        gs = [1.0] + [float(rng.uniform(0.4, 1.0)) for _ in range(nv - 1)]
        cents: List[Tuple[float, float]] = []
        while len(cents) < nv:
            rad = 1.5 * math.sqrt(float(rng.uniform()))
            ang = float(rng.uniform(0.0, TWO_PI))
            cand = (c + rad * math.cos(ang), c + rad * math.sin(ang))
            if all(math.hypot(cand[0] - q[0], cand[1] - q[1]) >= 2.5 * max(rs) for q in cents):
                cents.append(cand)
        J = int(rng.integers(J_range[0], J_range[1] + 1))
        re = float(10.0 ** rng.uniform(3.0, math.log10(4e4)))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        h = TWO_PI / (1 << J)
        vs = tuple(Vortex(g, r, cx, cy) for g, r, (cx, cy) in zip(gs, rs, cents))
        out.append((t, Problem(f"req{i}", J=J, p=2, eps=1e-4, re=re, cs=0.17, m=20,
                               dt=min(0.01, h), steps=steps, vortices=vs)))
    return out
