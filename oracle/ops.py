"""Collocation operators, Poisson solve, Smagorinsky viscosity, residual and
Jacobian-vector product on the dense finest grid, FP64.  Test infrastructure.

Vorticity-streamfunction statement of the barotropic flow (Section 4: the
model reduces to single-layer barotropic physics; the streamfunction solves a
Poisson equation):  laplacian(psi) = -omega, u = dpsi/dy, v = -dpsi/dx,
d omega/dt = F(omega) = -div(u omega) + (eddy diffusion) - mu omega.

* D1 is the collocation derivative of Section 2.5 (filter phi'(n)).
* D2 is the (2p+1)-point Lagrange second difference; L = D2_x + D2_y.
* Poisson: psi_hat = -omega_hat / lambda(k) with the exact symbol lambda of L,
  the k = 0 mode set to 0 (zero-mean gauge); numpy's FFT is the library step.
* Smagorinsky, eq. (5): nu_e = nu0 + (Cs*Delta)^2 |S|, Delta = h,
  |S| = sqrt(2 S_ij S_ij), S_ij = (du_i/dx_j + du_j/dx_i)/2 (mode 2); mode 1
  uses an a-priori |S| = s0 (as the paper did); mode 0 gives nu0 only.
* Diffusion in the symmetric conservative form
  (1/2)[L(nu w) + nu L w - w L nu], equal to nu L w for constant nu.
* The Jacobian-vector product freezes nu_e (the residual is then quadratic).
"""
from __future__ import annotations

import dataclasses
from typing import Dict

import numpy as np

from .dd import d1_coeffs, d2_coeffs


@dataclasses.dataclass
class Flow:
    nu0: float
    cs: float = 0.17
    s0: float = 0.0
    mu: float = 0.0
    smag_mode: int = 2
    advect: bool = True        # oracle-only switch for the linear special case


def d1(f: np.ndarray, axis: int, h: float, p: int) -> np.ndarray:
    """(D1 f)[k] = (1/h) sum_{n=1}^{2p-2} a_n (f[k+n] - f[k-n]) along axis
    (axis 1 = x, axis 0 = y)."""
    out = np.zeros_like(f)
    for n, a in enumerate(d1_coeffs(p), start=1):
        out += float(a) * (np.roll(f, -n, axis) - np.roll(f, n, axis))
    return out / h


def d2(f: np.ndarray, axis: int, h: float, p: int) -> np.ndarray:
    c = d2_coeffs(p)
    out = float(c[0]) * f
    for n in range(1, p + 1):
        out = out + float(c[n]) * (np.roll(f, -n, axis) + np.roll(f, n, axis))
    return out / (h * h)


def lap(f: np.ndarray, h: float, p: int) -> np.ndarray:
    return d2(f, 1, h, p) + d2(f, 0, h, p)


def d2_symbol(theta: np.ndarray, p: int) -> np.ndarray:
    """sigma_2(theta) = c_0 + 2 sum_n c_n cos(n theta) (times 1/h^2 gives D2's
    eigenvalue on exp(i k x))."""
    c = d2_coeffs(p)
    s = float(c[0]) * np.ones_like(theta)
    for n in range(1, p + 1):
        s = s + 2.0 * float(c[n]) * np.cos(n * theta)
    return s


def lap_symbol(N: int, h: float, p: int) -> np.ndarray:
    """lambda(ky, kx) on the rfft2 half spectrum [N][N/2+1]."""
    ty = 2.0 * np.pi * np.fft.fftfreq(N)
    tx = 2.0 * np.pi * np.fft.rfftfreq(N)
    return (d2_symbol(ty, p)[:, None] + d2_symbol(tx, p)[None, :]) / (h * h)


def poisson(omega: np.ndarray, h: float, p: int) -> np.ndarray:
    """psi with L psi = -(omega - mean omega), mean psi = 0."""
    N = omega.shape[0]
    lam = lap_symbol(N, h, p)
    w = np.fft.rfft2(omega)
    lam[0, 0] = 1.0
    ps = -w / lam
    ps[0, 0] = 0.0
    return np.fft.irfft2(ps, s=omega.shape)


def velocities(psi: np.ndarray, h: float, p: int):
    return d1(psi, 0, h, p), -d1(psi, 1, h, p)


def strain_rate(u: np.ndarray, v: np.ndarray, h: float, p: int) -> np.ndarray:
    s11 = d1(u, 1, h, p)
    s22 = d1(v, 0, h, p)
    s12 = 0.5 * (d1(u, 0, h, p) + d1(v, 1, h, p))
    return np.sqrt(2.0 * (s11 * s11 + s22 * s22 + 2.0 * s12 * s12))


def eddy_viscosity(u: np.ndarray, v: np.ndarray, h: float, p: int, fl: Flow) -> np.ndarray:
    if fl.smag_mode == 0:
        return np.full_like(u, fl.nu0)
    c2 = (fl.cs * h) ** 2
    if fl.smag_mode == 1:
        return np.full_like(u, fl.nu0 + c2 * fl.s0)
    return fl.nu0 + c2 * strain_rate(u, v, h, p)


def base_fields(omega: np.ndarray, h: float, p: int, fl: Flow) -> Dict[str, np.ndarray]:
    psi = poisson(omega, h, p)
    u, v = velocities(psi, h, p)
    nu = eddy_viscosity(u, v, h, p, fl)
    return dict(omega=omega, psi=psi, u=u, v=v, nu=nu)


def advection(u, v, w, h, p):
    return -(d1(u * w, 1, h, p) + d1(v * w, 0, h, p))


def diffusion(nu, w, h, p):
    return 0.5 * (lap(nu * w, h, p) + nu * lap(w, h, p) - w * lap(nu, h, p))


def rhs(omega: np.ndarray, h: float, p: int, fl: Flow, base=None) -> np.ndarray:
    """F(omega) at every finest node."""
    b = base if base is not None else base_fields(omega, h, p, fl)
    out = diffusion(b["nu"], omega, h, p) - fl.mu * omega
    if fl.advect:
        out = out + advection(b["u"], b["v"], omega, h, p)
    return out


def jvp(vt: np.ndarray, base: Dict[str, np.ndarray], h: float, p: int, fl: Flow) -> np.ndarray:
    """J v with nu_e frozen at the base state:
    -[D1_x(u_v w + u v~) + D1_y(v_v w + v v~)] + diffusion(nu, v~) - mu v~."""
    out = diffusion(base["nu"], vt, h, p) - fl.mu * vt
    if fl.advect:
        psv = poisson(vt, h, p)
        uv, vv = velocities(psv, h, p)
        w = base["omega"]
        out = out - (d1(uv * w + base["u"] * vt, 1, h, p) + d1(vv * w + base["v"] * vt, 0, h, p))
    return out


def nu_prime(base: Dict[str, np.ndarray], uv: np.ndarray, vv: np.ndarray, h: float, p: int,
             fl: Flow) -> np.ndarray:
    """Derivative of the eddy viscosity of eq. (5) in the direction whose
    velocity is (u_v, v_v): nu' = (Cs h)^2 d|S| with, for |S| = sqrt(2 Q),
    Q = S11^2 + S22^2 + 2 S12^2, d|S| = dQ / |S| = 2 (S11 S11' + S22 S22'
    + 2 S12 S12') / |S|.  |S| is not differentiable where it vanishes; there
    the numerator vanishes too and nu' is taken as 0 (reading S22).  Zero
    unless the viscosity follows the local strain (smag_mode 2)."""
    if fl.smag_mode != 2:
        return np.zeros_like(uv)
    u, v = base["u"], base["v"]
    s11, s22 = d1(u, 1, h, p), d1(v, 0, h, p)
    s12 = 0.5 * (d1(u, 0, h, p) + d1(v, 1, h, p))
    t11, t22 = d1(uv, 1, h, p), d1(vv, 0, h, p)
    t12 = 0.5 * (d1(uv, 0, h, p) + d1(vv, 1, h, p))
    S = np.sqrt(2.0 * (s11 * s11 + s22 * s22 + 2.0 * s12 * s12))
    num = 2.0 * (s11 * t11 + s22 * t22 + 2.0 * s12 * t12)
    dS = np.divide(num, S, out=np.zeros_like(num), where=S > 0.0)
    return (fl.cs * h) ** 2 * dS


def jvp_exact(vt: np.ndarray, base: Dict[str, np.ndarray], h: float, p: int, fl: Flow) -> np.ndarray:
    """The exact Jacobian-vector product of F: the frozen-viscosity product
    plus the viscosity's own variation, 1/2 [L(nu' w) + nu' L w - w L nu']."""
    out = jvp(vt, base, h, p, fl)
    if fl.smag_mode != 2:
        return out
    uv, vv = velocities(poisson(vt, h, p), h, p)
    return out + diffusion(nu_prime(base, uv, vv, h, p, fl), base["omega"], h, p)

