// Level-adapted evaluation of the residual and of the Jacobian-vector
// product at the active nodes.
//
// Section 2.1 places the method beside the adaptive wavelet collocation
// method, which takes the derivatives at an active node with the
// finite-difference stencil of the level that resolves the node's
// neighbourhood, on values of the interpolant at stencil points that are not
// active.  Here the local level lambda of an active node x is the finest level
// l of an active node of level l within periodic Chebyshev distance
// (2p - 2) 2^(J - l) of x (that node's first-derivative reach), at least the
// level of x itself; x is a node of G^lambda.  The flux divergence and the
// three Laplacians of the conservative diffusion at x then use the D1 and L
// stencils with node spacing s = 2^(J - lambda) (step s h) on the dense
// fields: w~ = Pi(omega) (the values at inactive stencil points are those of
// the interpolant), the velocity of the spectral Poisson solve and the eddy
// viscosity of the dense residual pass.  Every node active gives lambda = J,
// the dense evaluation.  One thread per active node, no tiles: the work is
// proportional to the active count.
#include "mra_internal.hpp"

namespace mra {

template <int P, typename T> __device__ inline T ad_d1(int n) {
  if constexpr (P == 2) return n == 1 ? T(2.0 / 3.0) : T(-1.0 / 12.0);
  else return n == 1 ? T(272.0 / 365.0) : n == 2 ? T(-53.0 / 365.0) : n == 3 ? T(16.0 / 1095.0) : T(1.0 / 2920.0);
}
template <int P, typename T> __device__ inline T ad_d2(int n) {
  if constexpr (P == 2) return n == 0 ? T(-2.5) : n == 1 ? T(4.0 / 3.0) : T(-1.0 / 12.0);
  else return n == 0 ? T(-49.0 / 18.0) : n == 1 ? T(1.5) : n == 2 ? T(-0.15) : T(1.0 / 90.0);
}

// lambda of every active node: the finest levels first, each scanning the
// (2R + 1)^2 nodes of its lattice around x for an active node new at it.
template <int P>
__global__ void __launch_bounds__(256) k_local_level(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int na = (int)*s.n_active;
  const int J = s.J, N = s.N, nm = N - 1, j0 = s.j0;
  constexpr int R = 2 * P - 2;
  const auto* rank = glb(s.rank);
  const auto* fine = glb(s.index_fine);
  for (int k = MRA_BX(b) * 256 + (int)threadIdx.x; k < na; k += MRA_GX(b) * 256) {
    const int f = fine[k];
    const int x = f & nm, y = f >> J;
    const int lev = level_of(x, y, J, j0);
    int lam = lev;
    for (int l = J; l > lev && lam == lev; --l) {
      const int sp = 1 << (J - l);
      for (int j = -R; j <= R && lam == lev; ++j) {
        const int yy = (y + j * sp) & nm;
        for (int i = -R; i <= R; ++i) {
          const int xx = (x + i * sp) & nm;
          if (((xx | yy) & sp) && rank[yy * N + xx] >= 0) {   // active, and new at level l
            lam = l;
            break;
          }
        }
      }
    }
    glb(s.lam)[k] = (uint8_t)lam;
  }
}

// field value at (x + dx, y + dy), periodic
template <typename T>
__device__ __forceinline__ T at(const T* f, int x, int y, int dx, int dy, int J, int nm) {
  return f[(((y + dy) & nm) << J) + ((x + dx) & nm)];
}

// 1/2 [L(nu a) + nu L a - a L nu] at x with step sp (times (sp h)^2)
template <int P, typename T>
__device__ __forceinline__ T diff_at(const T* nu, const T* a, int x, int y, int sp, int J, int nm) {
  const T n0 = at(nu, x, y, 0, 0, J, nm), a0 = at(a, x, y, 0, 0, J, nm);
  T lna = T(2) * ad_d2<P, T>(0) * (n0 * a0), la = T(2) * ad_d2<P, T>(0) * a0, ln = T(2) * ad_d2<P, T>(0) * n0;
#pragma unroll
  for (int n = 1; n <= P; ++n) {
    const int d = n * sp;
    const T nxp = at(nu, x, y, d, 0, J, nm), nxm = at(nu, x, y, -d, 0, J, nm);
    const T nyp = at(nu, x, y, 0, d, J, nm), nym = at(nu, x, y, 0, -d, J, nm);
    const T axp = at(a, x, y, d, 0, J, nm), axm = at(a, x, y, -d, 0, J, nm);
    const T ayp = at(a, x, y, 0, d, J, nm), aym = at(a, x, y, 0, -d, J, nm);
    const T c = ad_d2<P, T>(n);
    lna += c * ((nxp * axp + nxm * axm) + (nyp * ayp + nym * aym));
    la += c * ((axp + axm) + (ayp + aym));
    ln += c * ((nxp + nxm) + (nyp + nym));
  }
  return T(0.5) * (lna + n0 * la - a0 * ln);
}

// The residual at the active nodes: FP64 solves from wt, u, v, nu; solves
// with FP32 bulk fields (R64) in FP64 from res64, vel64 and the FP64 nu_e the
// fields pass left in dense64.
template <int P, typename T, bool R64>
__global__ void __launch_bounds__(256) k_rhs_adapt(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int na = (int)*s.n_active;
  const int J = s.J, N = s.N, nm = N - 1;
  const T* W = R64 ? reinterpret_cast<const T*>(s.res64) : reinterpret_cast<const T*>(s.wt);
  const T* U = R64 ? reinterpret_cast<const T*>(s.vel64) : reinterpret_cast<const T*>(s.u);
  const T* V = R64 ? reinterpret_cast<const T*>(s.vel64 + (size_t)N * N) : reinterpret_cast<const T*>(s.v);
  const T* NU = R64 ? reinterpret_cast<const T*>(s.dense64) : reinterpret_cast<const T*>(s.nu);
  const T mu = T(s.mu);
  for (int k = MRA_BX(b) * 256 + (int)threadIdx.x; k < na; k += MRA_GX(b) * 256) {
    const int f = s.index_fine[k];
    const int x = f & nm, y = f >> J;
    const int sp = 1 << (J - (int)s.lam[k]);
    const T H = T(sp * s.h);
    T fx = T(0), fy = T(0);
#pragma unroll
    for (int n = 1; n <= 2 * P - 2; ++n) {
      const int d = n * sp;
      const T a = ad_d1<P, T>(n);
      fx += a * (at(U, x, y, d, 0, J, nm) * at(W, x, y, d, 0, J, nm) -
                 at(U, x, y, -d, 0, J, nm) * at(W, x, y, -d, 0, J, nm));
      fy += a * (at(V, x, y, 0, d, J, nm) * at(W, x, y, 0, d, J, nm) -
                 at(V, x, y, 0, -d, J, nm) * at(W, x, y, 0, -d, J, nm));
    }
    const T adv = -(fx + fy) / H;
    const T dif = diff_at<P, T>(NU, W, x, y, sp, J, nm) / (H * H);
    s.out_rhs[k] = (double)(adv + dif - mu * at(W, x, y, 0, 0, J, nm));
  }
}

// The frozen-Jacobian product at the active nodes, in the bulk type: v~ (vt),
// the stream function psi~ of v~ (uv), w~, u, v, nu_e; u_v = D1_y psi~ and
// v_v = -D1_x psi~ (finest collocation stencil) at the flux points.
template <int P, typename T>
__global__ void __launch_bounds__(256) k_jvp_adapt(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  if (s.ctrl[C_DONE]) return;
  const int na = (int)*s.n_active;
  const int J = s.J, N = s.N, nm = N - 1;
  const T* VT = reinterpret_cast<const T*>(s.vt);
  const T* PS = reinterpret_cast<const T*>(s.uv);
  const T* W = reinterpret_cast<const T*>(s.wt);
  const T* U = reinterpret_cast<const T*>(s.u);
  const T* V = reinterpret_cast<const T*>(s.v);
  const T* NU = reinterpret_cast<const T*>(s.nu);
  const T ih = T(1.0 / s.h), mu = T(s.mu);
  for (int k = MRA_BX(b) * 256 + (int)threadIdx.x; k < na; k += MRA_GX(b) * 256) {
    const int f = s.index_fine[k];
    const int x = f & nm, y = f >> J;
    const int sp = 1 << (J - (int)s.lam[k]);
    const T H = T(sp * s.h);
    // the linearised fluxes at (x +- d, y) and (x, y +- d)
    auto fluxx = [&](int dx) {
      T uv = T(0);
#pragma unroll
      for (int m = 1; m <= 2 * P - 2; ++m)
        uv += ad_d1<P, T>(m) * (at(PS, x, y, dx, m, J, nm) - at(PS, x, y, dx, -m, J, nm));
      uv = ih * uv;
      return uv * at(W, x, y, dx, 0, J, nm) + at(U, x, y, dx, 0, J, nm) * at(VT, x, y, dx, 0, J, nm);
    };
    auto fluxy = [&](int dy) {
      T vx = T(0);
#pragma unroll
      for (int m = 1; m <= 2 * P - 2; ++m)
        vx += ad_d1<P, T>(m) * (at(PS, x, y, m, dy, J, nm) - at(PS, x, y, -m, dy, J, nm));
      const T vv = -(ih * vx);
      return vv * at(W, x, y, 0, dy, J, nm) + at(V, x, y, 0, dy, J, nm) * at(VT, x, y, 0, dy, J, nm);
    };
    T fx = T(0), fy = T(0);
#pragma unroll
    for (int n = 1; n <= 2 * P - 2; ++n) {
      const int d = n * sp;
      const T a = ad_d1<P, T>(n);
      fx += a * (fluxx(d) - fluxx(-d));
      fy += a * (fluxy(d) - fluxy(-d));
    }
    const T adv = -(fx + fy) / H;
    const T dif = diff_at<P, T>(NU, VT, x, y, sp, J, nm) / (H * H);
    s.out_jvp[k] = (double)(adv + dif - mu * at(VT, x, y, 0, 0, J, nm));
  }
}

// about 2048 blocks per launch, never more than the nodes need
static int adapt_grid(int J, int nbatch) {
  const int nf = 1 << (2 * J);
  int g = (2048 + nbatch - 1) / nbatch;
  const int cap = (nf + 255) / 256;
  return g < cap ? g : cap;
}

hipError_t launch_local_level(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  dim3 g(adapt_grid(c.J, b.n) * b.n);
  if (c.p == 2) hipLaunchKernelGGL(k_local_level<2>, g, dim3(256), 0, st, b);
  else hipLaunchKernelGGL(k_local_level<3>, g, dim3(256), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_rhs_adapted(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  dim3 g(adapt_grid(c.J, b.n) * b.n);
  const bool r64 = c.prec != 0;     // FP32 bulk fields: the residual in FP64 all the same
  if (c.p == 2) {
    if (r64) hipLaunchKernelGGL((k_rhs_adapt<2, double, true>), g, dim3(256), 0, st, b);
    else hipLaunchKernelGGL((k_rhs_adapt<2, double, false>), g, dim3(256), 0, st, b);
  } else {
    if (r64) hipLaunchKernelGGL((k_rhs_adapt<3, double, true>), g, dim3(256), 0, st, b);
    else hipLaunchKernelGGL((k_rhs_adapt<3, double, false>), g, dim3(256), 0, st, b);
  }
  return hipGetLastError();
}

hipError_t launch_jvp_adapted(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  dim3 g(adapt_grid(c.J, b.n) * b.n);
  if (c.prec == 0) {
    if (c.p == 2) hipLaunchKernelGGL((k_jvp_adapt<2, double>), g, dim3(256), 0, st, b);
    else hipLaunchKernelGGL((k_jvp_adapt<3, double>), g, dim3(256), 0, st, b);
  } else {
    if (c.p == 2) hipLaunchKernelGGL((k_jvp_adapt<2, float>), g, dim3(256), 0, st, b);
    else hipLaunchKernelGGL((k_jvp_adapt<3, float>), g, dim3(256), 0, st, b);
  }
  return hipGetLastError();
}

}  // namespace mra
