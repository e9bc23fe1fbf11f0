// Collocation stencils of the residual and of its Jacobian-vector product,
// and the diagnostics, on tiles of the dense finest grid staged in LDS.
//
// Section 2.5: first derivatives at a node use the DD collocation filter
// (D1 f)[k] = (1/h) sum_{n=1}^{2p-2} a_n (f[k+n] - f[k-n]), a_n = -phi'(n):
//   p = 2: (2/3, -1/12);  p = 3: (272/365, -53/365, 16/1095, 1/2920).
// Second derivatives use the (2p+1)-point Lagrange rule
//   p = 2: (-5/2; 4/3, -1/12)/h^2;  p = 3: (-49/18; 3/2, -3/20, 1/90)/h^2.
// Section 2.3, eq. (5): Smagorinsky eddy viscosity nu_e = nu0 + (Cs h)^2 |S|,
// |S| = sqrt(2 S_ij S_ij) from the resolved strain of the velocity
// u = D1_y psi, v = -D1_x psi (computed by the Fourier pass of the Poisson
// solve and read here for the residual; the products of the frozen Jacobian
// read psi~ and apply D1 themselves).
// Residual (flux form, symmetric conservative diffusion):
//   F = -[D1_x(u w) + D1_y(v w)] + 1/2 [L(nu w) + nu L w - w L nu] - mu w,
// evaluated only at the active nodes of a tile (written to their position in
// the active list through the dense rank map); tiles without an active node
// skip the residual.  The residual kernel also stores nu_e on the whole grid:
// the Jacobian-vector products of the step reuse it (frozen) with u and v.
#include <type_traits>

#include "mra_internal.hpp"

namespace mra {

template <int P, typename T> __device__ inline T d1c(int n) {
  if constexpr (P == 2) return n == 1 ? T(2.0 / 3.0) : T(-1.0 / 12.0);
  else return n == 1 ? T(272.0 / 365.0) : n == 2 ? T(-53.0 / 365.0) : n == 3 ? T(16.0 / 1095.0) : T(1.0 / 2920.0);
}
template <int P, typename T> __device__ inline T d2c(int n) {
  if constexpr (P == 2) return n == 0 ? T(-2.5) : n == 1 ? T(4.0 / 3.0) : T(-1.0 / 12.0);
  else return n == 0 ? T(-49.0 / 18.0) : n == 1 ? T(1.5) : n == 2 ? T(-0.15) : T(1.0 / 90.0);
}

// D1 along x / y at (r, c) of an LDS array with pitch W (times 1/h outside)
template <int P, typename T> __device__ inline T dx1(const T* a, int W, int r, int c) {
  T s = T(0);
#pragma unroll
  for (int n = 1; n <= 2 * P - 2; ++n) s += d1c<P, T>(n) * (a[r * W + c + n] - a[r * W + c - n]);
  return s;
}
template <int P, typename T> __device__ inline T dy1(const T* a, int W, int r, int c) {
  T s = T(0);
#pragma unroll
  for (int n = 1; n <= 2 * P - 2; ++n) s += d1c<P, T>(n) * (a[(r + n) * W + c] - a[(r - n) * W + c]);
  return s;
}
// L = D2_x + D2_y (times 1/h^2 outside)
template <int P, typename T> __device__ inline T lap5(const T* a, int W, int r, int c) {
  T s = T(2) * d2c<P, T>(0) * a[r * W + c];
#pragma unroll
  for (int n = 1; n <= P; ++n)
    s += d2c<P, T>(n) * ((a[r * W + c + n] + a[r * W + c - n]) + (a[(r + n) * W + c] + a[(r - n) * W + c]));
  return s;
}

// A W x W periodic region staged through registers: fetch() issues every
// global load of this thread at once, put() writes them to LDS, so the loads
// of several regions (and other register loads) are in flight together
// instead of one latency per loop trip.
template <int W, typename T, int NT = 256>
struct Region {
  static constexpr int NI = (W * W + NT - 1) / NT;
  T v[NI];
  __device__ inline void fetch(const T* __restrict__ src, int x0, int y0, int N) {
    const int nm = N - 1;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int q = threadIdx.x + NT * i;
      if (q < W * W) {
        const int r = q / W, c = q - r * W;
        v[i] = src[((y0 + r) & nm) * N + ((x0 + c) & nm)];
      }
    }
  }
  // the same through a buffer resource over an N x N field, N = 2^J: one
  // offset register per element and no 64-bit address
  __device__ inline void fetch_buf(__amdgpu_buffer_rsrc_t rs, int x0, int y0, int J) {
    const int nm = (1 << J) - 1;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int q = threadIdx.x + NT * i;
      if (q < W * W) {
        const int r = q / W, c = q - r * W;
        const unsigned f = ((unsigned)((y0 + r) & nm) << J) + (unsigned)((x0 + c) & nm);
        v[i] = buf_ld<T>(rs, f * (unsigned)sizeof(T), 0u);
      }
    }
  }
  __device__ inline void put(T* dst) const {
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int q = threadIdx.x + NT * i;
      if (q < W * W) dst[q] = v[i];
    }
  }
};


template <int P> struct Geo {
  static constexpr int R1 = 2 * P - 2;   // D1 reach
  static constexpr int HU = 3 * P - 2;   // u, v halo for the residual
};

template <int P, typename T>
__host__ __device__ inline size_t rhs_lds_elems(int TS) {
  using G = Geo<P>;
  const size_t Wu = TS + 2 * G::HU, Wn = TS + 2 * P, Ww = TS + 2 * G::R1;
  return 2 * Wu * Wu + 2 * Wn * Wn + Ww * Ww;
}
template <int P, typename T>
__host__ __device__ inline size_t jvp_lds_elems(int TS, bool exact = false) {
  using G = Geo<P>;
  const size_t Ww = TS + 2 * G::R1, Wn = TS + 2 * P;
  // frozen: v~, both fluxes, nu_e, and psi~ sharing its buffer with nu_e v~
  return exact ? 4 * Ww * Ww + 4 * Wn * Wn : 4 * Ww * Ww + Wn * Wn;
}

// R64: the residual of a solve whose bulk fields are FP32, evaluated in FP64
// from the FP64 prolongation res64 and its FP64 velocity vel64 (u, then v).
// Such a kernel also leaves the FP32 copies of w~, u, v (rounded) and nu_e in
// the bulk fields, which the Jacobian-vector products of the step read.
// FIELDS: only the fields (nu_e, and with R64 the FP32 copies and nu_e in FP64
// in dense64), no residual: the level-adapted residual follows.
template <int P, typename T, int TS, bool R64 = false, bool FIELDS = false, int NT = 256>
__global__ void __launch_bounds__(NT) k_rhs(Batch b) {
  static_assert(!R64 || sizeof(T) == 8, "the FP32-bulk residual runs in FP64");
  using G = Geo<P>;
  using TB = typename std::conditional<R64, float, T>::type;   // bulk field type
  extern __shared__ unsigned char smem[];
  const SolveDev& s = MRA_SOLVE(b);
  const int N = s.N, ntx = s.ntx;
  const int tile = tile_of_block(MRA_BX(b), ntx * ntx, b.n);
  const int x0 = (tile % ntx) * TS, y0 = (tile / ntx) * TS;
  constexpr int Wu = TS + 2 * G::HU, Wn = TS + 2 * P, Ww = TS + 2 * G::R1;
  T* uu = reinterpret_cast<T*>(smem);
  T* vv = uu + Wu * Wu;
  T* nu = vv + Wu * Wu;
  T* ww = nu + Wn * Wn;
  T* cn = ww + Ww * Ww;
  {
    const T* gu = R64 ? reinterpret_cast<const T*>(s.vel64) : reinterpret_cast<const T*>(s.u);
    const T* gv = R64 ? reinterpret_cast<const T*>(s.vel64 + (size_t)N * N) : reinterpret_cast<const T*>(s.v);
    const T* gw = R64 ? reinterpret_cast<const T*>(s.res64) : reinterpret_cast<const T*>(s.wt);
    Region<Wu, T, NT> ru, rv;
    Region<Ww, T, NT> rw;
    ru.fetch(gu, x0 - G::HU, y0 - G::HU, N);
    rv.fetch(gv, x0 - G::HU, y0 - G::HU, N);
    rw.fetch(gw, x0 - G::R1, y0 - G::R1, N);
    ru.put(uu);
    rv.put(vv);
    rw.put(ww);
  }
  __syncthreads();
  if constexpr (R64) {
    // the FP32 fields of the products: every tile writes its own nodes
    TB* bw = reinterpret_cast<TB*>(s.wt);
    TB* bu = reinterpret_cast<TB*>(s.u);
    TB* bv = reinterpret_cast<TB*>(s.v);
    for (int q = threadIdx.x; q < TS * TS; q += blockDim.x) {
      const int r = q / TS, c = q - r * TS;
      const size_t o = (size_t)(y0 + r) * N + x0 + c;
      bw[o] = (TB)ww[(r + G::R1) * Ww + c + G::R1];
      bu[o] = (TB)uu[(r + G::HU) * Wu + c + G::HU];
      bv[o] = (TB)vv[(r + G::HU) * Wu + c + G::HU];
    }
  }
  const T ih = T(1.0 / s.h), ih2 = T(1.0 / (s.h * s.h));
  // nu_e on the Wn region
  const T cs2 = T((s.cs * s.h) * (s.cs * s.h));
  const T nu0 = T(s.nu0);
  const T nuc = T(s.nu0 + (s.cs * s.h) * (s.cs * s.h) * s.s0);
  for (int q = threadIdx.x; q < Wn * Wn; q += blockDim.x) {
    const int r = q / Wn, c = q - r * Wn;
    T val;
    if (s.smag_mode == 2) {
      const int ru = r + G::R1, cu = c + G::R1;
      const T s11 = ih * dx1<P, T>(uu, Wu, ru, cu);
      const T s22 = ih * dy1<P, T>(vv, Wu, ru, cu);
      const T s12 = T(0.5) * ih * (dy1<P, T>(uu, Wu, ru, cu) + dx1<P, T>(vv, Wu, ru, cu));
      val = nu0 + cs2 * sqrt(T(2) * (s11 * s11 + s22 * s22 + T(2) * s12 * s12));
    } else {
      val = s.smag_mode == 1 ? nuc : nu0;
    }
    nu[q] = val;
  }
  __syncthreads();
  // store nu_e of the tile for the Jacobian-vector products
  TB* gn = reinterpret_cast<TB*>(s.nu);
  for (int q = threadIdx.x; q < TS * TS; q += blockDim.x) {
    const int r = q / TS, c = q - r * TS;
    gn[(y0 + r) * N + x0 + c] = (TB)nu[(r + P) * Wn + c + P];
  }
  if constexpr (FIELDS) {
    if constexpr (R64) {
      double* g64 = s.dense64;
      for (int q = threadIdx.x; q < TS * TS; q += blockDim.x) {
        const int r = q / TS, c = q - r * TS;
        g64[(y0 + r) * N + x0 + c] = nu[(r + P) * Wn + c + P];
      }
    }
    return;
  }
  if (s.tile_count[tile] == 0) return;
  __syncthreads();
  // fluxes u w, v w on the Ww region (in place of u, v), nu w on the Wn region
  const int ou = G::HU - G::R1;   // = P
  for (int q = threadIdx.x; q < Ww * Ww; q += blockDim.x) {
    const int r = q / Ww, c = q - r * Ww;
    const T wv = ww[q];
    uu[(r + ou) * Wu + c + ou] *= wv;
    vv[(r + ou) * Wu + c + ou] *= wv;
  }
  const int on = G::R1 - P;   // nu w with pitch Wn
  for (int q = threadIdx.x; q < Wn * Wn; q += blockDim.x) {
    const int r = q / Wn, c = q - r * Wn;
    cn[q] = nu[q] * ww[(r + on) * Ww + c + on];
  }
  __syncthreads();
  const int* rank = s.rank;
  const T mu = T(s.mu);
  double* out = s.out_rhs;
  for (int q = threadIdx.x; q < TS * TS; q += blockDim.x) {
    const int r = q / TS, c = q - r * TS;
    const int k = rank[(y0 + r) * N + x0 + c];
    if (k < 0) continue;
    const int ra = r + G::HU, ca = c + G::HU;
    const T adv = -ih * (dx1<P, T>(uu, Wu, ra, ca) + dy1<P, T>(vv, Wu, ra, ca));
    const int rw = r + G::R1, cw = c + G::R1, rn = r + P, cn_ = c + P;
    const T wv = ww[rw * Ww + cw];
    const T nv = nu[rn * Wn + cn_];
    const T diff = T(0.5) * ih2 * (lap5<P, T>(cn, Wn, rn, cn_) + nv * lap5<P, T>(ww, Ww, rw, cw) -
                                   wv * lap5<P, T>(nu, Wn, rn, cn_));
    out[k] = (double)(adv + diff - mu * wv);
  }
}

// Derivative of the eddy viscosity in the direction of the current Arnoldi
// vector, for the exact Jacobian: with S the strain of (u, v) and S' that of
// (u_v, v_v), nu' = (Cs h)^2 2 (S11 S11' + S22 S22' + 2 S12 S12') / |S|
// (0 where |S| = 0, where the numerator vanishes too; |nu'| <= (Cs h)^2 |S'|).
// Written to the solve's FP64 diagnostics buffer (unused during a step) as T,
// on every tile whose 3 x 3 tile neighbourhood holds an active node: the
// product on an active tile reads nu' within its halo.
template <int P, typename T, int TS>
__global__ void __launch_bounds__(256) k_nuprime(Batch b) {
  using G = Geo<P>;
  constexpr int W = TS + 2 * G::R1;
  __shared__ T su[W * W], sv[W * W], suv[W * W], svv[W * W];
  const SolveDev& s = MRA_SOLVE(b);
  const int N = s.N, ntx = s.ntx;
  const int tile = tile_of_block(MRA_BX(b), ntx * ntx, b.n);
  if (s.ctrl[C_DONE] || s.smag_mode != 2) return;
  const int tx = tile % ntx, ty = tile / ntx;
  int near = 0;
  for (int d = 0; d < 9; ++d) {
    const int nx = (tx + d % 3 - 1 + ntx) % ntx, ny = (ty + d / 3 - 1 + ntx) % ntx;
    near |= s.tile_count[ny * ntx + nx];
  }
  if (!near) return;
  const int x0 = tx * TS, y0 = ty * TS;
  {
    Region<W, T> ru, rv, ruv, rvv;
    ru.fetch(reinterpret_cast<const T*>(s.u), x0 - G::R1, y0 - G::R1, N);
    rv.fetch(reinterpret_cast<const T*>(s.v), x0 - G::R1, y0 - G::R1, N);
    ruv.fetch(reinterpret_cast<const T*>(s.uv), x0 - G::R1, y0 - G::R1, N);
    rvv.fetch(reinterpret_cast<const T*>(s.vv), x0 - G::R1, y0 - G::R1, N);
    ru.put(su);
    rv.put(sv);
    ruv.put(suv);
    rvv.put(svv);
  }
  __syncthreads();
  const T ih = T(1.0 / s.h);
  const T cs2 = T((s.cs * s.h) * (s.cs * s.h));
  T* out = reinterpret_cast<T*>(s.vel64);
  for (int q = threadIdx.x; q < TS * TS; q += blockDim.x) {
    const int r = q / TS, c = q - r * TS;
    const int ra = r + G::R1, ca = c + G::R1;
    const T s11 = ih * dx1<P, T>(su, W, ra, ca);
    const T s22 = ih * dy1<P, T>(sv, W, ra, ca);
    const T s12 = T(0.5) * ih * (dy1<P, T>(su, W, ra, ca) + dx1<P, T>(sv, W, ra, ca));
    const T t11 = ih * dx1<P, T>(suv, W, ra, ca);
    const T t22 = ih * dy1<P, T>(svv, W, ra, ca);
    const T t12 = T(0.5) * ih * (dy1<P, T>(suv, W, ra, ca) + dx1<P, T>(svv, W, ra, ca));
    const T sn = sqrt(T(2) * (s11 * s11 + s22 * s22 + T(2) * s12 * s12));
    const T num = T(2) * (s11 * t11 + s22 * t22 + T(2) * s12 * t12);
    out[(y0 + r) * N + x0 + c] = sn > T(0) ? cs2 * (num / sn) : T(0);
  }
}

// Jacobian-vector product on one tile.  Every global load is issued in one
// phase: v~ and nu_e regions into LDS; u, v, w~ at this thread's flux points
// and the ranks of its output nodes into registers.  The frozen Jacobian takes
// the stream function psi~ of v~ (into LDS) and forms u_v = D1_y psi~ and
// v_v = -D1_x psi~ with the collocation stencil: one field read instead of
// two, and the Poisson pass skips one inverse transform.  EX (the exact
// Jacobian, local strain) reads u_v and v_v, which k_nuprime differentiates
// as well, and adds the viscosity's variation
// 1/2 [L(nu' w~) + nu' L w~ - w~ L nu'] with nu' from k_nuprime.
template <int P, typename T, int TS, bool EX, int NT = 256>
__global__ void __launch_bounds__(NT) k_jvp(Batch b) {
  using G = Geo<P>;
  extern __shared__ unsigned char smem[];
  const SolveDev& s = MRA_SOLVE(b);
  const int N = s.N, J = s.J, ntx = s.ntx, nm = N - 1;
  // the fields through buffer resources (N x N each, formed while uniform)
  const size_t fbytes = (size_t)N * N * sizeof(T);
  const auto rU = buf_rsrc(s.u, fbytes), rV = buf_rsrc(s.v, fbytes), rW = buf_rsrc(s.wt, fbytes);
  const auto rVt = buf_rsrc(s.vt, fbytes), rNu = buf_rsrc(s.nu, fbytes), rUv = buf_rsrc(s.uv, fbytes);
  const auto rVv = buf_rsrc(s.vv, fbytes), rR = buf_rsrc(s.rank, (size_t)N * N * sizeof(int));
  const int tile = tile_of_block(MRA_BX(b), ntx * ntx, b.n);
  const int done = s.ctrl[C_DONE], cnt = s.tile_count[tile];
  if (done || cnt == 0) return;
  const int x0 = (tile % ntx) * TS, y0 = (tile / ntx) * TS;
  constexpr int Ww = TS + 2 * G::R1, Wn = TS + 2 * P;
  constexpr int NQ = (Ww * Ww + NT - 1) / NT;       // flux points per thread
  constexpr int NO = (TS * TS + NT - 1) / NT;       // output nodes per thread
  T* vt = reinterpret_cast<T*>(smem);
  T* fa = vt + Ww * Ww;
  T* fb = fa + Ww * Ww;
  T* nu = fb + Ww * Ww;
  T* cn = nu + Wn * Wn;
  // frozen Jacobian: psi~ (Ww region), whose D1 gives u~ and v~ in place; it
  // is dead once the fluxes are formed, so nu_e v~ (cn) takes its buffer
  T* ps = cn;
  // exact Jacobian: w~ (Ww region), nu' and nu' w~ (Wn regions)
  T* wl = cn + Wn * Wn;
  T* np = wl + Ww * Ww;
  T* cp = np + Wn * Wn;
  const bool ex = EX && s.smag_mode == 2;
  T ur[NQ], vr[NQ], wr[NQ], uvr[EX ? NQ : 1], vvr[EX ? NQ : 1];
  int kr[NO];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int q = threadIdx.x + NT * i;
    if (q < Ww * Ww) {
      const int r = q / Ww, c = q - r * Ww;
      const unsigned f = ((unsigned)((y0 - G::R1 + r) & nm) << J) + (unsigned)((x0 - G::R1 + c) & nm);
      const unsigned fo = f * (unsigned)sizeof(T);
      ur[i] = buf_ld<T>(rU, fo, 0u);
      vr[i] = buf_ld<T>(rV, fo, 0u);
      wr[i] = buf_ld<T>(rW, fo, 0u);
      if constexpr (EX) {
        uvr[i] = buf_ld<T>(rUv, fo, 0u);
        vvr[i] = buf_ld<T>(rVv, fo, 0u);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NO; ++i) {
    const int q = threadIdx.x + NT * i;
    const unsigned f = ((unsigned)(y0 + q / TS) << J) + (unsigned)(x0 + (q % TS));
    kr[i] = q < TS * TS ? buf_ld<int>(rR, f * 4u, 0u) : -1;
  }
  {
    Region<Wn, T, NT> rnu;
    Region<Ww, T, NT> rvt;
    rvt.fetch_buf(rVt, x0 - G::R1, y0 - G::R1, J);
    rnu.fetch_buf(rNu, x0 - P, y0 - P, J);
    if constexpr (EX) {
      if (ex) {
        Region<Wn, T, NT> rnp;
        rnp.fetch(reinterpret_cast<const T*>(s.vel64), x0 - P, y0 - P, N);
        rnp.put(np);
      }
      rvt.put(vt);
      rnu.put(nu);
    } else {
      Region<Ww, T, NT> rps;
      rps.fetch_buf(rUv, x0 - G::R1, y0 - G::R1, J);
      rvt.put(vt);
      rnu.put(nu);
      rps.put(ps);
    }
  }
  __syncthreads();
  const T ih = T(1.0 / s.h), ih2 = T(1.0 / (s.h * s.h));
  // fluxes of the linearised advection on the Ww region, nu v~ on the Wn region.
  // With psi~: D1_x of the x-flux is taken on the tile's rows only and D1_y of
  // the y-flux on its columns only, so u~ = D1_y psi~ is needed on rows
  // [R1, R1 + TS) and v~ = -D1_x psi~ on columns [R1, R1 + TS) of the region,
  // and their stencils stay inside it.
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int q = threadIdx.x + NT * i;
    if (q < Ww * Ww) {
      const T vtv = vt[q];
      if constexpr (EX) {
        fa[q] = uvr[i] * wr[i] + ur[i] * vtv;
        fb[q] = vvr[i] * wr[i] + vr[i] * vtv;
        wl[q] = wr[i];
      } else {
        const int r = q / Ww, c = q - r * Ww;
        if (r >= G::R1 && r < G::R1 + TS) fa[q] = (ih * dy1<P, T>(ps, Ww, r, c)) * wr[i] + ur[i] * vtv;
        if (c >= G::R1 && c < G::R1 + TS) fb[q] = -(ih * dx1<P, T>(ps, Ww, r, c)) * wr[i] + vr[i] * vtv;
      }
    }
  }
  constexpr int on = G::R1 - P;
  if constexpr (!EX) __syncthreads();   // every flux has read psi~ before cn overwrites it
  for (int q = threadIdx.x; q < Wn * Wn; q += blockDim.x) {
    const int r = q / Wn, c = q - r * Wn;
    cn[q] = nu[q] * vt[(r + on) * Ww + c + on];
  }
  __syncthreads();
  if constexpr (EX) {
    if (ex) {
      for (int q = threadIdx.x; q < Wn * Wn; q += blockDim.x) {
        const int r = q / Wn, c = q - r * Wn;
        cp[q] = np[q] * wl[(r + on) * Ww + c + on];
      }
      __syncthreads();
    }
  }
  const T mu = T(s.mu);
  double* out = s.out_jvp;
#pragma unroll
  for (int i = 0; i < NO; ++i) {
    const int q = threadIdx.x + NT * i;
    const int k = kr[i];
    if (k < 0) continue;
    const int r = q / TS, c = q - r * TS;
    const int ra = r + G::R1, ca = c + G::R1, rn = r + P, cn_ = c + P;
    const T adv = -ih * (dx1<P, T>(fa, Ww, ra, ca) + dy1<P, T>(fb, Ww, ra, ca));
    const T vv = vt[ra * Ww + ca];
    const T nv = nu[rn * Wn + cn_];
    const T diff = T(0.5) * ih2 * (lap5<P, T>(cn, Wn, rn, cn_) + nv * lap5<P, T>(vt, Ww, ra, ca) -
                                   vv * lap5<P, T>(nu, Wn, rn, cn_));
    T tot = adv + diff - mu * vv;
    if constexpr (EX) {
      if (ex) {
        const T wv = wl[ra * Ww + ca];
        const T pv = np[rn * Wn + cn_];
        tot += T(0.5) * ih2 * (lap5<P, T>(cp, Wn, rn, cn_) + pv * lap5<P, T>(wl, Ww, ra, ca) -
                               wv * lap5<P, T>(np, Wn, rn, cn_));
      }
    }
    out[k] = (double)tot;
  }
}

// Passive scalar (Section 3.6): L v~ = -[D1_x(u v~) + D1_y(v v~)]
// + 1/2 [L(kappa v~) + kappa L v~ - v~ L kappa] at the active nodes of one
// tile, with u, v (and the diffusivity kappa, stored in s.nu) the fields the
// scalar was coupled to.  The same kernel gives the residual (v~ = Pi(r),
// check_done = 0) and the products with the Arnoldi vectors.  Condensation
// (Section 2.6, rate c = scal[S_COND], 0 when off) adds -c f'(r) to the
// residual, f(r) = 1/2 r^2 (r - 1)^2, and its linearisation -c f''(r_n) v~ to
// the products, in FP64 from the active values r_n of the step's start.
template <int P, typename T, int TS>
__global__ void __launch_bounds__(256) k_scalar(Batch b, int check_done) {
  using G = Geo<P>;
  extern __shared__ unsigned char smem[];
  const SolveDev& s = MRA_SOLVE(b);
  const int N = s.N, ntx = s.ntx, nm = N - 1;
  const int tile = tile_of_block(MRA_BX(b), ntx * ntx, b.n);
  const int done = check_done ? s.ctrl[C_DONE] : 0, cnt = s.tile_count[tile];
  if (done || cnt == 0) return;
  const int x0 = (tile % ntx) * TS, y0 = (tile / ntx) * TS;
  constexpr int Ww = TS + 2 * G::R1, Wn = TS + 2 * P;
  constexpr int NQ = (Ww * Ww + 255) / 256;       // flux points per thread
  constexpr int NO = (TS * TS + 255) / 256;       // output nodes per thread
  T* vt = reinterpret_cast<T*>(smem);
  T* fa = vt + Ww * Ww;
  T* fb = fa + Ww * Ww;
  T* nu = fb + Ww * Ww;
  T* cn = nu + Wn * Wn;
  const T* gu = reinterpret_cast<const T*>(s.u);
  const T* gv = reinterpret_cast<const T*>(s.v);
  T ur[NQ], vr[NQ];
  int kr[NO];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int q = threadIdx.x + 256 * i;
    if (q < Ww * Ww) {
      const int r = q / Ww, c = q - r * Ww;
      const int f = ((y0 - G::R1 + r) & nm) * N + ((x0 - G::R1 + c) & nm);
      ur[i] = gu[f];
      vr[i] = gv[f];
    }
  }
#pragma unroll
  for (int i = 0; i < NO; ++i) {
    const int q = threadIdx.x + 256 * i;
    kr[i] = q < TS * TS ? s.rank[(y0 + q / TS) * N + x0 + (q % TS)] : -1;
  }
  {
    Region<Ww, T> rvt;
    Region<Wn, T> rnu;
    rvt.fetch(reinterpret_cast<const T*>(s.vt), x0 - G::R1, y0 - G::R1, N);
    rnu.fetch(reinterpret_cast<const T*>(s.nu), x0 - P, y0 - P, N);
    rvt.put(vt);
    rnu.put(nu);
  }
  __syncthreads();
  const T ih = T(1.0 / s.h), ih2 = T(1.0 / (s.h * s.h));
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int q = threadIdx.x + 256 * i;
    if (q < Ww * Ww) {
      const T vtv = vt[q];
      fa[q] = ur[i] * vtv;
      fb[q] = vr[i] * vtv;
    }
  }
  constexpr int on = G::R1 - P;
  for (int q = threadIdx.x; q < Wn * Wn; q += blockDim.x) {
    const int r = q / Wn, c = q - r * Wn;
    cn[q] = nu[q] * vt[(r + on) * Ww + c + on];
  }
  __syncthreads();
  double* out = s.out_jvp;
  const double cond = s.scal[S_COND];
  const auto* om = glb(s.omega);
#pragma unroll
  for (int i = 0; i < NO; ++i) {
    const int q = threadIdx.x + 256 * i;
    const int k = kr[i];
    if (k < 0) continue;
    const int r = q / TS, c = q - r * TS;
    const int ra = r + G::R1, ca = c + G::R1, rn = r + P, cn_ = c + P;
    const T adv = -ih * (dx1<P, T>(fa, Ww, ra, ca) + dy1<P, T>(fb, Ww, ra, ca));
    const T vv = vt[ra * Ww + ca];
    const T nv = nu[rn * Wn + cn_];
    const T diff = T(0.5) * ih2 * (lap5<P, T>(cn, Wn, rn, cn_) + nv * lap5<P, T>(vt, Ww, ra, ca) -
                                   vv * lap5<P, T>(nu, Wn, rn, cn_));
    double o = (double)(adv + diff);
    if (cond != 0.0) {
      const double rk = om[k];
      o -= check_done ? cond * ((6.0 * rk * rk - 6.0 * rk + 1.0) * (double)vv)
                      : cond * (rk * (rk - 1.0) * (2.0 * rk - 1.0));
    }
    out[k] = o;
  }
}

template <int P, typename T, int TS>
static hipError_t scalar_ts(const Batch& b, int N, int check_done, hipStream_t st) {
  const int nt = (N / TS) * (N / TS);
  using G = Geo<P>;
  const size_t Ww = TS + 2 * G::R1, Wn = TS + 2 * P;
  const size_t lds = (3 * Ww * Ww + 2 * Wn * Wn) * sizeof(T);   // v~, both fluxes; kappa, kappa v~
  hipLaunchKernelGGL((k_scalar<P, T, TS>), dim3(nt * b.n), dim3(256), lds, st, b, check_done);
  return hipGetLastError();
}

template <int P, typename T>
static hipError_t scalar_t(const Batch& b, const LaunchCfg& c, int check_done, hipStream_t st) {
  const int N = 1 << c.J;
  const int TS = c.tile;     // the tile the solves were laid out with
  if (!tile_valid(c.J, c.p, c.prec, TS)) return hipErrorInvalidValue;
  if (TS == 32) return scalar_ts<P, T, 32>(b, N, check_done, st);
  if (TS == 16) return scalar_ts<P, T, 16>(b, N, check_done, st);
  return scalar_ts<P, T, 8>(b, N, check_done, st);
}

hipError_t launch_scalar(const Batch& b, const LaunchCfg& c, int check_done, hipStream_t st) {
  if (c.prec == 0) return c.p == 2 ? scalar_t<2, double>(b, c, check_done, st) : scalar_t<3, double>(b, c, check_done, st);
  return c.p == 2 ? scalar_t<2, float>(b, c, check_done, st) : scalar_t<3, float>(b, c, check_done, st);
}

// fill n elements of a bulk field with a constant
template <typename T>
__global__ void k_fill(T* f, size_t n, double value) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    f[i] = (T)value;
}

hipError_t launch_fill(void* f, size_t n, int prec, double value, hipStream_t st) {
  const size_t gb = (n + 255) / 256;
  const int g = (int)(gb < 4096 ? gb : 4096);
  if (prec == 0) hipLaunchKernelGGL(k_fill<double>, dim3(g), dim3(256), 0, st, static_cast<double*>(f), n, value);
  else hipLaunchKernelGGL(k_fill<float>, dim3(g), dim3(256), 0, st, static_cast<float*>(f), n, value);
  return hipGetLastError();
}

template <int P, typename T, int TS, bool FIELDS>
static void rhs_launch(const Batch& b, int nt, hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    // FP32 bulk fields: the residual itself runs in FP64 (k_rhs R64)
    // on grids of 2048^2 and up, 1024 threads: the LDS of the FP64 tiles
    // holds two blocks per CU, 32 wavefronts against 8 with 256 threads
    const size_t lds = rhs_lds_elems<P, double>(TS) * sizeof(double);
    if (nt * TS * TS >= (1 << 22))
      hipLaunchKernelGGL((k_rhs<P, double, TS, true, FIELDS, 1024>), dim3((nt) * b.n), dim3(1024), lds, st, b);
    else
      hipLaunchKernelGGL((k_rhs<P, double, TS, true, FIELDS>), dim3((nt) * b.n), dim3(256), lds, st, b);
  } else {
    const size_t lds = rhs_lds_elems<P, T>(TS) * sizeof(T);
    hipLaunchKernelGGL((k_rhs<P, T, TS, false, FIELDS>), dim3((nt) * b.n), dim3(256), lds, st, b);
  }
}

template <int P, typename T, int TS>
static hipError_t rhs_ts(const Batch& b, int N, bool jvp, bool exact, hipStream_t st, bool fields = false) {
  const int nt = (N / TS) * (N / TS);
  if (!jvp) {
    if (fields) rhs_launch<P, T, TS, true>(b, nt, st);
    else rhs_launch<P, T, TS, false>(b, nt, st);
  } else if (!exact) {
    // FP32 products on 32-edge tiles of grids of 2048^2 and up: 512 threads,
    // two output nodes each (the LDS of a block allows four resident blocks,
    // 32 wavefronts per CU, against 20 with 256 threads).  Measured 2% faster
    // there, 2% slower on the sparse 512^2 batch, which keeps 256.
    const size_t lds = jvp_lds_elems<P, T>(TS) * sizeof(T);
    bool wide = false;
    if constexpr (sizeof(T) == 4 && TS == 32) {
      wide = N >= 2048;
      if (wide) hipLaunchKernelGGL((k_jvp<P, T, TS, false, 512>), dim3((nt) * b.n), dim3(512), lds, st, b);
    }
    if (!wide) hipLaunchKernelGGL((k_jvp<P, T, TS, false>), dim3((nt) * b.n), dim3(256), lds, st, b);
  } else {
    hipLaunchKernelGGL((k_nuprime<P, T, TS>), dim3((nt) * b.n), dim3(256), 0, st, b);
    const size_t lds = jvp_lds_elems<P, T>(TS, true) * sizeof(T);
    hipLaunchKernelGGL((k_jvp<P, T, TS, true>), dim3((nt) * b.n), dim3(256), lds, st, b);
  }
  return hipGetLastError();
}

template <int P, typename T>
static hipError_t rhs_t(const Batch& b, const LaunchCfg& c, bool jvp, hipStream_t st, bool fields = false) {
  const int N = 1 << c.J;
  const int TS = c.tile;     // the tile the solves were laid out with
  if (!tile_valid(c.J, c.p, c.prec, TS)) return hipErrorInvalidValue;
  const bool exact = jvp && c.jac == 1;
  if (TS == 32) return rhs_ts<P, T, 32>(b, N, jvp, exact, st, fields);
  if (TS == 16) return rhs_ts<P, T, 16>(b, N, jvp, exact, st, fields);
  return rhs_ts<P, T, 8>(b, N, jvp, exact, st, fields);
}

static hipError_t rhs_dispatch(const Batch& b, const LaunchCfg& c, bool jvp, hipStream_t st, bool fields = false) {
  if (c.prec == 0)
    return c.p == 2 ? rhs_t<2, double>(b, c, jvp, st, fields) : rhs_t<3, double>(b, c, jvp, st, fields);
  return c.p == 2 ? rhs_t<2, float>(b, c, jvp, st, fields) : rhs_t<3, float>(b, c, jvp, st, fields);
}

// Level-adapted evaluation (k_adapted.hip): the local levels of the step's
// active set, the residual's fields on the dense grid, then the residual at
// the active nodes; the products at the active nodes.
hipError_t launch_rhs(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  if (!c.adapt) return rhs_dispatch(b, c, false, st);
  hipError_t e;
  if ((e = launch_local_level(b, c, st)) != hipSuccess) return e;
  if ((e = rhs_dispatch(b, c, false, st, true)) != hipSuccess) return e;
  return launch_rhs_adapted(b, c, st);
}
hipError_t launch_jvp(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  if (c.adapt) return launch_jvp_adapted(b, c, st);
  return rhs_dispatch(b, c, true, st);
}

// ------------------------------------------------------------- diagnostics
// One block per row y of the FP64 field dense64 and its FP64 velocity
// vel64: row sums of w, u^2 + v^2, w^2, |grad w|^2 and the row max of |w|
// (Sections 3.3, 3.4).  The host adds the rows in order.
template <int P>
__global__ void __launch_bounds__(256) k_diag(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int N = s.N, nm = N - 1, y = MRA_BX(b);
  const double* w = s.dense64;
  const double* vu = s.vel64;
  const double* vv = s.vel64 + (size_t)N * N;
  const double ih = 1.0 / s.h;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
  for (int x = threadIdx.x; x < N; x += blockDim.x) {
    double gx = 0, gy = 0;
    for (int n = 1; n <= 2 * P - 2; ++n) {
      const double cn = d1c<P, double>(n);
      gy += cn * (w[((y + n) & nm) * N + x] - w[((y - n) & nm) * N + x]);
      gx += cn * (w[y * N + ((x + n) & nm)] - w[y * N + ((x - n) & nm)]);
    }
    gx *= ih; gy *= ih;
    const double u = vu[y * N + x], v = vv[y * N + x];
    const double wv = w[y * N + x];
    a0 += wv;
    a1 += u * u + v * v;
    a2 += wv * wv;
    a3 += gx * gx + gy * gy;
    a4 = fmax(a4, fabs(wv));
  }
  __shared__ double red[5][256];
  red[0][threadIdx.x] = a0; red[1][threadIdx.x] = a1; red[2][threadIdx.x] = a2;
  red[3][threadIdx.x] = a3; red[4][threadIdx.x] = a4;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
      red[4][threadIdx.x] = fmax(red[4][threadIdx.x], red[4][threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 5) s.diag[y * 5 + threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_diag(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  const int N = 1 << c.J;
  if (c.p == 2) hipLaunchKernelGGL(k_diag<2>, dim3((N) * b.n), dim3(256), 0, st, b);
  else hipLaunchKernelGGL(k_diag<3>, dim3((N) * b.n), dim3(256), 0, st, b);
  return hipGetLastError();
}

// ----------------------------------------------------------- centre tracking
// One block per row y of the FP64 field dense64: each node is given to the
// nearest of the K previous centres (periodic distance, ties to the lower
// index) and adds max(w, 0), and that weight times its periodic displacement
// from the centre, to the centre's row sums.  Row sums go to rows[y][K][3];
// the host adds the rows in order (Section 3.2: separation of the centres).
struct Centres {
  double x[kMaxTrack], y[kMaxTrack];
  int k;
};

__device__ inline double periodic_delta(double a, double c, double L) {
  const double t = a - c + 0.5 * L;
  return t - L * floor(t / L) - 0.5 * L;
}

__global__ void __launch_bounds__(256) k_track(Batch b, Centres cs, double* rows) {
  const SolveDev& s = MRA_SOLVE(b);
  const int N = s.N, y = MRA_BX(b);
  const double L = s.length, h = s.h;
  const double* w = s.dense64;
  double acc[kMaxTrack][3];
#pragma unroll
  for (int k = 0; k < kMaxTrack; ++k) acc[k][0] = acc[k][1] = acc[k][2] = 0.0;
  const double yy = y * h;
  for (int x = threadIdx.x; x < N; x += blockDim.x) {
    const double xx = x * h;
    int best = 0;
    double bd = 0.0, bx = 0.0, by = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxTrack; ++k) {
      if (k >= cs.k) break;
      const double dx = periodic_delta(xx, cs.x[k], L), dy = periodic_delta(yy, cs.y[k], L);
      const double d2 = dx * dx + dy * dy;
      if (k == 0 || d2 < bd) { best = k; bd = d2; bx = dx; by = dy; }
    }
    const double wv = fmax(w[y * N + x], 0.0);
#pragma unroll
    for (int k = 0; k < kMaxTrack; ++k)
      if (k == best) { acc[k][0] += wv; acc[k][1] += wv * bx; acc[k][2] += wv * by; }
  }
  __shared__ double red[kMaxTrack * 3][256];
#pragma unroll
  for (int k = 0; k < kMaxTrack; ++k)
    for (int c = 0; c < 3; ++c) red[k * 3 + c][threadIdx.x] = acc[k][c];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int q = 0; q < kMaxTrack * 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + o];
    __syncthreads();
  }
  if ((int)threadIdx.x < cs.k * 3) rows[(size_t)y * cs.k * 3 + threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_track(const Batch& b, const LaunchCfg& c, const double* cx, const double* cy, int k,
                        double* rows, hipStream_t st) {
  if (k < 1 || k > kMaxTrack) return hipErrorInvalidValue;
  Centres cs{};
  for (int i = 0; i < k; ++i) { cs.x[i] = cx[i]; cs.y[i] = cy[i]; }
  cs.k = k;
  hipLaunchKernelGGL(k_track, dim3((1 << c.J) * b.n), dim3(256), 0, st, b, cs, rows);
  return hipGetLastError();
}

}  // namespace mra
