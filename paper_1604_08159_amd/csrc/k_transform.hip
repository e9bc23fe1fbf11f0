// DD multiresolution kernels for gfx950: forward transform with the
// significance test and order-preserving compaction of the active set,
// inverse transform, nodal prolongation Pi, scatter / gather between the
// active list and the dense finest grid.
//
// Section 2.4 and eq. (6): nested dyadic meshes, DD prediction of order 2p
// from the next coarser mesh, details d = u - P(u|G^{l-1}), and the filtered
// trial solution whose unknowns are the nodal values at the active nodes.
//
// All levels of the forward transform are independent (coarse values are
// samples), so one launch covers every packed position.  The prolongation is
// sequential in the level: the levels up to kCoarseLevels are done by one
// workgroup per solve, finer levels by one launch each.
#include <type_traits>

#include "mra_internal.hpp"

namespace mra {

__global__ void k_write_desc(SolveDev* dst, SolveDev src) { *dst = src; }

hipError_t launch_write_desc(SolveDev* dst, const SolveDev& src, hipStream_t st) {
  hipLaunchKernelGGL(k_write_desc, dim3(1), dim3(1), 0, st, dst, src);
  return hipGetLastError();
}

template <typename T>
__device__ inline T* dense_target(const SolveDev& s, int target) {
  if (target == 0) return reinterpret_cast<T*>(s.wt);
  if (target == 1) return reinterpret_cast<T*>(s.vt);
  if (target == 3) return reinterpret_cast<T*>(s.res64);
  return reinterpret_cast<T*>(s.dense64);
}

// ------------------------------------------------------- active values
// The value of active node k in the prolongation of: src 0 the state omega,
// src 1 the first Arnoldi vector F * inv (inv = 0: no basis), src 2 a caller
// vector, src 3 basis slot j (for j > 0 the first-pass residual r_j that the
// Gram-Schmidt normalises after its product).  Vd is V_j of an FP64 basis; callers read a basis stored
// in FP32 (Vf) themselves.  Both pointers are taken once per kernel, so no
// descriptor load is repeated after a store.
__device__ inline double active_value(const SolveDev& s, int src, int k, double inv, const double* Vd) {
  if (src == 0) return glb(s.omega)[k];
  if (src == 2) return glb(s.vin)[k];
  if (src == 3) return glb(Vd)[k];
  return inv == 0.0 ? 0.0 : glb(s.w)[k] * inv;
}
// entry k of V_j, whichever precision the basis is stored in
__device__ inline double basis_value(const double* Vd, const float* Vf, int k) {
  return Vf ? (double)glb(Vf)[k] : glb(Vd)[k];
}
__device__ inline void basis_store(double* Vd, float* Vf, int k, double v) {
  if (Vf) glb(Vf)[k] = (float)v;
  else glb(Vd)[k] = v;
}

// ---------------------------------------------------------------- prolong
// mode 0: Pi (inactive nodes predicted, active nodes take their value);
// mode 1: inverse transform (every node = detail + prediction, details from
// the packed input in s.spec).
template <int P, typename T>
__device__ inline void prolong_node(T* __restrict__ f, const T* __restrict__ packed, int i, int l, int J,
                                    int j0) {
#pragma clang fp contract(off)
  int lv;
  const int fi = packed_to_fine(i, J, j0, &lv);
  const int N = 1 << J;
  const T pr = predict_node<P, T>(f, fi & (N - 1), fi >> J, l, J);
  f[fi] = packed[i] + pr;
}

// Inverse transform, levels j0+1 .. Lc (Lc = min(J, kCoarseLevels)), one
// block per solve: the 2^Lc x 2^Lc sub-grid of stride 2^(J-Lc) is swept in
// LDS (node = detail + prediction) and written back.  (mode 0, the
// prolongation of a source vector on the coarse levels, is kept for
// completeness; the step uses k_prolong_tiles.)
template <int P, typename T>
__global__ void __launch_bounds__(1024) k_prolong_coarse(Batch b, int target, int lmax, int mode, int src, int j) {
  const SolveDev& s = MRA_SOLVE(b);
  T* f = dense_target<T>(s, target);
  const T* packed = mode == 1 ? reinterpret_cast<const T*>(s.spec) : nullptr;
  const int J = s.J, j0 = s.j0;
  const int Lc = lmax < J ? lmax : J;
  const int n = 1 << Lc, S = 1 << (J - Lc);
  const int cnt = 1 << (2 * Lc);
  __shared__ T val[1 << (2 * kCoarseLevels)];
  __shared__ uint8_t act[1 << (2 * kCoarseLevels)];
  const int n0sq = 1 << (2 * j0);
  double inv = 0.0;
  if (mode == 0 && src == 1) {
    inv = first_scale(s, 0);
    if (threadIdx.x == 0) s.scal[S_INV] = inv;
  }
  double* Vd = s.V ? s.V + (size_t)j * s.vs : nullptr;
  float* Vf = s.V32 ? s.V32 + (size_t)j * s.vs : nullptr;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int fi = packed_to_fine(i, J, j0, nullptr);
    const int sub = ((fi >> J) / S) * n + (fi & (s.N - 1)) / S;
    const bool a = mode == 0 ? s.mask[i] != 0 : i < n0sq;
    act[sub] = a;
    if (a) {
      if (mode == 0) {
        const int k = s.rank[fi];
        const double v = src == 3 ? basis_value(Vd, Vf, k) : active_value(s, src, k, inv, Vd);
        if (src == 1 && inv != 0.0) basis_store(Vd, Vf, k, v);
        val[sub] = (T)v;
      } else {
        val[sub] = f[fi];
      }
    }
  }
  __syncthreads();
  for (int l = j0 + 1; l <= Lc; ++l) {
    const int lo = 1 << (2 * (l - 1)), hi = 1 << (2 * l);
    for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      int lv;
      const int sf = packed_to_fine(i, Lc, j0, &lv);   // node of the sub-grid
      if (act[sf]) continue;
      const T pr = predict_node<P, T>(val, sf & (n - 1), sf >> Lc, l, Lc);
      val[sf] = mode == 0 ? pr : packed[i] + pr;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int fi = packed_to_fine(i, J, j0, nullptr);
    f[fi] = val[((fi >> J) / S) * n + (fi & (s.N - 1)) / S];
  }
}

// Pi in one launch: one block per B x B tile of the finest grid (B =
// min(N, 32)) sweeps the lattices of levels j0 .. J in LDS, each a halo wider
// than the next (the reach of the next level's prediction), and writes the
// tile.  The level-j0 lattice is all active.  Halo nodes are recomputed by
// every tile that needs them, with identical arithmetic, so all tiles agree.
// Active nodes take their value through the rank map; for src 1 (the first
// Arnoldi vector) every block derives beta from the partial sums of k_norm0
// (block 0 records it) and the tile that owns a node writes its entry of V_0;
// later Arnoldi vectors (src 3) are read from V_j as the Gram-Schmidt stage
// wrote them.  The kernel is specialised per grid level J: every lattice
// size, halo and shift is a compile-time constant.
// FP32 tiles are 64 wide with 512 threads: against 32-wide tiles with 256
// threads a quarter of the blocks, each with 4 waves more, and fewer halo
// nodes per tile node (Pi per launch: 25.7 against 30.9 us for 24 solves of
// 512^2, 54 against 66 us for two of 2048^2; 1024 threads: 30.0 and 60 us).
// FP64 tiles stay 32 wide with 256 threads (their lattices take twice the LDS).
constexpr int kFineTile = 64;                      // tile edge of the FP32 prolongation
constexpr int kPiThreads = 512;                    // its threads per block
template <typename T> constexpr int pi_tile() { return sizeof(T) == 4 ? kFineTile : 32; }
template <typename T> constexpr int pi_threads() { return sizeof(T) == 4 ? kPiThreads : 256; }

// halo E_l of the level-l lattice (fine units) and its node count per side
// (independent of the tile offset; checked on the host for every offset)
__host__ __device__ constexpr int lat_halo(int J, int P, int l) {
  int E = 0;
  for (int q = J; q > l; --q) E += (2 * P - 1) << (J - q);
  return E;
}
__host__ __device__ constexpr int lat_floor(int v, int sh) {   // largest multiple of 2^sh <= v
  return v >= 0 ? (v >> sh) << sh : -((((-v) + (1 << sh) - 1) >> sh) << sh);
}
__host__ __device__ constexpr int lat_count(int J, int P, int B, int x0, int l) {
  const int sh = J - l, E = lat_halo(J, P, l);
  const int lo = x0 - E, hi = x0 + B - 1 + E;
  return ((hi - lat_floor(lo, sh)) >> sh) + 1;
}
template <int J, int P, int L>
__device__ inline int lat_origin(int x0) {
  constexpr int SH = J - L, E = lat_halo(J, P, L);
  return ((x0 - E) >> SH) << SH;         // floor to the lattice (arithmetic shift)
}

// Level L of the sweep (lattice of level L - 1 in buf[cur]), then the next.
// The tensor-product prediction is separable: pass 1 fills `half`, the level-L
// rows of the level-(L - 1) columns (a sample on even rows, the y-prediction
// on odd rows); pass 2 takes every node of level L from its row of `half` (a
// copy on even columns, the x-prediction on odd columns).  Odd-odd nodes thus
// get the x-prediction of the y-predictions, the canonical order, and every
// y-prediction is computed once per column instead of once per neighbour.
// Active nodes then take their value.
//
// Work is dealt in pairs: a node on the coarse lattice and the predicted node
// after it (two rows of one column in pass 1, two columns of one row in pass
// 2).  Both come from one window of 2P coarse values, the sample being the
// window's entry P - 1, so no lane branches on parity and a pair costs one
// window of loads.
//
// Pair geometry of level L along one axis: the level-L lattice starts at o
// (n nodes, spacing SV), the level-(L - 1) lattice at po (pn nodes, spacing
// 2 SV), and D = (o - po) / SV.  Pair jj holds lattice nodes 2 jj - e and
// 2 jj + 1 - e (e = D & 1) and coarse node (D >> 1) + jj.  Where 2 SV <= B
// every tile origin is a multiple of 2 SV, so D is a compile-time constant and
// the pairs cover the lattice exactly; on coarser levels D varies with the
// tile and one more pair is dealt.  A pair member outside the lattice (node
// -1, n or n + 1) is computed from in-buffer values and lands in a padding
// column or row that nothing reads as a value: lattice rows hold columns
// -1 .. n + 1 (stride n + 3) and P + 2 spare rows for the windows of such
// members; rows of `half` hold the coarse columns and the reach of such a
// window (stride pn + P + 1), and rows -1 .. n + 1.
template <int J, int P, int L, int B> struct Lvl {
  static constexpr int SH = J - L, SV = 1 << SH;
  static constexpr int n = lat_count(J, P, B, 0, L), pn = lat_count(J, P, B, 0, L - 1);
  static constexpr bool FIX = 2 * SV <= B;
  static constexpr int D0 = (lat_floor(-lat_halo(J, P, L), SH) - lat_floor(-lat_halo(J, P, L - 1), SH + 1)) >> SH;
  static constexpr int np = FIX ? ((D0 + n - 1) >> 1) - (D0 >> 1) + 1 : n / 2 + 1;
  static constexpr int RS = n + 3, RSP = pn + 3, RH = pn + P + 1;
};
template <int J, int P, int L, int B>
__device__ __forceinline__ int lvl_d(int x0) {
  using G = Lvl<J, P, L, B>;
  if constexpr (G::FIX) return G::D0;
  else return (lat_origin<J, P, L>(x0) - lat_origin<J, P, L - 1>(x0)) >> G::SH;
}
// coarsest swept lattice (every node of it active) and the LDS of the sweep:
// two lattice buffers (levels J0 .. J - 1; level J goes straight to the
// output) and the half-predicted lattice of each level
template <int P> constexpr int pi_j0() { return P == 2 ? 2 : 3; }
template <int J, int P, int TB> constexpr int pi_buf_len() {
  constexpr int B = (1 << J) < TB ? (1 << J) : TB;
  int m = 1;
  for (int l = pi_j0<P>(); l < J; ++l) {
    const int n = lat_count(J, P, B, 0, l), len = (n + P + 2) * (n + 3);
    m = len > m ? len : m;
  }
  return m;
}
template <int J, int P, int TB> constexpr int pi_half_len() {
  constexpr int B = (1 << J) < TB ? (1 << J) : TB;
  int m = 1;
  for (int L = pi_j0<P>() + 1; L <= J; ++L) {
    const int len = (lat_count(J, P, B, 0, L) + 3) * (lat_count(J, P, B, 0, L - 1) + P + 1);
    m = len > m ? len : m;
  }
  return m;
}
// pass-2 pairs of level L per thread
template <int J, int P, int L, int TB, int NT>
__host__ __device__ constexpr int pair_slots() {
  using G = Lvl<J, P, L, ((1 << J) < TB ? (1 << J) : TB)>;
  return (G::n * G::np + NT - 1) / NT;
}

template <typename T> using vec2 = T __attribute__((ext_vector_type(2)));

// Ranks of the two nodes of each of this thread's pass-2 pairs of level L (-1
// for a node of a coarser level, a node outside the lattice, a slot past the
// pairs).
template <int S> struct Ranks {
  int c[S], p[S];
};
template <int J, int P, int L, int TB, int NT>
__device__ __forceinline__ Ranks<pair_slots<J, P, L, TB, NT>()> level_ranks(const SolveDev& s, int x0, int y0) {
  constexpr int N = 1 << J, NM = N - 1, B = N < TB ? N : TB;
  using G = Lvl<J, P, L, B>;
  constexpr int NQ = G::n * G::np, S = pair_slots<J, P, L, TB, NT>();
  const int ox = lat_origin<J, P, L>(x0), oy = lat_origin<J, P, L>(y0);
  const int ex = lvl_d<J, P, L, B>(x0) & 1;
  const auto* __restrict__ rank = glb(s.rank);
  Ranks<S> r;
#pragma unroll
  for (int i = 0; i < S; ++i) {
    const int q = threadIdx.x + NT * i;
    r.c[i] = -1;
    r.p[i] = -1;
    if (NQ % NT == 0 || i + 1 < S || q < NQ) {
      const int iy = q / G::np, jj = q - iy * G::np;
      const int ixc = 2 * jj - ex;
      const int y = oy + (iy << G::SH), xc = ox + (ixc << G::SH);
      const int row = (y & NM) * N;
      if constexpr (L == J) {
        // the finest pair is two neighbours inside the tile, the first at an even x
        const vec2<int> kk = *glb(reinterpret_cast<const vec2<int>*>(s.rank + row + xc));
        r.c[i] = (y & 1) ? kk.x : -1;
        r.p[i] = kk.y;
      } else {
        if ((y & G::SV) && ixc >= 0 && ixc < G::n) r.c[i] = rank[row + (xc & NM)];
        if (ixc + 1 < G::n) r.p[i] = rank[row + ((xc + G::SV) & NM)];
      }
    }
  }
  return r;
}

// Raw source values of a level's new active nodes (before the first basis
// vector's scale is applied): FP64, or FP32 for a basis stored in FP32.
template <int S, bool FB> struct RawVals {
  double c[S], p[S];
  float fc[FB ? S : 1], fp[FB ? S : 1];
};
template <int S, bool FB>
__device__ __forceinline__ RawVals<S, FB> level_values(const SolveDev& s, const Ranks<S>& kr, int src,
                                                       const double* Vd, const float* Vf) {
  RawVals<S, FB> rv;
  if (FB && src == 3) {
    // loaded raw: a conversion next to the load would wait for each in turn
#pragma unroll
    for (int i = 0; i < S; ++i) {
      rv.fc[i] = 0.0f;
      rv.fp[i] = 0.0f;
      if (kr.c[i] >= 0) rv.fc[i] = glb(Vf)[kr.c[i]];
      if (kr.p[i] >= 0) rv.fp[i] = glb(Vf)[kr.p[i]];
    }
  } else {
    const double* base = src == 0 ? s.omega : (src == 2 ? s.vin : (src == 3 ? Vd : s.w));
#pragma unroll
    for (int i = 0; i < S; ++i) {
      rv.c[i] = 0.0;
      rv.p[i] = 0.0;
      if (kr.c[i] >= 0) rv.c[i] = glb(base)[kr.c[i]];
      if (kr.p[i] >= 0) rv.p[i] = glb(base)[kr.p[i]];
    }
  }
  return rv;
}


// The sweep keeps two levels of loads in flight: at level L the values of
// level L + 1 (whose ranks arrived during level L - 1) and the ranks of level
// L + 2 are issued before L's passes, so no global load sits on the path
// between two levels.  kin, vin: ranks and raw values of level L; kn1: ranks
// of level L + 1.  inv is uniform over the block (1 / beta for src 1).
template <int J, int L> constexpr int lvl_cap() { return L < J ? L : J; }
template <int P, typename T, int J, int L, bool FB, int TB, int NT>
__device__ __forceinline__ void prolong_level_ct(const SolveDev& s, T (*buf)[pi_buf_len<J, P, TB>()], T* half,
                                                 int cur, int x0, int y0, int src, double inv, double* Vd, float* Vf,
                                                 T* f, const Ranks<pair_slots<J, P, L, TB, NT>()>& kin,
                                                 const RawVals<pair_slots<J, P, L, TB, NT>(), FB>& vin,
                                                 const Ranks<pair_slots<J, P, lvl_cap<J, L + 1>(), TB, NT>()>& kn1) {
#pragma clang fp contract(off)
  constexpr int N = 1 << J, B = N < TB ? N : TB;
  using G = Lvl<J, P, L, B>;
  constexpr int SH = G::SH, SV = G::SV, n = G::n, pn = G::pn, np = G::np;
  constexpr int RS = G::RS, RSP = G::RSP, RH = G::RH;
  constexpr int N1 = np * pn, S1 = (N1 + NT - 1) / NT;               // pass 1: (row pair, coarse column)
  constexpr int N2 = n * np, S2 = pair_slots<J, P, L, TB, NT>();     // pass 2: (row, column pair)
  static_assert(S2 <= 16, "too many pairs of one level per thread");
  static_assert(L == J || (n + P + 2) * RS <= pi_buf_len<J, P, TB>(), "lattice of one level exceeds its buffer");
  static_assert((n + 3) * RH <= pi_half_len<J, P, TB>(), "half-predicted lattice exceeds its buffer");
  static_assert(L < J || (G::FIX && (G::D0 & 1) == 0 && 2 * np == n), "finest pairs are neighbours in the tile");
  const T* prev = buf[cur];
  T* nxt = buf[cur ^ 1];
  constexpr int L1 = lvl_cap<J, L + 1>(), L2 = lvl_cap<J, L + 2>();
  RawVals<pair_slots<J, P, L1, TB, NT>(), FB> vn1;
  Ranks<pair_slots<J, P, L2, TB, NT>()> kn2;
  if constexpr (L < J) vn1 = level_values<pair_slots<J, P, L1, TB, NT>(), FB>(s, kn1, src, Vd, Vf);
  if constexpr (L + 1 < J) kn2 = level_ranks<J, P, L2, TB, NT>(s, x0, y0);
  // pass 1: a sample row and a y-predicted row of one coarse column
  {
    const int dy = lvl_d<J, P, L, B>(y0);
    const int jr0 = (dy >> 1) - (P - 1), ey = dy & 1;
#pragma unroll
    for (int i = 0; i < S1; ++i) {
      const int q = threadIdx.x + NT * i;
      if (N1 % NT == 0 || i + 1 < S1 || q < N1) {
        const int rp = q / pn, c = q - rp * pn;
        const T* w = prev + (jr0 + rp) * RSP + c + 1;
        T cc[2 * P];
#pragma unroll
        for (int o = 0; o < 2 * P; ++o) cc[o] = w[o * RSP];
        T* h = half + (2 * rp - ey + 1) * RH + c;
        h[0] = cc[P - 1];
        h[RH] = dd_pred<P, T>(cc);
      }
    }
  }
  __syncthreads();
  // pass 2: a sample and an x-predicted node of one level-L row
  const int dx = lvl_d<J, P, L, B>(x0);
  const int jc0 = (dx >> 1) - (P - 1), ex = dx & 1;
  const bool s1 = src == 1, keep = s1 && inv != 0.0;
  const bool fsrc = FB && src == 3;
#pragma unroll
  for (int i = 0; i < S2; ++i) {
    const int q = threadIdx.x + NT * i;
    if (N2 % NT == 0 || i + 1 < S2 || q < N2) {
      const int iy = q / np, jj = q - iy * np;
      const T* w = half + (iy + 1) * RH + jc0 + jj;
      T cc[2 * P];
#pragma unroll
      for (int o = 0; o < 2 * P; ++o) cc[o] = w[o];
      T vc = cc[P - 1], vp = dd_pred<P, T>(cc);
      const int ixc = 2 * jj - ex;
      // active nodes take their value
      T ac, ap;
      if (fsrc) {
        ac = (T)vin.fc[i];
        ap = (T)vin.fp[i];
      } else {
        double dc = vin.c[i], dp = vin.p[i];
        if (s1) {
          dc = inv == 0.0 ? 0.0 : dc * inv;
          dp = inv == 0.0 ? 0.0 : dp * inv;
        }
        ac = (T)dc;
        ap = (T)dp;
        if (keep) {
          // the first basis vector, at this tile's own nodes
          const int ox = lat_origin<J, P, L>(x0), oy = lat_origin<J, P, L>(y0);
          const int y = oy + (iy << SH), xc = ox + (ixc << SH), xp = xc + SV;
          const bool rin = y >= y0 && y < y0 + B;
          if (kin.c[i] >= 0 && rin && xc >= x0 && xc < x0 + B) {
            if constexpr (FB) glb(Vf)[kin.c[i]] = (float)dc;
            else glb(Vd)[kin.c[i]] = dc;
          }
          if (kin.p[i] >= 0 && rin && xp >= x0 && xp < x0 + B) {
            if constexpr (FB) glb(Vf)[kin.p[i]] = (float)dp;
            else glb(Vd)[kin.p[i]] = dp;
          }
        }
      }
      vc = kin.c[i] >= 0 ? ac : vc;
      vp = kin.p[i] >= 0 ? ap : vp;
      if constexpr (L == J) {
        // finest lattice = the tile; the pair is two neighbours, the first at an even x
        *glb(reinterpret_cast<vec2<T>*>(f + (y0 + iy) * N + x0 + ixc)) = vec2<T>{vc, vp};
      } else {
        T* o = nxt + iy * RS + ixc + 1;
        o[0] = vc;
        o[1] = vp;
      }
    }
  }
  if constexpr (L < J) {
    __syncthreads();
    prolong_level_ct<P, T, J, L + 1, FB, TB, NT>(s, buf, half, cur ^ 1, x0, y0, src, inv, Vd, Vf, f, kn1, vn1,
                                                 kn2);
  }
}

// 1 / beta of the first basis vector, the same in every lane
__device__ inline double lane_uniform(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int P, typename T, int J, bool FB, int TB = pi_tile<T>(), int NT = pi_threads<T>()>
__global__ void __launch_bounds__(NT) k_prolong_tiles(Batch b, int target, int src, int j) {
#pragma clang fp contract(off)
  constexpr int N = 1 << J, NM = N - 1, B = N < TB ? N : TB, NTX = N / B;
  constexpr int J0 = pi_j0<P>();
  constexpr int pn = lat_count(J, P, B, 0, J0), SH0 = J - J0, RS0 = pn + 3;
  static_assert(pn * pn <= NT, "coarsest lattice exceeds one node per thread");
  static_assert(lat_count(J, P, B, 0, J) == B, "finest lattice is the tile");
  __shared__ T buf[2][pi_buf_len<J, P, TB>()];
  __shared__ T half[pi_half_len<J, P, TB>()];
  const SolveDev& s = MRA_SOLVE(b);
  // tiles in XCD-aware order: neighbours, which read each other's halo ranks
  // and values, share an L2
  const int t = tile_of_block(MRA_BX(b), NTX * NTX, b.n);
  const int x0 = (t % NTX) * B, y0 = (t / NTX) * B;
  T* f = dense_target<T>(s, target);
  double* Vd = s.V ? s.V + (size_t)j * s.vs : nullptr;      // V_j, FP64 basis
  float* Vf = s.V32 ? s.V32 + (size_t)j * s.vs : nullptr;   // V_j, FP32 basis
  const int pox = lat_origin<J, P, J0>(x0), poy = lat_origin<J, P, J0>(y0);
  // the coarsest lattice (all active, at most 256 nodes): rank and raw value
  // of this thread's node are fetched while the scale is being reduced
  const bool has0 = (int)threadIdx.x < pn * pn;
  int x0n = 0, y0n = 0, k0n = 0, q0 = 0;
  double raw = 0.0;
  // the first two swept levels' ranks, in flight meanwhile
  const auto k1 = level_ranks<J, P, J0 + 1, TB, NT>(s, x0, y0);
  Ranks<pair_slots<J, P, lvl_cap<J, J0 + 2>(), TB, NT>()> k2;
  if constexpr (J0 + 1 < J) k2 = level_ranks<J, P, J0 + 2, TB, NT>(s, x0, y0);
  if (has0) {
    const int q = threadIdx.x;
    const int iy = q / pn, ix = q - iy * pn;
    q0 = iy * RS0 + ix + 1;
    x0n = pox + (ix << SH0);
    y0n = poy + (iy << SH0);
    k0n = glb(s.rank)[(y0n & NM) * N + (x0n & NM)];
    raw = src == 0 ? glb(s.omega)[k0n]
                   : (src == 2 ? glb(s.vin)[k0n]
                               : (src == 3 ? (FB ? (double)glb(Vf)[k0n] : glb(Vd)[k0n]) : glb(s.w)[k0n]));
  }
  // A tile whose every node is active needs no sweep: each node takes its own
  // value.  Its stencil tiles (edge s.tile, dividing B) are then full.  On
  // grids of 1024^2 and up where most nodes are active, their counts are
  // loaded once the sweep's first loads are out and read after its first
  // barrier; elsewhere no tile is checked (on smaller grids the check's code
  // cost the sparse sweep more than it saved).
  constexpr bool kFullPath = J >= 10;
  __shared__ int tfull[kFullPath ? 64 : 1];
  const int ts = s.tile, nq = ts > 0 && B % ts == 0 ? B / ts : 0;
  bool cand = false;
  if constexpr (kFullPath) cand = nq > 0 && nq * nq <= 64 && 2 * *s.n_active > (int64_t)N * N;
  int tcv = 0;
  if (cand && (int)threadIdx.x < nq * nq) {
    const int a = threadIdx.x / nq, c = threadIdx.x - a * nq;
    tcv = glb(s.tile_count)[(y0 / ts + a) * s.ntx + x0 / ts + c];
  }
  const double inv = src == 1 ? lane_uniform(first_scale(s, t)) : 0.0;
  if (has0) {
    double a = raw;
    if (src == 1) {
      a = inv == 0.0 ? 0.0 : raw * inv;
      if (inv != 0.0 && x0n >= x0 && x0n < x0 + B && y0n >= y0 && y0n < y0 + B) {
        if constexpr (FB) glb(Vf)[k0n] = (float)a;
        else glb(Vd)[k0n] = a;
      }
    }
    buf[0][q0] = (T)a;
  }
  const auto v1 = level_values<pair_slots<J, P, J0 + 1, TB, NT>(), FB>(s, k1, src, Vd, Vf);
  if (cand && (int)threadIdx.x < nq * nq) tfull[threadIdx.x] = tcv == ts * ts;
  __syncthreads();
  bool full = cand;
  for (int i = 0; i < nq * nq && full; ++i) full = tfull[i] != 0;
  if (kFullPath && full) {
    // every rank, then every value, then the stores: a store between them
    // would order each load after it (the pointers may alias)
    constexpr int PT = (B * B + NT - 1) / NT;
    const auto* rank = glb(s.rank);
    const int nmine = (B * B - (int)threadIdx.x + NT - 1) / NT;   // nodes of this thread
    int fi[PT], kk[PT];
    double a[PT];
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int i = threadIdx.x + u * NT;
      fi[u] = (y0 + i / B) * N + x0 + i % B;
      if (u < nmine) kk[u] = rank[fi[u]];
    }
#pragma unroll
    for (int u = 0; u < PT; ++u)
      if (u < nmine) a[u] = (FB && src == 3) ? (double)glb(Vf)[kk[u]] : active_value(s, src, kk[u], inv, Vd);
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      if (u >= nmine) break;
      if (src == 1 && inv != 0.0) {
        if constexpr (FB) glb(Vf)[kk[u]] = (float)a[u];
        else glb(Vd)[kk[u]] = a[u];
      }
      glb(f)[fi[u]] = (T)a[u];
    }
    return;
  }
  prolong_level_ct<P, T, J, J0 + 1, FB, TB, NT>(s, buf, half, 0, x0, y0, src, inv, Vd, Vf, f, k1, v1, k2);
}

template <int P, typename T>
__global__ void __launch_bounds__(256) k_prolong_level(Batch b, int target, int l) {
  const SolveDev& s = MRA_SOLVE(b);
  T* f = dense_target<T>(s, target);
  const T* packed = reinterpret_cast<const T*>(s.spec);
  const int lo = 1 << (2 * (l - 1)), hi = 1 << (2 * l);
  const int i = lo + MRA_BX(b) * blockDim.x + threadIdx.x;
  if (i < hi) prolong_node<P, T>(f, packed, i, l, s.J, s.j0);
}

// coarse copy for the inverse transform: dense(coarse node) = packed[i]
template <typename T>
__global__ void k_inverse_coarse(Batch b, int target) {
  const SolveDev& s = MRA_SOLVE(b);
  T* f = dense_target<T>(s, target);
  const T* packed = reinterpret_cast<const T*>(s.spec);
  const int n0 = 1 << s.j0;
  for (int i = threadIdx.x; i < n0 * n0; i += blockDim.x) f[packed_to_fine(i, s.J, s.j0, nullptr)] = packed[i];
}

// Host check of k_prolong_tiles' assumptions for a grid, over every tile
// offset: each level's lattice count is the one the kernel was compiled for
// (the count at offset 0, so the x and y lattices of a tile have equal size).
static bool lattice_fits(int J, int P, int TB) {
  const int N = 1 << J, j0 = P == 2 ? 2 : 3;
  const int B = N < TB ? N : TB;
  for (int x0 = 0; x0 < N; x0 += B)
    for (int l = j0; l <= J; ++l)
      if (lat_count(J, P, B, x0, l) != lat_count(J, P, B, 0, l)) return false;
  return true;
}

template <int P, typename T, int J, bool FB>
static void prolong_j(const Batch& b, int target, int src, int j, hipStream_t st) {
  constexpr int TB = pi_tile<T>(), NT = pi_threads<T>();
  constexpr int N = 1 << J, B = N < TB ? N : TB;
  hipLaunchKernelGGL((k_prolong_tiles<P, T, J, FB>), dim3((N / B) * (N / B) * b.n), dim3(NT), 0, st, b, target,
                     src, j);
}

template <int P, typename T, bool FB>
static hipError_t prolong_p(const Batch& b, int J, int target, int src, int j, hipStream_t st) {
  switch (J) {
    case 3: if constexpr (P == 2) { prolong_j<P, T, 3, FB>(b, target, src, j, st); break; } return hipErrorInvalidValue;
    case 4: prolong_j<P, T, 4, FB>(b, target, src, j, st); break;
    case 5: prolong_j<P, T, 5, FB>(b, target, src, j, st); break;
    case 6: prolong_j<P, T, 6, FB>(b, target, src, j, st); break;
    case 7: prolong_j<P, T, 7, FB>(b, target, src, j, st); break;
    case 8: prolong_j<P, T, 8, FB>(b, target, src, j, st); break;
    case 9: prolong_j<P, T, 9, FB>(b, target, src, j, st); break;
    case 10: prolong_j<P, T, 10, FB>(b, target, src, j, st); break;
    case 11: prolong_j<P, T, 11, FB>(b, target, src, j, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The Arnoldi vectors (src 1 writes V_0, src 3 reads V_j) of a basis stored
// in FP32 take the FB kernels, which exist for FP32 tiles (the precision of
// such solves).
template <typename T>
static hipError_t prolong_t(const Batch& b, const LaunchCfg& c, int target, int src, int j, hipStream_t st) {
  if (!lattice_fits(c.J, c.p, pi_tile<T>())) return hipErrorInvalidValue;
  if ((src == 1 || src == 3) && c.vb) {
    if constexpr (std::is_same<T, float>::value)
      return c.p == 2 ? prolong_p<2, T, true>(b, c.J, target, src, j, st)
                      : prolong_p<3, T, true>(b, c.J, target, src, j, st);
    return hipErrorInvalidValue;
  }
  return c.p == 2 ? prolong_p<2, T, false>(b, c.J, target, src, j, st)
                  : prolong_p<3, T, false>(b, c.J, target, src, j, st);
}

// inverse transform: coarse copy, coarse kernel, one launch per finer level
template <typename T>
static hipError_t inverse_t(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  dim3 g1(b.n);
  hipLaunchKernelGGL(k_inverse_coarse<T>, g1, dim3(256), 0, st, b, 0);
  if (c.p == 2) hipLaunchKernelGGL((k_prolong_coarse<2, T>), g1, dim3(1024), 0, st, b, 0, kCoarseLevels, 1, 0, 0);
  else hipLaunchKernelGGL((k_prolong_coarse<3, T>), g1, dim3(1024), 0, st, b, 0, kCoarseLevels, 1, 0, 0);
  for (int l = kCoarseLevels + 1; l <= c.J; ++l) {
    const int cnt = 3 << (2 * (l - 1));
    dim3 g(((cnt + 255) / 256) * b.n);
    if (c.p == 2) hipLaunchKernelGGL((k_prolong_level<2, T>), g, dim3(256), 0, st, b, 0, l);
    else hipLaunchKernelGGL((k_prolong_level<3, T>), g, dim3(256), 0, st, b, 0, l);
  }
  return hipGetLastError();
}

hipError_t launch_prolong(const Batch& b, const LaunchCfg& c, int target, int as_double, int src, int j,
                          hipStream_t st) {
  if (as_double) return prolong_t<double>(b, c, target, src, j, st);
  return prolong_t<float>(b, c, target, src, j, st);
}

// inverse transform: packed input in s.spec (element type of prec), output wt.
hipError_t launch_inverse(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  if (c.prec == 0) return inverse_t<double>(b, c, st);
  return inverse_t<float>(b, c, st);
}

// ---------------------------------------------------------------- forward
__device__ inline double warp_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

__global__ void k_reset_max(Batch b) {
  if (threadIdx.x == 0) *MRA_SOLVE(b).umax = 0ull;
}

hipError_t launch_reset_max(const Batch& b, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_max, dim3((1) * b.n), dim3(64), 0, st, b);
  return hipGetLastError();
}

// src: 0 -> dense64 (double), 1 -> wt (T).  dst: 0 -> packed64 (double),
// 1 -> spec reinterpreted as a packed T array.  One thread per packed node
// below nlim (the levels below those of k_forward_tiles).
template <int P, typename T>
__global__ void __launch_bounds__(256) k_forward(Batch b, int src, int dst, int nlim) {
#pragma clang fp contract(off)
  const SolveDev& s = MRA_SOLVE(b);
  const auto* f = glb(src == 0 ? reinterpret_cast<const T*>(s.dense64) : reinterpret_cast<const T*>(s.wt));
  auto* out = glb(dst == 0 ? reinterpret_cast<T*>(s.packed64) : reinterpret_cast<T*>(s.spec));
  const int J = s.J, j0 = s.j0, N = s.N;
  const int i = MRA_BX(b) * blockDim.x + threadIdx.x;
  double am = 0.0;
  if (i < nlim) {
    int l;
    const int fi = packed_to_fine(i, J, j0, &l);
    const T val = f[fi];
    // a NaN would vanish in the fmax reduction: count it as +inf
    am = isfinite((double)val) ? fabs((double)val) : __builtin_huge_val();
    out[i] = l == j0 ? val : val - predict_node<P, T, decltype(f)>(f, fi & (N - 1), fi >> J, l, J);
  }
  __shared__ double red[4];
  am = warp_max(am);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = am;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    atomicMax(s.umax, (unsigned long long)__double_as_longlong(mx));
  }
}

// The three finest levels (98% of the nodes), tile by tile: the dense field
// of a TS x TS tile and the reach of its predictions (H = (2P - 1) 2^(J - LT)
// for the coarsest of those levels, LT) is staged in LDS once, and every node
// of the tile at a level >= LT takes its detail from there, with the
// arithmetic of predict_node (a node's parity from its global coordinates,
// its neighbours at the same offsets in the tile's window).  The max |f| is
// taken over every node of the tile.
template <int P> constexpr int fwd_lt(int J) {
  return J - 2 > pi_j0<P>() + 1 ? J - 2 : pi_j0<P>() + 1;
}
template <int P, typename T, int J>
__global__ void __launch_bounds__(256) k_forward_tiles(Batch b, int src, int dst) {
#pragma clang fp contract(off)
  constexpr int N = 1 << J, NM = N - 1, J0 = pi_j0<P>(), LT = fwd_lt<P>(J);
  constexpr int TS = N < 32 ? N : 32, NTX = N / TS;
  constexpr int H = (2 * P - 1) << (J - LT), W = TS + 2 * H;
  __shared__ T reg[W * W];
  const SolveDev& s = MRA_SOLVE(b);
  const auto* f = glb(src == 0 ? reinterpret_cast<const T*>(s.dense64) : reinterpret_cast<const T*>(s.wt));
  auto* out = glb(dst == 0 ? reinterpret_cast<T*>(s.packed64) : reinterpret_cast<T*>(s.spec));
  const int t = tile_of_block(MRA_BX(b), NTX * NTX, b.n);
  const int x0 = (t % NTX) * TS, y0 = (t / NTX) * TS;
  constexpr int NR = (W * W + 255) / 256;
  T v[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int q = threadIdx.x + 256 * i;
    if (q < W * W) {
      const int r = q / W, c = q - r * W;
      v[i] = f[((y0 - H + r) & NM) * N + ((x0 - H + c) & NM)];
    }
  }
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int q = threadIdx.x + 256 * i;
    if (q < W * W) reg[q] = v[i];
  }
  __syncthreads();
  double am = 0.0;
  for (int q = threadIdx.x; q < TS * TS; q += 256) {
    const int ly = q / TS, lx = q - ly * TS;
    const int x = x0 + lx, y = y0 + ly;
    const int cx = lx + H, cy = ly + H;
    const T val = reg[cy * W + cx];
    am = fmax(am, isfinite((double)val) ? fabs((double)val) : __builtin_huge_val());
    const int xy = x | y;
    const int l = xy == 0 ? J0 : (J - ntz((unsigned)xy) > J0 ? J - ntz((unsigned)xy) : J0);
    if (l < LT) continue;
    // predict_node's arithmetic on the window (same neighbours, same order)
    const int sv = 1 << (J - l), S = 2 * sv;
    const bool ox = (x & sv) != 0, oy = (y & sv) != 0;
    T c[2 * P];
    T pred;
    if (ox && !oy) {
      const int a = cx - sv - (P - 1) * S;
#pragma unroll
      for (int o = 0; o < 2 * P; ++o) c[o] = reg[cy * W + a + o * S];
      pred = dd_pred<P, T>(c);
    } else if (oy && !ox) {
      const int a = cy - sv - (P - 1) * S;
#pragma unroll
      for (int o = 0; o < 2 * P; ++o) c[o] = reg[(a + o * S) * W + cx];
      pred = dd_pred<P, T>(c);
    } else {
      T py[2 * P];
      const int ax = cx - sv - (P - 1) * S, ay = cy - sv - (P - 1) * S;
#pragma unroll
      for (int o2 = 0; o2 < 2 * P; ++o2) {
#pragma unroll
        for (int o = 0; o < 2 * P; ++o) c[o] = reg[(ay + o * S) * W + ax + o2 * S];
        py[o2] = dd_pred<P, T>(c);
      }
      pred = dd_pred<P, T>(py);
    }
    out[fine_to_packed(x, y, l, J, J0)] = val - pred;
  }
  __shared__ double red[4];
  am = warp_max(am);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = am;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    atomicMax(s.umax, (unsigned long long)__double_as_longlong(mx));
  }
}

template <int P, typename T>
static hipError_t forward_p(const Batch& b, int J, int src, int dst, hipStream_t st) {
  const int j0 = pi_j0<P>();
  if (J <= j0 || J > 11) return hipErrorInvalidValue;
  // coarse levels: one thread per packed node below level LT
  const int lt = J - 2 > j0 + 1 ? J - 2 : j0 + 1;
  const int nlim = 1 << (2 * (lt - 1));
  hipLaunchKernelGGL((k_forward<P, T>), dim3(((nlim + 255) / 256) * b.n), dim3(256), 0, st, b, src, dst, nlim);
  const int N = 1 << J, TS = N < 32 ? N : 32;
  const dim3 g((N / TS) * (N / TS) * b.n);
  switch (J) {
    case 3: if constexpr (P == 2) { hipLaunchKernelGGL((k_forward_tiles<P, T, 3>), g, dim3(256), 0, st, b, src, dst); break; } return hipErrorInvalidValue;
    case 4: hipLaunchKernelGGL((k_forward_tiles<P, T, 4>), g, dim3(256), 0, st, b, src, dst); break;
    case 5: hipLaunchKernelGGL((k_forward_tiles<P, T, 5>), g, dim3(256), 0, st, b, src, dst); break;
    case 6: hipLaunchKernelGGL((k_forward_tiles<P, T, 6>), g, dim3(256), 0, st, b, src, dst); break;
    case 7: hipLaunchKernelGGL((k_forward_tiles<P, T, 7>), g, dim3(256), 0, st, b, src, dst); break;
    case 8: hipLaunchKernelGGL((k_forward_tiles<P, T, 8>), g, dim3(256), 0, st, b, src, dst); break;
    case 9: hipLaunchKernelGGL((k_forward_tiles<P, T, 9>), g, dim3(256), 0, st, b, src, dst); break;
    case 10: hipLaunchKernelGGL((k_forward_tiles<P, T, 10>), g, dim3(256), 0, st, b, src, dst); break;
    case 11: hipLaunchKernelGGL((k_forward_tiles<P, T, 11>), g, dim3(256), 0, st, b, src, dst); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_forward(const Batch& b, const LaunchCfg& c, int src, int dst, hipStream_t st) {
  const bool dbl = src == 0 || c.prec == 0;
  if (dbl) return c.p == 2 ? forward_p<2, double>(b, c.J, src, dst, st) : forward_p<3, double>(b, c.J, src, dst, st);
  return c.p == 2 ? forward_p<2, float>(b, c.J, src, dst, st) : forward_p<3, float>(b, c.J, src, dst, st);
}

// ---------------------------------------------------------------- threshold
// Active set: the coarsest mesh, every significant node (|d| >= tau), and the
// adjacent zone of every significant node Q of level l > j0: the nodes of
// G^{min(l+1,J)} within periodic Chebyshev distance 2^(J-l) of Q.  Written as
// a scatter (each significant node marks its 5 x 5, on the finest level 3 x 3,
// zone), so the cost follows the number of significant nodes; concurrent
// marks all write 1.  Three passes: significance, zones, per-block counts.
template <typename TP>
__device__ inline const TP* packed_details(const SolveDev& s, int packed_is_double) {
  return packed_is_double ? reinterpret_cast<const TP*>(s.packed64) : reinterpret_cast<const TP*>(s.spec);
}

template <typename TP>
__global__ void __launch_bounds__(256) k_mask_sig(Batch b, int packed_is_double) {
  const SolveDev& s = MRA_SOLVE(b);
  const TP* d = packed_details<TP>(s, packed_is_double);
  const int Nf = s.N * s.N, n0 = 1 << (2 * s.j0);
  const double umax = __longlong_as_double((long long)*s.umax);
  // max|u| over the field is NaN or inf exactly when a value is: report it
  // (every comparison with tau would fail and silently drop the details)
  if (MRA_BX(b) == 0 && threadIdx.x == 0 && !isfinite(umax)) s.ctrl[C_STATUS] = 5;
  const double tau = s.eps * umax;
  for (int i = MRA_BX(b) * blockDim.x + threadIdx.x; i < Nf; i += MRA_GX(b) * blockDim.x)
    s.mask[i] = (i < n0 || fabs((double)d[i]) >= tau) ? 1 : 0;
}

template <typename TP>
__global__ void __launch_bounds__(256) k_mask_zone(Batch b, int packed_is_double) {
  const SolveDev& s = MRA_SOLVE(b);
  if (!s.adjacent_zone) return;
  const TP* d = packed_details<TP>(s, packed_is_double);
  const int J = s.J, j0 = s.j0, N = s.N, nm = N - 1, Nf = N * N, n0 = 1 << (2 * j0);
  const double tau = s.eps * __longlong_as_double((long long)*s.umax);
  for (int i = n0 + MRA_BX(b) * blockDim.x + threadIdx.x; i < Nf; i += MRA_GX(b) * blockDim.x) {
    if (!(fabs((double)d[i]) >= tau)) continue;
    int l;
    const int f = packed_to_fine(i, J, j0, &l);
    const int px = f & nm, py = f >> J;
    const int sp = l < J ? 1 << (J - l - 1) : 1;   // spacing of G^{min(l+1,J)}
    const int R = l < J ? 2 : 1;                    // 2^(J-l) / spacing
    for (int bq = -R; bq <= R; ++bq) {
      const int qy = (py + bq * sp) & nm;
      for (int aq = -R; aq <= R; ++aq) {
        const int qx = (px + aq * sp) & nm;
        s.mask[fine_to_packed(qx, qy, level_of(qx, qy, J, j0), J, j0)] = 1;
      }
    }
  }
}

// active count of each compaction block (kScanBlock threads x kScanItems)
__global__ void __launch_bounds__(kScanBlock) k_mask_count(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int Nf = s.N * s.N;
  const int base = MRA_BX(b) * (kScanBlock * kScanItems) + threadIdx.x * kScanItems;
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int i = base + q;
    if (i < Nf) cnt += s.mask[i];
  }
  __shared__ int red[kScanBlock / 64];
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kScanBlock / 64; ++w) t += red[w];
    s.block_off[MRA_BX(b)] = t;
  }
}

// exclusive block-wide scan of one int per thread (blockDim multiple of 64)
__device__ inline int block_exclusive_scan(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < nw; ++w) { int t = sh[w]; sh[w] = acc; acc += t; }
    sh[nw] = acc;
  }
  __syncthreads();
  const int res = sh[wid] + x - v;
  *total = sh[nw];
  __syncthreads();
  return res;
}

__global__ void __launch_bounds__(1024) k_scan(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int Nf = s.N * s.N;
  const int nblk = (Nf + kScanBlock * kScanItems - 1) / (kScanBlock * kScanItems);
  const int per = (nblk + blockDim.x - 1) / blockDim.x;
  __shared__ int sh[17];
  int loc[8];
  int sum = 0;
  for (int q = 0; q < per; ++q) {
    const int k = threadIdx.x * per + q;
    const int v = k < nblk ? s.block_off[k] : 0;
    loc[q] = sum;
    sum += v;
  }
  int total;
  const int off = block_exclusive_scan(sum, sh, &total);
  for (int q = 0; q < per; ++q) {
    const int k = threadIdx.x * per + q;
    if (k < nblk) s.block_off[k] = off + loc[q];
  }
  if (threadIdx.x == 0) {
    // more active nodes than the arrays hold: nothing is compacted, n_active
    // becomes 0 (every later step then moves no state) and the state stays
    // omega on the previous set, whose prolongation the next regrid (or a
    // move to a larger arena) takes up again
    const int over = total > s.cap;
    s.ctrl[C_OVER] = over;
    if (over) {
      s.ctrl[C_NEED] = total;
      s.ctrl[C_STATUS] = kStatusCapacity;
    }
    *s.n_active = over ? 0 : total;
  }
}

__global__ void __launch_bounds__(kScanBlock) k_compact(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  if (s.ctrl[C_OVER]) return;    // the previous set and rank map stay
  const int Nf = s.N * s.N;
  const int J = s.J, j0 = s.j0;
  const int base = MRA_BX(b) * (kScanBlock * kScanItems) + threadIdx.x * kScanItems;
  int m[kScanItems];
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int i = base + q;
    m[q] = i < Nf ? s.mask[i] : 0;
    cnt += m[q];
  }
  __shared__ int sh[kScanBlock / 64 + 1];
  int total;
  int pos = s.block_off[MRA_BX(b)] + block_exclusive_scan(cnt, sh, &total);
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int i = base + q;
    if (i >= Nf) break;
    const int f = packed_to_fine(i, J, j0, nullptr);
    if (m[q]) {
      s.index_packed[pos] = i;
      s.index_fine[pos] = f;
      s.rank[f] = pos;
      ++pos;
    } else {
      s.rank[f] = -1;
    }
  }
}

// Active nodes per stencil tile, from the rank map: one block per tile, a
// plain count (no atomics, so no contention on the counters of full tiles).
__global__ void __launch_bounds__(256) k_tile_count(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int T = s.tile, ntx = s.ntx, N = s.N;
  const auto* rank = glb(s.rank);
  __shared__ int part[4];
  for (int t = MRA_BX(b); t < ntx * ntx; t += MRA_GX(b)) {
    const int x0 = (t % ntx) * T, y0 = (t / ntx) * T;
    int c = 0;
    for (int q = threadIdx.x; q < T * T; q += blockDim.x) c += rank[(y0 + q / T) * N + x0 + q % T] >= 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) glb(s.tile_count)[t] = part[0] + part[1] + part[2] + part[3];
    __syncthreads();
  }
}

static hipError_t launch_tile_count(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  const int ntx = c.tile > 0 ? (1 << c.J) / c.tile : 1;
  const int per = ntx * ntx < 2048 ? ntx * ntx : 2048;
  hipLaunchKernelGGL(k_tile_count, dim3(per * b.n), dim3(256), 0, st, b);
  return hipGetLastError();
}

static int grid_blocks(int J);

hipError_t launch_threshold(const Batch& b, const LaunchCfg& c, int packed_is_double, hipStream_t st) {
  const int nf = 1 << (2 * c.J);
  const int nblk = (nf + kScanBlock * kScanItems - 1) / (kScanBlock * kScanItems);
  dim3 g((nblk) * b.n);
  dim3 gm(grid_blocks(c.J) * b.n);
  if (packed_is_double || c.prec == 0) {
    hipLaunchKernelGGL(k_mask_sig<double>, gm, dim3(256), 0, st, b, packed_is_double);
    hipLaunchKernelGGL(k_mask_zone<double>, gm, dim3(256), 0, st, b, packed_is_double);
  } else {
    hipLaunchKernelGGL(k_mask_sig<float>, gm, dim3(256), 0, st, b, packed_is_double);
    hipLaunchKernelGGL(k_mask_zone<float>, gm, dim3(256), 0, st, b, packed_is_double);
  }
  hipLaunchKernelGGL(k_mask_count, g, dim3(kScanBlock), 0, st, b);
  hipLaunchKernelGGL(k_scan, dim3((1) * b.n), dim3(1024), 0, st, b);
  hipLaunchKernelGGL(k_compact, g, dim3(kScanBlock), 0, st, b);
  return launch_tile_count(b, c, st);
}

// ---------------------------------------------------------------- gather
static int grid_blocks(int J) {
  const int nf = 1 << (2 * J);
  const int nb = (nf + 255) / 256;
  return nb < 1024 ? nb : 1024;
}

__global__ void __launch_bounds__(256) k_gather(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int na = (int)*s.n_active;
  for (int k = MRA_BX(b) * blockDim.x + threadIdx.x; k < na; k += MRA_GX(b) * blockDim.x)
    s.omega[k] = s.dense64[s.index_fine[k]];
}

hipError_t launch_gather(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3((grid_blocks(c.J)) * b.n), dim3(256), 0, st, b);
  return hipGetLastError();
}

// rank map and tile counts from a caller-given index list
__global__ void __launch_bounds__(256) k_rank_clear(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int Nf = s.N * s.N;
  for (int f = MRA_BX(b) * blockDim.x + threadIdx.x; f < Nf; f += MRA_GX(b) * blockDim.x) s.rank[f] = -1;
}

__global__ void __launch_bounds__(256) k_rank_scatter(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int na = (int)*s.n_active;
  for (int k = MRA_BX(b) * blockDim.x + threadIdx.x; k < na; k += MRA_GX(b) * blockDim.x)
    s.rank[s.index_fine[k]] = k;
}

hipError_t launch_rank_from_index(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  dim3 g((grid_blocks(c.J)) * b.n);
  hipLaunchKernelGGL(k_rank_clear, g, dim3(256), 0, st, b);
  hipLaunchKernelGGL(k_rank_scatter, g, dim3(256), 0, st, b);
  return launch_tile_count(b, c, st);
}

}  // namespace mra
