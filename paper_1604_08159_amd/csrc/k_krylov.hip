// Krylov part of the time steps, in FP64 arithmetic (the basis is stored in
// FP64, or in FP32 for precision MRA_FP32): Arnoldi with classical
// Gram-Schmidt and a reorthogonalisation delayed by one column (DCGS2); for the
// exponential Rosenbrock-Euler
// step phi_1(dt H) e_1 from the exponential of the augmented Hessenberg
// matrix and the update omega_M += dt beta V y; for the theta-scheme the
// Newton residual, the GMRES least squares and the Newton update.
//
// The paper advances the collocation system by projecting it onto a Krylov
// subspace (abstract; Section 2.1); the exponential Euler step with the
// Jacobian at frozen eddy viscosity is the reading implemented here.
//
// Reductions over the active nodes are deterministic and need no cross-block
// signalling: the active list is cut into the same fixed chunks in every
// kernel of a step (the chunk count depends only on N_a), each block reduces
// its chunk in a fixed order into a per-chunk partial (wavefront butterflies,
// then the wavefronts in order), and every block of the NEXT kernel adds the
// partials in the same fixed order (the kernel boundary orders the writes
// before the reads).
#include <utility>

#include "mra_internal.hpp"

namespace mra {

// Gram-Schmidt kernels.  A thread takes the elements lo + tid, lo + tid + 256,
// ... of its chunk; for each it loads w and all basis entries V_i[k], i <= j,
// at once (MJ >= j + 1 register slots, MJ fixed at compile time from m), so a
// chunk costs one dependent global round per element instead of one per group
// of basis vectors.
//
// Classical Gram-Schmidt with the reorthogonalisation delayed by one column
// (DCGS2: Swirydowicz, Langou, Ananthan, Yang and Thomas, "Low
// synchronization Gram-Schmidt and GMRES algorithms", 2020; Bielich et al.,
// 2022).  Every column gets its second pass, as in CGS2, but the second pass
// of column j - 1 shares the reads of the basis with the first pass of column
// j, so a column costs two passes over the basis, not three or four.  Slot j
// of the basis holds r_j, the residual of the first pass of column j - 1 (not
// normalised and not yet reorthogonalised; for j = 0 the normalised v_0), and
// the product w = A r_j is taken of it.  Column j:
//   stage 1 (k_gs_dot)   g = V_{<j}^T w, c = r_j^T w, ||w||^2, and
//     s = V_{<j}^T r_j, ||r_j||^2;
//   stage 2 (k_gs_update):
//       alpha = ||r_j - V s|| = sqrt(||r_j||^2 - ||s||^2)      (Pythagoras)
//       column j - 1 of H: h^(j-1) + s, and H[j][j-1] = alpha     (final)
//       v_j = (r_j - V s) / alpha
//       A v_j = (w - V_{<=j} u) / alpha,  u = H[0..j][0..j-1] s   (Arnoldi)
//       h^(j) = V_{<=j}^T A v_j: (g_i - u_i) / alpha for i < j,
//               (kappa - u_j) / alpha at j, kappa = (c - s^T g) / alpha
//       r_{j+1} = A v_j - V_{<=j} h^(j) = (w - V g - kappa v_j) / alpha;
//   the last column's stage 2 also sums V_{<m}^T r_m and ||r_m||^2 on the fly
//   (r_m is not stored), and k_gs_last ends column m - 1 from them.
// A breakdown of column j - 1 (alpha <= 1e-13 ||A v_{j-1}||, with
// ||A v_{j-1}||^2 = ||h^(j-1)||^2 + ||r_j||^2) or a non-finite value ends the
// basis at column j's stage 2 (m_eff = j).  The oracle's Arnoldi uses
// modified Gram-Schmidt; in exact arithmetic the two give the same basis and
// Hessenberg matrix.
//
// The second-pass sums of r_j (V_{<j}^T r_j, ||r_j||^2) are taken by column
// j's stage 1, which reads V_{<j} and r_j for its own sums anyway; stage 2
// then holds no sums of its own (except in the last column, for r_m).
// Partials: stage 1 writes buffers 0 and 1, stage 2 reads them, the last
// column's stage 2 writes buffer 2 for k_gs_last; no kernel overwrites
// partials that a block of the same kernel is still reading.  The first-pass
// coefficients h^(j) wait in hpart slot j & 1 until the next column ends them.

// ||F||^2 partials (buffer 1).
__global__ void __launch_bounds__(256) k_norm0(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int na = (int)*s.n_active;
  const int nb = nchunks(na);
  for (int ch = MRA_BX(b); ch < nb; ch += MRA_GX(b)) {
    const Chunk c = chunk_of(na, ch);
    double acc[1] = {0.0};
    const auto* W = glb(s.w);
    for (int k = c.lo + (int)threadIdx.x; k < c.hi; k += blockDim.x) acc[0] += W[k] * W[k];
    block_sums_store<1>(acc, 1, part_buf(s, 1) + (size_t)ch * (kMaxM + 2));
    __syncthreads();
  }
}

// Stage 1: V_{<=j}^T w (slot j holding r_j) and ||w||^2 partials (buffer 0)
// and, for j > 0, the second-pass sums of r_j, V_{<j}^T r_j and ||r_j||^2
// (buffer 1), from the same loads.
template <typename TV, int MJ, int JC>
__global__ void __launch_bounds__(256) k_gs_dot(Batch b, int jrt) {
  const int j = JC >= 0 ? JC : jrt;   // JC >= 0: the column is a compile-time constant
  const SolveDev& s = MRA_SOLVE(b);
  if (s.ctrl[C_DONE]) return;
  const int na = (int)*s.n_active;
  const int nb = nchunks(na);
  const size_t Nf = (size_t)s.vs;   // basis stride
  const unsigned vst = (unsigned)(Nf * sizeof(TV));
  const auto rV = buf_rsrc(vbasis<TV>(s), (size_t)(s.m + 1) * Nf * sizeof(TV));
  const auto rW = buf_rsrc(s.w, (size_t)s.cap * sizeof(double));
  for (int ch = MRA_BX(b); ch < nb; ch += MRA_GX(b)) {
    const Chunk c = chunk_of(na, ch);
    double acc[MJ + 1], acs[MJ + 1];
#pragma unroll
    for (int i = 0; i <= MJ; ++i) acc[i] = acs[i] = 0.0;
    for (int k = c.lo + (int)threadIdx.x; k < c.hi; k += blockDim.x) {
      const double wk = buf_ld<double>(rW, (unsigned)k * 8u, 0u);
      const unsigned ko = (unsigned)k * (unsigned)sizeof(TV);
      TV v[MJ];   // raw loads: a conversion here would wait for each load in turn
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i <= j) v[i] = buf_ld<TV>(rV, ko, (unsigned)i * vst);
      double rj = 0.0;
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i == j) rj = (double)v[i];
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i <= j) acc[i] += (double)v[i] * wk;
      acc[MJ] += wk * wk;
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i < j) acs[i] += (double)v[i] * rj;
      acs[MJ] += rj * rj;
    }
    // slot layouts: g[0 .. j - 1], c at j, ||w||^2 at j + 1; s[0 .. j - 1],
    // ||r_j||^2 at j (static register indices)
#pragma unroll
    for (int i = 0; i < MJ; ++i)
      if (i == j + 1) acc[i] = acc[MJ];
#pragma unroll
    for (int i = 0; i < MJ; ++i)
      if (i == j) acs[i] = acs[MJ];
    block_sums_store<MJ + 1>(acc, j + 2, part_buf(s, 0) + (size_t)ch * (kMaxM + 2));
    __syncthreads();
    if (j > 0) {
      block_sums_store<MJ + 1>(acs, j + 1, part_buf(s, 1) + (size_t)ch * (kMaxM + 2));
      __syncthreads();
    }
  }
}

// The end of column jj - 1 from the partials of V_{<jj}^T r_jj and
// ||r_jj||^2 (in sb, ||r_jj||^2 at jj) and its first-pass coefficients
// (hpart slot (jj - 1) & 1): alpha, and the breakdown and non-finite tests
// against ||A v_{jj-1}||.  Called by the first wavefront (lane i takes term i
// of both sums; jj <= kMaxM + 1 <= 64), every lane gets the result; *brk when
// the basis ends at column jj - 1, *bad when a value is not finite.
__device__ inline double end_column(const SolveDev& s, int jj, const double* sb, bool* brk, bool* bad) {
  static_assert(kMaxM + 1 <= 64, "one lane per coefficient");
  const double* hp = s.hpart + (size_t)((jj - 1) & 1) * (kMaxM + 1);
  const int lane = threadIdx.x & 63;
  double ss = 0.0, hh = 0.0;
  if (lane < jj) {
    const double a = sb[lane], h = hp[lane];
    ss = a * a;
    hh = h * h;
  }
  ss = wave_sum(ss);
  hh = wave_sum(hh);
  const double a = sb[jj];
  *bad = !isfinite(a) || !isfinite(ss) || !isfinite(hh);
  const double al = *bad ? 0.0 : sqrt(fmax(a - ss, 0.0));
  *brk = *bad || al <= kBreakdown * sqrt(hh + a);
  return al;
}

// Block 0: column jj - 1 of H made final (h^(jj-1) + s, subdiagonal alpha)
// and, if the basis ends there, the control words (m_eff = jj, or 0 with
// status 5 for a non-finite value).
__device__ inline void write_column(const SolveDev& s, int jj, const double* sb, double alpha, bool brk, bool bad) {
  const double* hp = s.hpart + (size_t)((jj - 1) & 1) * (kMaxM + 1);
  const int m = s.m;
  for (int i = threadIdx.x; i < jj; i += blockDim.x) s.H[i * m + jj - 1] = hp[i] + sb[i];
  if (threadIdx.x == 0) {
    s.H[jj * m + jj - 1] = alpha;
    if (bad) {
      s.ctrl[C_STATUS] = 5;
      s.ctrl[C_MEFF] = 0;
    } else if (brk && jj < s.ctrl[C_MEFF]) {
      s.ctrl[C_MEFF] = jj;
    }
    if (brk) s.ctrl[C_DONE] = 1;
  }
}

// Stage 2 (see above).  ACC: the last column, which also sums the
// second-pass partials of r_m for k_gs_last (buffer 2); the other columns'
// r_{j+1} get theirs from the next column's stage 1.
template <typename TV, int MJ, int JC, bool ACC>
__global__ void __launch_bounds__(256) k_gs_update(Batch b, int jrt) {
  const int j = JC >= 0 ? JC : jrt;   // JC >= 0: the column is a compile-time constant
  const SolveDev& s = MRA_SOLVE(b);
  if (s.ctrl[C_DONE]) return;
  const int na = (int)*s.n_active;
  const int nb = nchunks(na);
  if ((int)MRA_BX(b) >= nb) return;
  const int m = s.m;
  // the buffer resources, formed while every value they take is uniform
  const size_t Nf = (size_t)s.vs;   // basis stride
  const unsigned vst = (unsigned)(Nf * sizeof(TV));
  const auto rV = buf_rsrc(vbasis<TV>(s), (size_t)(m + 1) * Nf * sizeof(TV));
  const auto rW = buf_rsrc(s.w, (size_t)s.cap * sizeof(double));
  __shared__ double ga[kMaxM + 2];               // g[0 .. j - 1], c, ||w||^2
  __shared__ double sb[kMaxM + 2];               // s[0 .. j - 1], ||r_j||^2
  __shared__ double Hs[(kMaxM + 1) * kMaxM];     // H[0..j][0..j-1], column j - 1 made final
  __shared__ double u[kMaxM + 1];
  __shared__ double sc[3];                       // alpha, kappa, 1 / alpha
  __shared__ int brk_sh, bad_sh;
  // columns 0 .. j - 2 of H are final (earlier stage-2 kernels wrote them)
  for (int q = threadIdx.x; q < (j + 1) * j; q += blockDim.x) {
    const int r = q / j, cidx = q - r * j;
    Hs[q] = cidx < j - 1 ? s.H[r * m + cidx] : 0.0;
  }
  if (j > 0 && 2 * j + 3 <= 64) {
    reduce_partials2(part_buf(s, 0), j + 2, ga, part_buf(s, 1), j + 1, sb, nb);
  } else {
    reduce_partials<32>(part_buf(s, 0), nb, j + 2, ga);
    if (j > 0) reduce_partials<32>(part_buf(s, 1), nb, j + 1, sb);
  }
  if (threadIdx.x < 64) {
    double al = 1.0;
    bool brk = false, bad = false;
    if (j > 0) al = end_column(s, j, sb, &brk, &bad);
    if (threadIdx.x == 0) {
      bad |= !isfinite(ga[j + 1]);        // the product of r_j
      sc[0] = al;
      sc[2] = al > 0.0 ? 1.0 / al : 0.0;
      brk_sh = brk || bad;
      bad_sh = bad;
    }
  }
  __syncthreads();
  if (MRA_BX(b) == 0) {
    if (j > 0) write_column(s, j, sb, sc[0], brk_sh, bad_sh);
    else if (bad_sh && threadIdx.x == 0) {
      s.ctrl[C_STATUS] = 5;
      s.ctrl[C_MEFF] = 0;
      s.ctrl[C_DONE] = 1;
    }
  }
  if (brk_sh) return;
  // column j - 1 of the staged H made final, then u = H[0..j][0..j-1] s
  if (j > 0) {
    const double* hp = s.hpart + (size_t)((j - 1) & 1) * (kMaxM + 1);
    for (int r = threadIdx.x; r <= j; r += blockDim.x)
      Hs[r * j + j - 1] = r < j ? hp[r] + sb[r] : sc[0];
  }
  __syncthreads();
  for (int r = threadIdx.x; r <= j; r += blockDim.x) {
    // row r of the Hessenberg H[0..j][0..j-1] starts at column r - 1
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < MJ; ++i)
      if (i + 1 >= r && i < j) t += Hs[r * j + i] * sb[i];
    u[r] = t;
  }
  if (threadIdx.x >= 64 && threadIdx.x < 128) {
    const int lane = threadIdx.x - 64;
    const double sg = wave_sum(lane < j ? sb[lane] * ga[lane] : 0.0);
    if (lane == 0) sc[1] = (ga[j] - sg) * sc[2];
  }
  __syncthreads();
  // first-pass coefficients of column j, kept until the next column ends it
  if (MRA_BX(b) == 0) {
    double* hc = s.hpart + (size_t)(j & 1) * (kMaxM + 1);
    for (int r = threadIdx.x; r <= j; r += blockDim.x) hc[r] = ((r < j ? ga[r] : sc[1]) - u[r]) * sc[2];
  }
  const double ia = sc[2], kap = sc[1];
  const bool store_next = j + 1 < m;
  for (int ch = MRA_BX(b); ch < nb; ch += MRA_GX(b)) {
    const Chunk c = chunk_of(na, ch);
    double acc[ACC ? MJ + 1 : 1];
#pragma unroll
    for (int i = 0; i < (ACC ? MJ + 1 : 1); ++i) acc[i] = 0.0;
    for (int k = c.lo + (int)threadIdx.x; k < c.hi; k += blockDim.x) {
      // the coefficients sb, ga are read from LDS in every trip: held in
      // registers across the loop they would take 4 more per basis vector
      // beside the loaded entries, and cut the waves per SIMD
      asm volatile("" ::: "memory");
      const double wk = buf_ld<double>(rW, (unsigned)k * 8u, 0u);
      const unsigned ko = (unsigned)k * (unsigned)sizeof(TV);
      TV v[MJ];   // raw loads: a conversion here would wait for each load in turn
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i <= j) v[i] = buf_ld<TV>(rV, ko, (unsigned)i * vst);
      double rj = 0.0;
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i == j) rj = (double)v[i];
      double t = rj;
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i < j) t -= sb[i] * (double)v[i];
      // v_j as stored (j = 0: v_0 itself, already final)
      const TV vjs = j > 0 ? (TV)(t * ia) : (TV)rj;
      const double vj = (double)vjs;
      double q = wk;
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i < j) q -= ga[i] * (double)v[i];
      q -= kap * vj;
      const TV rns = (TV)(q * ia);
      const double rn = (double)rns;
      if (j > 0) buf_st<TV>(rV, ko, (unsigned)j * vst, vjs);
      if (store_next) buf_st<TV>(rV, ko, (unsigned)(j + 1) * vst, rns);
      if constexpr (ACC) {
#pragma unroll
        for (int i = 0; i < MJ; ++i)
          if (i < j) acc[i] += (double)v[i] * rn;
#pragma unroll
        for (int i = 0; i < MJ; ++i)
          if (i == j) acc[i] += vj * rn;
        acc[MJ] += rn * rn;
      }
    }
    if constexpr (ACC) {
      // slot layout: V_{<=j}^T r_{j+1} at 0 .. j, ||r_{j+1}||^2 at j + 1
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i == j + 1) acc[i] = acc[MJ];
      block_sums_store<MJ + 1>(acc, j + 2, part_buf(s, 2) + (size_t)ch * (kMaxM + 2));
      __syncthreads();
    }
  }
}

// The end of the last column m - 1: the second-pass coefficients of r_m and
// ||r_m||^2 from its stage 2 (r_m itself is not stored).  One block per solve.
__global__ void __launch_bounds__(256) k_gs_last(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  if (s.ctrl[C_DONE]) return;
  const int na = (int)*s.n_active;
  const int nb = nchunks(na);
  const int jj = s.m;
  __shared__ double sb[kMaxM + 2];
  __shared__ double al_sh;
  __shared__ int brk_sh, bad_sh;
  reduce_partials<32>(part_buf(s, 2), nb, jj + 1, sb);
  if (threadIdx.x < 64) {
    bool brk, bad;
    const double al = end_column(s, jj, sb, &brk, &bad);
    if (threadIdx.x == 0) {
      al_sh = al;
      brk_sh = brk;
      bad_sh = bad;
    }
  }
  __syncthreads();
  write_column(s, jj, sb, al_sh, brk_sh, bad_sh);
}

// Grid of the reductions, blocks per solve (blocks loop over chunks): at
// least kRedGrid, more for small batches so that the launch still has about
// kRedTarget blocks (four per CU; a batch of two 2048^2 solves would
// otherwise run 128 blocks), never more than the chunks a grid can have.
constexpr int kRedGrid = 64;
constexpr int kRedTarget = 2048;
static int red_grid(int J, int nbatch) {
  const int nf = 1 << (2 * J);
  int cap = (nf + kChunkMin - 1) / kChunkMin;
  if (cap > kRedBlocks) cap = kRedBlocks;
  int g = (kRedTarget + nbatch - 1) / nbatch;
  if (g < kRedGrid) g = kRedGrid;
  return g < cap ? g : cap;
}

hipError_t launch_norm0(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_norm0, dim3(red_grid(c.J, b.n) * b.n), dim3(256), 0, st, b);
  return hipGetLastError();
}

template <typename TV, int MJ, int JC>
static void arnoldi_mj(const Batch& b, dim3 g, int j, bool last, hipStream_t st) {
  hipLaunchKernelGGL((k_gs_dot<TV, MJ, JC>), g, dim3(256), 0, st, b, j);
  if (last) hipLaunchKernelGGL((k_gs_update<TV, MJ, JC, true>), g, dim3(256), 0, st, b, j);
  else hipLaunchKernelGGL((k_gs_update<TV, MJ, JC, false>), g, dim3(256), 0, st, b, j);
}

// Columns j < kFixedCols run kernels instantiated for that column (exactly
// j + 1 basis vectors, no per-vector predicates); later columns (m > 32) use
// a register bucket of 48 vectors with a run-time column.
constexpr int kFixedCols = 32;
template <typename TV, int... Js>
static void arnoldi_fixed(const Batch& b, dim3 g, int j, bool last, hipStream_t st,
                          std::integer_sequence<int, Js...>) {
  (void)((j == Js ? (arnoldi_mj<TV, Js + 1, Js>(b, g, j, last, st), true) : false) || ...);
}

template <typename TV>
static void arnoldi_t(const Batch& b, const LaunchCfg& c, dim3 g, int j, hipStream_t st) {
  const bool last = j == c.m - 1;
  if (j < kFixedCols) arnoldi_fixed<TV>(b, g, j, last, st, std::make_integer_sequence<int, kFixedCols>{});
  else arnoldi_mj<TV, 48, -1>(b, g, j, last, st);
}

hipError_t launch_arnoldi(const Batch& b, const LaunchCfg& c, int j, hipStream_t st) {
  dim3 g(red_grid(c.J, b.n) * b.n);
  if (j >= c.m || c.m > kMaxM) return hipErrorInvalidValue;
  if (c.vb) arnoldi_t<float>(b, c, g, j, st);
  else arnoldi_t<double>(b, c, g, j, st);
  if (j == c.m - 1) hipLaunchKernelGGL(k_gs_last, dim3(b.n), dim3(256), 0, st, b);
  return hipGetLastError();
}

// ---------------------------------------------------------------- phi_1
// y = phi_1(dt H_k) e_1 = last column of exp([[dt H_k, e_1], [0, 0]]) (first
// k entries), k = m_eff.  exp by scaling and squaring of a degree-18 Taylor
// polynomial: ||A/2^s||_1 <= 1/2 bounds the truncation by 1e-22 relative.
// The polynomial is evaluated in the Paterson-Stockmeyer form (Paterson and
// Stockmeyer 1973): with X = A^3 and B_k = c_3k I + c_3k+1 A + c_3k+2 A^2,
// p(A) = B_0 + X (B_1 + X (B_2 + X (B_3 + X (B_4 + X (B_5 + c_18 X))))),
// seven matrix products (A^2, A^3 and five in X) instead of Horner's 17.
constexpr int kTaylor = 18;
struct TaylorCoef {
  double c[kTaylor + 1];
  constexpr TaylorCoef() : c() {
    c[0] = 1.0;
    for (int i = 1; i <= kTaylor; ++i) c[i] = c[i - 1] / i;
  }
};
static_assert(kTaylor == 18, "the evaluation below is written for degree 3 * 6");

// C = A B (K x K, LDS).  The sum over l keeps its order; unrolled, the LDS
// loads of eight terms are issued before their products, so a term no longer
// waits for its own loads.
__device__ void mat_mul(const double* A, const double* B, double* C, int K) {
  for (int q = threadIdx.x; q < K * K; q += blockDim.x) {
    const int i = q / K, j = q - i * K;
    double t = 0.0;
#pragma unroll 8
    for (int l = 0; l < K; ++l) t += A[i * K + l] * B[l * K + j];
    C[q] = t;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_phi1(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int k = s.ctrl[C_MEFF];      // 0 after a non-finite value or for F = 0
  if (k <= 0) return;
  const int K = k + 1, m = s.m;
  __shared__ double A[(kMaxM + 1) * (kMaxM + 1)];
  __shared__ double A2[(kMaxM + 1) * (kMaxM + 1)];
  __shared__ double X[(kMaxM + 1) * (kMaxM + 1)];
  __shared__ double Pm[(kMaxM + 1) * (kMaxM + 1)];
  __shared__ double Tm[(kMaxM + 1) * (kMaxM + 1)];
  __shared__ double colsum[kMaxM + 1];
  __shared__ int sc;
  const double dt = s.dt;
  for (int q = threadIdx.x; q < K * K; q += blockDim.x) {
    const int i = q / K, j = q - i * K;
    double v = 0.0;
    if (i < k && j < k && i <= j + 1) v = dt * s.H[i * m + j];   // Hessenberg part only
    else if (i == 0 && j == k) v = 1.0;
    A[q] = v;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < K; j += blockDim.x) {
    double t = 0.0;
    for (int i = 0; i < K; ++i) t += fabs(A[i * K + j]);
    colsum[j] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double nrm = 0.0;
    for (int j = 0; j < K; ++j) nrm = fmax(nrm, colsum[j]);
    int e = 0;
    if (nrm > 0.5) e = (int)ceil(log2(nrm / 0.5));
    if (e > 60) e = 60;
    sc = e;
  }
  __syncthreads();
  const double scale = ldexp(1.0, -sc);
  for (int q = threadIdx.x; q < K * K; q += blockDim.x) A[q] *= scale;
  __syncthreads();
  constexpr TaylorCoef tc;
  mat_mul(A, A, A2, K);
  mat_mul(A2, A, X, K);
  // Pm = B_5 + c_18 X, then Pm = B_k + X Pm for k = 4 .. 0
  for (int q = threadIdx.x; q < K * K; q += blockDim.x) {
    const int i = q / K, j = q - i * K;
    Pm[q] = (i == j ? tc.c[15] : 0.0) + tc.c[16] * A[q] + tc.c[17] * A2[q] + tc.c[18] * X[q];
  }
  __syncthreads();
  for (int kb = 4; kb >= 0; --kb) {
    mat_mul(X, Pm, Tm, K);
    const double c0 = tc.c[3 * kb], c1 = tc.c[3 * kb + 1], c2 = tc.c[3 * kb + 2];
    for (int q = threadIdx.x; q < K * K; q += blockDim.x) {
      const int i = q / K, j = q - i * K;
      Pm[q] = (i == j ? c0 : 0.0) + c1 * A[q] + c2 * A2[q] + Tm[q];
    }
    __syncthreads();
  }
  for (int r = 0; r < sc; ++r) {
    mat_mul(Pm, Pm, Tm, K);
    for (int q = threadIdx.x; q < K * K; q += blockDim.x) Pm[q] = Tm[q];
    __syncthreads();
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) s.y[i] = Pm[i * K + k];
}

hipError_t launch_phi1(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_phi1, dim3((1) * b.n), dim3(256), 0, st, b);
  return hipGetLastError();
}

// State update from the Krylov solution y:
//   mode 0 (exponential step):   omega_M += dt beta V_k y, the time advances;
//   mode 1 (Newton iteration):   omega_M += V_k y (y carries beta);
//   mode 2 (last Newton iteration): as mode 1, then the time advances.
template <typename TV>
__global__ void __launch_bounds__(256) k_update(Batch b, int mode) {
  const SolveDev& s = MRA_SOLVE(b);
  const int k = s.ctrl[C_MEFF];
  const int na = (int)*s.n_active;
  if (MRA_BX(b) == 0 && threadIdx.x == 0) {
    // a frozen solve (capacity exceeded, n_active 0) does not advance
    if (mode != 1 && !s.ctrl[C_OVER]) {
      s.scal[S_T] += s.dt;
      s.scal[S_STEPS] += 1.0;
    }
    // active-point residual evaluations: one F and k products J v
    s.scal[S_EVALS] += (double)(1 + k) * (double)na;
  }
  if (k <= 0) return;
  const size_t Nf = (size_t)s.vs;   // basis stride
  __shared__ double yy[kMaxM + 1];
  const double f = mode == 0 ? s.dt * s.scal[S_BETA] : 1.0;
  for (int i = threadIdx.x; i < k; i += blockDim.x) yy[i] = f * s.y[i];
  __syncthreads();
  bool bad = false;
  const auto* V = glb(vbasis<TV>(s));
  auto* om = glb(s.omega);
  for (int q = MRA_BX(b) * blockDim.x + threadIdx.x; q < na; q += MRA_GX(b) * blockDim.x) {
    double t = 0.0;
    for (int i = 0; i < k; ++i) t += yy[i] * (double)V[i * Nf + q];
    const double nv = om[q] + t;
    bad |= !isfinite(nv);
    om[q] = nv;
  }
  if (bad) s.ctrl[C_STATUS] = 5;
}

static int update_grid(int J) {
  const int nf = 1 << (2 * J);
  int nb = (nf + 255) / 256;
  return nb > 1024 ? 1024 : nb;
}

hipError_t launch_update(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  if (!c.vb) hipLaunchKernelGGL(k_update<double>, dim3(update_grid(c.J) * b.n), dim3(256), 0, st, b, 0);
  else hipLaunchKernelGGL(k_update<float>, dim3(update_grid(c.J) * b.n), dim3(256), 0, st, b, 0);
  return hipGetLastError();
}

hipError_t launch_newton_update(const Batch& b, const LaunchCfg& c, int last, hipStream_t st) {
  const int mode = last ? 2 : 1;
  if (!c.vb) hipLaunchKernelGGL(k_update<double>, dim3(update_grid(c.J) * b.n), dim3(256), 0, st, b, mode);
  else hipLaunchKernelGGL(k_update<float>, dim3(update_grid(c.J) * b.n), dim3(256), 0, st, b, mode);
  return hipGetLastError();
}

// ------------------------------------------------- theta-scheme Newton
// The implicit alternative to the exponential step: the theta-scheme
//   G(omega) = omega - omega_n - dt [theta F(omega) + (1 - theta) F(omega_n)] = 0
// on the active set of the step's start, solved by a fixed number of Newton
// iterations (I - theta dt J(omega_k)) d = -G(omega_k), each linear system by
// one GMRES(m) cycle from a zero guess (Section 2.1 places the method among
// Newton-Krylov solvers).  J is the Jacobian at frozen eddy viscosity, the
// operator of the exponential step.

// w <- -G(omega_k) = (omega_n - omega_k) + dt (theta F(omega_k) + (1 - theta) F(omega_n)),
// with F(omega_k) in w on entry.  The first iteration (omega_0 = omega_n)
// keeps omega_n and F(omega_n) in the FP64 regrid buffers, which the step
// does not otherwise use before its regrid.
__global__ void __launch_bounds__(256) k_newton_rhs(Batch b, int first) {
  const SolveDev& s = MRA_SOLVE(b);
  const int na = (int)*s.n_active;
  const double th = s.scal[S_THETA], dt = s.dt;
  auto* wn = glb(s.packed64);
  auto* fn = glb(s.dense64);
  auto* W = glb(s.w);
  const auto* Om = glb(s.omega);
  for (int q = MRA_BX(b) * blockDim.x + threadIdx.x; q < na; q += MRA_GX(b) * blockDim.x) {
    const double f = W[q], om = Om[q];
    double on, f0;
    if (first) {
      wn[q] = om;
      fn[q] = f;
      on = om;
      f0 = f;
    } else {
      on = wn[q];
      f0 = fn[q];
    }
    W[q] = (on - om) + dt * (th * f + (1.0 - th) * f0);
  }
}

hipError_t launch_newton_rhs(const Batch& b, const LaunchCfg& c, int first, hipStream_t st) {
  hipLaunchKernelGGL(k_newton_rhs, dim3(update_grid(c.J) * b.n), dim3(256), 0, st, b, first);
  return hipGetLastError();
}

// GMRES least squares.  The Arnoldi basis of J started from r = -G spans the
// Krylov space of A = I - theta dt J, and A V_k = V_{k+1} (I~ - theta dt H_k)
// with I~ the k x k identity over a zero row; the correction is d = V_k y with
// y minimising ||beta e_1 - (I~ - theta dt H_k) y||.  Givens rotations reduce
// the (k+1) x k Hessenberg matrix to triangular form; one thread does the
// O(k^2) work (k <= 47).
__global__ void __launch_bounds__(256) k_gmres(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int k = s.ctrl[C_MEFF];      // 0 after a non-finite value or for -G = 0
  if (k <= 0) return;
  const int m = s.m;
  const double a = s.scal[S_THETA] * s.dt;
  __shared__ double R[(kMaxM + 1) * kMaxM];
  __shared__ double g[kMaxM + 1];
  for (int q = threadIdx.x; q < (k + 1) * k; q += blockDim.x) {
    const int i = q / k, j = q - i * k;
    double v = 0.0;
    if (i == k) {
      if (j == k - 1) v = -a * s.H[i * m + j];      // h_{k+1,k}, stored where the column ended
    } else if (i <= j + 1) {
      v = (i == j ? 1.0 : 0.0) - a * s.H[i * m + j];
    }
    R[q] = v;
  }
  for (int i = threadIdx.x; i <= k; i += blockDim.x) g[i] = i == 0 ? s.scal[S_BETA] : 0.0;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int j = 0; j < k; ++j) {
    const double x = R[j * k + j], y = R[(j + 1) * k + j];
    const double r = hypot(x, y);
    const double c = r > 0.0 ? x / r : 1.0, sn = r > 0.0 ? y / r : 0.0;
    for (int l = j; l < k; ++l) {
      const double p = R[j * k + l], q = R[(j + 1) * k + l];
      R[j * k + l] = c * p + sn * q;
      R[(j + 1) * k + l] = c * q - sn * p;
    }
    const double p = g[j], q = g[j + 1];
    g[j] = c * p + sn * q;
    g[j + 1] = c * q - sn * p;
  }
  bool bad = false;
  for (int j = k - 1; j >= 0; --j) {
    double t = g[j];
    for (int l = j + 1; l < k; ++l) t -= R[j * k + l] * g[l];
    const double d = R[j * k + j];
    g[j] = d != 0.0 ? t / d : 0.0;      // a singular projected system takes no step there
    bad |= !isfinite(g[j]);
  }
  for (int j = 0; j < k; ++j) s.y[j] = g[j];
  if (bad) {
    s.ctrl[C_STATUS] = 5;
    s.ctrl[C_MEFF] = 0;
  }
}

hipError_t launch_gmres(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres, dim3((1) * b.n), dim3(256), 0, st, b);
  return hipGetLastError();
}

// One device scalar of every solve of b (the theta of the theta-scheme, the
// condensation rate of a scalar), written in stream order.
__global__ void k_set_scal(Batch b, int idx, double value) {
  if (threadIdx.x == 0) MRA_SOLVE(b).scal[idx] = value;
}

hipError_t launch_set_scal(const Batch& b, int idx, double value, hipStream_t st) {
  if (idx < 0 || idx >= S_NSCAL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_set_scal, dim3((1) * b.n), dim3(64), 0, st, b, idx, value);
  return hipGetLastError();
}

__global__ void k_reset_ctrl(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  for (int i = threadIdx.x; i < C_NCTRL; i += blockDim.x) s.ctrl[i] = 0;
  for (int i = threadIdx.x; i < S_NSCAL; i += blockDim.x) s.scal[i] = 0.0;
}

__global__ void k_clear_done(Batch b) {
  if (threadIdx.x == 0) MRA_SOLVE(b).ctrl[C_DONE] = 0;
}

hipError_t launch_clear_done(const Batch& b, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_done, dim3((1) * b.n), dim3(64), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_reset_ctrl(const Batch& b, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_ctrl, dim3((1) * b.n), dim3(64), 0, st, b);
  return hipGetLastError();
}

}  // namespace mra
