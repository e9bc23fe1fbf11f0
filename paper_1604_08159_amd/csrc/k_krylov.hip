// Krylov part of the exponential Rosenbrock-Euler step, FP64:
// Arnoldi with classical Gram-Schmidt and one reorthogonalisation (CGS2),
// phi_1(dt H) e_1 from the exponential of the augmented Hessenberg matrix,
// and the state update omega_M += dt beta V y.
//
// The paper advances the collocation system by projecting it onto a Krylov
// subspace (abstract; Section 2.1); the exponential Euler step with the
// Jacobian at frozen eddy viscosity is the reading implemented here.
//
// Reductions over the active nodes are deterministic and need no cross-block
// signalling: the active list is cut into the same fixed chunks in every
// kernel of a step (the chunk count depends only on N_a), one wavefront per
// basis vector reduces a chunk in a fixed order into a per-chunk partial, and
// every block of the NEXT kernel adds the partials in the same fixed order
// (the kernel boundary orders the writes before the reads).
#include "mra_internal.hpp"

namespace mra {

// Gram-Schmidt kernels.  A thread takes the elements lo + tid, lo + tid + 256,
// ... of its chunk; for each it loads w and all basis entries V_i[k], i <= j,
// at once (MJ >= j + 1 register slots, MJ fixed at compile time from m), so a
// chunk costs one dependent global round per element instead of one per group
// of basis vectors.

// ||F||^2 partials (buffer B).
__global__ void __launch_bounds__(256) k_norm0(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int na = (int)*s.n_active;
  const int nb = nchunks(na);
  for (int ch = MRA_BX(b); ch < nb; ch += MRA_GX(b)) {
    const Chunk c = chunk_of(na, ch);
    double acc[1] = {0.0};
    for (int k = c.lo + (int)threadIdx.x; k < c.hi; k += blockDim.x) acc[0] += s.w[k] * s.w[k];
    block_sums_store<1>(acc, 1, part_buf(s, 1) + (size_t)ch * (kMaxM + 2));
    __syncthreads();
  }
}

// Stage 1: h1 = V_j^T w and ||w||^2 (= ||A v_j||^2) partials (buffer A).
template <int MJ>
__global__ void __launch_bounds__(256) k_gs_dot(Batch b, int j) {
  const SolveDev& s = MRA_SOLVE(b);
  if (s.ctrl[C_DONE]) return;
  const int na = (int)*s.n_active;
  const int nb = nchunks(na);
  const size_t Nf = (size_t)s.N * s.N;
  for (int ch = MRA_BX(b); ch < nb; ch += MRA_GX(b)) {
    const Chunk c = chunk_of(na, ch);
    double acc[MJ + 1];
#pragma unroll
    for (int i = 0; i <= MJ; ++i) acc[i] = 0.0;
    for (int k = c.lo + (int)threadIdx.x; k < c.hi; k += blockDim.x) {
      const double wk = s.w[k];
      double v[MJ];
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i <= j) v[i] = s.V[i * Nf + k];
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i <= j) acc[i] += v[i] * wk;
      acc[MJ] += wk * wk;
    }
    // slot layout: h1[0 .. j], then ||w||^2 at j + 1 (static register indices)
#pragma unroll
    for (int i = 0; i < MJ; ++i)
      if (i == j + 1) acc[i] = acc[MJ];
    block_sums_store<MJ + 1>(acc, j + 2, part_buf(s, 0) + (size_t)ch * (kMaxM + 2));
    __syncthreads();
  }
}

// Stage 2: h1 from A; w -= V_j h1; h2 = V_j^T w partials (buffer B).
template <int MJ>
__global__ void __launch_bounds__(256) k_gs_axpy_dot(Batch b, int j) {
  const SolveDev& s = MRA_SOLVE(b);
  if (s.ctrl[C_DONE]) return;
  const int na = (int)*s.n_active;
  const int nb = nchunks(na);
  if ((int)MRA_BX(b) >= nb) return;
  __shared__ double h[kMaxM + 2];
  reduce_partials(part_buf(s, 0), nb, j + 2, h);
  if (MRA_BX(b) == 0) {
    for (int i = threadIdx.x; i <= j; i += blockDim.x) s.hpart[i] = h[i];
    if (threadIdx.x == 0) s.scal[S_NRMAV] = sqrt(h[j + 1]);
  }
  const size_t Nf = (size_t)s.N * s.N;
  for (int ch = MRA_BX(b); ch < nb; ch += MRA_GX(b)) {
    const Chunk c = chunk_of(na, ch);
    double acc[MJ];
#pragma unroll
    for (int i = 0; i < MJ; ++i) acc[i] = 0.0;
    for (int k = c.lo + (int)threadIdx.x; k < c.hi; k += blockDim.x) {
      double t = s.w[k];
      double v[MJ];
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i <= j) v[i] = s.V[i * Nf + k];
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i <= j) t -= h[i] * v[i];
      s.w[k] = t;
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i <= j) acc[i] += v[i] * t;
    }
    block_sums_store<MJ>(acc, j + 1, part_buf(s, 1) + (size_t)ch * (kMaxM + 2));
    __syncthreads();
  }
}

// Stage 3: h2 from B; w -= V_j h2; H[:j+1, j] = h1 + h2; ||w||^2 partials
// (buffer A), consumed by the next scaling (next_scale) or by phi_1.
template <int MJ>
__global__ void __launch_bounds__(256) k_gs_axpy_norm(Batch b, int j) {
  const SolveDev& s = MRA_SOLVE(b);
  if (s.ctrl[C_DONE]) return;
  const int na = (int)*s.n_active;
  const int nb = nchunks(na);
  if ((int)MRA_BX(b) >= nb) return;
  __shared__ double h[kMaxM + 2];
  reduce_partials(part_buf(s, 1), nb, j + 1, h);
  if (MRA_BX(b) == 0)
    for (int i = threadIdx.x; i <= j; i += blockDim.x) s.H[i * s.m + j] = s.hpart[i] + h[i];
  const size_t Nf = (size_t)s.N * s.N;
  for (int ch = MRA_BX(b); ch < nb; ch += MRA_GX(b)) {
    const Chunk c = chunk_of(na, ch);
    double acc[1] = {0.0};
    for (int k = c.lo + (int)threadIdx.x; k < c.hi; k += blockDim.x) {
      double t = s.w[k];
      double v[MJ];
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i <= j) v[i] = s.V[i * Nf + k];
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i <= j) t -= h[i] * v[i];
      s.w[k] = t;
      acc[0] += t * t;
    }
    block_sums_store<1>(acc, 1, part_buf(s, 0) + (size_t)ch * (kMaxM + 2));
    __syncthreads();
  }
}

// Grid of the reductions: at most kRedGrid blocks per solve (blocks loop
// over chunks), fewer on grids too small to fill them.
constexpr int kRedGrid = 64;
static int red_grid(int J) {
  const int nf = 1 << (2 * J);
  int g = (nf + kChunkMin - 1) / kChunkMin;
  return g < kRedGrid ? g : kRedGrid;
}

hipError_t launch_norm0(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_norm0, dim3((red_grid(c.J)) * b.n), dim3(256), 0, st, b);
  return hipGetLastError();
}

template <int MJ>
static void arnoldi_mj(const Batch& b, dim3 g, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_gs_dot<MJ>, g, dim3(256), 0, st, b, j);
  hipLaunchKernelGGL(k_gs_axpy_dot<MJ>, g, dim3(256), 0, st, b, j);
  hipLaunchKernelGGL(k_gs_axpy_norm<MJ>, g, dim3(256), 0, st, b, j);
}

// basis-vector register slots: the smallest bucket holding m vectors
hipError_t launch_arnoldi(const Batch& b, const LaunchCfg& c, int j, hipStream_t st) {
  dim3 g((red_grid(c.J)) * b.n);
  if (j >= c.m || c.m > kMaxM) return hipErrorInvalidValue;
  if (c.m <= 8) arnoldi_mj<8>(b, g, j, st);
  else if (c.m <= 16) arnoldi_mj<16>(b, g, j, st);
  else if (c.m <= 24) arnoldi_mj<24>(b, g, j, st);
  else if (c.m <= 32) arnoldi_mj<32>(b, g, j, st);
  else arnoldi_mj<48>(b, g, j, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------- phi_1
// y = phi_1(dt H_k) e_1 = last column of exp([[dt H_k, e_1], [0, 0]]) (first
// k entries), k = m_eff.  exp by scaling and squaring of a degree-18 Taylor
// polynomial: ||A/2^s||_1 <= 1/2 bounds the truncation by 1e-22 relative.
constexpr int kTaylor = 18;

__device__ void mat_mul(const double* A, const double* B, double* C, int K) {
  for (int q = threadIdx.x; q < K * K; q += blockDim.x) {
    const int i = q / K, j = q - i * K;
    double t = 0.0;
    for (int l = 0; l < K; ++l) t += A[i * K + l] * B[l * K + j];
    C[q] = t;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_phi1(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  // the last column's norm (partials of stage 3): only its finiteness matters
  if (!s.ctrl[C_DONE]) {
    __shared__ double tot[2];
    reduce_partials(part_buf(s, 0), nchunks((int)*s.n_active), 1, tot);
    if (threadIdx.x == 0 && !isfinite(tot[0])) {
      s.ctrl[C_STATUS] = 5;
      s.ctrl[C_MEFF] = 0;
    }
    __syncthreads();
  }
  const int k = s.ctrl[C_MEFF];
  if (k <= 0) return;
  const int K = k + 1, m = s.m;
  __shared__ double A[(kMaxM + 1) * (kMaxM + 1)];
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
  for (int q = threadIdx.x; q < K * K; q += blockDim.x) {
    A[q] *= scale;
    const int i = q / K, j = q - i * K;
    Pm[q] = (i == j ? 1.0 : 0.0) + A[q] / kTaylor;
  }
  __syncthreads();
  for (int d = kTaylor - 1; d >= 1; --d) {
    mat_mul(A, Pm, Tm, K);
    const double inv = 1.0 / d;
    for (int q = threadIdx.x; q < K * K; q += blockDim.x) {
      const int i = q / K, j = q - i * K;
      Pm[q] = (i == j ? 1.0 : 0.0) + Tm[q] * inv;
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

// omega_M += dt beta V_k y; the time advances.
__global__ void __launch_bounds__(256) k_update(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int k = s.ctrl[C_MEFF];
  const int na = (int)*s.n_active;
  if (MRA_BX(b) == 0 && threadIdx.x == 0) {
    s.scal[S_T] += s.dt;
    s.scal[S_STEPS] += 1.0;
    // active-point residual evaluations of this step: F and k products J v
    s.scal[S_EVALS] += (double)(1 + k) * (double)na;
  }
  if (k <= 0) return;
  const size_t Nf = (size_t)s.N * s.N;
  __shared__ double yy[kMaxM + 1];
  const double f = s.dt * s.scal[S_BETA];
  for (int i = threadIdx.x; i < k; i += blockDim.x) yy[i] = f * s.y[i];
  __syncthreads();
  bool bad = false;
  for (int q = MRA_BX(b) * blockDim.x + threadIdx.x; q < na; q += MRA_GX(b) * blockDim.x) {
    double t = 0.0;
    for (int i = 0; i < k; ++i) t += yy[i] * s.V[i * Nf + q];
    const double nv = s.omega[q] + t;
    bad |= !isfinite(nv);
    s.omega[q] = nv;
  }
  if (bad) s.ctrl[C_STATUS] = 5;
}

hipError_t launch_update(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  const int nf = 1 << (2 * c.J);
  int nb = (nf + 255) / 256;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_update, dim3((nb) * b.n), dim3(256), 0, st, b);
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
