// Krylov part of the exponential Rosenbrock-Euler step, FP64:
// Arnoldi with classical Gram-Schmidt and one reorthogonalisation (CGS2),
// phi_1(dt H) e_1 from the exponential of the augmented Hessenberg matrix,
// and the state update omega_M += dt beta V y.
//
// The paper advances the collocation system by projecting it onto a Krylov
// subspace (abstract; Section 2.1); the exponential Euler step with the
// Jacobian at frozen eddy viscosity is the reading implemented here.
//
// Reductions over the active nodes are deterministic: the active list is cut
// into the same fixed chunks in every kernel of a step (the chunk count
// depends only on N_a), every block reduces its chunk in a fixed order, and
// the last block to finish (device-scope counter) adds the block partials in
// block order.
#include "mra_internal.hpp"

namespace mra {

constexpr double kBreakdown = 1e-13;
constexpr int kChunkMin = 2048;

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

struct Chunk {
  int nb, lo, hi;
};
__device__ inline Chunk chunk_of(int na) {
  int nb = (na + kChunkMin - 1) / kChunkMin;
  if (nb < 1) nb = 1;
  if (nb > kRedBlocks) nb = kRedBlocks;
  const int per = (na + nb - 1) / nb;
  Chunk c;
  c.nb = nb;
  c.lo = blockIdx.x * per;
  c.hi = c.lo + per < na ? c.lo + per : na;
  return c;
}

// Per block: partial sums of cnt values written to partials[blk][0..cnt).
// Returns true in exactly one block (the last to finish), after a device
// fence, with every block's partials visible.
__device__ bool publish_partials(const SolveDev& s, int nb, int cnt, double* red /*[4][kMaxM+2]*/,
                                 int counter) {
  __syncthreads();
  const int stride = kMaxM + 2;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    double t = red[i] + red[stride + i];
    t += red[2 * stride + i];
    t += red[3 * stride + i];
    s.partials[blockIdx.x * stride + i] = t;
  }
  __threadfence();
  __syncthreads();
  __shared__ int last;
  if (threadIdx.x == 0) {
    const int prev = atomicAdd(&s.ctrl[counter], 1);
    last = prev == nb - 1;
    if (last) s.ctrl[counter] = 0;
  }
  __syncthreads();
  if (last) __threadfence();
  return last != 0;
}

// In the last block: totals[i] = sum over blocks (in block order) of the
// partials, i < cnt.  One wave per value, lanes stride the blocks.
__device__ void reduce_partials(const SolveDev& s, int nb, int cnt, double* totals) {
  const int stride = kMaxM + 2;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i = wid; i < cnt; i += nw) {
    double t = 0.0;
    for (int b = lane; b < nb; b += 64) t += __hip_atomic_load(&s.partials[b * stride + i], __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT);
    t = wave_sum(t);
    if (lane == 0) totals[i] = t;
  }
  __syncthreads();
}

// ||w||^2 over a chunk, stored in red[wave][slot]
__device__ inline void chunk_dot(const double* a, const double* b, int lo, int hi, double* red, int slot) {
  double t = 0.0;
  for (int k = lo + threadIdx.x; k < hi; k += blockDim.x) t += a[k] * b[k];
  t = wave_sum(t);
  if ((threadIdx.x & 63) == 0) red[(threadIdx.x >> 6) * (kMaxM + 2) + slot] = t;
}

// beta = ||F||; v_1 scaling, flags.
__global__ void __launch_bounds__(256) k_norm0(Batch b) {
  const SolveDev& s = *b.s[blockIdx.y];
  const int na = (int)*s.n_active;
  const Chunk c = chunk_of(na);
  if ((int)blockIdx.x >= c.nb) return;
  __shared__ double red[4 * (kMaxM + 2)];
  __shared__ double tot[kMaxM + 2];
  chunk_dot(s.w, s.w, c.lo, c.hi, red, 0);
  if (!publish_partials(s, c.nb, 1, red, C_CNT0)) return;
  reduce_partials(s, c.nb, 1, tot);
  if (threadIdx.x == 0) {
    const double beta = sqrt(tot[0]);
    s.scal[S_BETA] = beta;
    const bool ok = isfinite(beta);
    if (!ok) s.ctrl[C_STATUS] = 5;
    const bool zero = !(beta > 0.0) || !ok;
    s.ctrl[C_DONE] = zero ? 1 : 0;
    s.ctrl[C_MEFF] = zero ? 0 : s.m;
    s.scal[S_INV] = zero ? 0.0 : 1.0 / beta;
  }
}

// Stage 1: h1 = V_j^T w, ||w||^2 (= ||A v_j||^2).
__global__ void __launch_bounds__(256) k_gs_dot(Batch b, int j) {
  const SolveDev& s = *b.s[blockIdx.y];
  if (s.ctrl[C_DONE]) return;
  const int na = (int)*s.n_active;
  const Chunk c = chunk_of(na);
  if ((int)blockIdx.x >= c.nb) return;
  const size_t Nf = (size_t)s.N * s.N;
  __shared__ double red[4 * (kMaxM + 2)];
  __shared__ double tot[kMaxM + 2];
  for (int i = 0; i <= j; ++i) chunk_dot(s.V + i * Nf, s.w, c.lo, c.hi, red, i);
  chunk_dot(s.w, s.w, c.lo, c.hi, red, j + 1);
  if (!publish_partials(s, c.nb, j + 2, red, C_CNT1)) return;
  reduce_partials(s, c.nb, j + 2, tot);
  for (int i = threadIdx.x; i <= j; i += blockDim.x) s.hpart[i] = tot[i];
  if (threadIdx.x == 0) s.scal[S_NRMAV] = sqrt(tot[j + 1]);
}

// Stage 2: w -= V_j h1; h2 = V_j^T w.
__global__ void __launch_bounds__(256) k_gs_axpy_dot(Batch b, int j) {
  const SolveDev& s = *b.s[blockIdx.y];
  if (s.ctrl[C_DONE]) return;
  const int na = (int)*s.n_active;
  const Chunk c = chunk_of(na);
  if ((int)blockIdx.x >= c.nb) return;
  const size_t Nf = (size_t)s.N * s.N;
  __shared__ double red[4 * (kMaxM + 2)];
  __shared__ double tot[kMaxM + 2];
  __shared__ double h[kMaxM + 1];
  for (int i = threadIdx.x; i <= j; i += blockDim.x) h[i] = s.hpart[i];
  __syncthreads();
  for (int k = c.lo + threadIdx.x; k < c.hi; k += blockDim.x) {
    double t = s.w[k];
    for (int i = 0; i <= j; ++i) t -= h[i] * s.V[i * Nf + k];
    s.w[k] = t;
  }
  __syncthreads();
  for (int i = 0; i <= j; ++i) chunk_dot(s.V + i * Nf, s.w, c.lo, c.hi, red, i);
  if (!publish_partials(s, c.nb, j + 1, red, C_CNT2)) return;
  reduce_partials(s, c.nb, j + 1, tot);
  for (int i = threadIdx.x; i <= j; i += blockDim.x) s.hpart[(kMaxM + 1) + i] = tot[i];
}

// Stage 3: w -= V_j h2; H[:, j] = h1 + h2, H[j+1, j] = ||w||; breakdown test.
__global__ void __launch_bounds__(256) k_gs_axpy_norm(Batch b, int j) {
  const SolveDev& s = *b.s[blockIdx.y];
  if (s.ctrl[C_DONE]) return;
  const int na = (int)*s.n_active;
  const Chunk c = chunk_of(na);
  if ((int)blockIdx.x >= c.nb) return;
  const size_t Nf = (size_t)s.N * s.N;
  __shared__ double red[4 * (kMaxM + 2)];
  __shared__ double tot[kMaxM + 2];
  __shared__ double h[kMaxM + 1];
  for (int i = threadIdx.x; i <= j; i += blockDim.x) h[i] = s.hpart[(kMaxM + 1) + i];
  __syncthreads();
  for (int k = c.lo + threadIdx.x; k < c.hi; k += blockDim.x) {
    double t = s.w[k];
    for (int i = 0; i <= j; ++i) t -= h[i] * s.V[i * Nf + k];
    s.w[k] = t;
  }
  __syncthreads();
  chunk_dot(s.w, s.w, c.lo, c.hi, red, 0);
  if (!publish_partials(s, c.nb, 1, red, C_CNT3)) return;
  reduce_partials(s, c.nb, 1, tot);
  const int m = s.m;
  for (int i = threadIdx.x; i <= j; i += blockDim.x) s.H[i * m + j] = s.hpart[i] + h[i];
  if (threadIdx.x == 0) {
    const double hn = sqrt(tot[0]);
    s.H[(j + 1) * m + j] = hn;
    const double nav = s.scal[S_NRMAV];
    if (!isfinite(hn) || !isfinite(nav)) {
      s.ctrl[C_STATUS] = 5;
      s.ctrl[C_DONE] = 1;
      s.ctrl[C_MEFF] = 0;
    } else if (hn <= kBreakdown * nav || j + 1 == m) {
      s.ctrl[C_DONE] = 1;
      s.ctrl[C_MEFF] = j + 1;
    } else {
      s.scal[S_INV] = 1.0 / hn;
    }
  }
}

hipError_t launch_norm0(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_norm0, dim3(kRedBlocks, b.n), dim3(256), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_arnoldi(const Batch& b, const LaunchCfg& c, int j, hipStream_t st) {
  dim3 g(kRedBlocks, b.n);
  hipLaunchKernelGGL(k_gs_dot, g, dim3(256), 0, st, b, j);
  hipLaunchKernelGGL(k_gs_axpy_dot, g, dim3(256), 0, st, b, j);
  hipLaunchKernelGGL(k_gs_axpy_norm, g, dim3(256), 0, st, b, j);
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
  const SolveDev& s = *b.s[blockIdx.y];
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
  hipLaunchKernelGGL(k_phi1, dim3(1, b.n), dim3(256), 0, st, b);
  return hipGetLastError();
}

// omega_M += dt beta V_k y; the time advances.
__global__ void __launch_bounds__(256) k_update(Batch b) {
  const SolveDev& s = *b.s[blockIdx.y];
  const int k = s.ctrl[C_MEFF];
  const int na = (int)*s.n_active;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
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
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < na; q += gridDim.x * blockDim.x) {
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
  hipLaunchKernelGGL(k_update, dim3(nb, b.n), dim3(256), 0, st, b);
  return hipGetLastError();
}

__global__ void k_reset_ctrl(Batch b) {
  const SolveDev& s = *b.s[blockIdx.y];
  for (int i = threadIdx.x; i < C_NCTRL; i += blockDim.x) s.ctrl[i] = 0;
  for (int i = threadIdx.x; i < S_NSCAL; i += blockDim.x) s.scal[i] = 0.0;
}

__global__ void k_clear_done(Batch b) {
  if (threadIdx.x == 0) b.s[blockIdx.y]->ctrl[C_DONE] = 0;
}

hipError_t launch_clear_done(const Batch& b, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_done, dim3(1, b.n), dim3(64), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_reset_ctrl(const Batch& b, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_ctrl, dim3(1, b.n), dim3(64), 0, st, b);
  return hipGetLastError();
}

}  // namespace mra
