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
  return reinterpret_cast<T*>(s.dense64);
}

// ---------------------------------------------------------------- scatter
// src 0: omega; src 1: V[j] = w * inv (stored), then scattered; src 2: vin.
template <typename T>
__global__ void __launch_bounds__(256) k_scatter(Batch b, int src, int target, int j) {
  const SolveDev& s = MRA_SOLVE(b);
  const int na = (int)*s.n_active;
  const int Nf = s.N * s.N;
  T* dense = dense_target<T>(s, target);
  const int* fi = s.index_fine;
  if (src == 0) {
    const double* om = s.omega;
    for (int k = MRA_BX(b) * blockDim.x + threadIdx.x; k < na; k += MRA_GX(b) * blockDim.x)
      dense[fi[k]] = (T)om[k];
  } else if (src == 2) {
    const double* vin = s.vin;
    for (int k = MRA_BX(b) * blockDim.x + threadIdx.x; k < na; k += MRA_GX(b) * blockDim.x)
      dense[fi[k]] = (T)vin[k];
  } else {
    const double inv = next_scale(s, j, MRA_BX(b));
    const bool done = inv == 0.0;
    double* Vj = s.V + (size_t)j * Nf;
    const double* w = s.w;
    for (int k = MRA_BX(b) * blockDim.x + threadIdx.x; k < na; k += MRA_GX(b) * blockDim.x) {
      double val = 0.0;
      if (!done) {
        val = w[k] * inv;
        Vj[k] = val;
      }
      dense[fi[k]] = (T)val;
    }
  }
}

static int scatter_blocks(int J) {
  int nf = 1 << (2 * J);
  int nb = (nf + 255) / 256;
  return nb < 1024 ? nb : 1024;
}

hipError_t launch_scatter(const Batch& b, const LaunchCfg& c, int src, int target, int j, hipStream_t st) {
  dim3 g((scatter_blocks(c.J)) * b.n);
  if (target == 2 || c.prec == 0)
    hipLaunchKernelGGL(k_scatter<double>, g, dim3(256), 0, st, b, src, target, j);
  else
    hipLaunchKernelGGL(k_scatter<float>, g, dim3(256), 0, st, b, src, target, j);
  return hipGetLastError();
}

// ---------------------------------------------------------------- prolong
// mode 0: Pi (inactive nodes predicted, active kept); mode 1: inverse
// transform (every node = detail + prediction, details from `packed`).
template <int P, typename T>
__device__ inline void prolong_node(T* __restrict__ f, const uint8_t* __restrict__ mask,
                                    const T* __restrict__ packed, int i, int l, int J, int j0,
                                    int mode) {
#pragma clang fp contract(off)
  if (mode == 0 && mask[i]) return;
  int lv;
  const int fi = packed_to_fine(i, J, j0, &lv);
  const int N = 1 << J;
  const T pr = predict_node<P, T>(f, fi & (N - 1), fi >> J, l, J);
  f[fi] = mode == 0 ? pr : packed[i] + pr;
}

// Levels j0+1 .. Lc (Lc = min(J, kCoarseLevels)) for one solve per block: the
// 2^Lc x 2^Lc sub-grid of stride 2^(J-Lc) is gathered into LDS (active
// values from the dense field, through the contiguous coarse part of the
// packed mask), every coarse level is swept in LDS with the same arithmetic
// as the fine levels, and the predicted nodes are written back.
// mode 1 (inverse transform) adds the details of the packed input instead.
template <int P, typename T>
__global__ void __launch_bounds__(1024) k_prolong_coarse(Batch b, int target, int lmax, int mode) {
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
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int fi = packed_to_fine(i, J, j0, nullptr);
    const int sub = ((fi >> J) / S) * n + (fi & (s.N - 1)) / S;
    const bool a = mode == 0 ? s.mask[i] != 0 : i < n0sq;
    act[sub] = a;
    if (a) val[sub] = f[fi];
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
  for (int i = n0sq + threadIdx.x; i < cnt; i += blockDim.x) {
    const int fi = packed_to_fine(i, J, j0, nullptr);
    const int sub = ((fi >> J) / S) * n + (fi & (s.N - 1)) / S;
    if (!act[sub]) f[fi] = val[sub];
  }
}

template <int P, typename T>
__global__ void __launch_bounds__(256) k_prolong_level(Batch b, int target, int l, int mode) {
  const SolveDev& s = MRA_SOLVE(b);
  T* f = dense_target<T>(s, target);
  const T* packed = mode == 1 ? reinterpret_cast<const T*>(s.spec) : nullptr;
  const int lo = 1 << (2 * (l - 1)), hi = 1 << (2 * l);
  const int i = lo + MRA_BX(b) * blockDim.x + threadIdx.x;
  if (i < hi) prolong_node<P, T>(f, s.mask, packed, i, l, s.J, s.j0, mode);
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

template <typename T>
static hipError_t prolong_t(const Batch& b, const LaunchCfg& c, int target, int mode, hipStream_t st) {
  const int j0 = c.p == 2 ? 2 : 3;
  dim3 g1((1) * b.n);
  if (mode == 1) hipLaunchKernelGGL(k_inverse_coarse<T>, g1, dim3(256), 0, st, b, target);
  if (c.p == 2)
    hipLaunchKernelGGL((k_prolong_coarse<2, T>), g1, dim3(1024), 0, st, b, target, kCoarseLevels, mode);
  else
    hipLaunchKernelGGL((k_prolong_coarse<3, T>), g1, dim3(1024), 0, st, b, target, kCoarseLevels, mode);
  for (int l = (kCoarseLevels > j0 ? kCoarseLevels : j0) + 1; l <= c.J; ++l) {
    const int cnt = 3 << (2 * (l - 1));
    dim3 g(((cnt + 255) / 256) * b.n);
    if (c.p == 2)
      hipLaunchKernelGGL((k_prolong_level<2, T>), g, dim3(256), 0, st, b, target, l, mode);
    else
      hipLaunchKernelGGL((k_prolong_level<3, T>), g, dim3(256), 0, st, b, target, l, mode);
  }
  return hipGetLastError();
}

hipError_t launch_prolong(const Batch& b, const LaunchCfg& c, int target, int as_double, hipStream_t st) {
  if (as_double) return prolong_t<double>(b, c, target, 0, st);
  return prolong_t<float>(b, c, target, 0, st);
}

hipError_t launch_prolong_level(const Batch& b, const LaunchCfg& c, int target, int as_double, int l,
                                hipStream_t st) {
  const int cnt = 3 << (2 * (l - 1));
  dim3 g(((cnt + 255) / 256) * b.n);
  if (as_double) {
    if (c.p == 2) hipLaunchKernelGGL((k_prolong_level<2, double>), g, dim3(256), 0, st, b, target, l, 0);
    else hipLaunchKernelGGL((k_prolong_level<3, double>), g, dim3(256), 0, st, b, target, l, 0);
  } else {
    if (c.p == 2) hipLaunchKernelGGL((k_prolong_level<2, float>), g, dim3(256), 0, st, b, target, l, 0);
    else hipLaunchKernelGGL((k_prolong_level<3, float>), g, dim3(256), 0, st, b, target, l, 0);
  }
  return hipGetLastError();
}

// inverse transform: packed input in s.spec (element type of prec), output wt.
hipError_t launch_inverse(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  if (c.prec == 0) return prolong_t<double>(b, c, 0, 1, st);
  return prolong_t<float>(b, c, 0, 1, st);
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
// 1 -> spec reinterpreted as a packed T array.
template <int P, typename T>
__global__ void __launch_bounds__(256) k_forward(Batch b, int src, int dst) {
#pragma clang fp contract(off)
  const SolveDev& s = MRA_SOLVE(b);
  const T* f = src == 0 ? reinterpret_cast<const T*>(s.dense64) : reinterpret_cast<const T*>(s.wt);
  T* out = dst == 0 ? reinterpret_cast<T*>(s.packed64) : reinterpret_cast<T*>(s.spec);
  const int J = s.J, j0 = s.j0, N = s.N;
  const int Nf = N * N;
  const int i = MRA_BX(b) * blockDim.x + threadIdx.x;
  double am = 0.0;
  if (i < Nf) {
    int l;
    const int fi = packed_to_fine(i, J, j0, &l);
    const T val = f[fi];
    am = fabs((double)val);
    out[i] = l == j0 ? val : val - predict_node<P, T>(f, fi & (N - 1), fi >> J, l, J);
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

hipError_t launch_forward(const Batch& b, const LaunchCfg& c, int src, int dst, hipStream_t st) {
  const int nf = 1 << (2 * c.J);
  dim3 g(((nf + 255) / 256) * b.n);
  const bool dbl = src == 0 || c.prec == 0;
  if (dbl) {
    if (c.p == 2) hipLaunchKernelGGL((k_forward<2, double>), g, dim3(256), 0, st, b, src, dst);
    else hipLaunchKernelGGL((k_forward<3, double>), g, dim3(256), 0, st, b, src, dst);
  } else {
    if (c.p == 2) hipLaunchKernelGGL((k_forward<2, float>), g, dim3(256), 0, st, b, src, dst);
    else hipLaunchKernelGGL((k_forward<3, float>), g, dim3(256), 0, st, b, src, dst);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- threshold
// Active test of packed position i: coarsest mesh, significant detail, or in
// the adjacent zone of a significant node Q of level l, i.e. this node lies on
// G^{min(l+1,J)} within periodic Chebyshev distance 2^(J-l) of Q.  Written as
// a gather: for every level l >= max(level-1, j0+1) the level-l nodes within
// that distance are examined.
template <typename TP>
__device__ inline bool is_active(const TP* __restrict__ d, int i, int J, int j0, double tau, int az) {
  if (i < (1 << (2 * j0))) return true;
  if (fabs((double)d[i]) >= tau) return true;
  if (!az) return false;
  int lp;
  const int f = packed_to_fine(i, J, j0, &lp);
  const int N = 1 << J, nm = N - 1;
  const int px = f & nm, py = f >> J;
  const int lmin = lp - 1 > j0 + 1 ? lp - 1 : j0 + 1;
  for (int l = lmin; l <= J; ++l) {
    const int s = 1 << (J - l), hs = s >> 1;
    int cx[3], cy[3], nx, ny;
    if ((px & (s - 1)) == 0) { cx[0] = px - s; cx[1] = px; cx[2] = px + s; nx = 3; }
    else { cx[0] = px - hs; cx[1] = px + hs; nx = 2; }
    if ((py & (s - 1)) == 0) { cy[0] = py - s; cy[1] = py; cy[2] = py + s; ny = 3; }
    else { cy[0] = py - hs; cy[1] = py + hs; ny = 2; }
    for (int a = 0; a < ny; ++a) {
      const int qy = cy[a] & nm;
      for (int c = 0; c < nx; ++c) {
        const int qx = cx[c] & nm;
        if (level_of(qx, qy, J, j0) != l) continue;
        if (fabs((double)d[fine_to_packed(qx, qy, l, J, j0)]) >= tau) return true;
      }
    }
  }
  return false;
}

template <typename TP>
__global__ void __launch_bounds__(kScanBlock) k_mask_count(Batch b, int packed_is_double) {
  const SolveDev& s = MRA_SOLVE(b);
  const TP* d = packed_is_double ? reinterpret_cast<const TP*>(s.packed64) : reinterpret_cast<const TP*>(s.spec);
  const int Nf = s.N * s.N;
  const double tau = s.eps * __longlong_as_double((long long)*s.umax);
  const int base = MRA_BX(b) * (kScanBlock * kScanItems) + threadIdx.x * kScanItems;
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    const int i = base + q;
    if (i < Nf) {
      const bool a = is_active<TP>(d, i, s.J, s.j0, tau, s.adjacent_zone);
      s.mask[i] = a ? 1 : 0;
      cnt += a;
    }
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
  if (threadIdx.x == 0) *s.n_active = total;
  const int ntiles = s.ntx * s.ntx;
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x) s.tile_count[t] = 0;
}

__global__ void __launch_bounds__(kScanBlock) k_compact(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int Nf = s.N * s.N;
  const int J = s.J, j0 = s.j0, N = s.N, T = s.tile, ntx = s.ntx;
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
      const int x = f & (N - 1), y = f >> J;
      atomicAdd(&s.tile_count[(y / T) * ntx + x / T], 1);
      ++pos;
    } else {
      s.rank[f] = -1;
    }
  }
}

hipError_t launch_threshold(const Batch& b, const LaunchCfg& c, int packed_is_double, hipStream_t st) {
  const int nf = 1 << (2 * c.J);
  const int nblk = (nf + kScanBlock * kScanItems - 1) / (kScanBlock * kScanItems);
  dim3 g((nblk) * b.n);
  if (packed_is_double || c.prec == 0)
    hipLaunchKernelGGL(k_mask_count<double>, g, dim3(kScanBlock), 0, st, b, packed_is_double);
  else
    hipLaunchKernelGGL(k_mask_count<float>, g, dim3(kScanBlock), 0, st, b, packed_is_double);
  hipLaunchKernelGGL(k_scan, dim3((1) * b.n), dim3(1024), 0, st, b);
  hipLaunchKernelGGL(k_compact, g, dim3(kScanBlock), 0, st, b);
  return hipGetLastError();
}

// ---------------------------------------------------------------- gather
__global__ void __launch_bounds__(256) k_gather(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int na = (int)*s.n_active;
  for (int k = MRA_BX(b) * blockDim.x + threadIdx.x; k < na; k += MRA_GX(b) * blockDim.x)
    s.omega[k] = s.dense64[s.index_fine[k]];
}

hipError_t launch_gather(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3((scatter_blocks(c.J)) * b.n), dim3(256), 0, st, b);
  return hipGetLastError();
}

// rank map and tile flags from a caller-given index list
__global__ void __launch_bounds__(256) k_rank_clear(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int Nf = s.N * s.N;
  for (int f = MRA_BX(b) * blockDim.x + threadIdx.x; f < Nf; f += MRA_GX(b) * blockDim.x) s.rank[f] = -1;
  const int ntiles = s.ntx * s.ntx;
  for (int t = MRA_BX(b) * blockDim.x + threadIdx.x; t < ntiles; t += MRA_GX(b) * blockDim.x)
    s.tile_count[t] = 0;
}

__global__ void __launch_bounds__(256) k_rank_scatter(Batch b) {
  const SolveDev& s = MRA_SOLVE(b);
  const int na = (int)*s.n_active;
  const int J = s.J, N = s.N, T = s.tile, ntx = s.ntx;
  for (int k = MRA_BX(b) * blockDim.x + threadIdx.x; k < na; k += MRA_GX(b) * blockDim.x) {
    const int f = s.index_fine[k];
    s.rank[f] = k;
    atomicAdd(&s.tile_count[((f >> J) / T) * ntx + (f & (N - 1)) / T], 1);
  }
}

hipError_t launch_rank_from_index(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  dim3 g((scatter_blocks(c.J)) * b.n);
  hipLaunchKernelGGL(k_rank_clear, g, dim3(256), 0, st, b);
  hipLaunchKernelGGL(k_rank_scatter, g, dim3(256), 0, st, b);
  return hipGetLastError();
}

}  // namespace mra
