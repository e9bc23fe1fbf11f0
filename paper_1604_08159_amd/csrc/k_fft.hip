// Streamfunction Poisson solve on the periodic grid: psi_hat = -omega_hat /
// lambda(k) with lambda the exact symbol of the discrete Laplacian
// L = D2_x + D2_y ((2p+1)-point Lagrange second differences), the k = 0 mode
// set to zero.  The paper states only that the streamfunction satisfies a
// Poisson equation (Section 4); the FFT inverse of the discrete L is the
// solver chosen here.
//
// Three passes over HBM, each a batch of 1-D FFTs staged in LDS:
//   A  rows: real-to-complex FFT of length N (complex FFT of length N/2 on
//      the packed even/odd samples), written transposed as spec[kx][y];
//   B  columns (contiguous rows of spec): forward FFT (decimation in
//      frequency, natural -> bit-reversed), multiply by -1/lambda / N^2 in
//      bit-reversed order, inverse FFT (decimation in time,
//      bit-reversed -> natural);
//   C  rows: complex-to-real inverse, read transposed.
// Twiddles come from one table of exp(-2 pi i k / 2048) set up once.
#include "mra_internal.hpp"

namespace mra {

__device__ double2 g_tw64[kTwN];
__device__ float2 g_tw32[kTwN];

__global__ void k_init_tw() {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < kTwN; k += gridDim.x * blockDim.x) {
    double sn, cs;
    sincospi(-(double)k / (kTwN / 2), &sn, &cs);
    g_tw64[k] = make_double2(cs, sn);
    g_tw32[k] = make_float2((float)cs, (float)sn);
  }
}

hipError_t fft_init_tables(hipStream_t st) {
  hipLaunchKernelGGL(k_init_tw, dim3(8), dim3(256), 0, st);
  return hipGetLastError();
}

template <typename T> struct C2;
template <> struct C2<double> {
  using t = double2;
  __device__ static t tw(int k) { return g_tw64[k]; }
};
template <> struct C2<float> {
  using t = float2;
  __device__ static t tw(int k) { return g_tw32[k]; }
};

template <typename V> __device__ inline V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ inline V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ inline V cmul(V a, V b) { return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <typename V> __device__ inline V cmulc(V a, V b) {   // a * conj(b)
  return V{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename V> __device__ inline V cconj(V a) { return V{a.x, -a.y}; }

__device__ inline int brev(int k, int bits) { return (int)(__brev((unsigned)k) >> (32 - bits)); }

// nvec vectors of length M = 2^lm in LDS (stride M).
// forward, decimation in frequency: natural in, bit-reversed out.
template <typename T>
__device__ void fft_dif(typename C2<T>::t* buf, int nvec, int lm) {
  using V = typename C2<T>::t;
  const int M = 1 << lm, half = M >> 1;
  const int nb = nvec * half;
  for (int lh = lm - 1; lh >= 0; --lh) {
    const int hs = 1 << lh;
    const int tws = kTwN >> (lh + 1);
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
      const int v = q >> (lm - 1), r = q & (half - 1);
      const int pos = r & (hs - 1);
      const int i0 = v * M + ((r >> lh) << (lh + 1)) + pos;
      const V a = buf[i0], b = buf[i0 + hs];
      buf[i0] = cadd(a, b);
      buf[i0 + hs] = cmul(csub(a, b), C2<T>::tw(pos * tws));
    }
    __syncthreads();
  }
}

// inverse (conjugate twiddles), decimation in time: bit-reversed in, natural
// out, unnormalised.
template <typename T>
__device__ void ifft_dit(typename C2<T>::t* buf, int nvec, int lm) {
  using V = typename C2<T>::t;
  const int M = 1 << lm, half = M >> 1;
  const int nb = nvec * half;
  for (int lh = 0; lh < lm; ++lh) {
    const int hs = 1 << lh;
    const int tws = kTwN >> (lh + 1);
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
      const int v = q >> (lm - 1), r = q & (half - 1);
      const int pos = r & (hs - 1);
      const int i0 = v * M + ((r >> lh) << (lh + 1)) + pos;
      const V a = buf[i0];
      const V b = cmulc(buf[i0 + hs], C2<T>::tw(pos * tws));
      buf[i0] = cadd(a, b);
      buf[i0 + hs] = csub(a, b);
    }
    __syncthreads();
  }
}

template <typename T>
__device__ inline const T* poisson_src(const SolveDev& s, int src) {
  if (src == 0) return reinterpret_cast<const T*>(s.wt);
  if (src == 1) return reinterpret_cast<const T*>(s.vt);
  return reinterpret_cast<const T*>(s.dense64);
}
template <typename T>
__device__ inline T* poisson_dst(const SolveDev& s, int src) {
  return reinterpret_cast<T*>(src == 1 ? s.psiv : s.psi);
}

// pass A: rows -> spec[kx][y], R rows per block
template <typename T>
__global__ void __launch_bounds__(256) k_fft_rows_fwd(Batch b, int src, int R) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem[];
  V* buf = reinterpret_cast<V*>(smem);
  const SolveDev& s = *b.s[blockIdx.y];
  const int J = s.J, N = s.N, M = N >> 1, lm = J - 1;
  const int y0 = blockIdx.x * R;
  const V* in = reinterpret_cast<const V*>(poisson_src<T>(s, src));
  for (int q = threadIdx.x; q < R * M; q += blockDim.x) {
    const int r = q / M, n = q - r * M;
    buf[q] = in[(size_t)(y0 + r) * M + n];
  }
  __syncthreads();
  fft_dif<T>(buf, R, lm);
  V* spec = reinterpret_cast<V*>(s.spec);
  const int twN = kTwN / N;
  for (int q = threadIdx.x; q < (M + 1) * R; q += blockDim.x) {
    const int k = q / R, r = q - k * R;
    const V* row = buf + r * M;
    const V zk = row[brev(k & (M - 1), lm)];
    const V zc = cconj(row[brev((M - k) & (M - 1), lm)]);
    const V e = cmul(csub(zk, zc), C2<T>::tw(k * twN));
    V x;
    x.x = T(0.5) * (zk.x + zc.x + e.y);
    x.y = T(0.5) * (zk.y + zc.y - e.x);
    spec[(size_t)k * N + y0 + r] = x;
  }
}

// sigma_2(theta_k) = c0 + 2 sum_n c_n cos(2 pi n k / N), FP64
template <int P>
__device__ inline double d2_sigma(int k, int N) {
  const int tws = kTwN / N;
  if constexpr (P == 2) {
    return -2.5 + 2.0 * ((4.0 / 3.0) * g_tw64[((k) & (N - 1)) * tws].x +
                         (-1.0 / 12.0) * g_tw64[((2 * k) & (N - 1)) * tws].x);
  } else {
    return -49.0 / 18.0 + 2.0 * (1.5 * g_tw64[((k) & (N - 1)) * tws].x +
                                 (-0.15) * g_tw64[((2 * k) & (N - 1)) * tws].x +
                                 (1.0 / 90.0) * g_tw64[((3 * k) & (N - 1)) * tws].x);
  }
}

// pass B: C spectrum rows (fixed kx) per block
template <int P, typename T>
__global__ void __launch_bounds__(256) k_fft_cols(Batch b, int C) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem[];
  V* buf = reinterpret_cast<V*>(smem);
  const SolveDev& s = *b.s[blockIdx.y];
  const int J = s.J, N = s.N, M = N >> 1;
  const int k0 = blockIdx.x * C;
  const int nr = (M + 1 - k0) < C ? (M + 1 - k0) : C;
  V* spec = reinterpret_cast<V*>(s.spec);
  for (int q = threadIdx.x; q < nr * N; q += blockDim.x) buf[q] = spec[(size_t)k0 * N + q];
  __syncthreads();
  fft_dif<T>(buf, nr, J);
  const double h2n = s.h * s.h / ((double)N * (double)N);
  for (int q = threadIdx.x; q < nr * N; q += blockDim.x) {
    const int r = q >> J, j = q & (N - 1);
    const int kx = k0 + r, ky = brev(j, J);
    const double den = d2_sigma<P>(kx, N) + d2_sigma<P>(ky, N);
    const T g = (kx == 0 && ky == 0) ? T(0) : (T)(-h2n / den);
    buf[q].x *= g;
    buf[q].y *= g;
  }
  __syncthreads();
  ifft_dit<T>(buf, nr, J);
  for (int q = threadIdx.x; q < nr * N; q += blockDim.x) spec[(size_t)k0 * N + q] = buf[q];
}

// pass C: spec[kx][y] -> real rows
template <typename T>
__global__ void __launch_bounds__(256) k_fft_rows_inv(Batch b, int src, int R) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem[];
  V* buf = reinterpret_cast<V*>(smem);
  const SolveDev& s = *b.s[blockIdx.y];
  const int J = s.J, N = s.N, M = N >> 1, lm = J - 1;
  const int y0 = blockIdx.x * R;
  const V* spec = reinterpret_cast<const V*>(s.spec);
  const int twN = kTwN / N;
  for (int q = threadIdx.x; q < M * R; q += blockDim.x) {
    const int k = q / R, r = q - k * R;
    const V xk = spec[(size_t)k * N + y0 + r];
    const V xc = cconj(spec[(size_t)(M - k) * N + y0 + r]);
    const V e = cmulc(csub(xk, xc), C2<T>::tw(k * twN));
    V z;
    z.x = xk.x + xc.x - e.y;
    z.y = xk.y + xc.y + e.x;
    buf[r * M + brev(k, lm)] = z;
  }
  __syncthreads();
  ifft_dit<T>(buf, R, lm);
  V* out = reinterpret_cast<V*>(poisson_dst<T>(s, src));
  for (int q = threadIdx.x; q < R * M; q += blockDim.x) {
    const int r = q / M, n = q - r * M;
    out[(size_t)(y0 + r) * M + n] = buf[q];
  }
}

static int rows_per_block(int N, size_t elem) {
  const size_t budget = 64 * 1024;
  size_t per = (size_t)(N / 2) * elem;
  int r = (int)(budget / per);
  if (r > 32) r = 32;
  if (r > N) r = N;
  if (r < 1) r = 1;
  int p2 = 1;
  while (p2 * 2 <= r) p2 *= 2;
  return p2;
}
static int cols_per_block(int N, size_t elem) {
  const size_t budget = 64 * 1024;
  int c = (int)(budget / ((size_t)N * elem));
  if (c > 16) c = 16;
  if (c < 1) c = 1;
  return c;
}

template <typename T>
static hipError_t poisson_t(const Batch& b, const LaunchCfg& c, int src, int pass, hipStream_t st) {
  using V = typename C2<T>::t;
  const int N = 1 << c.J, M = N / 2;
  const int R = rows_per_block(N, sizeof(V));
  const int C = cols_per_block(N, sizeof(V));
  if (pass < 0 || pass == 0)
    hipLaunchKernelGGL(k_fft_rows_fwd<T>, dim3(N / R, b.n), dim3(256), (size_t)R * M * sizeof(V), st, b, src, R);
  if (pass < 0 || pass == 1) {
    dim3 g((M + 1 + C - 1) / C, b.n);
    if (c.p == 2) hipLaunchKernelGGL((k_fft_cols<2, T>), g, dim3(256), (size_t)C * N * sizeof(V), st, b, C);
    else hipLaunchKernelGGL((k_fft_cols<3, T>), g, dim3(256), (size_t)C * N * sizeof(V), st, b, C);
  }
  if (pass < 0 || pass == 2)
    hipLaunchKernelGGL(k_fft_rows_inv<T>, dim3(N / R, b.n), dim3(256), (size_t)R * M * sizeof(V), st, b, src, R);
  return hipGetLastError();
}

hipError_t launch_poisson(const Batch& b, const LaunchCfg& c, int src, hipStream_t st) {
  if (src == 2 || c.prec == 0) return poisson_t<double>(b, c, src, -1, st);
  return poisson_t<float>(b, c, src, -1, st);
}

hipError_t launch_poisson_pass(const Batch& b, const LaunchCfg& c, int src, int pass, hipStream_t st) {
  if (src == 2 || c.prec == 0) return poisson_t<double>(b, c, src, pass, st);
  return poisson_t<float>(b, c, src, pass, st);
}

}  // namespace mra
