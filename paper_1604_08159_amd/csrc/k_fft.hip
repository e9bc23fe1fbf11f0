// Velocity from vorticity on the periodic grid: psi_hat = -omega_hat /
// lambda(k), lambda the exact symbol of the discrete Laplacian L = D2_x + D2_y
// ((2p+1)-point Lagrange second differences), the k = 0 mode set to zero; then
// u = D1_y psi and v = -D1_x psi with the collocation first derivative of
// Section 2.5.  D1 and L are circulant on the periodic grid, so both are
// diagonal in Fourier space: u_hat = i s1(ky) psi_hat, v_hat = -i s1(kx)
// psi_hat with s1(theta) = (2/h) sum_n a_n sin(n theta).  Applying them as
// multipliers gives the same discrete operator as differencing psi, with the
// rounding of the transforms relative to |u| instead of amplified by 1/h.
// The paper states only that the streamfunction satisfies a Poisson equation
// (Section 4); the FFT inverse of the discrete L is the solver chosen here.
//
// Three passes over HBM, each a batch of 1-D FFTs staged in LDS:
//   A  rows: real-to-complex FFT of length N (complex FFT of length N/2 on
//      the packed even/odd samples), written transposed as spec[kx][y];
//   B  columns (contiguous rows of spec): forward FFT, multiply by
//      -1/lambda / N^2, form the u and v spectra, two inverse FFTs;
//   C  rows: complex-to-real inverse of both, read transposed.
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

// ------------------------------------------------------------ FFT core
// Stockham autosort FFT (natural order in and out) of nfft vectors of length
// L = 2^lg held in LDS at stride L, by a block of 256 threads.  Passes of
// radix 8 (the last one of radix 2, 4 or 8 to complete L): every thread keeps
// 8 complex values in registers per pass, so a pass is one LDS read phase,
// one barrier, the small DFTs and twiddles in registers, one LDS write phase.
// The block handles nfft * L <= 2048 points.  S = -1 forward, +1 inverse
// (unnormalised).
constexpr int kFftThreads = 256;
constexpr int kFftPoints = 2048;

template <int S, typename V> __device__ inline V mul_i(V a) {   // (S i) * a
  return S < 0 ? V{a.y, -a.x} : V{-a.y, a.x};
}

template <int R, int S, typename T>
__device__ inline void small_dft(typename C2<T>::t* v) {
  using V = typename C2<T>::t;
  if constexpr (R == 2) {
    const V a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const V t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const V t2 = cadd(v[1], v[3]), t3 = mul_i<S>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  } else {
    V e[4] = {v[0], v[2], v[4], v[6]};
    V o[4] = {v[1], v[3], v[5], v[7]};
    small_dft<4, S, T>(e);
    small_dft<4, S, T>(o);
    const T c = T(0.70710678118654752440);
    const V w1 = V{c * (o[1].x - S * o[1].y), c * (o[1].y + S * o[1].x)};   // e^{S i pi/4} o1
    const V w2 = mul_i<S>(o[2]);
    const V w3 = V{c * (-o[3].x - S * o[3].y), c * (-o[3].y + S * o[3].x)}; // e^{S 3i pi/4} o3
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], w1);
    v[5] = csub(e[1], w1);
    v[2] = cadd(e[2], w2);
    v[6] = csub(e[2], w2);
    v[3] = cadd(e[3], w3);
    v[7] = csub(e[3], w3);
  }
}

template <int R, int S, typename T>
__device__ inline void stockham_pass(typename C2<T>::t* buf, int L, int nfft, int Ns) {
  using V = typename C2<T>::t;
  constexpr int IPT = 8 / R;               // work items per thread
  const int per = L / R;
  const int total = nfft * per;
  const int twstep = kTwN / (Ns * R);
  V v[IPT][R];
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const int q = threadIdx.x + it * kFftThreads;
    if (q < total) {
      const int f = q / per, j = q - f * per;
      const int k = j & (Ns - 1);
      const V* src = buf + f * L + j;
      v[it][0] = src[0];
      // twiddles w^r, w = exp(-2 pi i k / (Ns R)): one table load, then powers
      const V w1 = C2<T>::tw(k * twstep);
      V wr = w1;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const V x = src[r * per];
        v[it][r] = S < 0 ? cmul(x, wr) : cmulc(x, wr);
        wr = cmul(wr, w1);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const int q = threadIdx.x + it * kFftThreads;
    if (q < total) {
      const int f = q / per, j = q - f * per;
      const int k = j & (Ns - 1);
      small_dft<R, S, T>(v[it]);
      V* dst = buf + f * L + (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ns] = v[it][r];
    }
  }
  __syncthreads();
}

template <int S, typename T>
__device__ void fft_block(typename C2<T>::t* buf, int L, int nfft) {
  for (int Ns = 1; Ns < L;) {
    const int rem = L / Ns;
    if (rem >= 8) { stockham_pass<8, S, T>(buf, L, nfft, Ns); Ns *= 8; }
    else if (rem == 4) { stockham_pass<4, S, T>(buf, L, nfft, Ns); Ns *= 4; }
    else { stockham_pass<2, S, T>(buf, L, nfft, Ns); Ns *= 2; }
  }
}

template <typename T>
__device__ inline const T* poisson_src(const SolveDev& s, int src) {
  if (src == 0) return reinterpret_cast<const T*>(s.wt);
  if (src == 1) return reinterpret_cast<const T*>(s.vt);
  return reinterpret_cast<const T*>(s.dense64);
}
// velocity outputs: src 0 -> (u, v), src 1 -> (u_v, v_v), src 2 -> FP64 pair
template <typename T>
__device__ inline T* poisson_dst(const SolveDev& s, int src, int comp) {
  if (src == 0) return reinterpret_cast<T*>(comp == 0 ? s.u : s.v);
  if (src == 1) return reinterpret_cast<T*>(comp == 0 ? s.uv : s.vv);
  return reinterpret_cast<T*>(s.vel64 + (size_t)comp * s.N * s.N);
}

// pass A: rows -> spec[kx][y], R rows per block (R * N/2 <= 2048)
template <typename T>
__global__ void __launch_bounds__(kFftThreads) k_fft_rows_fwd(Batch b, int src, int R) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem[];
  V* buf = reinterpret_cast<V*>(smem);
  const SolveDev& s = MRA_SOLVE(b);
  const int N = s.N, M = N >> 1;
  const int y0 = MRA_BX(b) * R;
  const V* in = reinterpret_cast<const V*>(poisson_src<T>(s, src));
  for (int q = threadIdx.x; q < R * M; q += blockDim.x) buf[q] = in[(size_t)y0 * M + q];
  __syncthreads();
  fft_block<-1, T>(buf, M, R);
  V* spec = reinterpret_cast<V*>(s.spec);
  const int twN = kTwN / N;
  for (int q = threadIdx.x; q < (M + 1) * R; q += blockDim.x) {
    const int k = q / R, r = q - k * R;
    const V* row = buf + r * M;
    const V zk = row[k & (M - 1)];
    const V zc = cconj(row[(M - k) & (M - 1)]);
    const V e = cmul(csub(zk, zc), C2<T>::tw(k * twN));
    V x;
    x.x = T(0.5) * (zk.x + zc.x + e.y);
    x.y = T(0.5) * (zk.y + zc.y - e.x);
    spec[(size_t)k * N + y0 + r] = x;
  }
}

// Symbols at theta = 2 pi k / N, FP64: sigma_2 = c0 + 2 sum_n c_n cos(n theta)
// (h^2 times the eigenvalue of D2) and sigma_1 = 2 sum_n a_n sin(n theta)
// (h / i times the eigenvalue of D1).  Table entry m: exp(-2 pi i m / 2048).
template <int P>
__device__ inline void symbols(int k, int N, double* s1, double* s2) {
  const int tws = kTwN / N;
  double c[4], sn[5];
#pragma unroll
  for (int n = 1; n <= 2 * P - 2; ++n) {
    const double2 t = g_tw64[((n * k) & (N - 1)) * tws];
    if (n <= P) c[n] = t.x;
    sn[n] = -t.y;
  }
  if constexpr (P == 2) {
    *s2 = -2.5 + 2.0 * ((4.0 / 3.0) * c[1] + (-1.0 / 12.0) * c[2]);
    *s1 = 2.0 * ((2.0 / 3.0) * sn[1] + (-1.0 / 12.0) * sn[2]);
  } else {
    *s2 = -49.0 / 18.0 + 2.0 * (1.5 * c[1] + (-0.15) * c[2] + (1.0 / 90.0) * c[3]);
    *s1 = 2.0 * ((272.0 / 365.0) * sn[1] + (-53.0 / 365.0) * sn[2] + (16.0 / 1095.0) * sn[3] +
                 (1.0 / 2920.0) * sn[4]);
  }
}

// pass B: C spectrum rows (fixed kx) per block (C * N <= 2048).  LDS: A holds
// psi_hat, B the u (then the v) spectrum; 2 * 2048 complex values at most.
template <int P, typename T>
__global__ void __launch_bounds__(kFftThreads) k_fft_cols(Batch b, int C) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem[];
  V* A = reinterpret_cast<V*>(smem);
  V* Bv = A + C * (1 << MRA_SOLVE(b).J);
  const SolveDev& s = MRA_SOLVE(b);
  const int J = s.J, N = s.N, M = N >> 1;
  const int k0 = MRA_BX(b) * C;
  const int nr = (M + 1 - k0) < C ? (M + 1 - k0) : C;
  V* specU = reinterpret_cast<V*>(s.spec);
  V* specV = reinterpret_cast<V*>(s.spec2);
  for (int q = threadIdx.x; q < nr * N; q += blockDim.x) A[q] = specU[(size_t)k0 * N + q];
  __syncthreads();
  fft_block<-1, T>(A, N, nr);
  const double h2n = s.h * s.h / ((double)N * (double)N);
  const double ih = 1.0 / s.h;
  for (int q = threadIdx.x; q < nr * N; q += blockDim.x) {
    const int r = q >> J, ky = q & (N - 1);
    const int kx = k0 + r;
    double s1x, s2x, s1y, s2y;
    symbols<P>(kx, N, &s1x, &s2x);
    symbols<P>(ky, N, &s1y, &s2y);
    const T g = (kx == 0 && ky == 0) ? T(0) : (T)(-h2n / (s2x + s2y));
    const V z = A[q];
    const T sy = (T)(s1y * ih);
    A[q] = V{z.x * g, z.y * g};
    Bv[q] = V{-sy * (z.y * g), sy * (z.x * g)};          // i s1(ky) psi_hat
  }
  __syncthreads();
  fft_block<1, T>(Bv, N, nr);
  for (int q = threadIdx.x; q < nr * N; q += blockDim.x) specU[(size_t)k0 * N + q] = Bv[q];
  __syncthreads();
  for (int q = threadIdx.x; q < nr * N; q += blockDim.x) {
    const int r = q >> J;
    double s1x, s2x;
    symbols<P>(k0 + r, N, &s1x, &s2x);
    const T sx = (T)(s1x * ih);
    const V z = A[q];
    Bv[q] = V{sx * z.y, -sx * z.x};                       // -i s1(kx) psi_hat
  }
  __syncthreads();
  fft_block<1, T>(Bv, N, nr);
  for (int q = threadIdx.x; q < nr * N; q += blockDim.x) specV[(size_t)k0 * N + q] = Bv[q];
}

// pass C: spec[kx][y] -> real rows, R rows per block (R * N/2 <= 2048), for
// the u spectrum and then the v spectrum.
template <typename T>
__global__ void __launch_bounds__(kFftThreads) k_fft_rows_inv(Batch b, int src, int R) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem[];
  V* buf = reinterpret_cast<V*>(smem);
  const SolveDev& s = MRA_SOLVE(b);
  const int N = s.N, M = N >> 1;
  const int y0 = MRA_BX(b) * R;
  const int twN = kTwN / N;
  for (int comp = 0; comp < 2; ++comp) {
    const V* spec = reinterpret_cast<const V*>(comp == 0 ? s.spec : s.spec2);
    for (int q = threadIdx.x; q < M * R; q += blockDim.x) {
      const int k = q / R, r = q - k * R;
      const V xk = spec[(size_t)k * N + y0 + r];
      const V xc = cconj(spec[(size_t)(M - k) * N + y0 + r]);
      const V e = cmulc(csub(xk, xc), C2<T>::tw(k * twN));
      V z;
      z.x = xk.x + xc.x - e.y;
      z.y = xk.y + xc.y + e.x;
      buf[r * M + k] = z;
    }
    __syncthreads();
    fft_block<1, T>(buf, M, R);
    V* out = reinterpret_cast<V*>(poisson_dst<T>(s, src, comp));
    for (int q = threadIdx.x; q < R * M; q += blockDim.x) out[(size_t)y0 * M + q] = buf[q];
    __syncthreads();
  }
}

static int rows_per_block(int N) {
  int r = kFftPoints / (N / 2);
  return r < N ? r : N;
}
static int cols_per_block(int N) {
  int c = kFftPoints / N;
  return c < N / 2 + 1 ? c : N / 2 + 1;
}

template <typename T>
static hipError_t poisson_t(const Batch& b, const LaunchCfg& c, int src, int pass, hipStream_t st) {
  using V = typename C2<T>::t;
  const int N = 1 << c.J, M = N / 2;
  const int R = rows_per_block(N);
  const int C = cols_per_block(N);
  if (pass < 0 || pass == 0)
    hipLaunchKernelGGL(k_fft_rows_fwd<T>, dim3((N / R) * b.n), dim3(kFftThreads), (size_t)R * M * sizeof(V), st, b,
                       src, R);
  if (pass < 0 || pass == 1) {
    dim3 g(((M + 1 + C - 1) / C) * b.n);
    const size_t lds = 2 * (size_t)C * N * sizeof(V);
    if (c.p == 2) hipLaunchKernelGGL((k_fft_cols<2, T>), g, dim3(kFftThreads), lds, st, b, C);
    else hipLaunchKernelGGL((k_fft_cols<3, T>), g, dim3(kFftThreads), lds, st, b, C);
  }
  if (pass < 0 || pass == 2)
    hipLaunchKernelGGL(k_fft_rows_inv<T>, dim3((N / R) * b.n), dim3(kFftThreads), (size_t)R * M * sizeof(V), st, b,
                       src, R);
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
