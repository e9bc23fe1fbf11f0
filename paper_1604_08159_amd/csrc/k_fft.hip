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

// Operator symbols at theta = 2 pi k / N for every N = 2^J <= 2048, entry
// N + k (k < N), rows [p - 2][kind]:
//   kind 0: sigma_1 = 2 sum_n a_n sin(n theta)    (h / i times the eigenvalue of D1)
//   kind 1: sigma_2 = c0 + 2 sum_n c_n cos(n theta)  (h^2 times the eigenvalue of D2)
// with the D1 filter a_n and the Lagrange D2 weights c_n of the stencils.
constexpr int kSymN = 2 * kTwN;
__device__ double g_sym64[2][2][kSymN];
__device__ float g_sym32[2][2][kSymN];

__global__ void k_init_tw() {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < kTwN; k += gridDim.x * blockDim.x) {
    double sn, cs;
    sincospi(-(double)k / (kTwN / 2), &sn, &cs);
    g_tw64[k] = make_double2(cs, sn);
    g_tw32[k] = make_float2((float)cs, (float)sn);
  }
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < kSymN; e += gridDim.x * blockDim.x) {
    if (e < 2) continue;
    const int N = 1 << ilog2((unsigned)e), k = e - N;
    double c[5], sn[5];
    for (int n = 1; n <= 4; ++n) sincospi(2.0 * (double)((n * k) & (N - 1)) / N, &sn[n], &c[n]);
    const double s2a = -2.5 + 2.0 * ((4.0 / 3.0) * c[1] + (-1.0 / 12.0) * c[2]);
    const double s1a = 2.0 * ((2.0 / 3.0) * sn[1] + (-1.0 / 12.0) * sn[2]);
    const double s2b = -49.0 / 18.0 + 2.0 * (1.5 * c[1] + (-0.15) * c[2] + (1.0 / 90.0) * c[3]);
    const double s1b = 2.0 * ((272.0 / 365.0) * sn[1] + (-53.0 / 365.0) * sn[2] + (16.0 / 1095.0) * sn[3] +
                              (1.0 / 2920.0) * sn[4]);
    g_sym64[0][0][e] = s1a; g_sym64[0][1][e] = s2a;
    g_sym64[1][0][e] = s1b; g_sym64[1][1][e] = s2b;
    g_sym32[0][0][e] = (float)s1a; g_sym32[0][1][e] = (float)s2a;
    g_sym32[1][0][e] = (float)s1b; g_sym32[1][1][e] = (float)s2b;
  }
}

hipError_t fft_init_tables(hipStream_t st) {
  hipLaunchKernelGGL(k_init_tw, dim3(16), dim3(256), 0, st);
  return hipGetLastError();
}

template <typename T> struct C2;
template <> struct C2<double> {
  using t = double2;
  __device__ static t tw(int k) { return g_tw64[k]; }
  __device__ static double sym(int p, int kind, int e) { return g_sym64[p - 2][kind][e]; }
};
template <> struct C2<float> {
  using t = float2;
  __device__ static t tw(int k) { return g_tw32[k]; }
  __device__ static float sym(int p, int kind, int e) { return g_sym32[p - 2][kind][e]; }
};

// LDS slot of FFT element i: one pad slot per 32 elements spreads the
// strided writes of the early Stockham passes over the banks.
__device__ inline int lx(int i) { return i + (i >> 5); }
__host__ __device__ inline int lds_slots(int n) { return n + (n >> 5); }

// Global loads and stores of complex values through plain 2-vectors (the
// HIP vector types do not bind to address-space-qualified references).
template <typename V> struct Raw2;
template <> struct Raw2<float2> { typedef float t __attribute__((ext_vector_type(2))); };
template <> struct Raw2<double2> { typedef double t __attribute__((ext_vector_type(2))); };
template <typename V> __device__ inline V gload(const V* p, size_t i) {
  const auto r = glb(reinterpret_cast<const typename Raw2<V>::t*>(p))[i];
  return V{r.x, r.y};
}
template <typename V> __device__ inline void gstore(V* p, size_t i, V v) {
  typename Raw2<V>::t r;
  r.x = v.x;
  r.y = v.y;
  glb(reinterpret_cast<typename Raw2<V>::t*>(p))[i] = r;
}

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
// a barrier, the small DFTs and twiddles in registers, one LDS write phase.
// The block handles nfft * L <= 2048 points.  S = -1 forward, +1 inverse
// (unnormalised).
//
// Work items are dealt so that wavefront w handles exactly the elements
// [512 w, 512 (w + 1)) in every pass.  For L <= 512 each vector then lives in
// one wavefront, whose lanes exchange data through LDS with only a wavefront
// barrier: the four wavefronts of a block run their passes independently.
// Larger L takes block barriers.  The elementwise phases around the FFTs use
// the same ownership, so they need no block barrier either when L <= 512.
constexpr int kFftThreads = 256;
constexpr int kFftPoints = 2048;
constexpr int kWaveSpan = 512;             // elements owned by one wavefront

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ inline void fft_sync(bool wave_local) {
  if (wave_local) wave_sync();
  else __syncthreads();
}
// first element owned by this thread's wavefront, and its lane
__device__ inline int own0() { return (threadIdx.x >> 6) * kWaveSpan; }
__device__ inline int lane() { return threadIdx.x & 63; }

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

// The twiddle w = exp(-2 pi i k / (Ns R)) of each item of each pass, loaded
// from the table when a block starts (beside its data loads) instead of at
// each pass, where it would add one dependent load to every pass.  The
// passes of both signs use the same entries (the inverse takes conj(w)).
template <typename T, int LGL, int LGNS> struct TwSet {
  static constexpr int REM = LGL - LGNS, LGR = REM >= 3 ? 3 : REM, IPT = 8 >> LGR;
  typename C2<T>::t w[IPT];
  TwSet<T, LGL, LGNS + LGR> next;
};
template <typename T, int LGL> struct TwSet<T, LGL, LGL> {};

template <typename T, int LGL, int NF, int LGNS, int NT = kFftThreads>
__device__ __forceinline__ void load_twiddles(TwSet<T, LGL, LGNS>& ts, int nfft) {
  if constexpr (LGNS < LGL) {
    using S_ = TwSet<T, LGL, LGNS>;
    constexpr int LGR = S_::LGR, IPT = S_::IPT, LGIPT = 3 - LGR;
    constexpr int LGPER = LGL - LGR, PER = 1 << LGPER, NS = 1 << LGNS;
    constexpr int TWSHIFT = 11 - LGNS - LGR;
    constexpr bool FULL = NF * PER == NT * IPT;
    if constexpr (LGNS > 0) {
      const int total = nfft << LGPER;
      const int qbase = ((threadIdx.x >> 6) << (6 + LGIPT)) + (threadIdx.x & 63);
#pragma unroll
      for (int it = 0; it < IPT; ++it) {
        const int q = qbase + (it << 6);
        if (FULL || q < total) ts.w[it] = C2<T>::tw(((q & (PER - 1)) & (NS - 1)) << TWSHIFT);
      }
    }
    load_twiddles<T, LGL, NF, LGNS + LGR, NT>(ts.next, nfft);
  }
}

// One radix-2^LGR pass over NF vectors of length 2^LGL (Ns = 2^LGNS), all
// sizes compile-time, so index arithmetic is shifts and immediate offsets.
template <int S, typename T, int LGL, int NF, int LGNS, int LGR, int NT = kFftThreads>
__device__ __forceinline__ void stockham_pass(typename C2<T>::t* buf, int nfft, const TwSet<T, LGL, LGNS>& ts) {
  using V = typename C2<T>::t;
  constexpr int R = 1 << LGR, IPT = 8 / R, LGIPT = 3 - LGR;
  constexpr int LGPER = LGL - LGR, PER = 1 << LGPER;      // items per vector
  constexpr int NS = 1 << LGNS;
  constexpr int TWSHIFT = 11 - LGNS - LGR;                // kTwN = 2^11
  constexpr bool WL = LGL <= 9;
  constexpr bool FULL = NF * PER == NT * IPT;             // every (thread, it) has an item
  static_assert(NF * (1 << LGL) <= 8 * NT, "FFT block size");
  const int total = nfft << LGPER;
  // item of (thread, it): wavefront w takes items [64 IPT w, 64 IPT (w + 1))
  const int qbase = ((threadIdx.x >> 6) << (6 + LGIPT)) + (threadIdx.x & 63);
  V v[IPT][R];
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const int q = qbase + (it << 6);
    if (FULL || q < total) {
      const int j = q & (PER - 1);
      const int base = ((q >> LGPER) << LGL) + j;
      if constexpr (LGNS == 0) {             // first pass: every twiddle is 1
#pragma unroll
        for (int r = 0; r < R; ++r) v[it][r] = buf[lx(base + r * PER)];
      } else {
        // twiddles w^r, w = exp(-2 pi i k / (Ns R)): one preloaded entry, then
        // powers.  The empty asm keeps the powers here: formed when the entry
        // arrives they would hold R - 1 more values per pass across the block
        V w1 = ts.w[it];
        asm volatile("" : "+v"(w1.x), "+v"(w1.y));
        v[it][0] = buf[lx(base)];
        V wr = w1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const V x = buf[lx(base + r * PER)];
          v[it][r] = S < 0 ? cmul(x, wr) : cmulc(x, wr);
          wr = cmul(wr, w1);
        }
      }
    }
  }
  fft_sync(WL);
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const int q = qbase + (it << 6);
    if (FULL || q < total) {
      const int j = q & (PER - 1);
      const int k = j & (NS - 1);
      small_dft<R, S, T>(v[it]);
      const int base = ((q >> LGPER) << LGL) + ((j - k) << LGR) + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lx(base + r * NS)] = v[it][r];
    }
  }
  fft_sync(WL);
}

template <int S, typename T, int LGL, int NF, int LGNS, int NT = kFftThreads>
__device__ __forceinline__ void fft_passes(typename C2<T>::t* buf, int nfft, const TwSet<T, LGL, LGNS>& ts) {
  if constexpr (LGNS < LGL) {
    constexpr int REM = LGL - LGNS;
    constexpr int LGR = REM >= 3 ? 3 : REM;
    stockham_pass<S, T, LGL, NF, LGNS, LGR, NT>(buf, nfft, ts);
    fft_passes<S, T, LGL, NF, LGNS + LGR, NT>(buf, nfft, ts.next);
  }
}

// nfft <= NF vectors of length 2^LGL at stride 2^LGL; wavefront-local when
// L <= 512.  ts: the twiddles of (LGL, NF, NT, nfft) from load_twiddles.
template <int S, typename T, int LGL, int NF, int NT = kFftThreads>
__device__ __forceinline__ void fft_block(typename C2<T>::t* buf, int nfft, const TwSet<T, LGL, 0>& ts) {
  fft_passes<S, T, LGL, NF, 0, NT>(buf, nfft, ts);
}

template <typename T>
__device__ inline const T* poisson_src(const SolveDev& s, int src) {
  if (src == 0) return reinterpret_cast<const T*>(s.wt);
  if (src == 1) return reinterpret_cast<const T*>(s.vt);
  if (src == 3) return reinterpret_cast<const T*>(s.res64);
  return reinterpret_cast<const T*>(s.dense64);
}
// velocity outputs: src 0 -> (u, v), src 1 -> (u_v, v_v), or psi~ alone in u_v
// when only the stream function is formed, src 2 and 3 -> the FP64 pair
template <typename T>
__device__ inline T* poisson_dst(const SolveDev& s, int src, int comp) {
  if (src == 0) return reinterpret_cast<T*>(comp == 0 ? s.u : s.v);
  if (src == 1) return reinterpret_cast<T*>(comp == 0 ? s.uv : s.vv);
  return reinterpret_cast<T*>(s.vel64 + (size_t)comp * s.N * s.N);
}

// Launch geometry, compile-time per grid level J (N = 2^J, M = N/2):
// rows per row-pass block and spectrum rows per column-pass block.
// NT threads per row-pass block hold 8 NT points: the large grids take more
// threads so that a block holds several rows, and each spectrum access of the
// transposed layout covers R consecutive elements (at least 64 bytes).
template <int J, int NT = kFftThreads> struct FftGeo {
  static constexpr int N = 1 << J, M = N >> 1, LGM = J - 1;
  static constexpr int R = ((8 * NT) >> LGM) < N ? ((8 * NT) >> LGM) : N;
  static constexpr int C = (kFftPoints >> J) < M + 1 ? (kFftPoints >> J) : M + 1;
};
template <typename T, int J> constexpr int row_threads() {
  return J >= 10 ? (sizeof(T) == 4 ? 1024 : 512) : kFftThreads;
}

// pass A: rows -> spec[kx][y], R rows per block (R * N/2 <= 2048)
template <typename T, int J, int NT = row_threads<T, J>()>
__global__ void __launch_bounds__(NT) k_fft_rows_fwd(Batch b, int src) {
  using V = typename C2<T>::t;
  using G = FftGeo<J, NT>;
  constexpr int N = G::N, M = G::M, R = G::R;
  extern __shared__ unsigned char smem[];
  V* buf = reinterpret_cast<V*>(smem);
  const SolveDev& s = MRA_SOLVE(b);
  const int y0 = MRA_BX(b) * R;
  const V* in = reinterpret_cast<const V*>(poisson_src<T>(s, src));
  constexpr int n = R * M;
  constexpr int twN = kTwN / N;
  constexpr int PL = kWaveSpan / 64, PO = ((M + 1) * R + NT - 1) / NT;
  // the row data and the twiddles of every pass are all in flight before the
  // first is waited for
  const int e1 = min(own0() + kWaveSpan, n);
  V d[PL];
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int q = own0() + lane() + u * 64;
    if (q < e1) d[u] = gload(in, (size_t)y0 * M + q);
  }
  TwSet<T, G::LGM, 0> ts;
  load_twiddles<T, G::LGM, R, 0, NT>(ts, R);
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int q = own0() + lane() + u * 64;
    if (q < e1) buf[lx(q)] = d[u];
  }
  fft_sync(G::LGM <= 9);
  fft_block<-1, T, G::LGM, R, NT>(buf, R, ts);
  __syncthreads();
  V* spec = reinterpret_cast<V*>(s.spec);
  // the twiddles of the split into the real transform, loaded together
  V tk[PO];
#pragma unroll
  for (int u = 0; u < PO; ++u) {
    const int q = threadIdx.x + u * NT;
    if (q < (M + 1) * R) tk[u] = C2<T>::tw((q / R) * twN);
  }
#pragma unroll
  for (int u = 0; u < PO; ++u) {
    const int q = threadIdx.x + u * NT;
    if (q >= (M + 1) * R) break;
    const int k = q / R, r = q % R;
    const V zk = buf[lx(r * M + (k & (M - 1)))];
    const V zc = cconj(buf[lx(r * M + ((M - k) & (M - 1)))]);
    const V e = cmul(csub(zk, zc), tk[u]);
    V x;
    x.x = T(0.5) * (zk.x + zc.x + e.y);
    x.y = T(0.5) * (zk.y + zc.y - e.x);
    gstore(spec, (size_t)k * N + y0 + r, x);
  }
}

// pass B: C spectrum rows (fixed kx) per block (C * N <= 2048).  LDS: A holds
// psi_hat, B the u (then the v) spectrum; 2 * 2048 complex values at most.
// PSI: only the stream function is wanted (the products of the frozen
// Jacobian take u = D1_y psi and v = -D1_x psi with the collocation stencil,
// which is the same circulant operator as the symbol): psi_hat goes back
// along y in place and B is not used.
template <int P, typename T, int J, bool PSI>
__global__ void __launch_bounds__(kFftThreads) k_fft_cols(Batch b) {
  using V = typename C2<T>::t;
  using G = FftGeo<J>;
  constexpr int N = G::N, M = G::M, C = G::C;
  extern __shared__ unsigned char smem[];
  const SolveDev& s = MRA_SOLVE(b);
  V* A = reinterpret_cast<V*>(smem);
  V* Bv = A + (PSI ? 0 : lds_slots(C * N));
  const int k0 = MRA_BX(b) * C;
  const int nr = (M + 1 - k0) < C ? (M + 1 - k0) : C;
  V* specU = reinterpret_cast<V*>(s.spec);
  V* specV = reinterpret_cast<V*>(s.spec2);
  constexpr bool wl = J <= 9;
  constexpr int PL = kWaveSpan / 64;
  const int e1 = min(own0() + kWaveSpan, nr * N);
  // the spectrum rows and the twiddles of every pass are all in flight before
  // the first is waited for
  V d[PL];
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int q = own0() + lane() + u * 64;
    if (q < e1) d[u] = gload(specU, (size_t)k0 * N + q);
  }
  TwSet<T, J, 0> ts;
  load_twiddles<T, J, C, 0>(ts, nr);
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int q = own0() + lane() + u * 64;
    if (q < e1) A[lx(q)] = d[u];
  }
  fft_sync(wl);
  fft_block<-1, T, J, C>(A, nr, ts);
  const T h2n = T(-s.h * s.h / ((double)N * (double)N));
  const T ih = T(1.0 / s.h);
  // the symbols of this thread's elements, loaded together
  T s1x[PL], s1y[PL], s0y[PL];
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int q = own0() + lane() + u * 64;
    if (q < e1) {
      s1x[u] = C2<T>::sym(P, 1, N + k0 + (q >> J));
      s1y[u] = C2<T>::sym(P, 1, N + (q & (N - 1)));
      if constexpr (!PSI) s0y[u] = C2<T>::sym(P, 0, N + (q & (N - 1)));
    }
  }
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int q = own0() + lane() + u * 64;
    if (q >= e1) break;
    const int r = q >> J, ky = q & (N - 1);
    const int kx = k0 + r;
    const T den = s1x[u] + s1y[u];
    const T g = (kx == 0 && ky == 0) ? T(0) : h2n / den;
    const V z = A[lx(q)];
    const V ps = V{z.x * g, z.y * g};
    A[lx(q)] = ps;
    if constexpr (!PSI) {
      const T sy = s0y[u] * ih;
      Bv[lx(q)] = V{-sy * ps.y, sy * ps.x};   // i s1(ky) psi_hat
    }
  }
  fft_sync(wl);
  if constexpr (PSI) {
    fft_block<1, T, J, C>(A, nr, ts);
    for (int q = own0() + lane(); q < e1; q += 64) specU[(size_t)k0 * N + q] = A[lx(q)];
    return;
  }
  fft_block<1, T, J, C>(Bv, nr, ts);
  for (int q = own0() + lane(); q < e1; q += 64) specU[(size_t)k0 * N + q] = Bv[lx(q)];
  fft_sync(wl);
  T s0x[PL];
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int q = own0() + lane() + u * 64;
    if (q < e1) s0x[u] = C2<T>::sym(P, 0, N + k0 + (q >> J));
  }
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int q = own0() + lane() + u * 64;
    if (q >= e1) break;
    const T sx = s0x[u] * ih;
    const V z = A[lx(q)];
    Bv[lx(q)] = V{sx * z.y, -sx * z.x};                    // -i s1(kx) psi_hat
  }
  fft_sync(wl);
  fft_block<1, T, J, C>(Bv, nr, ts);
  for (int q = own0() + lane(); q < e1; q += 64) specV[(size_t)k0 * N + q] = Bv[lx(q)];
}

// pass C: spec[kx][y] -> real rows, R rows per block (R * N/2 <= 2048), for
// the u spectrum and then the v spectrum (NC = 2), or for psi alone (NC = 1).
template <typename T, int J, int NC, int NT = row_threads<T, J>()>
__global__ void __launch_bounds__(NT) k_fft_rows_inv(Batch b, int src) {
  using V = typename C2<T>::t;
  using G = FftGeo<J, NT>;
  constexpr int N = G::N, M = G::M, R = G::R;
  extern __shared__ unsigned char smem[];
  V* buf = reinterpret_cast<V*>(smem);
  const SolveDev& s = MRA_SOLVE(b);
  // row blocks in XCD-aware order: the blocks that read the two 64-byte
  // halves of a 128-byte line of the transposed spectrum share an L2 (the
  // forward pass, which writes such halves, measured slower in this order)
  const int y0 = tile_of_block(MRA_BX(b), N / R, b.n) * R;
  constexpr int twN = kTwN / N;
  constexpr int NP = (M / 2 + 1) * R, PP = (NP + NT - 1) / NT;
  TwSet<T, G::LGM, 0> ts;
  load_twiddles<T, G::LGM, R, 0, NT>(ts, R);
  for (int comp = 0; comp < NC; ++comp) {
    const V* spec = reinterpret_cast<const V*>(comp == 0 ? s.spec : s.spec2);
    // z_k = X_k + conj X_{M-k} + i tw_k (X_k - conj X_{M-k}): the pair (k,
    // M - k) gives z_k and z_{M-k} from the same two loads, so every entry of
    // the spectrum is read once; all of this thread's pairs are loaded first
    V xa[PP], xb[PP], ta[PP], tb[PP];
#pragma unroll
    for (int u = 0; u < PP; ++u) {
      const int q = threadIdx.x + u * NT;
      if (q < NP) {
        const int k = q / R, r = q % R;
        xa[u] = gload(spec, (size_t)k * N + y0 + r);
        xb[u] = gload(spec, (size_t)(M - k) * N + y0 + r);
        ta[u] = C2<T>::tw(k * twN);
        tb[u] = C2<T>::tw(((M - k) & (M - 1)) * twN);
      }
    }
#pragma unroll
    for (int u = 0; u < PP; ++u) {
      const int q = threadIdx.x + u * NT;
      if (q >= NP) break;
      const int k = q / R, r = q % R;
      {
        const V xc = cconj(xb[u]);
        const V e = cmulc(csub(xa[u], xc), ta[u]);
        V z;
        z.x = xa[u].x + xc.x - e.y;
        z.y = xa[u].y + xc.y + e.x;
        buf[lx(r * M + k)] = z;
      }
      if (k > 0 && k < M / 2) {
        const V xc = cconj(xa[u]);
        const V e = cmulc(csub(xb[u], xc), tb[u]);
        V z;
        z.x = xb[u].x + xc.x - e.y;
        z.y = xb[u].y + xc.y + e.x;
        buf[lx(r * M + M - k)] = z;
      }
    }
    __syncthreads();
    fft_block<1, T, G::LGM, R, NT>(buf, R, ts);
    V* out = reinterpret_cast<V*>(poisson_dst<T>(s, src, comp));
    const int e1 = min(own0() + kWaveSpan, R * M);
    for (int q = own0() + lane(); q < e1; q += 64) gstore(out, (size_t)y0 * M + q, buf[lx(q)]);
    __syncthreads();
  }
}

template <typename T, int J, bool PSI>
static void poisson_jp(const Batch& b, int p, int src, int pass, hipStream_t st) {
  using V = typename C2<T>::t;
  using G = FftGeo<J>;
  constexpr int NT = row_threads<T, J>();
  using GR = FftGeo<J, NT>;
  if (pass < 0 || pass == 0)
    hipLaunchKernelGGL((k_fft_rows_fwd<T, J>), dim3((GR::N / GR::R) * b.n), dim3(NT),
                       lds_slots(GR::R * GR::M) * sizeof(V), st, b, src);
  if (pass < 0 || pass == 1) {
    dim3 g(((G::M + 1 + G::C - 1) / G::C) * b.n);
    const size_t lds = (PSI ? 1 : 2) * (size_t)lds_slots(G::C * G::N) * sizeof(V);
    if (p == 2) hipLaunchKernelGGL((k_fft_cols<2, T, J, PSI>), g, dim3(kFftThreads), lds, st, b);
    else hipLaunchKernelGGL((k_fft_cols<3, T, J, PSI>), g, dim3(kFftThreads), lds, st, b);
  }
  if (pass < 0 || pass == 2)
    hipLaunchKernelGGL((k_fft_rows_inv<T, J, PSI ? 1 : 2>), dim3((GR::N / GR::R) * b.n), dim3(NT),
                       lds_slots(GR::R * GR::M) * sizeof(V), st, b, src);
}

template <typename T, int J>
static void poisson_j(const Batch& b, int p, int src, bool psi, int pass, hipStream_t st) {
  if (psi) poisson_jp<T, J, true>(b, p, src, pass, st);
  else poisson_jp<T, J, false>(b, p, src, pass, st);
}

// The products of the frozen Jacobian (src 1, Jacobian 0) need the stream
// function only; every other source needs both velocity components.
template <typename T>
static hipError_t poisson_t(const Batch& b, const LaunchCfg& c, int src, int pass, hipStream_t st) {
  const bool psi = src == 1 && c.jac == 0;
  switch (c.J) {
    case 3: poisson_j<T, 3>(b, c.p, src, psi, pass, st); break;
    case 4: poisson_j<T, 4>(b, c.p, src, psi, pass, st); break;
    case 5: poisson_j<T, 5>(b, c.p, src, psi, pass, st); break;
    case 6: poisson_j<T, 6>(b, c.p, src, psi, pass, st); break;
    case 7: poisson_j<T, 7>(b, c.p, src, psi, pass, st); break;
    case 8: poisson_j<T, 8>(b, c.p, src, psi, pass, st); break;
    case 9: poisson_j<T, 9>(b, c.p, src, psi, pass, st); break;
    case 10: poisson_j<T, 10>(b, c.p, src, psi, pass, st); break;
    case 11: poisson_j<T, 11>(b, c.p, src, psi, pass, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_poisson(const Batch& b, const LaunchCfg& c, int src, hipStream_t st) {
  if (src >= 2 || c.prec == 0) return poisson_t<double>(b, c, src, -1, st);
  return poisson_t<float>(b, c, src, -1, st);
}

hipError_t launch_poisson_pass(const Batch& b, const LaunchCfg& c, int src, int pass, hipStream_t st) {
  if (src >= 2 || c.prec == 0) return poisson_t<double>(b, c, src, pass, st);
  return poisson_t<float>(b, c, src, pass, st);
}

}  // namespace mra
