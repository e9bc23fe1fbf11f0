// Internal declarations of the gfx950 wavelet-collocation library.
//
// Every kernel works on a batch of solves of equal (J, p, precision): each
// block works for one solve (see MRA_SOLVE) whose buffers are described by a
// SolveDev record that lives in device memory (in the solve's arena, or in the
// workspace of a stand-alone call).  Sizes that change on the device (the
// active count) are read from device memory, so launch shapes depend only on
// (J, p, m) and a captured step stays valid.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace mra {

constexpr int kMaxJ = 11;
constexpr int kMaxM = 47;           // Krylov dimension cap (augmented size <= 48)
constexpr int kMaxBatch = 64;       // solves per launch
constexpr int kTile = 32;           // stencil tile edge (clamped to N)
constexpr int kRedBlocks = 512;     // max chunks per solve of the Krylov reductions
constexpr int kScanItems = 4;       // packed entries per thread in compaction
constexpr int kScanBlock = 256;     // threads per compaction block
constexpr int kCoarseLevels = 6;    // levels <= this are prolonged by one block
constexpr int kTwN = 2048;          // twiddle table size (largest FFT length)

// Control words (int) and scalars (double) of a solve.
// C_OVER: the last regrid found more active nodes (C_NEED) than the solve's
// capacity; the solve is frozen until it is moved to a larger arena.
enum Ctrl : int { C_MEFF = 0, C_DONE = 1, C_STATUS = 2, C_CNT0 = 4, C_CNT1 = 5, C_CNT2 = 6,
                  C_CNT3 = 7, C_OVER = 8, C_NEED = 9, C_NCTRL = 16 };
constexpr int kStatusCapacity = 7;   // the status word's value for MRA_E_CAPACITY
// Elements between consecutive basis vectors beyond the capacity: vectors of
// a power-of-two length would all start on the same DRAM channel and bank,
// and the Gram-Schmidt reads up to m + 1 of them at the same offset at once.
// 4 KB of FP64 (a 2 x 2048^2 step: 23.14 -> 22.40 ms; 2 KB and 12 KB within
// 0.5% of it).
constexpr int kBasisPad = 512;
enum Scal : int { S_BETA = 0, S_INV = 1, S_UMAX = 3, S_T = 4, S_EVALS = 5, S_STEPS = 6,
                  S_THETA = 7, S_COND = 8, S_NSCAL = 16 };

struct SolveDev {
  // geometry / numbers
  int J, j0, p, N;
  int prec;                 // 0 -> double bulk fields, 1 -> float bulk fields
  int vb32;                 // 1 -> Krylov basis stored in FP32 (precision MRA_FP32)
  int m;                    // Krylov dimension
  int adjacent_zone;
  int smag_mode;
  int tile, ntx;            // stencil tile edge and tiles per side
  int cap;                  // capacity: length of the active-value arrays and basis vectors (<= Nf)
  int vs;                   // stride of the basis vectors (cap, padded: kBasisPad)
  double h, length, eps, dt;
  double nu0, cs, s0, mu;
  // active set
  uint8_t* mask;            // [Nf] packed
  int32_t* index_packed;    // [cap]
  int32_t* index_fine;      // [cap]
  int32_t* rank;            // [Nf] dense: active position or -1
  int32_t* tile_count;      // [ntiles] active nodes per stencil tile
  int64_t* n_active;        // device scalar
  int32_t* block_off;       // [nscan] compaction block counts -> offsets
  unsigned long long* umax; // bits of max|u| (non-negative doubles order as integers)
  // Krylov (FP64 arithmetic)
  double* omega;            // [cap] active values
  double* V;                // [(m+1)][vs] basis in FP64 (null when stored in FP32)
  float* V32;               // [(m+1)][vs] basis in FP32, precision MRA_FP32 only (else null)
  double* w;                // [cap]
  double* H;                // [(m+1)][m]
  double* hpart;            // [2][kMaxM+1] first-pass Gram-Schmidt coefficients, by column parity
  double* y;                // [kMaxM + 1]
  double* partials;         // [3][kRedBlocks][kMaxM + 2]
  double* scal;             // [S_NSCAL]
  int* ctrl;                // [C_NCTRL]
  // dense fields (element type by prec)
  void* wt;                 // Pi(omega)
  void* u;                  // velocity of Pi(omega)
  void* v;
  void* nu;                 // eddy viscosity of Pi(omega)
  void* vt;                 // Pi(v)
  void* uv;                 // velocity of Pi(v)
  void* vv;
  void* spec;               // complex half spectrum [(N/2+1)][N]: omega, then u
  void* spec2;              // the v spectrum, same shape
  double* vel64;            // FP64 velocity [2][Nf] of dense64 (diagnostics), and of res64
  double* res64;            // FP32-bulk solves: Pi(omega) in FP64 for the residual [Nf] (it
                            // shares the Krylov basis storage, which a step fills only later,
                            // when that holds Nf values)
  double* dense64;          // FP64 regrid field [Nf]; F(omega_n) during Newton iterations
  double* packed64;         // FP64 packed pyramid [Nf]; omega_n during Newton iterations
  double* out_rhs;          // residual at the active nodes [cap]
  double* out_jvp;          // J v at the active nodes [cap]
  const double* vin;        // active vector scattered by src 2 of the scatter
  double* diag;             // [N][4] per-row diagnostic partial sums
  uint8_t* lam;             // level-adapted evaluation: local level of each active node [Nf]
};

struct Batch {
  const SolveDev* s[kMaxBatch];
  int n;
};

// Launch geometry of a batch: a 1-D grid of n * gx blocks in which block
// L works for solve L % n as its block L / n.  Workgroups are dealt to the 8
// XCDs round-robin by linear id, so (for n dividing 8 or a multiple of 8) all
// blocks of one solve run on the same XCD(s) and consecutive kernels of that
// solve meet its data in the same L2.
#define MRA_SOLVE(b) (*(b).s[blockIdx.x % (b).n])
#define MRA_BX(b) ((int)(blockIdx.x / (b).n))
#define MRA_GX(b) ((int)(gridDim.x / (b).n))

// ------------------------------------------------------------------ helpers
// XCD-aware order of tiles (or row blocks).  Block L of a batch of n solves
// runs on XCD L % 8 and serves solve L % n as its block L / n, so one solve's
// blocks are spread over nx = 8 / gcd(n, 8) XCDs, its block bx landing on XCD
// group bx % nx.  Give each of those XCDs a contiguous run of tiles so that
// shared halos (or shared cache lines) stay in its L2 (nx = 1: plain order).
__device__ inline int tile_of_block(int bid, int ntiles, int nbatch) {
  int g = nbatch & 7;
  const int nx = g == 0 ? 1 : (g == 4 ? 2 : (g == 2 || g == 6 ? 4 : 8));
  if (nx == 1 || ntiles % nx != 0) return bid;
  return (bid % nx) * (ntiles / nx) + bid / nx;
}

__host__ __device__ inline int ilog2(unsigned v) { return 31 - __builtin_clz(v); }
__host__ __device__ inline int ntz(unsigned v) { return __builtin_ctz(v); }

// packed index -> fine index y*N + x (also returns level).
__device__ inline int packed_to_fine(int i, int J, int j0, int* level) {
  int N = 1 << J;
  int n0 = 1 << j0;
  if (i < n0 * n0) {
    int s0 = 1 << (J - j0);
    if (level) *level = j0;
    return (i >> j0) * s0 * N + (i & (n0 - 1)) * s0;
  }
  int l = (ilog2((unsigned)i) >> 1) + 1;
  int lb = l - 1;
  int n2 = 1 << (2 * lb);
  int band = (i >> (2 * lb)) - 1;
  int r = i - (band + 1) * n2;
  int b = r >> lb, a = r & ((1 << lb) - 1);
  int s = 1 << (J - l);
  int x = (2 * a + (band != 1 ? 1 : 0)) * s;
  int y = (2 * b + (band != 0 ? 1 : 0)) * s;
  if (level) *level = l;
  return y * N + x;
}

// fine (x, y) -> level.
__device__ inline int level_of(int x, int y, int J, int j0) {
  unsigned t = (unsigned)(x | y);
  int tz = t == 0 ? J : ntz(t);
  int l = J - tz;
  return l < j0 ? j0 : l;
}

// fine (x, y) of level l > j0 -> packed index.
__device__ inline int fine_to_packed(int x, int y, int l, int J, int j0) {
  if (l <= j0) {
    int s0 = 1 << (J - j0);
    return (y / s0) * (1 << j0) + x / s0;
  }
  int s = J - l;
  int xs = x >> s, ys = y >> s;
  int band = (xs & 1) ? ((ys & 1) ? 2 : 0) : 1;
  int lb = l - 1;
  return ((band + 1) << (2 * lb)) + ((ys >> 1) << lb) + (xs >> 1);
}

// Order-2p DD midpoint prediction from c[0..2P-1] = coarse values at offsets
// -P+1 .. P; one rounding per operation, pairs nearest first.
template <int P, typename T>
__device__ inline T dd_pred(const T* c) {
#pragma clang fp contract(off)
  if constexpr (P == 2) {
    T s = T(0.5625) * (c[1] + c[2]);
    s = s + T(-0.0625) * (c[0] + c[3]);
    return s;
  } else {
    T s = T(0.5859375) * (c[2] + c[3]);
    s = s + T(-0.09765625) * (c[1] + c[4]);
    s = s + T(0.01171875) * (c[0] + c[5]);
    return s;
  }
}

// Prediction of a non-coarse node (x, y) of level l from the level-(l-1)
// values of the dense field f (coarse stride S = 2^(J-l+1)).
template <int P, typename T, typename Ptr = const T*>
__device__ inline T predict_node(Ptr __restrict__ f, int x, int y, int l, int J) {
  const int N = 1 << J;
  const int s = 1 << (J - l);
  const int S = 2 * s;
  const int nm = N - 1;
  const bool ox = (x & s) != 0, oy = (y & s) != 0;
  T c[2 * P];
  if (ox && !oy) {
    const int row = y * N;
    const int x0 = x - s - (P - 1) * S;
#pragma unroll
    for (int o = 0; o < 2 * P; ++o) c[o] = f[row + ((x0 + o * S) & nm)];
    return dd_pred<P, T>(c);
  } else if (oy && !ox) {
    const int y0 = y - s - (P - 1) * S;
#pragma unroll
    for (int o = 0; o < 2 * P; ++o) c[o] = f[((y0 + o * S) & nm) * N + x];
    return dd_pred<P, T>(c);
  } else {
    T py[2 * P];
    const int x0 = x - s - (P - 1) * S;
    const int y0 = y - s - (P - 1) * S;
#pragma unroll
    for (int ox2 = 0; ox2 < 2 * P; ++ox2) {
      const int xx = (x0 + ox2 * S) & nm;
#pragma unroll
      for (int o = 0; o < 2 * P; ++o) c[o] = f[((y0 + o * S) & nm) * N + xx];
      py[ox2] = dd_pred<P, T>(c);
    }
    return dd_pred<P, T>(py);
  }
}

// Stencil tile edge: 32, or 16 where a 32-tile would need more than 64 KB of
// LDS (FP64 with the 6-point rule); never more than N.
__host__ __device__ inline int tile_edge(int J, int p, int prec) {
  const int t = (prec == 0 && p == 3) ? 16 : kTile;
  const int N = 1 << J;
  return N < t ? N : t;
}
// Whether a stencil tile edge can serve (J, p, bulk precision): 8, 16 or 32,
// at most N, and not the excluded 32-tile of FP64 with the 6-point rule.
inline bool tile_valid(int J, int p, int prec, int t) {
  if (t != 8 && t != 16 && t != 32) return false;
  if (t > (1 << J)) return false;
  return !(prec == 0 && p == 3 && t == 32);
}
// The tile a new solve takes: the one set by mra_tune_set_tile for its
// (J, p, bulk precision), else tile_edge.
int tile_choice(int J, int p, int prec);

// Solve buffers are device (global) memory, but their pointers reach the
// kernels through the solve descriptor, where the compiler cannot tell and
// emits flat accesses, which on gfx9 also hold the LDS wait counter.  Hot
// loops take them through glb().
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* glb(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Vector memory through a buffer resource.  Element k of vector i of a basis
// (stride `stride` bytes) is at byte i * stride + k * sizeof(T): the vector's
// offset is a scalar register and the element's offset one vector register
// shared by every vector, so a loop over the basis spends no address
// arithmetic per vector and no register pair per address.  The resource
// covers `bytes` (below 2 GiB for every basis: (kMaxM + 1) vectors of at most
// 2^22 + kBasisPad doubles); an access past it reads zero and writes nothing.
constexpr int kBufWord3 = 0x00020000;   // 32-bit data format, no swizzle, no stride
static_assert((long long)(kMaxM + 1) * ((1 << 22) + kBasisPad) * 8 < (1ll << 31), "basis exceeds a buffer resource");
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufWord3);
}
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <typename T>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, T v) {
  if constexpr (sizeof(T) == 8) {
    using R = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(R, v), r, voff, soff, 0);
  } else {
    using R = decltype(__builtin_amdgcn_raw_buffer_load_b32(r, 0u, 0u, 0));
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(R, v), r, voff, soff, 0);
  }
}

// The Krylov basis is stored in FP64, or in FP32 for solves of precision
// MRA_FP32 (every sum over it stays FP64 either way; the FP32 products take
// the basis vectors rounded to FP32 in both cases).
template <typename TV> __device__ inline TV* vbasis(const SolveDev& s);
template <> __device__ inline double* vbasis<double>(const SolveDev& s) { return s.V; }
template <> __device__ inline float* vbasis<float>(const SolveDev& s) { return s.V32; }

// ------------------------------------------------- Krylov reductions
constexpr double kBreakdown = 1e-13;
constexpr int kChunkMin = 512;

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

struct Chunk {
  int lo, hi;
};
__device__ inline int nchunks(int na) {
  int nb = (na + kChunkMin - 1) / kChunkMin;
  if (nb < 1) nb = 1;
  return nb > kRedBlocks ? kRedBlocks : nb;
}
__device__ inline Chunk chunk_of(int na, int ch) {
  const int nb = nchunks(na);
  const int per = (na + nb - 1) / nb;
  Chunk c;
  c.lo = ch * per;
  c.hi = c.lo + per < na ? c.lo + per : na;
  return c;
}

// Partial-sum buffers: the Gram-Schmidt's first stage writes buffer 0, the
// residual norm buffer 1, and the second stage of column j buffer
// 1 + (j & 1), so that a kernel never overwrites partials another block of
// the same kernel is still reading.  One slot of kMaxM + 2 sums per chunk.
constexpr int kWavesPerBlock = 4;
constexpr int kPartSlots = kRedBlocks;
__device__ inline double* part_buf(const SolveDev& s, int which) {
  return s.partials + (size_t)which * kPartSlots * (kMaxM + 2);
}

// totals[i] = sum over the nb slots of buf[slot][i], i < cnt <= kMaxM + 2, in
// a fixed order (wavefront w adds slots w, w + 4, ... in turn, lane i holds
// sum i, then the four wavefronts in order): every block that calls this gets
// bit-identical totals.  totals is in LDS.  U slots per lane are in flight at
// once: the Gram-Schmidt stages take 32 (their sums over up to 512 slots sit
// in front of every block's pass), kernels where the reduction is a side
// path keep 8, so that it does not raise their register count.
template <int U = 8>
__device__ inline void reduce_partials(const double* buf, int nb, int cnt, double* totals) {
  __shared__ double part[kWavesPerBlock][kMaxM + 2];
  const int stride = kMaxM + 2;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const auto* g = glb(buf);
  double t = 0.0;
  if (lane < cnt) {
#pragma unroll U
    for (int q = wid; q < nb; q += kWavesPerBlock) t += g[q * stride + lane];
    part[wid][lane] = t;
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    double a = part[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kWavesPerBlock; ++w) a += part[w][threadIdx.x];
    totals[threadIdx.x] = a;
  }
  __syncthreads();
}

// Two reductions in one pass over the slots (cnt_a + cnt_b <= 64): lanes
// below cnt_a sum buffer a, the next cnt_b lanes buffer b, each in the order
// of reduce_partials (so the totals are bit-identical to two calls of it).
__device__ inline void reduce_partials2(const double* bufa, int cnta, double* tota, const double* bufb, int cntb,
                                        double* totb, int nb) {
  __shared__ double part[kWavesPerBlock][64];
  const int stride = kMaxM + 2;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const bool ina = lane < cnta, inb = !ina && lane < cnta + cntb;
  const auto* g = glb(ina ? bufa + lane : bufb + (lane - cnta));
  double t = 0.0;
  if (ina || inb) {
#pragma unroll 32
    for (int q = wid; q < nb; q += kWavesPerBlock) t += g[q * stride];
    part[wid][lane] = t;
  }
  __syncthreads();
  const int i = threadIdx.x;
  if (i < cnta + cntb) {
    double a = part[0][i];
#pragma unroll
    for (int w = 1; w < kWavesPerBlock; ++w) a += part[w][i];
    if (i < cnta) tota[i] = a;
    else totb[i - cnta] = a;
  }
  __syncthreads();
}

// Sums of acc[0 .. cnt) over the block (fixed order: within each wavefront a
// butterfly, then the wavefronts in order) written to out[0 .. cnt).
template <int NA>
__device__ inline void block_sums_store(double (&acc)[NA], int cnt, double* out) {
  __shared__ double part[kWavesPerBlock][NA];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    if (i < cnt) {
      double v = acc[i];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0) part[wid][i] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    double a = part[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kWavesPerBlock; ++w) a += part[w][threadIdx.x];
    glb(out)[threadIdx.x] = a;
  }
}

// The scaling of the first basis vector: beta = ||F|| from the partials of
// k_norm0 (buffer B).  Every block computes the same value; block 0 records
// beta and starts the basis (C_MEFF = m, or 0 and C_DONE when F = 0 or is not
// finite).  Returns 1 / beta, or 0.  Later basis vectors are normalised by
// the Gram-Schmidt stage of the column after theirs.
__device__ inline double first_scale(const SolveDev& s, int bx) {
  __shared__ double tot[2];
  __shared__ double inv_sh;
  const int na = (int)*s.n_active;
  const int nb = nchunks(na);
  reduce_partials(part_buf(s, 1), nb, 1, tot);
  if (threadIdx.x == 0) {
    const double nrm = sqrt(tot[0]);
    const bool ok = isfinite(nrm);
    const bool zero = !(nrm > 0.0) || !ok;
    if (bx == 0) {
      s.scal[S_BETA] = nrm;
      if (!ok) s.ctrl[C_STATUS] = 5;
      s.ctrl[C_DONE] = zero ? 1 : 0;
      s.ctrl[C_MEFF] = zero ? 0 : s.m;
    }
    inv_sh = zero ? 0.0 : 1.0 / nrm;
  }
  __syncthreads();
  return inv_sh;
}

// ------------------------------------------------------------- launchers
// Each returns hipSuccess or the launch error.  `nb` solves in `b`.
struct LaunchCfg {
  int J, p, prec, m;
  int kind = 0;   // 0 vorticity, 1 passive scalar coupled to a vorticity solve
  int integ = 0;  // 0 exponential Rosenbrock-Euler, 1 theta-scheme by Newton-GMRES
  int newton = 0; // Newton iterations per step (integ 1)
  int jac = 0;    // Jacobian of the Krylov products: 0 eddy viscosity frozen, 1 exact
  int vb = 0;     // Krylov basis stored in FP32 (precision MRA_FP32); FP64 otherwise
  int tile = 0;   // stencil tile edge of the solves (their SolveDev tile)
  int adapt = 0;  // evaluation: 0 dense, 1 level-adapted at the active nodes
};

hipError_t launch_write_desc(SolveDev* dst, const SolveDev& src, hipStream_t st);

// transforms
// Pi into target (0 wt, 1 vt, 2 dense64, 3 res64) from src (0 omega, 1 the
// next Arnoldi vector V_j, 2 vin); as_double selects the element type.
hipError_t launch_prolong(const Batch& b, const LaunchCfg& c, int target, int as_double, int src, int j,
                          hipStream_t st);
hipError_t launch_forward(const Batch& b, const LaunchCfg& c, int src /*0 dense64 (fp64), 1 wt*/,
                          int dst /*0 packed64, 1 spec-as-packed (T)*/, hipStream_t st);
hipError_t launch_inverse(const Batch& b, const LaunchCfg& c, hipStream_t st);
hipError_t launch_threshold(const Batch& b, const LaunchCfg& c, int packed_is_double, hipStream_t st);
hipError_t launch_gather(const Batch& b, const LaunchCfg& c, hipStream_t st);
hipError_t launch_rank_from_index(const Batch& b, const LaunchCfg& c, hipStream_t st);
hipError_t launch_reset_max(const Batch& b, hipStream_t st);

// Poisson
hipError_t fft_init_tables(hipStream_t st);
hipError_t launch_poisson(const Batch& b, const LaunchCfg& c,
                          int src /*0 wt->(u,v), 1 vt->(uv,vv), 2 dense64->vel64, 3 res64->vel64 (fp64)*/,
                          hipStream_t st);
hipError_t launch_poisson_pass(const Batch& b, const LaunchCfg& c, int src, int pass, hipStream_t st);

// stencils
// The residual: FP64 solves from wt, u, v; FP32-bulk solves in FP64 from res64
// and vel64, also writing the FP32 wt, u, v and nu_e that their products read.
hipError_t launch_rhs(const Batch& b, const LaunchCfg& c, hipStream_t st);
hipError_t launch_jvp(const Batch& b, const LaunchCfg& c, hipStream_t st);
// level-adapted evaluation: local levels, residual and products at the active nodes
hipError_t launch_local_level(const Batch& b, const LaunchCfg& c, hipStream_t st);
hipError_t launch_rhs_adapted(const Batch& b, const LaunchCfg& c, hipStream_t st);
hipError_t launch_jvp_adapted(const Batch& b, const LaunchCfg& c, hipStream_t st);
// passive-scalar operator at the active nodes (check_done: skip once the basis is complete)
hipError_t launch_scalar(const Batch& b, const LaunchCfg& c, int check_done, hipStream_t st);
hipError_t launch_fill(void* f, size_t n, int prec, double value, hipStream_t st);
// vortex-centre row sums of dense64 (K <= kMaxTrack centres) into rows[N][K][3]
constexpr int kMaxTrack = 4;
hipError_t launch_track(const Batch& b, const LaunchCfg& c, const double* cx, const double* cy, int k,
                        double* rows, hipStream_t st);
hipError_t launch_diag(const Batch& b, const LaunchCfg& c, hipStream_t st);

// Krylov
hipError_t launch_norm0(const Batch& b, const LaunchCfg& c, hipStream_t st);
hipError_t launch_arnoldi(const Batch& b, const LaunchCfg& c, int j, hipStream_t st);
hipError_t launch_phi1(const Batch& b, const LaunchCfg& c, hipStream_t st);
hipError_t launch_update(const Batch& b, const LaunchCfg& c, hipStream_t st);
// theta-scheme Newton iteration: w <- -G(omega_k) (first: keep omega_n, F_n);
// GMRES least squares on the shifted Hessenberg matrix; omega += V y
// (last: the step's time advance)
hipError_t launch_newton_rhs(const Batch& b, const LaunchCfg& c, int first, hipStream_t st);
hipError_t launch_gmres(const Batch& b, const LaunchCfg& c, hipStream_t st);
hipError_t launch_newton_update(const Batch& b, const LaunchCfg& c, int last, hipStream_t st);
hipError_t launch_set_scal(const Batch& b, int idx, double value, hipStream_t st);
hipError_t launch_reset_ctrl(const Batch& b, hipStream_t st);
hipError_t launch_clear_done(const Batch& b, hipStream_t st);

}  // namespace mra
