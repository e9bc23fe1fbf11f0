// C-ABI of the library: argument checks, workspace / arena layouts, the
// sequence of launches of one exponential step, HIP-graph capture of that
// step, batching of solves, read-back and diagnostics.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/mra.h"
#include "mra_internal.hpp"

using namespace mra;

// Workspace of mra_transform_noalloc: one per device, in module memory, for
// grids up to kScratchMaxJ (the transform's descriptor, max|u|, compaction
// offsets, rank map and tile counts: about 4.1 MB at J = 10).  Every call on a
// device shares it, so such calls must not overlap on that device.
constexpr int kScratchMaxJ = 10;
constexpr size_t kScratchBytes = (size_t)5 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

struct mra_solve_s {
  SolveDev host;          // pointers into the arena
  SolveDev* dev = nullptr;
  LaunchCfg cfg{};
  int device = 0;
  hipGraphExec_t graph = nullptr;
  hipGraph_t graph_def = nullptr;
  hipStream_t graph_stream = nullptr;
  std::vector<double> diag_rows;
  long steps = 0;                 // steps enqueued so far
  mra_solve_s* partner = nullptr; // passive scalar: the vorticity solve it rides on
  int riders = 0;                 // passive scalars riding on this solve
};

static_assert(kStatusCapacity == MRA_E_CAPACITY, "status word value of a capacity overflow");

namespace {

std::mutex g_mu;
bool g_init[64] = {};
void* g_scratch[64] = {};   // per device: the address of `scratch` on that device

#define MRA_TRY(expr)                                   \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return MRA_E_DEVICE;          \
  } while (0)

int32_t ensure_init() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MRA_E_DEVICE;
  if (dev < 0 || dev >= 64) return MRA_E_DEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_init[dev]) return MRA_OK;
  // the device copy of the no-allocation workspace: its address on this
  // device (the host-side name of the array is not a device address)
  void* sp = nullptr;
  if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) return MRA_E_DEVICE;
  g_scratch[dev] = sp;
  MRA_TRY(fft_init_tables(nullptr));
  MRA_TRY(hipDeviceSynchronize());
  g_init[dev] = true;
  return MRA_OK;
}

int32_t check_grid(const mra_grid_desc* g) {
  if (!g) return MRA_E_ARG;
  if (g->p != 2 && g->p != 3) return MRA_E_SIZE;
  const int j0 = g->p == 2 ? 2 : 3;
  if (g->j0 != j0) return MRA_E_SIZE;
  if (g->J < j0 + 1 || g->J > kMaxJ) return MRA_E_SIZE;
  if (!(g->length > 0.0) || !(g->eps >= 0.0) || !std::isfinite(g->eps)) return MRA_E_ARG;
  if (g->adjacent_zone != 0 && g->adjacent_zone != 1) return MRA_E_ARG;
  return MRA_OK;
}

int32_t check_flow(const mra_flow_desc* f) {
  if (!f) return MRA_E_ARG;
  if (!(f->nu0 >= 0.0) || !(f->mu >= 0.0) || !(f->cs >= 0.0) || !(f->s0 >= 0.0)) return MRA_E_ARG;
  if (f->smag_mode < 0 || f->smag_mode > 2) return MRA_E_ARG;
  return MRA_OK;
}

int prec_bulk(int32_t prec) { return prec == MRA_FP64 ? 0 : 1; }

// Tile edges set by mra_tune_set_tile, per (J, p - 2, bulk precision); 0 keeps
// the default rule.  Read when a solve or workspace is laid out.
static std::atomic<int> g_tile_set[kMaxJ + 1][2][2];


// Simple bump allocator over a caller buffer (null base = size query).  Each
// array is 256-byte aligned and followed by 4 KB, so that arrays of
// power-of-two size do not all start on the same DRAM channel (the stencils
// read six N^2 fields at the same node).
constexpr size_t kStagger = 4096;
struct Layout {
  char* base;
  size_t off = 0;
  explicit Layout(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T) + kStagger;
    return p;
  }
};

void fill_geometry(SolveDev& s, const mra_grid_desc* g, int32_t prec) {
  std::memset(&s, 0, sizeof(s));
  s.J = g->J;
  s.j0 = g->j0;
  s.p = g->p;
  s.N = 1 << g->J;
  s.prec = prec_bulk(prec);
  s.vb32 = prec == MRA_FP32;
  s.adjacent_zone = g->adjacent_zone;
  s.tile = tile_choice(s.J, s.p, s.prec);
  s.ntx = s.N / s.tile;
  s.cap = s.N * s.N;
  s.vs = s.cap + kBasisPad;
  s.length = g->length;
  s.h = g->length / s.N;
  s.eps = g->eps;
}

void fill_flow(SolveDev& s, const mra_flow_desc* f) {
  s.nu0 = f->nu0;
  s.cs = f->cs;
  s.s0 = f->s0;
  s.mu = f->mu;
  s.smag_mode = f->smag_mode;
}

int nscan_of(int J) {
  const int nf = 1 << (2 * J);
  return (nf + kScanBlock * kScanItems - 1) / (kScanBlock * kScanItems);
}

// Workspace of the stand-alone transform.
void transform_layout(Layout& L, SolveDev& s) {
  const size_t Nf = (size_t)s.N * s.N;
  (void)L.take<SolveDev>(1);
  s.umax = L.take<unsigned long long>(1);
  s.ctrl = L.take<int>(C_NCTRL);
  s.scal = L.take<double>(S_NSCAL);
  s.block_off = L.take<int32_t>(nscan_of(s.J));
  s.rank = L.take<int32_t>(Nf);
  s.tile_count = L.take<int32_t>((size_t)s.ntx * s.ntx);
}

// Workspace of the stand-alone residual / JVP.
void rhs_layout(Layout& L, SolveDev& s) {
  const size_t Nf = (size_t)s.N * s.N;
  const size_t esz = s.prec == 0 ? 8 : 4;
  (void)L.take<SolveDev>(1);
  s.ctrl = L.take<int>(C_NCTRL);
  s.scal = L.take<double>(S_NSCAL);
  s.rank = L.take<int32_t>(Nf);
  s.tile_count = L.take<int32_t>((size_t)s.ntx * s.ntx);
  s.wt = L.take<char>(Nf * esz);
  s.u = L.take<char>(Nf * esz);
  s.v = L.take<char>(Nf * esz);
  s.nu = L.take<char>(Nf * esz);
  s.vt = L.take<char>(Nf * esz);
  s.uv = L.take<char>(Nf * esz);
  s.vv = L.take<char>(Nf * esz);
  // the residual of FP32 bulk fields runs in FP64: its prolongation, velocity
  // and FP64 spectra
  s.spec = L.take<char>((size_t)(s.N / 2 + 1) * s.N * 16);
  s.spec2 = L.take<char>((size_t)(s.N / 2 + 1) * s.N * 16);
  if (s.prec != 0) {
    s.res64 = L.take<double>(Nf);
    s.vel64 = L.take<double>(2 * Nf);
    s.dense64 = L.take<double>(Nf);     // FP64 nu_e of the level-adapted residual
  }
  s.lam = L.take<uint8_t>(Nf);
  s.out_rhs = L.take<double>(Nf);
}

// Arena of a solve.  The active-length arrays and the basis vectors hold
// s.cap entries (at most N^2); everything indexed by grid node holds N^2.
void solve_layout(Layout& L, SolveDev& s) {
  const size_t Nf = (size_t)s.N * s.N;
  const size_t cap = (size_t)s.cap;
  const size_t esz = s.prec == 0 ? 8 : 4;
  (void)L.take<SolveDev>(1);
  s.ctrl = L.take<int>(C_NCTRL);
  s.scal = L.take<double>(S_NSCAL);
  s.umax = L.take<unsigned long long>(1);
  s.n_active = L.take<int64_t>(1);
  s.mask = L.take<uint8_t>(Nf);
  s.index_packed = L.take<int32_t>(cap);
  s.index_fine = L.take<int32_t>(cap);
  s.rank = L.take<int32_t>(Nf);
  s.tile_count = L.take<int32_t>((size_t)s.ntx * s.ntx);
  s.block_off = L.take<int32_t>(nscan_of(s.J));
  s.omega = L.take<double>(cap);
  s.V = nullptr;
  s.V32 = nullptr;
  s.vs = s.cap + kBasisPad;
  if (s.vb32) s.V32 = L.take<float>((size_t)(s.m + 1) * s.vs);
  else s.V = L.take<double>((size_t)(s.m + 1) * s.vs);
  s.w = L.take<double>(cap);
  s.H = L.take<double>((size_t)(s.m + 1) * s.m);
  s.hpart = L.take<double>(2 * (kMaxM + 1));
  s.y = L.take<double>(kMaxM + 1);
  s.partials = L.take<double>((size_t)3 * kPartSlots * (kMaxM + 2));
  s.wt = L.take<char>(Nf * esz);
  s.u = L.take<char>(Nf * esz);
  s.v = L.take<char>(Nf * esz);
  s.nu = L.take<char>(Nf * esz);
  s.vt = L.take<char>(Nf * esz);
  s.uv = L.take<char>(Nf * esz);
  s.vv = L.take<char>(Nf * esz);
  s.vel64 = L.take<double>(2 * Nf);  // FP64 for the diagnostics
  s.spec = L.take<char>((size_t)(s.N / 2 + 1) * s.N * 16);
  s.spec2 = L.take<char>((size_t)(s.N / 2 + 1) * s.N * 16);
  s.dense64 = L.take<double>(Nf);
  s.packed64 = L.take<double>(Nf);
  s.diag = L.take<double>((size_t)s.N * 5);
  s.lam = L.take<uint8_t>(cap);
  s.out_rhs = s.w;
  s.out_jvp = s.w;
  // FP32 bulk fields: the FP64 prolongation of the residual lives in the
  // basis storage ((m + 1) cap elements, m >= 1), which a step writes only
  // after the residual (V_0 = F / beta is written by the first product's Pi),
  // when that holds N^2 doubles; else in a buffer of its own
  if (s.prec != 0) {
    const size_t vbytes = (size_t)(s.m + 1) * s.vs * (s.vb32 ? 4 : 8);
    s.res64 = vbytes >= Nf * 8 ? (s.V ? s.V : reinterpret_cast<double*>(s.V32)) : L.take<double>(Nf);
  }
}

Batch one(const SolveDev* d) {
  Batch b;
  std::memset(&b, 0, sizeof(b));
  b.s[0] = d;
  b.n = 1;
  return b;
}

// The residual F(omega) at the active nodes, with u, v and nu_e of Pi(omega)
// left in the bulk fields for the Jacobian-vector products.  FP64 solves
// prolong, solve the Poisson equation and evaluate the stencil in their own
// fields; solves with FP32 bulk fields do all three in FP64 (res64, vel64)
// and the stencil kernel leaves the FP32 copies that the products read.
hipError_t enqueue_residual(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  hipError_t e;
  const bool dbl = c.prec == 0;
  if ((e = launch_prolong(b, c, dbl ? 0 : 3, 1, 0, 0, st)) != hipSuccess) return e;
  if ((e = launch_poisson(b, c, dbl ? 0 : 3, st)) != hipSuccess) return e;
  return launch_rhs(b, c, st);
}

// One exponential step of passive scalars: the operator is linear in the
// scalar, so its residual and its Arnoldi products are the same stencil on
// Pi(r) and Pi(v_j); no Poisson solve (the velocity is the partner's).
hipError_t enqueue_scalar_step(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  const int dbl = c.prec == 0;
  hipError_t e;
  if ((e = launch_prolong(b, c, 1, dbl, 0, 0, st)) != hipSuccess) return e;
  if ((e = launch_scalar(b, c, 0, st)) != hipSuccess) return e;
  if ((e = launch_norm0(b, c, st)) != hipSuccess) return e;
  for (int j = 0; j < c.m; ++j) {
    if ((e = launch_prolong(b, c, 1, dbl, j == 0 ? 1 : 3, j, st)) != hipSuccess) return e;
    if ((e = launch_scalar(b, c, 1, st)) != hipSuccess) return e;
    if ((e = launch_arnoldi(b, c, j, st)) != hipSuccess) return e;
  }
  if ((e = launch_phi1(b, c, st)) != hipSuccess) return e;
  if ((e = launch_update(b, c, st)) != hipSuccess) return e;
  if ((e = launch_prolong(b, c, 2, 1, 0, 0, st)) != hipSuccess) return e;
  if ((e = launch_reset_max(b, st)) != hipSuccess) return e;
  if ((e = launch_forward(b, c, 0, 0, st)) != hipSuccess) return e;
  if ((e = launch_threshold(b, c, 1, st)) != hipSuccess) return e;
  return launch_gather(b, c, st);
}

// One theta-scheme step by Newton-GMRES: Newton iteration k evaluates
// F(omega_k) (and the frozen fields of J at omega_k), forms -G(omega_k), runs
// the Arnoldi process of J from it, solves the GMRES least squares on the
// shifted Hessenberg matrix and adds V y; then the FP64 regrid.
hipError_t enqueue_theta_step(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  const int dbl = c.prec == 0;
  hipError_t e;
  for (int it = 0; it < c.newton; ++it) {
    if ((e = enqueue_residual(b, c, st)) != hipSuccess) return e;
    if ((e = launch_newton_rhs(b, c, it == 0, st)) != hipSuccess) return e;
    if ((e = launch_norm0(b, c, st)) != hipSuccess) return e;
    for (int j = 0; j < c.m; ++j) {
      if ((e = launch_prolong(b, c, 1, dbl, j == 0 ? 1 : 3, j, st)) != hipSuccess) return e;
      if ((e = launch_poisson(b, c, 1, st)) != hipSuccess) return e;
      if ((e = launch_jvp(b, c, st)) != hipSuccess) return e;
      if ((e = launch_arnoldi(b, c, j, st)) != hipSuccess) return e;
    }
    if ((e = launch_gmres(b, c, st)) != hipSuccess) return e;
    if ((e = launch_newton_update(b, c, it == c.newton - 1, st)) != hipSuccess) return e;
  }
  if ((e = launch_prolong(b, c, 2, 1, 0, 0, st)) != hipSuccess) return e;
  if ((e = launch_reset_max(b, st)) != hipSuccess) return e;
  if ((e = launch_forward(b, c, 0, 0, st)) != hipSuccess) return e;
  if ((e = launch_threshold(b, c, 1, st)) != hipSuccess) return e;
  return launch_gather(b, c, st);
}

// One exponential Rosenbrock-Euler step with regrid for every solve of b.
hipError_t enqueue_step(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  if (c.kind == 1) return enqueue_scalar_step(b, c, st);
  if (c.integ == 1) return enqueue_theta_step(b, c, st);
  const int dbl = c.prec == 0;
  hipError_t e;
  // residual F at omega
  if ((e = enqueue_residual(b, c, st)) != hipSuccess) return e;
  if ((e = launch_norm0(b, c, st)) != hipSuccess) return e;
  // Arnoldi
  for (int j = 0; j < c.m; ++j) {
    if ((e = launch_prolong(b, c, 1, dbl, j == 0 ? 1 : 3, j, st)) != hipSuccess) return e;
    if ((e = launch_poisson(b, c, 1, st)) != hipSuccess) return e;
    if ((e = launch_jvp(b, c, st)) != hipSuccess) return e;
    if ((e = launch_arnoldi(b, c, j, st)) != hipSuccess) return e;
  }
  if ((e = launch_phi1(b, c, st)) != hipSuccess) return e;
  if ((e = launch_update(b, c, st)) != hipSuccess) return e;
  // FP64 regrid: Pi on the old set, forward transform, threshold, gather
  if ((e = launch_prolong(b, c, 2, 1, 0, 0, st)) != hipSuccess) return e;
  if ((e = launch_reset_max(b, st)) != hipSuccess) return e;
  if ((e = launch_forward(b, c, 0, 0, st)) != hipSuccess) return e;
  if ((e = launch_threshold(b, c, 1, st)) != hipSuccess) return e;
  return launch_gather(b, c, st);
}

bool graphs_enabled() {
  const char* v = std::getenv("MRA_NO_GRAPH");
  return !(v && v[0] == '1');
}

struct GraphEntry {
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
};
std::map<std::pair<std::vector<const void*>, hipStream_t>, GraphEntry> g_batch_graphs;
constexpr size_t kMaxCachedGraphs = 32;

void drop_batch_graphs() {
  for (auto& kv : g_batch_graphs) {
    if (kv.second.x) (void)hipGraphExecDestroy(kv.second.x);
    if (kv.second.g) (void)hipGraphDestroy(kv.second.g);
  }
  g_batch_graphs.clear();
}

hipError_t capture(const Batch& b, const LaunchCfg& c, hipStream_t st, hipGraph_t* g, hipGraphExec_t* x) {
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t e1 = enqueue_step(b, c, st);
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(st, &graph);
  if (e1 != hipSuccess) { if (graph) (void)hipGraphDestroy(graph); return e1; }
  if (e2 != hipSuccess) return e2;
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) { (void)hipGraphDestroy(graph); return e; }
  *g = graph;
  *x = exec;
  return hipSuccess;
}

// One launch of a batch step: up to kMaxBatch solves of one configuration.
struct StepChunk {
  Batch b;
  LaunchCfg c;
};

// Side streams of the graph captures (per device, default priority); a
// captured graph does not refer to them once it is instantiated.
constexpr int kSideStreams = 16;
hipStream_t g_side[64][kSideStreams] = {};

hipError_t side_stream(int i, hipStream_t* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  hipStream_t& s = g_side[dev][i % kSideStreams];
  if (!s && (e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return e;
  *out = s;
  return hipSuccess;
}

// Captures one step of every chunk into one graph.  A single chunk is
// captured on `st` itself.  Several chunks become parallel branches: each is
// enqueued on a side stream that waits for a fork event of `st`, and `st`
// waits for each branch's join event before the capture ends.  Passive
// scalars read their partner's step, so their chunks fork only after every
// vorticity chunk has joined.
hipError_t capture_chunks(const std::vector<StepChunk>& chunks, hipStream_t st, hipGraph_t* g,
                          hipGraphExec_t* x) {
  if (chunks.size() == 1) return capture(chunks[0].b, chunks[0].c, st, g, x);
  std::vector<hipEvent_t> evs;
  auto new_event = [&](hipEvent_t* e) -> hipError_t {
    hipError_t r = hipEventCreateWithFlags(e, hipEventDisableTiming);
    if (r == hipSuccess) evs.push_back(*e);
    return r;
  };
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t e1 = hipSuccess;
  int next_side = 0;
  for (int kind = 0; kind <= 1 && e1 == hipSuccess; ++kind) {
    hipEvent_t fork;
    if ((e1 = new_event(&fork)) != hipSuccess || (e1 = hipEventRecord(fork, st)) != hipSuccess) break;
    for (const StepChunk& ch : chunks) {
      if (ch.c.kind != kind) continue;
      hipStream_t sd;
      hipEvent_t join;
      if ((e1 = side_stream(next_side++, &sd)) != hipSuccess || (e1 = hipStreamWaitEvent(sd, fork, 0)) != hipSuccess ||
          (e1 = enqueue_step(ch.b, ch.c, sd)) != hipSuccess || (e1 = new_event(&join)) != hipSuccess ||
          (e1 = hipEventRecord(join, sd)) != hipSuccess || (e1 = hipStreamWaitEvent(st, join, 0)) != hipSuccess)
        break;
    }
  }
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(st, &graph);
  for (hipEvent_t ev : evs) (void)hipEventDestroy(ev);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return e1 != hipSuccess ? e1 : e2;
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) { (void)hipGraphDestroy(graph); return e; }
  *g = graph;
  *x = exec;
  return hipSuccess;
}

}  // namespace

int mra::tile_choice(int J, int p, int prec) {
  if (J >= 0 && J <= kMaxJ && (p == 2 || p == 3) && (prec == 0 || prec == 1)) {
    const int t = g_tile_set[J][p - 2][prec].load(std::memory_order_relaxed);
    if (t != 0) return t;
  }
  return tile_edge(J, p, prec);
}

extern "C" {

const char* mra_status_str(int32_t st) {
  switch (st) {
    case MRA_OK: return "ok";
    case MRA_E_ARG: return "invalid argument";
    case MRA_E_SIZE: return "unsupported size";
    case MRA_E_NOMEM: return "buffer too small";
    case MRA_E_DEVICE: return "HIP error";
    case MRA_E_NONFINITE: return "non-finite value";
    case MRA_E_UNSUPPORTED: return "unsupported";
    case MRA_E_CAPACITY: return "active set exceeds the solve's capacity";
    default: return "unknown status";
  }
}

int32_t mra_abi_version(void) { return 1; }

int32_t mra_init(void) { return ensure_init(); }

int32_t mra_transform_ws_bytes(const mra_grid_desc* g, int32_t prec, size_t* bytes) {
  int32_t r = check_grid(g);
  if (r != MRA_OK) return r;
  if (!bytes || prec < 0 || prec > 2) return MRA_E_ARG;
  SolveDev s;
  fill_geometry(s, g, prec);
  Layout L(nullptr);
  transform_layout(L, s);
  *bytes = L.off + 256;
  return MRA_OK;
}

// Argument checks shared by mra_transform and mra_transform_noalloc.
static int32_t check_transform(const mra_grid_desc* g, int32_t prec, int32_t dir, const void* in, void* out,
                               uint8_t* mask, int32_t* index_packed, int32_t* index_fine, int64_t* n_active) {
  int32_t r = check_grid(g);
  if (r != MRA_OK) return r;
  if (prec < 0 || prec > 2 || !in || !out) return MRA_E_ARG;
  if (dir != MRA_FORWARD && dir != MRA_INVERSE && dir != MRA_PROLONG) return MRA_E_ARG;
  if (dir == MRA_FORWARD && mask && (!index_packed || !index_fine || !n_active)) return MRA_E_ARG;
  if (dir == MRA_PROLONG && (!mask || !index_fine || !n_active)) return MRA_E_ARG;
  return MRA_OK;
}

// The launches of a transform whose workspace (device address ws, already
// checked to be large enough) holds the descriptor and the scratch arrays.
static int32_t transform_enqueue(const mra_grid_desc* g, int32_t prec, int32_t dir, const void* in, void* out,
                                 uint8_t* mask, int32_t* index_packed, int32_t* index_fine, int64_t* n_active,
                                 void* ws, hipStream_t st) {
  SolveDev s;
  fill_geometry(s, g, prec);
  Layout L(ws);
  transform_layout(L, s);
  SolveDev* dev = reinterpret_cast<SolveDev*>(ws);
  const bool dbl = s.prec == 0;
  LaunchCfg c{s.J, s.p, s.prec, 0};
  c.tile = s.tile;
  s.mask = mask;
  s.index_packed = index_packed;
  s.index_fine = index_fine;
  s.n_active = n_active;
  if (dir == MRA_FORWARD) {
    if (dbl) { s.dense64 = (double*)in; s.packed64 = (double*)out; }
    else { s.wt = const_cast<void*>(in); s.spec = out; }
    MRA_TRY(launch_write_desc(dev, s, st));
    Batch b = one(dev);
    MRA_TRY(launch_reset_max(b, st));
    MRA_TRY(launch_forward(b, c, dbl ? 0 : 1, dbl ? 0 : 1, st));
    if (mask) MRA_TRY(launch_threshold(b, c, dbl ? 1 : 0, st));
  } else if (dir == MRA_INVERSE) {
    s.spec = const_cast<void*>(in);
    s.wt = out;
    MRA_TRY(launch_write_desc(dev, s, st));
    MRA_TRY(launch_inverse(one(dev), c, st));
  } else {
    s.omega = (double*)in;
    if (dbl) s.dense64 = (double*)out;
    else s.wt = out;
    MRA_TRY(launch_write_desc(dev, s, st));
    Batch b = one(dev);
    MRA_TRY(launch_rank_from_index(b, c, st));
    MRA_TRY(launch_prolong(b, c, dbl ? 2 : 0, dbl ? 1 : 0, 0, 0, st));
  }
  return MRA_OK;
}

int32_t mra_transform(const mra_grid_desc* g, int32_t prec, int32_t dir, const void* in, void* out,
                      uint8_t* mask, int32_t* index_packed, int32_t* index_fine, int64_t* n_active,
                      void* ws, size_t ws_bytes, void* stream) {
  int32_t r = check_transform(g, prec, dir, in, out, mask, index_packed, index_fine, n_active);
  if (r != MRA_OK) return r;
  if (!ws) return MRA_E_ARG;
  size_t need = 0;
  mra_transform_ws_bytes(g, prec, &need);
  if (ws_bytes < need) return MRA_E_NOMEM;
  if ((r = ensure_init()) != MRA_OK) return r;
  return transform_enqueue(g, prec, dir, in, out, mask, index_packed, index_fine, n_active, ws,
                           static_cast<hipStream_t>(stream));
}

int32_t mra_transform_noalloc(const mra_grid_desc* g, int32_t prec, int32_t dir, const void* in, void* out,
                              uint8_t* mask, int32_t* index_packed, int32_t* index_fine, int64_t* n_active,
                              void* stream) {
  int32_t r = check_transform(g, prec, dir, in, out, mask, index_packed, index_fine, n_active);
  if (r != MRA_OK) return r;
  size_t need = 0;
  mra_transform_ws_bytes(g, prec, &need);
  if (g->J > kScratchMaxJ || need > kScratchBytes) return MRA_E_SIZE;
  if ((r = ensure_init()) != MRA_OK) return r;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MRA_E_DEVICE;
  return transform_enqueue(g, prec, dir, in, out, mask, index_packed, index_fine, n_active, g_scratch[dev],
                           static_cast<hipStream_t>(stream));
}

int32_t mra_rhs_ws_bytes(const mra_grid_desc* g, int32_t prec, size_t* bytes) {
  int32_t r = check_grid(g);
  if (r != MRA_OK) return r;
  if (!bytes || prec < 0 || prec > 2) return MRA_E_ARG;
  SolveDev s;
  fill_geometry(s, g, prec);
  Layout L(nullptr);
  rhs_layout(L, s);
  *bytes = L.off + 256;
  return MRA_OK;
}

static int32_t rhs_impl(const mra_grid_desc* g, const mra_flow_desc* f, int32_t prec, const uint8_t* mask,
                        const int32_t* index_fine, const int64_t* n_active, const double* omega_active,
                        const double* v_active, double* out_active, void* vel_dense_or_null, void* ws,
                        size_t ws_bytes, void* stream, int adapt) {
  int32_t r = check_grid(g);
  if (r != MRA_OK) return r;
  if ((r = check_flow(f)) != MRA_OK) return r;
  if (prec < 0 || prec > 2 || !mask || !index_fine || !n_active || !omega_active || !out_active || !ws)
    return MRA_E_ARG;
  size_t need = 0;
  mra_rhs_ws_bytes(g, prec, &need);
  if (ws_bytes < need) return MRA_E_NOMEM;
  if ((r = ensure_init()) != MRA_OK) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  SolveDev s;
  fill_geometry(s, g, prec);
  fill_flow(s, f);
  Layout L(ws);
  rhs_layout(L, s);
  SolveDev* dev = reinterpret_cast<SolveDev*>(ws);
  s.mask = const_cast<uint8_t*>(mask);
  s.index_fine = const_cast<int32_t*>(index_fine);
  s.n_active = const_cast<int64_t*>(n_active);
  s.omega = const_cast<double*>(omega_active);
  if (vel_dense_or_null) {
    s.u = vel_dense_or_null;
    s.v = static_cast<char*>(vel_dense_or_null) + (size_t)s.N * s.N * (s.prec == 0 ? 8 : 4);
  }
  if (v_active) {
    s.out_jvp = out_active;
    s.vin = v_active;
  } else {
    s.out_rhs = out_active;
  }
  const int dbl = s.prec == 0;
  LaunchCfg c{s.J, s.p, s.prec, 0};
  c.tile = s.tile;
  c.adapt = adapt;
  MRA_TRY(launch_write_desc(dev, s, st));
  Batch b = one(dev);
  MRA_TRY(launch_reset_ctrl(b, st));
  MRA_TRY(launch_rank_from_index(b, c, st));
  MRA_TRY(enqueue_residual(b, c, st));
  if (v_active) {
    MRA_TRY(launch_prolong(b, c, 1, dbl, 2, 0, st));
    MRA_TRY(launch_poisson(b, c, 1, st));
    MRA_TRY(launch_jvp(b, c, st));
  }
  return MRA_OK;
}

int32_t collocation_rhs(const mra_grid_desc* g, const mra_flow_desc* f, int32_t prec, const uint8_t* mask,
                        const int32_t* index_fine, const int64_t* n_active, const double* omega_active,
                        const double* v_active, double* out_active, void* vel_dense_or_null, void* ws,
                        size_t ws_bytes, void* stream) {
  return rhs_impl(g, f, prec, mask, index_fine, n_active, omega_active, v_active, out_active, vel_dense_or_null,
                  ws, ws_bytes, stream, 0);
}

int32_t collocation_rhs_adapted(const mra_grid_desc* g, const mra_flow_desc* f, int32_t prec, const uint8_t* mask,
                                const int32_t* index_fine, const int64_t* n_active, const double* omega_active,
                                const double* v_active, double* out_active, void* vel_dense_or_null, void* ws,
                                size_t ws_bytes, void* stream) {
  return rhs_impl(g, f, prec, mask, index_fine, n_active, omega_active, v_active, out_active, vel_dense_or_null,
                  ws, ws_bytes, stream, 1);
}

// capacity 0: N^2; otherwise between the coarsest mesh's node count and N^2
static int32_t check_capacity(const mra_grid_desc* g, int64_t capacity) {
  const int64_t nf = (int64_t)1 << (2 * g->J);
  const int64_t n0 = (int64_t)1 << (2 * g->j0);
  if (capacity != 0 && (capacity < n0 || capacity > nf)) return MRA_E_SIZE;
  return MRA_OK;
}

int32_t mra_solve_footprint_cap(const mra_grid_desc* g, int32_t prec, int32_t m, int64_t capacity,
                                size_t* bytes) {
  int32_t r = check_grid(g);
  if (r != MRA_OK) return r;
  if (!bytes || prec < 0 || prec > 2) return MRA_E_ARG;
  if (m < 1 || m > kMaxM) return MRA_E_SIZE;
  if ((r = check_capacity(g, capacity)) != MRA_OK) return r;
  SolveDev s;
  fill_geometry(s, g, prec);
  s.m = m;
  if (capacity) s.cap = (int)capacity;
  Layout L(nullptr);
  solve_layout(L, s);
  *bytes = L.off + 256;
  return MRA_OK;
}

int32_t mra_solve_footprint(const mra_grid_desc* g, int32_t prec, int32_t m, size_t* bytes) {
  return mra_solve_footprint_cap(g, prec, m, 0, bytes);
}

// The launches that turn the FP64 field in s.dense64 into the active set and
// values of an arena (the regrid without its prolongation).
static hipError_t enqueue_regrid_from_dense(const Batch& b, const LaunchCfg& c, hipStream_t st) {
  hipError_t e;
  if ((e = launch_reset_max(b, st)) != hipSuccess || (e = launch_forward(b, c, 0, 0, st)) != hipSuccess ||
      (e = launch_threshold(b, c, 1, st)) != hipSuccess)
    return e;
  return launch_gather(b, c, st);
}

int32_t mra_solve_init_cap(const mra_grid_desc* g, const mra_flow_desc* f, int32_t prec, int32_t m, double dt,
                           const double* omega0_dense, int64_t capacity, void* arena, size_t arena_bytes,
                           void* stream, mra_solve* out, int64_t* needed) {
  int32_t r = check_grid(g);
  if (r != MRA_OK) return r;
  if ((r = check_flow(f)) != MRA_OK) return r;
  if (!omega0_dense || !arena || !out || prec < 0 || prec > 2) return MRA_E_ARG;
  if (m < 1 || m > kMaxM) return MRA_E_SIZE;
  if ((r = check_capacity(g, capacity)) != MRA_OK) return r;
  if (!(dt > 0.0) || !std::isfinite(dt)) return MRA_E_ARG;
  if ((reinterpret_cast<uintptr_t>(arena) & 255) != 0) return MRA_E_ARG;
  size_t need = 0;
  mra_solve_footprint_cap(g, prec, m, capacity, &need);
  if (arena_bytes < need) return MRA_E_NOMEM;
  if ((r = ensure_init()) != MRA_OK) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  mra_solve_s* h = new (std::nothrow) mra_solve_s();
  if (!h) return MRA_E_NOMEM;
  SolveDev& s = h->host;
  fill_geometry(s, g, prec);
  fill_flow(s, f);
  s.m = m;
  s.dt = dt;
  if (capacity) s.cap = (int)capacity;
  Layout L(arena);
  solve_layout(L, s);
  h->dev = reinterpret_cast<SolveDev*>(arena);
  h->cfg = LaunchCfg{s.J, s.p, s.prec, m};
  h->cfg.vb = s.vb32;
  h->cfg.tile = s.tile;
  (void)hipGetDevice(&h->device);
  h->diag_rows.resize((size_t)s.N * 5);
  const size_t Nf = (size_t)s.N * s.N;
  Batch b = one(h->dev);
  hipError_t e;
  if ((e = launch_write_desc(h->dev, s, st)) != hipSuccess ||
      (e = launch_reset_ctrl(b, st)) != hipSuccess ||
      (e = hipMemcpyAsync(s.dense64, omega0_dense, Nf * sizeof(double), hipMemcpyDeviceToDevice, st)) !=
          hipSuccess ||
      (e = enqueue_regrid_from_dense(b, h->cfg, st)) != hipSuccess) {
    delete h;
    return MRA_E_DEVICE;
  }
  if (s.cap < (int)Nf) {
    // the first active set must fit: a solve frozen before its first regrid
    // would have no previous set to fall back on
    int ctrl[C_NCTRL];
    if (hipMemcpyAsync(ctrl, s.ctrl, sizeof(ctrl), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      delete h;
      return MRA_E_DEVICE;
    }
    if (ctrl[C_OVER]) {
      if (needed) *needed = ctrl[C_NEED];
      delete h;
      return MRA_E_CAPACITY;
    }
  }
  *out = h;
  return MRA_OK;
}

int32_t mra_solve_init(const mra_grid_desc* g, const mra_flow_desc* f, int32_t prec, int32_t m, double dt,
                       const double* omega0_dense, void* arena, size_t arena_bytes, void* stream,
                       mra_solve* out) {
  return mra_solve_init_cap(g, f, prec, m, dt, omega0_dense, 0, arena, arena_bytes, stream, out, nullptr);
}

int32_t mra_solve_capacity(mra_solve h, int64_t* capacity, int64_t* needed, int32_t* frozen, void* stream) {
  if (!h || !capacity || !needed || !frozen) return MRA_E_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int ctrl[C_NCTRL];
  int64_t na = 0;
  MRA_TRY(hipMemcpyAsync(ctrl, h->host.ctrl, sizeof(ctrl), hipMemcpyDeviceToHost, st));
  MRA_TRY(hipMemcpyAsync(&na, h->host.n_active, sizeof(na), hipMemcpyDeviceToHost, st));
  MRA_TRY(hipStreamSynchronize(st));
  *capacity = h->host.cap;
  *frozen = ctrl[C_OVER] ? 1 : 0;
  *needed = ctrl[C_OVER] ? (int64_t)ctrl[C_NEED] : na;
  return MRA_OK;
}

static void drop_graphs_of(mra_solve h);

int32_t mra_solve_migrate(mra_solve h, int64_t capacity, void* arena, size_t arena_bytes, void* stream) {
  if (!h || !arena) return MRA_E_ARG;
  if (h->cfg.kind != 0 || h->riders) return MRA_E_UNSUPPORTED;
  if ((reinterpret_cast<uintptr_t>(arena) & 255) != 0) return MRA_E_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const SolveDev& o = h->host;
  mra_grid_desc g{};
  g.J = o.J;
  g.j0 = o.j0;
  g.p = o.p;
  g.eps = o.eps;
  g.length = o.length;
  g.adjacent_zone = o.adjacent_zone;
  const int32_t prec = o.prec == 0 ? MRA_FP64 : (o.vb32 ? MRA_FP32 : MRA_MIXED);
  int32_t r = check_capacity(&g, capacity);
  if (r != MRA_OK) return r;
  size_t need = 0;
  mra_solve_footprint_cap(&g, prec, o.m, capacity, &need);
  if (arena_bytes < need) return MRA_E_NOMEM;
  // the old arena's state: control words and counters, after its work
  MRA_TRY(hipStreamSynchronize(st));
  int ctrl[C_NCTRL];
  int64_t na = 0;
  MRA_TRY(hipMemcpy(ctrl, o.ctrl, sizeof(ctrl), hipMemcpyDeviceToHost));
  MRA_TRY(hipMemcpy(&na, o.n_active, sizeof(na), hipMemcpyDeviceToHost));
  const bool frozen = ctrl[C_OVER] != 0;
  const int64_t cap = capacity ? capacity : (int64_t)o.N * o.N;
  if ((frozen ? (int64_t)ctrl[C_NEED] : na) > cap) return MRA_E_SIZE;
  drop_graphs_of(h);
  SolveDev s = o;
  s.cap = (int)cap;
  Layout L(arena);
  solve_layout(L, s);
  SolveDev* dev = reinterpret_cast<SolveDev*>(arena);
  LaunchCfg c = h->cfg;
  Batch b = one(dev);
  const size_t Nf = (size_t)s.N * s.N;
  MRA_TRY(launch_write_desc(dev, s, st));
  MRA_TRY(launch_reset_ctrl(b, st));
  // time, step and evaluation counters, theta, ...
  MRA_TRY(hipMemcpyAsync(s.scal, o.scal, S_NSCAL * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (frozen) {
    // the pending regrid: the FP64 prolongation of omega on the old set
    MRA_TRY(launch_prolong(one(h->dev), c, 2, 1, 0, 0, st));
    MRA_TRY(hipMemcpyAsync(s.dense64, o.dense64, Nf * sizeof(double), hipMemcpyDeviceToDevice, st));
    MRA_TRY(enqueue_regrid_from_dense(b, c, st));
  } else {
    // the state as it is: active set, values and the tile counts
    MRA_TRY(hipMemcpyAsync(s.n_active, o.n_active, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
    MRA_TRY(hipMemcpyAsync(s.mask, o.mask, Nf, hipMemcpyDeviceToDevice, st));
    MRA_TRY(hipMemcpyAsync(s.rank, o.rank, Nf * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    MRA_TRY(hipMemcpyAsync(s.tile_count, o.tile_count, (size_t)s.ntx * s.ntx * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, st));
    if (na > 0) {
      MRA_TRY(hipMemcpyAsync(s.index_packed, o.index_packed, na * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
      MRA_TRY(hipMemcpyAsync(s.index_fine, o.index_fine, na * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
      MRA_TRY(hipMemcpyAsync(s.omega, o.omega, na * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
  }
  // the old arena is read until here: the caller may free it on return
  MRA_TRY(hipStreamSynchronize(st));
  h->host = s;
  h->dev = dev;
  return MRA_OK;
}

int32_t mra_scalar_init(mra_solve partner, const mra_grid_desc* g, int32_t m, double dt, double kappa0,
                        int32_t eddy, const double* r0_dense, void* arena, size_t arena_bytes, void* stream,
                        mra_solve* out) {
  if (!partner || partner->cfg.kind != 0) return MRA_E_ARG;
  // a scalar holds pointers into its partner's arena, which a move to a
  // larger one would leave behind
  if (partner->host.cap != partner->host.N * partner->host.N) return MRA_E_UNSUPPORTED;
  // a scalar step reads the partner's flow at the start of its step, which a
  // Newton step overwrites with the flow at its last iterate
  if (partner->cfg.integ != 0) return MRA_E_UNSUPPORTED;
  int32_t r = check_grid(g);
  if (r != MRA_OK) return r;
  if (g->J != partner->cfg.J || g->p != partner->cfg.p) return MRA_E_ARG;
  if (!r0_dense || !arena || !out) return MRA_E_ARG;
  if (m < 1 || m > kMaxM) return MRA_E_SIZE;
  if (!(dt > 0.0) || !std::isfinite(dt) || !(kappa0 >= 0.0) || !std::isfinite(kappa0)) return MRA_E_ARG;
  if ((reinterpret_cast<uintptr_t>(arena) & 255) != 0) return MRA_E_ARG;
  // the scalar takes its partner's precision, basis storage included
  const int32_t prec = partner->host.prec == 0 ? MRA_FP64 : (partner->host.vb32 ? MRA_FP32 : MRA_MIXED);
  size_t need = 0;
  mra_solve_footprint(g, prec, m, &need);
  if (arena_bytes < need) return MRA_E_NOMEM;
  if ((r = ensure_init()) != MRA_OK) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  mra_solve_s* h = new (std::nothrow) mra_solve_s();
  if (!h) return MRA_E_NOMEM;
  SolveDev& s = h->host;
  fill_geometry(s, g, prec);
  s.m = m;
  s.dt = dt;
  Layout L(arena);
  solve_layout(L, s);
  // the flow the scalar rides on: the partner's velocity and, for eddy
  // diffusion, its nu_e; otherwise a constant field of the scalar's own
  s.u = partner->host.u;
  s.v = partner->host.v;
  const size_t Nf = (size_t)s.N * s.N;
  if (eddy) s.nu = partner->host.nu;
  h->dev = reinterpret_cast<SolveDev*>(arena);
  h->cfg = LaunchCfg{s.J, s.p, s.prec, m, 1};
  h->cfg.vb = s.vb32;
  h->cfg.tile = s.tile;
  h->partner = partner;
  partner->riders += 1;
  h->steps = partner->steps;   // the next scalar step follows the partner's next step
  (void)hipGetDevice(&h->device);
  h->diag_rows.resize((size_t)s.N * 5);
  Batch b = one(h->dev);
  hipError_t e;
  if ((e = launch_write_desc(h->dev, s, st)) != hipSuccess || (e = launch_reset_ctrl(b, st)) != hipSuccess ||
      (!eddy && (e = launch_fill(s.nu, Nf, s.prec, kappa0, st)) != hipSuccess) ||
      (e = hipMemcpyAsync(s.dense64, r0_dense, Nf * sizeof(double), hipMemcpyDeviceToDevice, st)) != hipSuccess ||
      (e = launch_reset_max(b, st)) != hipSuccess || (e = launch_forward(b, h->cfg, 0, 0, st)) != hipSuccess ||
      (e = launch_threshold(b, h->cfg, 1, st)) != hipSuccess || (e = launch_gather(b, h->cfg, st)) != hipSuccess) {
    partner->riders -= 1;
    delete h;
    return MRA_E_DEVICE;
  }
  *out = h;
  return MRA_OK;
}

// A passive scalar's step k uses the velocity of its partner's step k, which
// lives in the partner's fields from that step's start until the next step.
static bool scalar_step_ready(const mra_solve_s* h) {
  return h->cfg.kind == 0 || (h->partner && h->partner->steps == h->steps + 1);
}

int32_t krylov_step(mra_solve h, int32_t nsteps, void* stream) {
  if (!h || nsteps < 0) return MRA_E_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Batch b = one(h->dev);
  if (nsteps == 0) return MRA_OK;
  if (h->cfg.kind == 1 && (nsteps != 1 || !scalar_step_ready(h))) return MRA_E_ARG;
  h->steps += nsteps;
  if (!st || !graphs_enabled()) {
    for (int i = 0; i < nsteps; ++i) MRA_TRY(enqueue_step(b, h->cfg, st));
    return MRA_OK;
  }
  if (!h->graph || h->graph_stream != st) {
    if (h->graph) { (void)hipGraphExecDestroy(h->graph); h->graph = nullptr; }
    if (h->graph_def) { (void)hipGraphDestroy(h->graph_def); h->graph_def = nullptr; }
    MRA_TRY(capture(b, h->cfg, st, &h->graph_def, &h->graph));
    h->graph_stream = st;
  }
  for (int i = 0; i < nsteps; ++i) MRA_TRY(hipGraphLaunch(h->graph, st));
  return MRA_OK;
}

int32_t solve_batch(mra_solve* solves, int32_t n, const int32_t* nsteps, void* stream) {
  if (!solves || !nsteps || n < 0) return MRA_E_ARG;
  for (int i = 0; i < n; ++i)
    if (!solves[i] || nsteps[i] < 0) return MRA_E_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int maxs = 0;
  for (int i = 0; i < n; ++i) maxs = std::max(maxs, nsteps[i]);
  const bool use_graph = st && graphs_enabled();
  for (int t = 0; t < maxs; ++t) {
    // the solves still running, grouped by launch configuration (vorticity
    // solves first: a scalar's step reads its partner's step) and cut into
    // launches of at most kMaxBatch solves
    std::map<std::tuple<int, int, int, int, int, int, int, int, int, int, int>, std::vector<mra_solve>> groups;
    for (int i = 0; i < n; ++i)
      if (nsteps[i] > t) {
        const LaunchCfg& c = solves[i]->cfg;
        groups[std::make_tuple(c.kind, c.J, c.p, c.prec, c.m, c.integ, c.newton, c.jac, c.vb, c.tile, c.adapt)]
            .push_back(solves[i]);
      }
    std::vector<StepChunk> chunks;
    std::vector<const void*> key;   // the composition: each launch's handles, then a null separator
    for (auto& kv : groups) {
      auto& v = kv.second;
      // groups in order, vorticity first: a scalar is ready once its
      // partner's step of this round is counted
      for (mra_solve h : v) {
        if (!scalar_step_ready(h)) return MRA_E_ARG;
        h->steps += 1;
      }
      for (size_t o = 0; o < v.size(); o += kMaxBatch) {
        StepChunk ch;
        std::memset(&ch.b, 0, sizeof(ch.b));
        ch.b.n = (int)std::min<size_t>(kMaxBatch, v.size() - o);
        for (int k = 0; k < ch.b.n; ++k) {
          ch.b.s[k] = v[o + k]->dev;
          key.push_back(v[o + k]);
        }
        key.push_back(nullptr);
        ch.c = v[o]->cfg;
        chunks.push_back(ch);
      }
    }
    if (!use_graph) {
      for (const StepChunk& ch : chunks) MRA_TRY(enqueue_step(ch.b, ch.c, st));
      continue;
    }
    // one graph per composition: every launch of the step is a branch of it,
    // so a step of the whole batch, whatever its sizes, is one graph launch
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_batch_graphs.find({key, st});
    if (it == g_batch_graphs.end()) {
      // bounded cache: a serving loop changes the batch composition often.
      // Drop this stream's graphs first (after the stream's work), and all
      // graphs only if it holds none.
      if (g_batch_graphs.size() >= kMaxCachedGraphs) {
        MRA_TRY(hipStreamSynchronize(st));
        bool dropped = false;
        for (auto d = g_batch_graphs.begin(); d != g_batch_graphs.end();) {
          if (d->first.second != st) { ++d; continue; }
          if (d->second.x) (void)hipGraphExecDestroy(d->second.x);
          if (d->second.g) (void)hipGraphDestroy(d->second.g);
          d = g_batch_graphs.erase(d);
          dropped = true;
        }
        if (!dropped) {
          MRA_TRY(hipDeviceSynchronize());   // cached graphs may be in flight on any stream
          drop_batch_graphs();
        }
      }
      GraphEntry ge;
      MRA_TRY(capture_chunks(chunks, st, &ge.g, &ge.x));
      it = g_batch_graphs.emplace(std::make_pair(key, st), ge).first;
    }
    MRA_TRY(hipGraphLaunch(it->second.x, st));
  }
  return MRA_OK;
}

int32_t mra_solve_read(mra_solve h, double* omega_dense_out, double* diag_out, void* stream) {
  if (!h) return MRA_E_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const SolveDev& s = h->host;
  const size_t Nf = (size_t)s.N * s.N;
  Batch b = one(h->dev);
  LaunchCfg c = h->cfg;
  MRA_TRY(launch_prolong(b, c, 2, 1, 0, 0, st));
  if (omega_dense_out)
    MRA_TRY(hipMemcpyAsync(omega_dense_out, s.dense64, Nf * sizeof(double), hipMemcpyDeviceToDevice, st));
  int64_t na = 0;
  int ctrl[C_NCTRL];
  double scal[S_NSCAL];
  if (diag_out) {
    MRA_TRY(launch_poisson(b, c, 2, st));
    MRA_TRY(launch_diag(b, c, st));
    MRA_TRY(hipMemcpyAsync(h->diag_rows.data(), s.diag, (size_t)s.N * 5 * sizeof(double),
                           hipMemcpyDeviceToHost, st));
  }
  MRA_TRY(hipMemcpyAsync(&na, s.n_active, sizeof(na), hipMemcpyDeviceToHost, st));
  MRA_TRY(hipMemcpyAsync(ctrl, s.ctrl, sizeof(ctrl), hipMemcpyDeviceToHost, st));
  MRA_TRY(hipMemcpyAsync(scal, s.scal, sizeof(scal), hipMemcpyDeviceToHost, st));
  MRA_TRY(hipStreamSynchronize(st));
  if (diag_out) {
    double sw = 0, suv = 0, sw2 = 0, sg = 0, mx = 0;
    for (int y = 0; y < s.N; ++y) {
      const double* r = &h->diag_rows[(size_t)y * 5];
      sw += r[0]; suv += r[1]; sw2 += r[2]; sg += r[3]; mx = std::max(mx, r[4]);
    }
    const double h2 = s.h * s.h;
    diag_out[0] = scal[S_T];
    diag_out[1] = 0.5 * h2 * suv;
    diag_out[2] = 0.5 * h2 * sw2;
    diag_out[3] = 0.5 * h2 * sg;
    diag_out[4] = h2 * sw;
    diag_out[5] = mx;
    diag_out[6] = (double)na;
    diag_out[7] = (double)ctrl[C_STATUS];
  }
  if (ctrl[C_STATUS] == kStatusCapacity) return MRA_E_CAPACITY;
  return ctrl[C_STATUS] == 0 ? MRA_OK : MRA_E_NONFINITE;
}

int32_t mra_solve_track(mra_solve h, int32_t k, double* centres, void* stream) {
  if (!h || !centres || k < 1 || k > kMaxTrack) return MRA_E_ARG;
  const SolveDev& s = h->host;
  for (int i = 0; i < 2 * k; ++i)
    if (!std::isfinite(centres[i])) return MRA_E_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Batch b = one(h->dev);
  const LaunchCfg& c = h->cfg;
  double cx[kMaxTrack], cy[kMaxTrack];
  for (int i = 0; i < k; ++i) { cx[i] = centres[2 * i]; cy[i] = centres[2 * i + 1]; }
  std::vector<double> rows((size_t)s.N * k * 3);
  MRA_TRY(launch_prolong(b, c, 2, 1, 0, 0, st));
  MRA_TRY(launch_track(b, c, cx, cy, k, s.vel64, st));
  MRA_TRY(hipMemcpyAsync(rows.data(), s.vel64, rows.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  MRA_TRY(hipStreamSynchronize(st));
  const double L = s.length;
  for (int i = 0; i < k; ++i) {
    double sw = 0.0, sx = 0.0, sy = 0.0;
    for (int y = 0; y < s.N; ++y) {
      const double* r = &rows[((size_t)y * k + i) * 3];
      sw += r[0]; sx += r[1]; sy += r[2];
    }
    if (!(sw > 0.0)) continue;                 // no positive vorticity: the centre stays
    const double nx = cx[i] + sx / sw, ny = cy[i] + sy / sw;
    centres[2 * i] = nx - L * std::floor(nx / L);
    centres[2 * i + 1] = ny - L * std::floor(ny / L);
  }
  return MRA_OK;
}

int32_t mra_solve_ptrs_get(mra_solve h, mra_solve_ptrs* out) {
  if (!h || !out) return MRA_E_ARG;
  const SolveDev& s = h->host;
  out->omega_active = s.omega;
  out->mask = s.mask;
  out->index_packed = s.index_packed;
  out->index_fine = s.index_fine;
  out->n_active = s.n_active;
  out->krylov_V = s.vb32 ? (void*)s.V32 : (void*)s.V;
  out->hessenberg = s.H;
  out->scalars = s.scal;
  out->control = s.ctrl;
  out->capacity = s.cap;
  out->basis_stride = s.vs;
  return MRA_OK;
}

// Drops every captured graph that launches h (its own and the cached batch
// graphs), after the work they may still have in flight.
static void drop_graphs_of(mra_solve h) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_batch_graphs.begin(); it != g_batch_graphs.end();) {
      const auto& key = it->first.first;
      if (std::find(key.begin(), key.end(), static_cast<const void*>(h)) == key.end()) { ++it; continue; }
      // the graph was launched only on its key's stream: wait for that stream
      (void)hipStreamSynchronize(it->first.second);
      if (it->second.x) (void)hipGraphExecDestroy(it->second.x);
      if (it->second.g) (void)hipGraphDestroy(it->second.g);
      it = g_batch_graphs.erase(it);
    }
  }
  if (h->graph) {
    (void)hipStreamSynchronize(h->graph_stream);
    (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
  }
  if (h->graph_def) {
    (void)hipGraphDestroy(h->graph_def);
    h->graph_def = nullptr;
  }
  h->graph_stream = nullptr;
}

int32_t mra_solve_set_integrator(mra_solve h, int32_t integrator, double theta, int32_t newton_iters,
                                 void* stream) {
  if (!h) return MRA_E_ARG;
  if (integrator != MRA_EXPONENTIAL && integrator != MRA_THETA_NEWTON) return MRA_E_ARG;
  if (integrator == MRA_THETA_NEWTON) {
    if (!(theta >= 0.0 && theta <= 1.0)) return MRA_E_ARG;
    if (newton_iters < 1 || newton_iters > MRA_MAX_NEWTON) return MRA_E_ARG;
  }
  if (h->cfg.kind != 0) return MRA_E_UNSUPPORTED;
  if (integrator == MRA_THETA_NEWTON && (h->riders > 0 || h->cfg.adapt)) return MRA_E_UNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  drop_graphs_of(h);
  if (integrator == MRA_THETA_NEWTON) MRA_TRY(launch_set_scal(one(h->dev), S_THETA, theta, st));
  h->cfg.integ = integrator;
  h->cfg.newton = integrator == MRA_THETA_NEWTON ? newton_iters : 0;
  return MRA_OK;
}

int32_t mra_solve_set_evaluation(mra_solve h, int32_t evaluation) {
  if (!h) return MRA_E_ARG;
  if (evaluation != MRA_EVAL_DENSE && evaluation != MRA_EVAL_ADAPTED) return MRA_E_ARG;
  if (h->cfg.kind != 0) return MRA_E_UNSUPPORTED;
  // the adapted residual keeps the FP64 eddy viscosity in the regrid field,
  // which the theta-scheme's Newton iterations hold; its products are the
  // frozen-viscosity ones
  if (evaluation == MRA_EVAL_ADAPTED && (h->cfg.integ != 0 || h->cfg.jac != 0)) return MRA_E_UNSUPPORTED;
  drop_graphs_of(h);
  h->cfg.adapt = evaluation;
  return MRA_OK;
}

int32_t mra_tune_set_tile(int32_t J, int32_t p, int32_t prec, int32_t tile) {
  if (J < 3 || J > kMaxJ || (p != 2 && p != 3) || prec < 0 || prec > 2) return MRA_E_ARG;
  const int bulk = prec_bulk(prec);
  if (tile != 0 && !tile_valid(J, p, bulk, tile)) return MRA_E_ARG;
  g_tile_set[J][p - 2][bulk].store(tile, std::memory_order_relaxed);
  return MRA_OK;
}

int32_t mra_tune_get_tile(int32_t J, int32_t p, int32_t prec, int32_t* tile) {
  if (!tile || J < 3 || J > kMaxJ || (p != 2 && p != 3) || prec < 0 || prec > 2) return MRA_E_ARG;
  *tile = tile_choice(J, p, prec_bulk(prec));
  return MRA_OK;
}

int32_t mra_scalar_set_condensation(mra_solve h, double rate, void* stream) {
  if (!h || !(rate >= 0.0) || !std::isfinite(rate)) return MRA_E_ARG;
  if (h->cfg.kind != 1) return MRA_E_UNSUPPORTED;
  MRA_TRY(launch_set_scal(one(h->dev), S_COND, rate, static_cast<hipStream_t>(stream)));
  return MRA_OK;
}

int32_t mra_solve_set_jacobian(mra_solve h, int32_t jacobian) {
  if (!h) return MRA_E_ARG;
  if (jacobian != MRA_JAC_FROZEN && jacobian != MRA_JAC_EXACT) return MRA_E_ARG;
  if (h->cfg.kind != 0) return MRA_E_UNSUPPORTED;
  if (jacobian == MRA_JAC_EXACT && h->cfg.adapt) return MRA_E_UNSUPPORTED;
  drop_graphs_of(h);
  h->cfg.jac = jacobian;
  return MRA_OK;
}

int32_t mra_solve_destroy(mra_solve h) {
  if (!h) return MRA_E_ARG;
  if (h->riders > 0) return MRA_E_ARG;          // passive scalars still read its fields
  drop_graphs_of(h);
  if (h->partner) h->partner->riders -= 1;
  delete h;
  return MRA_OK;
}

// Phases of one exponential step, in launch order, for mra_step_profile.
enum StepPhase : int { P_RES_PI = 0, P_RES_FFT_ROWS, P_RES_FFT_COLS, P_RES_FFT_INV, P_RES_STENCIL, P_NORM0,
                       P_PI, P_FFT_ROWS, P_FFT_COLS, P_FFT_INV, P_JVP, P_GS, P_PHI1, P_UPDATE, P_REGRID_PI,
                       P_REGRID_FWD, P_REGRID_MASK, P_NPHASE };

int32_t mra_step_profile(mra_solve* solves, int32_t n, void* stream, double* ms_out, int32_t n_out) {
  if (!solves || n < 1 || n > kMaxBatch || !ms_out || n_out < P_NPHASE) return MRA_E_ARG;
  Batch b;
  std::memset(&b, 0, sizeof(b));
  b.n = n;
  for (int i = 0; i < n; ++i) {
    if (!solves[i]) return MRA_E_ARG;
    const LaunchCfg& c0 = solves[0]->cfg;
    const LaunchCfg& ci = solves[i]->cfg;
    if (ci.J != c0.J || ci.p != c0.p || ci.prec != c0.prec || ci.m != c0.m || ci.vb != c0.vb ||
        ci.tile != c0.tile || ci.kind != c0.kind || ci.integ != c0.integ || ci.jac != c0.jac ||
        ci.adapt != c0.adapt)
      return MRA_E_ARG;
    b.s[i] = solves[i]->dev;
  }
  const LaunchCfg& c = solves[0]->cfg;
  if (c.kind != 0 || c.integ != 0) return MRA_E_UNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<hipEvent_t> ev;
  std::vector<int> phase;   // phase of the launches between event i - 1 and event i
  auto mark = [&](int ph) -> hipError_t {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    ev.push_back(e);
    phase.push_back(ph);
    return hipEventRecord(e, st);
  };
  auto run = [&]() -> hipError_t {
    hipError_t e;
    const bool dbl = c.prec == 0;
    const int rsrc = dbl ? 0 : 3;
    if ((e = mark(-1)) != hipSuccess) return e;
    // the launches of enqueue_step (exponential integrator), phase by phase
    if ((e = launch_prolong(b, c, rsrc, 1, 0, 0, st)) != hipSuccess || (e = mark(P_RES_PI)) != hipSuccess) return e;
    for (int pass = 0; pass < 3; ++pass)
      if ((e = launch_poisson_pass(b, c, rsrc, pass, st)) != hipSuccess || (e = mark(P_RES_FFT_ROWS + pass)) != hipSuccess)
        return e;
    if ((e = launch_rhs(b, c, st)) != hipSuccess || (e = mark(P_RES_STENCIL)) != hipSuccess) return e;
    if ((e = launch_norm0(b, c, st)) != hipSuccess || (e = mark(P_NORM0)) != hipSuccess) return e;
    for (int j = 0; j < c.m; ++j) {
      if ((e = launch_prolong(b, c, 1, dbl, j == 0 ? 1 : 3, j, st)) != hipSuccess || (e = mark(P_PI)) != hipSuccess)
        return e;
      for (int pass = 0; pass < 3; ++pass)
        if ((e = launch_poisson_pass(b, c, 1, pass, st)) != hipSuccess || (e = mark(P_FFT_ROWS + pass)) != hipSuccess)
          return e;
      if ((e = launch_jvp(b, c, st)) != hipSuccess || (e = mark(P_JVP)) != hipSuccess) return e;
      if ((e = launch_arnoldi(b, c, j, st)) != hipSuccess || (e = mark(P_GS)) != hipSuccess) return e;
    }
    if ((e = launch_phi1(b, c, st)) != hipSuccess || (e = mark(P_PHI1)) != hipSuccess) return e;
    if ((e = launch_update(b, c, st)) != hipSuccess || (e = mark(P_UPDATE)) != hipSuccess) return e;
    if ((e = launch_prolong(b, c, 2, 1, 0, 0, st)) != hipSuccess || (e = mark(P_REGRID_PI)) != hipSuccess) return e;
    if ((e = launch_reset_max(b, st)) != hipSuccess || (e = launch_forward(b, c, 0, 0, st)) != hipSuccess ||
        (e = mark(P_REGRID_FWD)) != hipSuccess)
      return e;
    if ((e = launch_threshold(b, c, 1, st)) != hipSuccess || (e = launch_gather(b, c, st)) != hipSuccess ||
        (e = mark(P_REGRID_MASK)) != hipSuccess)
      return e;
    return hipEventSynchronize(ev.back());
  };
  hipError_t e = run();
  for (int i = 0; i < P_NPHASE; ++i) ms_out[i] = 0.0;
  if (e == hipSuccess) {
    for (size_t i = 1; i < ev.size(); ++i) {
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, ev[i - 1], ev[i])) != hipSuccess) break;
      ms_out[phase[i]] += ms;
    }
  }
  for (hipEvent_t x : ev) (void)hipEventDestroy(x);
  if (e != hipSuccess) return MRA_E_DEVICE;
  for (int i = 0; i < n; ++i) solves[i]->steps += 1;
  return MRA_OK;
}

int32_t mra_time_kernel(mra_solve* solves, int32_t n, int32_t which, int32_t reps, void* stream,
                        float* avg_ms) {
  if (!solves || n < 1 || n > kMaxBatch || !avg_ms || reps < 1) return MRA_E_ARG;
  if (which < 0 || which > 6) return MRA_E_ARG;
  Batch b;
  std::memset(&b, 0, sizeof(b));
  b.n = n;
  for (int i = 0; i < n; ++i) {
    if (!solves[i]) return MRA_E_ARG;
    const LaunchCfg& c0 = solves[0]->cfg;
    const LaunchCfg& ci = solves[i]->cfg;
    if (ci.J != c0.J || ci.p != c0.p || ci.prec != c0.prec || ci.m != c0.m || ci.vb != c0.vb || ci.tile != c0.tile ||
        ci.adapt != c0.adapt)
      return MRA_E_ARG;
    b.s[i] = solves[i]->dev;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const LaunchCfg& c = solves[0]->cfg;
  // the end of a step leaves the Arnoldi flag set; clear it so that the
  // timed Jacobian-vector stencil does its work (the next step resets it)
  MRA_TRY(launch_clear_done(b, st));
  hipEvent_t e0, e1;
  MRA_TRY(hipEventCreate(&e0));
  MRA_TRY(hipEventCreate(&e1));
  MRA_TRY(hipEventRecord(e0, st));
  for (int i = 0; i < reps; ++i) {
    hipError_t e = hipSuccess;
    switch (which) {
      case 0: e = launch_jvp(b, c, st); break;
      case 1: e = launch_poisson_pass(b, c, 1, 0, st); break;
      case 2: e = launch_poisson_pass(b, c, 1, 1, st); break;
      case 3: e = launch_poisson_pass(b, c, 1, 2, st); break;
      case 4: e = launch_prolong(b, c, 1, c.prec == 0, 0, 0, st); break;
      case 5: e = launch_forward(b, c, 0, 0, st); break;
      case 6: e = launch_rhs(b, c, st); break;
      default: e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return MRA_E_DEVICE;
  }
  MRA_TRY(hipEventRecord(e1, st));
  MRA_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  MRA_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = ms / reps;
  return MRA_OK;
}

}  // extern "C"
