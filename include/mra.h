/*
 * mra.h -- C-ABI of the MI355X (gfx950) wavelet-collocation vortex library.
 *
 * The library evaluates, on one GPU, the hot path of the weighted-residual
 * collocation method of Walsh & Alam (arXiv:1604.08159) for the barotropic
 * vorticity-streamfunction equations on the periodic square [0, L)^2:
 *
 *   laplacian(psi) = -omega,  u = d psi/dy,  v = -d psi/dx,
 *   d omega/dt = -div(u omega) + eddy diffusion (Smagorinsky, eq. (5)).
 *
 * Grid: N = 2^J nodes per side, h = L/N, arrays f[y][x] row-major (x fastest).
 * Multiresolution (Section 2.4, eq. (6)): nested meshes G^{j0} .. G^J, the
 * order-2p Deslauriers-Dubuc (DD) prediction, details d = u - P(u|G^{l-1}),
 * an active set M of nodes whose detail is significant (plus an adjacent zone
 * and the coarsest mesh); the unknowns are the nodal values at M.
 * Derivatives (Section 2.5): collocation first derivative with the DD filter
 * phi'(n); the second derivative is the (2p+1)-point Lagrange rule.
 * Time step: exponential Rosenbrock-Euler in a Krylov subspace (the paper's
 * Krylov projection, abstract and Section 2.1).
 *
 * Packed pyramid layout (N*N entries): the 2^j0 x 2^j0 coarse values at
 * offset 0, then for l = j0+1..J three bands of 2^(l-1) x 2^(l-1) entries,
 * row-major [b][a], at offsets 4^(l-1) (X: node ((2a+1)s, 2bs)),
 * 2*4^(l-1) (Y: node (2as, (2b+1)s)) and 3*4^(l-1) (XY: ((2a+1)s, (2b+1)s)),
 * s = 2^(J-l).  The mask and index_packed use packed positions; index_fine
 * holds y*N + x of the same nodes, both ascending in packed order.
 *
 * Conventions
 *   - Every pointer argument named *_dev, and every array argument unless
 *     stated otherwise, is DEVICE memory owned by the caller.  The library
 *     never allocates or frees device memory; it keeps only small constant
 *     tables and the 5 MiB workspace of mra_transform_noalloc in module
 *     memory (set up by mra_init) and, per solve handle, a small host object
 *     plus captured HIP graphs.
 *   - `stream` is a hipStream_t (NULL = default stream).  Every call is
 *     asynchronous on it except mra_solve_read, which synchronises it.
 *   - Argument and size errors are returned before anything is launched.
 *     Device-side conditions (non-finite values) go to the solve's status
 *     word, read back by mra_solve_read.  No C++ exception crosses the ABI.
 *   - Sizes that change on the device (the active count N_a) live in device
 *     memory so that captured graphs stay valid.
 *   - Distinct solves on distinct streams are independent; calls that share
 *     a workspace or a solve must not overlap.
 */
#ifndef MRA_H
#define MRA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MRA_OK = 0,
  MRA_E_ARG = 1,          /* bad argument (null pointer, unknown enum)          */
  MRA_E_SIZE = 2,         /* grid, order, Krylov size or buffer size unsupported */
  MRA_E_NOMEM = 3,        /* arena / workspace smaller than required             */
  MRA_E_DEVICE = 4,       /* a HIP call failed                                   */
  MRA_E_NONFINITE = 5,    /* a non-finite value was met (status word only)       */
  MRA_E_UNSUPPORTED = 6,
  MRA_E_CAPACITY = 7      /* a regrid found more active nodes than the solve's
                             capacity (status word; see mra_solve_migrate)      */
};

/* Precision.  MRA_FP64: every field and sum in FP64.  MRA_MIXED: the bulk
 * fields of the Jacobian-vector products (Pi of the Arnoldi vectors, their
 * Poisson solve, the product stencil, and the base fields w~, u, v, nu_e they
 * read) are FP32; the residual F itself (its Pi, Poisson solve and stencil,
 * once per step), the Krylov basis and its sums, the Hessenberg exponential
 * or solve, the update and the regrid are FP64.  MRA_FP32 (solves): as
 * MIXED, with the Krylov basis stored in FP32 (its sums stay FP64). */
enum { MRA_FP64 = 0, MRA_FP32 = 1, MRA_MIXED = 2 };
enum { MRA_FORWARD = 1, MRA_INVERSE = -1, MRA_PROLONG = 2 };
enum { MRA_EXPONENTIAL = 0, MRA_THETA_NEWTON = 1 };   /* time integrator of a solve */
enum { MRA_JAC_FROZEN = 0, MRA_JAC_EXACT = 1 };        /* Jacobian of its Krylov products */
enum { MRA_EVAL_DENSE = 0, MRA_EVAL_ADAPTED = 1 };     /* evaluation of the residual / products */
#define MRA_MAX_NEWTON 8

/* Grid: J in [j0+1, 11]; p in {2, 3} (4- and 6-point DD); j0 must equal
 * ceil(log2(2p)) (2 for p = 2, 3 for p = 3); length > 0 is the side of the
 * periodic square; eps >= 0 the relative threshold (tau = eps * max|u|);
 * adjacent_zone 0/1. */
typedef struct {
  int32_t J, j0, p, adjacent_zone;
  double length, eps;
} mra_grid_desc;

/* Flow: nu0 >= 0 molecular/base viscosity; cs Smagorinsky constant; s0 the
 * a-priori |S| of smag_mode 1; mu >= 0 linear friction; smag_mode 0 (nu0
 * only), 1 (nu0 + (cs h)^2 s0) or 2 (nu0 + (cs h)^2 |S| from the resolved
 * strain).  Eq. (5) with Delta = h. */
typedef struct {
  double nu0, cs, s0, mu;
  int32_t smag_mode, reserved;
} mra_flow_desc;

typedef struct mra_solve_s* mra_solve;

/* Device pointers into a solve's arena (for inspection by tests/tools). */
typedef struct {
  double* omega_active;      /* [capacity] FP64, first N_a valid                */
  uint8_t* mask;             /* [N*N] packed layout, 1 = active                  */
  int32_t* index_packed;     /* [capacity], first N_a valid                      */
  int32_t* index_fine;       /* [capacity], first N_a valid                      */
  int64_t* n_active;         /* device scalar (0 while the solve is frozen)      */
  void* krylov_V;            /* [(m+1)][basis_stride] Arnoldi basis: double, or float for
                                precision MRA_FP32 (sums over it are FP64); after
                                a step rows 0 .. m_eff-1 hold the orthonormal
                                basis, the next row a work vector              */
  double* hessenberg;        /* [(m+1)][m] FP64                                  */
  double* scalars;           /* [16] FP64: [0] beta, [4] t,
                                [5] active-point residual evaluations so far
                                (sum over steps of (1 + m_eff) N_a), [6] steps */
  int32_t* control;          /* [16] int: [0] m_eff, [1] done, [2] status, [8] 1
                                while frozen, [9] the N_a a frozen regrid found  */
  int64_t capacity;          /* entries of the active-length arrays             */
  int64_t basis_stride;      /* elements from one basis vector to the next
                                (capacity plus a padding)                       */
} mra_solve_ptrs;

const char* mra_status_str(int32_t status);
int32_t mra_abi_version(void);

/* Set up the library's constant tables (FFT twiddles) on the CURRENT device.
 * Idempotent per device; called implicitly by the other entry points. */
int32_t mra_init(void);

/* ------------------------------------------------------------------------
 * mra_transform -- DD multiresolution transform (Section 2.4, eq. (6)).
 *
 * prec selects the element type of the dense / packed arrays: MRA_FP64 ->
 * double, MRA_FP32 or MRA_MIXED -> float.  Active values are always double.
 *
 * MRA_FORWARD: in = dense [N][N]; out = packed pyramid [N*N] (coarse values,
 *   then details d = u - P(u|G^{l-1}) of every level, the 2-D prediction
 *   being the tensor-product DD rule applied along y, then x).  If mask is
 *   non-NULL the active set is also built: tau = eps * max|in|,
 *   S = {non-coarse nodes with |d| >= tau}, M = G^{j0} + S + adjacent zone
 *   (nodes of G^{min(l+1,J)} within periodic Chebyshev distance 2^(J-l) of a
 *   node of S at level l); mask [N*N] (packed), index_packed / index_fine
 *   [N*N capacity] and *n_active (device int64) are written.  In FP64 the
 *   details are computed with one rounding per operation and no fused
 *   multiply-add, so they and the active set are reproducible bit for bit.
 * MRA_INVERSE: in = packed pyramid, out = dense: u = d + P(u|G^{l-1}),
 *   coarse to fine.
 * MRA_PROLONG (nodal inverse transform Pi): in = active values (double,
 *   n_active entries in index_fine order); mask and index_fine describe M;
 *   out = dense [N][N]: active nodes keep their value, an inactive node of
 *   level l gets the DD prediction from the final level-(l-1) values.
 *
 * ws: device workspace of at least mra_transform_ws_bytes bytes.
 * ------------------------------------------------------------------------ */
int32_t mra_transform_ws_bytes(const mra_grid_desc* g, int32_t prec, size_t* bytes);
int32_t mra_transform(const mra_grid_desc* g, int32_t prec, int32_t dir,
                      const void* in, void* out,
                      uint8_t* mask, int32_t* index_packed, int32_t* index_fine,
                      int64_t* n_active, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * mra_transform_noalloc -- mra_transform for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same arguments without the workspace, the same
 * kernels and the same results bit for bit.  The workspace is a
 * library-owned array in module memory of 5 MiB per device, held from the
 * first call on a device until the process ends; the call itself allocates
 * nothing (no hipMalloc, hipFree or allocating library routine).  Grids up to
 * J = 10 only: a larger J returns MRA_E_SIZE before anything is launched.
 * The array is shared by every call on a device and keeps the last call's
 * contents (each call initialises what it reads), so calls on one device
 * must not overlap: issue them on one stream, or order them by events or
 * synchronisation; calls that overlap race.  Other errors as mra_transform.
 * ------------------------------------------------------------------------ */
int32_t mra_transform_noalloc(const mra_grid_desc* g, int32_t prec, int32_t dir,
                              const void* in, void* out,
                              uint8_t* mask, int32_t* index_packed, int32_t* index_fine,
                              int64_t* n_active, void* stream);

/* ------------------------------------------------------------------------
 * collocation_rhs -- residual F(omega) or the Jacobian-vector product J v at
 * the active nodes (Sections 2.3 and 2.5; vorticity-streamfunction form):
 *
 *   w~ = Pi(omega), psi = -L^{-1} w~ (k = 0 mode dropped), u = D1_y psi,
 *   v = -D1_x psi (L and D1 are circulant: all three are applied as Fourier
 *   multipliers of w~), nu_e from eq. (5),
 *   F = -[D1_x(u w~) + D1_y(v w~)] + 1/2[L(nu_e w~) + nu_e L w~ - w~ L nu_e]
 *       - mu w~,
 *   J v (nu_e frozen at omega): with v~ = Pi(v), psi_v = -L^{-1} v~,
 *   -[D1_x(u_v w~ + u v~) + D1_y(v_v w~ + v v~)]
 *       + 1/2[L(nu_e v~) + nu_e L v~ - v~ L nu_e] - mu v~.
 *
 * mask / index_fine / n_active: the active set (as from mra_transform).
 * omega_active, v_active (NULL -> F), out_active: double [n_active].
 * vel_dense_or_null: if non-NULL receives the velocity of w~ as [2][N][N]
 *   (u then v; element type of prec), caller-owned.
 * prec: element type of the dense fields (FP64, or FP32 for FP32/MIXED).
 *   With FP32 fields the residual F is still evaluated in FP64 (its Pi,
 *   Poisson solve and stencil) and the FP32 base fields of the product are
 *   its values rounded; only J v runs in FP32.
 * ------------------------------------------------------------------------ */
int32_t mra_rhs_ws_bytes(const mra_grid_desc* g, int32_t prec, size_t* bytes);
int32_t collocation_rhs(const mra_grid_desc* g, const mra_flow_desc* f, int32_t prec,
                        const uint8_t* mask, const int32_t* index_fine,
                        const int64_t* n_active, const double* omega_active,
                        const double* v_active, double* out_active,
                        void* vel_dense_or_null, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * collocation_rhs_adapted -- collocation_rhs with the level-adapted
 * evaluation of the adaptive wavelet collocation method that Section 2.1
 * cites: the derivatives at an active node x take the stencils of its local
 * level lambda(x), the finest level l of an active node of level l within
 * periodic Chebyshev distance (2p - 2) 2^(J - l) of x (at least the level of x
 * itself).  The flux divergence and the three Laplacians of the conservative
 * diffusion at x use the D1 and L stencils with node spacing 2^(J - lambda)
 * (step 2^(J - lambda) h) on the dense w~ = Pi(omega) (values of the
 * interpolant at inactive stencil points), the velocity of the spectral
 * Poisson solve and the eddy viscosity; where every node is active this is
 * collocation_rhs.  The stencil work is one thread per active node; Pi and
 * the Poisson solve stay dense.  Same arguments, workspace and errors as
 * collocation_rhs (mra_rhs_ws_bytes covers both).
 * ------------------------------------------------------------------------ */
int32_t collocation_rhs_adapted(const mra_grid_desc* g, const mra_flow_desc* f, int32_t prec,
                                const uint8_t* mask, const int32_t* index_fine,
                                const int64_t* n_active, const double* omega_active,
                                const double* v_active, double* out_active,
                                void* vel_dense_or_null, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Solves.  A solve keeps its whole state in a caller-owned device arena of
 * mra_solve_footprint bytes: active values (FP64), active set, Krylov basis
 * V [(m+1) x N*N] (FP64, or FP32 for MRA_FP32), Hessenberg matrix,
 * dense work fields and FFT spectra.  1 <= m <= 47.
 *
 * mra_solve_init: omega0_dense (device, double [N][N]) is transformed and
 *   thresholded to the first active set; the host handle is written to *out.
 *   The solve's capacity is N*N.
 * krylov_step: nsteps exponential Rosenbrock-Euler steps
 *   omega_M <- omega_M + dt beta V_m phi_1(dt H_m) e_1, with Arnoldi
 *   (classical Gram-Schmidt with a second pass for every column, delayed to
 *   the next column's reads of the basis (DCGS2); happy breakdown
 *   h_{j+1,j} <= 1e-13 ||A v_j||, beta = 0 -> no update) and
 *   an FP64 regrid (Pi, forward transform, threshold, gather) after each
 *   step.  The first call captures one step into a HIP graph on `stream`;
 *   later calls replay it.
 * solve_batch: advances solves[i] by nsteps[i] steps; solves of equal
 *   (J, p, precision, m, integrator, Newton iterations, Jacobian, tile) share
 *   every kernel launch (up to 64 solves per launch).  On a non-default
 *   stream one step of the whole call, whatever its grid sizes, is one
 *   captured HIP graph launch: each group of equal configuration is a branch
 *   of the graph, the branches run concurrently, and passive scalars' branches
 *   follow their partners'.  A graph is captured once per composition of the
 *   call (which solves, in which groups) and replayed while it stays the
 *   same.  Results are bit for bit those of krylov_step on each solve alone.
 * mra_solve_read: synchronises `stream`; omega_dense_out (device double
 *   [N][N], may be NULL) receives Pi(omega_M); diag_out (HOST double[8],
 *   may be NULL) receives t, energy, enstrophy, palinstrophy, circulation,
 *   max|omega|, N_a, status (Sections 3.3 and 3.4).
 * ------------------------------------------------------------------------ */
int32_t mra_solve_footprint(const mra_grid_desc* g, int32_t prec, int32_t m, size_t* bytes);
int32_t mra_solve_init(const mra_grid_desc* g, const mra_flow_desc* f, int32_t prec,
                       int32_t m, double dt, const double* omega0_dense,
                       void* arena, size_t arena_bytes, void* stream, mra_solve* out);
int32_t krylov_step(mra_solve s, int32_t nsteps, void* stream);

/* ------------------------------------------------------------------------
 * Capacity.  The active set of the adaptive grid (Section 2.4) is usually a
 * small part of the N*N nodes; a solve can size its active values, index
 * lists and Krylov basis for `capacity` active nodes instead of N*N (the
 * node-indexed fields stay N*N), so that an arena holds what the active set
 * needs.  capacity 0 means N*N; otherwise 2^(2 j0) <= capacity <= N*N, else
 * MRA_E_SIZE.
 *
 * mra_solve_footprint_cap / mra_solve_init_cap: as mra_solve_footprint and
 *   mra_solve_init, for that capacity.  Below N*N, mra_solve_init_cap
 *   synchronises `stream` and checks the first active set: when it exceeds
 *   the capacity no handle is made, *needed (if not NULL) receives its size
 *   and the call returns MRA_E_CAPACITY.
 * When a later regrid finds more active nodes than the capacity, nothing
 *   beyond it is written: the solve is frozen.  Its state
 *   stays omega on the previous active set, advanced by the step that
 *   overflowed; its status word becomes MRA_E_CAPACITY (mra_solve_read
 *   returns it) and n_active reads 0; later steps leave it unchanged and do
 *   not advance t.
 * mra_solve_capacity: the capacity, the active-node count (for a frozen
 *   solve, the count the regrid needed) and the frozen flag.  Synchronises
 *   `stream`.
 * mra_solve_migrate: moves the solve into a new caller-owned arena of
 *   mra_solve_footprint_cap(capacity) bytes.  A frozen solve completes its
 *   pending regrid there (the same FP64 field, so the run continues exactly as
 *   with a larger capacity); any other solve is copied as it is.  The handle
 *   stays valid and now lives in the new arena, which the caller keeps; the
 *   old arena is no longer read once the call returns (it synchronises
 *   `stream`).  The solve's captured graphs are dropped.  Errors: MRA_E_ARG;
 *   MRA_E_SIZE when the capacity is out of range or below the active (or
 *   needed) count; MRA_E_NOMEM for a small arena; MRA_E_UNSUPPORTED for a
 *   passive scalar or a solve that carries one (mra_scalar_init also refuses
 *   a partner whose capacity is below N*N).
 * ------------------------------------------------------------------------ */
int32_t mra_solve_footprint_cap(const mra_grid_desc* g, int32_t prec, int32_t m, int64_t capacity,
                                size_t* bytes);
int32_t mra_solve_init_cap(const mra_grid_desc* g, const mra_flow_desc* f, int32_t prec, int32_t m,
                           double dt, const double* omega0_dense, int64_t capacity, void* arena,
                           size_t arena_bytes, void* stream, mra_solve* out, int64_t* needed);
int32_t mra_solve_capacity(mra_solve s, int64_t* capacity, int64_t* needed, int32_t* frozen, void* stream);
int32_t mra_solve_migrate(mra_solve s, int64_t capacity, void* arena, size_t arena_bytes, void* stream);

/* ------------------------------------------------------------------------
 * mra_solve_track -- vortex centres for the separation b(t) of Section 3.2.
 * centres: HOST double [k][2] (x, y), 1 <= k <= 4, the previous centres on
 * input and the updated ones on output.  Each finest node of Pi(omega_M) is
 * given to the nearest previous centre (periodic distance, ties to the lower
 * index); a centre moves by the mean periodic displacement of its nodes
 * weighted by max(omega, 0), and stays if that weight is zero.  One call is one
 * update: track a run by calling it after every step (or every few steps,
 * while the centres move much less than their spacing).  Synchronises
 * `stream`.
 * ------------------------------------------------------------------------ */
int32_t mra_solve_track(mra_solve s, int32_t k, double* centres, void* stream);

/* ------------------------------------------------------------------------
 * mra_scalar_init -- a passive scalar (the water vapor mixing ratio of
 * Section 3.6: eq. (3) with only a diffusion term) carried by the flow of the
 * vorticity solve `partner`:
 *
 *   dr/dt = -[D1_x(u r~) + D1_y(v r~)]
 *           + 1/2 [L(kappa r~) + kappa L r~ - r~ L kappa],   r~ = Pi(r),
 *
 * on its own adaptive grid (g: same J and p as the partner, its own eps) with
 * the same exponential step (the operator is linear in r) and FP64 regrid.
 * kappa = the partner's nu_e (eddy != 0) or the constant kappa0 >= 0.
 * Coupling is first-order splitting: the scalar's step k uses u, v (and
 * nu_e) of the partner's step k, i.e. of the vorticity at the start of that
 * step.  So a scalar step must follow its partner's step and precede the
 * next: krylov_step on a scalar takes nsteps = 1 right after one partner step
 * (else MRA_E_ARG); solve_batch orders every step itself when the partner is
 * in the same call.  Precision follows the partner; the arena is
 * mra_solve_footprint(g, precision, m) bytes.  The partner must outlive the
 * scalar: mra_solve_destroy refuses (MRA_E_ARG) a solve that still carries
 * scalars, so destroy scalars first.  r0_dense: device double [N][N].
 * mra_solve_read on a scalar returns its field and its mass as diag[4].
 * ------------------------------------------------------------------------ */
int32_t mra_scalar_init(mra_solve partner, const mra_grid_desc* g, int32_t m, double dt, double kappa0,
                        int32_t eddy, const double* r0_dense, void* arena, size_t arena_bytes,
                        void* stream, mra_solve* out);

/* ------------------------------------------------------------------------
 * Vapor condensation (Section 2.6, the moving air-vapor interface).  The
 * loss of vapor there is the variational derivative of the functional
 * int 1/2 r^2 (r - 1)^2 + D_v |grad r|^2, read as its gradient flow (the
 * sign under which a vapor patch shrinks, as the section's experiment
 * describes).  mra_scalar_set_condensation sets the rate c >= 0 of the
 * reaction part: the scalar's right-hand side gains -c f'(r) at every active
 * node, f'(r) = r (r - 1) (2 r - 1), and its Krylov products the
 * linearisation -c f''(r_n) v, f''(r) = 6 r^2 - 6 r + 1, at the state r_n of
 * the step's start (exponential Rosenbrock-Euler), both in FP64.  The
 * section's functional has c = 1; its gradient term is the scalar's
 * diffusion with the constant kappa0 = 2 D_v (eddy = 0).  c = 0 (the default)
 * is pure transport.  The rate is written in stream order on `stream`, so
 * steps enqueued after the call use it.  Errors: MRA_E_ARG for a null handle
 * or a negative or non-finite rate; MRA_E_UNSUPPORTED for a vorticity solve.
 * ------------------------------------------------------------------------ */
int32_t mra_scalar_set_condensation(mra_solve s, double rate, void* stream);

/* ------------------------------------------------------------------------
 * Tile autotuning.  The stencil kernels (residual, Jacobian-vector products,
 * scalar transport) work on square tiles of the finest grid staged in LDS;
 * the edge trades halo re-reads (larger tiles read fewer halo nodes) against
 * LDS per block (smaller tiles fit more blocks per CU).  By default it is 32,
 * 16 for FP64 with the 6-point rule, never more than N.
 * mra_tune_set_tile sets the edge (8, 16 or 32) that solves and residual
 * workspaces laid out from now on take for (J, p, precision); tile 0 restores
 * the default.  A solve keeps the tile it was created with, and solve_batch
 * groups solves by tile, so solves of either tile can share a call.
 * Errors: MRA_E_ARG for J outside 3..11, p outside {2, 3}, an unknown
 * precision, a tile other than 0, 8, 16, 32, a tile larger than N, or the
 * 32-tile of FP64 with the 6-point rule.  mra_tune_get_tile writes the edge
 * a new solve of (J, p, precision) would take.  The table is process-wide;
 * the Python autotuner (paper_1604_08159_amd/autotune.py) times the
 * candidates on the GPU and keeps the choices in a JSON cache.
 * ------------------------------------------------------------------------ */
int32_t mra_tune_set_tile(int32_t J, int32_t p, int32_t prec, int32_t tile);
int32_t mra_tune_get_tile(int32_t J, int32_t p, int32_t prec, int32_t* tile);
int32_t solve_batch(mra_solve* solves, int32_t n, const int32_t* nsteps, void* stream);
int32_t mra_solve_read(mra_solve s, double* omega_dense_out, double* diag_out, void* stream);
int32_t mra_solve_ptrs_get(mra_solve s, mra_solve_ptrs* out);
int32_t mra_solve_destroy(mra_solve s);

/* ------------------------------------------------------------------------
 * mra_solve_set_integrator -- the time scheme of later steps of a vorticity
 * solve.  Section 2.1 places the method among Newton-Krylov solvers of the
 * collocation system; besides the default exponential step
 * (MRA_EXPONENTIAL) a solve can take the implicit theta-scheme
 *
 *   G(w) = w - w_n - dt [theta F(w) + (1 - theta) F(w_n)] = 0
 *
 * on the active set of the step's start (MRA_THETA_NEWTON; theta in [0, 1]:
 * 1/2 Crank-Nicolson, 1 backward Euler, 0 explicit Euler), solved by
 * newton_iters (1..MRA_MAX_NEWTON) Newton iterations from w_0 = w_n:
 * (I - theta dt J(w_k)) d = -G(w_k), w_{k+1} = w_k + d, with J the Jacobian at
 * eddy viscosity frozen at w_k (the exponential step's operator) and each
 * linear system solved by one GMRES(m) cycle from a zero guess: the Arnoldi
 * process of J from -G (the same Gram-Schmidt and breakdown rule), then the least-squares
 * problem on I~ - theta dt H (Givens rotations).  Each step ends with the
 * FP64 regrid.  No extra arena memory.  theta and newton_iters are ignored for
 * MRA_EXPONENTIAL.  Takes effect for steps enqueued after the call (theta is
 * written on `stream`); drops the captured graphs that launch the solve.
 * Errors: MRA_E_ARG (null handle, unknown integrator, theta or newton_iters out
 * of range); MRA_E_UNSUPPORTED on a passive scalar, or for MRA_THETA_NEWTON
 * while a passive scalar rides on the solve (its coupling reads the flow at
 * the start of the partner's step, which Newton iterations overwrite);
 * mra_scalar_init likewise refuses a partner with MRA_THETA_NEWTON.
 * ------------------------------------------------------------------------ */
int32_t mra_solve_set_integrator(mra_solve s, int32_t integrator, double theta, int32_t newton_iters,
                                 void* stream);

/* ------------------------------------------------------------------------
 * mra_solve_set_jacobian -- the Jacobian J in the Krylov products of later
 * steps of a vorticity solve (either integrator).  MRA_JAC_FROZEN (default):
 * eddy viscosity frozen at the linearisation point.  MRA_JAC_EXACT: the
 * viscosity of eq. (5) is linearised too, adding
 *
 *   1/2 [L(nu' w~) + nu' L w~ - w~ L nu'],
 *   nu' = (Cs h)^2 2 (S11 S11' + S22 S22' + 2 S12 S12') / |S|,
 *
 * with S the strain of the base velocity and S' that of (u_v, v_v); nu' = 0
 * where |S| = 0 (the numerator vanishes there too; |nu'| <= (Cs h)^2 |S'|).
 * Only the local-strain model (smag_mode 2) depends on omega; for the other
 * modes both choices give the same products.  With it the exponential step is
 * second order in dt and the theta-scheme's Newton iteration is Newton's
 * method proper.  Each product also evaluates nu' on the tiles around the
 * active ones (one more stencil pass, no extra arena memory).  Drops the
 * captured graphs that launch the solve.  Errors: MRA_E_ARG (null handle,
 * unknown value); MRA_E_UNSUPPORTED on a passive scalar (its operator is
 * linear).
 * ------------------------------------------------------------------------ */
int32_t mra_solve_set_jacobian(mra_solve s, int32_t jacobian);

/* ------------------------------------------------------------------------
 * mra_solve_set_evaluation -- how later steps of a vorticity solve evaluate
 * the residual and the Krylov products: MRA_EVAL_DENSE (default: the stencils
 * of the finest level at every node, Section 2.5) or MRA_EVAL_ADAPTED (the
 * level-adapted evaluation of collocation_rhs_adapted; the local levels are
 * taken once per step from the step's active set).  Drops the captured graphs
 * that launch the solve.  Errors: MRA_E_ARG (null handle, unknown value);
 * MRA_E_UNSUPPORTED on a passive scalar, with the theta-scheme or with the
 * exact Jacobian (mra_solve_set_integrator and mra_solve_set_jacobian refuse
 * those in turn on an adapted solve).
 * ------------------------------------------------------------------------ */
int32_t mra_solve_set_evaluation(mra_solve s, int32_t evaluation);

/* Profiling hook: times `reps` back-to-back launches of one kernel of the
 * step, launched exactly as the step launches it for the batch `solves`
 * (n solves of equal J, p, precision and m): 0 Jacobian-vector stencil,
 * 1/2/3 Poisson FFT passes (rows, columns, inverse rows), 4 prolongation of
 * the finest level, 5 forward transform (FP64 regrid), 6 residual stencil.
 * HIP events on `stream`; *avg_ms receives the mean launch duration.  Only
 * work buffers are overwritten: call it between steps. */
int32_t mra_time_kernel(mra_solve* solves, int32_t n, int32_t which, int32_t reps, void* stream,
                        float* avg_ms);

/* Profiling hook: advances the batch `solves` (n solves of one launch
 * configuration, exponential integrator, vorticity solves) by ONE step with
 * the launches of krylov_step / solve_batch, issued directly (not from a
 * graph) with a HIP event on `stream` after every phase, and writes the GPU
 * time of each phase, summed over the step, to ms_out[0 .. 16]: the
 * residual's Pi, its three Poisson passes (rows, columns, inverse rows) and
 * its stencil; ||F||; the m products' Pi, their three Poisson passes and their
 * stencil; the m Gram-Schmidt columns; phi_1; the update; the regrid's Pi, its
 * forward transform, and its threshold, compaction and gather.  n_out >= 17.
 * Synchronises `stream`.  Errors: MRA_E_ARG (bad handles, mixed
 * configurations, n_out too small), MRA_E_UNSUPPORTED (passive scalars, the
 * theta-scheme). */
int32_t mra_step_profile(mra_solve* solves, int32_t n, void* stream, double* ms_out, int32_t n_out);

#ifdef __cplusplus
}
#endif
#endif /* MRA_H */
