"""MI355X (gfx950) wavelet-collocation vortex solver: Python binding.

A thin layer over the C-ABI of ``libmra.so`` (declared in include/mra.h):
PyTorch provides device memory and streams, every step of the method runs
in the library's HIP kernels.  The names follow the C entry points:

  mra_transform      DD forward / inverse transform, threshold, prolongation
  collocation_rhs    residual F(omega) or Jacobian-vector product at the active nodes
  Solve              one solve (arena, init, krylov_step, read)
  solve_batch        advance several solves with shared launches

Method: Walsh & Alam, "Fujiwhara interaction of tropical cyclone scale
vortices using a weighted residual collocation method" (arXiv:1604.08159),
Sections 2.3-2.5 (Smagorinsky closure, DD multiresolution, collocation) and
its Krylov-projected time integration.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import (FlowDesc, GridDesc, MraError, SolvePtrs, MRA_FORWARD, MRA_INVERSE, MRA_PROLONG,
                   MRA_FP64, MRA_FP32, MRA_MIXED, MRA_OK, MRA_E_NONFINITE, MRA_E_UNSUPPORTED, MRA_E_CAPACITY,
                   MRA_EXPONENTIAL,
                   MRA_THETA_NEWTON, MRA_MAX_NEWTON, MRA_JAC_FROZEN, MRA_JAC_EXACT, MRA_EVAL_DENSE,
                   MRA_EVAL_ADAPTED)

_LIB: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    """The loaded library; raises if it is missing (no fallback path exists)."""
    global _LIB
    if _LIB is None:
        _LIB = _lib.load()
    return _LIB


def _check(fn: str, st: int) -> None:
    if st != MRA_OK:
        raise MraError(fn, st, lib().mra_status_str(st).decode())


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def coarsest_level(p: int) -> int:
    return int(math.ceil(math.log2(2 * p)))


def grid_desc(J: int, p: int, eps: float, length: float = 2.0 * math.pi, adjacent_zone: int = 1,
              j0: Optional[int] = None) -> GridDesc:
    return GridDesc(J, coarsest_level(p) if j0 is None else j0, p, adjacent_zone, length, eps)


def flow_desc(nu0: float, cs: float = 0.17, s0: float = 0.0, mu: float = 0.0, smag_mode: int = 2) -> FlowDesc:
    return FlowDesc(nu0, cs, s0, mu, smag_mode, 0)


def bulk_dtype(prec: int) -> torch.dtype:
    return torch.float64 if prec == MRA_FP64 else torch.float32


def _alloc(nbytes: int, device) -> torch.Tensor:
    # 256-byte alignment: over-allocate and slice
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw[off: off + nbytes]


def transform_ws_bytes(g: GridDesc, prec: int) -> int:
    n = C.c_size_t()
    _check("mra_transform_ws_bytes", lib().mra_transform_ws_bytes(C.byref(g), prec, C.byref(n)))
    return n.value


def mra_transform(g: GridDesc, prec: int, direction: int, inp: torch.Tensor, out: torch.Tensor,
                  mask: Optional[torch.Tensor] = None, index_packed: Optional[torch.Tensor] = None,
                  index_fine: Optional[torch.Tensor] = None, n_active: Optional[torch.Tensor] = None,
                  ws: Optional[torch.Tensor] = None, stream=None) -> None:
    if ws is None:
        ws = _alloc(transform_ws_bytes(g, prec), inp.device)
    st = lib().mra_transform(C.byref(g), prec, direction, _ptr(inp), _ptr(out), _ptr(mask),
                             _ptr(index_packed), _ptr(index_fine), _ptr(n_active), _ptr(ws),
                             ws.numel(), _stream(stream))
    _check("mra_transform", st)


def mra_transform_noalloc(g: GridDesc, prec: int, direction: int, inp: torch.Tensor, out: torch.Tensor,
                          mask: Optional[torch.Tensor] = None, index_packed: Optional[torch.Tensor] = None,
                          index_fine: Optional[torch.Tensor] = None, n_active: Optional[torch.Tensor] = None,
                          stream=None) -> None:
    """mra_transform without a workspace argument: the library's own
    per-device workspace serves (grids up to J = 10; calls on one device must
    not overlap)."""
    st = lib().mra_transform_noalloc(C.byref(g), prec, direction, _ptr(inp), _ptr(out), _ptr(mask),
                                     _ptr(index_packed), _ptr(index_fine), _ptr(n_active), _stream(stream))
    _check("mra_transform_noalloc", st)


def rhs_ws_bytes(g: GridDesc, prec: int) -> int:
    n = C.c_size_t()
    _check("mra_rhs_ws_bytes", lib().mra_rhs_ws_bytes(C.byref(g), prec, C.byref(n)))
    return n.value


def collocation_rhs(g: GridDesc, f: FlowDesc, prec: int, mask: torch.Tensor, index_fine: torch.Tensor,
                    n_active: torch.Tensor, omega_active: torch.Tensor, v_active: Optional[torch.Tensor],
                    out_active: torch.Tensor, velocity: Optional[torch.Tensor] = None,
                    ws: Optional[torch.Tensor] = None, stream=None) -> None:
    if ws is None:
        ws = _alloc(rhs_ws_bytes(g, prec), omega_active.device)
    st = lib().collocation_rhs(C.byref(g), C.byref(f), prec, _ptr(mask), _ptr(index_fine), _ptr(n_active),
                               _ptr(omega_active), _ptr(v_active), _ptr(out_active), _ptr(velocity), _ptr(ws),
                               ws.numel(), _stream(stream))
    _check("collocation_rhs", st)


def collocation_rhs_adapted(g: GridDesc, f: FlowDesc, prec: int, mask: torch.Tensor, index_fine: torch.Tensor,
                            n_active: torch.Tensor, omega_active: torch.Tensor, v_active: Optional[torch.Tensor],
                            out_active: torch.Tensor, velocity: Optional[torch.Tensor] = None,
                            ws: Optional[torch.Tensor] = None, stream=None) -> None:
    """collocation_rhs with the level-adapted evaluation (derivatives at each
    active node on the stencils of its local level)."""
    if ws is None:
        ws = _alloc(rhs_ws_bytes(g, prec), omega_active.device)
    st = lib().collocation_rhs_adapted(C.byref(g), C.byref(f), prec, _ptr(mask), _ptr(index_fine), _ptr(n_active),
                                       _ptr(omega_active), _ptr(v_active), _ptr(out_active), _ptr(velocity),
                                       _ptr(ws), ws.numel(), _stream(stream))
    _check("collocation_rhs_adapted", st)


def solve_footprint(g: GridDesc, prec: int, m: int, capacity: int = 0) -> int:
    """Arena bytes of a solve whose active-length arrays hold `capacity`
    nodes (0: N^2)."""
    n = C.c_size_t()
    _check("mra_solve_footprint_cap", lib().mra_solve_footprint_cap(C.byref(g), prec, m, int(capacity), C.byref(n)))
    return n.value


def tune_set_tile(J: int, p: int, prec: int, tile: int) -> None:
    """Stencil tile edge (8, 16 or 32; 0: the default) that solves of
    (J, p, prec) created from now on take (mra_tune_set_tile)."""
    _check("mra_tune_set_tile", lib().mra_tune_set_tile(J, p, prec, tile))


def tune_get_tile(J: int, p: int, prec: int) -> int:
    t = C.c_int32()
    _check("mra_tune_get_tile", lib().mra_tune_get_tile(J, p, prec, C.byref(t)))
    return t.value


DIAG_KEYS = ("t", "energy", "enstrophy", "palinstrophy", "gamma", "max_abs", "n_active", "status")


class Solve:
    """One solve whose whole state lives in a torch-allocated device arena.

    capacity: active nodes the arena holds (0: N^2).  A solve whose active set
    outgrows it is moved to an arena `grow` times the needed count (capped at
    N^2) by step() and solve_batch(), and then runs on exactly as it would
    have with the larger capacity."""

    def __init__(self, g: GridDesc, f: FlowDesc, prec: int, m: int, dt: float, omega0: torch.Tensor,
                 stream=None, arena: Optional[torch.Tensor] = None, capacity: int = 0, grow: float = 1.5):
        N = 1 << g.J
        if omega0.dtype != torch.float64 or tuple(omega0.shape) != (N, N):
            raise ValueError("omega0 must be a float64 [N, N] device tensor")
        self.g, self.f, self.prec, self.m, self.dt = g, f, prec, m, dt
        self.N = N
        self.capacity = int(capacity) if capacity else N * N
        self.grow = float(grow)
        self.migrations = 0
        w0 = omega0.contiguous()
        while True:
            self.nbytes = solve_footprint(g, prec, m, self.capacity)
            self.arena = arena if arena is not None else _alloc(self.nbytes, omega0.device)
            h, need = C.c_void_p(), C.c_int64()
            st = lib().mra_solve_init_cap(C.byref(g), C.byref(f), prec, m, dt, _ptr(w0), self.capacity,
                                          _ptr(self.arena), self.arena.numel(), _stream(stream), C.byref(h),
                                          C.byref(need))
            if st != MRA_E_CAPACITY or arena is not None:
                break
            # the first active set is larger than the capacity: a larger arena
            self.capacity = min(N * N, max(need.value, int(math.ceil(need.value * self.grow))))
            self.migrations += 1
        _check("mra_solve_init_cap", st)
        self.handle = h

    def capacity_state(self, stream=None) -> Tuple[int, int, bool]:
        """(capacity, active or needed node count, frozen); synchronises."""
        cap, need, frozen = C.c_int64(), C.c_int64(), C.c_int32()
        _check("mra_solve_capacity", lib().mra_solve_capacity(self.handle, C.byref(cap), C.byref(need),
                                                               C.byref(frozen), _stream(stream)))
        return cap.value, need.value, bool(frozen.value)

    def migrate(self, capacity: int, stream=None) -> None:
        """Move the solve to a new arena of `capacity` active nodes
        (mra_solve_migrate); a frozen solve completes its regrid there."""
        nbytes = solve_footprint(self.g, self.prec, self.m, capacity)
        arena = _alloc(nbytes, self.arena.device)
        _check("mra_solve_migrate", lib().mra_solve_migrate(self.handle, int(capacity), _ptr(arena), arena.numel(),
                                                             _stream(stream)))
        self.arena, self.nbytes, self.capacity = arena, nbytes, int(capacity)
        self.migrations += 1

    def fit(self, stream=None) -> bool:
        """If the solve is frozen, move it to a larger arena; returns whether it was."""
        if self.capacity >= self.N * self.N:
            return False
        _, need, frozen = self.capacity_state(stream)
        if frozen:
            self.migrate(min(self.N * self.N, max(need, int(math.ceil(need * self.grow)))), stream)
        return frozen

    def steps_done(self, stream=None) -> int:
        return int(round(self.scalars(stream=stream)["steps"]))

    def step(self, nsteps: int = 1, stream=None) -> None:
        if self.capacity >= self.N * self.N:
            _check("krylov_step", lib().krylov_step(self.handle, nsteps, _stream(stream)))
            return
        target = self.steps_done(stream) + nsteps
        while True:
            done = self.steps_done(stream)
            if done >= target:
                return
            _check("krylov_step", lib().krylov_step(self.handle, target - done, _stream(stream)))
            self.fit(stream)

    def set_integrator(self, integrator: int, theta: float = 0.5, newton_iters: int = 2, stream=None) -> None:
        """Time scheme of later steps: MRA_EXPONENTIAL, or MRA_THETA_NEWTON
        (theta-scheme by newton_iters Newton-GMRES iterations)."""
        _check("mra_solve_set_integrator",
               lib().mra_solve_set_integrator(self.handle, integrator, float(theta), int(newton_iters),
                                              _stream(stream)))

    def set_evaluation(self, evaluation: int) -> None:
        """Evaluation of later steps: MRA_EVAL_DENSE or MRA_EVAL_ADAPTED."""
        _check("mra_solve_set_evaluation", lib().mra_solve_set_evaluation(self.handle, int(evaluation)))

    def set_jacobian(self, jacobian: int) -> None:
        """Jacobian of later steps' Krylov products: MRA_JAC_FROZEN or MRA_JAC_EXACT."""
        _check("mra_solve_set_jacobian", lib().mra_solve_set_jacobian(self.handle, int(jacobian)))

    def read(self, dense: bool = True, stream=None) -> Tuple[Optional[torch.Tensor], Dict[str, float]]:
        out = torch.empty((self.N, self.N), dtype=torch.float64, device=self.arena.device) if dense else None
        diag = (C.c_double * 8)()
        st = lib().mra_solve_read(self.handle, _ptr(out), diag, _stream(stream))
        if st not in (MRA_OK, MRA_E_NONFINITE, MRA_E_CAPACITY):
            _check("mra_solve_read", st)
        return out, dict(zip(DIAG_KEYS, list(diag)))

    def track(self, centres, stream=None):
        """One update of the vortex centres [(x, y), ...] (mra_solve_track)."""
        k = len(centres)
        buf = (C.c_double * (2 * k))(*[float(v) for c in centres for v in c])
        _check("mra_solve_track", lib().mra_solve_track(self.handle, k, buf, _stream(stream)))
        return [(buf[2 * i], buf[2 * i + 1]) for i in range(k)]

    def ptrs(self) -> SolvePtrs:
        p = SolvePtrs()
        _check("mra_solve_ptrs_get", lib().mra_solve_ptrs_get(self.handle, C.byref(p)))
        return p

    def _arena_view(self, addr: int, n: int, dtype: torch.dtype) -> torch.Tensor:
        """View of n elements at device address addr inside this solve's arena."""
        esz = torch.empty((), dtype=dtype).element_size()
        off = addr - self.arena.data_ptr()
        if off < 0 or off + n * esz > self.arena.numel():
            raise ValueError("address outside the arena")
        return self.arena[off: off + n * esz].view(dtype)

    def active_set(self) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor, torch.Tensor]:
        """(omega_M, mask, index_packed, index_fine) copied out of the arena."""
        p = self.ptrs()
        torch.cuda.synchronize(self.arena.device)
        na = int(self._arena_view(p.n_active, 1, torch.int64).item())
        nf = self.N * self.N
        return (self._arena_view(p.omega_active, na, torch.float64).clone(),
                self._arena_view(p.mask, nf, torch.uint8).clone(),
                self._arena_view(p.index_packed, na, torch.int32).clone(),
                self._arena_view(p.index_fine, na, torch.int32).clone())

    def scalars(self, stream=None) -> Dict[str, float]:
        """t, steps and the active-point residual evaluations counted on the
        device: after all work on the device, or, with `stream`, after the work
        enqueued on that stream (the solve's stream) only."""
        p = self.ptrs()
        view = self._arena_view(p.scalars, 16, torch.float64)
        if stream is None:
            torch.cuda.synchronize(self.arena.device)
            v = view.cpu().tolist()
        else:
            with torch.cuda.stream(stream):
                v = view.cpu().tolist()
        return {"t": v[4], "evals": v[5], "steps": v[6], "beta": v[0]}

    def close(self) -> None:
        if getattr(self, "handle", None):
            _check("mra_solve_destroy", lib().mra_solve_destroy(self.handle))   # refused while scalars ride on it
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ScalarSolve(Solve):
    """A passive scalar carried by the flow of a vorticity solve (mra_scalar_init):
    its own adaptive grid and Krylov state, the partner's velocity.  Keep the
    partner alive while this solve exists."""

    def __init__(self, partner: Solve, g: GridDesc, m: int, dt: float, r0: torch.Tensor, kappa0: float = 0.0,
                 eddy: bool = True, stream=None, arena: Optional[torch.Tensor] = None):
        N = 1 << g.J
        if r0.dtype != torch.float64 or tuple(r0.shape) != (N, N):
            raise ValueError("r0 must be a float64 [N, N] device tensor")
        self.g, self.f, self.prec, self.m, self.dt = g, partner.f, partner.prec, m, dt
        self.N = N
        self.partner = partner
        self.capacity, self.grow, self.migrations = N * N, 1.5, 0
        self.nbytes = solve_footprint(g, partner.prec, m)
        self.arena = arena if arena is not None else _alloc(self.nbytes, r0.device)
        h = C.c_void_p()
        st = lib().mra_scalar_init(partner.handle, C.byref(g), m, dt, kappa0, 1 if eddy else 0,
                                   _ptr(r0.contiguous()), _ptr(self.arena), self.arena.numel(), _stream(stream),
                                   C.byref(h))
        _check("mra_scalar_init", st)
        self.handle = h

    def set_condensation(self, rate: float, stream=None) -> None:
        """Vapor condensation at rate c (mra_scalar_set_condensation): the
        right-hand side gains -c r (r - 1) (2 r - 1); 0 turns it off."""
        _check("mra_scalar_set_condensation",
               lib().mra_scalar_set_condensation(self.handle, float(rate), _stream(stream)))


KERNELS = {"jvp": 0, "fft_rows": 1, "fft_cols": 2, "fft_rows_inv": 3, "prolong_finest": 4,
           "forward": 5, "rhs": 6}


def time_kernel(solves: Sequence[Solve], which: str, reps: int, stream=None) -> float:
    """Mean duration [ms] of one launch of a step kernel for this batch (HIP events)."""
    n = len(solves)
    hs = (C.c_void_p * n)(*[s.handle for s in solves])
    ms = C.c_float()
    _check("mra_time_kernel", lib().mra_time_kernel(hs, n, KERNELS[which], reps, _stream(stream), C.byref(ms)))
    return ms.value


STEP_PHASES = ("res_prolong", "res_fft_rows", "res_fft_cols", "res_fft_rows_inv", "res_stencil", "norm0",
               "prolong", "fft_rows", "fft_cols", "fft_rows_inv", "jvp", "gram_schmidt", "phi1", "update",
               "regrid_prolong", "regrid_forward", "regrid_mask")


def step_profile(solves: Sequence[Solve], stream=None) -> Dict[str, float]:
    """One step of the batch with a HIP event after every phase
    (mra_step_profile): GPU milliseconds per phase, summed over the step."""
    n = len(solves)
    hs = (C.c_void_p * n)(*[s.handle for s in solves])
    out = (C.c_double * len(STEP_PHASES))()
    _check("mra_step_profile", lib().mra_step_profile(hs, n, _stream(stream), out, len(STEP_PHASES)))
    return dict(zip(STEP_PHASES, list(out)))


def _solve_batch(solves: Sequence[Solve], nsteps: Sequence[int], stream=None) -> None:
    n = len(solves)
    hs = (C.c_void_p * n)(*[s.handle for s in solves])
    ns = (C.c_int32 * n)(*[int(k) for k in nsteps])
    _check("solve_batch", lib().solve_batch(hs, n, ns, _stream(stream)))


def solve_batch(solves: Sequence[Solve], nsteps: Sequence[int], stream=None, fit: bool = True) -> None:
    """Advance solves[i] by nsteps[i] steps in shared launches (solve_batch).
    Solves below full capacity that freeze on the way are moved to larger
    arenas and finish their steps (fit=False leaves that to the caller: the
    call then does not synchronise)."""
    small = [i for i, s in enumerate(solves) if s.capacity < s.N * s.N]
    if not fit or not small:
        _solve_batch(solves, nsteps, stream)
        return
    target = {i: solves[i].steps_done(stream) + int(nsteps[i]) for i in small}
    _solve_batch(solves, nsteps, stream)
    while True:
        rest = []
        for i in small:
            solves[i].fit(stream)
            k = target[i] - solves[i].steps_done(stream)
            if k > 0:
                rest.append((solves[i], k))
        if not rest:
            return
        _solve_batch([s for s, _ in rest], [k for _, k in rest], stream)
