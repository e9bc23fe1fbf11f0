"""Continuous batching of vortex solves on one GPU.

Host-side orchestration only: every step of every solve runs in the
library's kernels through solve_batch.  Requests (initial vortices, grid,
Reynolds number, step count) arrive over time; a request is admitted as soon
as its arena fits in the HBM budget (footprint from mra_solve_footprint_cap,
for a capacity of N^2 nodes or a set fraction of them) and stays resident --
active set, Krylov basis, dense work fields -- until its last step.  Resident solves of equal (J, p, m) form a group with a stream of
its own; a group advances in rounds of a few steps (one solve_batch call, so
its solves share every kernel launch and a captured step graph), and groups
run independently of each other: there is no barrier across groups.  The
host polls each group's completion event; when a round ends it retires the
group's finished solves (result read back, latency recorded, arena
released), admits the requests that now fit, and starts the group's next
round, so a small request never waits for a large group's round, and
requests that arrive while others run join as soon as memory allows.

Results do not depend on the mix: kernels and reductions are per solve, so a
solve gives bit-identical results alone and inside any batch.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import torch

from . import MRA_MIXED, Solve, flow_desc, grid_desc, solve_batch, solve_footprint


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds after the start of the run
    J: int
    p: int
    eps: float
    nu0: float
    cs: float
    m: int
    dt: float
    steps: int
    omega0: object                 # host FP64 [N][N] (numpy)


@dataclasses.dataclass
class Record:
    rid: int
    J: int
    steps: int
    arrival: float
    admitted: float = -1.0
    finished: float = -1.0
    evals: float = 0.0
    n_active: int = 0
    status: int = 0
    diag: Optional[Dict[str, float]] = None
    omega: Optional[torch.Tensor] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    """Admission by HBM footprint, resident state, batched rounds of steps."""

    def __init__(self, hbm_budget: int, prec: int = MRA_MIXED, round_steps: int = 20,
                 device: str = "cuda:0", keep_results: bool = False,
                 progress: Optional[Callable[[int, int, int], None]] = None,
                 capacity_fraction: Optional[float] = None):
        """capacity_fraction: size each solve's active-length arrays and Krylov
        basis for that fraction of its N^2 nodes (None: N^2).  A solve whose
        active set outgrows its capacity is moved to a larger arena when its
        round ends, and then continues exactly as with full capacity; the
        move may take the bytes in use above the budget (the solve cannot go
        on in its old arena), and admission then waits until they fall below
        it."""
        self.budget = int(hbm_budget)
        self.cap_frac = capacity_fraction
        self.peak_used = 0
        self.migrations = 0
        self.progress = progress          # called after each round: (done, resident, waiting)
        self.prec = prec
        self.round_steps = round_steps
        self.dev = torch.device(device)
        self.keep = keep_results
        self.streams: Dict[Tuple[int, int, int], torch.cuda.Stream] = {}
        self.used = 0
        self.live: Dict[int, Tuple[Solve, Request, Record, int]] = {}   # rid -> (solve, req, rec, steps done)

    def capacity(self, r: Request) -> int:
        if not self.cap_frac:
            return 0
        nf = 1 << (2 * r.J)
        return min(nf, max(4096, int(math.ceil(self.cap_frac * nf))))

    def footprint(self, r: Request) -> int:
        return solve_footprint(grid_desc(r.J, r.p, r.eps), self.prec, r.m, self.capacity(r))

    def _stream(self, r: Request) -> torch.cuda.Stream:
        key = (r.J, r.p, r.m)
        if key not in self.streams:
            self.streams[key] = torch.cuda.Stream(device=self.dev)
        return self.streams[key]

    def _admit(self, r: Request, rec: Record, now: float) -> None:
        st = self._stream(r)
        with torch.cuda.stream(st):
            # an asynchronous copy from pinned memory on the group's stream: the
            # host does not wait for a round of that group still in flight
            host = torch.from_numpy(r.omega0).pin_memory()
            w0 = host.to(self.dev, non_blocking=True)
            s = Solve(grid_desc(r.J, r.p, r.eps), flow_desc(r.nu0, r.cs), self.prec, r.m, r.dt, w0, stream=st,
                      capacity=self.capacity(r))
        s._staging = (host, w0)          # alive until the copy and the init have run
        self.used += s.nbytes
        self.peak_used = max(self.peak_used, self.used)
        rec.admitted = now
        self.live[r.rid] = (s, r, rec, 0)

    def _retire(self, rid: int, now: float) -> Record:
        s, r, rec, _ = self.live.pop(rid)
        st = self._stream(r)
        dense, diag = s.read(dense=self.keep, stream=st)
        rec.finished = now
        rec.diag = diag
        rec.n_active = int(diag["n_active"])
        rec.status = int(diag["status"])
        rec.evals = s.scalars(stream=st)["evals"]
        rec.omega = dense
        self.used -= s.nbytes
        s.close()
        return rec

    def _event(self):
        return torch.cuda.Event()

    def run(self, requests: Sequence[Request], realtime: bool = True) -> List[Record]:
        """Serve the requests (sorted by arrival); returns their records.  A
        request whose footprint alone exceeds the budget is rejected
        (status -1) without affecting the others.  realtime=False: arrival
        times only order the queue (a virtual clock advances with them)."""
        records: Dict[int, Record] = {r.rid: Record(r.rid, r.J, r.steps, r.arrival) for r in requests}
        done: List[Record] = []
        ok = []
        for r in requests:
            if self.footprint(r) > self.budget:
                rec = records[r.rid]
                rec.status, rec.admitted, rec.finished = -1, r.arrival, r.arrival
                done.append(rec)
            else:
                ok.append(r)
        pending = collections.deque(sorted(ok, key=lambda r: r.arrival))
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else None
        vclock = [0.0]
        now = (lambda: clock()) if realtime else (lambda: vclock[0])
        # per group: the round in flight, as (event, solve ids, steps)
        inflight: Dict[Tuple[int, int, int], Tuple[object, List[int], int]] = {}
        while pending or self.live:
            progressed = False
            # retire: every group whose round has ended
            for key in list(inflight):
                ev, rids, k = inflight[key]
                if not ev.query():
                    continue
                del inflight[key]
                progressed = True
                for i in rids:
                    s, r, rec, d = self.live[i]
                    if s.capacity < s.N * s.N:
                        # a solve that outgrew its capacity froze during the
                        # round: move it, and count the steps it really took
                        before = s.nbytes
                        if s.fit(stream=self.streams[key]):
                            self.migrations += 1
                            self.used += s.nbytes - before
                            self.peak_used = max(self.peak_used, self.used)
                        d = s.steps_done(stream=self.streams[key])
                    else:
                        d += k
                    self.live[i] = (s, r, rec, d)
                for i in [i for i in rids if self.live[i][3] >= self.live[i][1].steps]:
                    done.append(self._retire(i, now()))
            # admission: FIFO, while the head fits in the remaining budget
            while pending and (not realtime or pending[0].arrival <= now()):
                r = pending[0]
                if self.used + self.footprint(r) > self.budget and self.live:
                    break
                pending.popleft()
                if not realtime:
                    vclock[0] = max(vclock[0], r.arrival)
                self._admit(r, records[r.rid], now())
                progressed = True
            # launch: the next round of every idle group
            groups: Dict[Tuple[int, int, int], List[int]] = collections.defaultdict(list)
            for rid, (s, r, rec, k) in self.live.items():
                groups[(r.J, r.p, r.m)].append(rid)
            for key, rids in groups.items():
                if key in inflight:
                    continue
                k = min(self.round_steps, min(self.live[i][1].steps - self.live[i][3] for i in rids))
                st = self.streams[key]
                solve_batch([self.live[i][0] for i in rids], [k] * len(rids), stream=st, fit=False)
                ev = self._event()
                ev.record(st)
                inflight[key] = (ev, list(rids), k)
                progressed = True
            if self.progress and progressed:
                self.progress(len(done), len(self.live), len(pending))
            if not progressed:
                # nothing ended, arrived or started: wait a little for a round or an arrival
                if realtime or inflight:
                    time.sleep(0.0002)
        return done


def summarize(records: Sequence[Record], wall: float) -> Dict[str, float]:
    served = [r for r in records if r.status >= 0]
    lat = sorted(r.latency for r in served)

    def pct(q):
        if not lat:
            return float("nan")
        i = min(len(lat) - 1, max(0, int(round(q * (len(lat) - 1)))))
        return lat[i]

    by_size = {}
    for J in sorted({r.J for r in served}):
        lj = sorted(r.latency for r in served if r.J == J)
        q = lambda f: lj[min(len(lj) - 1, max(0, int(round(f * (len(lj) - 1)))))]
        by_size[str(1 << J)] = {"requests": len(lj), "p50_latency_s": q(0.50), "p99_latency_s": q(0.99)}
    return {"requests": len(records), "wall_s": wall, "solves_per_s": len(served) / wall if wall > 0 else 0.0,
            "p50_latency_s": pct(0.50), "p99_latency_s": pct(0.99), "max_latency_s": lat[-1] if lat else 0.0,
            "active_pt_evals_per_s": sum(r.evals for r in records) / wall if wall > 0 else 0.0,
            "failed": sum(1 for r in records if r.status > 0),
            "rejected": sum(1 for r in records if r.status < 0),
            "latency_by_finest_size": by_size}


def requests_from_problems(timed_problems, omega_fn) -> List[Request]:
    """Requests from (arrival, workloads.Problem) pairs; omega_fn(problem) -> host field."""
    out = []
    for i, (t, pb) in enumerate(timed_problems):
        out.append(Request(i, t, pb.J, pb.p, pb.eps, pb.nu0, pb.cs, pb.m, pb.dt, pb.steps, omega_fn(pb)))
    return out
