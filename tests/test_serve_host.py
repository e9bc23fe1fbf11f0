"""Host logic of the continuous-batching server without a GPU: the solve, the
batched step and the streams are replaced by fakes that count steps, so the
admission by footprint, FIFO order, rejection of oversized requests, the
exact step count of every solve, the round size and the latency summary are
checked on the CPU (virtual clock)."""
import contextlib

import numpy as np
import pytest

from paper_1604_08159_amd import serve


class FakeSolve:
    live = 0
    peak = 0
    bytes_live = 0
    peak_bytes = 0

    def __init__(self, g, f, prec, m, dt, w0, stream=None, capacity=0):
        self.J, self.m = g.J, m
        self.N = 1 << g.J
        self.capacity = self.N * self.N
        self.nbytes = FOOTPRINT[g.J]
        self.steps = 0
        FakeSolve.live += 1
        FakeSolve.peak = max(FakeSolve.peak, FakeSolve.live)
        FakeSolve.bytes_live += self.nbytes
        FakeSolve.peak_bytes = max(FakeSolve.peak_bytes, FakeSolve.bytes_live)

    def read(self, dense=True, stream=None):
        return None, {"n_active": 10.0, "status": 0.0}

    def scalars(self, stream=None):
        return {"evals": 21.0 * 10 * self.steps}

    def close(self):
        FakeSolve.live -= 1
        FakeSolve.bytes_live -= self.nbytes


FOOTPRINT = {6: 100, 7: 400, 8: 1600}
BATCHES = []


def fake_solve_batch(solves, nsteps, stream=None, fit=True):
    assert len({s.J for s in solves}) == 1            # one launch configuration per batch
    BATCHES.append((solves[0].J, len(solves), nsteps[0]))
    for s, k in zip(solves, nsteps):
        s.steps += k


class FakeStream:
    def synchronize(self):
        pass


class FakeEvent:
    """A round's completion event: the fake batch has run when it is recorded."""

    def record(self, stream=None):
        pass

    def query(self):
        return True


@pytest.fixture
def fakes(monkeypatch):
    FakeSolve.live = FakeSolve.peak = FakeSolve.bytes_live = FakeSolve.peak_bytes = 0
    BATCHES.clear()
    monkeypatch.setattr(serve, "Solve", FakeSolve)
    monkeypatch.setattr(serve, "solve_batch", fake_solve_batch)
    monkeypatch.setattr(serve, "solve_footprint", lambda g, prec, m, capacity=0: FOOTPRINT[g.J])
    monkeypatch.setattr(serve.torch.cuda, "Stream", lambda device=None: FakeStream())
    monkeypatch.setattr(serve.torch.cuda, "stream", lambda st: contextlib.nullcontext())
    monkeypatch.setattr(serve.torch, "from_numpy", lambda a: a)          # host arrays stay put
    monkeypatch.setattr(serve.Server, "_event", lambda self: FakeEvent())
    yield


class _Host(np.ndarray):
    def to(self, *a, **k):
        return self

    def pin_memory(self):
        return self


def _req(rid, arrival, J, steps):
    w = np.zeros((1 << J, 1 << J)).view(_Host)
    return serve.Request(rid, arrival, J, 2, 1e-4, 1e-4, 0.17, 20, 0.01, steps, w)


def test_admission_rounds_and_step_counts(fakes):
    reqs = [_req(0, 0.0, 6, 45), _req(1, 0.1, 8, 30), _req(2, 0.2, 7, 10), _req(3, 0.3, 6, 20),
            _req(4, 0.4, 8, 5)]
    srv = serve.Server(hbm_budget=2000, round_steps=20, device="cpu")
    recs = {r.rid: r for r in srv.run(reqs, realtime=False)}
    assert sorted(recs) == [0, 1, 2, 3, 4]
    assert all(r.status == 0 for r in recs.values())
    # every solve ran exactly its steps, in rounds of at most 20
    for J, n, k in BATCHES:
        assert 1 <= k <= 20
    assert all(recs[r.rid].evals == 21.0 * 10 * r.steps for r in reqs)
    # the budget (2000) is never exceeded: the two 1600-byte solves never coexist,
    # so request 4 (J = 8) waits for request 1, and every arena is released
    assert FakeSolve.peak_bytes <= 2000 and FakeSolve.live == 0
    assert recs[4].admitted >= recs[1].finished
    for rec in recs.values():
        assert rec.admitted >= rec.arrival and rec.finished >= rec.admitted


def test_oversized_request_is_rejected_alone(fakes):
    reqs = [_req(0, 0.0, 8, 10), _req(1, 0.0, 6, 10)]
    srv = serve.Server(hbm_budget=1000, round_steps=20, device="cpu")
    recs = {r.rid: r for r in srv.run(reqs, realtime=False)}
    assert recs[0].status == -1 and recs[1].status == 0
    s = serve.summarize(list(recs.values()), 1.0)
    assert s["rejected"] == 1 and s["failed"] == 0 and s["requests"] == 2


def test_budget_limits_residency(fakes):
    reqs = [_req(i, 0.0, 7, 40) for i in range(6)]          # 400 bytes each
    srv = serve.Server(hbm_budget=1000, round_steps=20, device="cpu")
    srv.run(reqs, realtime=False)
    assert FakeSolve.peak == 2                              # 2 x 400 <= 1000 < 3 x 400


def test_summary_percentiles():
    recs = []
    for i, lat in enumerate([1.0, 2.0, 3.0, 4.0, 10.0]):
        r = serve.Record(i, 6, 10, 0.0, admitted=0.0, finished=lat, evals=5.0)
        recs.append(r)
    s = serve.summarize(recs, 2.0)
    assert s["p50_latency_s"] == 3.0 and s["p99_latency_s"] == 10.0 and s["max_latency_s"] == 10.0
    assert s["solves_per_s"] == 2.5 and s["active_pt_evals_per_s"] == 12.5


def test_groups_advance_without_a_barrier(fakes, monkeypatch):
    """A large group's round still in flight does not hold a small group
    back: the small request runs all its rounds and is retired first, and a
    request arriving meanwhile (queued behind the budget) is admitted as soon
    as the small one's arena is released."""
    class SlowEvent(FakeEvent):
        def __init__(self, slow):
            self.slow, self.left = slow, 40 if slow else 0

        def query(self):
            if self.left > 0:
                self.left -= 1
                return False
            return True

    srv = serve.Server(hbm_budget=1700, round_steps=20, device="cpu")
    # the event recorded after a J = 8 round (the last batch launched) takes 40 polls
    monkeypatch.setattr(srv, "_event", lambda: SlowEvent(BATCHES[-1][0] == 8))
    reqs = [_req(0, 0.0, 8, 20), _req(1, 0.0, 6, 60), _req(2, 0.0, 6, 20)]
    recs = srv.run(reqs, realtime=False)
    order = [r.rid for r in recs]
    assert order.index(1) < order.index(0) and order.index(2) < order.index(0)
    # the J = 6 rounds (3 for request 1, 1 for request 2) ran while the J = 8 round was in flight
    j6 = [b for b in BATCHES if b[0] == 6]
    assert sum(k for _, n, k in j6 if n >= 1) >= 60 and BATCHES.index((8, 1, 20)) < BATCHES.index(j6[-1])
    assert all(r.status == 0 for r in recs) and FakeSolve.live == 0


def test_capacity_sized_solves_refit_and_finish(fakes, monkeypatch):
    """With capacity_fraction the server admits by the smaller footprint; a
    solve that outgrows its capacity freezes partway through a round (fewer
    steps done than the round asked for), is moved to a larger arena when the
    round ends (bytes in use updated, migration counted), and still runs
    exactly its steps."""
    class CapSolve(FakeSolve):
        def __init__(self, g, f, prec, m, dt, w0, stream=None, capacity=0):
            super().__init__(g, f, prec, m, dt, w0, stream)
            self.capacity = capacity or self.N * self.N
            self.nbytes_full = self.nbytes
            FakeSolve.bytes_live -= self.nbytes
            self.nbytes = self.nbytes // 4 if self.capacity < self.N * self.N else self.nbytes
            FakeSolve.bytes_live += self.nbytes
            self.freeze_at = 7 if self.J == 7 else None      # the J = 7 solves outgrow their capacity
            self.frozen = False

        def fit(self, stream=None):
            if not self.frozen:
                return False
            FakeSolve.bytes_live += self.nbytes_full - self.nbytes
            FakeSolve.peak_bytes = max(FakeSolve.peak_bytes, FakeSolve.bytes_live)
            self.nbytes, self.capacity, self.frozen, self.freeze_at = self.nbytes_full, self.N * self.N, False, None
            return True

        def steps_done(self, stream=None):
            return self.steps

    def cap_batch(solves, nsteps, stream=None, fit=True):
        assert not fit                                     # the server refits at the end of a round
        BATCHES.append((solves[0].J, len(solves), nsteps[0]))
        for s, k in zip(solves, nsteps):
            if s.frozen:
                continue
            if s.freeze_at is not None and s.steps + k > s.freeze_at:
                s.steps, s.frozen = s.freeze_at, True
            else:
                s.steps += k

    monkeypatch.setattr(serve, "Solve", CapSolve)
    monkeypatch.setattr(serve, "solve_batch", cap_batch)
    monkeypatch.setattr(serve, "solve_footprint",
                        lambda g, prec, m, capacity=0: FOOTPRINT[g.J] // (4 if capacity else 1))
    reqs = [_req(0, 0.0, 7, 30), _req(1, 0.0, 6, 25), _req(2, 0.0, 7, 12), _req(3, 0.0, 8, 10)]
    srv = serve.Server(hbm_budget=1200, round_steps=10, device="cpu", capacity_fraction=0.25)
    recs = {r.rid: r for r in srv.run(reqs, realtime=False)}
    assert all(r.status == 0 for r in recs.values())
    assert all(recs[r.rid].evals == 21.0 * 10 * r.steps for r in reqs)     # exactly its steps
    assert srv.migrations == 2                                              # both J = 7 solves
    # admitted at a quarter of 1600 + 400 + 400 + 100 bytes, all resident at once
    assert FakeSolve.peak >= 3 and srv.used == 0 and FakeSolve.live == 0
    # admission keeps to the budget; a refit may take the bytes in use above it
    # (the solve cannot go on in its old arena) by at most what the refits added
    assert srv.peak_used <= 1200 + 2 * (400 - 100)
