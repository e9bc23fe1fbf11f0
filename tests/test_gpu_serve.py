"""Continuous batching: a request served inside a changing mix of solves of
different sizes gives bit-identical results to the same request run alone;
admission respects the HBM budget; an oversize request is rejected without
affecting the others."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1604_08159_amd import serve
    return serve


def _requests(S):
    timed = W.serving_requests(6, seed=7, J_range=(5, 7), steps_range=(7, 30))
    return S.requests_from_problems(timed, W.initial_field)


def test_mix_equals_alone(S):
    reqs = _requests(S)
    srv = S.Server(hbm_budget=8 << 30, round_steps=5, keep_results=True)
    mixed = {r.rid: r for r in srv.run(reqs, realtime=False)}
    assert len(mixed) == len(reqs)
    for q in reqs:
        alone = S.Server(hbm_budget=8 << 30, round_steps=11, keep_results=True).run([q], realtime=False)[0]
        a, b = mixed[q.rid], alone
        assert a.status == 0 and b.status == 0
        assert torch.equal(a.omega, b.omega), q.rid
        assert a.diag["n_active"] == b.diag["n_active"]


def test_budget_admission_and_rejection(S):
    reqs = _requests(S)
    big = max(S.Server(1).footprint(r) for r in reqs)
    # a budget for about two solves: everything is served, never above budget
    srv = S.Server(hbm_budget=2 * big, round_steps=5)
    peak = [0]
    orig = srv._admit

    def admit(r, rec, now):
        orig(r, rec, now)
        peak[0] = max(peak[0], srv.used)
    srv._admit = admit
    recs = srv.run(reqs, realtime=False)
    assert len(recs) == len(reqs) and all(r.status == 0 for r in recs)
    assert peak[0] <= 2 * big
    # a budget below one footprint: that request is rejected, the rest run
    srv = S.Server(hbm_budget=big - 1, round_steps=5)
    recs = srv.run(reqs, realtime=False)
    assert sum(r.status < 0 for r in recs) >= 1
    assert all(r.status == 0 for r in recs if r.status >= 0)
    summ = S.summarize(recs, 1.0)
    assert summ["rejected"] >= 1 and summ["failed"] == 0


def test_staggered_arrivals_tight_budget_equal_alone(S):
    """Poisson-like arrivals on the wall clock and a budget of about two
    solves: requests are admitted while others are resident and mid-run
    (no barrier across groups), and each result is still bit-identical to
    the request served alone."""
    timed = W.serving_requests(8, seed=11, rate=40.0, J_range=(5, 7), steps_range=(10, 40))
    reqs = S.requests_from_problems(timed, W.initial_field)
    big = max(S.Server(1).footprint(r) for r in reqs)
    srv = S.Server(hbm_budget=2 * big, round_steps=4, keep_results=True)
    recs = {r.rid: r for r in srv.run(reqs, realtime=True)}
    assert all(r.status == 0 for r in recs.values())
    # some request was admitted while another one was resident and unfinished
    overlap = [(a.rid, b.rid) for a in recs.values() for b in recs.values()
               if a.rid != b.rid and b.admitted < a.admitted < b.finished]
    assert overlap, "no request joined while another was running"
    for q in reqs:
        alone = S.Server(hbm_budget=8 << 30, round_steps=7, keep_results=True).run([q], realtime=False)[0]
        assert torch.equal(recs[q.rid].omega, alone.omega), q.rid
