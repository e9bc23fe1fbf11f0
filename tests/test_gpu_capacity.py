"""Solves sized by capacity (mra_solve_init_cap, mra_solve_migrate): the
active-length arrays and the Krylov basis hold `capacity` nodes.  A solve
whose active set outgrows its capacity freezes without writing past it, and
once moved to a larger arena continues exactly as a solve of full capacity:
masks and values bit-identical after the same steps."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_08159_amd as m
    m.lib()
    return m


def _make(M, pb, prec, capacity=0, stream=None):
    w0 = torch.from_numpy(W.initial_field(pb)).to(DEV)
    return M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), prec, pb.m, pb.dt, w0,
                   stream=stream, capacity=capacity)


def _state(s):
    om, mask, ip, fi = s.active_set()
    return om.cpu().numpy(), mask.cpu().numpy(), fi.cpu().numpy()


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("prec", ["MRA_FP64", "MRA_MIXED"])
def test_small_capacity_runs_like_full(M, prec):
    pb = W.fujiwhara_pair(1000, J=8)
    pr = getattr(M, prec)
    full = _make(M, pb, pr)
    na0 = int(full.read(dense=False)[1]["n_active"])
    # an initial capacity below the first active set: refused by the init,
    # which the constructor repeats with a larger arena
    small = _make(M, pb, pr, capacity=max(64, na0 // 4))
    print(f"{prec}: N_a0 {na0}, capacity after init {small.capacity}, migrations {small.migrations}", flush=True)
    assert small.migrations == 1 and na0 <= small.capacity < full.capacity
    assert small.nbytes < full.nbytes
    assert _same(_state(full), _state(small))
    # exactly the active count: any growth freezes the solve within the run
    small.migrate(na0)
    assert small.capacity == na0
    for k in range(4):
        full.step(5)
        small.step(5)
        assert _same(_state(full), _state(small)), f"after {5 * (k + 1)} steps"
    df, dgf = full.read()
    ds, dgs = small.read()
    print(f"  after 20 steps: N_a {int(dgf['n_active'])}, capacity {small.capacity}, migrations "
          f"{small.migrations}, t {dgf['t']:.4f} / {dgs['t']:.4f}")
    assert torch.equal(df, ds)
    assert dgf["t"] == dgs["t"] and dgs["status"] == 0
    full.close()
    small.close()


def test_frozen_solve_is_inert_until_moved(M):
    pb = W.fujiwhara_pair(1001, J=8)
    st = torch.cuda.Stream(device=DEV)
    ref = _make(M, pb, M.MRA_MIXED, stream=st)
    M.solve_batch([ref], [6], stream=st)
    na = [int(ref.read(dense=False, stream=st)[1]["n_active"])]
    s = _make(M, pb, M.MRA_MIXED, stream=st)
    # the capacity of the initial set, and steps enqueued without refitting
    _, na0, _ = s.capacity_state(stream=st)
    s.migrate(na0, stream=st)
    M.solve_batch([s], [6], stream=st, fit=False)
    cap, need, frozen = s.capacity_state(stream=st)
    if not frozen:
        pytest.skip(f"the active set did not outgrow {na0} nodes in 6 steps (N_a {need})")
    dense, diag = s.read(stream=st)
    t_frozen = diag["t"]
    assert diag["status"] == M.MRA_E_CAPACITY and diag["n_active"] == 0
    M.solve_batch([s], [3], stream=st, fit=False)          # steps of a frozen solve move nothing
    dense2, diag2 = s.read(stream=st)
    assert diag2["t"] == t_frozen and torch.equal(dense, dense2)
    steps = s.steps_done(stream=st)
    assert steps < 6
    assert s.fit(stream=st) and s.capacity >= need
    M.solve_batch([s], [6 - steps], stream=st)
    print(f"frozen at {steps} steps with capacity {cap} (needed {need}); moved to {s.capacity}")
    assert _same(_state(ref), _state(s))
    ref.close()
    s.close()


def test_batch_mixes_capacities_and_sizes(M):
    pbs = [W.fujiwhara_pair(1010 + i, J=J) for i, J in enumerate((7, 8, 8, 9))]
    st = torch.cuda.Stream(device=DEV)
    alone = []
    for pb in pbs:
        s = _make(M, pb, M.MRA_MIXED, stream=st)
        M.solve_batch([s], [8], stream=st)
        alone.append(_state(s))
        s.close()
    solves = []
    for i, pb in enumerate(pbs):
        s = _make(M, pb, M.MRA_MIXED, stream=st)
        if i % 2 == 0:
            _, na0, _ = s.capacity_state(stream=st)
            s.migrate(na0, stream=st)                      # tight: likely to refit during the batch
        solves.append(s)
    M.solve_batch(solves, [8] * len(solves), stream=st)
    print("capacities", [s.capacity for s in solves], "migrations", [s.migrations for s in solves])
    for s, a in zip(solves, alone):
        assert _same(_state(s), a)
        assert s.steps_done(stream=st) == 8
    for s in solves:
        s.close()


def test_capacity_refusals(M):
    pb = W.fujiwhara_pair(1020, J=7)
    s = _make(M, pb, M.MRA_MIXED, capacity=4096)
    with pytest.raises(M.MraError) as e:                    # a scalar rides only on a full-capacity solve
        M.ScalarSolve(s, M.grid_desc(pb.J, pb.p, pb.eps), 8, pb.dt,
                      torch.zeros((1 << pb.J, 1 << pb.J), dtype=torch.float64, device=DEV))
    assert e.value.status == M.MRA_E_UNSUPPORTED
    _, na, _ = s.capacity_state()
    with pytest.raises(M.MraError) as e:                    # below the active count
        s.migrate(max(16, na // 2))
    assert e.value.status == 2
    with pytest.raises(M.MraError) as e:
        s.migrate((1 << (2 * pb.J)) + 1)
    assert e.value.status == 2
    s.close()
