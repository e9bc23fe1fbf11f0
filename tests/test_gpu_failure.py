"""Failure handling on the GPU: a non-finite value in a solve's state is
reported through its status word (mra_solve_read returns MRA_E_NONFINITE,
diag[7] = 5) without an update of the state, and a failing solve does not
disturb the solves it is batched with (every index the kernels use comes from
masks, ranks and positions, never from field values)."""
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


def _make(M, pb, prec, bad=False, m=10, stream=None):
    w0 = W.initial_field(pb)
    if bad:
        w0 = w0.copy()
        w0[pb.N // 3, pb.N // 5] = np.nan      # not a coarsest-level node
    st = stream if stream is not None else torch.cuda.current_stream(DEV)
    with torch.cuda.stream(st):
        return M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), prec, m, pb.dt,
                       torch.from_numpy(w0).to(DEV), stream=stream)


@pytest.mark.parametrize("prec", [0, 2])
def test_nonfinite_state_is_reported(M, prec):
    pb = W.plain_pair()
    print(f"non-finite initial field, precision {prec}", flush=True)
    s = _make(M, pb, prec, bad=True)
    _, diag = s.read()
    assert int(diag["status"]) == M.MRA_E_NONFINITE        # caught by the first threshold
    s.step(2)
    _, diag = s.read()
    assert int(diag["status"]) == M.MRA_E_NONFINITE
    sc = s.scalars()
    assert sc["steps"] == 2                 # the steps still run; the status word is sticky
    s.close()


def test_failing_solve_does_not_disturb_its_batch(M):
    pbs = [W.fujiwhara_pair(5000 + i, J=6) for i in range(3)]
    st = torch.cuda.Stream(device=DEV)
    alone = []
    for i in (0, 2):
        s = _make(M, pbs[i], M.MRA_MIXED, stream=st)
        s.step(2, stream=st)
        alone.append(s.read(stream=st)[0].cpu().numpy())
        s.close()
    solves = [_make(M, pb, M.MRA_MIXED, bad=(i == 1), stream=st) for i, pb in enumerate(pbs)]
    M.solve_batch(solves, [2, 2, 2], stream=st)
    d0, g0 = solves[0].read(stream=st)
    d2, g2 = solves[2].read(stream=st)
    _, gb = solves[1].read(stream=st)
    assert int(gb["status"]) == M.MRA_E_NONFINITE
    assert int(g0["status"]) == 0 and int(g2["status"]) == 0
    assert np.array_equal(d0.cpu().numpy(), alone[0])
    assert np.array_equal(d2.cpu().numpy(), alone[1])
    for s in solves:
        s.close()


def test_partner_cannot_be_destroyed_before_its_scalar(M):
    pb = W.plain_pair()
    s = _make(M, pb, M.MRA_MIXED)
    sc = M.ScalarSolve(s, M.grid_desc(pb.J, pb.p, 1e-3), 10, pb.dt,
                       torch.from_numpy(W.vapor_field(pb.N)).to(DEV))
    with pytest.raises(M.MraError) as e:
        s.close()
    assert e.value.status == 1 and s.handle is not None
    s.step(1)
    sc.step(1)                                  # both still usable
    sc.close()
    s.close()
    assert s.handle is None

