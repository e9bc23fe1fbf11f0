"""mra_transform_noalloc (the transform for callers that cannot allocate)
against mra_transform with a caller workspace: the same kernels, so the
outputs must agree bit for bit, on two calls in a row, the second on a
smaller grid; and grids beyond the library's workspace are refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mra as om
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


def _field(N, seed):
    vs = [W.Vortex(1.0, 0.4, 2.6, 3.1), W.Vortex(0.8, 0.3, 3.9, 3.3)]
    return W.vorticity_field(N, vs) + 1e-3 * W.random_field(N, seed)


def _forward(M, fn, J, p, eps, prec, u):
    N = 1 << J
    dt = M.bulk_dtype(prec)
    g = M.grid_desc(J, p, eps)
    inp = torch.from_numpy(u).to(DEV, dt)
    out = torch.full((N * N,), float("nan"), dtype=dt, device=DEV)
    mask = torch.full((N * N,), 7, dtype=torch.uint8, device=DEV)
    ip = torch.full((N * N,), -5, dtype=torch.int32, device=DEV)
    fi = torch.full((N * N,), -5, dtype=torch.int32, device=DEV)
    na = torch.full((1,), -1, dtype=torch.int64, device=DEV)
    fn(g, prec, M.MRA_FORWARD, inp, out, mask, ip, fi, na)
    torch.cuda.synchronize()
    n = int(na.item())
    return out.cpu().numpy(), mask.cpu().numpy(), ip[:n].cpu().numpy(), fi[:n].cpu().numpy()


def _prolong(M, fn, J, p, eps, prec, mask, fi, vals):
    N = 1 << J
    g = M.grid_desc(J, p, eps)
    out = torch.full((N, N), float("nan"), dtype=M.bulk_dtype(prec), device=DEV)
    fn(g, prec, M.MRA_PROLONG, torch.from_numpy(vals).to(DEV), out, torch.from_numpy(mask).to(DEV),
       None, torch.from_numpy(fi).to(DEV), torch.tensor([fi.size], dtype=torch.int64, device=DEV))
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 2])
@pytest.mark.parametrize("p", [2, 3])
def test_noalloc_equals_workspace_call(M, prec, p):
    eps = 1e-3
    for J in (10, 9, 6):     # consecutive calls, each on a smaller grid than the last
        u = _field(1 << J, J)
        ref = _forward(M, M.mra_transform, J, p, eps, prec, u)
        got = _forward(M, M.mra_transform_noalloc, J, p, eps, prec, u)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b, equal_nan=True), f"forward J={J}"
        if prec == M.MRA_FP64:
            # and the FP64 active set is the oracle's (bit-exact)
            mask, ip, fi = om.threshold(om.forward(u, J, p), u, eps, J, p)
            assert np.array_equal(got[1], mask) and np.array_equal(got[3], fi)
        _, mask, _, fi = got
        vals = W.random_field(1 << J, 3).ravel()[fi]
        pr = _prolong(M, M.mra_transform, J, p, eps, prec, mask, fi, vals)
        pg = _prolong(M, M.mra_transform_noalloc, J, p, eps, prec, mask, fi, vals)
        assert np.array_equal(pr, pg), f"prolong J={J}"


def test_noalloc_refuses_grids_beyond_its_workspace(M):
    J = 11
    N = 1 << J
    t = torch.zeros(N * N, dtype=torch.float64, device=DEV)
    with pytest.raises(M.MraError) as e:
        M.mra_transform_noalloc(M.grid_desc(J, 2, 0.0), M.MRA_FP64, M.MRA_FORWARD, t, torch.empty_like(t))
    assert e.value.status == 2     # MRA_E_SIZE, before any launch
