"""Tile autotuning on the GPU: the stencil tile edge changes only how tiles
are staged in LDS, never a node's arithmetic, so solves laid out with tiles
8, 16 and 32 step bit-identically (FP64 and mixed); solves of different tiles
share a solve_batch call and each equals itself stepped alone; a condensing
scalar steps bit-identically whatever its and its partner's tiles; the autotuner
times the candidates, applies its choice and round-trips its JSON cache."""
import json

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
    yield m
    for prec in (m.MRA_FP64, m.MRA_MIXED):
        m.tune_set_tile(7, 2, prec, 0)


def _solve(M, pb, prec, tile, stream=None):
    M.tune_set_tile(pb.J, pb.p, prec, tile)
    try:
        return M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), prec, pb.m, pb.dt,
                       torch.from_numpy(W.initial_field(pb)).to(DEV), stream=stream)
    finally:
        M.tune_set_tile(pb.J, pb.p, prec, 0)


@pytest.mark.parametrize("prec", [0, 2])
def test_tiles_step_bit_identically(M, prec):
    pb = W.fujiwhara_pair(1003, J=7)
    out = {}
    for tile in (8, 16, 32):
        s = _solve(M, pb, prec, tile)
        s.step(3)
        out[tile] = s.read()[0].cpu().numpy()
        s.close()
    print(f"128^2 precision {prec}: tiles 8, 16, 32 after 3 steps")
    assert np.array_equal(out[8], out[16]) and np.array_equal(out[16], out[32])


def test_mixed_tiles_share_a_batch(M):
    pbs = [W.fujiwhara_pair(1010 + i, J=7) for i in range(3)]
    tiles = [16, 32, 16]
    st = torch.cuda.Stream(device=DEV)
    alone = []
    for pb, t in zip(pbs, tiles):
        with torch.cuda.stream(st):
            s = _solve(M, pb, M.MRA_MIXED, t, stream=st)
        s.step(2, stream=st)
        alone.append(s.read(stream=st)[0].cpu().numpy())
        s.close()
    with torch.cuda.stream(st):
        solves = [_solve(M, pb, M.MRA_MIXED, t, stream=st) for pb, t in zip(pbs, tiles)]
    M.solve_batch(solves, [2, 2, 2], stream=st)
    for s, ref in zip(solves, alone):
        assert np.array_equal(s.read(stream=st)[0].cpu().numpy(), ref)
        s.close()


def test_autotuner_choice_and_cache(M, tmp_path):
    from paper_1604_08159_amd import autotune as at
    cache = str(tmp_path / "tiles.json")
    ent = at.autotune([(7, 2, M.MRA_MIXED)], cache=cache, nsolves=2, steps=3, warmup=1)
    e = ent["J7_p2_prec2"]
    print(f"128^2 mixed: ms per step by tile {e['ms_per_step']}, chosen {e['tile']}")
    assert set(e["ms_per_step"]) == {"8", "16", "32"} and e["tile"] in (8, 16, 32)
    assert M.tune_get_tile(7, 2, M.MRA_MIXED) == e["tile"]
    M.tune_set_tile(7, 2, M.MRA_MIXED, 0)
    data = json.load(open(cache))
    assert data["entries"]["J7_p2_prec2"]["tile"] == e["tile"]
    assert at.apply_cache(cache) == 1 and M.tune_get_tile(7, 2, M.MRA_MIXED) == e["tile"]
    # a cached entry is not timed again
    again = at.autotune([(7, 2, M.MRA_MIXED)], cache=cache)
    assert again["J7_p2_prec2"] == data["entries"]["J7_p2_prec2"]
    M.tune_set_tile(7, 2, M.MRA_MIXED, 0)


def test_scalar_tiles_step_bit_identically(M):
    """A passive scalar (with condensation) laid out with tile 16 or 32 on a
    partner of either tile steps bit-identically."""
    pb = W.fujiwhara_pair(1004, J=7)
    r0 = torch.from_numpy(W.vapor_patch(pb.N, 1.0, 0.005)).to(DEV)
    out = []
    for tv, ts in ((32, 32), (16, 32), (32, 16)):
        v = _solve(M, pb, M.MRA_MIXED, tv)
        M.tune_set_tile(pb.J, pb.p, M.MRA_MIXED, ts)
        try:
            s = M.ScalarSolve(v, M.grid_desc(pb.J, pb.p, 1e-3), 10, pb.dt, r0, kappa0=0.01, eddy=False)
        finally:
            M.tune_set_tile(pb.J, pb.p, M.MRA_MIXED, 0)
        s.set_condensation(1.0)
        M.solve_batch([v, s], [3, 3])
        out.append(s.read()[0].cpu().numpy())
        s.close()
        v.close()
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
