"""Mixed precision against the FP64 path over many steps at the full 2048^2
size of the three-vortex configuration (6-point DD, eps 1e-4, m = 30,
dt = 0.002), both on the GPU through the C-ABI (the FP64 path is pinned to
the oracle by the parity tests).

* with its seeded noise, 100 steps: the active sets agree and the fields are
  within 1e-8 (the products' FP32 rounding enters every step; measured
  2.7e-10);
* without the noise, 500 steps: the same sets and within 1e-8 (measured
  2.9e-9, growing linearly).

Both bars sit far below the 1e-5 accuracy target; they guard the mixed path
against a regression of its arithmetic, which would show here long before a
short parity test.
"""
import dataclasses

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


def _run_pair(M, pb, steps):
    out = {}
    st = torch.cuda.Stream()
    for prec in (M.MRA_FP64, M.MRA_MIXED):
        with torch.cuda.stream(st):
            s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), prec, pb.m, pb.dt,
                        torch.from_numpy(W.initial_field(pb)).to(DEV), stream=st)
        M.solve_batch([s], [steps], stream=st)
        dense, diag = s.read(stream=st)
        mask = s.active_set()[1].cpu().numpy()
        out[prec] = (dense.cpu().numpy(), diag, mask)
        s.close()
    a, da, ma = out[M.MRA_FP64]
    b, db, mb = out[M.MRA_MIXED]
    rel = float(np.linalg.norm(a - b) / np.linalg.norm(a))
    flips = int((ma != mb).sum())
    dE = abs(da["energy"] - db["energy"]) / da["energy"]
    dZ = abs(da["enstrophy"] - db["enstrophy"]) / da["enstrophy"]
    return rel, flips, dE, dZ, int(da["n_active"])


@pytest.mark.parametrize("noise,steps", [(1e-3, 100), (0.0, 500)])
def test_three2048_mixed_tracks_fp64(M, noise, steps):
    pb = dataclasses.replace(W.three_vortex(), noise_amp=noise)
    rel, flips, dE, dZ, na = _run_pair(M, pb, steps)
    print(f"2048^2 noise {noise:g}, {steps} steps: mixed vs FP64 rel L2 {rel:.2e}, dE/E {dE:.1e}, "
          f"dZ/Z {dZ:.1e}, flips {flips}, N_a {na}")
    assert flips == 0
    assert rel <= 1e-8
    assert dE <= 1e-8 and dZ <= 1e-8
