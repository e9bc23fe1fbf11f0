"""Benchmark of the wavelet-collocation vortex step on one MI355X.

Headline workload: the three-vortex Re = 37440 configuration at its full
size, 2048 x 2048 finest grid (J = 11), 6-point DD, threshold 1e-4,
Smagorinsky Cs = 0.17, Krylov dimension 30, dt = 0.002, seeded white-noise
vorticity of amplitude 1e-3 (nearly every node active at first); a batch of
two solves (noise seeds 37440, 37441) in mixed precision.  One step = one
exponential Rosenbrock-Euler step of every solve of the batch (residual,
30 Jacobian-vector products, Arnoldi, phi_1, update and FP64 regrid),
launched together through solve_batch and replayed as a HIP graph.

Metric: active-point residual evaluations per second, summed over the batch
((1 + m_eff) N_a per solve and step, counted on the device).  Also reported
in the same JSON line:
  roofline        the dominant kernel of the step (largest share of one
                  step's GPU time, from per-phase HIP events inside a step)
                  against 8 TB/s, with algorithmic bytes per launch from the
                  per-unit byte model of each kernel (kernel_bytes), and the
                  same for every other kernel of the step;
  rhs_pipeline    the HBM fraction of the residual and product kernels
                  together: (B_F + m B_Jv) / (t_F + m t_Jv) / 8 TB/s;
  cpu_baseline    the FP64 CPU oracle on a bounded sample of the same
                  workload (one residual and 17 products at 2048^2, one
                  core, about 10 s), whose outputs also give the accuracy of the GPU's
                  residual and product against the oracle;
  sub-records     the 512^2 Fujiwhara batch of 24 (with its accuracy against
                  the oracle after the timed steps and its 2000-step drift),
                  the 2048^2 configuration's 5000-step drift (mixed against
                  FP64, beside a perturbed FP64 run), the 256-solve ensemble (solves/s against the FP64 per-solve
                  GPU path and the oracle), and the serving configuration's
                  request mix (p50 / p99 latency at 70% of capacity).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ...]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CALIB_BYTES = 64 << 20          # plain device copy of known size (PMC byte-counter scale)
KERNEL_SOURCES = {"jvp": "k_stencil.hip", "res_stencil": "k_stencil.hip", "prolong": "k_transform.hip",
                  "res_prolong": "k_transform.hip", "fft_rows": "k_fft.hip", "fft_cols": "k_fft.hip",
                  "fft_rows_inv": "k_fft.hip", "res_fft_rows": "k_fft.hip", "res_fft_cols": "k_fft.hip",
                  "res_fft_rows_inv": "k_fft.hip", "gram_schmidt": "k_krylov.hip"}
SEEDS = list(range(1000, 1024))   # 24 resident solves: the throughput-optimal batch on one MI355X
METRIC = "active-pt RHS evals/s"
ORACLE_ENV = {"OMP_NUM_THREADS": "1", "OPENBLAS_NUM_THREADS": "1", "MKL_NUM_THREADS": "1",
              "NUMEXPR_NUM_THREADS": "1"}


def kernel_bytes(phase: str, N: int, na: float, phi_t: float, esz: int, m: int) -> float:
    """Algorithmic HBM bytes of one launch of a step phase for ONE solve: the
    per-unit byte model of each kernel (what the method must move), with N_f
    terms at the bulk element size esz (4 for FP32 fields, 8 for FP64):
      Pi                 esz N_f written + 12 N_a (FP64 value + int32 index)
      Poisson pass       2 esz N_f (read + write of the real-field equivalent)
      product stencil    6 esz N_f phi_t (v~, psi_v, w~, u, v, nu_e on the
                         tiles holding an active node) + 12 N_a (FP64 out + index)
      residual stencil   2 esz N_f phi_t (w~, psi) + 12 N_a
      Gram-Schmidt       16 m (m+1) N_a + 64 m N_a per step for CGS2 with the
                         second pass in every column and every pass reading
                         the basis twice, per column: that over m (gs_bytes
                         gives what the delayed second pass reads, about half)
    The residual of a solve with FP32 bulk fields runs in FP64 (esz 8 for its
    phases).  The dense int32 rank map that the kernels read is implementation
    traffic and is reported apart (rank_map_bytes)."""
    nf = N * N
    if phase in ("prolong", "res_prolong", "regrid_prolong"):
        return esz * nf + 12 * na
    if phase in ("fft_rows", "fft_cols", "fft_rows_inv", "res_fft_rows", "res_fft_cols", "res_fft_rows_inv"):
        return 2 * esz * nf
    if phase == "jvp":
        return 6 * esz * nf * phi_t + 12 * na
    if phase == "res_stencil":
        return 2 * esz * nf * phi_t + 12 * na
    if phase == "gram_schmidt":
        return (16 * m * (m + 1) * na + 64 * m * na) / m
    raise KeyError(phase)


def gs_bytes(N_a: float, m: int, vsz: int = 8) -> float:
    """Bytes of the Gram-Schmidt of one step as the delayed-reorthogonalisation
    CGS2 runs it: column j reads slots 0..j of the basis (vsz bytes per entry)
    and w (FP64) twice, once per stage, and writes v_j (j > 0) and r_{j+1}
    (j < m - 1).  Every column gets its second pass within these two reads."""
    tot = 0.0
    for j in range(m):
        rd = (j + 1) * vsz + 8
        tot += 2 * rd + vsz * ((1 if j > 0 else 0) + (1 if j < m - 1 else 0))
    return tot * N_a


# launches of each phase in one step (the rest run once)
PER_COLUMN = ("prolong", "fft_rows", "fft_cols", "fft_rows_inv", "jvp", "gram_schmidt")
RESIDUAL = ("res_prolong", "res_fft_rows", "res_fft_cols", "res_fft_rows_inv", "res_stencil")
MODELLED = RESIDUAL + PER_COLUMN


def roofline_from_profile(prof: dict, N: int, na: float, phi_t: float, nbatch: int, bulk_esz: int, m: int,
                          residual_esz: int = 8, gs_step_bytes: float = None) -> dict:
    """Per-kernel achieved bandwidth from one profiled step (GPU ms per phase,
    summed over the step): algorithmic bytes per launch / average launch time.
    gs_step_bytes: the Gram-Schmidt bytes of the profiled step over the batch
    (gs_bytes); else the CGS2 model of kernel_bytes."""
    step_ms = sum(prof.values())
    out = {}
    for ph in MODELLED:
        launches = m if ph in PER_COLUMN else 1
        esz = residual_esz if ph in RESIDUAL else bulk_esz
        if ph == "gram_schmidt":
            esz = 8
        nbytes = kernel_bytes(ph, N, na, phi_t, esz, m) * nbatch
        if ph == "gram_schmidt" and gs_step_bytes is not None:
            nbytes = gs_step_bytes / m
        avg = prof[ph] / launches
        gbs = nbytes / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
        out[ph] = {"launches_per_step": launches, "avg_launch_ms": avg, "share_of_step": prof[ph] / step_ms,
                   "algorithmic_bytes_per_launch": nbytes, "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS}
    return out


def rhs_pipeline(kern: dict, m: int) -> dict:
    """HBM fraction of the residual and product kernels together:
    (B_F + m B_Jv) / (t_F + m t_Jv) against the peak."""
    bf = sum(kern[p]["algorithmic_bytes_per_launch"] for p in RESIDUAL)
    tf = sum(kern[p]["avg_launch_ms"] for p in RESIDUAL)
    prod = ("prolong", "fft_rows", "fft_cols", "fft_rows_inv", "jvp")
    bj = sum(kern[p]["algorithmic_bytes_per_launch"] for p in prod)
    tj = sum(kern[p]["avg_launch_ms"] for p in prod)
    gbs = (bf + m * bj) / ((tf + m * tj) * 1e-3) / 1e9
    return {"bytes_F": bf, "ms_F": tf, "bytes_Jv": bj, "ms_Jv": tj, "achieved_gbs": gbs,
            "frac": gbs / HBM_PEAK_GBS,
            "kernels": "residual: Pi, 3 Poisson passes, stencil (FP64); product: Pi, 3 Poisson passes, stencil"}


def active_tile_fraction(solves, N: int, ts: int = 32) -> float:
    """Fraction of the stencil tiles holding an active node, over the batch."""
    import torch
    fr = []
    for s in solves:
        _, _, _, fi = s.active_set()
        f = fi.long()
        t = ((f // N) // ts) * (N // ts) + (f % N) // ts
        fr.append(torch.unique(t).numel() / (N // ts) ** 2)
    return sum(fr) / len(fr)


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    runs, if they were taken on the current source of the kernel."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_1604_08159_amd", "csrc", KERNEL_SOURCES[kernel])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    return rec.get("bytes_per_launch")


def fp64_per_solve(m, W, dev, steps: int) -> dict:
    """The 512^2 Fujiwhara workload, one solve at a time, all bulk fields in FP64."""
    import torch
    stream = torch.cuda.Stream(device=dev)
    pb = W.fujiwhara_pair(SEEDS[0])
    with torch.cuda.stream(stream):
        w0 = torch.from_numpy(W.initial_field(pb)).to(dev)
        s = m.Solve(m.grid_desc(pb.J, pb.p, pb.eps), m.flow_desc(pb.nu0, pb.cs), m.MRA_FP64, pb.m, pb.dt, w0,
                    stream=stream)
    s.step(3, stream=stream)
    stream.synchronize()
    e0 = s.scalars()["evals"]
    t0 = time.perf_counter()
    s.step(steps, stream=stream)
    stream.synchronize()
    wall = time.perf_counter() - t0
    e1 = s.scalars()["evals"]
    s.close()
    return {"value": (e1 - e0) / wall, "ms_per_step": wall / steps * 1e3, "steps": steps,
            "solves_per_s_at_2000_steps": 1.0 / (wall / steps * 2000)}


def compare_fields(a, b, da: dict, db: dict) -> dict:
    """Relative L2 of two dense vorticity fields and the relative differences
    of energy and enstrophy (a is the reference)."""
    rel = float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(a)))
    return {"rel_l2_vorticity": rel, "rel_energy": abs(da["energy"] - db["energy"]) / da["energy"],
            "rel_enstrophy": abs(da["enstrophy"] - db["enstrophy"]) / da["enstrophy"]}


def start_oracle(code: str) -> subprocess.Popen:
    """An oracle run in a single-threaded child process (it overlaps the GPU legs)."""
    env = dict(os.environ, **ORACLE_ENV)
    return subprocess.Popen([sys.executable, "-c", code], env=env, stdout=subprocess.PIPE,
                            stderr=subprocess.PIPE, text=True)


def finish_oracle(pr: subprocess.Popen) -> dict:
    out, err = pr.communicate()
    if pr.returncode != 0:
        raise RuntimeError("oracle run failed: " + err[-2000:])
    return json.loads(out.strip().splitlines()[-1])


# products in the oracle's timed sample of the 2048^2 headline: about 10 s of
# one core, in a child process that overlaps the GPU legs
THREE_CPU_PRODUCTS = 17

ORACLE_THREE = """
import json, sys, time, dataclasses
sys.path.insert(0, {root!r})
import numpy as np
import workloads as W
from oracle import krylov as ok, ops as oo
pb = dataclasses.replace(W.three_vortex(), noise_seed={seed})
g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps); fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
st = ok.init_state(W.initial_field(pb), g)
op = ok.Operator(g, fl, st.index_fine)
t0 = time.perf_counter()
F = op.F(st.omega_M)
v = F / np.linalg.norm(F)
outs = []
for _ in range({nprod}):
    w = op.Av(v)
    outs.append((v, w))
    v = w / np.linalg.norm(w)
sec = time.perf_counter() - t0
np.save({d!r} + "/omega.npy", st.omega_M); np.save({d!r} + "/fi.npy", st.index_fine)
np.save({d!r} + "/mask.npy", st.mask); np.save({d!r} + "/F.npy", F)
np.save({d!r} + "/v.npy", outs[0][0]); np.save({d!r} + "/Av.npy", outs[0][1])
print(json.dumps({{"evals": (1 + {nprod}) * int(st.omega_M.size), "sec": sec, "n_active": int(st.omega_M.size)}}))
"""

ORACLE_PAIR = """
import json, sys, time
sys.path.insert(0, {root!r})
import numpy as np
import workloads as W
from oracle import krylov as ok, mra as om, ops as oo
pb = W.fujiwhara_pair({seed})
g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps); fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
st = ok.init_state(W.initial_field(pb), g)
ev = 0; t0 = time.perf_counter()
for _ in range({steps}):
    na = st.omega_M.size; st = ok.step(st, g, fl, pb.m, pb.dt); ev += (1 + st.last_m_eff) * na
sec = time.perf_counter() - t0
ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
np.save({d!r} + "/pair_ref.npy", ref); np.save({d!r} + "/pair_mask.npy", st.mask)
print(json.dumps({{"evals": ev, "sec": sec, "n_active": int(st.omega_M.size), "diag": ok.diagnostics(ref, g)}}))
"""


def ensemble_cpu_baseline(probs, steps: int = 2) -> dict:
    """The FP64 oracle for the ensemble: for every grid size, one solve of the
    ensemble is timed over `steps` steps, single-threaded, in its own process
    (the sizes run side by side); the per-step times, applied to every solve's
    step count and spread over the host's cores one solve per process, give
    the oracle's ensemble rate."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               NUMEXPR_NUM_THREADS="1")
    code = (
        "import json,sys,time; sys.path.insert(0, %r)\n"
        "import workloads as W\n"
        "from oracle import krylov as ok, ops as oo\n"
        "pb = W.ensemble(%d, steps=%d)[%d]\n"
        "g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps); fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)\n"
        "st = ok.init_state(W.initial_field(pb), g)\n"
        "t0 = time.perf_counter()\n"
        "for _ in range(%d):\n"
        "    st = ok.step(st, g, fl, pb.m, pb.dt)\n"
        "print(json.dumps({'sec_per_step': (time.perf_counter() - t0) / %d}))\n")
    first = {}
    for i, pb in enumerate(probs):
        first.setdefault(pb.J, i)
    procs = {J: subprocess.Popen([sys.executable, "-c", code % (ROOT, len(probs), probs[0].steps, i, steps, steps)],
                                 env=env, stdout=subprocess.PIPE, text=True) for J, i in first.items()}
    per_step = {}
    for J, pr in procs.items():
        out, _ = pr.communicate()
        if pr.returncode != 0:
            raise RuntimeError(f"oracle ensemble timing failed for J={J}")
        per_step[J] = json.loads(out.strip().splitlines()[-1])["sec_per_step"]
    cores = min(len(os.sched_getaffinity(0)), 16)
    total = sum(per_step[pb.J] * pb.steps for pb in probs) / cores
    return {"value": len(probs) / total, "unit": "ensemble solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} oracle steps of one solve per grid size ({', '.join(str(1 << J) + '^2' for J in sorted(per_step))}), "
                      f"single-threaded; per-step seconds {', '.join(f'{per_step[J]:.2f}' for J in sorted(per_step))}, "
                      f"applied to every solve's step count over {cores} cores, one solve per process (extrapolated)"}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def progress_printer(every: float = 10.0):
    """Round callback of the server: one stderr line every `every` seconds."""
    last = [time.perf_counter()]

    def cb(done: int, live: int, pending: int) -> None:
        now = time.perf_counter()
        if now - last[0] >= every:
            last[0] = now
            log(f"  {done} done, {live} resident, {pending} waiting")
    return cb


def tune_tiles(Js, cache: str = "") -> dict:
    """Tile autotuning for the grid sizes of a workload (outside any timed
    region): each size J (with its count in Js) is tuned at the batch it runs
    at, up to 16 resident solves, 6 steps per candidate.  Returns the choices
    and timings for the JSON line."""
    import collections
    from paper_1604_08159_amd import MRA_MIXED, autotune
    ta = time.perf_counter()
    counts = collections.Counter(Js)
    tuned = {}
    for J in sorted(counts):
        tuned.update(autotune.autotune([(J, 2, MRA_MIXED)], cache=cache or None,
                                       nsolves=min(16, counts[J]), steps=6, warmup=2))
    out = {"tiles": {str(J): tuned[autotune.entry_key(J, 2, MRA_MIXED)]["tile"] for J in sorted(counts)},
           "ms_per_step_by_tile": {str(J): tuned[autotune.entry_key(J, 2, MRA_MIXED)]["ms_per_step"]
                                   for J in sorted(counts)},
           "seconds": time.perf_counter() - ta,
           "note": "per size, a batch of up to 16 two-vortex solves, 6 steps per candidate, before the run"}
    log("autotune: " + ", ".join(f"J={J} tile {t}" for J, t in out["tiles"].items()))
    return out


def untune_tiles(tuned: dict) -> None:
    import paper_1604_08159_amd as m
    for J in tuned["tiles"]:
        m.tune_set_tile(int(J), 2, m.MRA_MIXED, 0)


def ensemble_leg(args, with_cpu: bool = True) -> dict:
    """Batched ensemble: two-vortex solves of sizes 128^2..1024^2, mixed
    precision, all resident, advanced by the continuous-batching server."""
    import torch
    import workloads as W
    import paper_1604_08159_amd as m
    from paper_1604_08159_amd import MRA_FP64, MRA_MIXED, serve
    probs = W.ensemble(args.solves, steps=args.ens_steps)
    tuned = tune_tiles([pb.J for pb in probs], args.tune_cache)
    reqs = serve.requests_from_problems([(0.0, pb) for pb in probs], W.initial_field)
    srv = serve.Server(hbm_budget=args.hbm_gb << 30, prec=MRA_MIXED, round_steps=args.round_steps,
                       progress=progress_printer())
    log(f"ensemble: {len(probs)} solves, {args.ens_steps} steps each")
    t0 = time.perf_counter()
    recs = srv.run(reqs, realtime=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    summ = serve.summarize(recs, wall)
    full_peak = srv.peak_used
    # the same ensemble with arenas sized for a fraction of N^2 active nodes:
    # residency, refits and the same results
    srv2 = serve.Server(hbm_budget=args.hbm_gb << 30, prec=MRA_MIXED, round_steps=args.round_steps,
                        progress=progress_printer(), capacity_fraction=args.cap_frac)
    t0 = time.perf_counter()
    recs2 = srv2.run(reqs, realtime=False)
    torch.cuda.synchronize()
    wall2 = time.perf_counter() - t0
    by_id = {r.rid: r for r in recs}
    same = all(r.status == 0 and r.diag == by_id[r.rid].diag for r in recs2)
    cap_rec = {"capacity_fraction": args.cap_frac, "solves_per_s": len(recs2) / wall2, "wall_s": wall2,
               "peak_resident_bytes": srv2.peak_used, "full_capacity_peak_resident_bytes": full_peak,
               "refits": srv2.migrations, "diagnostics_identical_to_full_capacity": same,
               "note": "every solve resident at once in both runs; a solve whose active set outgrows its "
                       "capacity is moved to a larger arena when its round ends"}
    log(f"capacity-sized ensemble: peak {srv2.peak_used / 2**30:.2f} GiB against {full_peak / 2**30:.2f} GiB, "
        f"{srv2.migrations} refits, identical {same}")
    # baseline: the FP64 GPU path, one solve at a time: per grid size, one
    # solve is warmed up (graph captured) and timed over a few steps, and that
    # per-step time is applied to every solve's step count
    per_step = {}
    for J in sorted({pb.J for pb in probs}):
        pb = next(q for q in probs if q.J == J)
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            s = m.Solve(m.grid_desc(pb.J, pb.p, pb.eps), m.flow_desc(pb.nu0, pb.cs), MRA_FP64, pb.m, pb.dt,
                        torch.from_numpy(W.initial_field(pb)).cuda(), stream=st)
        s.step(2, stream=st)
        st.synchronize()
        ta = time.perf_counter()
        s.step(8, stream=st)
        st.synchronize()
        per_step[J] = (time.perf_counter() - ta) / 8
        s.close()
        log(f"fp64 per-solve J={J}: {per_step[J] * 1e3:.2f} ms/step")
    fp64_total = sum(per_step[pb.J] * pb.steps for pb in probs)
    accuracy = ensemble_accuracy(m, W, probs)
    cpu = ensemble_cpu_baseline(probs) if with_cpu else None
    out = ({"workload": f"ensemble of {len(probs)} two-vortex solves, finest 128^2..1024^2, "
                                  f"{args.ens_steps} steps each, mixed precision, one GPU",
                      "metric": "ensemble solves/s", "value": summ["solves_per_s"], "wall_s": wall,
                      "active_pt_evals_per_s": summ["active_pt_evals_per_s"], "failed": summ["failed"],
                      "fp64_per_solve_gpu": {"solves_per_s_extrapolated": len(probs) / fp64_total,
                                             "sec_per_step_by_J": per_step,
                                             "note": "one warmed solve per size timed over 8 steps, "
                                                     "applied to every solve's step count"},
                      "accuracy_vs_fp64_gpu": accuracy,
                      "autotune": tuned, "capacity_sized": cap_rec,
                      "cpu_baseline": cpu})
    untune_tiles(tuned)
    return out


def ensemble_accuracy(m, W, probs) -> dict:
    """The first solve of each grid size of the ensemble over its full step
    count, mixed precision (the tiles the ensemble ran with) against the FP64
    GPU path on the same problem: vorticity, energy and enstrophy, and the
    active sets."""
    import torch
    rows = {}
    worst = 0.0
    for J in sorted({pb.J for pb in probs}):
        pb = next(q for q in probs if q.J == J)
        st = torch.cuda.Stream()
        res = {}
        for name, prec in (("fp64", m.MRA_FP64), ("mixed", m.MRA_MIXED)):
            with torch.cuda.stream(st):
                s = m.Solve(m.grid_desc(pb.J, pb.p, pb.eps), m.flow_desc(pb.nu0, pb.cs), prec, pb.m, pb.dt,
                            torch.from_numpy(W.initial_field(pb)).cuda(), stream=st)
            s.step(pb.steps, stream=st)
            dense, diag = s.read(stream=st)
            _, mask, _, _ = s.active_set()
            res[name] = (dense.cpu().numpy(), diag, mask.cpu().numpy())
            s.close()
        a, da, ma = res["fp64"]
        b, db, mb = res["mixed"]
        row = {"steps": pb.steps, "eps": pb.eps, **compare_fields(a, b, da, db),
               "mask_flips": int((ma != mb).sum()), "n_active_fp64": int(da["n_active"])}
        worst = max(worst, row["rel_l2_vorticity"], row["rel_energy"], row["rel_enstrophy"])
        rows[str(1 << J)] = row
        log(f"ensemble accuracy {1 << J}^2: rel L2 {row['rel_l2_vorticity']:.2e}, flips {row['mask_flips']}")
    return {"by_finest_size": rows, "worst": worst, "tolerance": 1e-5, "within": worst <= 1e-5,
            "note": "the first solve of each size, its full step count, mixed against FP64 on the GPU"}


def run_ensemble(args) -> int:
    print(json.dumps(ensemble_leg(args, not args.no_cpu)))
    return 0


def run_serving(args) -> int:
    """Poisson arrivals of 1-3 vortex solves of sizes 64^2..2048^2, admitted
    by HBM footprint, served by continuous batching; latency percentiles."""
    import torch
    import workloads as W
    from paper_1604_08159_amd import MRA_MIXED, serve
    timed = W.serving_requests(args.requests, rate=args.rate, J_range=(6, args.max_J),
                               steps_range=(args.min_steps, args.max_steps))
    tuned = tune_tiles([pb.J for _, pb in timed], args.tune_cache)
    reqs = serve.requests_from_problems(timed, W.initial_field)
    srv = serve.Server(hbm_budget=args.hbm_gb << 30, prec=MRA_MIXED, round_steps=args.round_steps,
                       progress=progress_printer())
    log(f"serving: {len(reqs)} requests over {timed[-1][0]:.2f} s of arrivals")
    t0 = time.perf_counter()
    recs = srv.run(reqs, realtime=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    summ = serve.summarize(recs, wall)
    offered = args.rate
    print(json.dumps({"workload": f"serving: {args.requests} requests, Poisson arrivals at {args.rate}/s, "
                                  f"finest 64^2..{1 << args.max_J}^2, {args.min_steps}-{args.max_steps} steps",
                      **summ, "offered_req_per_s": offered,
                      "achieved_req_per_s": summ["solves_per_s"], "autotune": tuned}))
    untune_tiles(tuned)
    return 0


def serving_spec_leg(args) -> dict:
    """The serving configuration's request mix (1-3 vortices, finest 64^2..2048^2
    log-uniform over levels, 200-2000 steps, Re 1e3..4e4) on a bounded sample:
    capacity from a closed-loop run (every request queued at once), then
    Poisson arrivals at 70% of that capacity for the latency percentiles.  The
    configuration's 50 req/s is far above one GPU's capacity for this mix, so
    its queue would grow without bound."""
    import torch
    import workloads as W
    from paper_1604_08159_amd import MRA_MIXED, serve
    n = args.spec_requests

    def server():
        return serve.Server(hbm_budget=args.hbm_gb << 30, prec=MRA_MIXED, round_steps=args.round_steps,
                            progress=progress_printer())

    timed = W.serving_requests(n, seed=50, rate=50.0, J_range=(6, 11), steps_range=(200, 2000))
    log(f"serving_spec: capacity run, {n} requests queued at once")
    t0 = time.perf_counter()
    recs = server().run(serve.requests_from_problems(timed, W.initial_field), realtime=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cap = {k: v for k, v in serve.summarize(recs, wall).items() if "latency" not in k}   # no arrival clock here
    rate = 0.7 * cap["solves_per_s"]
    timed70 = W.serving_requests(n, seed=51, rate=rate, J_range=(6, 11), steps_range=(200, 2000))
    log(f"serving_spec: {n} Poisson arrivals at {rate:.2f}/s (70% of capacity)")
    t0 = time.perf_counter()
    recs70 = server().run(serve.requests_from_problems(timed70, W.initial_field), realtime=True)
    torch.cuda.synchronize()
    wall70 = time.perf_counter() - t0
    at70 = serve.summarize(recs70, wall70)
    return ({"workload": f"serving configuration mix: 1-3 vortices, finest 64^2..2048^2, 200-2000 steps, "
                                  f"{n} requests per run, mixed precision",
                      "metric": "solves/s and p50/p99 latency",
                      "capacity_closed_loop": cap, "offered_req_per_s_at_70pct": rate, "at_70pct_of_capacity": at70,
                      "configured_rate_req_per_s": 50.0})


def run_serving_spec(args) -> int:
    print(json.dumps(serving_spec_leg(args)))
    return 0


def run_vapor(args) -> int:
    """Passive vapor (Section 3.6) carried by the Fujiwhara flow: each of the
    batch's 512^2 vortex solves has a vapor solve on its own adaptive grid,
    both advanced in one solve_batch per step."""
    import torch
    import workloads as W
    import paper_1604_08159_amd as m
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    seeds = [SEEDS[i % len(SEEDS)] + 100 * (i // len(SEEDS)) for i in range(args.batch)]
    pairs = []
    with torch.cuda.stream(stream):
        for sd in seeds:
            pb = W.fujiwhara_pair(sd)
            v = m.Solve(m.grid_desc(pb.J, pb.p, pb.eps), m.flow_desc(pb.nu0, pb.cs), m.MRA_MIXED, pb.m, pb.dt,
                        torch.from_numpy(W.initial_field(pb)).to(dev), stream=stream)
            r0 = torch.from_numpy(W.vapor_field(pb.N, 8.0)).to(dev)
            sc = m.ScalarSolve(v, m.grid_desc(pb.J, pb.p, 1e-4), pb.m, pb.dt, r0, eddy=True, stream=stream)
            pairs.append((v, sc))
    handles = [x for pr in pairs for x in pr]
    _, d0 = pairs[0][1].read(stream=stream)
    r0_0, _ = pairs[0][1].read(stream=stream)
    m.solve_batch(handles, [args.warmup] * len(handles), stream=stream)
    stream.synchronize()
    ev0 = [h.scalars()["evals"] for h in handles]
    t0 = time.perf_counter()
    m.solve_batch(handles, [args.steps] * len(handles), stream=stream)
    stream.synchronize()
    wall = time.perf_counter() - t0
    ev1 = [h.scalars()["evals"] for h in handles]
    dv = sum(ev1[i] - ev0[i] for i in range(0, len(handles), 2))
    ds = sum(ev1[i] - ev0[i] for i in range(1, len(handles), 2))
    r1, d1 = pairs[0][1].read(stream=stream)
    nas = [int(sc.read(dense=False, stream=stream)[1]["n_active"]) for _, sc in pairs]
    print(json.dumps({"workload": f"vapor carried by the Fujiwhara pair, 512^2, batch of {len(pairs)} vortex + "
                                  f"{len(pairs)} vapor solves, mixed precision, {args.steps} steps",
                      "metric": "active-pt RHS evals/s", "value": (dv + ds) / wall,
                      "vortex_evals_per_s": dv / wall, "vapor_evals_per_s": ds / wall,
                      "ms_per_step": wall / args.steps * 1e3, "mean_vapor_active_points": sum(nas) / len(nas),
                      "vapor_mass_rel_change": abs(d1["gamma"] - d0["gamma"]) / abs(d0["gamma"]),
                      "vapor_min_max_initial": [float(r0_0.min()), float(r0_0.max())],
                      "vapor_min_max_final": [float(r1.min()), float(r1.max())]}))
    return 0


def run_condensation(args) -> int:
    """Vapor condensation (Section 2.6's moving interface) at 512^2 in calm
    air: a batch of circular patches of radii 0.6 .. 1.3 (D_v = 1e-3, rate 1,
    kappa = 2 D_v) riding one vorticity solve at rest, dt = 0.1 to t = 80 as in
    the section's figure.  Reports the scalars' active-point evaluations per
    second, and for the R0 = 1 patch the squared radius sqrt(A / pi)^2 at
    t = 40 and 80 against the curvature law R0^2 - 2 kappa t and the extremes
    of r (the section's point: no oscillation at the interface)."""
    import torch
    import workloads as W
    import paper_1604_08159_amd as m
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    J, dt, kappa = 9, 0.1, 2 * W.COND_DV
    N = 1 << J
    radii = [0.6 + 0.1 * i for i in range(args.cond_batch)]
    with torch.cuda.stream(stream):
        v = m.Solve(m.grid_desc(J, 2, 1e-3), m.flow_desc(1e-4, 0.17), m.MRA_MIXED, 20, dt,
                    torch.zeros((N, N), dtype=torch.float64, device=dev), stream=stream)
        scs = []
        for R0 in radii:
            r0 = torch.from_numpy(W.vapor_patch(N, R0)).to(dev)
            sc = m.ScalarSolve(v, m.grid_desc(J, 2, 1e-4), 20, dt, r0, kappa0=kappa, eddy=False, stream=stream)
            sc.set_condensation(1.0, stream=stream)
            scs.append(sc)
    handles = [v] + scs
    i1 = min(range(len(radii)), key=lambda i: abs(radii[i] - 1.0))
    h = 2 * np.pi / N
    r_init, _ = scs[i1].read(stream=stream)
    R2 = {0.0: h * h * float(r_init.sum()) / np.pi}
    ev0 = sum(sc.scalars()["evals"] for sc in scs)
    wall, half = 0.0, args.cond_steps // 2
    ext = [float(r_init.min()), float(r_init.max())]
    for k in range(2):
        stream.synchronize()
        t0 = time.perf_counter()
        m.solve_batch(handles, [half] * len(handles), stream=stream)
        stream.synchronize()
        wall += time.perf_counter() - t0
        r, _ = scs[i1].read(stream=stream)
        R2[(k + 1) * half * dt] = h * h * float(r.sum()) / np.pi
        ext = [min(ext[0], float(r.min())), max(ext[1], float(r.max()))]
    ev1 = sum(sc.scalars()["evals"] for sc in scs)
    nas = [int(sc.read(dense=False, stream=stream)[1]["n_active"]) for sc in scs]
    law = {t: R2[0.0] - 2 * kappa * t for t in R2}
    print(json.dumps({"workload": f"vapor condensation, 512^2, calm air, {len(scs)} patches of radius "
                                  f"{radii[0]:.1f}..{radii[-1]:.1f}, D_v={W.COND_DV}, dt={dt}, {2 * half} steps "
                                  f"(t = {2 * half * dt:g}), mixed precision",
                      "metric": "active-pt RHS evals/s", "value": (ev1 - ev0) / wall,
                      "ms_per_step": wall / (2 * half) * 1e3, "mean_active_points": sum(nas) / len(nas),
                      "R0_1_patch_R2": {f"{t:g}": R2[t] for t in R2},
                      "curvature_law_R2": {f"{t:g}": law[t] for t in law},
                      "r_min_max": ext}))
    for sc in scs:
        sc.close()
    v.close()
    return 0


def run_three(args) -> int:
    """The three-vortex Re = 37440 configuration at 2048^2 (6-point DD, m = 30,
    noise everywhere at first, so nearly every node is active): a batch of
    args.batch3 solves with noise seeds 37440 + i, mixed precision."""
    import dataclasses
    import torch
    import workloads as W
    import paper_1604_08159_amd as m
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    pbs = [dataclasses.replace(W.three_vortex(), noise_seed=37440 + i) for i in range(args.batch3)]
    prec = m.MRA_FP32 if args.prec3 == "fp32" else m.MRA_MIXED
    solves = []
    with torch.cuda.stream(stream):
        for pb in pbs:
            solves.append(m.Solve(m.grid_desc(pb.J, pb.p, pb.eps), m.flow_desc(pb.nu0, pb.cs), prec, pb.m,
                                  pb.dt, torch.from_numpy(W.initial_field(pb)).to(dev), stream=stream))
    m.solve_batch(solves, [2] * len(solves), stream=stream)
    stream.synchronize()
    ev0 = sum(s.scalars()["evals"] for s in solves)
    t0 = time.perf_counter()
    m.solve_batch(solves, [args.steps3] * len(solves), stream=stream)
    stream.synchronize()
    wall = time.perf_counter() - t0
    ev1 = sum(s.scalars()["evals"] for s in solves)
    nas = [int(s.read(dense=False, stream=stream)[1]["n_active"]) for s in solves]
    N = pbs[0].N
    k_ms = m.time_kernel(solves, "jvp", 10, stream=stream)
    nbytes = kernel_bytes("jvp", N, sum(nas) / len(nas), 1.0, 4, pbs[0].m) * len(solves)
    print(json.dumps({"workload": f"three vortices Re=37440 + noise, finest 2048^2 (J=11), 6-point DD, eps=1e-4, "
                                  f"m=30, dt=0.002; batch of {len(solves)}, mixed precision"
                                  f"{' (Krylov basis in FP32)' if args.prec3 == 'fp32' else ''}, {args.steps3} steps",
                      "metric": "active-pt RHS evals/s", "value": (ev1 - ev0) / wall,
                      "ms_per_step": wall / args.steps3 * 1e3, "mean_active_points": sum(nas) / len(nas),
                      "active_fraction": sum(nas) / len(nas) / (N * N),
                      "jvp_ms": k_ms, "jvp_algorithmic_gbs": nbytes / (k_ms * 1e-3) / 1e9}))
    return 0


def run_longrun(args) -> int:
    """The Fujiwhara configuration over its full length (2000 steps) for one
    seed, in mixed precision and in FP64: vortex separation b(t*)/b(0) from
    the centre tracker every 20 steps, and the mixed run against the FP64 run
    at the end (vorticity, energy, enstrophy)."""
    import torch
    import workloads as W
    import paper_1604_08159_amd as m
    dev = torch.device("cuda:0")
    pb = W.fujiwhara_pair(SEEDS[0])
    gamma = pb.vortices[0].gamma
    c0 = [(v.cx, v.cy) for v in pb.vortices]
    b0 = float(np.hypot(c0[1][0] - c0[0][0], c0[1][1] - c0[0][1]))
    tc = 2.0 * np.pi * b0 * b0 / gamma
    out = {"workload": f"Fujiwhara pair Re=5000, 512^2, seed {SEEDS[0]}, {args.long_steps} steps",
           "b0": b0, "t_c": tc}
    res = {}
    for name, prec in (("mixed", m.MRA_MIXED), ("fp64", m.MRA_FP64)):
        stream = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(stream):
            s = m.Solve(m.grid_desc(pb.J, pb.p, pb.eps), m.flow_desc(pb.nu0, pb.cs), prec, pb.m, pb.dt,
                        torch.from_numpy(W.initial_field(pb)).to(dev), stream=stream)
        cs = list(c0)
        curve = []
        t0 = time.perf_counter()
        for k in range(0, args.long_steps, 20):
            n = min(20, args.long_steps - k)
            s.step(n, stream=stream)
            cs = s.track(cs, stream=stream)
            b = float(np.hypot(*[((cs[1][i] - cs[0][i] + np.pi) % (2 * np.pi)) - np.pi for i in range(2)]))
            curve.append([round((k + n) * pb.dt / tc, 4), round(b / b0, 5)])
        wall = time.perf_counter() - t0
        dense, diag = s.read(stream=stream)
        res[name] = (dense, diag)
        out[name] = {"seconds": wall, "b_over_b0_vs_tstar": curve[::5] + ([curve[-1]] if len(curve) % 5 != 1 else []),
                     "n_active_final": int(diag["n_active"]), "status": int(diag["status"])}
        s.close()
        log(f"{name}: {wall:.1f} s")
    a, da = res["fp64"]
    b_, db = res["mixed"]
    out["mixed_vs_fp64"] = {"rel_l2_vorticity": float(torch.linalg.vector_norm(a - b_) / torch.linalg.vector_norm(a)),
                            "rel_energy": abs(da["energy"] - db["energy"]) / da["energy"],
                            "rel_enstrophy": abs(da["enstrophy"] - db["enstrophy"]) / da["enstrophy"]}
    print(json.dumps(out))
    return 0


def run_implicit(args) -> int:
    """The benchmark's 512^2 batch advanced by the implicit theta-scheme
    (args.newton Newton iterations of one GMRES(m) cycle each, args.jacobian
    Jacobian), then the time discretisation error of both integrators with
    both Jacobians on seed 1000 in FP64 against an exact-Jacobian exponential
    run at a quarter of the step, with the benchmark's threshold and with
    every node active."""
    import torch
    import workloads as W
    import paper_1604_08159_amd as m
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    seeds = [SEEDS[i % len(SEEDS)] + 100 * (i // len(SEEDS)) for i in range(args.batch)]
    solves = []
    with torch.cuda.stream(stream):
        for sd in seeds:
            pb = W.fujiwhara_pair(sd)
            s = m.Solve(m.grid_desc(pb.J, pb.p, pb.eps), m.flow_desc(pb.nu0, pb.cs), m.MRA_MIXED, pb.m, pb.dt,
                        torch.from_numpy(W.initial_field(pb)).to(dev), stream=stream)
            s.set_integrator(m.MRA_THETA_NEWTON, args.theta, args.newton, stream=stream)
            s.set_jacobian(m.MRA_JAC_EXACT if args.jacobian == "exact" else m.MRA_JAC_FROZEN)
            solves.append(s)
    m.solve_batch(solves, [args.warmup] * len(solves), stream=stream)
    stream.synchronize()
    ev0 = sum(s.scalars()["evals"] for s in solves)
    t0 = time.perf_counter()
    m.solve_batch(solves, [args.steps] * len(solves), stream=stream)
    stream.synchronize()
    wall = time.perf_counter() - t0
    ev1 = sum(s.scalars()["evals"] for s in solves)
    status = [int(s.read(dense=False, stream=stream)[1]["status"]) for s in solves]
    for s in solves:
        s.close()
    log("batch done; time-discretisation check")
    pb = W.fujiwhara_pair(SEEDS[0])
    T = 50

    def run(dt, nsteps, integ, exact, eps=pb.eps):
        with torch.cuda.stream(stream):
            s = m.Solve(m.grid_desc(pb.J, pb.p, eps), m.flow_desc(pb.nu0, pb.cs), m.MRA_FP64, pb.m, dt,
                        torch.from_numpy(W.initial_field(pb)).to(dev), stream=stream)
        if integ:
            s.set_integrator(m.MRA_THETA_NEWTON, args.theta, args.newton, stream=stream)
        s.set_jacobian(m.MRA_JAC_EXACT if exact else m.MRA_JAC_FROZEN)
        s.step(nsteps, stream=stream)
        out = s.read(stream=stream)[0]
        s.close()
        return out

    variants = (("exponential", False, False), ("exponential_exact_jacobian", False, True),
                ("theta", True, False), ("theta_exact_jacobian", True, True))
    err = {}
    for tag, eps in (("", pb.eps), ("_eps0", 0.0)):
        ref = run(pb.dt / 4, 4 * T, False, True, eps)
        nrm = float(torch.linalg.vector_norm(ref))
        for name, integ, exact in variants:
            err[name + tag] = float(torch.linalg.vector_norm(run(pb.dt, T, integ, exact, eps) - ref)) / nrm
    print(json.dumps({"workload": f"Fujiwhara pair Re=5000, 512^2, batch of {len(solves)}, theta-scheme "
                                  f"theta={args.theta} by {args.newton} Newton-GMRES(m=20) iterations per step, "
                                  f"{args.jacobian} Jacobian, mixed precision, {args.steps} steps",
                      "metric": "active-pt RHS evals/s", "value": (ev1 - ev0) / wall,
                      "ms_per_step": wall / args.steps * 1e3, "failed": sum(1 for x in status if x),
                      "time_error_vs_dt_over_4": {"steps": T, "dt": pb.dt, "precision": "fp64",
                                                  "reference": "exponential step, exact Jacobian, dt/4",
                                                  "rel_l2": err}}))
    return 0


def run_families(args) -> int:
    """The unequal-strength (Section 3.3: U2/U1 = 1 .. 0.5 at equal size) and
    unequal-size (Section 3.4: equal peak vorticity, R2/R1 = 0.9, 0.7, 0.5)
    pairs at 512^2 in one batch: energy and enstrophy relative to their
    initial values and the tracked separation at the paper's output times
    9.375 h, 18.75 h and 37.5 h.  Time is converted with R/U1: 100 km at
    46.8 m/s against the model's r0 / (Gamma1 / (2 pi r0))."""
    import torch
    import workloads as W
    import paper_1604_08159_amd as m
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    pbs = [W.unequal_strength_pair(r) for r in W.E6_U2_OVER_U1] + [W.unequal_size_pair(r) for r in W.E7_R2_OVER_R1]
    r0 = pbs[0].vortices[0].r0
    t_model_per_hour = (r0 / (1.0 / (2 * np.pi * r0))) / (100e3 / 46.8 / 3600.0)
    marks = [int(round(hrs * t_model_per_hour / pbs[0].dt)) for hrs in (9.375, 18.75, 37.5)]
    if args.fam_steps <= 0:
        args.fam_steps = marks[-1]
    marks = [min(k, args.fam_steps) for k in marks]
    solves = []
    with torch.cuda.stream(stream):
        for pb in pbs:
            solves.append(m.Solve(m.grid_desc(pb.J, pb.p, pb.eps), m.flow_desc(pb.nu0, pb.cs), m.MRA_MIXED, pb.m,
                                  pb.dt, torch.from_numpy(W.initial_field(pb)).to(dev), stream=stream))
    d0 = [s.read(dense=False, stream=stream)[1] for s in solves]
    cs = [[(v.cx, v.cy) for v in pb.vortices] for pb in pbs]
    hist = [[] for _ in pbs]
    done, wall, ev = 0, 0.0, 0.0
    ev0 = sum(s.scalars()["evals"] for s in solves)
    for target in sorted(set(list(range(50, args.fam_steps + 1, 50)) + marks)):
        t0 = time.perf_counter()
        m.solve_batch(solves, [target - done] * len(solves), stream=stream)
        stream.synchronize()
        wall += time.perf_counter() - t0
        done = target
        for i, s in enumerate(solves):
            cs[i] = s.track(cs[i], stream=stream)
            if target in marks:
                _, d = s.read(dense=False, stream=stream)
                b = float(np.hypot(*[((cs[i][1][k] - cs[i][0][k] + np.pi) % (2 * np.pi)) - np.pi for k in range(2)]))
                b0 = abs(pbs[i].vortices[1].cx - pbs[i].vortices[0].cx)
                hist[i].append({"hours": round(target * pbs[i].dt / t_model_per_hour, 3),
                                "E_over_E0": d["energy"] / d0[i]["energy"],
                                "Z_over_Z0": d["enstrophy"] / d0[i]["enstrophy"],
                                "b_over_b0": b / b0, "n_active": int(d["n_active"]), "status": int(d["status"])})
        log(f"families: {done} steps")
    ev = sum(s.scalars()["evals"] for s in solves) - ev0
    print(json.dumps({"workload": f"unequal-strength (U2/U1 = 1, 0.80, 0.70, 0.60, 0.50) and unequal-size "
                                  f"(R2/R1 = 0.9, 0.7, 0.5) pairs, Re=37440, 512^2, batch of {len(pbs)}, mixed "
                                  f"precision, {args.fam_steps} steps",
                      "metric": "active-pt RHS evals/s", "value": ev / wall, "wall_s": wall,
                      "model_time_per_hour": t_model_per_hour,
                      "runs": {pb.name: h for pb, h in zip(pbs, hist)}}))
    return 0


def make_batch(m, W, dev, stream, pbs, prec):
    import torch
    solves = []
    with torch.cuda.stream(stream):
        for pb in pbs:
            solves.append(m.Solve(m.grid_desc(pb.J, pb.p, pb.eps), m.flow_desc(pb.nu0, pb.cs), prec, pb.m, pb.dt,
                                  torch.from_numpy(W.initial_field(pb)).to(dev), stream=stream))
    return solves


def timed_batch(m, solves, stream, warmup: int, steps: int) -> dict:
    """warmup untimed steps, then `steps` timed steps of the batch (graph
    replay), bracketed by device synchronisation."""
    import torch
    n = len(solves)
    m.solve_batch(solves, [warmup] * n, stream=stream)
    stream.synchronize()
    ev0 = sum(s.scalars()["evals"] for s in solves)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.solve_batch(solves, [steps] * n, stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev1 = sum(s.scalars()["evals"] for s in solves)
    diags = [s.read(dense=False, stream=stream)[1] for s in solves]
    if any(d["status"] != 0 for d in diags):
        raise RuntimeError(f"a solve reported status {[d['status'] for d in diags]}")
    return {"value": (ev1 - ev0) / wall, "wall": wall, "ms_per_step": wall / steps * 1e3,
            "n_active": [int(d["n_active"]) for d in diags]}


def step_roofline(m, solves, stream, N: int, m_kry: int, bulk_esz: int) -> dict:
    """Per-phase GPU time of one more step (mra_step_profile) turned into
    achieved bandwidth per kernel, the dominant kernel and the fraction of the
    residual and product pipeline."""
    phi_t = active_tile_fraction(solves, N)
    nas = [int(s.read(dense=False, stream=stream)[1]["n_active"]) for s in solves]   # the profiled step's N_a
    na = sum(nas) / len(nas)
    prof = m.step_profile(solves, stream=stream)
    gsb = sum(gs_bytes(a, m_kry) for a in nas)
    kern = roofline_from_profile(prof, N, na, phi_t, len(solves), bulk_esz, m_kry, gs_step_bytes=gsb)
    kern["gram_schmidt"]["cgs2_two_reads_per_pass_bytes_per_launch"] = \
        kernel_bytes("gram_schmidt", N, na, phi_t, 8, m_kry) * len(solves)
    step_ms = sum(prof.values())
    dom = max(kern, key=lambda k: kern[k]["avg_launch_ms"] * kern[k]["launches_per_step"])
    # phases with no byte model (phi_1, update, regrid, norm) keep their share
    others = {k: {"ms_per_step": v, "share_of_step": v / step_ms} for k, v in prof.items() if k not in kern}
    return {"phi_t": phi_t, "n_active_mean": na, "profile_ms": prof, "step_ms_profiled": step_ms,
            "kernels": kern, "other_phases": others, "dominant": dom,
            "rhs_pipeline": rhs_pipeline(kern, m_kry)}


def copy_ceiling(dev) -> float:
    """Plain device copy: the byte-counter scale of profiled runs (64 MiB) and,
    timed, the practical streaming ceiling of this device (1 GiB)."""
    import torch
    cal_a = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
    cal_b = torch.empty_like(cal_a)
    cal_b.copy_(cal_a)
    torch.cuda.synchronize()
    big_a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    big_b = torch.empty_like(big_a)
    big_b.copy_(big_a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        big_b.copy_(big_a)
    e1.record()
    e1.synchronize()
    gbs = 2 * big_a.numel() * 4 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del cal_a, cal_b, big_a, big_b
    torch.cuda.empty_cache()
    return gbs


def three_leg(args, m, W, dev, tmpdir: str) -> dict:
    """The headline: the three-vortex configuration at 2048^2, a batch of
    args.batch3 solves (noise seeds 37440 + i), mixed precision."""
    import dataclasses
    import torch
    stream = torch.cuda.Stream(device=dev)
    pbs = [dataclasses.replace(W.three_vortex(), noise_seed=37440 + i) for i in range(args.batch3)]
    pb = pbs[0]
    solves = make_batch(m, W, dev, stream, pbs, m.MRA_MIXED)
    log(f"three-vortex 2048^2 batch of {len(solves)}: {args.warmup} + {args.steps} steps")
    t = timed_batch(m, solves, stream, args.warmup, args.steps)
    rl = step_roofline(m, solves, stream, pb.N, pb.m, 4)
    k_jvp = m.time_kernel(solves, "jvp", 10, stream=stream)
    out = {"timed": t, "roofline": rl, "jvp_back_to_back_ms": k_jvp}
    if args.no_compare:
        for s in solves:
            s.close()
        return out
    # mixed against the FP64 GPU path over the same steps (warm-up, timed, profiled)
    nst = args.warmup + args.steps + 1
    ref = make_batch(m, W, dev, stream, [pb], m.MRA_FP64)[0]
    ref.step(nst, stream=stream)
    a, da = ref.read(stream=stream)
    b, db = solves[0].read(stream=stream)
    _, ma, _, _ = ref.active_set()
    _, mb, _, _ = solves[0].active_set()
    out["mixed_vs_fp64_gpu"] = {"steps": nst, **compare_fields(a.cpu().numpy(), b.cpu().numpy(), da, db),
                                "mask_flips": int((ma != mb).sum()), "n_active_fp64": int(da["n_active"])}
    ref.close()
    for s in solves:
        s.close()
    del a, b
    torch.cuda.empty_cache()
    return out


def three_oracle_accuracy(m, W, dev, tmpdir: str) -> dict:
    """The mixed path's residual and product at 2048^2 against the FP64 oracle
    on the same FP64 inputs (the initial state of seed 37440 and a unit-norm
    Krylov-like vector), from the oracle's cpu_baseline sample."""
    import torch
    pb = W.three_vortex()
    ld = lambda n: np.load(os.path.join(tmpdir, n + ".npy"))
    omega, fi, mask, F, v, Av = ld("omega"), ld("fi"), ld("mask"), ld("F"), ld("v"), ld("Av")
    n = fi.size
    g, f = m.grid_desc(pb.J, pb.p, pb.eps), m.flow_desc(pb.nu0, pb.cs)
    t = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)
    mk, fk, nk = t(mask, torch.uint8), t(fi, torch.int32), t(np.array([n]), torch.int64)
    out = torch.empty(n, dtype=torch.float64, device=dev)
    m.collocation_rhs(g, f, m.MRA_MIXED, mk, fk, nk, t(omega), None, out)
    eF = float(np.abs(out.cpu().numpy() - F).max() / np.abs(F).max())
    m.collocation_rhs(g, f, m.MRA_MIXED, mk, fk, nk, t(omega), t(v), out)
    eJ = float(np.abs(out.cpu().numpy() - Av).max() / np.abs(Av).max())
    return {"residual_max_rel": eF, "product_max_rel": eJ, "n_active": n, "tolerance": 2e-5,
            "within": eF <= 2e-5 and eJ <= 2e-5,
            "note": "max |GPU - oracle| / max |oracle| at every active node of 2048^2; the product takes the "
                    "FP64 vector rounded to FP32, the residual runs in FP64"}


def pair_leg(args, m, W, dev, tmpdir: str, orc: dict) -> dict:
    """The 512^2 Fujiwhara batch of 24 in mixed precision, with its accuracy
    against the FP64 oracle after the warm-up and timed steps."""
    import torch
    stream = torch.cuda.Stream(device=dev)
    pbs = [W.fujiwhara_pair(sd) for sd in SEEDS[:args.batch]]
    solves = make_batch(m, W, dev, stream, pbs, m.MRA_MIXED)
    log(f"Fujiwhara 512^2 batch of {len(solves)}: {args.warmup} + {args.steps} steps")
    t = timed_batch(m, solves, stream, args.warmup, args.steps)
    dense, diag = solves[0].read(stream=stream)
    _, mask, _, _ = solves[0].active_set()
    ref = np.load(os.path.join(tmpdir, "pair_ref.npy"))
    rmask = np.load(os.path.join(tmpdir, "pair_mask.npy"))
    acc = {"seed": SEEDS[0], "steps": args.warmup + args.steps,
           **compare_fields(ref, dense.cpu().numpy(), orc["diag"], diag),
           "mask_flips": int((mask.cpu().numpy() != rmask).sum()), "n_active_oracle": orc["n_active"],
           "n_active_mixed": int(diag["n_active"]), "tolerance": 1e-5}
    acc["within"] = acc["rel_l2_vorticity"] <= 1e-5
    rl = step_roofline(m, solves, stream, pbs[0].N, pbs[0].m, 4)
    for s in solves:
        s.close()
    return {"workload": f"Fujiwhara pair Re=5000, finest 512^2 (J=9), 4-point DD, eps=1e-4, m=20, dt=0.01; "
                        f"batch of {len(pbs)} seeded solves, mixed precision",
            "metric": METRIC, "value": t["value"], "ms_per_step": t["ms_per_step"], "steps": args.steps,
            "mean_active_points": sum(t["n_active"]) / len(t["n_active"]),
            "accuracy_vs_oracle": acc,
            "roofline_dominant": {"kernel": rl["dominant"], **rl["kernels"][rl["dominant"]]},
            "kernels": rl["kernels"], "other_phases": rl["other_phases"],
            "jvp": rl["kernels"]["jvp"], "rhs_pipeline": rl["rhs_pipeline"], "phi_t": rl["phi_t"],
            "fp64_per_solve_gpu": fp64_per_solve(m, W, dev, max(10, args.steps // 2)),
            "cpu_baseline": {"value": orc["evals"] / orc["sec"], "unit": METRIC, "cores": 1, "kind": "oracle",
                             "sample": f"{args.warmup + args.steps} steps of seed {SEEDS[0]}, {orc['sec']:.1f} s"}}


def adapted_leg(args, m, W, dev) -> dict:
    """The 512^2 Fujiwhara batch with the level-adapted evaluation (the
    residual and products at the active nodes on the stencils of each node's
    local level; Pi and the Poisson solve stay dense): throughput, the
    products' stencil time against the dense tile stencil of the same batch,
    and the distance of the adapted run from the dense one after the timed
    steps."""
    import torch
    stream = torch.cuda.Stream(device=dev)
    pbs = [W.fujiwhara_pair(sd) for sd in SEEDS[:args.batch]]
    out = {}
    fields = {}
    for name, ev in (("dense", m.MRA_EVAL_DENSE), ("adapted", m.MRA_EVAL_ADAPTED)):
        solves = make_batch(m, W, dev, stream, pbs, m.MRA_MIXED)
        for s in solves:
            s.set_evaluation(ev)
        t = timed_batch(m, solves, stream, args.warmup, args.steps)
        dense, diag = solves[0].read(stream=stream)
        fields[name] = (dense.cpu().numpy(), diag)
        prof = m.step_profile(solves, stream=stream)
        out[name] = {"value": t["value"], "ms_per_step": t["ms_per_step"],
                     "product_stencil_ms": prof["jvp"] / pbs[0].m, "residual_stencil_ms": prof["res_stencil"],
                     "step_profile_ms": sum(prof.values())}
        for s in solves:
            s.close()
    a, da = fields["dense"]
    b, db = fields["adapted"]
    out["adapted_vs_dense"] = {"steps": args.warmup + args.steps, **compare_fields(a, b, da, db),
                               "note": "the two evaluations are different discrete operators (distance O(eps))"}
    out["workload"] = (f"Fujiwhara pair Re=5000, 512^2, batch of {len(pbs)}, mixed precision, level-adapted "
                       f"evaluation against the dense one")
    return out


def run_drift_three(args) -> int:
    import torch
    import workloads as W
    import paper_1604_08159_amd as m
    print(json.dumps(drift_three_leg(m, W, torch.device("cuda:0"), args.long_steps3, args.noise3)))
    return 0


def drift_three_leg(m, W, dev, steps: int, noise_amp: float = None) -> dict:
    """The three-vortex 2048^2 configuration over its full length for noise
    seed 37440: one solve in mixed precision against one in FP64, both on the
    GPU, and beside it an FP64 solve whose initial field carries relative
    white noise of 1e-10 against the same FP64 run (the threshold's own
    sensitivity), compared every 100 steps up to step 1000 and every 500
    after (vorticity, energy, enstrophy, mask flips)."""
    import dataclasses
    import torch
    pb = W.three_vortex()
    if noise_amp is not None:
        pb = dataclasses.replace(pb, noise_amp=noise_amp)
    w0 = W.initial_field(pb)
    w0p = w0 * (1.0 + 1e-10 * np.random.default_rng(7).standard_normal(w0.shape))
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        mk = lambda prec, w: m.Solve(m.grid_desc(pb.J, pb.p, pb.eps), m.flow_desc(pb.nu0, pb.cs), prec, pb.m,
                                     pb.dt, torch.from_numpy(w).to(dev), stream=stream)
        runs = {"fp64": mk(m.MRA_FP64, w0), "mixed": mk(m.MRA_MIXED, w0), "perturbed_fp64": mk(m.MRA_FP64, w0p)}
    t0 = time.perf_counter()
    curve, done = [], 0
    first_flip = {"mixed": None, "perturbed_fp64": None}
    while done < steps:
        k = min(100 if done < 1000 else 500, steps - done)
        m.solve_batch(list(runs.values()), [k] * len(runs), stream=stream)
        done += k
        got = {}
        for name, sv in runs.items():
            dense, diag = sv.read(stream=stream)
            got[name] = (dense.cpu().numpy(), diag, sv.active_set()[1].cpu().numpy())
        a, da, ma = got["fp64"]
        row = {"step": done, "n_active_fp64": int(da["n_active"])}
        for name in ("mixed", "perturbed_fp64"):
            b, db, mb = got[name]
            row[name] = {**compare_fields(a, b, da, db), "mask_flips": int((ma != mb).sum())}
            if row[name]["mask_flips"] and first_flip[name] is None:
                first_flip[name] = done
        curve.append(row)
        log(f"step {done}: mixed {row['mixed']['rel_l2_vorticity']:.2e} ({row['mixed']['mask_flips']} flips), "
            f"perturbed FP64 {row['perturbed_fp64']['rel_l2_vorticity']:.2e} "
            f"({row['perturbed_fp64']['mask_flips']} flips), N_a {row['n_active_fp64']} "
            f"({time.perf_counter() - t0:.0f} s)")
    for sv in runs.values():
        sv.close()
    return {"workload": f"three vortices Re=37440 + noise of amplitude {pb.noise_amp:g} (seed 37440), 2048^2, "
                        f"6-point DD, m=30, dt=0.002, {steps} steps; mixed against FP64 on the GPU",
            "reference": "the FP64 GPU path", "final": curve[-1], "first_flip_by": first_flip, "tolerance": 1e-5,
            "curve": curve, "seconds": time.perf_counter() - t0}


def drift_leg(m, W, dev, steps: int, every: int = 100) -> dict:
    """Mixed precision against FP64 over the Fujiwhara configuration's full
    length for one seed, both on the GPU (the FP64 GPU path is pinned to the
    oracle by the parity tests: 2.4e-15 over the plain configuration's 100
    steps), and beside it the flow's own sensitivity: FP64 runs whose initial
    vortex moves by 1e-9 (a smooth perturbation, about the size of the
    difference the mixed precision leaves after the first steps) or whose
    initial field carries white noise of relative size 1e-10, each against
    the unperturbed FP64 run.  Thresholding is discontinuous: once the runs
    differ enough to move one detail across tau they carry different active
    sets.  Every `every` steps: relative L2 of each pair and its mask flips."""
    import dataclasses
    import torch
    pb = W.fujiwhara_pair(SEEDS[0])
    w0 = W.initial_field(pb)
    v0 = pb.vortices[0]
    shifted = dataclasses.replace(pb, vortices=(dataclasses.replace(v0, cx=v0.cx + 1e-9),) + pb.vortices[1:])
    w0s = W.initial_field(shifted)
    rng = np.random.default_rng(7)
    w0p = w0 * (1.0 + 1e-10 * rng.standard_normal(w0.shape))
    stream = torch.cuda.Stream(device=dev)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        mk = lambda prec, w: m.Solve(m.grid_desc(pb.J, pb.p, pb.eps), m.flow_desc(pb.nu0, pb.cs), prec, pb.m,
                                     pb.dt, torch.from_numpy(w).to(dev), stream=stream)
        ref, mix, per, sft = mk(m.MRA_FP64, w0), mk(m.MRA_MIXED, w0), mk(m.MRA_FP64, w0p), mk(m.MRA_FP64, w0s)
    runs = (("fp64", ref), ("mixed", mix), ("perturbed_fp64", per), ("shifted_fp64", sft))
    curve = []
    first_flip = {"mixed": None, "perturbed_fp64": None, "shifted_fp64": None}
    done = 0
    while done < steps:
        k = min(every, steps - done)
        m.solve_batch([r for _, r in runs], [k] * len(runs), stream=stream)
        done += k
        fields = {}
        for name, s in runs:
            dense, diag = s.read(stream=stream)
            _, mask, _, _ = s.active_set()
            fields[name] = (dense.cpu().numpy(), diag, mask.cpu().numpy())
        a, da, ma = fields["fp64"]
        row = {"step": done}
        for name in ("mixed", "perturbed_fp64", "shifted_fp64"):
            b, db, mb = fields[name]
            flips = int((ma != mb).sum())
            row[name] = {"rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(a)), "mask_flips": flips}
            if flips and first_flip[name] is None:
                first_flip[name] = done
        curve.append(row)
    a, da, ma = fields["fp64"]
    b, db, mb = fields["mixed"]
    c, dc, mc = fields["perturbed_fp64"]
    e, de, me = fields["shifted_fp64"]
    for _, s in runs:
        s.close()
    return {"seed": SEEDS[0], "steps": steps, "reference": "the FP64 GPU path", **compare_fields(a, b, da, db),
            "mask_flips": int((ma != mb).sum()), "n_active_fp64": int(da["n_active"]),
            "n_active_mixed": int(db["n_active"]),
            "perturbed_fp64_vs_fp64": {"perturbation": "relative 1e-10 N(0,1) on the initial field",
                                       **compare_fields(a, c, da, dc), "mask_flips": int((ma != mc).sum())},
            "shifted_fp64_vs_fp64": {"perturbation": "the first vortex's centre moved by 1e-9 in x",
                                     "initial_rel_l2": float(np.linalg.norm(w0s - w0) / np.linalg.norm(w0)),
                                     **compare_fields(a, e, da, de), "mask_flips": int((ma != me).sum())},
            "first_flip_by": first_flip, "every": every, "curve": curve, "seconds": time.perf_counter() - t0}


def run_fujiwhara(args) -> int:
    """The 512^2 Fujiwhara batch alone, with its oracle accuracy and baseline."""
    import torch
    import paper_1604_08159_amd as m
    import workloads as W
    tmp = tempfile.TemporaryDirectory(prefix="mra_bench_")
    orc = start_oracle(ORACLE_PAIR.format(root=ROOT, seed=SEEDS[0], steps=args.warmup + args.steps, d=tmp.name))
    r = finish_oracle(orc)
    print(json.dumps(pair_leg(args, m, W, torch.device("cuda:0"), tmp.name, r)))
    tmp.cleanup()
    return 0


def run_default(args) -> int:
    """The headline line: the three-vortex 2048^2 batch, with the roofline of
    its step, the oracle beside it, and the sub-records of the other
    configurations."""
    import torch
    import paper_1604_08159_amd as m
    import workloads as W
    T0 = time.perf_counter()
    dev = torch.device("cuda:0")
    tmp = tempfile.TemporaryDirectory(prefix="mra_bench_")
    orc3 = orc2 = None
    if not args.no_cpu:
        orc3 = start_oracle(ORACLE_THREE.format(root=ROOT, seed=37440, nprod=THREE_CPU_PRODUCTS, d=tmp.name))
        orc2 = start_oracle(ORACLE_PAIR.format(root=ROOT, seed=SEEDS[0], steps=args.warmup + args.steps,
                                               d=tmp.name))
    ceiling = copy_ceiling(dev)
    three = three_leg(args, m, W, dev, tmp.name)
    t, rl = three["timed"], three["roofline"]
    dom = rl["dominant"]
    kd = rl["kernels"][dom]
    out = {
        "metric": METRIC, "value": t["value"], "unit": METRIC, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "three Gaussian vortices at Re=37440 plus seeded white noise of amplitude 1e-3, "
                               "finest 2048^2 (J=11), 6-point DD, eps=1e-4, Cs=0.17, m=30, dt=0.002; "
                               f"batch of {args.batch3} solves (noise seeds 37440..{37440 + args.batch3 - 1}), "
                               "mixed precision (FP32 products, FP64 residual, Krylov and regrid)",
                   "batch": args.batch3, "finest_points": 1 << 22,
                   "mean_active_points": sum(t["n_active"]) / len(t["n_active"]),
                   "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": kd["achieved_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": kd["frac"], "traffic": measured_traffic(dom),
                     "avg_launch_ms": kd["avg_launch_ms"], "launches_per_step": kd["launches_per_step"],
                     "algorithmic_bytes_per_launch": kd["algorithmic_bytes_per_launch"],
                     "share_of_step": kd["share_of_step"], "active_tile_fraction": rl["phi_t"],
                     "mean_active_points": rl["n_active_mean"],
                     "timing": "HIP events after every phase of one step on the step's stream (mra_step_profile)",
                     "copy_ceiling_gbs": ceiling, "frac_of_copy_ceiling": kd["achieved_gbs"] / ceiling},
        "rhs_pipeline": rl["rhs_pipeline"],
        "kernels": rl["kernels"], "other_phases": rl["other_phases"],
        "jvp_back_to_back_ms": three["jvp_back_to_back_ms"],
        "finest_pt_evals_per_s": t["value"] * (1 << 22) / (sum(t["n_active"]) / len(t["n_active"])),
        "mixed_vs_fp64_gpu": three.get("mixed_vs_fp64_gpu"),
    }
    log("three-vortex leg done")
    if orc3 is not None:
        r3 = finish_oracle(orc3)
        out["cpu_baseline"] = {"value": r3["evals"] / r3["sec"], "unit": METRIC, "cores": 1, "kind": "oracle",
                               "sample": f"one residual and {THREE_CPU_PRODUCTS} Jacobian-vector products of the FP64 oracle at "
                                         f"2048^2 on the initial state of noise seed 37440 "
                                         f"({r3['n_active']} active nodes), one core, {r3['sec']:.1f} s"}
        out["accuracy_vs_oracle"] = three_oracle_accuracy(m, W, dev, tmp.name)
    if not args.no_sub:
        r2 = finish_oracle(orc2) if orc2 is not None else None
        if r2 is not None:
            out["fujiwhara512"] = pair_leg(args, m, W, dev, tmp.name, r2)
        out["drift_fujiwhara512"] = drift_leg(m, W, dev, args.long_steps)
        log("drift leg done")
        out["drift_three2048"] = drift_three_leg(m, W, dev, args.long_steps3)
        log("2048^2 drift leg done")
        out["adapted_fujiwhara512"] = adapted_leg(args, m, W, dev)
        log("adapted leg done")
        out["ensemble"] = ensemble_leg(args, not args.no_cpu)
        log("ensemble leg done")
        out["serving"] = serving_spec_leg(args)
        log("serving leg done")
    tmp.cleanup()
    out["bench_wall_s"] = time.perf_counter() - T0
    print(json.dumps(out))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["default", "fujiwhara", "adapted", "ensemble", "serving", "vapor", "three2048",
                                           "longrun", "implicit", "families", "serving_spec", "condensation", "drift_three"],
                    default="default",
                    help="default: the three-vortex 2048^2 headline with every sub-record")
    ap.add_argument("--no-sub", action="store_true", help="default workload: the headline only")
    ap.add_argument("--no-compare", action="store_true",
                    help="default workload: skip the FP64 GPU comparison run (kernel profiles of the step)")
    ap.add_argument("--batch3", type=int, default=2)
    ap.add_argument("--steps3", type=int, default=10)
    ap.add_argument("--tune-cache", default="", help="ensemble: JSON cache of the tile autotuner")
    ap.add_argument("--cond-batch", type=int, default=8)
    ap.add_argument("--cond-steps", type=int, default=800)
    ap.add_argument("--prec3", choices=["mixed", "fp32"], default="mixed",
                    help="three2048: fp32 stores the Krylov basis in FP32")
    ap.add_argument("--long-steps", type=int, default=2000)
    ap.add_argument("--long-steps3", type=int, default=5000, help="drift_three: steps of the 2048^2 run")
    ap.add_argument("--noise3", type=float, default=None, help="drift_three: noise amplitude in place of 1e-3")
    ap.add_argument("--fam-steps", type=int, default=0, help="0: up to 37.5 h")
    ap.add_argument("--spec-requests", type=int, default=24)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--newton", type=int, default=2)
    ap.add_argument("--jacobian", choices=["frozen", "exact"], default="frozen")
    ap.add_argument("--solves", type=int, default=256)
    ap.add_argument("--ens-steps", type=int, default=200)
    ap.add_argument("--round-steps", type=int, default=20)
    ap.add_argument("--hbm-gb", type=int, default=200)
    ap.add_argument("--cap-frac", type=float, default=0.25,
                    help="ensemble: active-node capacity of the second run's arenas, as a fraction of N^2")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--max-J", type=int, default=10)
    ap.add_argument("--min-steps", type=int, default=20)
    ap.add_argument("--max-steps", type=int, default=200)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--prec", choices=["mixed", "fp64", "fp32"], default="mixed",
                    help="fp32: mixed with the Krylov basis stored in FP32")
    ap.add_argument("--batch", type=int, default=len(SEEDS))
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 (independent solves shard across GPUs by a host router)"}))
        return 2
    if args.workload == "ensemble":
        return run_ensemble(args)
    if args.workload == "serving":
        return run_serving(args)
    if args.workload == "vapor":
        return run_vapor(args)
    if args.workload == "condensation":
        return run_condensation(args)
    if args.workload == "three2048":
        return run_three(args)
    if args.workload == "serving_spec":
        return run_serving_spec(args)
    if args.workload == "families":
        return run_families(args)
    if args.workload == "implicit":
        return run_implicit(args)
    if args.workload == "drift_three":
        return run_drift_three(args)
    if args.workload == "longrun":
        return run_longrun(args)

    if args.workload == "fujiwhara":
        return run_fujiwhara(args)
    if args.workload == "adapted":
        import torch
        import paper_1604_08159_amd as m
        import workloads as W
        print(json.dumps(adapted_leg(args, m, W, torch.device("cuda:0"))))
        return 0
    return run_default(args)


if __name__ == "__main__":
    sys.exit(main())
