"""Benchmark of the wavelet-collocation vortex step on one MI355X.

Workload: the Fujiwhara pair at Re = 5000 on a 512 x 512 finest grid
(J = 9), 4-point DD, threshold 1e-4, Krylov dimension 20, dt = 0.01; a batch
of 24 solves whose radii and separations are drawn from seeds 1000..1023.
One step = one exponential Rosenbrock-Euler step of every solve of the batch
(residual, 20 Jacobian-vector products, Arnoldi, phi_1, update and FP64
regrid), launched together through solve_batch and replayed as a HIP graph.

Metric: active-point residual evaluations per second, summed over the batch
((1 + m_eff) N_a per solve and step, counted on the device).  Also reported:
the roofline fraction of the dominant kernel (HIP events on the launching
stream) and the FP64 CPU oracle timed on a bounded sample on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec mixed|fp64]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CALIB_BYTES = 64 << 20          # plain device copy of known size (PMC byte-counter scale)
KERNEL_SOURCES = {"jvp": "k_stencil.hip", "rhs": "k_stencil.hip", "fft_rows": "k_fft.hip",
                  "fft_cols": "k_fft.hip", "fft_rows_inv": "k_fft.hip", "prolong_finest": "k_transform.hip",
                  "forward": "k_transform.hip"}
SEEDS = list(range(1000, 1024))   # 24 resident solves: the throughput-optimal batch on one MI355X
METRIC = "active-pt RHS evals/s"


def kernel_bytes(name: str, N: int, na: int, tiles_active_frac: float, nbatch: int, esz: int) -> float:
    """Algorithmic HBM bytes of one launch of a step kernel for the batch."""
    nf = N * N
    if name == "jvp":
        # psi~, v~, w~, u, v, nu_e on active tiles + rank map; J v out (FP64)
        per = (6 * esz + 4) * nf * tiles_active_frac + 8 * na
    elif name == "rhs":
        # u, v, w~ in; nu_e out; rank map; F out (FP64)
        per = (4 * esz + 4) * nf + 8 * na
    elif name == "fft_rows":
        per = esz * nf + 2 * esz * (N // 2 + 1) * N
    elif name == "fft_rows_inv":
        # the products' pass: psi~ alone
        per = esz * nf + 2 * esz * (N // 2 + 1) * N
    elif name == "fft_cols":
        # spectrum in, psi~ spectrum out
        per = 2 * (2 * esz * (N // 2 + 1) * N)
    elif name == "prolong_finest":
        lev = 3 * nf // 4
        per = lev * (1 + esz)          # mask byte + written value (inputs are re-read coarse values)
    elif name == "forward":
        per = nf * (8 + 8)
    else:
        raise KeyError(name)
    return per * nbatch


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
    """The same workload, one solve at a time, all bulk fields in FP64."""
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


def accuracy_vs_fp64(m, W, dev, solve, seed: int, steps: int) -> dict:
    """Mixed-precision solve against the same solve run with FP64 bulk fields
    for the same number of steps: relative L2 of the vorticity field and the
    relative differences of energy and enstrophy."""
    import torch
    stream = torch.cuda.Stream(device=dev)
    pb = W.fujiwhara_pair(seed)
    with torch.cuda.stream(stream):
        w0 = torch.from_numpy(W.initial_field(pb)).to(dev)
        ref = m.Solve(m.grid_desc(pb.J, pb.p, pb.eps), m.flow_desc(pb.nu0, pb.cs), m.MRA_FP64, pb.m, pb.dt, w0,
                      stream=stream)
    ref.step(steps, stream=stream)
    a, da = ref.read(stream=stream)
    b, db = solve.read(stream=stream)
    stream.synchronize()
    ref.close()
    rel = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(a))
    return {"seed": seed, "steps": steps, "rel_l2_vorticity": rel,
            "rel_energy": abs(da["energy"] - db["energy"]) / da["energy"],
            "rel_enstrophy": abs(da["enstrophy"] - db["enstrophy"]) / da["enstrophy"],
            "n_active_fp64": int(da["n_active"]), "n_active_mixed": int(db["n_active"]),
            "tolerance": 1e-5, "within": rel <= 1e-5}


def cpu_baseline(steps: int) -> dict:
    """The FP64 oracle on one solve of the batch, single-threaded, timed here."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               NUMEXPR_NUM_THREADS="1")
    code = (
        "import json,sys,time; sys.path.insert(0, %r)\n"
        "import workloads as W\n"
        "from oracle import krylov as ok, ops as oo\n"
        "pb = W.fujiwhara_pair(%d)\n"
        "g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps); fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)\n"
        "st = ok.init_state(W.initial_field(pb), g)\n"
        "ev = 0; t0 = time.perf_counter()\n"
        "for _ in range(%d):\n"
        "    na = st.omega_M.size; st = ok.step(st, g, fl, pb.m, pb.dt); ev += (1 + st.last_m_eff) * na\n"
        "dt = time.perf_counter() - t0\n"
        "print(json.dumps({'evals': ev, 'sec': dt}))\n" % (ROOT, SEEDS[0], steps))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    r = json.loads(out.stdout.strip().splitlines()[-1])
    return {"value": r["evals"] / r["sec"], "unit": "active-pt RHS evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of one 512^2 Fujiwhara solve (seed {SEEDS[0]}), FP64 NumPy/SciPy, "
                      f"{r['sec']:.1f} s"}


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


def run_ensemble(args) -> int:
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
    cpu = None if args.no_cpu else ensemble_cpu_baseline(probs)
    print(json.dumps({"workload": f"ensemble of {len(probs)} two-vortex solves, finest 128^2..1024^2, "
                                  f"{args.ens_steps} steps each, mixed precision, one GPU",
                      "metric": "ensemble solves/s", "value": summ["solves_per_s"], "wall_s": wall,
                      "active_pt_evals_per_s": summ["active_pt_evals_per_s"], "failed": summ["failed"],
                      "fp64_per_solve_gpu": {"solves_per_s_extrapolated": len(probs) / fp64_total,
                                             "sec_per_step_by_J": per_step,
                                             "note": "one warmed solve per size timed over 8 steps, "
                                                     "applied to every solve's step count"},
                      "autotune": tuned,
                      "cpu_baseline": cpu}))
    untune_tiles(tuned)
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


def run_serving_spec(args) -> int:
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
    print(json.dumps({"workload": f"serving configuration mix: 1-3 vortices, finest 64^2..2048^2, 200-2000 steps, "
                                  f"{n} requests per run, mixed precision",
                      "metric": "solves/s and p50/p99 latency",
                      "capacity_closed_loop": cap, "offered_req_per_s_at_70pct": rate, "at_70pct_of_capacity": at70,
                      "configured_rate_req_per_s": 50.0}))
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
    nbytes = kernel_bytes("jvp", N, int(sum(nas) / len(nas)), 1.0, len(solves), 4)
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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["fujiwhara", "ensemble", "serving", "vapor", "three2048", "longrun",
                                           "implicit", "families", "serving_spec", "condensation"],
                    default="fujiwhara")
    ap.add_argument("--batch3", type=int, default=2)
    ap.add_argument("--steps3", type=int, default=10)
    ap.add_argument("--tune-cache", default="", help="ensemble: JSON cache of the tile autotuner")
    ap.add_argument("--cond-batch", type=int, default=8)
    ap.add_argument("--cond-steps", type=int, default=800)
    ap.add_argument("--prec3", choices=["mixed", "fp32"], default="mixed",
                    help="three2048: fp32 stores the Krylov basis in FP32")
    ap.add_argument("--long-steps", type=int, default=2000)
    ap.add_argument("--fam-steps", type=int, default=0, help="0: up to 37.5 h")
    ap.add_argument("--spec-requests", type=int, default=40)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--newton", type=int, default=2)
    ap.add_argument("--jacobian", choices=["frozen", "exact"], default="frozen")
    ap.add_argument("--solves", type=int, default=256)
    ap.add_argument("--ens-steps", type=int, default=200)
    ap.add_argument("--round-steps", type=int, default=20)
    ap.add_argument("--hbm-gb", type=int, default=200)
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--max-J", type=int, default=10)
    ap.add_argument("--min-steps", type=int, default=20)
    ap.add_argument("--max-steps", type=int, default=200)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--prec", choices=["mixed", "fp64", "fp32"], default="mixed",
                    help="fp32: mixed with the Krylov basis stored in FP32")
    ap.add_argument("--batch", type=int, default=len(SEEDS))
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kernel", default="jvp")
    ap.add_argument("--no-fp64-compare", action="store_true")
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
    if args.workload == "longrun":
        return run_longrun(args)

    import torch
    import paper_1604_08159_amd as m
    import workloads as W

    dev = torch.device("cuda:0")
    prec = {"mixed": m.MRA_MIXED, "fp64": m.MRA_FP64, "fp32": m.MRA_FP32}[args.prec]
    stream = torch.cuda.Stream(device=dev)
    seeds = [SEEDS[i % len(SEEDS)] + 100 * (i // len(SEEDS)) for i in range(args.batch)]
    pbs = [W.fujiwhara_pair(s) for s in seeds]
    solves = []
    with torch.cuda.stream(stream):
        for pb in pbs:
            w0 = torch.from_numpy(W.initial_field(pb)).to(dev)
            solves.append(m.Solve(m.grid_desc(pb.J, pb.p, pb.eps), m.flow_desc(pb.nu0, pb.cs), prec, pb.m,
                                  pb.dt, w0, stream=stream))
    n = len(solves)
    m.solve_batch(solves, [args.warmup] * n, stream=stream)
    stream.synchronize()
    ev0 = sum(s.scalars()["evals"] for s in solves)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.solve_batch(solves, [args.steps] * n, stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev1 = sum(s.scalars()["evals"] for s in solves)
    value = (ev1 - ev0) / wall

    # state after the timed region
    nas = []
    for s in solves:
        _, diag = s.read(dense=False, stream=stream)
        nas.append(int(diag["n_active"]))
        if diag["status"] != 0:
            print(json.dumps({"error": f"solve reported status {diag['status']}"}))
            return 1
    N = 1 << pbs[0].J
    esz = 8 if prec == m.MRA_FP64 else 4

    # dominant kernel: HIP events around back-to-back launches of the same
    # launch configuration, on the stream the step runs on
    reps = 50
    k_ms = m.time_kernel(solves, args.kernel, reps, stream=stream)
    # fraction of stencil tiles holding an active node (the stencil skips the rest)
    ts = 32
    act_tiles = []
    for s in solves:
        _, mask, ip, fi = s.active_set()
        f = fi.long()
        t = ((f // N) // ts) * (N // ts) + (f % N) // ts
        act_tiles.append(torch.unique(t).numel() / (N // ts) ** 2)
    frac_t = sum(act_tiles) / len(act_tiles)
    nbytes = kernel_bytes(args.kernel, N, int(sum(nas) / len(nas)), frac_t, n, esz)
    achieved = nbytes / (k_ms * 1e-3) / 1e9

    # plain copy of known size: the byte-counter scale of profiled runs, and
    # (timed) the practical streaming ceiling of this device
    cal_a = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
    cal_b = torch.empty_like(cal_a)
    cal_b.copy_(cal_a)
    torch.cuda.synchronize()
    big_a = torch.empty(1 << 28, dtype=torch.float32, device=dev)      # 1 GiB, far beyond the caches
    big_b = torch.empty_like(big_a)
    big_b.copy_(big_a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        big_b.copy_(big_a)
    e1.record()
    e1.synchronize()
    copy_gbs = 2 * big_a.numel() * 4 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del cal_a, cal_b, big_a, big_b
    compare = None
    accuracy = None
    if not args.no_fp64_compare and prec != m.MRA_FP64:
        compare = fp64_per_solve(m, W, dev, max(10, args.steps // 10))
        accuracy = accuracy_vs_fp64(m, W, dev, solves[0], seeds[0], args.warmup + args.steps)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "active-pt RHS evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == m.MRA_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"Fujiwhara pair Re=5000, finest 512^2 (J=9), 4-point DD, eps=1e-4, m=20, "
                               f"dt=0.01; batch of {n} seeded solves",
                   "batch": n, "finest_points": N * N, "mean_active_points": sum(nas) / len(nas),
                   "precision": args.prec, "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "hbm", "kernel": args.kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.kernel),
                     "avg_launch_ms": k_ms, "algorithmic_bytes_per_launch": nbytes,
                     "active_tile_fraction": frac_t,
                     "copy_ceiling_gbs": copy_gbs, "frac_of_copy_ceiling": achieved / copy_gbs},
        "finest_pt_evals_per_s": value * N * N / (sum(nas) / len(nas)),
    }
    step_s = wall / args.steps
    out["ensemble"] = {"solves_per_s_at_2000_steps": n / (step_s * 2000),
                       "note": "batch solves/s if each solve ran the configuration's 2000 steps"}
    if compare is not None:
        out["fp64_per_solve_gpu"] = compare
    if accuracy is not None:
        out["fp32_vs_fp64"] = accuracy
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    for s in solves:
        s.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
