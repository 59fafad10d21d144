"""Benchmark: certified MPC solves per second on one MI355X.

Workload: 4096 problems, horizon 20, dt 0.03 s, mixed single and double
support, pushes on the initial velocity (the "plain_b4096_n20" generator
configuration), inputs resident in HBM.  One step = one pinmpc_solve of the
whole batch: setup, the ADMM sweeps, FP64 refinement and certificate.  Only
problems whose reported KKT residuals are all <= 1e-5 count as solves.

Prints one JSON line.  Also reports p50/p99 latency of a batch solve, the
roofline of the dominant kernel measured with HIP events inside the library,
and the FP64 oracle timed on the host cores as a reference baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MPC solves/sec at KKT resid ≤1e-5 (batch 4096, N=20); p99 solve latency"
WORKLOAD = "plain_b4096_n20"
KKT_BAR = 1e-5
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

# Algorithmic bytes of one plain ADMM sweep per stage (FP32):
#   operators A 676 + Bt 624 + H packed 1300 + M packed 312 + qbar 100
#   + e 52 + contact 2 + force scale 4 = 3070 B read,
#   iterates (current and extrapolated, 5 x 25 each) 1000 B read + 1000 B written
SWEEP_BYTES_PER_STAGE = 3070 + 2000
# Algorithmic flops of one sweep per stage: block 1 (Abar^T y 338, Bt^T w 312,
# M t 288, H htilde 1250, vector ops 100), block 2 (Abar xi 650, Bbar du 312,
# vector ops + projection 150), block 3 and the restart test 200
SWEEP_FLOPS_PER_STAGE = 338 + 312 + 288 + 1250 + 100 + 650 + 312 + 150 + 200
FP32_PEAK_TFLOPS = 157.3
# Algorithmic work of the FP64 refinement per pass-stage (one stage of one
# equality-constrained pass or of one interior-point iteration): about 30 kflop
# and 4.5 KB of stage data (the survey's per-unit figures for this step)
REFINE_FLOPS_PER_PASS_STAGE = 30_000
REFINE_BYTES_PER_PASS_STAGE = 4_500
# the same pass-stage counted densely from the kernel's own products (13-state,
# 12-input shapes, 2 flops per multiply-add): backward recursion Bp = B P 3744,
# d = B c + e 312, W A 4394, W d 338, W Bp 4056, Bp^T W Bp 3744,
# Bp^T [W A | W d] 4368, P R P and P R c 3744, Gauss-Jordan on [H | Hwx | hw]
# 5904, S and s 9100 (39 704 per factored stage); forward rollout 1250,
# costates and gradient 650, multipliers and residuals 500 (2 400 per stage of
# every pass)
REFINE_DENSE_BACKWARD = 3744 + 312 + 4394 + 338 + 4056 + 3744 + 4368 + 3744 + 5904 + 9100
REFINE_DENSE_FORWARD = 1250 + 650 + 500
# The four-contact refinement (feet and hands, 24 inputs) per stage of one
# interior-point iteration: two backward recursions, the predictor's a
# factorisation of the stage system (W B 8112, W A 4394, B^T W B 14976, B^T W A
# 8112, B^T w 624, Gauss-Jordan on the 24 x 38 system 41952, S and s 13468:
# 91 638), the corrector's the vector part with the kept inverse (B^T w 624,
# H^-1 hw 1152, A^T w 338, Hwx^T kappa 624: 2738) except near the optimum, where
# it factors again; and two rollouts of the gains (1586 each).  The kernel
# reports the stages its factoring recursions covered, so the flops of a solve
# are counted from that mix.  Bytes: the iteration's data flow, each array crossing HBM once
# per phase that uses it: the factorisation reads A, B (FP32), the stage terms
# and x, and writes K, kappa, H^-1 and Hwx (13 216 B); the corrector's vector
# pass reads B, A, rho, x, H^-1 and Hwx and writes kappa (9568 B); two rollouts
# of the gains (4908 B each); two builds of the stage terms (2592 B each); two
# slack and multiplier steps (2144 B each); the step and the next residuals
# (3736 B); the corrector's target (1760 B)
WIDE_FACTOR_FLOPS = 8112 + 4394 + 14976 + 8112 + 624 + 41952 + 13468
WIDE_VECTOR_FLOPS = 624 + 1152 + 338 + 624
WIDE_ROLLOUT_FLOPS = 1586
WIDE_BYTES_PER_IPM_STAGE = 13216 + 9568 + 2 * 4908 + 2 * 2592 + 2 * 2144 + 3736 + 1760
# its sweep per stage: operators A 676 + Bt 1248 + H packed 2812 + M packed
# 1200 + qbar 148 + e 52 + contact 4 + force scale 4 = 6144 B read, iterates
# (5 x 37 each) 1480 B read + 1480 B written; setup per stage: A_k, A_{k+1},
# B_k, B_{k+1} read (3848 B), Bt, H, M, qbar written (5408 B)
WIDE_SWEEP_BYTES_PER_STAGE = 6144 + 2960
WIDE_SETUP_BYTES_PER_STAGE = 3848 + 5408
# setup, once per stage: operators read, H, M, qbar and the scaled B written
SETUP_BYTES_PER_STAGE = 3_200
# interior-point cap, polish passes and certificate threshold for horizons
# beyond 64 stages (the multiplier-sign residual is normalised by terms that
# grow with the costates over a long horizon)
LONG_BASE = dict(ipm_iters=150, polish_passes=20, kkt_tol=1e-10)
# FP64 peak of the chip: vector FMA units and matrix cores have the same rate
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=100, help="ADMM sweeps per solve")
    ap.add_argument("--form", type=int, default=0, help="0 plain, 1 fused, -1 packed")
    ap.add_argument("--rho", type=float, default=10.0)
    ap.add_argument("--refine-passes", type=int, default=8,
                    help="active-set passes before the interior-point fallback")
    ap.add_argument("--first-passes", type=int, default=4,
                    help="active-set passes every problem runs in the first refinement launch")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: choose form/K/rho with the autotuner on a held-out batch "
                         "(problems 4096..8191 of the same generator) before timing")
    ap.add_argument("--cpu-sample", type=int, default=4096,
                    help="problems in the oracle CPU-baseline sample (0: skip); the default "
                         "is the whole batch, about 20 core-seconds of oracle work")
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a plain streaming kernel over this many bytes (read once, "
                         "written once), to scale the HBM byte counters")
    ap.add_argument("--pmc-summary", default="",
                    help="only summarise rocprofv3 --pmc runs found under this folder "
                         "(pmc_fetch, pmc_write, pmc_copy_fetch, pmc_copy_write) into "
                         "profiles/traffic.json")
    ap.add_argument("--pmc-args", default=TUNED,
                    help="the benchmark arguments of those runs (recorded with each kernel's "
                         "entry; entries of kernels the runs did not see are kept)")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="generator configuration of the timed batch (the metric is quoted on "
                         "plain_b4096_n20; the others are reported beside it)")
    ap.add_argument("--precision", type=int, default=0, help="1: BF16 operators")
    ap.add_argument("--serving", type=int, default=0,
                    help="1: run the serving loop instead (continuous batching of Poisson "
                         "request arrivals, warm start across control ticks)")
    ap.add_argument("--serving-load", type=float, default=1.0,
                    help="offered load as a fraction of the serving configuration's nominal "
                         "32768 problems per 20 ms tick (the tick is stretched by 1 / load)")
    ap.add_argument("--serving-ticks", type=int, default=3)
    ap.add_argument("--lanes", type=int, default=3)
    ap.add_argument("--lane-capacity", type=int, default=8192)
    ap.add_argument("--streams", type=int, default=2,
                    help="solves in flight: S library contexts on S streams (default "
                         "priority) take the timed solves round robin, so one solve's "
                         "refinement tail overlaps the next solve's setup and sweeps")
    ap.add_argument("--scan", type=int, default=0,
                    help="refinement backward recursion: 0 sequential, 2/4/8 associative "
                         "scan over that many chunks of the horizon")
    ap.add_argument("--graph", type=int, default=0,
                    help="1: time captured-graph replays (phase times then come from a "
                         "second, uncaptured loop)")
    return ap.parse_args()


def _oracle_chunk(idx):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import mpcgen
    from oracle import qp
    batch = mpcgen.make_batch(WORKLOAD, indices=idx)
    t = time.perf_counter()
    for b in range(len(idx)):
        qp.solve(mpcgen.problem_fp64(batch, b))
    return time.perf_counter() - t


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _admm_chunk(args):
    idx, K, rho = args
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import mpcgen
    from oracle import admm
    batch = mpcgen.make_batch(WORKLOAD, indices=idx)
    t = time.perf_counter()
    for b in range(len(idx)):
        admm.solve(mpcgen.problem_fp64(batch, b), iters=K, rho=rho, scaling=True, accel=True)
    return time.perf_counter() - t


def cpu_baseline(sample, workers, admm_k=None, rho=10.0):
    """The FP64 oracle on the host cores: `sample` problems of the workload,
    one process per worker, BLAS single-threaded per process.  The worker
    count is capped at 16, the host-core share of one GPU on the GPU machine.
    With admm_k, also the FP64 ADMM reference (the same algorithm as the GPU's
    sweeps, no refinement, not certified) at the GPU's sweep count on the
    same sample."""
    import multiprocessing as mp
    if workers <= 0:
        workers = min(16, os.cpu_count() or 1)
    chunks = [list(range(i, sample, workers)) for i in range(workers)]
    chunks = [c for c in chunks if c]
    env_keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in env_keys}
    for k in env_keys:
        os.environ[k] = "1"
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(len(chunks)) as pool:
        busy = pool.map(_oracle_chunk, chunks)
        wall = time.perf_counter() - t0
        admm_rec = None
        if admm_k:
            t1 = time.perf_counter()
            busy2 = pool.map(_admm_chunk, [(c, admm_k, rho) for c in chunks])
            wall2 = time.perf_counter() - t1
            admm_rec = {"value": sample / wall2, "unit": "solves/s", "cores": len(chunks),
                        "kind": "oracle ADMM reference (same algorithm, FP64, not certified)",
                        "sweeps": admm_k,
                        "sample": f"{sample} problems of {WORKLOAD}, {sum(busy2):.1f} core-s"}
    for k, v in saved.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v
    return {
        "value": sample / wall,
        "unit": "solves/s",
        "cores": len(chunks),
        "nproc": os.cpu_count(),
        "cpu_model": _cpu_model(),
        "worker_cap": "16 processes: the host-core share of one GPU on the GPU box",
        "kind": "oracle",
        "same_algorithm_admm": admm_rec,
        "sample": f"{sample} problems of {WORKLOAD} (problem indices 0..{sample - 1}), "
                  f"dense-condensed FP64 interior point + certified active-set polish, "
                  f"{sum(busy):.1f} core-s",
    }


KERNEL_SOURCES = {
    "refine_kernel<1>": "refine.hip",
    "refine_kernel<2>": "refine.hip",
    "setup_kernel<2>": "setup.hip",
    "setup_kernel<4>": "setup.hip",
    "admm_fused_kernel": "admm_fused.hip",
    "admm_sweep_kernel": "admm_plain.hip",
    "dynamics_kernel": "dynamics.hip",
    "refine_wide_kernel": "refine_wide.hip",
}


def _kernel_sha(path):
    """Hash of a kernel's source together with the shared internal header."""
    h = hashlib.sha256()
    for f in (path, os.path.join(os.path.dirname(path), "pinmpc_internal.h")):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _counter_rows(run_dir):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(run_dir, "*counter_collection.csv")):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


TUNED = "--autotune 0 --form 1 --iters 2 --rho 1 --refine-passes 12 --first-passes 0 --cpu-sample 0 --streams 1"


def pmc_commands(run_args):
    """The rocprofv3 counter runs that a summary reads, for benchmark
    arguments `run_args`."""
    return [
        f"rocprofv3 --pmc FETCH_SIZE -d gpurun_out/pmc_fetch -o f --output-format csv -- "
        f"python3 bench.py {run_args} --steps 2 --warmup 1",
        f"rocprofv3 --pmc WRITE_SIZE -d gpurun_out/pmc_write -o w --output-format csv -- "
        f"python3 bench.py {run_args} --steps 2 --warmup 1",
        "rocprofv3 --pmc FETCH_SIZE -d gpurun_out/pmc_copy_fetch -o cf --output-format csv -- "
        "python3 bench.py --copy-calibration 1073741824",
        "rocprofv3 --pmc WRITE_SIZE -d gpurun_out/pmc_copy_write -o cw --output-format csv -- "
        "python3 bench.py --copy-calibration 1073741824",
        f"python3 bench.py --pmc-summary gpurun_out --pmc-args '{run_args}'",
    ]


def _kernel_match(kernel, name):
    """Whether a demangled kernel name is `kernel` ("refine_kernel<1>" also
    matches the instantiation refine_kernel<1, false>, and a plain name any
    instantiation of it)."""
    if "<" in kernel:
        head = "::" + kernel[:-1]
        return head + ">" in name or head + "," in name
    return "::" + kernel + "(" in name or "::" + kernel + "<" in name


def pmc_summary(prof_dir, run_args):
    """HBM bytes per launch of the library's kernels from two rocprofv3 --pmc
    runs of the benchmark (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each
    scaled by what the same counter reads for the --copy-calibration kernel,
    whose bytes are known.  Updates profiles/traffic.json (one entry per
    kernel, with the calibration and commands it was taken with); returns a
    text summary."""
    cal = {}
    for counter, sub in (("FETCH_SIZE", "pmc_copy_fetch"), ("WRITE_SIZE", "pmc_copy_write")):
        vals = [float(r["Counter_Value"]) for r in _counter_rows(os.path.join(prof_dir, sub))
                if r["Counter_Name"] == counter and "AUnaryFunctor" in r["Kernel_Name"]]
        known_kib = 1073741824 / 1024.0
        cal[counter] = {"dispatches": len(vals), "mean_kib": sum(vals) / len(vals),
                        "scale": known_kib / (sum(vals) / len(vals))}
    calib = {"kernel": "elementwise multiply by 1 over 1 GiB (read 1 GiB, write 1 GiB)",
             "FETCH_SIZE": cal["FETCH_SIZE"], "WRITE_SIZE": cal["WRITE_SIZE"]}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    out = {}
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    for k in ("calibration", "commands"):   # the single-run layout of earlier records
        out.pop(k, None)
    seen = {}
    lines = ["| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled bytes per launch |",
             "|---|---|---|---|---|"]
    for kernel, src in KERNEL_SOURCES.items():
        per = {}
        for counter, sub in (("FETCH_SIZE", "pmc_fetch"), ("WRITE_SIZE", "pmc_write")):
            vals = [float(r["Counter_Value"]) for r in _counter_rows(os.path.join(prof_dir, sub))
                    if r["Counter_Name"] == counter and _kernel_match(kernel, r["Kernel_Name"])]
            if vals:
                per[counter] = (len(vals), sum(vals) / len(vals))
        if len(per) < 2:
            continue
        nb = per["FETCH_SIZE"][1] * 1024 * cal["FETCH_SIZE"]["scale"] + \
            per["WRITE_SIZE"][1] * 1024 * cal["WRITE_SIZE"]["scale"]
        seen[kernel] = {"source_sha": _kernel_sha(os.path.join(ROOT, "paper_2606_05687_amd", "csrc", src)),
                        "fetch_kib": per["FETCH_SIZE"][1], "write_kib": per["WRITE_SIZE"][1],
                        "bytes_per_launch": nb, "calibration": calib,
                        "commands": pmc_commands(run_args)}
        lines.append(f"| {kernel} | {per['FETCH_SIZE'][0]} | {per['FETCH_SIZE'][1]:.0f} | "
                     f"{per['WRITE_SIZE'][1]:.0f} | {nb / 1e9:.3f} GB |")
    # the refinement runs as a pair of launches per solve (every problem's
    # active-set passes, then the problems they leave): its bytes per solve
    if "refine_kernel<1>" in seen and "refine_kernel<2>" in seen:
        seen["refine_kernel"] = {
            "source_sha": seen["refine_kernel<1>"]["source_sha"],
            "bytes_per_launch": seen["refine_kernel<1>"]["bytes_per_launch"] +
            seen["refine_kernel<2>"]["bytes_per_launch"],
            "note": "sum of the two refinement launches of one solve",
            "commands": pmc_commands(run_args)}
        lines.append(f"| refine_kernel<1> + <2> (per solve) | | | | "
                     f"{seen['refine_kernel']['bytes_per_launch'] / 1e9:.3f} GB |")
    out.update(seen)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    lines += ["", f"FETCH_SIZE scale {cal['FETCH_SIZE']['scale']:.4f} "
              f"(calibration kernel reads {cal['FETCH_SIZE']['mean_kib']:.0f} KiB for 1 GiB read), "
              f"WRITE_SIZE scale {cal['WRITE_SIZE']['scale']:.4f} "
              f"({cal['WRITE_SIZE']['mean_kib']:.0f} KiB for 1 GiB written)"]
    return "\n".join(lines)


def measured_traffic(kernel_src, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel calibration),
    if it was taken on the current source of the kernel; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f).get(kernel)
    if not t or t.get("source_sha") != _kernel_sha(kernel_src):
        return None
    return t.get("bytes_per_launch")


def _slice(batch, rows):
    """Problems `rows` of a generator batch, stage arrays trimmed to their
    longest horizon."""
    import numpy as np
    n = int(batch["N"][rows].max())
    out = {}
    for k, v in batch.items():
        if v is None or not hasattr(v, "shape") or v.ndim == 0:
            out[k] = v
            continue
        v = v[rows]
        if k in ("A", "B", "e", "x_ref", "u_ref", "contact"):
            v = v[:, :n]
        out[k] = np.ascontiguousarray(v)
    return out


def serving(args, settings):
    """Serving loop: per control tick, 512 requests of 64 problems (one per
    environment, 64 environment groups of 512) arrive as a Poisson process
    over the tick and are continuously batched onto the server's lanes; each
    environment keeps its warm-start slot across ticks.  Arrivals follow the
    clock (open loop); a request waits only for its own group's previous
    request.  Reports certified solves/s over the whole run (first arrival to
    last result) and p50/p99 request latency (arrival to results ready)."""
    import ctypes
    import numpy as np
    import torch
    import mpcgen
    from paper_2606_05687_amd import binding
    per_tick, per_req = 32768, 64
    n_req = per_tick // per_req
    tick_s = 0.020 / max(args.serving_load, 1e-6)
    full = mpcgen.make_batch("serving_tick")
    reqs = [_slice(full, np.arange(r * per_req, (r + 1) * per_req)) for r in range(n_req)]
    devs = [binding.to_device(r, "cuda:0") for r in reqs]
    lib = binding.load()
    srv = binding.Server(0, lanes=args.lanes, capacity=args.lane_capacity,
                         warm_slots=per_tick, **settings)
    outs = [binding.Solver.alloc_out(None, d) for d in devs]
    bstructs = [binding.make_batch_struct(d) for d in devs]
    ostructs = [binding._out_struct(o) for o in outs]
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    lat, ok_total = [], 0
    ticket = ctypes.c_int64()
    # open loop over ticks: tick t's requests arrive on the clock whether or
    # not earlier ticks are done; only an environment group's own previous
    # request must be done before its next one (its warm-start slots and output
    # buffers are the same), which is the control loop's own dependency
    pending = {}

    def finish(r):
        nonlocal ok_total
        t, delay_ms = pending.pop(r)
        # arrival to results ready: the client-side delay behind the group's
        # previous request plus the server's submit-to-ready latency
        lat.append(srv.wait(t) + delay_ms)
        o = outs[r]
        ok_total += int(((o["status"] == 0) & (o["res"].max(dim=1).values <= KKT_BAR)).sum().item())

    t_first = time.perf_counter()
    for tick in range(args.serving_ticks):
        arrive = np.sort(rng.uniform(0.0, tick_s, size=n_req)) + tick * tick_s
        order = rng.permutation(n_req)
        for a, r in zip(arrive, order):
            while time.perf_counter() - t_first < a:
                pass
            if r in pending:
                finish(r)
            delay_ms = (time.perf_counter() - t_first - a) * 1e3
            binding._check(lib.pinmpc_submit(srv._h, ctypes.byref(bstructs[r]),
                                             ctypes.byref(ostructs[r]), int(r * per_req),
                                             ctypes.byref(ticket)))
            pending[r] = (ticket.value, delay_ms)
    for r in list(pending):
        finish(r)
    t_end = time.perf_counter()
    st = srv.stats()
    srv.close()
    return {
        "metric": "serving: certified MPC solves/s and request latency (serving_tick)",
        "value": ok_total / (t_end - t_first), "unit": "solves/s", "n_gpus": 1,
        "ticks": args.serving_ticks, "offered_load": args.serving_load,
        "offered_solves_per_s": per_tick / tick_s,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "requests": len(lat), "problems_per_request": per_req,
        "launches": st["launches"], "problems": st["problems"],
        "certified_frac": ok_total / (per_tick * args.serving_ticks),
        "lanes": args.lanes, "lane_capacity": args.lane_capacity,
        "config": {"workload": "serving_tick", "settings": settings},
        "data": "synthetic",
    }


# Algorithmic bytes of the step before the solve (stage matrices from compact
# physics) per stage: A and B written (169 + 156 floats), yaw, reference CoM
# and two contact positions read (1 + 3 + 6 floats); per problem mass,
# principal moments, dt and horizon (6 words)
DYN_BYTES_PER_STAGE = (169 + 156) * 4 + (1 + 3 + 6) * 4
DYN_BYTES_PER_PROBLEM = 6 * 4


def before_after(batch, reps=20):
    """The steps before and after the solve on the metric workload, timed
    with HIP events on the current stream: the stage matrices of all 4096 x 20
    stages built from compact physics, and one landmark push (5 landmarks)
    plus one reward evaluation for 4096 environments."""
    import numpy as np
    import torch
    from paper_2606_05687_amd import binding
    keys = ("N", "yaw_k", "c_ref", "feet", "mass", "inertia", "dt")
    phys = {k: torch.from_numpy(np.ascontiguousarray(batch[k])).cuda() for k in keys}
    Bn, n = batch["yaw_k"].shape
    A = torch.empty((Bn, n, 13, 13), dtype=torch.float32, device="cuda")
    B = torch.empty((Bn, n, 13, 12), dtype=torch.float32, device="cuda")
    for _ in range(3):
        binding.build_dynamics(phys, A, B)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        binding.build_dynamics(phys, A, B)
    ev[1].record()
    torch.cuda.synchronize()
    dyn_ms = ev[0].elapsed_time(ev[1]) / reps
    dyn_bytes = Bn * n * DYN_BYTES_PER_STAGE + Bn * DYN_BYTES_PER_PROBLEM
    ring = binding.LandmarkRing(Bn, 5, n + 1)
    ring.clear()
    x = torch.zeros((Bn, n + 1, 13), dtype=torch.float32, device="cuda")
    Nd = phys["N"]
    com = torch.zeros((Bn, 3), dtype=torch.float32, device="cuda")
    alpha = torch.tensor([0.5, 0.25, 0.15, 0.07, 0.03], dtype=torch.float32, device="cuda")
    qc = torch.ones(3, dtype=torch.float32, device="cuda")
    for t in range(3):
        ring.push(x, Nd, t)
        ring.reward(com, t, alpha, qc, 0.1)
    ev[0].record()
    for t in range(3, 3 + reps):
        ring.push(x, Nd, t)
        ring.reward(com, t, alpha, qc, 0.1)
    ev[1].record()
    torch.cuda.synchronize()
    lm_ms = ev[0].elapsed_time(ev[1]) / reps
    return {"dynamics": {"ms": dyn_ms, "bytes": dyn_bytes,
                         "gbs": dyn_bytes / (dyn_ms * 1e-3) / 1e9,
                         "hbm_frac": dyn_bytes / (dyn_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "stages": int(Bn * n)},
            "landmark_push_and_reward_ms": lm_ms, "envs": int(Bn), "landmarks": 5}


def main():
    args = parse()
    if args.pmc_summary:
        print(pmc_summary(args.pmc_summary, args.pmc_args))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the batch shards across GPUs with no communication, see DESIGN.md",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"copy_kernel": "elementwise multiply by 1", "bytes_read": n * 4,
                          "bytes_written": n * 4, "reps": 3}), flush=True)
        return

    import mpcgen
    from paper_2606_05687_amd import binding

    torch.cuda.set_device(0)
    settings = dict(iters=args.iters, form=args.form, rho=args.rho,
                    refine_passes=args.refine_passes, first_passes=args.first_passes,
                    precision=args.precision, scan=args.scan)
    if args.serving:
        if args.autotune:
            # the schedule tuned on a held-out slice of the serving workload
            from paper_2606_05687_amd import autotune
            held = mpcgen.make_batch("serving_tick", indices=range(32768, 32768 + 4096))
            hdev = binding.to_device(held, "cuda:0")
            settings.update(autotune.tune(hdev, cache_path=os.path.join(ROOT, "gpurun_out",
                                                                        "tune.json"),
                                          force=True, in_flight=1))
            del hdev
        print(json.dumps(serving(args, settings)), flush=True)
        return
    tuned = None
    tune_curve = None
    if args.autotune:
        from paper_2606_05687_amd import autotune
        nb = mpcgen.CONFIGS[args.workload]["batch"]
        held = mpcgen.make_batch(args.workload, indices=range(nb, 2 * nb))
        hdev = binding.to_device(held, "cuda:0")
        # hundreds of stages need a larger interior-point cap than the default
        base = LONG_BASE if int(held["A"].shape[1]) > 64 else None
        tuned = autotune.tune(hdev, cache_path=os.path.join(ROOT, "gpurun_out", "tune.json"),
                              force=True, in_flight=max(1, args.streams), base=base)
        if tuned is None:   # no candidate certified enough: the base schedule
            tuned = dict(base or {})
        settings.update(tuned)
        tune_curve = [{k: r[k] for k in ("iters", "rho", "ms", "certified", "eq_passes",
                                          "ipm_iters")}
                      for r in autotune.LAST_LOG
                      if r["rho"] == tuned.get("rho") and r["refine_passes"] == 12
                      and r["first_passes"] == 0 and r["precision"] == tuned.get("precision")]
        del hdev
    batch = mpcgen.make_batch(args.workload)
    Bn, n = batch["A"].shape[0], batch["A"].shape[1]
    wide = batch["contact"].shape[-1] == 4   # feet and hands: the interior-point refinement
    stages = int(batch["N"].sum())
    if n > 64:   # the long-horizon refinement budget (also for a fixed schedule)
        for k, v in LONG_BASE.items():
            settings.setdefault(k, v)
    dev = binding.to_device(batch, "cuda:0")
    nst = max(1, args.streams)
    solvers = [binding.Solver(0, **settings) for _ in range(nst)]
    for sv in solvers:
        sv.set(graph=int(args.graph))
    outs = [sv.alloc_out(dev) for sv in solvers]
    bstruct = binding.make_batch_struct(dev)
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(nst - 1)]
    solver, out, stream = solvers[0], outs[0], streams[0]

    for _ in range(args.warmup):
        for sv, o, st in zip(solvers, outs, streams):
            sv.solve(dev, o, stream=st, batch_struct=bstruct)
    torch.cuda.synchronize()

    # timed region: K solves enqueued back to back (round robin over the
    # streams when more than one solve is in flight), bracketed by device
    # synchronisation; per-solve latency from HIP events recorded around each
    # solve on its stream, per-kernel times from the library's own HIP events
    # on the same stream (kept for the last STATS_RING solves)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        sv, o, st = solvers[i % nst], outs[i % nst], streams[i % nst]
        evs[i][0].record(st)
        sv.solve(dev, o, stream=st, batch_struct=bstruct)
        evs[i][1].record(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_ms = [a.elapsed_time(b) for a, b in evs]
    # every step solves the same batch deterministically: the last outputs
    # are every step's outputs
    certified = 0
    for i in range(args.steps):
        o = outs[i % nst]
        ok = (o["status"] == 0) & (o["res"].max(dim=1).values <= KKT_BAR)
        certified += int(ok.sum().item())
    ms_per_step = elapsed * 1e3 / args.steps
    value = certified / elapsed

    if args.graph:
        # graph replays report totals only: per-kernel times from an
        # uncaptured loop of the same length right after
        solver.set(graph=0)
        for _ in range(args.steps):
            solver.solve(dev, out, stream=stream, batch_struct=bstruct)
        torch.cuda.synchronize()
    nk = min((args.steps + nst - 1) // nst, binding.STATS_RING)
    phases = [solver.stats(back=i) for i in range(nk)]
    setup_ms = float(np.mean([ph["setup_ms"] for ph in phases]))
    admm_ms = float(np.mean([ph["admm_ms"] for ph in phases]))
    refine_ms = float(np.mean([ph["refine_ms"] for ph in phases]))

    single = None
    if nst > 1:
        # the same solves one at a time on one stream, for comparison
        evs1 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for _ in range(args.steps)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(args.steps):
            evs1[i][0].record(stream)
            solver.solve(dev, out, stream=stream, batch_struct=bstruct)
            evs1[i][1].record(stream)
        torch.cuda.synchronize()
        el1 = time.perf_counter() - t1
        ms1 = [a.elapsed_time(b) for a, b in evs1]
        ok1 = (out["status"] == 0) & (out["res"].max(dim=1).values <= KKT_BAR)
        single = {"value": int(ok1.sum().item()) * args.steps / el1,
                  "ms_per_step": el1 * 1e3 / args.steps,
                  "p50_ms": float(np.percentile(ms1, 50)), "p99_ms": float(np.percentile(ms1, 99))}
        # kernel durations for the roofline: from these solves, where no other
        # solve shares the GPU (with solves in flight, the stream events of a
        # phase also count time its kernels wait for the other stream's)
        single["kernel_ms_in_flight"] = {"setup": setup_ms, "admm": admm_ms, "refine": refine_ms}
        nk1 = min(args.steps, binding.STATS_RING)
        ph1 = [solver.stats(back=i) for i in range(nk1)]
        setup_ms = float(np.mean([ph["setup_ms"] for ph in ph1]))
        admm_ms = float(np.mean([ph["admm_ms"] for ph in ph1]))
        refine_ms = float(np.mean([ph["refine_ms"] for ph in ph1]))

    K = settings["iters"]
    iters_out = out["iters"].cpu().numpy().astype(np.int64)
    passes = iters_out - K
    N_b = batch["N"].astype(np.int64)
    det = out["detail"].cpu().numpy().astype(np.int64)
    eq_p, ipm_p, stf = det[:, 0], det[:, 1], det[:, 2]
    # pass-stages: one stage of one equality-constrained pass or interior-point
    # iteration, the unit of the refinement's algorithmic work
    pass_stages = int((N_b * (eq_p + ipm_p)).sum())
    dense_flops = float(stf.sum() * REFINE_DENSE_BACKWARD +
                        (N_b * eq_p).sum() * REFINE_DENSE_FORWARD +
                        (N_b * ipm_p).sum() * (REFINE_DENSE_BACKWARD + 2 * REFINE_DENSE_FORWARD))
    if wide:   # two recursions and two rollouts per iteration-stage
        factored = int(stf.sum())
        dense_flops = float(factored * WIDE_FACTOR_FLOPS +
                            (2 * pass_stages - factored) * WIDE_VECTOR_FLOPS +
                            2 * pass_stages * WIDE_ROLLOUT_FLOPS)
    sweep_b = WIDE_SWEEP_BYTES_PER_STAGE if wide else SWEEP_BYTES_PER_STAGE
    setup_b = WIDE_SETUP_BYTES_PER_STAGE if wide else SETUP_BYTES_PER_STAGE
    work = {"pass_stages": pass_stages,
            "equality_passes_mean": float(eq_p.mean()),
            "interior_point_iters_mean": float(ipm_p.mean()),
            "frac_reaching_interior_point": float((ipm_p > 0).mean()),
            "frac_finished_in_second_launch": float((det[:, 3] == 2).mean()),
            "stages_factored_per_equality_pass": float(stf.sum() / max(1, eq_p.sum())),
            "dense_flops_per_solve": dense_flops}
    # four contacts take the streamed sweep whatever the form (all sweeps in one
    # launch unless the form is 0)
    form_name = ("streamed" if wide and settings["form"] != 0 else
                 {0: "plain", 1: "fused", -1: "packed", 2: "split"}[settings["form"]])
    kernels = {
        "setup_kernel": {"ms": setup_ms},
        "admm": {"ms": admm_ms, "form": form_name},
        "refine_kernel": {"ms": refine_ms},
    }
    # algorithmic work of each phase per launch
    flops_ps = (dense_flops / max(1, pass_stages)) if wide else REFINE_FLOPS_PER_PASS_STAGE
    bytes_ps = WIDE_BYTES_PER_IPM_STAGE if wide else REFINE_BYTES_PER_PASS_STAGE
    refine_flops = float(pass_stages) * flops_ps
    refine_bytes = float(pass_stages) * bytes_ps
    kernels["refine_kernel"]["tflops"] = refine_flops / (refine_ms * 1e-3) / 1e12
    kernels["refine_kernel"]["gbs"] = refine_bytes / (refine_ms * 1e-3) / 1e9
    kernels["refine_kernel"]["dense_tflops"] = dense_flops / (refine_ms * 1e-3) / 1e12
    if settings["form"] == 0 or wide:
        sweep_bytes = stages * sweep_b
        kernels["admm"]["gbs"] = sweep_bytes * K / (admm_ms * 1e-3) / 1e9
    else:
        kernels["admm"]["tflops"] = stages * SWEEP_FLOPS_PER_STAGE * K / (admm_ms * 1e-3) / 1e12
    dominant = max(kernels, key=lambda k: kernels[k]["ms"])
    if dominant == "refine_kernel":
        kname = "refine_wide_kernel" if wide else "refine_kernel"
        src = os.path.join(ROOT, "paper_2606_05687_amd", "csrc",
                           "refine_wide.hip" if wide else "refine.hip")
        achieved = kernels["refine_kernel"]["tflops"]
        # FP64 arithmetic on the vector units and matrix cores (the same FP64
        # peak on this chip); the HBM fraction of the same launch beside it
        roof = {"kernel": kname if wide else "refine_kernel<1>+<2>", "bound": "alu",
                "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS,
                "traffic": measured_traffic(src, kname),
                "launch_ms": refine_ms, "flops_per_launch": refine_flops,
                "pass_stages": pass_stages, "flops_per_pass_stage": flops_ps,
                "hbm_gbs": kernels["refine_kernel"]["gbs"],
                "hbm_frac": kernels["refine_kernel"]["gbs"] / HBM_PEAK_GBS,
                "bytes_per_pass_stage": bytes_ps, "dtype": "f64"}
    elif dominant == "admm" and (settings["form"] == 0 or wide):
        src = os.path.join(ROOT, "paper_2606_05687_amd", "csrc", "admm_plain.hip")
        achieved = kernels["admm"]["gbs"]
        roof = {"kernel": "admm_sweep_kernel", "bound": "hbm", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(src, "admm_sweep_kernel"),
                "launch_ms": admm_ms / max(1, K), "bytes_per_launch": stages * sweep_b}
    elif dominant == "admm":
        src = os.path.join(ROOT, "paper_2606_05687_amd", "csrc", "admm_fused.hip")
        achieved = kernels["admm"]["tflops"]
        roof = {"kernel": "admm_fused_kernel", "bound": "alu", "achieved": achieved,
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                "traffic": measured_traffic(src, "admm_fused_kernel"), "launch_ms": admm_ms,
                "flops_per_launch": stages * SWEEP_FLOPS_PER_STAGE * K}
    else:
        src = os.path.join(ROOT, "paper_2606_05687_amd", "csrc", "setup.hip")
        roof = {"kernel": "setup_kernel", "bound": "alu", "achieved": None,
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": None,
                "traffic": measured_traffic(src, "setup_kernel<4>" if wide else "setup_kernel<2>"),
                "launch_ms": setup_ms}
    # the whole solve against HBM: setup once per stage, K sweeps of operators
    # and iterates, the refinement's pass-stages, over the throughput interval
    # (solves in flight) and over one uncontended solve
    solve_bytes = float(stages * (setup_b + K * sweep_b) + refine_bytes)
    whole = {"bytes_per_solve": solve_bytes,
             "interval_ms": ms_per_step,
             "gbs": solve_bytes / (ms_per_step * 1e-3) / 1e9,
             "frac": solve_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if single is not None:
        whole["one_in_flight_ms"] = single["ms_per_step"]
        whole["one_in_flight_frac"] = (solve_bytes / (single["ms_per_step"] * 1e-3) / 1e9 /
                                       HBM_PEAK_GBS)
    status = out["status"].cpu().numpy()
    line = {
        "metric": METRIC if args.workload == WORKLOAD else
        f"certified MPC solves/s at KKT resid <=1e-5 ({args.workload})",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (ADMM) + f64 (refinement)",
        "data": "synthetic",
        "config": {"workload": args.workload, "batch": int(Bn), "horizon": int(n),
                   "admm_iters": K, "rho": settings["rho"],
                   "form": form_name,
                   "precision": "bf16" if settings.get("precision") else "fp32",
                   "refine_passes": int(settings.get("refine_passes", 8)),
                   "first_passes": int(settings.get("first_passes", 4)),
                   "autotuned": bool(tuned)},
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "certified_frac": certified / (Bn * args.steps),
        "status_counts": {str(k): int((status == k).sum()) for k in range(5)},
        "refine_passes": {"mean": float(passes.mean()), "p99": float(np.percentile(passes, 99)),
                          "max": int(passes.max())},
        "refine_work": work,
        "whole_solve_hbm": whole,
        "phase_ms": {"setup": setup_ms, "admm": admm_ms, "refine": refine_ms},
        "kernels": kernels,
        "timed_graph": bool(args.graph),
        "solves_in_flight": nst,
        "one_in_flight": single,
        "roofline": roof,
    }
    for sv in solvers:
        sv.close()
    if tune_curve:
        # the autotuner's measurements at the chosen rho: sweep count K against
        # solve time and the refinement's mean passes (held-out batch)
        line["passes_vs_sweeps"] = tune_curve
    if args.workload == WORKLOAD:
        line["steps_before_after"] = before_after(batch)
    if args.cpu_sample > 0 and args.workload == WORKLOAD:
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample, args.cpu_workers,
                                            admm_k=K, rho=float(settings["rho"]))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
