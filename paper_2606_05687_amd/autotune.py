"""Autotuner for the solve schedule (driver over the C ABI).

Chooses, by measurement on a sample of the workload, the number of ADMM
sweeps K (from one to 200: more sweeps cost sweep time but may give the FP64
refinement a better active set and fewer passes), the penalty rho (1 to 30),
the operator precision, then, at the best of those, the active-set pass budget,
how many of those passes run for every problem before the uncertified ones are
handed to the second refinement launch, and how many problems share one
workgroup of the fused sweep (1, 2 or 4 where they fit); last, at the best of
everything so far, whether the refinement's backward recursion runs
sequentially over the horizon or as an associative scan over 2, 4 or 8 chunks
of it (one wave per chunk).  The sweep form follows the
horizon (fused up to 40 stages, packed by horizon class beyond).  Every
candidate's mean refinement work is logged beside its time, which gives the
refinement-passes-versus-K curve of the workload.  The score
is certified solves per second: problems whose status is certified and whose
reported KKT residuals are all <= the bar, divided by the measured solve time;
a candidate that certifies fewer than ``min_certified`` of the sample is
rejected.  Results are cached in a JSON file keyed by device architecture,
batch size, horizon mix and precision policy.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time

import numpy as np

from . import binding

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pinmpc_tune.json")
LAST_LOG: list = []   # measurements of the last tune() (or its cache entry)


def _key(dev, allow_bf16):
    import torch
    N = dev["N"].cpu().numpy() if "N" in dev else np.full(int(dev["A"].shape[0]),
                                                          int(dev["A"].shape[1]))
    hist = np.bincount(N, minlength=65)
    mix = hashlib.sha1(np.round(hist / max(1, len(N)), 2).tobytes()).hexdigest()[:10]
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return f"{arch}|B{int(dev['A'].shape[0])}|n{int(dev['A'].shape[1])}|mix{mix}|bf16{int(allow_bf16)}"


RHOS = (1.0, 3.0, 10.0, 30.0)
ITERS = (1, 2, 3, 5, 10, 20, 50, 100, 200)
PASSES = (2, 4, 8, 12, 16)
FIRSTS = (0, 2, 4)
GROUPS = (1, 2, 4)
SCANS = (0, 2, 4, 8)
BASE_PASSES, BASE_FIRST = 12, 0


def groups_for(n_max):
    """Problems per workgroup of the fused sweep that fit one workgroup of at
    most 1024 threads (round_up(25 N, 64) threads per problem); the packed
    form (beyond 40 stages) packs its shortest class (20 stages) so."""
    n = n_max if n_max <= 40 else 20
    tpp = ((25 * n + 63) // 64) * 64
    return tuple(g for g in GROUPS if g * tpp <= 1024)


def form_for(n_max):
    """Fused sweeps up to 40 stages, horizon-class packing beyond."""
    return 1 if n_max <= 40 else -1


def stage_a(n_max, allow_bf16=False):
    """First stage of the search: the ADMM schedule (penalty rho and sweep
    count K, from a single sweep up to 200) under the base refinement budget."""
    precs = [0, 1] if allow_bf16 else [0]
    for r, k, p in itertools.product(RHOS, ITERS, precs):
        yield dict(form=form_for(n_max), iters=k, rho=r, refine_passes=BASE_PASSES,
                   first_passes=BASE_FIRST, precision=p, group=1, scan=0)


def stage_b(best, n_max=20):
    """Second stage: the refinement's pass budget and launch split, and the
    problems per workgroup of the fused sweep, at the best ADMM schedule of the
    first stage."""
    for pa, p1, g in itertools.product(PASSES, FIRSTS, groups_for(n_max)):
        if (pa, p1, g) == (best["refine_passes"], best["first_passes"], best["group"]):
            continue
        yield dict(best, refine_passes=pa, first_passes=p1, group=g)


def stage_c(best, n_max=20):
    """Third stage: the refinement's backward recursion, sequential or an
    associative scan over 2, 4 or 8 chunks of the horizon, at the best
    schedule of the first two stages (horizons under 8 stages always run
    sequentially, so only longer ones try the scan)."""
    if n_max < 8:
        return
    for w in SCANS:
        if w != best.get("scan", 0):
            yield dict(best, scan=w)


def candidates(n_max, allow_bf16=False):
    """Every candidate the search can measure (both stages over all first-stage
    winners); the search itself measures stage_a, then stage_b of its best."""
    seen = set()
    for a in stage_a(n_max, allow_bf16):
        for c in [a, *stage_b(a, n_max), *stage_c(a, n_max)]:
            key = tuple(sorted(c.items()))
            if key not in seen:
                seen.add(key)
                yield c


def measure(solvers, streams, dev, outs, bs, settings, reps=4, kkt_bar=1e-5):
    """Seconds per solve with len(solvers) solves in flight (round robin over
    the streams), the certified fraction, and the mean refinement work per
    problem (equality-constrained passes, interior-point iterations)."""
    import torch
    for sv in solvers:
        sv.set(**settings)
    for sv, o, st in zip(solvers, outs, streams):
        sv.solve(dev, o, stream=st, batch_struct=bs)   # warm-up (and graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(reps):
        k = i % len(solvers)
        solvers[k].solve(dev, outs[k], stream=streams[k], batch_struct=bs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    out = outs[0]
    ok = (out["status"] == 0) & (out["res"].max(dim=1).values <= kkt_bar)
    frac = float(ok.float().mean().item())
    det = out["detail"].float()
    return dt, frac, float(det[:, 0].mean().item()), float(det[:, 1].mean().item())


def tune(dev, allow_bf16=False, cache_path=DEFAULT_CACHE, min_certified=0.999, verbose=False,
         force=False, in_flight=1, base=None):
    """Best settings (dict) for batches shaped like ``dev``, measured with
    `in_flight` solves on as many streams, every candidate on top of the
    settings in ``base`` (for example a larger interior-point cap for long
    horizons); cached."""
    import torch
    key = _key(dev, allow_bf16) + f"|inflight{int(in_flight)}"
    if base:
        key += "|" + ",".join(f"{k}={v}" for k, v in sorted(base.items()))
    cache = {}
    if os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    global LAST_LOG
    if key in cache and not force:
        LAST_LOG = cache[key].get("log", [])
        return cache[key]["settings"]
    n = max(1, int(in_flight))
    solvers = [binding.Solver(0, **(base or {})) for _ in range(n)]
    outs = [sv.alloc_out(dev) for sv in solvers]
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(n - 1)]
    bs = binding.make_batch_struct(dev)
    Bn = int(dev["A"].shape[0])
    best, best_score, log = None, -1.0, []

    def run(cands):
        nonlocal best, best_score
        for cand in cands:
            dt, frac, eq, ipm = measure(solvers, streams, dev, outs, bs, cand)
            score = frac * Bn / dt if frac >= min_certified else 0.0
            log.append(dict(cand, ms=dt * 1e3, certified=frac, score=score, eq_passes=eq,
                            ipm_iters=ipm))
            if verbose:
                print(f"  {cand} {dt * 1e3:.2f} ms certified {frac:.4f} passes {eq:.2f}+{ipm:.2f}"
                      f" -> {score:.0f}/s", flush=True)
            if score > best_score:
                best, best_score = cand, score

    run(stage_a(int(dev["A"].shape[1]), allow_bf16))
    if best is not None:
        run(list(stage_b(best, int(dev["A"].shape[1]))))
    if best is not None:
        run(list(stage_c(best, int(dev["A"].shape[1]))))
    for sv in solvers:
        sv.close()
    LAST_LOG = log
    if best is not None and base:
        best = dict(base, **best)
    cache[key] = {"settings": best, "score": best_score, "log": log}
    os.makedirs(os.path.dirname(cache_path) or ".", exist_ok=True)
    with open(cache_path, "w") as f:
        json.dump(cache, f, indent=1)
    return best
