"""Per-bucket launch shapes of the pair passes, chosen by timed trials on the
whole batch.

Replicas fall into buckets of equal diameter and temperature class.  For each
bucket the tuner tries every candidate launch shape, made of the tiles per
pair-pass block (1, 2 or 4) and the stage class (1152 or 1536 neighbour
positions staged in LDS per block).  Smaller blocks give more, shorter
workgroups.  The smaller stage lets the density pass keep more workgroups
resident per CU, but blocks whose slot window exceeds it read their
neighbours from global memory.  Every trial times the whole batch, with the
other buckets at their current choice, so per-bucket shapes are chosen for
the way they run together: one batch, one HIP graph, one launch per stage
class per pass.  Shapes change where work runs, not what is computed: the
tuned batch's trajectories equal the untuned ones bit for bit.

The trial rate is the median of a few timed windows (HIP events on the
launch stream) after a short warm-up.  A candidate replaces the current
choice only when it is faster by more than the tolerance.  Choices are
cached as JSON, keyed by the workload's bucket signature, the precision, the
Verlet skin and pruning width, and the candidate grid.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, List, Sequence, Tuple

import numpy as np
import torch

from . import _abi as A
from .engine import WireBatch

CANDIDATES = tuple(A.shape(t, c) for t in (4, 2, 1) for c in (1, 0))


def bucket_of(rp) -> Tuple[float, str]:
    return (float(rp.D), "cold" if rp.T < 100.0 else "warm")


def buckets(replicas: Sequence) -> Dict[Tuple[float, str], List[int]]:
    out: Dict[Tuple[float, str], List[int]] = {}
    for r, rp in enumerate(replicas):
        out.setdefault(bucket_of(rp), []).append(r)
    return dict(sorted(out.items()))


def bucket_key(b) -> str:
    return f"D{b[0]:g}-{b[1]}"


def shape_name(s: int) -> str:
    return f"{s & 15} tiles/block, stage {1152 if (s >> 4) == 0 else 1536}"


def cache_key(wb: WireBatch, candidates: Sequence[int]) -> str:
    sig = {"buckets": {bucket_key(b): [len(idx), int(sum(int(wb.n_atoms[r]) for r in idx))]
                       for b, idx in buckets(wb.replicas).items()},
           "precision": wb.precision, "skin": wb.skin, "prune": wb.prune,
           "candidates": list(candidates)}
    return hashlib.sha1(json.dumps(sig, sort_keys=True).encode()).hexdigest()[:16]


def measure(wb: WireBatch, steps: int, warmup: int, windows: int, spg: int) -> float:
    """Median atom-timesteps/s of `windows` timed windows of `steps` steps."""
    n = float(wb.n_atoms.sum())
    wb.run_batch(warmup, spg)
    rates = []
    stream = torch.cuda.current_stream()
    for _ in range(windows):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        wb.run_batch(steps, spg)
        e1.record(stream)
        torch.cuda.synchronize()
        rates.append(n * steps / (e0.elapsed_time(e1) * 1e-3))
    return float(np.median(rates))


def tune(wb: WireBatch, *, candidates: Sequence[int] = CANDIDATES, steps: int = 100,
         warmup: int = 50, windows: int = 3, steps_per_graph: int = 50, tol: float = 0.005,
         cache: str | None = None, log=print) -> dict:
    """Chooses one launch shape per bucket of wb's replicas by coordinate
    descent over the buckets on the whole batch, applies the choices to wb
    (set_shapes) and returns them with the trial rates."""
    key = cache_key(wb, candidates)
    blist = buckets(wb.replicas)
    cached = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            cached = json.load(fh)
    if key in cached:
        res = cached[key]
        shapes = [A.SHAPE_DEFAULT] * wb.R
        for b, idx in blist.items():
            for r in idx:
                shapes[r] = res["choice"][bucket_key(b)]
        wb.set_shapes(shapes)
        log(f"[autotune] cached choices {res['choice']}")
        return res
    t0 = time.perf_counter()
    shapes = list(wb.shapes) if wb.shapes is not None else [A.SHAPE_DEFAULT] * wb.R
    wb.set_shapes(shapes)
    best_rate = measure(wb, steps, warmup, windows, steps_per_graph)
    untuned = best_rate
    log(f"[autotune] start: {best_rate:.4e} atom-steps/s")
    choice, trials = {}, []
    for b, idx in blist.items():
        k = bucket_key(b)
        cur = shapes[idx[0]]
        for cand in candidates:
            if cand == cur:
                continue
            trial = list(shapes)
            for r in idx:
                trial[r] = cand
            wb.set_shapes(trial)
            rate = measure(wb, steps, warmup, windows, steps_per_graph)
            trials.append({"bucket": k, "shape": cand, "rate": rate})
            log(f"[autotune] {k}: {shape_name(cand)}: {rate:.4e} atom-steps/s "
                f"(best {best_rate:.4e})")
            if rate > best_rate * (1.0 + tol):
                best_rate, cur = rate, cand
        for r in idx:
            shapes[r] = cur
        choice[k] = cur
    wb.set_shapes(shapes)
    res = {"choice": choice, "names": {k: shape_name(v) for k, v in choice.items()},
           "untuned_trial_rate": untuned, "tuned_trial_rate": best_rate, "trials": trials,
           "seconds": time.perf_counter() - t0}
    if cache:
        merged = dict(cached)
        merged[key] = res
        with open(cache, "w") as fh:
            json.dump(merged, fh, indent=1)
    return res


def per_bucket_rates(replicas: Sequence, choice: dict, precision: str, *, skin: float,
                     prune: float, k_cap: int = 176, steps: int = 200, warmup: int = 200,
                     steps_per_graph: int = 50, log=print) -> dict:
    """Rate of each bucket alone (one batch of its replicas, with its tuned
    shape): the per-replica-size throughput.  Context for the one-batch
    rate, which is the one a workload runs at."""
    out = {}
    for b, idx in buckets(replicas).items():
        k = bucket_key(b)
        wb = WireBatch([replicas[r] for r in idx], precision, skin=skin, prune=prune,
                       k_cap=k_cap, n_log=steps_per_graph, shapes=[choice[k]] * len(idx))
        wb.prepare()
        rate = measure(wb, steps, warmup, 1, steps_per_graph)
        out[k] = {"replicas": len(idx), "atoms": int(wb.n_atoms.sum()),
                  "shape": shape_name(choice[k]), "atom_timesteps_per_s": rate}
        log(f"[autotune] bucket {k} alone: {out[k]}")
        del wb
        torch.cuda.empty_cache()
    return out


def main(argv=None):
    """Tunes the launch shapes of a workload's buckets in one batch and
    prints one JSON object: the choices, the one-batch rate before and after
    (timed windows of --steps after the tuning), and each bucket's rate
    alone."""
    import argparse
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as W
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--workload", default="batch2048-mixed", choices=sorted(W.WORKLOADS))
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--thermalize", type=int, default=1000)
    ap.add_argument("--trial-steps", type=int, default=100)
    ap.add_argument("--cache", default=None, help="JSON file of earlier choices")
    ap.add_argument("--no-per-bucket", action="store_true")
    a = ap.parse_args(argv)
    log = lambda *m: print(*m, file=sys.stderr, flush=True)
    wl = W.WORKLOADS[a.workload]()
    torch.cuda.set_device(0)
    wb = WireBatch(wl.replicas, wl.precision, skin=wl.skin, prune=wl.prune, n_log=50,
                   gamma=wl.gamma, k_cap=wl.k_cap)
    wb.prepare()
    wb.run_batch(a.thermalize, 50)
    untuned = measure(wb, a.steps, 50, 1, 50)
    res = tune(wb, steps=a.trial_steps, cache=a.cache, log=log)
    tuned = measure(wb, a.steps, 50, 1, 50)
    out = {"workload": wl.name, "atoms": int(wb.n_atoms.sum()), "steps": a.steps,
           "untuned_atom_timesteps_per_s": untuned, "tuned_atom_timesteps_per_s": tuned,
           "choice": res["names"], "tuning_seconds": res.get("seconds")}
    del wb
    torch.cuda.empty_cache()
    if not a.no_per_bucket:
        out["per_bucket"] = per_bucket_rates(wl.replicas, res["choice"], wl.precision,
                                             skin=wl.skin, prune=wl.prune, k_cap=wl.k_cap,
                                             log=log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
