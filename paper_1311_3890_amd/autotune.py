"""Per-bucket launch settings chosen by short timed trials.

Replicas are grouped into buckets of equal diameter and temperature class.
For each bucket a sample of its replicas is run through the batched graph
path for every candidate Verlet skin (with the cell edge r_cut + skin),
pruning half-width and graph chunk length; the fastest setting in
atom-timesteps/s is kept.  The skin trades the length of the full lists
(the work of each rebuild and pruning) against rebuild frequency, which
depends on temperature and diameter; the pruning half-width trades the length
of the lists the pair passes read against pruning frequency; the chunk length
trades graph launch overhead against the step granularity of the host loop.
Choices are cached as JSON so later runs reuse them.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import asdict, dataclass
from typing import Dict, List, Sequence, Tuple

import numpy as np
import torch

from .engine import WireBatch


@dataclass
class Choice:
    skin: float
    prune: float
    steps_per_graph: int
    rate: float          # atom-timesteps/s of the trial
    trials: list


def bucket_of(rp) -> Tuple[float, str]:
    return (float(rp.D), "cold" if rp.T < 100.0 else "warm")


def buckets(replicas: Sequence) -> Dict[Tuple[float, str], List[int]]:
    out: Dict[Tuple[float, str], List[int]] = {}
    for r, rp in enumerate(replicas):
        out.setdefault(bucket_of(rp), []).append(r)
    return dict(sorted(out.items()))


def _key(b) -> str:
    return f"D{b[0]:g}-{b[1]}"


def _time_batch(reps, skin, prune, spg, trial_steps, warmup, precision):
    wb = WireBatch(reps, precision, skin=skin, prune=prune, n_log=spg)
    wb.prepare()
    wb.run_batch(warmup, spg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wb.run_batch(trial_steps, spg)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rate = float(wb.n_atoms.sum()) * trial_steps / dt
    del wb
    return rate


def tune(replicas: Sequence, precision: str = "mixed", *,
         skins=(1.0, 1.3, 1.6, 2.0), prunes=(0.1, 0.15, 0.2), chunks=(50,),
         sample: int = 32, trial_steps: int = 100, warmup: int = 100,
         cache: str | None = None, log=print) -> Dict[str, Choice]:
    """Best (skin, prune, steps_per_graph) per bucket of `replicas`."""
    cached = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            cached = json.load(fh)
    result: Dict[str, Choice] = {}
    for b, idx in buckets(replicas).items():
        k = _key(b)
        if k in cached:
            result[k] = Choice(**cached[k])
            continue
        pick = np.linspace(0, len(idx) - 1, min(sample, len(idx))).round().astype(int)
        reps = [replicas[idx[p]] for p in pick]
        trials = []
        for skin in skins:
            for prune in (prunes if precision == "mixed" else (0.0,)):
                for spg in chunks:
                    rate = _time_batch(reps, skin, prune, spg, trial_steps, warmup, precision)
                    trials.append((skin, prune, spg, rate))
                    log(f"[autotune] {k}: skin {skin} prune {prune} chunk {spg}: "
                        f"{rate:.3e} atom-steps/s")
        skin, prune, spg, rate = max(trials, key=lambda t: t[3])
        result[k] = Choice(skin, prune, spg, rate, trials)
    if cache:
        merged = dict(cached)
        merged.update({k: asdict(v) for k, v in result.items()})
        with open(cache, "w") as fh:
            json.dump(merged, fh, indent=1)
    return result


class BucketRun:
    """The replicas of a workload as one WireBatch per bucket, each with its
    tuned settings, advanced in turn."""

    def __init__(self, replicas: Sequence, choices: Dict[str, Choice],
                 precision: str = "mixed", n_log: int = 100):
        self.parts = []
        for b, idx in buckets(replicas).items():
            c = choices[_key(b)]
            wb = WireBatch([replicas[r] for r in idx], precision, skin=c.skin, prune=c.prune,
                           n_log=n_log)
            self.parts.append((_key(b), idx, c, wb))
        self.n_atoms = sum(int(wb.n_atoms.sum()) for _, _, _, wb in self.parts)

    def prepare(self):
        for _, _, _, wb in self.parts:
            wb.prepare()

    def run(self, n: int):
        for _, _, c, wb in self.parts:
            wb.run_batch(n, c.steps_per_graph)


def _pass_us(wb, p: int, n: int = 10) -> float:
    """Average launch time (us) of force pass p on wb's current state, HIP
    events on the launch stream."""
    import ctypes as C
    from . import _abi as A
    lib = A.lib()
    args = (C.byref(wb.params), C.byref(wb.sys), C.byref(wb.nlist), C.byref(wb.out), wb.work)
    A.check(lib.tbsma_forces_pass(*args, p, wb.stream()))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(n):
        A.check(lib.tbsma_forces_pass(*args, p, wb.stream()))
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n * 1e3


def main(argv=None):
    """Tunes the buckets of a workload, then times each bucket's batch with its
    chosen settings; prints one JSON object."""
    import argparse
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as W
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--workload", default="batch2048-mixed", choices=sorted(W.WORKLOADS))
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--sample", type=int, default=32)
    ap.add_argument("--trial-steps", type=int, default=100)
    ap.add_argument("--cache", default=None, help="JSON file of earlier choices")
    a = ap.parse_args(argv)
    log = lambda *m: print(*m, file=sys.stderr, flush=True)
    wl = W.WORKLOADS[a.workload]()
    choices = tune(wl.replicas, wl.precision, sample=a.sample, trial_steps=a.trial_steps,
                   warmup=a.warmup, cache=a.cache, log=log)
    run = BucketRun(wl.replicas, choices, wl.precision)
    run.prepare()
    out = {"workload": wl.name, "atoms": run.n_atoms, "steps": a.steps, "buckets": {}}
    total_s = 0.0
    for k, idx, c, wb in run.parts:
        wb.run_batch(a.warmup, c.steps_per_graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        wb.run_batch(a.steps, c.steps_per_graph)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        total_s += dt
        n = int(wb.n_atoms.sum())
        kbar, kp = wb.list_lengths()
        t3 = _pass_us(wb, 3)
        out["buckets"][k] = {
            "replicas": len(idx), "atoms": n, "skin_A": c.skin, "prune_A": c.prune,
            "steps_per_graph": c.steps_per_graph,
            "atom_timesteps_per_s": n * a.steps / dt,
            "mean_listed_neighbours": kbar,
            "mean_pruned_list": kp,
            "force_pass_us": t3,
            "force_pass_GB_per_s": n * (4.0 * kp + 32.0) / (t3 * 1e-6) / 1e9}
        log(f"[autotune] {k}: {out['buckets'][k]}")
    out["atom_timesteps_per_s"] = run.n_atoms * a.steps / total_s
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
