"""The paper's simulation protocol on a batch of replicas (Simulation
details; Results).

1. Equilibration at the starting temperature T0 (0.01 K in the paper) with
   the Nose-Hoover thermostat and the axial barostat on the grip separation
   at zero load.
2. A temperature ramp from T0 to each replica's T, barostat off, grips held
   where the barostat left them; then a hold at T.
3. Elongation: the grips are moved apart by grip_step each every grip_hold
   steps (0.05 A every 20 ps in the paper) under Nose-Hoover at T, until
   every replica has failed and been retired (`retire` A of grip travel after
   the first logged rupture; the paper stops 2 A past failure) or the step
   budget ends.  Strain (eq 4) is measured from the equilibrated length.

Every step runs in libtbsma's kernels; this module only sequences the
phases, switches the dynamics settings between calls and collects the
records (analysis.Recorder).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

from .analysis import Recorder
from .engine import WireBatch


@dataclass
class Protocol:
    T0: float = 0.01             # K, equilibration temperature
    nh_tau: float = 0.1          # ps, Nose-Hoover relaxation time
    baro_steps: int = 50000      # 100 ps at 2 fs
    ramp_steps: int = 200000     # 400 ps
    hold_steps: int = 200000     # 400 ps
    baro_mass: float = 1.0e4     # amu
    baro_damp: float = 1.0       # 1/ps
    grip_step: float = 0.05      # A per grip per hold
    grip_hold: int = 10000       # steps (20 ps)
    max_steps: int = 2000000     # elongation budget
    retire: float = 2.0          # A of grip travel after the first rupture
    notch: tuple | None = (3, 4.08)
    steps_per_graph: int = 50
    n_log: int = 1000
    compact: bool = True


@dataclass
class Result:
    recorder: Recorder
    L0: np.ndarray                          # equilibrated lengths (A)
    properties: List[dict] = field(default_factory=list)


def run(replicas: Sequence, proto: Protocol = Protocol(), precision: str = "mixed",
        log=print, **batch_kw) -> Result:
    """Runs the three phases on all replicas in one batch; returns the
    recorder of the elongation and the properties of each replica."""
    b = WireBatch(replicas, precision, gamma=0.0, nh_tau=proto.nh_tau,
                  baro_mass=proto.baro_mass, baro_damp=proto.baro_damp, T_start=proto.T0,
                  ramp_begin=proto.baro_steps, ramp_steps=proto.ramp_steps,
                  notch=proto.notch, retire=proto.retire, n_log=proto.n_log, **batch_kw)
    b.prepare()
    spg = proto.steps_per_graph
    log(f"[protocol] {b.R} replicas, {int(b.n_atoms.sum())} atoms: barostat at "
        f"{proto.T0} K for {proto.baro_steps} steps")
    b.run_batch(proto.baro_steps, spg)
    # grips stay where the barostat left them: references there, no pulling
    s = b.t["baro_s"].view(b.R, 2)[:, 0].cpu().numpy()
    b.t["z0"].copy_(b.t["z"])
    b.t["v_pull"].zero_()
    b.set_dynamics(baro_mass=0.0)
    log(f"[protocol] grip travel at zero load: {s.min():+.3f} .. {s.max():+.3f} A; "
        f"ramp {proto.ramp_steps} + hold {proto.hold_steps} steps")
    b.run_batch(proto.ramp_steps + proto.hold_steps, spg)
    # elongation from the equilibrated state (rebase grows L0 by the
    # barostat's 2 s, still held in baro_s)
    b.rebase()
    b.set_dynamics(grip_step=proto.grip_step, grip_hold=proto.grip_hold, ramp_steps=0)
    L0 = b.L0.copy()
    log(f"[protocol] elongation: {proto.grip_step} A per grip every {proto.grip_hold} "
        f"steps, at most {proto.max_steps} steps")
    rec = Recorder(b)
    rec.run(proto.max_steps, spg, compact=proto.compact)
    props = rec.properties()
    return Result(rec, L0, props)


def summary(result: Result) -> dict:
    """Ensemble statistics of the properties (mean and standard deviation
    over the replicas that failed), as in Table 3."""
    out = {}
    props = result.properties
    failed = [p for p in props if np.isfinite(p["eps_f"])]
    for k in ("E", "sigma_y", "eps_y", "eps_f", "eps_after_yield"):
        v = np.array([p[k] for p in failed], dtype=float)
        out[k] = {"mean": float(v.mean()) if v.size else float("nan"),
                  "std": float(v.std(ddof=1)) if v.size > 1 else float("nan")}
    out["replicas"] = len(props)
    out["failed"] = len(failed)
    return out


def main(argv=None):
    """Runs the protocol on an ensemble of identical wires with distinct
    velocity seeds and prints the per-replica properties and their ensemble
    statistics as one JSON object.  --fast shortens every phase (a
    demonstration; the paper's protocol is the default)."""
    import argparse
    import json
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as W
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--diameter", type=float, default=31.0, help="A")
    ap.add_argument("--length", type=float, default=204.0, help="A")
    ap.add_argument("--T", type=float, default=298.0, help="K")
    ap.add_argument("--replicas", type=int, default=16)
    ap.add_argument("--fast", action="store_true")
    a = ap.parse_args(argv)
    reps = [W.Replica(a.diameter, W.snap_length(a.length), a.T, 0.0, W.seed_of(r), r)
            for r in range(a.replicas)]
    proto = Protocol()
    if a.fast:
        proto = Protocol(baro_steps=2000, ramp_steps=4000, hold_steps=2000, grip_hold=200,
                         max_steps=400000, retire=2.0, n_log=200)
    log = lambda *m: print(*m, file=sys.stderr, flush=True)
    res = run(reps, proto, log=log)
    print(json.dumps({"protocol": proto.__dict__, "L0": res.L0.tolist(),
                      "properties": res.properties, "summary": summary(res)},
                     default=float), flush=True)


if __name__ == "__main__":
    main()
