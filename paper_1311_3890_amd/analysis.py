"""Stress-strain products of elongation runs (Results; eq 4, eq 6, Table 3).

Host-side post-processing of the per-replica observables the step loops log
(`WireBatch.obs`): strain (eq 4), axial stress (eq 5) and status bits.  It
does no simulation arithmetic.

* `Recorder` drains a batch's observable ring after each chunk of steps, so
  runs longer than n_log * n_slots steps keep every record.
* `properties` reduces one replica's curve to Young's modulus (slope of the
  initial linear part), yield stress and strain (the stress maximum before
  failure), failure strain (the first logged step with a rupture) and the
  strain after yielding (the paper's measure of ductility, Figure 9).
* `critical_length` is eq 6: L_C = D0 cot(alpha) / eps_y.
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

from . import _abi as A


def critical_length(D0: float, eps_y: float, cot_alpha: float) -> float:
    """Eq 6: critical initial length above which a wire of diameter D0 and
    yield strain eps_y fails by brittle shear; cot(alpha) is 1 for perfect
    and sqrt(2) for partial dislocations in [100] wires."""
    return D0 / eps_y * cot_alpha


def properties(strain, stress, status=None, eps_lin: float = 0.02) -> Dict[str, float]:
    """Mechanical properties of one stress-strain curve (records in step
    order; stress in GPa).

    E        slope (GPa) of the least-squares line through the records with
             strain <= eps_lin (and before failure);
    sigma_y  largest stress before failure; eps_y its strain;
    eps_f    strain of the first record whose status has the rupture bit
             (nan if the wire has not failed);
    eps_after_yield  eps_f - eps_y.
    """
    e = np.asarray(strain, dtype=float)
    s = np.asarray(stress, dtype=float)
    n = e.size
    fail = n
    if status is not None:
        st = np.asarray(status).astype(np.int64)
        hit = np.nonzero(st & A.ST_RUPTURED)[0]
        if hit.size:
            fail = int(hit[0])
    eps_f = float(e[fail]) if fail < n else math.nan
    pre = slice(0, max(fail, 1))
    k = int(np.argmax(s[pre]))
    lin = np.nonzero(e[pre] <= eps_lin)[0]
    E = float(np.polyfit(e[lin], s[lin], 1)[0]) if lin.size >= 2 else math.nan
    return {"E": E, "sigma_y": float(s[k]), "eps_y": float(e[k]), "eps_f": eps_f,
            "eps_after_yield": eps_f - float(e[k])}


class Recorder:
    """Keeps every observable record of a WireBatch: run() advances it in
    chunks that fit the ring and drains the ring after each.  With
    compact=True the batch is replaced, after each chunk in which a replica
    was retired, by its compacted copy (WireBatch.compact); records stay
    keyed by the replica's index in the original batch."""

    def __init__(self, batch):
        self.b = batch
        self.ids = np.arange(batch.R)                # original index of each batch row
        self.rows: List[List[np.ndarray]] = [[] for _ in range(batch.R)]
        self.last = np.full(batch.R, -1, dtype=np.int64)

    def drain(self):
        ring = self.b.obs()                          # [n_slots, R, NOBS]
        steps = ring[:, :, A.OBS_STEP].astype(np.int64)
        for j, r in enumerate(self.ids):
            # a retired replica repeats its last record: only newer steps count
            for slot in np.argsort(steps[:, j], kind="stable"):
                st = int(steps[slot, j])
                if st > self.last[r] and st > 0:
                    self.rows[r].append(ring[slot, j].copy())
                    self.last[r] = st

    def compact(self) -> bool:
        """Drops retired replicas from the batch; False once none is left."""
        st = np.asarray(self.b.status()).astype(np.int64)
        keep = [j for j in range(len(self.ids)) if not st[j] & A.ST_DONE]
        if len(keep) == len(self.ids):
            return True
        nb = self.b.compact(keep) if keep else None
        self.ids = self.ids[keep]
        if nb is None:
            return False
        self.b = nb
        return True

    def run(self, n_steps: int, steps_per_graph: int = 50, compact: bool = False):
        chunk = self.b.n_log * self.b.n_slots
        chunk -= chunk % steps_per_graph if chunk > steps_per_graph else 0
        done = 0
        while done < n_steps:
            k = min(chunk, n_steps - done)
            self.b.run_batch(k, steps_per_graph)
            done += k
            self.drain()
            if compact and not self.compact():
                break

    def curve(self, r: int):
        """(strain, stress GPa, status) of original replica r, one entry per
        logged step."""
        if not self.rows[r]:
            return np.zeros(0), np.zeros(0), np.zeros(0, dtype=np.int64)
        a = np.stack(self.rows[r])
        return a[:, A.OBS_STRAIN], a[:, A.OBS_SZZ], a[:, A.OBS_STATUS].astype(np.int64)

    def properties(self, eps_lin: float = 0.02):
        return [properties(*self.curve(r), eps_lin=eps_lin) for r in range(len(self.rows))]
