"""Stress-strain post-processing (CPU): eq 6 against the paper's worked
example, the property extraction on curves with known answers, and the
observable-ring recorder on a stand-in batch."""
import math
import os

import numpy as np

from paper_1311_3890_amd import _abi as A
from paper_1311_3890_amd import analysis as AN

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_critical_length_matches_the_papers_example():
    rows = np.loadtxt(os.path.join(GOLD, "critical_length_example.txt"))
    for D0, eps_y, cot, lc in rows:
        assert abs(AN.critical_length(D0, eps_y, cot) - lc) < 0.05


def test_properties_of_a_known_curve():
    # linear elastic 100 GPa up to strain 0.05, then a drop and a plateau,
    # rupture reported at strain 0.15
    e = np.linspace(0.0, 0.2, 201)
    s = np.where(e <= 0.05, 100.0 * e, 1.0)
    st = np.where(e >= 0.15, A.ST_RUPTURED, 0)
    p = AN.properties(e, s, st)
    assert abs(p["E"] - 100.0) < 1e-9
    assert p["sigma_y"] == 5.0 and abs(p["eps_y"] - 0.05) < 1e-12
    assert abs(p["eps_f"] - 0.15) < 1e-12
    assert abs(p["eps_after_yield"] - 0.10) < 1e-12
    # no rupture: eps_f is nan
    q = AN.properties(e, s, np.zeros_like(st))
    assert math.isnan(q["eps_f"]) and q["sigma_y"] == 5.0


class _FakeBatch:
    """Logs (step, strain = step/1000) for 2 replicas into an 8-slot ring
    every 5 steps, like the device does."""

    def __init__(self):
        self.n_log, self.n_slots, self.R = 5, 8, 2
        self.ring = np.zeros((self.n_slots, self.R, A.NOBS))
        self.step = 0

    def run_batch(self, n, spg):
        for _ in range(n):
            self.step += 1
            if self.step % self.n_log == 0:
                slot = (self.step // self.n_log) % self.n_slots
                self.ring[slot, :, A.OBS_STEP] = self.step
                self.ring[slot, :, A.OBS_STRAIN] = self.step / 1000.0

    def obs(self):
        return self.ring.copy()


def test_recorder_keeps_every_record_of_a_long_run():
    b = _FakeBatch()
    rec = AN.Recorder(b)
    rec.run(300, steps_per_graph=10)
    eps, _, _ = rec.curve(0)
    assert np.array_equal(eps, np.arange(5, 301, 5) / 1000.0)
