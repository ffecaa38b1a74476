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
    """Logs (step, strain = step/1000 + replica/10) for its replicas into an
    8-slot ring every 5 steps, like the device does; replica r retires at
    logged step done_at[r] and then repeats its last record."""

    def __init__(self, reps=(0, 1), done_at=None, step=0, compactions=None):
        self.reps = list(reps)
        self.n_log, self.n_slots, self.R = 5, 8, len(self.reps)
        self.done_at = done_at or {}
        self.ring = np.zeros((self.n_slots, self.R, A.NOBS))
        self.st = np.zeros(self.R, dtype=np.uint32)
        self.step = step
        self.compactions = compactions if compactions is not None else []

    def run_batch(self, n, spg):
        for _ in range(n):
            self.step += 1
            if self.step % self.n_log:
                continue
            slot = (self.step // self.n_log) % self.n_slots
            prev = ((self.step // self.n_log) - 1) % self.n_slots
            for j, r in enumerate(self.reps):
                if self.st[j] & A.ST_DONE:
                    self.ring[slot, j] = self.ring[prev, j]
                    continue
                self.ring[slot, j, A.OBS_STEP] = self.step
                self.ring[slot, j, A.OBS_STRAIN] = self.step / 1000.0 + r / 10.0
                if self.step >= self.done_at.get(r, 1 << 30):
                    self.st[j] |= A.ST_DONE | A.ST_RUPTURED
                    self.ring[slot, j, A.OBS_STATUS] = self.st[j]

    def obs(self):
        return self.ring.copy()

    def status(self):
        return self.st.copy()

    def compact(self, keep):
        nb = _FakeBatch([self.reps[j] for j in keep], self.done_at, self.step,
                        self.compactions)
        nb.ring = self.ring[:, keep].copy()
        nb.st = self.st[keep].copy()
        self.compactions.append([self.reps[j] for j in keep])
        return nb


def test_recorder_keeps_every_record_of_a_long_run():
    b = _FakeBatch()
    rec = AN.Recorder(b)
    rec.run(300, steps_per_graph=10)
    eps, _, _ = rec.curve(0)
    assert np.array_equal(eps, np.arange(5, 301, 5) / 1000.0)


def test_recorder_skips_repeated_records_of_retired_replicas():
    # replica 0 retires at step 100: its records stop there, replica 1's go on
    b = _FakeBatch(done_at={0: 100})
    rec = AN.Recorder(b)
    rec.run(300, steps_per_graph=10)
    e0, _, s0 = rec.curve(0)
    e1, _, _ = rec.curve(1)
    assert np.array_equal(e0, np.arange(5, 101, 5) / 1000.0)
    assert s0[-1] & A.ST_DONE and not s0[:-1].any()
    assert np.array_equal(e1, np.arange(5, 301, 5) / 1000.0 + 0.1)


def test_recorder_compaction_keeps_records_by_original_index():
    b = _FakeBatch(reps=(0, 1, 2), done_at={1: 40, 0: 120, 2: 200})
    rec = AN.Recorder(b)
    rec.run(400, steps_per_graph=10, compact=True)
    # chunks of 40 steps: replica 1 dropped after the chunk ending at 40,
    # replica 0 after 120, and the run stops once replica 2 retires at 200
    assert b.compactions == [[0, 2], [2]]
    assert rec.b.step == 200 and len(rec.ids) == 0
    for r, end in ((0, 120), (1, 40), (2, 200)):
        e, _, s = rec.curve(r)
        assert np.array_equal(e, np.arange(5, end + 1, 5) / 1000.0 + r / 10.0)
        assert s[-1] & A.ST_DONE


def test_protocol_summary_over_failed_replicas():
    from paper_1311_3890_amd import protocol as P
    props = [dict(E=80.0, sigma_y=4.0, eps_y=0.05, eps_f=0.30, eps_after_yield=0.25),
             dict(E=90.0, sigma_y=5.0, eps_y=0.07, eps_f=0.40, eps_after_yield=0.33),
             dict(E=99.0, sigma_y=9.0, eps_y=0.09, eps_f=math.nan, eps_after_yield=math.nan)]
    s = P.summary(P.Result(None, np.zeros(3), props))
    assert s["replicas"] == 3 and s["failed"] == 2
    assert abs(s["E"]["mean"] - 85.0) < 1e-12 and abs(s["E"]["std"] - math.sqrt(50.0)) < 1e-12
    assert abs(s["eps_f"]["mean"] - 0.35) < 1e-12
