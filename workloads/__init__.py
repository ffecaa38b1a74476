"""Seeded synthetic workloads: which nanowire replicas to build.

This module is shared by the tests, the benchmark and both compute sides (the
HIP library and the CPU oracle).  It holds none of the method's arithmetic:
only the geometry and thermostat settings of each replica, drawn from a fixed
seed, in the shapes of the paper's wires (Simulation details: [100] Au wires,
diameters of a few nm, lengths of tens of nm, 10 K and 298 K).  The paper
measures on its own generated wires, not a public dataset; these stand in for
them.

Lengths are snapped to whole (002) layers of the FCC lattice (spacing a/2),
so that the wire builder keeps exactly n_layers planes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

S0 = 13113890          # master seed of every workload
A_LAT = 4.08           # Angstrom, FCC lattice constant of the generated wires
DT = 0.002             # ps (Simulation details: 2.0 fs)


@dataclass
class Replica:
    D: float            # Angstrom, cylinder diameter
    L: float            # Angstrom, generated length (whole (002) layers)
    T: float            # K
    v_pull: float       # Angstrom/ps, speed of the pulled grip
    seed: int           # 64-bit Philox key of this replica
    rep_id: int         # persistent replica id (a Philox counter word)
    jitter: float = 0.0  # Angstrom, uniform position jitter amplitude
    n_grip: int = 2     # (002) planes per grip


@dataclass
class Workload:
    name: str
    replicas: List[Replica]
    precision: str      # "fp64" or "mixed"
    steps: int          # protocol length (steps)
    gamma: float = 1.0  # 1/ps
    skin: float = 1.0   # Angstrom, Verlet skin of the full lists
    prune: float = 0.15  # Angstrom, half-width of the pruned lists (mixed)
    k_cap: int = 176    # Verlet-list capacity per atom (grown at the first build)
    notes: str = ""
    extra: dict = field(default_factory=dict)


def snap_length(L: float, a: float = A_LAT) -> float:
    """Length of the nearest whole number of (002) layers (>= 4 layers)."""
    n = max(4, int(round(L / (0.5 * a))))
    return n * (0.5 * a)


def seed_of(r: int) -> int:
    return S0 * 1000 + r


def wire_d1p5_l3_fp64() -> Workload:
    """One D 1.5 nm x L 3 nm wire, FP64, 10 K, 1000 steps at 0.5 A/ps."""
    return Workload("plain-fp64 D1.5xL3nm", [
        Replica(15.0, snap_length(30.0), 10.0, 0.5, seed_of(0), 0)],
        "fp64", 1000)


def wire_d3_l20_mixed() -> Workload:
    """One D 3 nm x L 20 nm wire with +-0.02 A jitter, mixed precision, 10 K."""
    return Workload("single-mixed D3xL20nm", [
        Replica(30.0, snap_length(200.0), 10.0, 0.5, seed_of(0), 0, jitter=0.02)],
        "mixed", 50000)


def batch512_d3(n_rep: int = 512) -> Workload:
    """512 D 3 nm wires, lengths uniform in 5-40 nm, 298 K, 0.5 A/ps."""
    rng = np.random.default_rng(S0)
    Ls = rng.uniform(50.0, 400.0, size=n_rep)
    reps = [Replica(30.0, snap_length(float(Ls[r])), 298.0, 0.5, seed_of(r), r)
            for r in range(n_rep)]
    # skin 2.6 A: with pruned lists the pair work does not grow with the
    # skin, and the pruning reads only the part of each row beyond its core,
    # so longer rows cost little while rebuilds become rare (measured fastest
    # of 1.6-3.2 A); the capacity leaves room for rows to grow in the run
    return Workload(f"batched {n_rep}x D3nm L5-40nm 298K", reps, "mixed", 20000, skin=2.6,
                    k_cap=264)


def batch2048_mixed_shapes(n_rep: int = 2048) -> Workload:
    """2048 wires: D in {1.5, 2, 2.5, 3} nm (r mod 4), L uniform in 3-30 nm,
    10 K for even r and 298 K for odd r, 0.1/0.5/1.0 A/ps (r mod 3)."""
    rng = np.random.default_rng(S0 + 4)
    Ls = rng.uniform(30.0, 300.0, size=n_rep)
    Ds = (15.0, 20.0, 25.0, 30.0)
    rates = (0.1, 0.5, 1.0)
    reps = [Replica(Ds[r % 4], snap_length(float(Ls[r])), 10.0 if r % 2 == 0 else 298.0,
                    rates[r % 3], seed_of(r), r) for r in range(n_rep)]
    return Workload(f"mixed-shapes {n_rep}x D1.5-3nm L3-30nm", reps, "mixed", 20000, skin=2.6,
                    k_cap=264)


def wire_d10_l100() -> Workload:
    """One D 10 nm x L 100 nm wire, mixed precision, 298 K, 20k steps."""
    return Workload("large D10xL100nm", [
        Replica(100.0, snap_length(1000.0), 298.0, 0.5, seed_of(0), 0)],
        "mixed", 20000)


WORKLOADS = {
    "d1.5-l3-fp64": wire_d1p5_l3_fp64,
    "d3-l20": wire_d3_l20_mixed,
    "batch512-d3": batch512_d3,
    "batch2048-mixed": batch2048_mixed_shapes,
    "d10-l100": wire_d10_l100,
}
