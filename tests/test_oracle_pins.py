"""Pins of the FP64 oracle to facts outside itself (CPU only).

Each test fixes part of the oracle with something the paper or the
mathematics determines: closed-form lattice sums with textbook FCC shell
counts, the dimer closed form, finite differences of the energy, Newton's
third law, invariances, the open-boundary virial identity, Hermite tail
conditions, NVE conservation and time reversibility of velocity Verlet, the
Langevin equipartition, and the published Philox known-answer vectors.
"""
import math
import os

import numpy as np
import pytest

import oracle

AU = oracle.Pot()
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def fcc_shell_energy(pot, a, shells):
    """Energy of one atom in a perfect FCC crystal from (count, r/a) shells,
    written with math.exp independently of the oracle."""
    rho = 0.0
    rep = 0.0
    for cnt, ra in shells:
        r = ra * a
        rho += cnt * pot.xi ** 2 * math.exp(-2 * pot.q * (r / pot.r0 - 1))
        rep += cnt * pot.A * math.exp(-pot.p * (r / pot.r0 - 1))
    return -math.sqrt(rho) + rep


# FCC coordination shells: 12 at a/sqrt2, 6 at a, 24 at a sqrt(3/2),
# 12 at a sqrt2, 24 at a sqrt(5/2); the next (8 at a sqrt3 = 7.07 A) lies
# beyond the 7.0 A cutoff.
FCC5 = [(12, math.sqrt(0.5)), (6, 1.0), (24, math.sqrt(1.5)), (12, math.sqrt(2.0)),
        (24, math.sqrt(2.5))]


def center_energy(pot, a):
    x, y, z, _ = oracle.build_wire(a, 3.2 * pot.r_cut, 3.2 * pot.r_cut, 0)
    L = 3.2 * pot.r_cut
    k = int(round(0.5 * L / (0.5 * a)))
    zc = k * 0.5 * a
    i = int(np.argmin(x ** 2 + y ** 2 + (z - zc) ** 2))
    assert x[i] == 0 and y[i] == 0
    # the central atom must be farther than r_cut from every surface
    r_surf = min(1.6 * pot.r_cut, zc, z.max() - zc)
    assert r_surf > pot.r_cut + 0.5
    r = oracle.forces(pot, x, y, z, 1)
    return r["e_atom"][i]


def test_cohesive_energy_closed_form():
    """Table 1 with r0 = 2.884 A: central atom of a large FCC cluster at
    a = 4.08 A equals the 5-shell closed form and the Au cohesive energy the
    parameters were fitted to (about -3.78 eV/atom)."""
    e = center_energy(AU, 4.08)
    ref = fcc_shell_energy(AU, 4.08, FCC5)
    assert abs(e - ref) < 1e-12
    assert abs(e - (-3.7792)) < 1e-3


def test_equilibrium_lattice_constant():
    """The fit reproduces the lattice parameter: dE/da = 0 near a = 4.079 A,
    which is the value Table 1 prints in its r0 column."""
    h = 1e-4
    a_grid = np.linspace(4.070, 4.090, 11)
    dE = [(center_energy(AU, a + h) - center_energy(AU, a - h)) / (2 * h) for a in a_grid]
    dE = np.array(dE)
    assert dE[0] < 0 < dE[-1]
    j = int(np.argmax(dE > 0))
    a_eq = a_grid[j - 1] - dE[j - 1] * (a_grid[j] - a_grid[j - 1]) / (dE[j] - dE[j - 1])
    assert abs(a_eq - 4.079) < 1e-3


def test_r0_as_printed_gives_unbound_crystal():
    """Reading check: with r0 = 4.079 A (the printed column) the crystal has a
    large positive energy, so the printed value cannot be the pair distance."""
    pot = oracle.Pot(r0=4.079)
    assert fcc_shell_energy(pot, 4.08, FCC5) > 10.0


def test_hard_cut_mode():
    """r_tail == r_cut reproduces the paper's hard cut at 5.8 A (4 shells)."""
    pot = oracle.Pot(r_tail=5.8, r_cut=5.8)
    e = center_energy(pot, 4.08)
    assert abs(e - fcc_shell_energy(pot, 4.08, FCC5[:4])) < 1e-12


def test_dimer_closed_form():
    """Two atoms: E = 2 [V(r) - xi exp(-q (r/r0 - 1))] and the force on each
    is dE/dr along the bond (attractive beyond the dimer minimum)."""
    for r in (2.3, 2.884, 3.5, 5.0, 6.0):
        x = np.array([0.0, r])
        y = np.zeros(2)
        z = np.zeros(2)
        out = oracle.forces(AU, x, y, z, 0)
        s = r / AU.r0 - 1
        E = 2 * (AU.A * math.exp(-AU.p * s) - AU.xi * math.exp(-AU.q * s))
        dE = 2 * (-AU.p / AU.r0 * AU.A * math.exp(-AU.p * s)
                  + AU.q / AU.r0 * AU.xi * math.exp(-AU.q * s))
        assert abs(out["E"] - E) < 1e-13
        assert abs(out["fx"][0] - dE) < 1e-12
        assert abs(out["fx"][1] + dE) < 1e-12
    out = oracle.forces(AU, np.array([0.0, AU.r0]), np.zeros(2), np.zeros(2), 0)
    assert abs(out["E"] - 2 * (AU.A - AU.xi)) < 1e-13


def test_linear_trimer_closed_form():
    """Three collinear atoms at 0, a, a+b: closed-form energy."""
    a, b = 2.8, 3.3
    x = np.array([0.0, a, a + b])
    out = oracle.forces(AU, x, np.zeros(3), np.zeros(3), 0)
    phi = lambda r: AU.xi ** 2 * math.exp(-2 * AU.q * (r / AU.r0 - 1))
    V = lambda r: AU.A * math.exp(-AU.p * (r / AU.r0 - 1))
    c = a + b
    E = (-math.sqrt(phi(a) + phi(c)) - math.sqrt(phi(a) + phi(b)) - math.sqrt(phi(b) + phi(c))
         + 2 * (V(a) + V(b) + V(c)))
    assert abs(out["E"] - E) < 1e-12


def random_cluster(n, seed, box=9.0, dmin=2.3):
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        p = rng.uniform(0, box, 3)
        if all(np.linalg.norm(p - q) > dmin for q in pts):
            pts.append(p)
    P = np.array(pts)
    return P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy()


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_forces_are_minus_energy_gradient(seed):
    """Central finite differences of the oracle energy, h = 1e-5 A."""
    x, y, z = random_cluster(30, seed)
    out = oracle.forces(AU, x, y, z, 0)
    # the cluster must exercise the cubic tail
    d = np.sqrt((x[:, None] - x) ** 2 + (y[:, None] - y) ** 2 + (z[:, None] - z) ** 2)
    assert np.any((d > AU.r_tail) & (d < AU.r_cut))
    h = 1e-5
    F = np.stack([out["fx"], out["fy"], out["fz"]], 1)
    fmax = np.abs(F).max()
    for i in range(0, 30, 3):
        for c, arr in enumerate((x, y, z)):
            arr[i] += h
            ep = oracle.forces(AU, x, y, z, 0)["E"]
            arr[i] -= 2 * h
            em = oracle.forces(AU, x, y, z, 0)["E"]
            arr[i] += h
            fd = -(ep - em) / (2 * h)
            assert abs(fd - F[i, c]) < 1e-7 * max(1.0, fmax), (i, c, fd, F[i, c])


from hypothesis import given, settings, strategies as st


@settings(max_examples=40, deadline=None)
@given(n=st.integers(2, 36), seed=st.integers(0, 10 ** 6), k=st.integers(0, 10 ** 6))
def test_force_invariants_on_random_clusters(n, seed, k):
    """For any cluster: the forces sum to zero (Newton's third law), the
    energy does not change under a translation, the cell-list mode equals
    brute force, and one randomly chosen force component equals minus the
    central difference of the energy (h = 1e-5 A)."""
    x, y, z = random_cluster(n, seed, box=9.0 * (n / 30.0) ** (1.0 / 3.0) + 2.0)
    out = oracle.forces(AU, x, y, z, 0)
    F = np.stack([out["fx"], out["fy"], out["fz"]], 1)
    assert np.abs(F.sum(0)).max() <= 1e-12 * np.abs(F).sum() + 1e-14
    t = oracle.forces(AU, x + 31.7, y - 4.2, z + 0.9, 0)
    assert abs(t["E"] - out["E"]) < 1e-11
    c = oracle.forces(AU, x, y, z, 1)
    for key in ("e_atom", "fx", "fy", "fz", "rho"):
        assert np.abs(c[key] - out[key]).max() < 1e-12
    i, comp = k % n, (k // n) % 3
    arr = (x, y, z)[comp]
    h = 1e-5
    arr[i] += h
    ep = oracle.forces(AU, x, y, z, 0)["E"]
    arr[i] -= 2 * h
    em = oracle.forces(AU, x, y, z, 0)["E"]
    arr[i] += h
    assert abs(-(ep - em) / (2 * h) - F[i, comp]) < 1e-7 * max(1.0, np.abs(F).max())


def test_newton_third_law_and_invariance():
    x, y, z = random_cluster(36, 7)
    out = oracle.forces(AU, x, y, z, 0)
    F = np.stack([out["fx"], out["fy"], out["fz"]], 1)
    assert np.abs(F.sum(0)).max() < 1e-12 * np.abs(F).sum()
    # translation
    t = oracle.forces(AU, x + 123.4, y - 7.7, z + 0.3, 0)
    assert abs(t["E"] - out["E"]) < 1e-11
    # rotation: energy invariant, forces rotate
    th = 0.7
    Rm = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    Rm = Rm @ np.array([[1, 0, 0], [0, math.cos(1.1), -math.sin(1.1)], [0, math.sin(1.1), math.cos(1.1)]])
    P = np.stack([x, y, z], 1) @ Rm.T
    r = oracle.forces(AU, P[:, 0], P[:, 1], P[:, 2], 0)
    assert abs(r["E"] - out["E"]) < 1e-11
    Fr = np.stack([r["fx"], r["fy"], r["fz"]], 1)
    assert np.abs(Fr - F @ Rm.T).max() < 1e-11


def test_virial_open_boundary_identity():
    """For a finite cluster with central pair forces, the pair virial
    -sum_{i<j} E' d d / r equals sum_i r_i (x) F_i (W symmetric)."""
    x, y, z = random_cluster(36, 11)
    out = oracle.forces(AU, x, y, z, 0)
    P = np.stack([x, y, z], 1)
    F = np.stack([out["fx"], out["fy"], out["fz"]], 1)
    M = P.T @ F
    W = out["w6"]
    full = np.array([[W[0], W[3], W[4]], [W[3], W[1], W[5]], [W[4], W[5], W[2]]])
    assert np.abs(M - M.T).max() < 1e-10
    assert np.abs(full - M).max() < 1e-10


def test_cubic_tail_conditions():
    """The tail matches value and slope at r_tail and vanishes with zero
    slope at r_cut; beyond r_cut both functions are zero."""
    eps = 1e-9
    for kind in (0, 1):
        f_in, d_in = oracle.radial(AU, kind, AU.r_tail)
        f_out, d_out = oracle.radial(AU, kind, AU.r_tail + eps)
        assert abs(f_in - f_out) < 1e-8 * abs(f_in)
        assert abs(d_in - d_out) < 1e-6 * abs(d_in)
        f_c, d_c = oracle.radial(AU, kind, AU.r_cut)
        assert abs(f_c) < 1e-15 and abs(d_c) < 1e-15
        assert oracle.radial(AU, kind, AU.r_cut + 1e-6) == (0.0, 0.0)
        # inside: the plain exponential of eq 1 / eq 2
        r = 3.1
        f, d = oracle.radial(AU, kind, r)
        pre, k = (AU.xi ** 2, 2 * AU.q) if kind == 0 else (AU.A, AU.p)
        assert abs(f - pre * math.exp(-k * (r / AU.r0 - 1))) < 1e-14
        # derivative by finite differences inside the tail
        r = 6.8
        h = 1e-6
        fd = (oracle.radial(AU, kind, r + h)[0] - oracle.radial(AU, kind, r - h)[0]) / (2 * h)
        assert abs(fd - oracle.radial(AU, kind, r)[1]) < 1e-8


def test_cell_list_mode_equals_brute_force():
    x, y, z, _ = oracle.build_wire(4.08, 20.0, 40.0, 2)
    rng = np.random.default_rng(5)
    x = x + rng.uniform(-0.1, 0.1, x.size)
    a = oracle.forces(AU, x, y, z, 0)
    b = oracle.forces(AU, x, y, z, 1)
    for k in ("e_atom", "fx", "fy", "fz", "rho"):
        assert np.abs(a[k] - b[k]).max() < 1e-12
    s = oracle.forces_sampled(AU, x, y, z, np.array([0, 17, 100, x.size - 1]))
    for k in ("fx", "fy", "fz", "e_atom", "rho"):
        assert np.abs(s[k] - a[k][[0, 17, 100, x.size - 1]]).max() < 1e-12


def test_wire_geometry():
    """[100] FCC cylinder: even-parity sites of the a/2 cubic grid inside the
    radius, nearest-neighbour distance a/sqrt2, (002) spacing a/2, 4-fold
    symmetry, two grip planes per end, and the atom count within 1 % of the
    bulk density 4/a^3 times the cylinder volume for a 10 nm wire."""
    a = 4.08
    x, y, z, f = oracle.build_wire(a, 30.0, 200.0, 2)
    ijk = np.round(np.stack([x, y, z], 1) / (a / 2)).astype(int)
    assert np.all(ijk.sum(1) % 2 == 0)
    assert np.all(x ** 2 + y ** 2 <= 15.0 ** 2 + 1e-9)
    assert z.min() == 0 and z.max() < 200.0
    layers = np.unique(z)
    assert np.allclose(np.diff(layers), a / 2)
    assert set(np.unique(f)) == {0, 1, 2}
    assert np.all(f[z <= layers[1]] == 1) and np.all(f[z >= layers[-2]] == 2)
    assert np.all(f[(z > layers[1]) & (z < layers[-2])] == 0)
    # 4-fold rotation maps the lattice onto itself
    s1 = {(int(i), int(j), int(k)) for i, j, k in ijk}
    s2 = {(-j, i, k) for i, j, k in s1}
    assert s1 == s2
    xb, _, _, _ = oracle.build_wire(a, 100.0, 40.8, 2)
    vol = math.pi * 50.0 ** 2 * 40.8
    assert abs(xb.size / (4 / a ** 3 * vol) - 1) < 0.01
    # nearest-neighbour distance
    P = np.stack([x, y, z], 1)[:300]
    d = np.sqrt(((P[:, None] - P) ** 2).sum(-1)) + np.eye(300) * 100
    assert abs(d.min() - a / math.sqrt(2)) < 1e-12


def read_kat():
    rows = []
    with open(os.path.join(GOLD, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(t, 16) for t in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers():
    for ctr, key, exp in read_kat():
        assert list(oracle.philox4x32_10(ctr, key)) == exp


def _py_philox(ctr, key):
    """Independent pure-Python Philox4x32-10 (integer arithmetic)."""
    c = list(ctr)
    k0, k1 = key
    for rnd in range(10):
        if rnd:
            k0 = (k0 + 0x9E3779B9) & 0xFFFFFFFF
            k1 = (k1 + 0xBB67AE85) & 0xFFFFFFFF
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & 0xFFFFFFFF, p1 & 0xFFFFFFFF,
             ((p0 >> 32) ^ c[3] ^ k1) & 0xFFFFFFFF, p0 & 0xFFFFFFFF]
    return c


def test_philox_random_counters_match_python():
    rng = np.random.default_rng(3)
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2 ** 32, 4)]
        key = [int(v) for v in rng.integers(0, 2 ** 32, 2)]
        assert list(oracle.philox4x32_10(ctr, key)) == _py_philox(ctr, key)


def test_uniform_and_gauss_definition_and_moments():
    seed = 13113890000 + 5
    u = oracle.uniform4(seed, 3, 77, 123456, 0)
    o = _py_philox([77, 123456, 3, 0], [seed & 0xFFFFFFFF, seed >> 32])
    assert np.allclose(u, [(v + 0.5) / 2 ** 32 for v in o], rtol=0, atol=0)
    g = np.array([oracle.gauss3(seed, 3, t, 9, 0) for t in range(20000)])
    assert abs(g.mean()) < 0.02
    assert abs(g.var() - 1) < 0.03
    # Box-Muller of the first pair
    u = oracle.uniform4(seed, 3, 0, 9, 0)
    r = math.sqrt(-2 * math.log(u[0]))
    assert abs(g[0, 0] - r * math.cos(2 * math.pi * u[1])) < 1e-14
    assert abs(g[0, 1] - r * math.sin(2 * math.pi * u[1])) < 1e-14


def small_wire_state(T, jitter=0.0, v_pull=0.5, gamma=1.0, D=15.0, L=30.6, seed=99):
    x, y, z, f = oracle.build_wire(4.08, D, L, 2)
    st = oracle.State(x, y, z, f)
    zlo = z[f == 1].max()
    zhi = z[f == 2].min()
    md = oracle.MD(T=T, v_pull=v_pull, gamma=gamma, z_lo=zlo, z_hi=zhi, seed=seed, rep_id=1)
    oracle.init_state(md, st, jitter)
    oracle.compute_forces(AU, st, 0)
    return st, md


def test_init_state_exact_temperature_and_zero_momentum():
    kb, acc, _ = oracle.constants()
    st, md = small_wire_state(298.0, jitter=0.02, v_pull=0.0)
    dyn = st.flag == 0
    m = oracle.MASS_AU
    assert abs(st.vx[dyn].sum()) < 1e-10 and abs(st.vz[dyn].sum()) < 1e-10
    ke = 0.5 * m * (st.vx[dyn] ** 2 + st.vy[dyn] ** 2 + st.vz[dyn] ** 2).sum() / acc
    T = 2 * ke / ((3 * dyn.sum() - 3) * kb)
    assert abs(T - 298.0) < 1e-9
    x0, _, _, _ = oracle.build_wire(4.08, 15.0, 30.6, 2)
    dx = st.x - x0
    assert 0.015 < np.abs(dx).max() <= 0.02
    assert np.all(st.vz[st.flag == 1] == 0)
    obs = oracle.observe(AU, md, st, 1.0, 30.6)
    assert abs(obs[2] - 298.0) < 1e-9


def test_nve_energy_conservation():
    """gamma = 0 and static grips: velocity Verlet conserves the total energy
    (bounded fluctuation, no secular drift) with the C1 cubic tail."""
    kb, acc, _ = oracle.constants()
    st, md = small_wire_state(50.0, v_pull=0.0, gamma=0.0)
    m = oracle.MASS_AU

    def etot():
        ke = 0.5 * m * (st.vx ** 2 + st.vy ** 2 + st.vz ** 2).sum() / acc
        return st.e_atom.sum() + ke

    e0 = etot()
    es = []
    for _ in range(20):
        oracle.run(AU, md, st, 50, 0)
        es.append(etot())
    es = np.array(es)
    n = st.x.size
    assert np.abs(es - e0).max() / n < 2e-5     # eV/atom
    slope = np.polyfit(np.arange(es.size) * 50 * md.dt, es, 1)[0] / n
    assert abs(slope) < 1e-5                   # eV/atom/ps


def test_velocity_verlet_time_reversible():
    st, md = small_wire_state(30.0, v_pull=0.0, gamma=0.0)
    x0, y0, z0 = st.x.copy(), st.y.copy(), st.z.copy()
    oracle.run(AU, md, st, 100, 0)
    assert np.abs(st.x - x0).max() > 1e-3
    st.vx, st.vy, st.vz = -st.vx, -st.vy, -st.vz
    st.step = 0
    oracle.run(AU, md, st, 100, 0)
    assert max(np.abs(st.x - x0).max(), np.abs(st.y - y0).max(), np.abs(st.z - z0).max()) < 1e-9


def test_free_atom_ballistic_and_grip_motion():
    """An isolated dynamic atom moves ballistically under velocity Verlet;
    grips sit at z0 and z0 + v_pull n dt."""
    x = np.array([0.0, 50.0, 100.0])
    st = oracle.State(x, np.zeros(3), np.zeros(3), np.array([0, 1, 2], np.uint8))
    st.vx[0], st.vy[0], st.vz[0] = 1.5, -0.5, 2.0
    md = oracle.MD(gamma=0.0, v_pull=0.7, z_lo=0, z_hi=0)
    oracle.compute_forces(AU, st, 0)
    oracle.run(AU, md, st, 37, 0)
    t = 37 * md.dt
    assert abs(st.x[0] - 1.5 * t) < 1e-13 and abs(st.z[0] - 2.0 * t) < 1e-13
    assert st.z[1] == 0.0 and abs(st.z[2] - 0.7 * 37 * md.dt) < 1e-15
    assert st.vz[2] == 0.7 and st.vz[1] == 0.0


def test_langevin_equipartition():
    """BAOAB samples the Maxwell-Boltzmann velocities: <T> -> T."""
    st, md = small_wire_state(300.0, v_pull=0.0, gamma=5.0)
    Ts = []
    for _ in range(40):
        oracle.run(AU, md, st, 50, 1)
        Ts.append(oracle.observe(AU, md, st, 1.0, 30.6)[2])
    Ts = np.array(Ts[10:])
    assert abs(Ts.mean() - 300.0) < 12.0


def test_observe_gap_and_stress_sign():
    """A wire cut in two by a gap reports that gap; a wire stretched
    affinely along z is in tension (positive sigma_zz)."""
    x, y, z, f = oracle.build_wire(4.08, 15.0, 40.8, 2)
    z2 = np.where(z > 20.0, z + 9.0, z)
    st = oracle.State(x, y, z2, f)
    md = oracle.MD(v_pull=0.0)
    obs = oracle.observe(AU, md, st, 1000.0, 40.8)
    assert abs(obs[6] - (9.0 + 2.04)) < 1e-12
    st2 = oracle.State(x * 0.99, y * 0.99, z * 1.02, f)
    obs2 = oracle.observe(AU, md, st2, 1000.0, 40.8)
    assert obs2[4] > 0
    st3 = oracle.State(x, y, z * 0.98, f)
    assert oracle.observe(AU, md, st3, 1000.0, 40.8)[4] < obs2[4]


# --- the streaming profile, eq 5's kinetic term and the pair counter ---------
# SI values (CODATA 2018, exact since the 2019 SI) written here independently
# of the oracle: one amu A^2/ps^2 in eV, one eV/A^3 in GPa, k_B in eV/K.
AMU_A2_PS2_EV = 1.66053906660e-27 * 1e-20 / 1e-24 / 1.602176634e-19
EVA3_GPA = 1.602176634e-19 / 1e-30 / 1e9
KB_EV = 1.380649e-23 / 1.602176634e-19


def _free_atoms():
    """Atoms that never interact: two columns of dynamic atoms along z (10 A
    apart within a column, the columns 12 A apart in x and staggered by 5 A),
    a bottom grip atom under each column at z = 0 and a top grip atom over
    each at z = 100; no two atoms are within r_cut, and a stretch along z only
    separates them further."""
    za = np.arange(10.0, 91.0, 10.0)
    zb = np.arange(15.0, 86.0, 10.0)
    x = np.concatenate([[0.0, 12.0], np.zeros(za.size), np.full(zb.size, 12.0), [0.0, 12.0]])
    z = np.concatenate([[0.0, 0.0], za, zb, [100.0, 100.0]])
    f = np.concatenate([[1, 1], np.zeros(za.size + zb.size), [2, 2]]).astype(np.uint8)
    return oracle.State(x, np.zeros(x.size), z, f)


def test_free_atoms_stay_on_the_affine_stretch_profile():
    """Reading 8: the Langevin O step acts on the velocity relative to the
    affine stretch u(z) = v_pull (z - z_lo) / (z_hi - z_lo + D), D the pulled
    grip's travel.  Free atoms started on that profile at T = 0 move
    ballistically while the grip is pulled and stay exactly on it, since
    z - z_lo grows in proportion to z_hi - z_lo + D.  So the O step must leave
    their velocities unchanged (a profile that missed the + D, or took D at
    another time than the positions, would pull them off it), and their
    peculiar kinetic energy and temperature are zero at every step."""
    st = _free_atoms()
    md = oracle.MD(T=0.0, gamma=5.0, v_pull=0.5, z_lo=0.0, z_hi=100.0, seed=7, rep_id=2)
    oracle.init_state(md, st, 0.0)
    dyn = st.flag == 0
    # at t = 0 the dynamic atoms move with the profile, the pulled grip at v_pull
    assert np.array_equal(st.vz[dyn], 0.5 * st.z[dyn] / 100.0)
    assert np.all(st.vz[st.flag == 2] == 0.5) and np.all(st.vz[st.flag == 1] == 0.0)
    assert np.all(st.vx == 0.0) and np.all(st.vy == 0.0)
    oracle.compute_forces(AU, st, 0)
    assert np.abs(np.stack([st.fx, st.fy, st.fz])).max() == 0.0
    v0, z_init = st.vz.copy(), st.z.copy()
    for _ in range(5):
        oracle.run(AU, md, st, 400, 0)
        t = st.step * md.dt
        assert np.abs(st.vz[dyn] - v0[dyn]).max() <= 1e-11 * v0.max()
        assert np.abs(st.z[dyn] - (z_init[dyn] + v0[dyn] * t)).max() < 1e-10
        assert np.all(st.vx == 0.0) and np.all(st.vy == 0.0)
        ob = oracle.observe(AU, md, st, 1.0, 100.0)
        assert ob[1] < 1e-26 and ob[2] < 1e-20, ob   # peculiar KE (eV) and T (K)
        assert abs(ob[7] - 0.5 * t) < 1e-12 and abs(ob[5] - 0.5 * t / 100.0) < 1e-14
    # the top grip moved rigidly at v_pull, the bottom one rested
    assert abs(st.z[-1] - (100.0 + 0.5 * st.step * md.dt)) < 1e-12 and st.z[0] == 0.0


def test_stress_of_an_ideal_gas_is_its_kinetic_term():
    """Eq 5 for atoms that do not interact: the virial term vanishes and
    sigma_zz is the kinetic term alone, -sum_i m v_z,i^2 / V over the dynamic
    atoms (reading 12: the printed m v_x,i v_x,j is m v_z,i^2; reading 13: V
    is the volume passed in).  Transverse velocities enter the kinetic energy
    and the temperature (3 N_dyn - 3 degrees of freedom), not sigma_zz; grip
    velocities enter none of them."""
    st = _free_atoms()
    rng = np.random.default_rng(5)
    st.vx, st.vy, st.vz = (rng.normal(size=st.x.size) * 3.0 for _ in range(3))
    md = oracle.MD(v_pull=0.0, z_lo=0.0, z_hi=100.0)   # at rest: u = 0
    vol = 1234.5
    ob = oracle.observe(AU, md, st, vol, 100.0)
    dyn = st.flag == 0
    m = oracle.MASS_AU
    kz = m * (st.vz[dyn] ** 2).sum() * AMU_A2_PS2_EV
    ke = 0.5 * m * (st.vx[dyn] ** 2 + st.vy[dyn] ** 2 + st.vz[dyn] ** 2).sum() * AMU_A2_PS2_EV
    assert ob[3] == 0.0                                            # -W_zz
    assert abs(ob[4] - (-kz / vol * EVA3_GPA)) <= 1e-12 * abs(ob[4])
    assert abs(ob[1] - ke) <= 1e-12 * ke
    assert abs(ob[2] - 2.0 * ke / ((3 * dyn.sum() - 3) * KB_EV)) <= 1e-9 * ob[2]
    # the lab frame and a pulled grip change nothing when u is the lab velocity
    md2 = oracle.MD(v_pull=0.5, z_lo=0.0, z_hi=100.0, lab_frame=1)
    assert np.array_equal(oracle.observe(AU, md2, st, vol, 100.0)[[1, 2, 3, 4]], ob[[1, 2, 3, 4]])


def test_pair_counter_equals_brute_force_at_the_radius():
    """The pair counter that checks the neighbour lists (count_pairs) equals
    an independent numpy brute force on a jittered wire, and counts strictly
    inside the radius: of two isolated pairs placed 1e-9 A inside and 1e-9 A
    outside it, only the first counts, for both of its atoms."""
    x, y, z, _ = oracle.build_wire(4.08, 20.0, 30.6, 2)
    rng = np.random.default_rng(11)
    P = np.stack([x, y, z], 1) + rng.uniform(-0.3, 0.3, (x.size, 3))
    rc = 8.0
    for k, d in enumerate((rc - 1e-9, rc + 1e-9)):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        c = np.array([200.0 + 50.0 * k, 0.0, 0.0])
        P = np.vstack([P, c, c + d * u])
    cnt = oracle.count_pairs(P[:, 0], P[:, 1], P[:, 2], rc)
    d2 = ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.inf)
    ref = (d2 < rc * rc).sum(1)
    assert np.array_equal(cnt, ref)
    assert list(cnt[-4:]) == [1, 1, 0, 0]
    assert ref[:-4].min() > 20


# --- the paper's protocol: Nose-Hoover thermostat, stepwise grips, notch ----
def _nh_extended_energy(st, md, kb, acc):
    dyn = st.flag == 0
    g = 3 * int(dyn.sum()) - 3
    m = oracle.MASS_AU
    ke = 0.5 * m * (st.vx[dyn] ** 2 + st.vy[dyn] ** 2 + st.vz[dyn] ** 2).sum() / acc
    gkT = g * kb * md.T
    Q = gkT * md.nh_tau ** 2
    return st.e_atom.sum() + ke + 0.5 * Q * st.zeta[0] ** 2 + gkT * st.eta[0], ke, g


def test_nose_hoover_conserves_its_extended_energy():
    """With resting grips, E_pot + K + Q zeta^2/2 + g kB T eta is a constant
    of the Nose-Hoover equations; a wire started at twice the target
    temperature is driven towards it while that sum stays put."""
    kb, acc, _ = oracle.constants()
    st, md = small_wire_state(600.0, v_pull=0.0, gamma=0.0)
    md.T, md.nh_tau = 300.0, 0.1
    h0, _, g = _nh_extended_energy(st, md, kb, acc)
    hs, Ts = [], []
    for _ in range(30):
        oracle.run(AU, md, st, 50, 1)
        h, ke, _ = _nh_extended_energy(st, md, kb, acc)
        hs.append(h)
        Ts.append(2 * ke / (g * kb))
    n = st.x.size
    hs = np.array(hs)
    assert np.abs(hs - h0).max() / n < 2e-5          # eV/atom
    assert abs(np.polyfit(np.arange(hs.size), hs, 1)[0]) / n < 2e-7
    assert abs(st.zeta[0]) > 0 and st.eta[0] != 0
    # the kinetic temperature leaves 600 K and ends near the 300 K target
    assert abs(np.mean(Ts[15:]) - 300.0) < 40.0


def test_nose_hoover_free_gas_converges_to_its_ode():
    """Non-interacting atoms (spacing > r_cut): all velocities share one
    scale, so K and zeta follow dK/dt = -2 zeta K, dzeta/dt =
    (2K/(g kB T) - 1)/tau^2, solved here by scipy.  The splitting must
    converge to that solution at second order in dt."""
    from scipy.integrate import solve_ivp
    kb, acc, _ = oracle.constants()
    g1 = np.arange(3) * 20.0
    X, Y, Z = np.meshgrid(g1, g1, g1, indexing="ij")
    x, y, z = X.ravel(), Y.ravel(), Z.ravel()
    f = np.zeros(x.size, np.uint8)
    rng = np.random.default_rng(5)
    v0 = rng.normal(size=(x.size, 3)) * 3.0
    m = oracle.MASS_AU
    n_dof = 3 * x.size - 3
    T, tau, t_end = 200.0, 0.2, 0.8
    K0 = 0.5 * m * (v0 ** 2).sum() / acc
    gkT = n_dof * kb * T

    def rhs(_, s):
        K, zeta = s
        return [-2.0 * zeta * K, (2.0 * K / gkT - 1.0) / tau ** 2]

    ref = solve_ivp(rhs, (0.0, t_end), [K0, 0.0], rtol=1e-12, atol=1e-14).y[:, -1]
    errs = []
    for dt in (0.004, 0.002):
        st = oracle.State(x, y, z, f)
        st.vx, st.vy, st.vz = (v0[:, k].copy() for k in range(3))
        oracle.compute_forces(AU, st, 0)
        assert np.abs(st.fx).max() == 0.0
        md = oracle.MD(dt=dt, gamma=0.0, T=T, v_pull=0.0, nh_tau=tau)
        oracle.run(AU, md, st, int(round(t_end / dt)), 0)
        K = 0.5 * m * (st.vx ** 2 + st.vy ** 2 + st.vz ** 2).sum() / acc
        errs.append((abs(K / ref[0] - 1.0), abs(st.zeta[0] - ref[1])))
    assert errs[1][0] < 2e-4 and errs[1][1] < 2e-3
    for k in range(2):
        assert 3.0 < errs[0][k] / errs[1][k] < 5.0   # second order


def test_nose_hoover_with_infinite_mass_is_velocity_verlet():
    st, md = small_wire_state(300.0, v_pull=0.0, gamma=0.0)
    st2 = st.copy()
    md2 = oracle.MD(**{**md.__dict__, "nh_tau": 1e12})
    oracle.run(AU, md, st, 40, 0)
    oracle.run(AU, md2, st2, 40, 0)
    assert np.abs(st.vx - st2.vx).max() < 1e-12 and np.abs(st.z - st2.z).max() < 1e-12


def test_stepwise_symmetric_grips():
    """Each hold begins with both grips moving grip_step outwards; they rest
    in between, and the elongation D of eq 4 is the sum of both moves."""
    x = np.array([0.0, 50.0, 100.0])
    st = oracle.State(x, np.zeros(3), np.array([0.0, 10.0, 20.0]),
                      np.array([0, 1, 2], np.uint8))
    md = oracle.MD(gamma=0.0, v_pull=0.7, z_lo=10.0, z_hi=20.0, grip_step=0.05, grip_hold=25)
    oracle.compute_forces(AU, st, 0)
    for n_done, moves in ((1, 1), (25, 1), (26, 2), (75, 3), (76, 4)):
        oracle.run(AU, md, st, n_done - st.step, 0)
        assert st.z[1] == 10.0 - 0.05 * moves and st.z[2] == 20.0 + 0.05 * moves
        assert st.vz[1] == 0.0 and st.vz[2] == 0.0
        obs = oracle.observe(AU, md, st, 1.0, 10.0)
        assert abs(obs[7] - 0.1 * moves) < 1e-15 and abs(obs[5] - 0.01 * moves) < 1e-15


def test_ring_notch_geometry():
    """The notch of Figure 1: three middle (002) planes lose exactly the sites
    farther than D/2 - depth from the axis; nothing else changes."""
    a, D, L = 4.08, 31.0, 204.0
    x, y, z, f = oracle.build_wire(a, D, L, 2)
    xn, yn, zn, fn = oracle.build_wire(a, D, L, 2, notch_layers=3, notch_depth=a)
    key = lambda X, Y, Z: set(zip(np.round(X / (a / 2)).astype(int),
                                  np.round(Y / (a / 2)).astype(int),
                                  np.round(Z / (a / 2)).astype(int)))
    full, notched = key(x, y, z), key(xn, yn, zn)
    assert notched < full
    planes = np.unique(np.round(z / (a / 2)).astype(int))
    mid = planes.size // 2
    ks = set(planes[mid - 1:mid + 2].tolist())
    rin = D / 2 - a
    want = {(i, j, k) for i, j, k in full
            if k in ks and math.hypot(i * a / 2, j * a / 2) > rin}
    assert full - notched == want and len(want) > 0
    # every removed plane keeps its core; the notch sits mid-wire
    for k in ks:
        assert any(kk == k for _, _, kk in notched)
    zc = np.mean([k * a / 2 for k in ks])
    assert abs(zc - 0.5 * z.max()) <= a / 2
    assert np.array_equal(np.unique(fn), [0, 1, 2])


def test_temperature_ramp_target_and_tracking():
    """Equilibration ramp: the target rises linearly from T_start to T over
    the ramp and is constant outside it; initial velocities are drawn at the
    target of step 0; a Nose-Hoover wire follows the ramp."""
    kb, acc, _ = oracle.constants()
    md = oracle.MD(T=300.0, T_start=20.0, ramp_begin=100, ramp_steps=400)
    for t, want in ((0, 20.0), (100, 20.0), (300, 160.0), (500, 300.0), (900, 300.0),
                    (100.5, 20.0 + 280.0 * 0.5 / 400)):
        assert abs(oracle.target_temperature(md, t) - want) < 1e-12
    assert oracle.target_temperature(oracle.MD(T=77.0), 12345) == 77.0
    x, y, z, f = oracle.build_wire(4.08, 15.0, 30.6, 2)
    st = oracle.State(x, y, z, f)
    md = oracle.MD(T=300.0, T_start=50.0, ramp_begin=0, ramp_steps=1500, gamma=0.0,
                   nh_tau=0.1, v_pull=0.0, z_lo=z[f == 1].max(), z_hi=z[f == 2].min(),
                   seed=7, rep_id=3)
    oracle.init_state(md, st, 0.0)
    dyn = st.flag == 0
    g = 3 * int(dyn.sum()) - 3
    m = oracle.MASS_AU

    def temp():
        ke = 0.5 * m * (st.vx[dyn] ** 2 + st.vy[dyn] ** 2 + st.vz[dyn] ** 2).sum() / acc
        return 2 * ke / (g * kb)

    assert abs(temp() - 50.0) < 1e-9
    oracle.compute_forces(AU, st, 1)
    Ts = []
    for _ in range(40):
        oracle.run(AU, md, st, 50, 1)
        Ts.append(temp())
    # the second half of the ramp averages near its mean target (~240 K),
    # the hold after it near 300 K
    assert abs(np.mean(Ts[15:30]) - 238.0) < 45.0
    assert abs(np.mean(Ts[32:]) - 300.0) < 45.0


# --- equilibration barostat: the grip separation as an extended coordinate --
def _piston_wire(T, **md_kw):
    x, y, z, f = oracle.build_wire(4.08, 15.0, 30.6, 2)
    st = oracle.State(x, y, z, f)
    md = oracle.MD(T=T, v_pull=0.0, z_lo=z[f == 1].max(), z_hi=z[f == 2].min(), seed=11,
                   rep_id=2, **md_kw)
    oracle.init_state(md, st, 0.0)
    oracle.compute_forces(AU, st, 1)
    return st, md


def test_barostat_force_is_minus_the_energy_slope():
    """The barostat's generalized force Q = sum_top F_z - sum_bottom F_z is
    -dE/ds for both grips moved outwards by s (central differences)."""
    x, y, z, f = oracle.build_wire(4.08, 15.0, 30.6, 2)
    z = z + np.random.default_rng(1).normal(scale=0.05, size=z.size)
    r = oracle.forces(AU, x, y, z, 0)
    q = r["fz"][f == 2].sum() - r["fz"][f == 1].sum()
    h = 1e-5
    e = lambda s: oracle.forces(AU, x, y, np.where(f == 2, z + s, np.where(f == 1, z - s, z)),
                                0)["E"]
    assert abs((e(-h) - e(h)) / (2 * h) - q) < 1e-6 * max(1.0, abs(q))


def test_barostat_conserves_energy_with_the_piston():
    """Without thermostat, E_pot + K + W (ds/dt)^2/2 stays constant while the
    free grips move (the freshly cut wire is not at zero axial stress)."""
    kb, acc, _ = oracle.constants()
    W = 3000.0
    st, md = _piston_wire(50.0, gamma=0.0, baro_mass=W)
    m = oracle.MASS_AU

    def h():
        ke = 0.5 * m * (st.vx ** 2 + st.vy ** 2 + st.vz ** 2).sum() / acc
        return st.e_atom.sum() + ke + 0.5 * W * st.piston[1] ** 2 / acc

    h0 = h()
    hs, ss = [], []
    for _ in range(30):
        oracle.run(AU, md, st, 50, 1)
        hs.append(h())
        ss.append(st.piston[0])
    n = st.x.size
    assert np.ptp(ss) > 0.02
    assert np.abs(np.array(hs) - h0).max() / n < 2e-5
    f = st.flag
    z0 = st.z0
    assert np.allclose(st.z[f == 2], z0[f == 2] + st.piston[0], atol=1e-12)
    assert np.allclose(st.z[f == 1], z0[f == 1] - st.piston[0], atol=1e-12)
    obs = oracle.observe(AU, md, st, 1.0, 30.6)
    assert abs(obs[7] - 2 * st.piston[0]) < 1e-15


def test_barostat_settles_at_the_load():
    """A damped piston on a cold Nose-Hoover wire settles where the grips'
    net force balances the load (Q = -2 F_load): the mean Q at rest is a
    small fraction of the cut wire's initial Q, and an outward load leaves
    the wire longer."""
    runs = {}
    for load in (0.0, 1.0):
        st, md = _piston_wire(5.0, gamma=0.0, nh_tau=0.05, baro_mass=500.0, baro_load=load,
                              baro_damp=5.0)
        q = lambda: st.fz[st.flag == 2].sum() - st.fz[st.flag == 1].sum()
        q0 = q()
        qs, ss = [], []
        for k in range(60):
            oracle.run(AU, md, st, 50, 1)
            if k >= 40:
                qs.append(q())
                ss.append(st.piston[0])
        runs[load] = (q0, np.mean(qs), np.mean(ss))
    for load, (q0, qm, _) in runs.items():
        assert abs(qm + 2 * load) < 0.1 * abs(q0), (load, q0, qm)
    assert runs[1.0][2] > runs[0.0][2] + 0.01


def test_philox_matches_rocrand():
    """The oracle's Philox4x32-10 words equal those of rocRAND's own
    header-only generator (compiled here, run on the host) for the counters
    (tag, lo32(step), rep_id, stream) the method uses."""
    import ctypes as C
    lib_path = os.path.join(os.path.dirname(__file__), "rocrand_ref", "librocrand_ref.so")
    if not os.path.exists(lib_path):
        pytest.skip("the rocRAND reference is compiled by __graft_entry__.build()")
    rr = C.CDLL(lib_path)
    rng = np.random.default_rng(7)
    for _ in range(20):
        seed = int(rng.integers(0, 2 ** 63))
        rep, stream = int(rng.integers(0, 2 ** 32)), int(rng.integers(0, 3))
        step = int(rng.integers(0, 2 ** 40))
        n = 16
        out = np.zeros(4 * n, np.uint32)
        rr.rocrand_philox_words(C.c_uint64(seed), C.c_uint32(rep), C.c_uint64(step),
                                C.c_uint32(stream), C.c_int64(n),
                                out.ctypes.data_as(C.c_void_p))
        for t in range(n):
            w = oracle.philox4x32_10([t, step & 0xffffffff, rep, stream],
                                     [seed & 0xffffffff, seed >> 32])
            assert list(w) == list(out[4 * t:4 * t + 4]), (seed, rep, step, stream, t)
