"""GPU parity of libtbsma against the FP64 oracle (run on an MI355X).

Every comparison feeds the oracle the same seeded inputs, or the positions the
GPU reached, and compares element by element:
  * random numbers: Philox words bit-exact, Box-Muller normals to 1e-14;
  * Verlet lists: exact set equality with brute force (r < r_cut + skin);
  * forces: FP64 mode eps_F <= 1e-12, mixed mode eps_F <= 1e-5, where
    eps_F = max_i |F_i - F_i^ref| / max_i |F_i^ref|; energies alike;
  * dynamics: FP64 lockstep with the oracle integrator; batched == alone and
    graph == eager bit for bit.
"""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_1311_3890_amd import _abi as A
from paper_1311_3890_amd.engine import WireBatch

pytestmark = pytest.mark.gpu
AU = oracle.Pot()


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def eps_F(F, Fr):
    F, Fr = np.asarray(F), np.asarray(Fr)
    return np.sqrt(((F - Fr) ** 2).sum(1)).max() / np.sqrt((Fr ** 2).sum(1)).max()


def stackF(t):
    return np.stack(t, 1)


def orc_state(b: WireBatch, r: int):
    x, y, z = b.positions(r)
    st = oracle.State(x, y, z, b.flags(r))
    st.vx, st.vy, st.vz = b.velocities(r)
    o = int(b.rep_off[r])
    n = int(b.n_atoms[r])
    st.z0 = b._slice("z0", r).copy()
    st.step = b.step_index()
    st.zeta[0] = float(b.t["nh_xi"][r])
    st.eta[0] = float(b.t["nh_eta"][r])
    st.piston[:] = b.t["baro_s"][2 * r:2 * r + 2].cpu().numpy()
    return st


def orc_md(b: WireBatch, r: int):
    rp = b.replicas[r]
    return oracle.MD(dt=b.dt, gamma=b.gamma, T=rp.T, v_pull=rp.v_pull, z_lo=b.z_lo[r],
                     z_hi=b.z_hi[r], seed=rp.seed, rep_id=rp.rep_id, lab_frame=b.lab_frame,
                     nh_tau=b.nh_tau, grip_step=b.grip_step, grip_hold=b.grip_hold,
                     T_start=float(b.t["T_start"][r]), ramp_begin=b.ramp_begin,
                     ramp_steps=b.ramp_steps, baro_mass=b.baro_mass, baro_load=b.baro_load,
                     baro_damp=b.baro_damp)


# the paper's protocol: Nose-Hoover, stepwise symmetric grips (short holds so
# that tests see several moves), ring notch three planes wide, a deep
PROTOCOL = dict(gamma=0.0, nh_tau=0.1, grip_step=0.05, grip_hold=20, notch=(3, 4.08))
# its equilibration: Nose-Hoover with a temperature ramp and the axial
# barostat on the grip separation (a light, damped piston so that tests see
# it move)
EQUIL = dict(gamma=0.0, nh_tau=0.1, notch=(3, 4.08), T_start=50.0, ramp_begin=0,
             ramp_steps=60, baro_mass=300.0, baro_load=0.0, baro_damp=2.0)


def R(D, L, T=10.0, v=0.5, r=0, jitter=0.0):
    return W.Replica(D, W.snap_length(L), T, v, W.seed_of(r), r, jitter=jitter)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "these tests need the GPU"
    torch.cuda.set_device(0)
    yield


def test_rng_words_and_normals():
    n = 2048
    for seed, rep, step, strm in [(0, 0, 0, 0), (W.seed_of(7), 7, 123456789, 0),
                                  (2 ** 64 - 1, 2 ** 32 - 1, 2 ** 40 + 5, 2)]:
        note(f"rng seed={seed} rep={rep} step={step} stream={strm}")
        w = torch.zeros(4 * n, dtype=torch.int32, device="cuda")
        g = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
        A.check(A.lib().tbsma_rng_fill(seed, rep, step, strm, n, C.c_void_p(w.data_ptr()),
                                       C.c_void_p(g.data_ptr()), None))
        torch.cuda.synchronize()
        wh = w.cpu().numpy().view(np.uint32).reshape(n, 4)
        gh = g.cpu().numpy().reshape(n, 3)
        key = [seed & 0xFFFFFFFF, seed >> 32]
        for t in range(0, n, 7):
            ref = oracle.philox4x32_10([t, step & 0xFFFFFFFF, rep, strm], key)
            assert np.array_equal(wh[t], ref), t
            assert np.abs(gh[t] - oracle.gauss3(seed, rep, t, step, strm)).max() < 1e-14


def test_fp32_normals_match_the_fp64_normals():
    """The normals of the mixed-precision Langevin O step are the FP64
    Box-Muller normals of the same Philox words within a few FP32 ulp:
    |n32 - n64| <= 2^-20 (1 + a), a = sqrt(-2 ln u) the Box-Muller radius of
    the normal.  (FP32 uniforms of relative precision 2^-24, the log-near-1
    correction and sin/cos of pi x give a relative error of about 3e-7 on a
    and an absolute one of about 3e-7 on the sine and cosine.)  Checked on
    all 2^24 counters of one step against the GPU's FP64 normals, and on
    every counter whose words sit within 2^-20 of 0, 1/2 or 1 against the
    oracle."""
    n = 1 << 24
    seed, rep, step, strm = W.seed_of(3), 3, 987654321, 0
    note(f"fp32 normals, {n} counters")
    w = torch.empty(4 * n, dtype=torch.int32, device="cuda")
    g64 = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    g32 = torch.empty(3 * n, dtype=torch.float32, device="cuda")
    lib = A.lib()
    A.check(lib.tbsma_rng_fill(seed, rep, step, strm, n, C.c_void_p(w.data_ptr()),
                               C.c_void_p(g64.data_ptr()), None))
    A.check(lib.tbsma_rng_normals_f32(seed, rep, step, strm, n, C.c_void_p(g32.data_ptr()),
                                      None))
    torch.cuda.synchronize()
    wu = w.view(n, 4).to(torch.int64) & 0xFFFFFFFF
    u = (wu.double() + 0.5) * 2.0 ** -32
    rad = torch.sqrt(-2.0 * torch.log(u))  # radius of (u0) and of (u2)
    tol = 2.0 ** -20 * (1.0 + torch.stack([rad[:, 0], rad[:, 0], rad[:, 2]], 1))
    err = (g32.view(n, 3).double() - g64.view(n, 3)).abs()
    note(f"  max |n32 - n64| = {err.max().item():.2e}, max err/tol = "
         f"{(err / tol).max().item():.3f}")
    assert bool((err <= tol).all())
    # words at the ends of (0, 1) and at 1/2, where the uniforms round most
    edge = 1 << 12
    near = ((wu < edge) | (wu >= (1 << 32) - edge) | ((wu - (1 << 31)).abs() < edge)).any(1)
    tags = torch.nonzero(near).flatten().cpu().numpy()
    assert tags.size >= 50, tags.size
    g32h = g32.view(n, 3).double().cpu().numpy()
    tolh = tol.cpu().numpy()
    for t in tags:
        ref = oracle.gauss3(seed, rep, int(t), step, strm)
        assert np.all(np.abs(g32h[t] - ref) <= tolh[t]), (t, g32h[t], ref)


def brute_sets(x, y, z, rl):
    P = np.stack([x, y, z], 1)
    out = []
    for i in range(P.shape[0]):
        d2 = ((P - P[i]) ** 2).sum(1)
        d2[i] = np.inf
        out.append(np.nonzero(d2 < rl * rl)[0])
    return out


@pytest.mark.parametrize("precision,cell", [("fp64", None), ("mixed", None), ("fp64", 12.0),
                                            ("mixed", 12.0)])
def test_neighbor_lists_are_exact_sets(precision, cell):
    # the 4.4 nm wire's z-slabs hold more candidates than LDS stages, so its
    # mixed-precision lists come from the cell walk; 12 A cells hold about
    # 100 atoms inside the wires, more than the 64 the cell sort ranks in
    # registers (larger cells take its insertion sort)
    reps = [R(15.0, 30.0, r=0, jitter=0.1), R(20.0, 20.0, T=298.0, r=1, jitter=0.1),
            R(30.0, 40.0, r=2, jitter=0.1), R(44.0, 30.0, r=3, jitter=0.1)]
    note(f"nlist sets {precision} cell={cell} R={len(reps)}")
    b = WireBatch(reps, precision, cell=cell)
    b.prepare()
    torch.cuda.synchronize()
    cs = b.t["cell_start"].cpu().numpy()
    if cell is not None:
        assert np.diff(cs).max() > 64
    rl = b.pot.r_cut + b.skin
    # FP64 lists are exact; mixed ones compare quantised positions, so pairs
    # within 1e-5 A of r_cut + skin may fall on either side
    tol = 0.0 if precision == "fp64" else 1e-5
    for r in range(b.R):
        x, y, z = b.positions(r)
        sure = brute_sets(x, y, z, rl - tol)
        loose = brute_sets(x, y, z, rl + tol)
        got = b.neighbor_rows(r)
        for i in range(len(sure)):
            g = set(got[i].tolist())
            assert len(g) == got[i].size
            assert set(sure[i].tolist()) <= g <= set(loose[i].tolist()), (r, i)
    if precision == "mixed":
        # per-atom counts of pairs within r_tail and within (r_tail, r_cut]
        # from the density pass (pairs within 1e-4 A of a boundary may fall
        # on either side in FP32)
        rt, rc = b.pot.r_tail, b.pot.r_cut
        for r in range(b.R):
            x, y, z = b.positions(r)
            P = np.stack([x, y, z], 1)
            cnt = b.active_counts(r)
            for i in range(P.shape[0]):
                d = np.sqrt(((P - P[i]) ** 2).sum(1))
                d[i] = np.inf
                edge_t = int(np.count_nonzero(np.abs(d - rt) < 1e-4))
                edge_c = int(np.count_nonzero(np.abs(d - rc) < 1e-4))
                assert abs(cnt[i, 0] - np.count_nonzero(d <= rt)) <= edge_t, (r, i)
                assert abs(cnt[i].sum() - np.count_nonzero(d <= rc)) <= edge_c, (r, i)
    if cell is not None:
        # every cell's slots in ascending order, and every real atom binned once
        ca = b.t["cell_atoms"].cpu().numpy()
        for r in range(b.R):
            st = cs[int(b.cell_off[r]) + r:int(b.cell_off[r + 1]) + r + 1]
            for c in range(st.size - 1):
                assert np.all(np.diff(ca[st[c]:st[c + 1]]) > 0), (r, c)
            o = int(b.rep_off[r])
            assert np.array_equal(np.sort(ca[st[0]:st[-1]]), o + np.arange(int(b.n_atoms[r])))
        forces = stackF(b.forces(2))
        x, y, z = b.positions(2)
        ref = oracle.forces(AU, x, y, z, 0)
        assert eps_F(forces, stackF((ref["fx"], ref["fy"], ref["fz"]))) <= (
            1e-12 if precision == "fp64" else 1e-5)
    # rows are stored in ascending cell-scan order: check determinism
    b2 = WireBatch(reps, precision, cell=cell)
    b2.prepare()
    torch.cuda.synchronize()
    assert torch.equal(b.t["nl"], b2.t["nl"]) and torch.equal(b.t["nn"], b2.t["nn"])


def _tile_box_counts(b, r, rl):
    """Atoms of replica r within rl of the box of each tile's positions (the
    candidates the list build stages for a tile whose slabs exceed LDS)."""
    from scipy.spatial import cKDTree
    x, y, z = (b._slice(k, r) for k in ("x", "y", "z"))
    tag = b.slot_tag[r]
    P = np.stack([x, y, z], 1)
    Ps = P if tag is None else P[tag]  # slot order
    tree = cKDTree(P)
    out = []
    for t0 in range(0, Ps.shape[0], 64):
        T = Ps[t0:t0 + 64]
        lo, hi = T.min(0), T.max(0)
        c = 0.5 * (lo + hi)
        cand = tree.query_ball_point(c, np.linalg.norm(0.5 * (hi - lo)) + rl)
        d = np.maximum(np.maximum(lo - P[cand], P[cand] - hi), 0.0)
        out.append(int(np.count_nonzero((d ** 2).sum(1) < rl * rl)))
    return np.array(out)


@pytest.mark.parametrize("order", ["blocked", "axial"])
def test_thick_wire_lists_from_the_box_scan_and_the_cell_walk(order):
    """Lists of wires whose z-slabs exceed LDS.  A tile whose box (its
    atoms' extent, widened by the list radius) holds at most 2560 atoms
    stages them in LDS (box scan); others walk the 27 cells around each atom.
    In the blocked order tiles are compact and all of a 5 nm wire's take the
    box scan; in the axial order a tile of a 7 nm wire is a strip across the
    wire and about one in eight takes the cell walk.  Either way the lists
    equal brute force."""
    from scipy.spatial import cKDTree
    D = 50.0 if order == "blocked" else 70.0
    rp = R(D, 120.0, T=298.0, r=7, jitter=0.1)
    note(f"thick-wire lists, {order} order, D {D / 10:.0f} nm")
    b = WireBatch([rp], "mixed", order=order)
    b.prepare()
    torch.cuda.synchronize()
    rl = b.pot.r_cut + b.skin
    counts = _tile_box_counts(b, 0, rl)
    # the blocked tiles take the box scan; the axial ones both paths
    fit = np.mean(counts <= 2560)
    note(f"  tiles whose box candidates fit in LDS: {fit:.2f}")
    if order == "blocked":
        assert fit > 0.9
    else:
        assert 0.0 < fit < 0.9
    x, y, z = b.positions(0)
    P = np.stack([x, y, z], 1)
    tree = cKDTree(P)
    got = b.neighbor_rows(0)
    for i in range(P.shape[0]):
        sure = set(tree.query_ball_point(P[i], rl - 1e-5)) - {i}
        loose = set(tree.query_ball_point(P[i], rl + 1e-5)) - {i}
        g = set(got[i].tolist())
        assert len(g) == got[i].size and sure <= g <= loose, i
    ref = oracle.forces(AU, x, y, z, 1)
    assert eps_F(stackF(b.forces(0)), stackF((ref["fx"], ref["fy"], ref["fz"]))) <= 1e-5


def _check_lists(b, r):
    rl = b.pot.r_cut + b.skin
    rt, rc = b.pot.r_tail, b.pot.r_cut
    # the Verlet lists are exact at the positions of their last build
    xr, yr, zr = (b._slice(k, r).astype(np.float64) for k in ("x_ref", "y_ref", "z_ref"))
    sure = brute_sets(xr, yr, zr, rl - 1e-5)
    loose = brute_sets(xr, yr, zr, rl + 1e-5)
    got = b.neighbor_rows(r)
    for i in range(len(sure)):
        g = set(got[i].tolist())
        assert len(g) == got[i].size
        assert set(sure[i].tolist()) <= g <= set(loose[i].tolist()), (r, i)
    if b.precision == "mixed":
        # mixed rows list the pairs within r_cut - min(skin/2, 0.8 A) at the
        # build first
        P0 = np.stack([xr, yr, zr], 1)
        rcore = b.pot.r_cut - min(0.5 * b.skin, 0.8)
        for i, row in enumerate(b.neighbor_rows(r, sort=False)):
            d = np.sqrt(((P0[row] - P0[i]) ** 2).sum(1))
            inner = np.flatnonzero(d < rcore - 1e-4)
            outer = np.flatnonzero(d > rcore + 1e-4)
            if inner.size and outer.size:
                assert inner[-1] < outer[0], (r, i)
    # the pruned lists the pair passes read hold every pair within r_tail
    # and within (r_tail, r_cut) at the current positions
    x, y, z = b.positions(r)
    P = np.stack([x, y, z], 1)
    cnt = b.active_counts(r)
    for i in range(P.shape[0]):
        d = np.sqrt(((P - P[i]) ** 2).sum(1))
        d[i] = np.inf
        edge_t = int(np.count_nonzero(np.abs(d - rt) < 1e-4))
        edge_c = int(np.count_nonzero(np.abs(d - rc) < 1e-4))
        assert abs(cnt[i, 0] - np.count_nonzero(d <= rt)) <= edge_t, (r, i)
        assert abs(cnt[i].sum() - np.count_nonzero(d <= rc)) <= edge_c, (r, i)


def test_lists_stay_exact_through_in_step_rebuilds_and_pruning():
    # a short skin makes the wires rebuild and prune several times in the
    # step loops, at different steps (a few replicas at a time, through the
    # per-step work lists)
    reps = [R(20.0, 30.0, T=298.0, r=0), R(15.0, 40.0, T=10.0, r=1),
            R(25.0, 20.0, T=298.0, r=2), R(20.0, 25.0, T=298.0, r=3)]
    note(f"lists through in-step rebuilds R={len(reps)}")
    b = WireBatch(reps, "mixed", skin=0.6, prune=0.1)
    b.prepare()
    b.run_batch(120, 40)
    torch.cuda.synchronize()
    st = b.status()
    assert not np.any(st & (A.ST_OVERFLOW | A.ST_NONFINITE | A.ST_OUTSIDE))
    assert st[0] & A.ST_REBUILT and st[2] & A.ST_REBUILT and st[3] & A.ST_REBUILT
    for r in range(b.R):
        _check_lists(b, r)


def test_lists_stay_exact_past_the_first_1024_replicas():
    # the work lists are made 1024 replicas at a time: replicas after the
    # first 1024 rebuild and prune through them as the first ones do
    reps = [R(15.0, 20.0, T=298.0, r=k) for k in range(1100)]
    note(f"lists through in-step rebuilds R={len(reps)}")
    b = WireBatch(reps, "mixed", skin=0.6, prune=0.1)
    b.prepare()
    b.run_batch(120, 40)
    torch.cuda.synchronize()
    st = b.status()
    assert not np.any(st & (A.ST_OVERFLOW | A.ST_NONFINITE | A.ST_OUTSIDE))
    second = [r for r in range(1024, b.R) if st[r] & A.ST_REBUILT]
    assert len(second) >= 10, len(second)
    for r in [0, 1023] + second[:3] + [b.R - 1]:
        _check_lists(b, r)


def test_forces_fp64_d1p5_wire():
    wl = W.wire_d1p5_l3_fp64()
    rp = wl.replicas[0]
    rp.jitter = 0.02
    note("forces fp64 D1.5 x L3 nm")
    b = WireBatch([rp], "fp64")
    b.prepare()
    torch.cuda.synchronize()
    x, y, z = b.positions(0)
    ref = oracle.forces(AU, x, y, z, 0)
    F = stackF(b.forces(0))
    Fr = stackF((ref["fx"], ref["fy"], ref["fz"]))
    assert eps_F(F, Fr) <= 1e-12
    assert np.abs(b.energies(0) - ref["e_atom"]).max() <= 1e-12
    assert abs(b.t["rep_energy"][0].item() - ref["E"]) <= 1e-12 * abs(ref["E"])
    assert abs(b.t["rep_wzz"][0].item() + ref["w6"][2]) <= 1e-10 * max(1.0, abs(ref["w6"][2]))


def test_forces_mixed_single_wire():
    rp = W.wire_d3_l20_mixed().replicas[0]
    note(f"forces mixed D={rp.D} L={rp.L}")
    b = WireBatch([rp], "mixed")
    b.prepare()
    torch.cuda.synchronize()
    x, y, z = b.positions(0)
    ref = oracle.forces(AU, x, y, z, 1)
    F = stackF(b.forces(0))
    Fr = stackF((ref["fx"], ref["fy"], ref["fz"]))
    e = eps_F(F, Fr)
    note(f"  eps_F = {e:.3e}  max|F| = {np.abs(Fr).max():.3f}")
    assert e <= 1e-5
    E = b.t["rep_energy"][0].item()
    assert abs(E - ref["E"]) <= 1e-6 * abs(ref["E"])
    assert np.abs(b.energies(0) - ref["e_atom"]).max() <= 2e-5
    wz = b.t["rep_wzz"][0].item()
    assert abs(wz + ref["w6"][2]) <= 1e-4 * max(1.0, abs(ref["w6"][2]))


def test_forces_mixed_ragged_batch():
    reps = [R(15.0, 12.0, r=0, jitter=0.02), R(30.0, 60.0, T=298.0, r=1, jitter=0.02),
            R(20.0, 33.0, r=2, jitter=0.02), R(25.0, 8.2, r=3, jitter=0.02)]
    note("forces mixed ragged batch")
    b = WireBatch(reps, "mixed")
    b.prepare()
    torch.cuda.synchronize()
    assert np.any(b.n_atoms % 64 != 0)
    for r in range(b.R):
        x, y, z = b.positions(r)
        ref = oracle.forces(AU, x, y, z, 0)
        F = stackF(b.forces(r))
        assert eps_F(F, stackF((ref["fx"], ref["fy"], ref["fz"]))) <= 1e-5, r
        assert abs(b.t["rep_energy"][r].item() - ref["E"]) <= 1e-6 * abs(ref["E"])
    # padding slots carry no force or energy
    for r in range(b.R):
        o, n, e = int(b.rep_off[r]), int(b.n_atoms[r]), int(b.rep_off[r + 1])
        assert torch.all(b.t["fx"][o + n:e] == 0) and torch.all(b.t["e_atom"][o + n:e] == 0)


from hypothesis import HealthCheck, given, settings, strategies as st


@settings(max_examples=12, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow])
@given(D=st.floats(8.0, 45.0), L=st.floats(6.0, 60.0), jitter=st.floats(0.0, 0.15),
       precision=st.sampled_from(["fp64", "mixed"]), order=st.sampled_from(["axial", "blocked"]),
       r=st.integers(0, 999))
def test_lists_and_forces_on_random_wires(D, L, jitter, precision, order, r):
    """Wires of random diameter, length and jitter, in either slot order and
    precision: the Verlet lists equal brute force and the forces and energy
    match the oracle at the GPU's positions (derandomised examples, so that
    every run checks the same wires)."""
    rp = R(D, L, T=298.0, r=r, jitter=jitter)
    note(f"random wire D {D:.2f} L {L:.2f} jitter {jitter:.3f} {precision} {order}")
    b = WireBatch([rp], precision, order=order)
    b.prepare()
    torch.cuda.synchronize()
    x, y, z = b.positions(0)
    rl = b.pot.r_cut + b.skin
    sure = brute_sets(x, y, z, rl - 1e-5)
    loose = brute_sets(x, y, z, rl + 1e-5)
    got = b.neighbor_rows(0)
    for i in range(x.size):
        g = set(got[i].tolist())
        assert len(g) == got[i].size and set(sure[i].tolist()) <= g <= set(loose[i].tolist()), i
    ref = oracle.forces(AU, x, y, z, 1)
    tol, etol = (1e-12, 1e-12) if precision == "fp64" else (1e-5, 1e-6)
    if x.size > 1:
        assert eps_F(stackF(b.forces(0)), stackF((ref["fx"], ref["fy"], ref["fz"]))) <= tol
    assert abs(b.t["rep_energy"][0].item() - ref["E"]) <= etol * max(1.0, abs(ref["E"]))


@pytest.mark.parametrize("kw", [{}, dict(baro_mass=300.0, baro_damp=2.0)],
                         ids=["pulled", "barostat"])
def test_init_state_matches_oracle(kw):
    """Jitter and Maxwell-Boltzmann velocities equal the oracle's; the pulled
    grip starts at v_pull, or at rest when the barostat moves the grips."""
    rp = R(20.0, 30.0, T=298.0, v=0.5, r=5, jitter=0.02)
    note(f"init state fp64 {kw}")
    b = WireBatch([rp], "fp64", gamma=0.0 if kw else 1.0, **kw)
    b.init_state()
    torch.cuda.synchronize()
    x0, y0, z0, f = oracle.build_wire(4.08, rp.D, rp.L, 2)
    st = oracle.State(x0, y0, z0, f)
    md = orc_md(b, 0)
    oracle.init_state(md, st, rp.jitter)
    x, y, z = b.positions(0)
    assert max(np.abs(x - st.x).max(), np.abs(y - st.y).max(), np.abs(z - st.z).max()) < 1e-14
    v = stackF(b.velocities(0))
    vr = stackF((st.vx, st.vy, st.vz))
    assert np.abs(v - vr).max() < 1e-12 * np.abs(vr).max()
    o = oracle.observe(AU, md, st, 1.0, rp.L)
    assert abs(o[2] - 298.0) < 1e-8
    vz_grip = v[b.flags(0) == A.GRIP_PULL, 2]
    assert np.all(vz_grip == (0.0 if kw else 0.5))


def test_step_fp64_lockstep_with_oracle():
    wl = W.wire_d1p5_l3_fp64()
    rp = wl.replicas[0]
    note("fp64 lockstep 20 steps")
    b = WireBatch([rp], "fp64", n_log=10)
    b.prepare()
    torch.cuda.synchronize()
    st = orc_state(b, 0)
    oracle.compute_forces(AU, st, 0)
    md = orc_md(b, 0)
    for k in range(4):
        b.step(5)
        oracle.run(AU, md, st, 5, 0)
        torch.cuda.synchronize()
        x, y, z = b.positions(0)
        dx = max(np.abs(x - st.x).max(), np.abs(y - st.y).max(), np.abs(z - st.z).max())
        v = stackF(b.velocities(0))
        dv = np.abs(v - stackF((st.vx, st.vy, st.vz))).max()
        note(f"  after {5 * (k + 1)} steps: |dx| {dx:.2e}  |dv| {dv:.2e}")
        assert dx < 1e-11 and dv < 1e-9
    assert b.step_index() == 20
    ob = b.obs_at(20)[0]
    orf = oracle.observe(AU, md, st, b.vol[0], b.L0[0])
    assert ob[A.OBS_STEP] == 20
    for k_gpu, k_or in ((A.OBS_EPOT, 0), (A.OBS_KE, 1), (A.OBS_T, 2), (A.OBS_WZZ, 3),
                        (A.OBS_SZZ, 4), (A.OBS_STRAIN, 5), (A.OBS_D, 7)):
        assert abs(ob[k_gpu] - orf[k_or]) <= 1e-9 * max(1.0, abs(orf[k_or])), (k_gpu, ob, orf)


@pytest.mark.parametrize("precision,ramp", [("fp64", False), ("mixed", False), ("fp64", True)])
def test_paper_protocol_lockstep_with_oracle(precision, ramp):
    """Nose-Hoover at 298 K, stepwise symmetric grips and a notched wire:
    positions, velocities, zeta and eta follow the oracle step for step
    (FP64 to rounding; mixed within its force error), and the elongation and
    strain of the records are the grips' travel.  With ramp, the target
    rises from 100 K to 298 K between steps 5 and 45."""
    rp = R(20.0, 40.0, T=298.0, v=0.0, r=3, jitter=0.01)
    note(f"paper protocol lockstep {precision} ramp={ramp}, 60 steps")
    rkw = dict(T_start=100.0, ramp_begin=5, ramp_steps=40) if ramp else {}
    b = WireBatch([rp], precision, n_log=10, **PROTOCOL, **rkw)
    b.prepare()
    torch.cuda.synchronize()
    st = orc_state(b, 0)
    assert st.x.size == oracle.build_wire(4.08, rp.D, rp.L, 2, 3, 4.08)[0].size
    oracle.compute_forces(AU, st, 0)
    md = orc_md(b, 0)
    # mixed: FP32 pair terms (eps_F ~ 1e-6) against the FP64 oracle
    # (measured: about 3e-7, 4e-6, 8e-6 and 4e-7 after 60 mixed steps)
    tol_x, tol_v, tol_z, tol_e = ((1e-11, 1e-9, 1e-9, 1e-11) if precision == "fp64"
                                  else (1e-5, 1e-4, 1e-4, 1e-5))
    for k in range(6):
        b.step(10)
        oracle.run(AU, md, st, 10, 0)
        torch.cuda.synchronize()
        x, y, z = b.positions(0)
        dx = max(np.abs(x - st.x).max(), np.abs(y - st.y).max(), np.abs(z - st.z).max())
        dv = np.abs(stackF(b.velocities(0)) - stackF((st.vx, st.vy, st.vz))).max()
        dzeta = abs(float(b.t["nh_xi"][0]) - st.zeta[0])
        deta = abs(float(b.t["nh_eta"][0]) - st.eta[0])
        note(f"  after {10 * (k + 1)} steps: |dx| {dx:.2e} |dv| {dv:.2e} "
             f"|dzeta| {dzeta:.2e} |deta| {deta:.2e}")
        assert dx < tol_x and dv < tol_v
        assert dzeta < tol_z and deta < tol_e
    assert abs(st.zeta[0]) > 1e-3
    ob = b.obs_at(60)[0]
    orf = oracle.observe(AU, md, st, b.vol[0], b.L0[0])
    assert ob[A.OBS_D] == orf[7] and abs(ob[A.OBS_D] - 2 * 0.05 * 3) < 1e-15
    assert abs(ob[A.OBS_STRAIN] - orf[5]) < 1e-15
    for k_gpu, k_or in ((A.OBS_EPOT, 0), (A.OBS_KE, 1), (A.OBS_T, 2), (A.OBS_WZZ, 3)):
        tol = 1e-9 if precision == "fp64" else 1e-4
        assert abs(ob[k_gpu] - orf[k_or]) <= tol * max(1.0, abs(orf[k_or])), (k_gpu, ob, orf)
    # the grips rest between moves and sit at z0 -+ 3 moves after 60 steps
    f = b.flags(0)
    z0 = b.t["z0"][:int(b.n_atoms[0])].cpu().numpy()
    assert np.all(z[f == A.GRIP_FIXED] == z0[f == A.GRIP_FIXED] - 0.05 * 3)
    assert np.all(z[f == A.GRIP_PULL] == z0[f == A.GRIP_PULL] + 0.05 * 3)
    assert np.all(b.velocities(0)[2][f != 0] == 0.0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_equilibration_barostat_lockstep_with_oracle(precision):
    """The equilibration protocol (Nose-Hoover on a temperature ramp and the
    axial barostat on the grip separation): atoms, thermostat and barostat
    variables follow the oracle step for step; the records carry D = 2 s."""
    rp = R(20.0, 40.0, T=298.0, v=0.0, r=8, jitter=0.01)
    note(f"equilibration lockstep {precision}, 60 steps")
    b = WireBatch([rp], precision, n_log=10, **EQUIL)
    b.prepare()
    torch.cuda.synchronize()
    st = orc_state(b, 0)
    oracle.compute_forces(AU, st, 0)
    md = orc_md(b, 0)
    # (measured in mixed precision: about 6e-7, 4e-6 and 3e-5 after 60 steps)
    tol_x, tol_v, tol_s = ((1e-11, 1e-9, 1e-10) if precision == "fp64" else (1e-5, 1e-4, 5e-4))
    for k in range(6):
        b.step(10)
        oracle.run(AU, md, st, 10, 0)
        torch.cuda.synchronize()
        x, y, z = b.positions(0)
        dx = max(np.abs(x - st.x).max(), np.abs(y - st.y).max(), np.abs(z - st.z).max())
        dv = np.abs(stackF(b.velocities(0)) - stackF((st.vx, st.vy, st.vz))).max()
        ps = b.t["baro_s"][:2].cpu().numpy()
        ds = np.abs(ps - st.piston).max()
        note(f"  after {10 * (k + 1)} steps: |dx| {dx:.2e} |dv| {dv:.2e} |ds| {ds:.2e} "
             f"s {ps[0]:.4f} ds/dt {ps[1]:.4f}")
        assert dx < tol_x and dv < tol_v and ds < tol_s
    assert abs(st.piston[0]) > 1e-3  # the piston moved
    ob = b.obs_at(60)[0]
    assert abs(ob[A.OBS_D] - 2 * float(b.t["baro_s"][0])) < 1e-15
    f = b.flags(0)
    z0 = b.t["z0"][:int(b.n_atoms[0])].cpu().numpy()
    s = float(b.t["baro_s"][0])
    assert np.allclose(z[f == A.GRIP_PULL], z0[f == A.GRIP_PULL] + s, atol=1e-12)
    assert np.allclose(z[f == A.GRIP_FIXED], z0[f == A.GRIP_FIXED] - s, atol=1e-12)


def test_langevin_with_temperature_ramp_lockstep_with_oracle():
    """BAOAB Langevin at a ramped target (mid-step noise amplitude), FP64,
    continuous pulling: the same trajectory as the oracle."""
    rp = R(20.0, 30.0, T=298.0, v=0.5, r=6, jitter=0.01)
    note("langevin ramp lockstep fp64, 40 steps")
    b = WireBatch([rp], "fp64", n_log=10, T_start=20.0, ramp_begin=0, ramp_steps=30)
    b.prepare()
    torch.cuda.synchronize()
    st = orc_state(b, 0)
    md = orc_md(b, 0)
    x0, y0, z0, f0 = oracle.build_wire(4.08, rp.D, rp.L, 2)
    st0 = oracle.State(x0, y0, z0, f0)
    oracle.init_state(md, st0, rp.jitter)
    assert np.abs(stackF((st.vx, st.vy, st.vz)) - stackF((st0.vx, st0.vy, st0.vz))).max() < 1e-12
    oracle.compute_forces(AU, st, 0)
    for k in range(4):
        b.step(10)
        oracle.run(AU, md, st, 10, 0)
        torch.cuda.synchronize()
        x, y, z = b.positions(0)
        dx = max(np.abs(x - st.x).max(), np.abs(y - st.y).max(), np.abs(z - st.z).max())
        dv = np.abs(stackF(b.velocities(0)) - stackF((st.vx, st.vy, st.vz))).max()
        note(f"  after {10 * (k + 1)} steps: |dx| {dx:.2e} |dv| {dv:.2e}")
        assert dx < 1e-11 and dv < 1e-9


@pytest.mark.parametrize("precision,lab", [("mixed", 0), ("mixed", 1), ("fp64", 1)])
def test_langevin_pulled_lockstep_with_oracle(precision, lab):
    """The benchmark's dynamics: BAOAB Langevin at 298 K with the top grip
    pulled at 0.5 A/ps, in the thermostat frame of the stretch profile or in
    the lab frame.  The GPU draws its noise from the same Philox counters as
    the oracle (FP32 normals in mixed precision), and in mixed precision
    leaves the second half kick of the 9 unlogged steps of each 10-step call
    to the next step's position update.  Positions and velocities follow the
    oracle step for step (FP64 to rounding, mixed within its force error),
    and so do the observables of the logged steps."""
    rp = R(20.0, 40.0, T=298.0, v=0.5, r=11, jitter=0.01)
    note(f"langevin pulled lockstep {precision} lab_frame={lab}, 60 steps")
    b = WireBatch([rp], precision, n_log=10, lab_frame=lab)
    b.prepare()
    torch.cuda.synchronize()
    st = orc_state(b, 0)
    oracle.compute_forces(AU, st, 0)
    md = orc_md(b, 0)
    assert md.lab_frame == lab and md.gamma == 1.0 and md.v_pull == 0.5
    tol_x, tol_v, tol_o = ((1e-11, 1e-9, 1e-9) if precision == "fp64" else (1e-5, 1e-4, 1e-4))
    for k in range(6):
        b.step(10)
        oracle.run(AU, md, st, 10, 0)
        torch.cuda.synchronize()
        x, y, z = b.positions(0)
        dx = max(np.abs(x - st.x).max(), np.abs(y - st.y).max(), np.abs(z - st.z).max())
        dv = np.abs(stackF(b.velocities(0)) - stackF((st.vx, st.vy, st.vz))).max()
        note(f"  after {10 * (k + 1)} steps: |dx| {dx:.2e} |dv| {dv:.2e}")
        assert dx < tol_x and dv < tol_v
        ob = b.obs_at(10 * (k + 1))[0]
        orf = oracle.observe(AU, md, st, b.vol[0], b.L0[0])
        for k_gpu, k_or in ((A.OBS_EPOT, 0), (A.OBS_KE, 1), (A.OBS_T, 2), (A.OBS_WZZ, 3),
                            (A.OBS_SZZ, 4), (A.OBS_STRAIN, 5), (A.OBS_D, 7)):
            assert abs(ob[k_gpu] - orf[k_or]) <= tol_o * max(1.0, abs(orf[k_or])), (k_gpu, ob, orf)
    f = b.flags(0)
    assert np.all(b.velocities(0)[2][f == A.GRIP_PULL] == 0.5)


def test_deferred_kick_leaves_trajectories_unchanged_bitwise():
    """In mixed precision the second half kick of an unlogged step is done by
    the next step's position update instead of the force pass, and the force
    pass takes its energy branch on logged steps only.  Logging every step
    (no deferred kicks, energies every step) or every 25th step (deferred
    kicks, energies rarely) gives the same positions, velocities and forces
    bit for bit, in the graph loop and in the plain loop."""
    reps = _three_replicas()
    note("deferred kick: n_log 1 vs 25 vs 7, 100 steps mixed")
    a = WireBatch(reps, "mixed", n_log=1)
    a.prepare()
    a.run_batch(100, 50)
    b = WireBatch(reps, "mixed", n_log=25, qbits=a.qbits)
    b.prepare()
    b.run_batch(100, 50)
    c = WireBatch(reps, "mixed", n_log=7, qbits=a.qbits)
    c.prepare()
    c.step(100)  # the call ends on an unlogged step, which then kicks itself
    for k in ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz"):
        assert torch.equal(a.t[k], b.t[k]), k
        assert torch.equal(a.t[k], c.t[k]), k
    assert a.step_index() == b.step_index() == c.step_index() == 100
    assert np.array_equal(a.obs_at(100), b.obs_at(100))


def test_nose_hoover_extended_energy_is_conserved_in_mixed_precision():
    """Resting grips, Nose-Hoover from 600 K towards 300 K in the batched
    graph loop: E_pot + K + Q zeta^2/2 + g kB T eta stays within the mixed
    force error while the temperature relaxes."""
    kb, _, _ = oracle.constants()
    rp = R(20.0, 40.0, T=600.0, v=0.0, r=4, jitter=0.01)
    note("nose-hoover invariant, mixed, 2000 steps")
    b = WireBatch([rp], "mixed", n_log=100, gamma=0.0, nh_tau=0.1, grip_step=0.0,
                  grip_hold=1000)
    b.prepare()
    b.t["T"].fill_(300.0)  # drawn at 600 K, thermostatted towards 300 K
    g = int(b.dof[0])
    Q = g * kb * 300.0 * 0.1 ** 2
    hs, Ts = [], []
    for _ in range(20):
        b.run_batch(100, 50)
        ob = b.obs_at(b.step_index())[0]
        xi, eta = float(b.t["nh_xi"][0]), float(b.t["nh_eta"][0])
        hs.append(ob[A.OBS_EPOT] + ob[A.OBS_KE] + 0.5 * Q * xi ** 2 + g * kb * 300.0 * eta)
        Ts.append(ob[A.OBS_T])
    n = int(b.n_atoms[0])
    hs = np.array(hs)
    note(f"  H spread {np.ptp(hs) / n:.2e} eV/atom, T {Ts[0]:.0f} -> {np.mean(Ts[10:]):.0f} K")
    assert np.ptp(hs) / n < 5e-5
    assert abs(np.mean(Ts[10:]) - 300.0) < 40.0


def test_d1p5_wire_end_to_end_forces_every_step():
    """The D 1.5 x L 3 nm wire: 1000 FP64 steps at 10 K with the top grip pulled at 0.5 A/ps;
    forces and per-atom energies checked against the oracle at every step."""
    wl = W.wire_d1p5_l3_fp64()
    note("D1.5 x L3 nm end-to-end 1000 steps fp64")
    b = WireBatch(wl.replicas, "fp64", n_log=100)
    b.prepare()
    worst = 0.0
    for s in range(wl.steps):
        b.step(1)
        x, y, z = b.positions(0)
        ref = oracle.forces(AU, x, y, z, 0)
        e = eps_F(stackF(b.forces(0)), stackF((ref["fx"], ref["fy"], ref["fz"])))
        worst = max(worst, e)
        assert e <= 1e-12, s
        assert np.abs(b.energies(0) - ref["e_atom"]).max() <= 1e-12, s
        if (s + 1) % 100 == 0:
            note(f"  step {s + 1}: worst eps_F {worst:.2e}")
    assert b.step_index() == 1000
    ob = b.obs_at(1000)[0]
    assert abs(ob[A.OBS_D] - 0.5 * 1000 * 0.002) < 1e-12
    assert abs(ob[A.OBS_STRAIN] - 1.0 / b.L0[0]) < 1e-12
    assert b.status()[0] & (A.ST_NONFINITE | A.ST_OVERFLOW) == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_paper_hard_cut(precision):
    """The paper's potential: a hard cut at 5.8 A (r_tail = r_cut, no tail).
    Forces and energies at a jittered wire equal the oracle's with the same
    cut; the jitter (0.005 A) keeps every pair at least 0.01 A from the cut,
    where FP32 distances could otherwise put a pair on either side.  Then 40
    FP64 steps (10 K, pulled) follow the oracle step for step."""
    from paper_1311_3890_amd.engine import Potential
    pot_g = Potential(r_tail=5.8, r_cut=5.8)
    pot_o = oracle.Pot(r_tail=5.8, r_cut=5.8)
    rp = R(25.0, 30.0, T=10.0, v=0.5, r=12, jitter=0.005)
    note(f"hard cut 5.8 A, {precision}")
    b = WireBatch([rp], precision, pot=pot_g, n_log=10)
    b.prepare()
    torch.cuda.synchronize()
    x, y, z = b.positions(0)
    P = np.stack([x, y, z], 1)
    d = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(2))
    assert np.abs(d - 5.8).min() > 0.01
    ref = oracle.forces(pot_o, x, y, z, 0)
    e = eps_F(stackF(b.forces(0)), stackF((ref["fx"], ref["fy"], ref["fz"])))
    note(f"  eps_F {e:.2e}")
    assert e <= (1e-12 if precision == "fp64" else 1e-5)
    assert abs(b.t["rep_energy"][0].item() - ref["E"]) <= (
        1e-12 if precision == "fp64" else 1e-6) * abs(ref["E"])
    # not the 7 A tail: the fifth shell (6.45 A) is cut off
    ref7 = oracle.forces(AU, x, y, z, 0)
    assert abs(ref7["E"] - ref["E"]) > 1e-5 * x.size
    if precision == "fp64":
        st = orc_state(b, 0)
        oracle.compute_forces(pot_o, st, 0)
        md = orc_md(b, 0)
        for k in range(4):
            b.step(10)
            oracle.run(pot_o, md, st, 10, 0)
            torch.cuda.synchronize()
            x, y, z = b.positions(0)
            dx = max(np.abs(x - st.x).max(), np.abs(y - st.y).max(), np.abs(z - st.z).max())
            dv = np.abs(stackF(b.velocities(0)) - stackF((st.vx, st.vy, st.vz))).max()
            note(f"  after {10 * (k + 1)} steps: |dx| {dx:.2e} |dv| {dv:.2e}")
            assert dx < 1e-11 and dv < 1e-9


def _three_replicas():
    return [R(15.0, 24.0, T=298.0, v=0.5, r=0), R(20.0, 40.0, T=10.0, v=1.0, r=1),
            R(30.0, 16.0, T=298.0, v=0.1, r=2)]


VARIANTS = pytest.mark.parametrize("kw", [{}, PROTOCOL, EQUIL],
                                   ids=["langevin", "protocol", "equilibration"])


@VARIANTS
def test_batched_equals_one_replica_at_a_time_bitwise(kw):
    reps = _three_replicas()
    note(f"batched vs alone, 120 steps mixed {kw}")
    b = WireBatch(reps, "mixed", n_log=40, **kw)
    b.prepare()
    b.run_batch(120, steps_per_graph=40)
    for r, rp in enumerate(reps):
        s = WireBatch([rp], "mixed", n_log=40, qbits=b.qbits, **kw)
        s.prepare()
        s.step(120)
        for a_, b_ in zip(b.positions(r) + b.velocities(r), s.positions(0) + s.velocities(0)):
            assert np.array_equal(a_, b_), r
        assert np.array_equal(b.obs_at(120)[r], s.obs_at(120)[0])


def test_pruned_lists_leave_trajectories_unchanged_bitwise():
    """The pair passes read lists pruned to r_cut + 2d and re-pruned when an
    atom moves more than d; the pairs they drop contribute exactly zero, so
    with the rebuild test on the build positions (the one used without
    pruning, so that both rebuild on the same steps) the trajectory equals
    the one on full lists bit for bit (several prunings and rebuilds happen
    at 298 K in 300 steps).  The default rebuild test bounds the
    displacement from the pruning instead: it rebuilds at least as often."""
    reps = _three_replicas()
    note("pruned vs full lists, 300 steps mixed")
    a = WireBatch(reps, "mixed", n_log=50, prune=0.1, rebuild_exact=True)
    a.prepare()
    a.run_batch(300, steps_per_graph=50)
    b = WireBatch(reps, "mixed", n_log=50, prune=0.0, qbits=a.qbits)
    b.prepare()
    b.run_batch(300, steps_per_graph=50)
    for k in ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz"):
        assert torch.equal(a.t[k], b.t[k]), k
    assert torch.equal(a.t["obs"], b.t["obs"])
    assert np.all(a.status() & A.ST_REBUILT)
    # the bound: the first rebuild of each replica comes no later
    c = WireBatch(reps, "mixed", n_log=1, n_slots=300, prune=0.1, qbits=a.qbits)
    c.prepare()
    e = WireBatch(reps, "mixed", n_log=1, n_slots=300, prune=0.1, qbits=a.qbits,
                  rebuild_exact=True)
    e.prepare()
    c.run_batch(300, steps_per_graph=50)
    e.run_batch(300, steps_per_graph=50)
    def first_rebuild(bb, r):
        o = bb.obs()[:, r]
        hit = (o[:, A.OBS_STATUS].astype(np.int64) & A.ST_REBUILT) != 0
        assert hit.any()
        return o[hit, A.OBS_STEP].min()
    for r in range(len(reps)):
        assert first_rebuild(c, r) <= first_rebuild(e, r), r


@VARIANTS
def test_graph_replay_equals_eager_bitwise(kw):
    reps = _three_replicas()
    note(f"graph vs eager, 100 steps {kw}")
    g = WireBatch(reps, "mixed", n_log=25, **kw)
    g.prepare()
    g.run_batch(100, steps_per_graph=30)  # 3 replays + 10 eager steps
    e = WireBatch(reps, "mixed", n_log=25, **kw)
    e.prepare()
    e.step(100)
    assert torch.equal(g.t["x"], e.t["x"]) and torch.equal(g.t["vz"], e.t["vz"])
    assert torch.equal(g.t["obs"], e.t["obs"])
    assert g.step_index() == e.step_index() == 100


@VARIANTS
def test_checkpoint_resume_is_bitwise(tmp_path, kw):
    reps = _three_replicas()
    note(f"checkpoint / resume {kw}")
    a = WireBatch(reps, "mixed", n_log=20, **kw)
    a.prepare()
    a.run_batch(60, 20)
    path = str(tmp_path / "ck.npz")
    a.save(path)
    a.run_batch(60, 20)
    b = WireBatch(reps, "mixed", n_log=20, qbits=a.qbits, **kw)
    b.load(path)
    assert b.step_index() == 60
    b.run_batch(60, 20)
    for k in ("x", "y", "z", "vx", "vy", "vz", "obs", "status", "nh_xi", "nh_eta", "baro_s"):
        assert torch.equal(a.t[k], b.t[k]), k


def test_barostat_runs_split_into_calls_repeat_bit_for_bit():
    """Without Nose-Hoover every call boundary is invisible: the barostat's
    grip force is re-formed at a call's start by the same sums the steps
    form, so 100 steps in one call equal 60 + 40 in two (Langevin, graph
    chunks of different lengths)."""
    reps = _three_replicas()
    note("barostat split calls, 100 steps mixed")
    kw = dict(gamma=1.0, baro_mass=300.0, baro_damp=2.0, T_start=50.0, ramp_steps=80)
    a = WireBatch(reps, "mixed", n_log=20, **kw)
    a.prepare()
    a.run_batch(100, 50)
    b = WireBatch(reps, "mixed", n_log=20, qbits=a.qbits, **kw)
    b.prepare()
    b.run_batch(60, 20)
    b.run_batch(40, 20)
    for k in ("x", "y", "z", "vx", "vy", "vz", "baro_s", "obs"):
        assert torch.equal(a.t[k], b.t[k]), k
    assert float(a.t["baro_s"].abs().max()) > 0


def test_mixed_dynamics_track_fp64_oracle_forces():
    """Mixed precision over 200 steps at 298 K: the forces at the GPU's
    positions stay within eps_F <= 1e-5 of the oracle and lists get rebuilt."""
    rp = R(30.0, 40.0, T=298.0, v=0.5, r=9, jitter=0.02)
    note("mixed 298K 200 steps with rebuilds")
    b = WireBatch([rp], "mixed", n_log=50)
    b.prepare()
    for k in range(4):
        b.run_batch(50, 25)
        x, y, z = b.positions(0)
        ref = oracle.forces(AU, x, y, z, 1)
        assert eps_F(stackF(b.forces(0)), stackF((ref["fx"], ref["fy"], ref["fz"]))) <= 1e-5
    assert b.status()[0] & A.ST_REBUILT
    T = b.obs()[:, 0, A.OBS_T]
    assert np.all(np.isfinite(T))


def test_neighbor_overflow_is_reported_and_regrown():
    rp = R(30.0, 30.0, r=1, jitter=0.02)
    note("nlist overflow k_cap=40")
    b = WireBatch([rp], "mixed", k_cap=40)
    b.init_state()
    lib = A.lib()
    A.check(lib.tbsma_build_cells(C.byref(b.params), C.byref(b.sys), C.byref(b.cells), b.work,
                                  b.stream()))
    need = C.c_int32()
    rc = lib.tbsma_neighbors(C.byref(b.params), C.byref(b.sys), C.byref(b.cells),
                             C.byref(b.nlist), b.work, C.byref(need), b.stream())
    assert rc == A.ECAPACITY
    x, y, z = b.positions(0)
    cnt = oracle.count_pairs(x, y, z, b.pot.r_cut + b.skin)
    assert need.value == cnt.max()
    b.build_lists()
    assert b.k_cap >= cnt.max()
    b.compute_forces()
    torch.cuda.synchronize()
    ref = oracle.forces(AU, x, y, z, 0)
    assert eps_F(stackF(b.forces(0)), stackF((ref["fx"], ref["fy"], ref["fz"]))) <= 1e-5


def test_degenerate_systems():
    note("degenerate: single atom, dimer, empty batch")
    # a single atom: no neighbours, zero density, zero force and energy
    one = W.Replica(1.0, 2.04, 10.0, 0.0, 1, 0, n_grip=0)
    b = WireBatch([one], "fp64")
    assert b.n_atoms[0] == 1
    b.prepare()
    torch.cuda.synchronize()
    assert b.t["fx"][0].item() == 0.0 and b.t["e_atom"][0].item() == 0.0
    # a dimer at r0 along z: E = 2 (A - xi)
    dim = W.Replica(1.0, 4.08 * 0.7068, 10.0, 0.0, 1, 0, n_grip=0)
    x = np.zeros(2)
    y = np.zeros(2)
    z = np.array([0.0, 2.884])
    f = np.zeros(2, dtype=np.uint8)
    for prec, tol in (("fp64", 1e-13), ("mixed", 1e-6)):
        b2 = WireBatch([dim], prec, wires=[(x, y, z, f)], gamma=0.0)
        b2.prepare(jitter=0.0)
        torch.cuda.synchronize()
        assert abs(b2.t["rep_energy"][0].item() - 2 * (AU.A - AU.xi)) < tol * 4
    # an empty system is a no-op
    s = A.System()
    s.R = 0
    out = A.ForcesOut()
    nl = A.NList()
    assert A.lib().tbsma_forces(C.byref(b.params), C.byref(s), C.byref(b.nlist),
                                C.byref(b.out), b.work, None) == A.OK


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_atom_outside_its_grid_is_reported_and_kept_exact(precision):
    """An atom moved 20 A beyond its replica's cell grid is binned into a
    border cell (the lists stay exact) and raises TBSMA_ST_OUTSIDE for that
    replica only; its neighbour replica evolves exactly as without it."""
    reps = [R(15.0, 24.0, T=298.0, v=0.5, r=0), R(15.0, 24.0, T=298.0, v=0.5, r=1)]
    note(f"atom outside the grid, {precision}")
    a = WireBatch(reps, precision, n_log=10)
    a.prepare()
    o, k = int(a.rep_off[1]), int(a.n_atoms[1]) // 2  # a dynamic atom mid-wire
    assert a.flags(1)[k] == 0
    a.t["x"][o + k] = float(a.grid_lo[1][0]) - 20.0
    a.build_lists()
    a.compute_forces()
    a.step(20)
    st = a.status()
    assert st[1] & A.ST_OUTSIDE and not st[0] & A.ST_OUTSIDE
    assert not np.any(st & A.ST_NONFINITE)
    fx, fy, fz = a.forces(1)
    assert fx[k] == 0.0 and fy[k] == 0.0 and fz[k] == 0.0  # nobody within r_cut
    b = WireBatch([reps[0]], precision, n_log=10, qbits=a.qbits)
    b.prepare()
    b.step(20)
    for p_, q_ in zip(a.positions(0) + a.velocities(0), b.positions(0) + b.velocities(0)):
        assert np.array_equal(p_, q_)


def test_rupture_gap_and_nonfinite_status():
    reps = [R(15.0, 40.0, r=0), R(15.0, 40.0, r=1)]
    note("rupture gap + NaN status")
    b = WireBatch(reps, "fp64", n_log=1, gamma=0.0)
    b.prepare()
    # cut replica 0 in two: move its upper half up by 9 A
    o, n = int(b.rep_off[0]), int(b.n_atoms[0])
    zz = b.t["z"][o:o + n]
    up = zz > 20.0
    zz[up] += 9.0
    b.t["z0"][o:o + n][up] += 9.0
    # poison one velocity of replica 1
    b.t["vx"][int(b.rep_off[1]) + 100] = float("nan")
    b.compute_forces()
    b.step(1)
    st = b.status()
    ob = b.obs_at(1)
    x, y, z = b.positions(0)
    zs = np.sort(z)
    gap = np.diff(zs).max()
    assert gap >= 9.0
    assert ob[0, A.OBS_GAP] == gap
    assert st[0] & A.ST_RUPTURED and not st[0] & A.ST_NONFINITE
    assert st[1] & A.ST_NONFINITE and not st[1] & A.ST_RUPTURED


def test_retired_replica_freezes_and_the_rest_are_unaffected():
    """A replica cut in two is ruptured at the first logged step; after
    `retire` A more grip travel it is retired: its atoms stop moving and its
    record repeats, while the other replica evolves exactly as it does alone."""
    reps = [R(20.0, 40.0, T=298.0, v=0.5, r=0), R(20.0, 40.0, T=298.0, v=0.5, r=1)]
    note("retirement after rupture, 200 steps mixed")
    # retirement is decided at logged steps; 0.045 A sits between two of them
    # (0.01 A apart) so that rounding of the grip travel cannot move it
    b = WireBatch(reps, "mixed", n_log=10, retire=0.045)
    b.prepare()
    o, n = int(b.rep_off[0]), int(b.n_atoms[0])
    zz = b.t["z"][o:o + n]
    up = zz > 20.0
    zz[up] += 9.0
    b.t["z0"][o:o + n][up] += 9.0
    b.compute_forces()
    b.run_batch(100, 50)
    st = b.status()
    assert st[0] & A.ST_RUPTURED and st[0] & A.ST_DONE
    assert not st[1] & (A.ST_RUPTURED | A.ST_DONE)
    x100 = [a.copy() for a in b.positions(0)]
    rec100 = b.obs_at(100)[0].copy()
    b.run_batch(100, 50)
    for a, c in zip(b.positions(0), x100):
        assert np.array_equal(a, c)
    assert np.array_equal(b.obs_at(200)[0], rec100)
    # retired at the first logged step with 0.045 A of travel (0.001 A/step)
    # after the rupture seen at step 10
    assert rec100[A.OBS_STEP] == 60.0
    s = WireBatch([reps[1]], "mixed", n_log=10, qbits=b.qbits, retire=0.045)
    s.prepare()
    s.run_batch(200, 50)
    for a_, c_ in zip(b.positions(1) + b.velocities(1), s.positions(0) + s.velocities(0)):
        assert np.array_equal(a_, c_)


def test_compacted_batch_continues_the_kept_replicas_exactly():
    """After a replica is retired, the compacted batch of the other two
    continues them bit for bit as the full batch does after a list rebuild and
    force evaluation at the same step; the step index, status and records
    carry over."""
    reps = [R(20.0, 40.0, T=298.0, v=0.5, r=k) for k in range(3)]
    note("compaction of 3 replicas after a retirement, 100 + 100 steps mixed")
    b = WireBatch(reps, "mixed", n_log=10, retire=0.045)
    b.prepare()
    o, n = int(b.rep_off[1]), int(b.n_atoms[1])
    zz = b.t["z"][o:o + n]
    up = zz > 20.0
    zz[up] += 9.0
    b.t["z0"][o:o + n][up] += 9.0
    b.compute_forces()
    b.run_batch(100, 50)
    assert b.status()[1] & A.ST_DONE and not (b.status()[[0, 2]] & A.ST_DONE).any()
    c = b.compact()
    assert c.R == 2 and c.step_index() == 100
    assert np.array_equal(c.status(), b.status()[[0, 2]])
    assert np.array_equal(c.obs(), b.obs()[:, [0, 2]])
    b.build_lists()
    b.compute_forces()
    b.run_batch(100, 50)
    c.run_batch(100, 50)
    for j, r in enumerate((0, 2)):
        for a_, c_ in zip(b.positions(r) + b.velocities(r), c.positions(j) + c.velocities(j)):
            assert np.array_equal(a_, c_)
    assert np.array_equal(c.obs(), b.obs()[:, [0, 2]])
    assert b.compact([1]).status()[0] & A.ST_DONE
    assert WireBatch.compact(c, []) is None


def test_paper_protocol_runs_to_failure_and_reports_properties():
    """Equilibration (barostat at 0.01 K), ramp and hold, then stepwise
    elongation until every replica has failed and been retired (fast
    settings: 0.05 A per grip every 20 steps); the curves and properties
    come out per original replica."""
    from paper_1311_3890_amd import protocol
    reps = [R(15.0, 30.0, T=300.0, v=0.0, r=k) for k in range(3)]
    note("paper protocol end to end, 3 x D1.5 L3 nm")
    proto = protocol.Protocol(baro_steps=300, ramp_steps=300, hold_steps=200, baro_mass=300.0,
                              baro_damp=5.0, grip_step=0.05, grip_hold=20, max_steps=20000,
                              retire=1.0, n_log=20, steps_per_graph=20)
    res = protocol.run(reps, proto, log=note)
    for r in range(len(reps)):
        eps, sig, st = res.recorder.curve(r)
        p = res.properties[r]
        note(f"  replica {r}: {eps.size} records, L0 {res.L0[r]:.2f} A, E {p['E']:.1f} GPa, "
             f"sigma_y {p['sigma_y']:.2f} GPa at {p['eps_y']:.3f}, eps_f {p['eps_f']:.3f}")
        assert st[-1] & A.ST_DONE and st[-1] & A.ST_RUPTURED
        # strain grows by 2 grip steps per hold, measured from the equilibrated length
        d = np.diff(eps)
        step = 2 * 0.05 / res.L0[r]
        assert np.all(np.isclose(d, 0.0, atol=1e-12) | np.isclose(d, step, rtol=1e-9))
        assert p["E"] > 0 and p["sigma_y"] > 0 and 0 < p["eps_y"] < p["eps_f"]
    assert len(res.recorder.ids) == 0  # all retired and compacted away


def _sampled_parity(b: WireBatch, reps_to_check, tol=1e-5, mode=1, etol=1e-6):
    """eps_F of the sampled replicas, and the relative error of their
    energies (per-atom e_i summed, and the record of the current step, which
    must be a logged one) against the oracle at the GPU's positions."""
    worst = 0.0
    rec = b.obs_at(b.step_index())
    assert b.step_index() % b.n_log == 0
    for r in reps_to_check:
        x, y, z = b.positions(r)
        ref = oracle.forces(AU, x, y, z, mode)
        e = eps_F(stackF(b.forces(r)), stackF((ref["fx"], ref["fy"], ref["fz"])))
        worst = max(worst, e)
        assert e <= tol, r
        E = float(np.sum(b.energies(r)))
        assert abs(E - ref["E"]) <= etol * abs(ref["E"]), (r, E, ref["E"])
        assert abs(rec[r][A.OBS_EPOT] - ref["E"]) <= etol * abs(ref["E"]), (r, rec[r], ref["E"])
    return worst


def test_blocked_order_fp64_lockstep_with_oracle():
    """A 4 nm wire whose atoms sit in the blocked slot order: the initial
    state and 20 FP64 Langevin steps follow the oracle, whose atoms are in
    generation order (noise keyed by the tag, not the slot)."""
    rp = R(40.0, 20.0, T=298.0, v=0.5, r=6, jitter=0.02)
    note("blocked order fp64 lockstep 20 steps")
    b = WireBatch([rp], "fp64", n_log=10, order="blocked")
    assert b.slot_tag[0] is not None
    assert not np.array_equal(b.slot_tag[0], np.arange(int(b.n_atoms[0])))
    b.init_state()
    torch.cuda.synchronize()
    x0, y0, z0, f = oracle.build_wire(4.08, rp.D, rp.L, 2)
    st = oracle.State(x0, y0, z0, f)
    md = orc_md(b, 0)
    oracle.init_state(md, st, rp.jitter)
    x, y, z = b.positions(0)
    assert max(np.abs(x - st.x).max(), np.abs(y - st.y).max(), np.abs(z - st.z).max()) < 1e-14
    assert np.array_equal(b.flags(0), f)
    b.build_lists()
    b.compute_forces()
    oracle.compute_forces(AU, st, 0)
    for k in range(4):
        b.step(5)
        oracle.run(AU, md, st, 5, 0)
        torch.cuda.synchronize()
        x, y, z = b.positions(0)
        dx = max(np.abs(x - st.x).max(), np.abs(y - st.y).max(), np.abs(z - st.z).max())
        dv = np.abs(stackF(b.velocities(0)) - stackF((st.vx, st.vy, st.vz))).max()
        note(f"  after {5 * (k + 1)} steps: |dx| {dx:.2e}  |dv| {dv:.2e}")
        assert dx < 1e-11 and dv < 1e-9


def test_thick_wire_blocks_stage_their_neighbours_by_gather_list():
    """A 5 nm wire (blocked slot order by default): after in-step rebuilds
    and prunings every block of the pair passes stages the exact set of its
    neighbours through a gather list, the Verlet lists are exact at their
    build positions, the pruned lists complete at the current ones, and
    forces and energies match the oracle."""
    rp = R(50.0, 60.0, T=298.0, v=0.5, r=3, jitter=0.02)
    note("D5 nm blocked order, gather staging, 150 steps mixed")
    # a short skin makes the wire rebuild and prune within the run
    b = WireBatch([rp], "mixed", n_log=25, skin=0.6, prune=0.1)
    assert b.slot_tag[0] is not None
    b.prepare()
    b.run_batch(150, 50)
    torch.cuda.synchronize()
    assert b.status()[0] & A.ST_REBUILT
    stg = b.staging()
    note(f"  staging {stg}")
    assert stg["gather"] > 0 and stg["unstaged"] == 0
    assert 0 < stg["mean_gathered"] <= 1536
    _check_lists(b, 0)
    worst = _sampled_parity(b, [0])
    note(f"  eps_F {worst:.2e}")


def test_gather_staging_leaves_trajectories_unchanged_bitwise():
    """Gather staging changes only where the pair passes read neighbour
    positions from (LDS instead of global memory), not the arithmetic or its
    order: 200 steps at 298 K with rebuilds and prunings, on and off, agree
    bit for bit.  So does gather staging with a list capacity above 256,
    where the pruning kernel's row-writing sweep repeats the distance tests
    instead of reading back the kept masks of its marking sweep."""
    rp = R(50.0, 40.0, T=298.0, v=0.5, r=4, jitter=0.02)
    note("gather staging on vs off, and with k_cap 264, 200 steps mixed")
    a = WireBatch([rp], "mixed", n_log=25, skin=0.6, prune=0.1, gather=1)
    assert a.k_cap <= 256
    a.prepare()
    a.run_batch(200, 50)
    g = WireBatch([rp], "mixed", n_log=25, skin=0.6, prune=0.1, gather=0, qbits=a.qbits)
    g.prepare()
    g.run_batch(200, 50)
    h = WireBatch([rp], "mixed", n_log=25, skin=0.6, prune=0.1, gather=1, qbits=a.qbits,
                  k_cap=264)
    h.prepare()
    h.run_batch(200, 50)
    torch.cuda.synchronize()
    assert a.status()[0] & A.ST_REBUILT
    assert a.staging()["gather"] > 0 and g.staging()["gather"] == 0
    assert h.k_cap == 264 and h.staging()["gather"] == a.staging()["gather"]
    for k in ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz", "obs", "status"):
        assert torch.equal(a.t[k], g.t[k]), k
        assert torch.equal(a.t[k], h.t[k]), k


def test_config2_pulled_to_rupture_forces_stay_within_parity():
    """The single D 3 x L 20 nm wire (+-0.02 A jitter, 10 K Langevin, mixed
    precision) pulled at 0.5 A/ps until it ruptures (at 10 K the wire draws
    out far beyond its yield point; at most 250 000 steps, strain 1.25):
    eps_F against the FP64 oracle at the GPU's positions every 5000 steps
    stays within 1e-5, energies within 1e-6."""
    wl = W.wire_d3_l20_mixed()
    note("D3 x L20 nm mixed, 10 K, pulled to rupture")
    b = WireBatch(wl.replicas, "mixed", n_log=500, n_slots=128, skin=wl.skin, prune=wl.prune,
                  k_cap=wl.k_cap, retire=2.0, strain_max=1.3)
    b.prepare()
    rows = []
    while b.step_index() < 250000:
        b.run_batch(5000, 500)
        torch.cuda.synchronize()
        st = int(b.status()[0])
        assert not st & (A.ST_NONFINITE | A.ST_OVERFLOW | A.ST_OUTSIDE), st
        rec = b.obs_at(b.step_index())[0]
        eps = _sampled_parity(b, [0])
        rows.append((b.step_index(), rec[A.OBS_STRAIN], rec[A.OBS_T], rec[A.OBS_SZZ], eps, st))
        note(f"  step {b.step_index():6d} strain {rec[A.OBS_STRAIN]:.4f} T {rec[A.OBS_T]:6.2f} K "
             f"sigma_zz {rec[A.OBS_SZZ]:6.3f} GPa eps_F {eps:.2e} status {st}")
        if st & A.ST_DONE:
            break
    assert rows[-1][5] & A.ST_RUPTURED, "the wire did not rupture within 250 000 steps"
    note(f"  max eps_F over {len(rows)} samples: {max(r[4] for r in rows):.2e}")


def test_launch_shapes_leave_trajectories_unchanged_bitwise():
    """Per-replica launch shapes (tiles per pair-pass block, stage class)
    change only where work runs: a batch with a mix of shapes follows the
    default batch bit for bit through rebuilds and prunings (150 steps at
    298 K, energies logged)."""
    reps = [R(15.0, 30.0, T=298.0, r=0), R(20.0, 40.0, T=10.0, r=1),
            R(25.0, 25.0, T=298.0, r=2), R(30.0, 35.0, T=298.0, r=3),
            R(15.0, 12.0, T=298.0, r=4)]
    shapes = [A.shape(1, 0), A.shape(2, 1), A.shape(4, 0), A.shape(2, 0), A.shape(1, 1)]
    note("launch shapes vs default, 150 steps mixed")
    a = WireBatch(reps, "mixed", n_log=25, skin=0.6, prune=0.1)
    a.prepare()
    a.run_batch(150, 50)
    b = WireBatch(reps, "mixed", n_log=25, skin=0.6, prune=0.1, qbits=a.qbits, shapes=shapes)
    b.prepare()
    b.run_batch(150, 50)
    torch.cuda.synchronize()
    assert np.all(a.status() & A.ST_REBUILT)
    for k in ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz", "e_atom", "obs", "status"):
        assert torch.equal(a.t[k], b.t[k]), k
    assert b.nbmap_blocks() == sum(-(-(int(n) // 64) // (s & 15))
                                   for n, s in zip(b.rep_off[1:] - b.rep_off[:-1], shapes))
    assert b.nbmap_blocks() > a.nbmap_blocks()


def test_autotune_chooses_a_shape_per_bucket_in_one_batch(tmp_path):
    """The tuner's trials run on the whole batch, one bucket at a time; the
    chosen shapes are applied to the batch, which stays within parity, and a
    cached choice is reused without trials."""
    from paper_1311_3890_amd import autotune
    reps = [R(15.0 if k % 2 else 30.0, 20.0 + 3 * k, T=298.0, r=k) for k in range(8)]
    note("autotune smoke, 8 replicas in 2 buckets")
    b = WireBatch(reps, "mixed", n_log=20)
    b.prepare()
    cache = str(tmp_path / "tune.json")
    cands = (A.shape(4, 1), A.shape(2, 0))
    res = autotune.tune(b, candidates=cands, steps=20, warmup=10, windows=1,
                        steps_per_graph=20, cache=cache, log=note)
    assert set(res["choice"]) == {"D15-warm", "D30-warm"}
    assert len(res["trials"]) == 2
    for r, rp in enumerate(reps):
        assert b.shapes[r] == res["choice"][autotune.bucket_key(autotune.bucket_of(rp))]
    b.run_batch(40 + (-b.step_index()) % 20, 20)  # to a logged step
    torch.cuda.synchronize()
    _sampled_parity(b, [0, 1])
    c = WireBatch(reps, "mixed", n_log=20)
    c.prepare()
    again = autotune.tune(c, candidates=cands, cache=cache, log=note)
    assert again["choice"] == res["choice"] and c.shapes == b.shapes


def test_replica_constants_and_rebase():
    """tbsma_replica_constants gives each replica's degrees of freedom, the
    hard-sphere volume of eq 5 and the inner grip faces exactly as their
    definitions over the wire's sites (notched, blocked order, and a wire
    without grips included); tbsma_rebase moves the grip references to the
    current positions and grows L0 by the barostat's elongation 2 s."""
    reps = [R(15.0, 30.0, T=10.0, r=0), R(40.0, 20.0, T=298.0, r=1),
            W.Replica(20.0, W.snap_length(25.0), 298.0, 0.5, W.seed_of(2), 2, n_grip=0)]
    note("replica constants and rebase")
    b = WireBatch(reps, "mixed", n_log=10, notch=(3, 4.08))
    torch.cuda.synchronize()
    for r, (x, y, z, f) in enumerate(b.wires):
        ndyn = int((f == A.DYN).sum())
        assert b.dof[r] == max(0, 3 * ndyn - 3)
        assert b.z_lo[r] == (z[f == A.GRIP_FIXED].max() if np.any(f == A.GRIP_FIXED) else z.min())
        assert b.z_hi[r] == (z[f == A.GRIP_PULL].min() if np.any(f == A.GRIP_PULL) else z.max())
        v = x.size * (4.0 / 3.0) * np.pi * (0.5 * AU.r0) ** 3
        assert abs(b.vol[r] - v) <= 1e-14 * v
    assert b.slot_tag[1] is not None
    # rebase after a barostat run: z0 = z and L0 + 2 s
    e = WireBatch(reps[:2], "mixed", n_log=10, gamma=0.0, nh_tau=0.1, baro_mass=300.0,
                  baro_damp=2.0)
    e.prepare()
    e.run_batch(60, 20)
    torch.cuda.synchronize()
    s = e.t["baro_s"].view(e.R, 2)[:, 0].cpu().numpy().copy()
    L0 = e.L0.copy()
    assert np.all(s != 0.0)
    e.rebase()
    assert torch.equal(e.t["z0"], e.t["z"])
    assert np.array_equal(e.L0, L0 + 2.0 * s)
    assert torch.all(e.t["baro_s"] == 0) and e.step_index() == 0


def test_full_size_batch512_sampled():
    """The 512-wire D 3 nm batch at full size in the benchmark's launch shape:
    graph-replayed steps, then sampled replicas against the oracle."""
    wl = W.batch512_d3()
    note(f"512-wire batch full size R={len(wl.replicas)}")
    b = WireBatch(wl.replicas, "mixed", n_log=50, skin=wl.skin, prune=wl.prune, k_cap=wl.k_cap)
    b.prepare()
    b.run_batch(100, 50)
    torch.cuda.synchronize()
    st = b.status()
    assert not np.any(st & (A.ST_NONFINITE | A.ST_OVERFLOW))
    idx = [0, 1, 77, 200, 311, 450, 510, 511]
    worst = _sampled_parity(b, idx)
    note(f"  worst eps_F over {len(idx)} replicas: {worst:.2e}")
    # 0.2 ps after a 298 K start on the perfect lattice, equipartition has
    # moved about half of the kinetic energy into the potential energy and the
    # 1/ps thermostat has only begun to restore it
    T = b.obs_at(100)[:, A.OBS_T]
    assert T.min() > 150.0 and T.max() < 320.0, (T.min(), T.max())


def test_full_size_d10_wire_sampled():
    wl = W.wire_d10_l100()
    note("D10 x L100 nm full size")
    b = WireBatch(wl.replicas, "mixed", n_log=50, strain_max=0.1)
    b.prepare()
    b.run_batch(50, 25)
    torch.cuda.synchronize()
    assert not b.status()[0] & (A.ST_NONFINITE | A.ST_OVERFLOW)
    worst = _sampled_parity(b, [0])
    stg = b.staging()
    note(f"  eps_F {worst:.2e}, staging {stg}")
    assert stg["gather"] > 0.9 * b.nbmap_blocks()


def test_batch2048_mixed_shapes_sampled():
    wl = W.batch2048_mixed_shapes()
    note(f"2048 mixed shapes R={len(wl.replicas)}")
    b = WireBatch(wl.replicas, "mixed", n_log=20, skin=wl.skin, prune=wl.prune, k_cap=wl.k_cap)
    b.prepare()
    b.run_batch(40, 20)
    torch.cuda.synchronize()
    assert not np.any(b.status() & (A.ST_NONFINITE | A.ST_OVERFLOW))
    _sampled_parity(b, [0, 1, 2, 3, 1001, 2047], mode=1)
