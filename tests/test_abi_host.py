"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and its host-side wire builder and argument checks behave (no device
work is started here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_1311_3890_amd import _abi as A
from paper_1311_3890_amd.engine import build_wire_host

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "tbsma.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tbsma_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_five_calls():
    names = declared_functions()
    for n in ("tbsma_build_cells", "tbsma_neighbors", "tbsma_forces", "tbsma_step",
              "tbsma_run_batch"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = C.CDLL(A.LIB_PATH)
    for n in declared_functions():
        assert hasattr(L, n), n
    assert set(declared_functions()) == set(A.SIGNATURES)


@pytest.mark.parametrize("D,L", [(15.0, 30.6), (30.0, 200.0), (20.0, 12.24), (25.0, 100.0)])
def test_host_wire_builder_equals_oracle(D, L):
    x, y, z, f = build_wire_host(4.08, D, L, 2)
    xo, yo, zo, fo = oracle.build_wire(4.08, D, L, 2)
    assert x.size == xo.size
    assert np.array_equal(x, xo) and np.array_equal(y, yo) and np.array_equal(z, zo)
    assert np.array_equal(f, fo)


from hypothesis import given, settings, strategies as st


@settings(max_examples=60, deadline=None)
@given(a=st.floats(3.6, 4.4), D=st.floats(0.0, 40.0), L=st.floats(0.0, 90.0),
       n_grip=st.integers(0, 4), layers=st.integers(0, 6), depth=st.floats(0.0, 25.0))
def test_host_wire_builder_equals_oracle_on_random_geometries(a, D, L, n_grip, layers, depth):
    """The library's wire builder and the oracle's, written apart, give the
    same sites, order and flags for any lattice constant, diameter, length,
    grip thickness and notch."""
    x, y, z, f = build_wire_host(a, D, L, n_grip, layers, depth)
    xo, yo, zo, fo = oracle.build_wire(a, D, L, n_grip, layers, depth)
    assert x.size == xo.size
    assert np.array_equal(x, xo) and np.array_equal(y, yo) and np.array_equal(z, zo)
    assert np.array_equal(f, fo)
    # the blocked slot order of thick wires is a permutation of the sites
    from paper_1311_3890_amd.engine import blocked_order
    perm = blocked_order(x, y, z, a)
    assert np.array_equal(np.sort(perm), np.arange(x.size))


def test_wire_builder_capacity_and_errors():
    lib = A.lib()
    n = C.c_int64()
    assert lib.tbsma_build_wire(4.08, 15.0, 30.0, 2, 0, 0.0, None, None, None, None, 0,
                                C.byref(n)) == A.ECAPACITY
    assert n.value == 336
    assert lib.tbsma_build_wire(-1.0, 15.0, 30.0, 2, 0, 0.0, None, None, None, None, 0,
                                C.byref(n)) == A.EINVAL
    assert b"bad wire" in lib.tbsma_last_error()
    # empty wire
    assert lib.tbsma_build_wire(4.08, 15.0, 0.0, 2, 0, 0.0, None, None, None, None, 0,
                                C.byref(n)) == A.OK
    assert n.value == 0
    assert lib.tbsma_build_wire(4.08, 15.0, 30.0, 2, -1, 0.0, None, None, None, None, 0,
                                C.byref(n)) == A.EINVAL
    assert b"notch" in lib.tbsma_last_error()


@pytest.mark.parametrize("D,L,layers,depth", [(31.0, 204.0, 3, 4.08), (15.0, 30.6, 2, 2.04),
                                               (20.0, 40.8, 5, 100.0)])
def test_notched_wire_builder_equals_oracle(D, L, layers, depth):
    x, y, z, f = build_wire_host(4.08, D, L, 2, layers, depth)
    xo, yo, zo, fo = oracle.build_wire(4.08, D, L, 2, layers, depth)
    assert x.size == xo.size < build_wire_host(4.08, D, L, 2)[0].size
    assert np.array_equal(x, xo) and np.array_equal(y, yo) and np.array_equal(z, zo)
    assert np.array_equal(f, fo)


def _params(**kw):
    p = A.Params(0.2061, 1.790, 10.229, 4.036, 2.884, 6.5, 7.0, 1.0, 8.0, 196.96657, A.MIXED, 21,
                 0.15)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("kw,msg", [
    (dict(cell=7.5), b"cell edge"),
    (dict(r_tail=7.5), b"r_tail"),
    (dict(qbits=30), b"qbits"),
    (dict(precision=7), b"precision"),
    (dict(cell=20.0), b"cell/2"),
    (dict(prune=0.6), b"prune"),
    (dict(prune=-0.1), b"prune"),
    (dict(gather=2), b"gather"),
    (dict(rebuild_exact=2), b"rebuild_exact"),
])
def test_parameter_checks(kw, msg):
    sysm = A.System()
    sysm.R = 0
    nb = C.c_size_t()
    rc = A.lib().tbsma_workspace_query(C.byref(_params(**kw)), C.byref(sysm), C.byref(nb))
    assert rc == A.EINVAL
    assert msg in A.lib().tbsma_last_error()


def test_layout_checks():
    """Offsets that are not multiples of 64 or do not end at N are refused."""
    rep = (C.c_int64 * 2)(0, 100)
    cel = (C.c_int64 * 2)(0, 10)
    s = A.System(1, 4, 100, 10, C.cast(rep, C.c_void_p), C.cast(cel, C.c_void_p))
    nb = C.c_size_t()
    assert A.lib().tbsma_workspace_query(C.byref(_params()), C.byref(s), C.byref(nb)) == A.EINVAL
    rep2 = (C.c_int64 * 2)(0, 128)
    s2 = A.System(1, 4, 128, 10, C.cast(rep2, C.c_void_p), C.cast(cel, C.c_void_p))
    assert A.lib().tbsma_workspace_query(C.byref(_params()), C.byref(s2), C.byref(nb)) == A.EINVAL
    assert b"NULL" in A.lib().tbsma_last_error()


def test_autotune_buckets_group_by_diameter_and_temperature():
    import workloads as W
    from paper_1311_3890_amd import autotune
    wl = W.batch2048_mixed_shapes(64)
    b = autotune.buckets(wl.replicas)
    # diameters go round-robin by r mod 4 and temperatures by r mod 2, so each
    # diameter comes with one temperature class
    assert len(b) == 4
    seen = sorted(r for idx in b.values() for r in idx)
    assert seen == list(range(64))
    for (D, cls), idx in b.items():
        for r in idx:
            assert wl.replicas[r].D == D
            assert (wl.replicas[r].T < 100) == (cls == "cold")


def test_workloads_are_seeded_and_snapped():
    import workloads as W
    a = W.batch512_d3()
    b = W.batch512_d3()
    assert [r.L for r in a.replicas] == [r.L for r in b.replicas]
    assert len(a.replicas) == 512
    for r in a.replicas:
        n = r.L / (W.A_LAT / 2)
        assert abs(n - round(n)) < 1e-9 and 50 - 2.04 <= r.L <= 400 + 2.04
    assert len({r.seed for r in a.replicas}) == 512


def _dummy_step_args(R=1, **md_kw):
    """Structures that pass every host-side check up to the dynamics
    settings; their device pointers are placeholders that the checks only
    compare with NULL (nothing runs: the checks fail first)."""
    ph = C.c_void_p(0x1000)
    rep = (C.c_int64 * (R + 1))(*[64 * r for r in range(R + 1)])
    cel = (C.c_int64 * (R + 1))(*[8 * r for r in range(R + 1)])
    s = A.System(R, 4, 64 * R, 8 * R, C.cast(rep, C.c_void_p), C.cast(cel, C.c_void_p),
                 *([ph] * 14), ph)
    cells = A.Cells(ph, ph)
    nl = A.NList(ph, ph, 8, 0, ph, ph, ph, None, ph)
    out = A.ForcesOut(ph, ph, ph, ph, None, ph, ph)
    md = A.MD(0.002, 0.0, 0, 10, 4, 0, *([ph] * 11), 0.0, None)
    for k, v in md_kw.items():
        setattr(md, k, v)
    return s, cells, nl, out, md, (rep, cel)


@pytest.mark.parametrize("R,kw,msg", [
    (0, dict(gamma=1.0, nh_tau=0.1), b"exclude"),
    (0, dict(nh_tau=-1.0), b"nh_tau"),
    (1, dict(nh_tau=0.1), b"nh_xi"),
    (0, dict(grip_hold=-5), b"grip_hold"),
    (0, dict(grip_hold=10, grip_step=float("nan")), b"grip_step"),
    (0, dict(baro_mass=100.0, grip_hold=10), b"exclude"),
    (0, dict(baro_mass=-1.0), b"baro_mass"),
    (1, dict(baro_mass=100.0), b"baro_s"),
])
def test_dynamics_setting_checks(R, kw, msg):
    s, cells, nl, out, md, keep = _dummy_step_args(R, **kw)
    rc = A.lib().tbsma_step(C.byref(_params()), C.byref(s), C.byref(cells), C.byref(nl),
                            C.byref(out), C.byref(md), None, 1, None)
    assert rc == A.EINVAL
    assert msg in A.lib().tbsma_last_error()


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})])
def test_bench_refuses_more_than_one_gpu(argv, env):
    # one GPU only: the refusal comes before any device or library is touched
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), *argv],
                       capture_output=True, text=True, timeout=120,
                       env={**os.environ, **env})
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_bench_counter_records_match_the_kernel_source():
    """The profiler counter records that bench.py reports beside its timing
    (HBM bytes, VALU instructions) are read only while the kernel source
    still has the hash they were taken on, and the VALU issue fraction is the
    recorded instructions over the launch time, against one wave64
    instruction per CU per cycle on 256 CUs at 2.4 GHz."""
    import importlib.util
    import json
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    with open(os.path.join(root, "profiles", "hbm_traffic.json")) as f:
        recs = json.load(f)["k_force_mixed"]
    rec = bench.counter_record("k_force_mixed", recs[0]["workload"])
    if rec is None:  # kernels changed since the counters were taken
        assert bench.counter_traffic(None) is None and bench.valu_issue(None, 1e-3) is None
        return
    assert bench.counter_traffic(rec) == pytest.approx(
        (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024)
    v = bench.valu_issue(rec, 400e-6)
    assert v["peak_instr_per_s"] == pytest.approx(256 * 2.4e9)
    assert v["frac"] == pytest.approx(rec["valu_instr"] / 400e-6 / (256 * 2.4e9))
    assert bench.counter_record("k_force_mixed", "no such workload") is None


def test_noalloc_step_refuses_a_system_beyond_its_scratch_on_the_host():
    """tbsma_step_noalloc checks the system's workspace against its static
    scratch before any device work (placeholders only, nothing runs)."""
    R = 1
    N = 64 * 40000  # 2.56 M slots: about 60 MB of workspace
    ph = C.c_void_p(0x1000)
    rep = (C.c_int64 * 2)(0, N)
    cel = (C.c_int64 * 2)(0, 8)
    s = A.System(R, 4, N, 8, C.cast(rep, C.c_void_p), C.cast(cel, C.c_void_p),
                 *([ph] * 14), ph)
    nb = C.c_size_t()
    A.check(A.lib().tbsma_workspace_query(C.byref(_params()), C.byref(s), C.byref(nb)))
    assert nb.value > (32 << 20)
    cells = A.Cells(ph, ph)
    nl = A.NList(ph, ph, 8, 0, ph, ph, ph, None, ph)
    out = A.ForcesOut(ph, ph, ph, ph, None, ph, ph)
    md = A.MD(0.002, 1.0, 0, 10, 4, 0, *([ph] * 11), 0.0, None)
    rc = A.lib().tbsma_step_noalloc(C.byref(_params()), C.byref(s), C.byref(cells),
                                    C.byref(nl), C.byref(out), C.byref(md), 1, None)
    assert rc == A.ECAPACITY
    assert b"static scratch" in A.lib().tbsma_last_error()


@pytest.mark.parametrize("shape,ok", [(A.shape(4, 1), True), (A.shape(1, 0), True),
                                      (A.shape(2, 1), True), (A.shape(3, 0), False),
                                      (A.shape(4, 2), False), (A.shape(8, 0), False)])
def test_launch_shape_checks(shape, ok):
    """Per-replica launch shapes: 1, 2 or 4 tiles per block and stage class
    0 or 1; the workspace holds a block map of ceil(tiles / tiles_per_block)
    blocks per replica."""
    R, N = 2, 64 * 10
    ph = C.c_void_p(0x1000)
    rep = (C.c_int64 * 3)(0, 64 * 6, N)
    cel = (C.c_int64 * 3)(0, 8, 16)
    s = A.System(R, 4, N, 16, C.cast(rep, C.c_void_p), C.cast(cel, C.c_void_p),
                 *([ph] * 14), ph)
    nb0 = C.c_size_t()
    A.check(A.lib().tbsma_workspace_query(C.byref(_params()), C.byref(s), C.byref(nb0)))
    sh = (C.c_int32 * R)(A.SHAPE_DEFAULT, shape)
    s.shape_h = C.cast(sh, C.c_void_p)
    nb = C.c_size_t()
    rc = A.lib().tbsma_workspace_query(C.byref(_params()), C.byref(s), C.byref(nb))
    assert rc == A.EINVAL and b"both" in A.lib().tbsma_last_error()  # device copy missing
    s.shape = ph
    rc = A.lib().tbsma_workspace_query(C.byref(_params()), C.byref(s), C.byref(nb))
    if ok:
        assert rc == A.OK
        assert (nb.value >= nb0.value) == ((shape & 15) <= 4)
    else:
        assert rc == A.EINVAL and b"launch shape" in A.lib().tbsma_last_error()


def test_replica_constants_and_rebase_check_their_outputs():
    ph = C.c_void_p(0x1000)
    rep = (C.c_int64 * 2)(0, 64)
    cel = (C.c_int64 * 2)(0, 8)
    s = A.System(1, 4, 64, 8, C.cast(rep, C.c_void_p), C.cast(cel, C.c_void_p),
                 *([ph] * 14), ph)
    lib = A.lib()
    assert lib.tbsma_replica_constants(C.byref(_params()), C.byref(s), ph, None, ph, ph,
                                       None) == A.EINVAL
    assert b"required" in lib.tbsma_last_error()
    assert lib.tbsma_rebase(C.byref(_params()), C.byref(s), None, None, None) == A.EINVAL
    assert b"L0" in lib.tbsma_last_error()
