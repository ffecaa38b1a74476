"""tbsma_step_noalloc (the step loop on the library's static device scratch)
against tbsma_step on a caller's workspace.

Both start from the same initial state.  The reference is the documented
equivalent sequence on a freshly initialised workspace (cell binning, lists
and forces at the current positions, then tbsma_step); the variant does the
same on its own scratch.  Same kernels, same order, same inputs: positions,
velocities, forces, observables and status must agree bit for bit.  Two calls
in a row, the second on a smaller system, so the second starts from a
scratch that holds the first call's contents.
"""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

import workloads as W
from paper_1311_3890_amd import _abi as A
from paper_1311_3890_amd.engine import WireBatch

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rep(D, L, T, v, r):
    return W.Replica(D, W.snap_length(L), T, v, W.seed_of(r), r, jitter=0.02)


def _noalloc(b: WireBatch, n: int):
    A.check(A.lib().tbsma_step_noalloc(C.byref(b.params), C.byref(b.sys), C.byref(b.cells),
                                       C.byref(b.nlist), C.byref(b.out), C.byref(b.md),
                                       int(n), b.stream()))
    torch.cuda.synchronize()


def _reference(b: WireBatch, n: int):
    lib = A.lib()
    A.check(lib.tbsma_workspace_init(C.byref(b.params), C.byref(b.sys), b.work, b.stream()))
    b.build_lists()
    b.compute_forces()
    b.step(n)
    torch.cuda.synchronize()


KEYS = ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz", "obs", "status", "step",
        "rep_energy", "rep_wzz")


def _compare(reps, precision, n, **kw):
    note(f"noalloc vs step: {len(reps)} replicas, {precision}, {n} steps {kw}")
    a = WireBatch(reps, precision, n_log=10, **kw)
    a.prepare()
    b = WireBatch(reps, precision, n_log=10, qbits=a.qbits, **kw)
    b.prepare()
    if precision == "mixed" and any(t is not None for t in a.slot_tag):
        assert a.staging()["gather"] > 0
    for k in KEYS:
        assert torch.equal(a.t[k], b.t[k]), f"initial state differs in {k}"
    _reference(a, n)
    _noalloc(b, n)
    for k in KEYS:
        assert torch.equal(a.t[k], b.t[k]), k
    assert b.step_index() == n
    assert np.isfinite(b.t["obs"].cpu().numpy()).all()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "these tests need the GPU"
    torch.cuda.set_device(0)
    yield


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_equals_step_on_a_workspace_twice_second_smaller(precision):
    big = [_rep(30.0, 20.0, 298.0, 0.5, 0), _rep(20.0, 12.0, 10.0, 1.0, 1),
           _rep(15.0, 6.0, 298.0, 0.1, 2)]
    small = [_rep(15.0, 4.0, 298.0, 0.5, 3)]
    _compare(big, precision, 60)
    _compare(small, precision, 30)


def test_noalloc_thick_wire_with_gather_staging_and_launch_shapes():
    """The scratch also holds the gather lists of a thick wire in the
    blocked slot order, and the block map of non-default launch shapes."""
    reps = [_rep(50.0, 60.0, 298.0, 0.5, 4), _rep(20.0, 30.0, 10.0, 0.5, 5)]
    shapes = [A.shape(4, 1), A.shape(2, 0)]
    _compare(reps, "mixed", 40, shapes=shapes)
    _compare([_rep(15.0, 4.0, 298.0, 0.5, 6)], "mixed", 20)


def test_noalloc_rejects_a_system_beyond_its_scratch_and_zero_steps():
    b = WireBatch([_rep(15.0, 4.0, 298.0, 0.5, 0)], "mixed", n_log=10)
    b.prepare()
    x0 = b.t["x"].clone()
    assert A.lib().tbsma_step_noalloc(C.byref(b.params), C.byref(b.sys), C.byref(b.cells),
                                      C.byref(b.nlist), C.byref(b.out), C.byref(b.md), 0,
                                      b.stream()) == A.OK
    assert torch.equal(b.t["x"], x0)
    # a system whose workspace exceeds the scratch (a D 20 x L 100 nm wire,
    # about 1.85 M atoms) is refused before any work is enqueued
    big = WireBatch([_rep(200.0, 1000.0, 298.0, 0.5, 1)], "mixed", n_log=10)
    nb = C.c_size_t()
    A.check(A.lib().tbsma_workspace_query(C.byref(big.params), C.byref(big.sys), C.byref(nb)))
    assert nb.value > (32 << 20)
    torch.cuda.synchronize()
    x1 = big.t["x"].clone()
    rc = A.lib().tbsma_step_noalloc(C.byref(big.params), C.byref(big.sys), C.byref(big.cells),
                                    C.byref(big.nlist), C.byref(big.out), C.byref(big.md), 5,
                                    big.stream())
    assert rc == A.ECAPACITY
    assert b"static scratch" in A.lib().tbsma_last_error()
    torch.cuda.synchronize()
    assert torch.equal(big.t["x"], x1) and big.step_index() == 0
