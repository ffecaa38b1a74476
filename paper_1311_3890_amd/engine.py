"""Replica batches on the GPU: layout, device buffers and calls into libtbsma.

``WireBatch`` packs R nanowire replicas into one slot space (each replica's
slots padded to a multiple of 64), sizes one cell grid per replica, allocates
every buffer as a torch tensor on the current device, and forwards each
operation to the C ABI of libtbsma (include/tbsma.h).  Nothing here computes
any part of the method; PyTorch provides device memory and the stream only.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np
import torch

from . import _abi as A

MASS_AU = 196.96657  # amu


@dataclass
class Potential:
    """TB-SMA parameters for Au (Table 1), r0 read as the nearest-neighbour
    distance 2.884 A; cubic tail from r_tail to r_cut."""
    A: float = 0.2061
    xi: float = 1.790
    p: float = 10.229
    q: float = 4.036
    r0: float = 2.884
    r_tail: float = 6.5
    r_cut: float = 7.0


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


def build_wire_host(a: float, D: float, L: float, n_grip: int = 2, notch_layers: int = 0,
                    notch_depth: float = 0.0):
    """Host-side wire geometry from libtbsma (tbsma_build_wire), optionally
    with the ring notch of Figure 1 at mid-length."""
    lib = A.lib()
    n = C.c_int64()
    rc = lib.tbsma_build_wire(a, D, L, n_grip, notch_layers, notch_depth, None, None, None,
                              None, 0, C.byref(n))
    if rc not in (A.OK, A.ECAPACITY):
        A.check(rc)
    x, y, z = (np.empty(n.value) for _ in range(3))
    f = np.empty(n.value, dtype=np.uint8)
    A.check(lib.tbsma_build_wire(a, D, L, n_grip, notch_layers, notch_depth, x.ctypes.data,
                                 y.ctypes.data, z.ctypes.data, f.ctypes.data, n.value,
                                 C.byref(n)))
    return x, y, z, f


def blocked_order(x, y, z, a: float):
    """Slot order of a thick wire in which every 256 consecutive atoms are a
    compact piece of it: atoms grouped by supercells of 4a x 4a x 4a (256
    lattice sites), supercells visited slab by slab along the axis and
    row by row in each slab, rows in alternating directions (so that
    consecutive supercells touch), sites within a supercell by plane, row and
    column.  Returns the tags (generation indices) in slot order.  The pair
    passes can then stage each block's neighbours in LDS (gather staging)."""
    h = 0.5 * a
    i = np.rint(np.asarray(x) / h).astype(np.int64)
    j = np.rint(np.asarray(y) / h).astype(np.int64)
    k = np.rint(np.asarray(z) / h).astype(np.int64)
    sx, sy, sz = np.floor_divide(i + 4, 8), np.floor_divide(j + 4, 8), np.floor_divide(k, 8)
    row = np.where(sz % 2 == 0, sy, -sy)
    col = np.where(sy % 2 == 0, sx, -sx)
    return np.lexsort((i, j, k, col, row, sz)).astype(np.int32)


# wires at least this thick (A) get the blocked slot order under order="auto":
# their axial (generation) order puts about 1700 or more atoms in the slot
# window of a block of 256, more than the pair passes stage in LDS
BLOCKED_MIN_D = 36.0


class WireBatch:
    """R independent [100] Au nanowires advanced together on one GPU.

    replicas      objects with D, L (A), T (K), v_pull (A/ps), seed, rep_id,
                  n_grip and jitter (workloads.Replica).
    precision     "mixed" (FP32 pair terms, FP64 state and sums) or "fp64".
    skin, cell    Verlet skin and cell edge (A; cell defaults to the smallest
                  allowed, at least 8 A); k_cap: list capacity (grows on
                  overflow at build_lists).
    prune         half-width d of the pair lists' pruning (mixed; 0: off).
    gamma         Langevin friction (1/ps); nh_tau > 0 selects Nose-Hoover
                  instead (gamma must then be 0).
    dt, n_log, n_slots  time step (ps), logging interval and record ring.
    strain_max    strain the cell grids leave room for.
    lab_frame     1: the Langevin O step acts on lab-frame velocities.
    grip_step, grip_hold  stepwise symmetric grips (grip_hold > 0).
    notch         (planes, depth in A) of the ring notch, or None.
    T_start, ramp_begin, ramp_steps  temperature ramp (ramp_steps > 0).
    baro_mass, baro_load, baro_damp  axial barostat on the grip separation
                  (baro_mass > 0).
    retire        grip travel (A) after the first rupture before a replica is
                  retired (0: never).
    qbits         position quantum 2^-qbits A (mixed; default from the grid).
    order         slot order of each replica's atoms: "axial" (generation
                  order, along the wire), "blocked" (blocked_order), or
                  "auto" (blocked for D >= BLOCKED_MIN_D).  Accessors return
                  per-atom arrays by tag whatever the order.
    gather        gather staging of the pair passes (mixed; tbsma_params);
                  default: on when some replica is in the blocked order.
    shapes        launch shape of each replica's pair-pass blocks
                  (_abi.shape(tiles_per_block, stage_class)), or None for
                  the default; see set_shapes.
    rebuild_exact with pruning, test the displacement since the list build
                  on the FP64 build positions instead of bounding it from
                  the pruning (tbsma_params.rebuild_exact): the lists then
                  rebuild on the same steps as without pruning.
    The settings mean what include/tbsma.h says of tbsma_md and tbsma_params.
    """

    def __init__(self, replicas: Sequence, precision: str = "mixed", *, skin: float = 1.0,
                 cell: float | None = None, k_cap: int = 176, gamma: float = 1.0, dt: float = 0.002,
                 n_log: int = 100, n_slots: int = 64, strain_max: float = 0.5,
                 lab_frame: int = 0, a: float = 4.08, pot: Potential | None = None,
                 device=None, wires=None, qbits: int | None = None, prune: float = 0.15,
                 retire: float = 0.0, nh_tau: float = 0.0, grip_step: float = 0.0,
                 grip_hold: int = 0, notch: tuple | None = None, T_start=None,
                 ramp_begin: int = 0, ramp_steps: int = 0, baro_mass: float = 0.0,
                 baro_load: float = 0.0, baro_damp: float = 0.0, order: str = "auto",
                 gather: int | None = None, shapes: Sequence[int] | None = None,
                 rebuild_exact: bool = False):
        self.replicas = list(replicas)
        if not self.replicas:
            raise ValueError("a batch needs at least one replica")
        self.pot = pot or Potential()
        if nh_tau > 0 and gamma > 0:
            raise ValueError("the Nose-Hoover thermostat (nh_tau > 0) needs gamma = 0")
        # settings a compacted copy of this batch is built with
        self._kw = dict(skin=skin, cell=cell, gamma=gamma, dt=dt, n_log=n_log, n_slots=n_slots,
                        strain_max=strain_max, lab_frame=lab_frame, a=a, pot=self.pot,
                        device=device, prune=prune, retire=retire, nh_tau=nh_tau,
                        grip_step=grip_step, grip_hold=grip_hold, notch=notch,
                        T_start=T_start, ramp_begin=ramp_begin, ramp_steps=ramp_steps,
                        baro_mass=baro_mass, baro_load=baro_load, baro_damp=baro_damp,
                        order=order, gather=gather, rebuild_exact=rebuild_exact)
        self.shapes = None if shapes is None else [int(v) for v in shapes]
        if self.shapes is not None and len(self.shapes) != len(self.replicas):
            raise ValueError("shapes needs one launch shape per replica")
        self.baro_mass, self.baro_load = float(baro_mass), float(baro_load)
        self.baro_damp = float(baro_damp)
        self.nh_tau, self.grip_step, self.grip_hold = float(nh_tau), float(grip_step), int(grip_hold)
        self.notch = notch
        self.precision = precision
        k_cap = (int(k_cap) + 7) // 8 * 8
        if cell is None:  # the smallest cell the 27-cell scan allows, at least 8 A
            cell = max(8.0, self.pot.r_cut + skin)
        self.skin, self.cell, self.k_cap = skin, cell, k_cap
        self.gamma, self.dt, self.lab_frame = gamma, dt, lab_frame
        self.n_log, self.n_slots = n_log, n_slots
        self.a = a
        self.device = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        R = len(self.replicas)
        self.R = R
        # --- host geometry and layout -------------------------------------------------
        nl_, nd_ = notch if notch is not None else (0, 0.0)
        self.wires = wires if wires is not None else [
            build_wire_host(a, rp.D, rp.L, rp.n_grip, nl_, nd_) for rp in self.replicas]
        self.n_atoms = np.array([w[0].size for w in self.wires], dtype=np.int64)
        if order not in ("auto", "axial", "blocked"):
            raise ValueError(f"unknown slot order {order!r}")
        self.order = order
        # tags of each replica's slots (None: slot order = tag order)
        self.slot_tag = [
            blocked_order(w[0], w[1], w[2], a)
            if order == "blocked" or (order == "auto" and rp.D >= BLOCKED_MIN_D) else None
            for w, rp in zip(self.wires, self.replicas)]
        pad = (self.n_atoms + A.TILE - 1) // A.TILE * A.TILE
        self.rep_off = np.zeros(R + 1, dtype=np.int64)
        self.rep_off[1:] = np.cumsum(pad)
        N = int(self.rep_off[-1])
        self.N = N
        margin = cell
        gdim = np.zeros((R, 3), dtype=np.int32)
        glo = np.zeros((R, 3), dtype=np.float64)
        for r, rp in enumerate(self.replicas):
            gxy = int(math.ceil((rp.D + 2 * margin) / cell))
            gz = int(math.ceil((rp.L * (1.0 + strain_max) + 2 * margin) / cell))
            gdim[r] = (gxy, gxy, gz)
            # symmetric grips stretch the wire both ways
            below = 0.5 * strain_max * rp.L if grip_hold > 0 or baro_mass > 0 else 0.0
            glo[r] = (-0.5 * gxy * cell, -0.5 * gxy * cell, -margin - below)
        self.grid_dim, self.grid_lo = gdim, glo
        ncell = gdim.prod(axis=1).astype(np.int64)
        self.cell_off = np.zeros(R + 1, dtype=np.int64)
        self.cell_off[1:] = np.cumsum(ncell)
        self.C = int(self.cell_off[-1])
        self.max_zbins = int(2 * gdim[:, 2].max())
        half = float((gdim * cell).max()) / 2.0
        self.qbits = int(qbits) if qbits is not None else int(
            min(24, math.floor(31 - math.log2(1.1 * half + 16.0))))
        # --- host arrays of the atoms -----------------------------------------------
        xh = np.zeros(N)
        yh = np.zeros(N)
        zh = np.zeros(N)
        fh = np.full(N, A.PAD, dtype=np.uint8)
        tagh = np.zeros(N, dtype=np.int32)
        for r, (x, y, z, f) in enumerate(self.wires):
            o = self.rep_off[r]
            n = x.size
            perm = self.slot_tag[r]
            sl = slice(None) if perm is None else perm
            xh[o:o + n], yh[o:o + n], zh[o:o + n], fh[o:o + n] = x[sl], y[sl], z[sl], f[sl]
            npad = int(self.rep_off[r + 1] - o)
            tagh[o:o + npad] = np.arange(npad, dtype=np.int32)
            if perm is not None:
                tagh[o:o + n] = perm
        # pads sit at the replica's grid corner (never used)
        self.L0 = np.array([rp.L for rp in self.replicas], dtype=np.float64)
        tile_rep = np.repeat(np.arange(R, dtype=np.int32), pad // A.TILE)
        # --- device buffers ------------------------------------------------------------
        dev = self.device
        f64 = dict(dtype=torch.float64, device=dev)
        ft = torch.float32 if precision == "mixed" else torch.float64
        self.t = {}
        T = self.t
        T["rep_off"] = torch.tensor(self.rep_off, device=dev)
        T["cell_off"] = torch.tensor(self.cell_off, device=dev)
        T["tile_rep"] = torch.tensor(tile_rep, device=dev)
        T["grid_dim"] = torch.tensor(gdim.reshape(-1), device=dev)
        T["grid_lo"] = torch.tensor(glo.reshape(-1), device=dev)
        T["rep_id"] = torch.tensor([rp.rep_id for rp in self.replicas], dtype=torch.int32,
                                   device=dev)
        T["x"] = torch.tensor(xh, **f64)
        T["y"] = torch.tensor(yh, **f64)
        T["z"] = torch.tensor(zh, **f64)
        for k in ("vx", "vy", "vz", "z0", "x_ref", "y_ref", "z_ref"):
            T[k] = torch.zeros(N, **f64)
        T["flag"] = torch.tensor(fh, device=dev)
        self.permuted = any(t is not None for t in self.slot_tag)
        if gather is None:  # gather staging where a replica is in the blocked order
            gather = 1 if self.permuted else 0
        T["tag"] = torch.tensor(tagh if self.permuted else np.zeros(1, np.int32), device=dev)
        T["qpos"] = torch.zeros(4 * N, dtype=torch.int32, device=dev)
        T["cell_start"] = torch.zeros(self.C + R, dtype=torch.int32, device=dev)
        T["cell_atoms"] = torch.zeros(max(N, 1), dtype=torch.int32, device=dev)
        T["nl"] = torch.zeros(k_cap * N, dtype=torch.int32, device=dev)
        T["nl_lane"] = torch.zeros(k_cap * N if precision == "mixed" else 1, dtype=torch.int32,
                                   device=dev)
        T["nn"] = torch.zeros(N, dtype=torch.int32, device=dev)
        mixed = precision == "mixed"
        T["nact"] = torch.zeros(2 * N if mixed else 1, dtype=torch.int32, device=dev)
        for k in ("fx", "fy", "fz", "e_atom"):
            T[k] = torch.zeros(N, dtype=ft, device=dev)
        T["g"] = torch.zeros(N, **f64)
        T["rep_energy"] = torch.zeros(R, **f64)
        T["rep_wzz"] = torch.zeros(R, **f64)
        T["T"] = torch.tensor([rp.T for rp in self.replicas], **f64)
        T["v_pull"] = torch.tensor([rp.v_pull for rp in self.replicas], **f64)
        # dof, hard-sphere volume and grip faces: tbsma_replica_constants
        T["z_lo"] = torch.zeros(R, **f64)
        T["z_hi"] = torch.zeros(R, **f64)
        T["vol"] = torch.zeros(R, **f64)
        T["L0"] = torch.tensor(self.L0, **f64)
        seeds = np.array([rp.seed for rp in self.replicas], dtype=np.uint64).view(np.int64)
        T["seed"] = torch.tensor(seeds, device=dev)
        T["dof"] = torch.zeros(R, dtype=torch.int32, device=dev)
        T["step"] = torch.zeros(1, dtype=torch.int64, device=dev)
        T["obs"] = torch.zeros(n_slots * R * A.NOBS, **f64)
        T["status"] = torch.zeros(R, dtype=torch.int32, device=dev)
        T["dfail"] = torch.full((R,), -1.0, **f64)
        # target temperatures at the start of a ramp (scalar or per replica)
        t0 = np.broadcast_to(np.asarray(T_start if T_start is not None else
                                        [rp.T for rp in self.replicas], dtype=np.float64), (R,))
        T["T_start"] = torch.tensor(np.ascontiguousarray(t0), **f64)
        self.ramp_begin, self.ramp_steps = int(ramp_begin), int(ramp_steps)
        T["baro_s"] = torch.zeros(2 * R, **f64)
        T["nh_xi"] = torch.zeros(R, **f64)
        T["nh_eta"] = torch.zeros(R, **f64)
        # --- ABI structs -------------------------------------------------------------------
        self.prune = float(prune) if precision == "mixed" else 0.0
        self.params = A.Params(self.pot.A, self.pot.xi, self.pot.p, self.pot.q, self.pot.r0,
                               self.pot.r_tail, self.pot.r_cut, skin, cell, MASS_AU,
                               A.MIXED if precision == "mixed" else A.FP64, self.qbits,
                               self.prune, int(gather) if precision == "mixed" else 0,
                               int(bool(rebuild_exact)))
        self._rep_off_h = (C.c_int64 * (R + 1))(*self.rep_off.tolist())
        self._shape_h = None
        self._cell_off_h = (C.c_int64 * (R + 1))(*self.cell_off.tolist())
        self.sys = A.System(R, self.max_zbins, N, self.C,
                            C.cast(self._rep_off_h, C.c_void_p),
                            C.cast(self._cell_off_h, C.c_void_p),
                            *[_ptr(T[k]) for k in ("rep_off", "cell_off", "tile_rep", "grid_dim",
                                                   "grid_lo", "rep_id", "x", "y", "z", "vx",
                                                   "vy", "vz", "z0", "flag")],
                            _ptr(T["qpos"]) if precision == "mixed" else None,
                            _ptr(T["tag"]) if self.permuted else None)
        self.cells = A.Cells(_ptr(T["cell_start"]), _ptr(T["cell_atoms"]))
        # the per-atom pair counts are a diagnostic: the step loop runs
        # without them, count_pairs() asks for them
        self.nlist = A.NList(_ptr(T["nl"]), _ptr(T["nn"]), k_cap, 0, _ptr(T["x_ref"]),
                             _ptr(T["y_ref"]), _ptr(T["z_ref"]), None,
                             _ptr(T["nl_lane"]) if mixed else None)
        self.out = A.ForcesOut(_ptr(T["fx"]), _ptr(T["fy"]), _ptr(T["fz"]), _ptr(T["e_atom"]),
                               _ptr(T["g"]) if precision == "fp64" else None,
                               _ptr(T["rep_energy"]), _ptr(T["rep_wzz"]))
        self.md = A.MD(dt, gamma, lab_frame, n_log, n_slots, 0,
                       *[_ptr(T[k]) for k in ("T", "v_pull", "z_lo", "z_hi", "vol", "L0", "seed",
                                              "dof", "step", "obs", "status")], float(retire),
                       _ptr(T["dfail"]), self.nh_tau, _ptr(T["nh_xi"]), _ptr(T["nh_eta"]),
                       self.grip_step, self.grip_hold, _ptr(T["T_start"]), self.ramp_begin,
                       self.ramp_steps, self.baro_mass, self.baro_load, self.baro_damp,
                       _ptr(T["baro_s"]))
        self._attach_shapes()
        # the per-replica constants from the lattice sites (before any jitter)
        A.check(A.lib().tbsma_replica_constants(C.byref(self.params), C.byref(self.sys),
                                                _ptr(T["dof"]), _ptr(T["vol"]), _ptr(T["z_lo"]),
                                                _ptr(T["z_hi"]), self.stream()))
        torch.cuda.synchronize(dev)
        self.z_lo = T["z_lo"].cpu().numpy().copy()
        self.z_hi = T["z_hi"].cpu().numpy().copy()
        self.dof = T["dof"].cpu().numpy().copy()
        self.vol = T["vol"].cpu().numpy().copy()
        self._new_workspace()

    def _attach_shapes(self):
        if self.shapes is None:
            self._shape_h = None
            self.sys.shape_h = self.sys.shape = None
            return
        self._shape_h = (C.c_int32 * self.R)(*self.shapes)
        self.t["shape"] = torch.tensor(self.shapes, dtype=torch.int32, device=self.device)
        self.sys.shape_h = C.cast(self._shape_h, C.c_void_p)
        self.sys.shape = _ptr(self.t["shape"])

    def _new_workspace(self):
        nb = C.c_size_t()
        A.check(A.lib().tbsma_workspace_query(C.byref(self.params), C.byref(self.sys),
                                              C.byref(nb)))
        self.t["work"] = torch.zeros(int(nb.value), dtype=torch.uint8, device=self.device)
        self.work = _ptr(self.t["work"])
        A.check(A.lib().tbsma_workspace_init(C.byref(self.params), C.byref(self.sys), self.work,
                                             self.stream()))

    def set_shapes(self, shapes: Sequence[int] | None):
        """New launch shapes for the pair passes (one per replica, or None for
        the default) between calls: a fresh workspace for them, then lists and
        forces rebuilt at the current positions (the step index, positions and
        velocities carry on).  Shapes never change a result bit, but the
        rebuild at this step reorders list entries as any rebuild does."""
        if shapes is not None:
            shapes = [int(v) for v in shapes]
            if len(shapes) != self.R:
                raise ValueError("shapes needs one launch shape per replica")
        self.shapes = shapes
        self._attach_shapes()
        self._new_workspace()
        self.build_lists()
        self.compute_forces()

    # ------------------------------------------------------------------------------------
    def stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def init_state(self, jitter: float | None = None):
        """Jitter + Maxwell-Boltzmann velocities (tbsma_init_state)."""
        if jitter is None:
            js = {rp.jitter for rp in self.replicas}
            if len(js) != 1:
                raise ValueError("replicas disagree on the jitter amplitude")
            jitter = js.pop()
        A.check(A.lib().tbsma_init_state(C.byref(self.params), C.byref(self.sys),
                                         C.byref(self.md), self.work, float(jitter),
                                         self.stream()))

    def build_lists(self):
        """Cells and Verlet lists of every replica; grows k_cap on overflow."""
        lib = A.lib()
        A.check(lib.tbsma_build_cells(C.byref(self.params), C.byref(self.sys),
                                      C.byref(self.cells), self.work, self.stream()))
        need = C.c_int32()
        rc = lib.tbsma_neighbors(C.byref(self.params), C.byref(self.sys), C.byref(self.cells),
                                 C.byref(self.nlist), self.work, C.byref(need), self.stream())
        if rc == A.ECAPACITY:
            self.resize_nlist(int(need.value * 1.15) + 8)
            return self.build_lists()
        A.check(rc)

    def resize_nlist(self, k_cap: int):
        k_cap = (int(k_cap) + 7) // 8 * 8
        self.k_cap = k_cap
        self.t["nl"] = torch.zeros(k_cap * self.N, dtype=torch.int32, device=self.device)
        self.nlist.nl = _ptr(self.t["nl"])
        if self.precision == "mixed":
            self.t["nl_lane"] = torch.zeros(k_cap * self.N, dtype=torch.int32,
                                            device=self.device)
            self.nlist.nl_lane = _ptr(self.t["nl_lane"])
        self.nlist.k_cap = k_cap

    def compute_forces(self):
        A.check(A.lib().tbsma_forces(C.byref(self.params), C.byref(self.sys),
                                     C.byref(self.nlist), C.byref(self.out), self.work,
                                     self.stream()))

    def prepare(self, jitter: float | None = None):
        """Initial state, lists and forces: ready for step / run_batch."""
        self.init_state(jitter)
        self.build_lists()
        self.compute_forces()

    def step(self, n: int):
        """n plain steps (one launch per kernel per step)."""
        A.check(A.lib().tbsma_step(C.byref(self.params), C.byref(self.sys), C.byref(self.cells),
                                   C.byref(self.nlist), C.byref(self.out), C.byref(self.md),
                                   self.work, int(n), self.stream()))

    def run_batch(self, n: int, steps_per_graph: int = 50):
        """n steps replayed from a captured HIP graph.  The legacy default
        stream cannot be captured, so the call then runs on a side stream
        ordered after, and before, the caller's stream."""
        cur = torch.cuda.current_stream(self.device)
        side = None
        if cur.cuda_stream == 0:
            if not hasattr(self, "_side"):
                self._side = torch.cuda.Stream(self.device)
            side = self._side
            side.wait_stream(cur)
        s = C.c_void_p(side.cuda_stream) if side is not None else self.stream()
        try:
            A.check(A.lib().tbsma_run_batch(C.byref(self.params), C.byref(self.sys),
                                            C.byref(self.cells), C.byref(self.nlist),
                                            C.byref(self.out), C.byref(self.md), self.work,
                                            int(n), int(steps_per_graph), s))
        finally:
            if side is not None:
                cur.wait_stream(side)

    # ------------------------------------------------------------------------------------
    def _by_tag(self, a, r):
        """Per-slot values of replica r (first axis) in tag order."""
        perm = self.slot_tag[r]
        if perm is None:
            return a
        out = np.empty_like(a)
        out[perm] = a
        return out

    def _slice(self, key, r):
        o = int(self.rep_off[r])
        return self._by_tag(self.t[key][o:o + int(self.n_atoms[r])].detach().cpu().numpy(), r)

    def positions(self, r: int):
        return tuple(self._slice(k, r).astype(np.float64) for k in ("x", "y", "z"))

    def velocities(self, r: int):
        return tuple(self._slice(k, r).astype(np.float64) for k in ("vx", "vy", "vz"))

    def forces(self, r: int):
        return tuple(self._slice(k, r).astype(np.float64) for k in ("fx", "fy", "fz"))

    def energies(self, r: int):
        return self._slice("e_atom", r).astype(np.float64)

    def flags(self, r: int):
        return self._slice("flag", r)

    def neighbor_rows(self, r: int, sort: bool = True):
        """Neighbour tag arrays of replica r, by tag: sorted, or with
        sort=False in list order."""
        nn = self.t["nn"].cpu().numpy()
        # chunks of 8: entry k of slot i at ((k // 8) * N + i) * 8 + k % 8
        nl = self.t["nl"].view(self.k_cap // 8, self.N, 8).cpu().numpy()
        o = int(self.rep_off[r])
        perm = self.slot_tag[r]
        rows = []
        for i in range(int(self.n_atoms[r])):
            j = nl[:, o + i, :].reshape(-1)[:nn[o + i]] - o
            j = j if perm is None else perm[j]
            rows.append(np.sort(j) if sort else j)
        return rows if perm is None else [rows[s] for s in np.argsort(perm)]

    def count_pairs(self):
        """Runs a density pass at the current positions that also counts,
        per atom, the list entries with 0 < r <= r_tail and r_tail < r < r_cut
        (mixed precision only; g_i is rewritten with the same values)."""
        if self.precision != "mixed":
            raise ValueError("pair counts are kept in mixed precision only")
        nl = A.NList(self.nlist.nl, self.nlist.nn, self.nlist.k_cap, 0, self.nlist.x_ref,
                     self.nlist.y_ref, self.nlist.z_ref, _ptr(self.t["nact"]),
                     self.nlist.nl_lane)
        A.check(A.lib().tbsma_forces_pass(C.byref(self.params), C.byref(self.sys), C.byref(nl),
                                          C.byref(self.out), self.work, 1, self.stream()))
        torch.cuda.synchronize(self.device)

    def active_counts(self, r: int):
        """(core, tail) numbers of list entries within r_tail and within
        (r_tail, r_cut) per atom of replica r at the current positions
        (mixed precision only)."""
        self.count_pairs()
        na = self.t["nact"].view(self.N, 2).cpu().numpy()
        o = int(self.rep_off[r])
        return self._by_tag(na[o:o + int(self.n_atoms[r])].copy(), r)

    # ------------------------------------------------------------------------------------
    # checkpoint / resume: the device state that the next step reads.  With the
    # lists saved too, a resumed run repeats the original bit for bit (the
    # noise is keyed by the step index, which is part of the state).
    _STATE = ("x", "y", "z", "vx", "vy", "vz", "z0", "qpos", "nl", "nl_lane", "nn", "x_ref", "y_ref",
              "z_ref", "fx", "fy", "fz", "e_atom", "g", "step", "status", "dfail", "nh_xi",
              "nh_eta", "baro_s", "obs", "work")

    def state_dict(self):
        return {k: self.t[k].detach().cpu().numpy().copy() for k in self._STATE}

    def load_state_dict(self, st):
        for k in self._STATE:
            src = torch.from_numpy(np.ascontiguousarray(st[k]))
            if src.shape != self.t[k].shape:
                raise ValueError(f"checkpoint field {k} has shape {tuple(src.shape)}, "
                                 f"expected {tuple(self.t[k].shape)}")
            self.t[k].copy_(src.to(self.device))
        torch.cuda.synchronize(self.device)

    def save(self, path: str):
        np.savez(path, **self.state_dict())

    def load(self, path: str):
        with np.load(path, allow_pickle=False) as f:
            self.load_state_dict({k: f[k] for k in self._STATE})

    def status(self):
        return self.t["status"].cpu().numpy().view(np.uint32)

    _DYNAMICS = {"gamma": float, "nh_tau": float, "grip_step": float, "grip_hold": int,
                 "baro_mass": float, "baro_load": float, "baro_damp": float,
                 "ramp_begin": int, "ramp_steps": int, "retire": float}

    def set_dynamics(self, **kw):
        """Changes dynamics settings between calls (the protocol's phases):
        any of gamma, nh_tau, grip_step, grip_hold, baro_mass, baro_load,
        baro_damp, ramp_begin, ramp_steps, retire.  The library checks the
        combination at the next call."""
        for k, v in kw.items():
            if k not in self._DYNAMICS:
                raise ValueError(f"not a dynamics setting: {k}")
            v = self._DYNAMICS[k](v)
            setattr(self.md, k, v)
            setattr(self, k, v)
            self._kw[k] = v

    def rebase(self):
        """Makes the current state the start of a new stretch: grip
        references z0 = z, step index 0, initial lengths L0 grown by the
        barostat's elongation 2 s (which is then zeroed), status, rupture
        marks and records cleared.  Grips then rest where they are unless
        the settings move them (v_pull is zeroed)."""
        A.check(A.lib().tbsma_rebase(C.byref(self.params), C.byref(self.sys),
                                     _ptr(self.t["L0"]), _ptr(self.t["baro_s"]), self.stream()))
        self.t["v_pull"].zero_()
        self.t["step"].zero_()
        self.t["status"].zero_()
        self.t["dfail"].fill_(-1.0)
        self.t["obs"].zero_()
        torch.cuda.synchronize(self.device)
        self.L0 = self.t["L0"].cpu().numpy().copy()

    def compact(self, keep: Sequence[int] | None = None) -> "WireBatch | None":
        """A new batch of the replicas in `keep` (default: those not retired),
        in that order, or None when none is left.  Positions, velocities, grip
        references, the step index, status, rupture displacements and the
        observable ring carry over; cells, lists and forces are rebuilt from
        the carried positions.  Every replica evolves independently of the
        others, so a kept replica continues exactly as it would in this batch
        after a list rebuild and force evaluation (build_lists and
        compute_forces) at the same step."""
        if keep is None:
            st = self.status()
            keep = [r for r in range(self.R) if not st[r] & A.ST_DONE]
        keep = [int(r) for r in keep]
        if not keep:
            return None
        if min(keep) < 0 or max(keep) >= self.R or len(set(keep)) != len(keep):
            raise ValueError("keep must list distinct replica indices of this batch")
        nb = WireBatch([self.replicas[r] for r in keep], self.precision,
                       wires=[self.wires[r] for r in keep], qbits=self.qbits,
                       k_cap=self.k_cap,
                       shapes=None if self.shapes is None else [self.shapes[r] for r in keep],
                       **dict(self._kw, device=self.device,
                              T_start=self.t["T_start"].cpu().numpy()[keep]))
        for j, r in enumerate(keep):
            o, oj, n = int(self.rep_off[r]), int(nb.rep_off[j]), int(self.n_atoms[r])
            for k in ("x", "y", "z", "vx", "vy", "vz", "z0"):
                nb.t[k][oj:oj + n].copy_(self.t[k][o:o + n])
        idx = torch.tensor(keep, dtype=torch.int64, device=self.device)
        nb.t["step"].copy_(self.t["step"])
        nb.t["status"].copy_(self.t["status"][idx])
        nb.t["dfail"].copy_(self.t["dfail"][idx])
        nb.t["nh_xi"].copy_(self.t["nh_xi"][idx])
        nb.t["nh_eta"].copy_(self.t["nh_eta"][idx])
        nb.t["baro_s"].view(nb.R, 2).copy_(self.t["baro_s"].view(self.R, 2)[idx])
        for k in ("T", "T_start", "v_pull", "L0"):  # may differ from the replicas'
            nb.t[k].copy_(self.t[k][idx])
        ring = self.t["obs"].view(self.n_slots, self.R, A.NOBS)
        nb.t["obs"].view(nb.n_slots, nb.R, A.NOBS).copy_(ring[:, idx])
        nb.build_lists()
        nb.compute_forces()
        return nb

    def step_index(self) -> int:
        return int(self.t["step"].item())

    def obs(self):
        """Observable ring buffer as [n_slots, R, NOBS]."""
        return self.t["obs"].view(self.n_slots, self.R, A.NOBS).cpu().numpy()

    def obs_at(self, step: int):
        slot = (step // self.n_log) % self.n_slots
        return self.obs()[slot]

    def mean_neighbors(self) -> float:
        nn = self.t["nn"].double()
        return float(nn.sum().item() / max(1, int(self.n_atoms.sum())))

    def list_lengths(self):
        """(mean Verlet-list length, mean length of the lists the pair passes
        read) per real atom; they differ in mixed precision with pruning."""
        out = self._list_stats()
        n = max(1, int(self.n_atoms.sum()))
        return out[0] / n, out[1] / n

    def _list_stats(self):
        out = (C.c_int64 * 6)()
        A.check(A.lib().tbsma_list_stats(C.byref(self.params), C.byref(self.sys),
                                         C.byref(self.nlist), self.work, out, self.stream()))
        return list(out)

    def nbmap_blocks(self) -> int:
        """Blocks of the pair passes (up to tiles_per_block tiles of one
        replica, four by default)."""
        tiles = (self.rep_off[1:] - self.rep_off[:-1]) // A.TILE
        tpb = np.array([4] * self.R if self.shapes is None else [s & 15 for s in self.shapes])
        return int(((tiles + tpb - 1) // tpb).sum())

    def staging(self):
        """How the pair passes reach each block's neighbours (mixed):
        blocks whose window fits LDS, blocks staged by gather list, blocks
        gathering from global memory, and the mean gather-list length."""
        out = self._list_stats()
        return dict(window=out[2], gather=out[3], unstaged=out[4],
                    mean_gathered=out[5] / out[3] if out[3] else 0.0)

    def mean_active_pairs(self) -> float:
        """Mean number of pairs within r_cut per real atom at the current
        positions (mixed precision)."""
        if self.precision != "mixed":
            return float("nan")
        self.count_pairs()
        na = self.t["nact"].double()
        return float(na.sum().item() / max(1, int(self.n_atoms.sum())))
