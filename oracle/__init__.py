"""FP64 CPU oracle for TB-SMA nanowire MD (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
the two share no code: the arithmetic lives in ``tbsma_oracle.c`` (plain C,
FP64, OpenMP), which this module compiles with gcc and calls through ctypes.

Each wrapper names the passage of the paper (French et al., Probing the
Statistical Validity of the Ductile-to-Brittle Transition in Metallic
Nanowires using GPU Computing) that the C function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tbsma_oracle.c")
_LIB = os.path.join(_HERE, "libtbsma_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, -O2, OpenMP; no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
             "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Pot(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("A", "xi", "p", "q", "r0", "r_tail", "r_cut")]


class _MD(C.Structure):
    _fields_ = [("dt", C.c_double), ("gamma", C.c_double), ("T", C.c_double),
                ("v_pull", C.c_double), ("z_lo", C.c_double), ("z_hi", C.c_double),
                ("mass", C.c_double), ("seed", C.c_uint64), ("rep_id", C.c_uint32),
                ("lab_frame", C.c_int32), ("nh_tau", C.c_double), ("grip_step", C.c_double),
                ("grip_hold", C.c_int64), ("T_start", C.c_double), ("ramp_begin", C.c_int64),
                ("ramp_steps", C.c_int64), ("baro_mass", C.c_double), ("baro_load", C.c_double),
                ("baro_damp", C.c_double)]


@dataclass
class Pot:
    """TB-SMA parameters for Au (Table 1), with r0 read as a/sqrt(2)."""
    A: float = 0.2061
    xi: float = 1.790
    p: float = 10.229
    q: float = 4.036
    r0: float = 2.884
    r_tail: float = 6.5
    r_cut: float = 7.0

    def c(self) -> _Pot:
        return _Pot(self.A, self.xi, self.p, self.q, self.r0, self.r_tail, self.r_cut)


MASS_AU = 196.96657


@dataclass
class MD:
    """Integrator settings for one replica (Simulation details)."""
    dt: float = 0.002
    gamma: float = 1.0
    T: float = 10.0
    v_pull: float = 0.5
    z_lo: float = 0.0
    z_hi: float = 0.0
    mass: float = MASS_AU
    seed: int = 0
    rep_id: int = 0
    lab_frame: int = 0
    nh_tau: float = 0.0     # > 0: Nose-Hoover thermostat (gamma must be 0)
    grip_step: float = 0.0  # stepwise grips: displacement per side per hold (A)
    grip_hold: int = 0      # > 0: stepwise symmetric grips, steps per hold
    T_start: float = 0.0    # temperature ramp from T_start at step ramp_begin
    ramp_begin: int = 0     # to T at ramp_begin + ramp_steps (0: no ramp)
    ramp_steps: int = 0
    baro_mass: float = 0.0  # > 0: axial barostat on the grip separation (amu)
    baro_load: float = 0.0  # outward pull on each grip (eV/A)
    baro_damp: float = 0.0  # friction on the barostat coordinate (1/ps)

    def c(self) -> _MD:
        return _MD(self.dt, self.gamma, self.T, self.v_pull, self.z_lo, self.z_hi,
                   self.mass, self.seed, self.rep_id, self.lab_frame, self.nh_tau,
                   self.grip_step, self.grip_hold, self.T_start, self.ramp_begin,
                   self.ramp_steps, self.baro_mass, self.baro_load, self.baro_damp)


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        L.orc_const_kb.restype = C.c_double
        L.orc_const_acc.restype = C.c_double
        L.orc_const_eva3_gpa.restype = C.c_double
        L.orc_radial_eval.restype = C.c_double
        L.orc_radial_eval.argtypes = [C.POINTER(_Pot), C.c_int, C.c_double, C.POINTER(C.c_double)]
        L.orc_build_wire.restype = C.c_int64
        L.orc_build_wire.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                     C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_int64]
        L.orc_forces.restype = C.c_double
        L.orc_forces.argtypes = [C.POINTER(_Pot), C.c_int64, dp, dp, dp, C.c_int,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p]
        L.orc_forces_sampled.restype = None
        L.orc_forces_sampled.argtypes = [C.POINTER(_Pot), C.c_int64, dp, dp, dp, C.c_int64, i64p,
                                         dp, dp, dp, dp, dp]
        L.orc_count_pairs.restype = C.c_int64
        L.orc_count_pairs.argtypes = [C.c_int64, dp, dp, dp, C.c_double, i32p]
        L.orc_philox4x32_10.restype = None
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_uniform4.restype = None
        L.orc_uniform4.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32, dp]
        L.orc_gauss3.restype = None
        L.orc_gauss3.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32, dp]
        L.orc_init_state.restype = None
        L.orc_init_state.argtypes = [C.POINTER(_MD), C.c_int64, dp, dp, dp, dp, dp, dp, u8p,
                                     C.c_double]
        L.orc_run.restype = None
        L.orc_run.argtypes = [C.POINTER(_Pot), C.POINTER(_MD), C.c_int64, dp, dp, dp, dp, dp, dp,
                              dp, u8p, dp, dp, dp, C.c_void_p, C.c_int64, C.c_int64, C.c_int,
                              dp, dp, dp]
        L.orc_observe.restype = None
        L.orc_observe.argtypes = [C.POINTER(_Pot), C.POINTER(_MD), C.c_int64, dp, dp, dp, dp, dp,
                                  dp, u8p, C.c_int64, C.c_double, C.c_double, dp, dp]
        L.orc_target_temperature.restype = C.c_double
        L.orc_target_temperature.argtypes = [C.POINTER(_MD), C.c_double]
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


KB = None
ACC = None
EVA3_GPA = None


def constants():
    """(k_B in eV/K, 1 eV/(A amu) in A/ps^2, 1 eV/A^3 in GPa)."""
    L = lib()
    return L.orc_const_kb(), L.orc_const_acc(), L.orc_const_eva3_gpa()


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def radial(pot: Pot, kind: int, r: float):
    """phi (kind 0, eq 1 summand) or V (kind 1, eq 2 summand) with its tail:
    returns (f(r), f'(r))."""
    d = C.c_double()
    f = lib().orc_radial_eval(C.byref(pot.c()), kind, float(r), C.byref(d))
    return f, d.value


def build_wire(a: float, D: float, L: float, n_grip: int = 2, notch_layers: int = 0,
               notch_depth: float = 0.0):
    """[100] FCC cylinder of diameter D and length L (Simulation details,
    Figure 1), optionally with the ring notch of Figure 1's caption at its
    middle.  Returns x, y, z (float64) and flag (uint8: 0 dynamic,
    1 bottom grip, 2 top grip)."""
    n = lib().orc_build_wire(a, D, L, n_grip, notch_layers, notch_depth, None, None, None,
                             None, 0)
    x, y, z = (np.empty(n) for _ in range(3))
    flag = np.empty(n, dtype=np.uint8)
    lib().orc_build_wire(a, D, L, n_grip, notch_layers, notch_depth, x.ctypes.data,
                         y.ctypes.data, z.ctypes.data, flag.ctypes.data, n)
    return x, y, z, flag


def forces(pot: Pot, x, y, z, mode: int = 0):
    """Energies, forces and virial of eqs 1-3 (mode 0 brute force, 1 cell
    list).  Returns a dict with E, e_atom, fx, fy, fz, rho, w6."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    out = {k: np.zeros(n) for k in ("e_atom", "fx", "fy", "fz", "rho")}
    w6 = np.zeros(6)
    E = lib().orc_forces(C.byref(pot.c()), n, x, y, z, mode, out["rho"].ctypes.data,
                         out["e_atom"].ctypes.data, out["fx"].ctypes.data,
                         out["fy"].ctypes.data, out["fz"].ctypes.data, w6.ctypes.data)
    out["E"] = E
    out["w6"] = w6
    return out


def forces_sampled(pot: Pot, x, y, z, idx):
    """Forces, per-atom energies and densities of the atoms listed in idx
    only (same definitions as forces)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    m = idx.size
    fx, fy, fz, e, rho = (np.zeros(m) for _ in range(5))
    lib().orc_forces_sampled(C.byref(pot.c()), x.size, x, y, z, m, idx, fx, fy, fz, e, rho)
    return {"fx": fx, "fy": fy, "fz": fz, "e_atom": e, "rho": rho}


def count_pairs(x, y, z, rc: float):
    """Per-atom number of j != i with r_ij < rc (brute force)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    cnt = np.zeros(x.size, dtype=np.int32)
    lib().orc_count_pairs(x.size, x, y, z, rc, cnt)
    return cnt


def philox4x32_10(ctr, key):
    """Philox4x32-10 block function (Salmon et al., SC'11)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c, k, o)
    return o


def uniform4(seed, rep_id, tag, step, stream):
    u = np.zeros(4)
    lib().orc_uniform4(seed, rep_id, tag, step, stream, u)
    return u


def gauss3(seed, rep_id, tag, step, stream):
    g = np.zeros(3)
    lib().orc_gauss3(seed, rep_id, tag, step, stream, g)
    return g


class State:
    """Positions, velocities, forces and grip references of one replica."""

    def __init__(self, x, y, z, flag):
        self.x, self.y, self.z = _f64(x).copy(), _f64(y).copy(), _f64(z).copy()
        self.flag = np.ascontiguousarray(flag, dtype=np.uint8).copy()
        n = self.x.size
        self.vx, self.vy, self.vz = np.zeros(n), np.zeros(n), np.zeros(n)
        self.fx, self.fy, self.fz = np.zeros(n), np.zeros(n), np.zeros(n)
        self.e_atom = np.zeros(n)
        self.z0 = self.z.copy()
        self.step = 0
        self.zeta = np.zeros(1)   # Nose-Hoover friction (1/ps)
        self.eta = np.zeros(1)    # its time integral
        self.piston = np.zeros(2)  # barostat: grip travel s (A) and ds/dt

    def copy(self):
        s = State(self.x, self.y, self.z, self.flag)
        for k in ("vx", "vy", "vz", "fx", "fy", "fz", "e_atom", "z0", "zeta", "eta", "piston"):
            setattr(s, k, getattr(self, k).copy())
        s.step = self.step
        return s


def init_state(md: MD, st: State, jitter: float = 0.0):
    """Jitter, Maxwell-Boltzmann velocities (Simulation details); sets z0."""
    lib().orc_init_state(C.byref(md.c()), st.x.size, st.x, st.y, st.z, st.vx, st.vy, st.vz,
                         st.flag, jitter)
    st.z0 = st.z.copy()


def compute_forces(pot: Pot, st: State, mode: int = 0):
    r = forces(pot, st.x, st.y, st.z, mode)
    st.fx, st.fy, st.fz, st.e_atom = r["fx"], r["fy"], r["fz"], r["e_atom"]
    return r


def run(pot: Pot, md: MD, st: State, n_steps: int, mode: int = 0):
    """n_steps of velocity Verlet with grips and the Langevin (BAOAB) or
    Nose-Hoover thermostat, or none (orc_run)."""
    lib().orc_run(C.byref(pot.c()), C.byref(md.c()), st.x.size, st.x, st.y, st.z,
                  st.vx, st.vy, st.vz, st.z0, st.flag, st.fx, st.fy, st.fz,
                  st.e_atom.ctypes.data, st.step, n_steps, mode, st.zeta, st.eta, st.piston)
    st.step += n_steps


def observe(pot: Pot, md: MD, st: State, vol: float, L0: float):
    """E_pot, KE, T, -W_zz, sigma_zz (GPa), strain, max axial gap, D."""
    out = np.zeros(8)
    lib().orc_observe(C.byref(pot.c()), C.byref(md.c()), st.x.size, st.x, st.y, st.z,
                      st.vx, st.vy, st.vz, st.flag, st.step, vol, L0, st.piston, out)
    return out


def target_temperature(md: MD, t: float) -> float:
    """Target temperature at time t (in steps) of the thermostats (ramp)."""
    return lib().orc_target_temperature(C.byref(md.c()), float(t))


def num_threads() -> int:
    return lib().orc_num_threads()
