#!/usr/bin/env python3
"""Throughput of the TB-SMA nanowire-elongation step on one MI355X.

Workload (default): 512 independent Au [100] nanowires, diameter 3 nm,
lengths uniform in 5-40 nm (whole (002) layers), 298 K Langevin, dt = 2 fs,
top grips pulled at 0.5 A/ps; FP32 pair arithmetic, FP64 integration; all
replicas advanced together by a HIP graph of steps.  One step = integrator,
per-replica neighbour-list rebuilds where needed, density pass, force pass,
second half-kick and per-replica reductions.

Printed (one JSON line on stdout): batched atom-timesteps/s over the timed
steps, the same replicas run one per launch (plain path), the force kernel
against the HBM roofline (algorithmic bytes / average launch time measured
with HIP events on the launch stream), and the FP64 CPU oracle timed on a
bounded sample on this host's cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# unpacked VALU issue: 256 CUs x 1 wave64 instruction per cycle x 2.4 GHz
VALU_PEAK_IPS = 256 * 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def counter_record(kernel: str, workload: str):
    """The committed profiler counter record of `kernel` on `workload`
    (profiles/hbm_traffic.json), or None when there is none or the kernel
    source has changed since it was taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as f:
            recs = json.load(f)[kernel]
        with open(os.path.join(ROOT, "paper_1311_3890_amd", "csrc", "tbsma_kernels.hip"),
                  "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, KeyError, ValueError):
        return None
    for rec in recs:
        if rec.get("source_sha256") == sha and rec.get("workload") == workload:
            return rec
    return None


def counter_traffic(rec):
    """HBM bytes per launch from a counter record: FETCH_SIZE and WRITE_SIZE,
    each scaled by what it reads for a plain elementwise kernel of known
    size."""
    if rec is None:
        return None
    return (rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"]) * 1024.0


def valu_issue(rec, launch_s: float):
    """VALU issue of a launch: the wavefront VALU instructions the counter run
    recorded per launch, over the launch time measured here, against one
    unpacked wave64 instruction per CU per cycle (4 SIMDs of 16 lanes, a
    wave64 instruction every 4 cycles each) on 256 CUs at 2.4 GHz."""
    if rec is None or "valu_instr" not in rec:
        return None
    achieved = rec["valu_instr"] / launch_s
    return {"instr_per_launch": rec["valu_instr"], "achieved_instr_per_s": achieved,
            "peak_instr_per_s": VALU_PEAK_IPS, "frac": achieved / VALU_PEAK_IPS}


# The paper's Table 2: one unstretched wire per row, timesteps/s at 10 K and
# at 298 K on one GTX 680 in FP32 (atoms, 10 K, 298 K).
PAPER_TABLE2 = ((8823, 2536, 2286), (17673, 1723, 1507), (26523, 1311, 1141),
                (35373, 1045, 897), (44223, 881, 717), (53073, 758, 616),
                (61923, 655, 550), (70773, 584, 484), (79623, 514, 409),
                (88473, 470, 354), (97323, 427, 330), (106173, 396, 300))


def paper_table(steps: int, warmup: int, spg: int):
    """Single unstretched wires at the sizes of the paper's Table 2 with the
    settings of its benchmark (Simulation details, TB-SMA benchmarks):
    Nose-Hoover NVT at 10 K and 298 K, dt 2 fs, a hard cut at 5.8 A, a 0.29 A
    list buffer, atoms ordered along [100] (no blocked order at D 3 nm), FP32
    pair arithmetic, static grips.  Wires of D 3 nm and 100 k (002) layers
    hold 8850 k atoms, within 0.3 % of the table's rows.  Each wire runs
    alone: one replica per batch, `steps` timed steps of the graph loop after
    `warmup` untimed ones."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1311_3890_amd import _abi as A
    from paper_1311_3890_amd.engine import Potential, WireBatch
    pot = Potential(r_tail=5.8, r_cut=5.8)
    rows = []
    for k, (pa, p10, p298) in enumerate(PAPER_TABLE2, start=1):
        for T, pts in ((10.0, p10), (298.0, p298)):
            rp = W.Replica(30.0, W.snap_length(204.0 * k), T, 0.0, W.seed_of(k), k)
            b = WireBatch([rp], "mixed", skin=0.29, prune=0.0, gamma=0.0, nh_tau=0.1,
                          pot=pot, n_log=100)
            b.prepare()
            b.run_batch(warmup, spg)
            stream = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            b.run_batch(steps, spg)
            e1.record(stream)
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3
            n = int(b.n_atoms[0])
            bad = int(np.count_nonzero(b.status() & (A.ST_NONFINITE | A.ST_OVERFLOW)))
            rows.append({"atoms": n, "T_K": T, "timesteps_per_s": steps / sec,
                         "atom_timesteps_per_s": n * steps / sec, "paper_atoms": pa,
                         "paper_timesteps_per_s": pts,
                         "atom_timesteps_over_paper": (n * steps / sec) / (pa * pts),
                         "bad": bad})
            log(f"[bench] paper table: {rows[-1]}")
            del b
            torch.cuda.empty_cache()
    return {"steps": steps, "warmup": warmup, "potential": "hard cut 5.8 A",
            "skin_A": 0.29, "thermostat": "Nose-Hoover, tau 0.1 ps", "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="batch512-d3", choices=["d3-l20", "batch512-d3", "batch2048-mixed", "d10-l100"])
    ap.add_argument("--steps-per-graph", type=int, default=50,
                    help="steps per captured graph (clamped to --steps, so that every "
                         "timed step runs from a graph whenever it divides --steps)")
    ap.add_argument("--thermalize", type=int, default=3000,
                    help="untimed steps run in setup before the warmup, so that the "
                         "timed window starts from thermal positions with lists "
                         "rebuilt there (not from the perfect lattice); with the "
                         "batched workloads' 2.6 A skin the rebuild rate settles "
                         "after some 2000 steps")
    ap.add_argument("--per-replica", type=int, default=32,
                    help="replicas timed one per launch for the plain-path rate")
    ap.add_argument("--per-replica-steps", type=int, default=20)
    ap.add_argument("--pass-launches", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-replica", action="store_true")
    ap.add_argument("--no-protocols", action="store_true",
                    help="skip the timing of the paper's elongation and equilibration "
                         "protocols on the same replicas")
    ap.add_argument("--paper-table", action="store_true",
                    help="also time single wires at the sizes and settings of the paper's "
                         "Table 2 (12 sizes x 10 K, 298 K)")
    ap.add_argument("--paper-table-steps", type=int, default=1000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 512 MiB device copy (counter calibration)")
    ap.add_argument("--drift-steps", type=int, default=0,
                    help="also measure NVE energy drift over this many steps (D1.5xL3nm and "
                         "D3xL20nm wires at 10 K, static grips, FP64 and mixed)")
    ap.add_argument("--skin", type=float, default=None,
                    help="Verlet skin (A); default: the workload's")
    ap.add_argument("--prune", type=float, default=None,
                    help="pruning half-width (A); default: the workload's")
    ap.add_argument("--autotune", action="store_true",
                    help="choose the pair passes' launch shapes per bucket of replicas in "
                         "untimed trials on the whole batch before the timed window "
                         "(paper_1311_3890_amd.autotune); the line also reports the rate "
                         "with the default shapes")
    ap.add_argument("--autotune-cache", default=None, help="JSON cache of earlier choices")
    ap.add_argument("--oracle-workloads", action="store_true",
                    help="also time the oracle on the D1.5xL3nm, D3xL20nm and D10xL100nm wires")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(replica ensembles would shard by replica with no exchange); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import ctypes as C

    import numpy as np
    import torch

    import workloads as W
    from paper_1311_3890_amd import _abi as A
    from paper_1311_3890_amd.engine import WireBatch

    torch.cuda.set_device(0)
    wl = W.WORKLOADS[args.workload]()
    strain_max = 0.1 if args.workload == "d10-l100" else 0.5
    log(f"[bench] workload {wl.name}: building {len(wl.replicas)} replicas")
    skin = wl.skin if args.skin is None else args.skin
    prune = wl.prune if args.prune is None else args.prune
    b = WireBatch(wl.replicas, wl.precision, n_log=100, strain_max=strain_max,
                  skin=skin, prune=prune, gamma=wl.gamma, k_cap=wl.k_cap)
    b.prepare()
    n_real = int(b.n_atoms.sum())
    S = max(1, min(args.steps_per_graph, args.steps))
    log(f"[bench] {b.R} replicas, {n_real} atoms ({b.N} slots), qbits {b.qbits}; "
        f"thermalize {args.thermalize}, warmup {args.warmup}, {S} steps per graph")
    lib = A.lib()

    def events():
        out = (C.c_int64 * 2)()
        A.check(lib.tbsma_event_counts(C.byref(b.params), C.byref(b.sys), b.work, out,
                                       b.stream()))
        return out[0], out[1]

    if args.thermalize > 0:
        b.run_batch(args.thermalize, S)
    tuned = untuned_value = None
    if args.autotune:
        from paper_1311_3890_amd import autotune
        untuned_value = autotune.measure(b, args.steps, args.warmup, 1, S)
        log(f"[bench] default launch shapes: {untuned_value:.4e} atom-steps/s")
        tuned = autotune.tune(b, steps_per_graph=S, cache=args.autotune_cache, log=log)
    b.run_batch(args.warmup, S)
    torch.cuda.synchronize()
    ev_before = events()

    # ---- timed region: K steps of the batched graph path -----------------------------
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    b.run_batch(args.steps, S)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    value = n_real * args.steps / (ms * 1e-3)
    ev_after = events()
    window = {"graph_replays": args.steps // S, "eager_steps": args.steps % S,
              "replica_rebuilds": ev_after[0] - ev_before[0],
              "replica_prunings": ev_after[1] - ev_before[1],
              "first_step": b.step_index() - args.steps}
    log(f"[bench] batched: {args.steps} steps in {ms:.1f} ms -> {value:.4e} atom-steps/s; "
        f"window {window}")
    st = b.status()
    bad = int(np.count_nonzero(st & (A.ST_NONFINITE | A.ST_OVERFLOW)))

    # ---- per-kernel timing of the two force passes (HIP events, same stream) ----------
    kbar = b.mean_neighbors()

    def time_pass(p):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        A.check(lib.tbsma_forces_pass(C.byref(b.params), C.byref(b.sys), C.byref(b.nlist),
                                      C.byref(b.out), b.work, p, b.stream()))
        torch.cuda.synchronize()
        evs[0].record(stream)
        for _ in range(args.pass_launches):
            A.check(lib.tbsma_forces_pass(C.byref(b.params), C.byref(b.sys), C.byref(b.nlist),
                                          C.byref(b.out), b.work, p, b.stream()))
        evs[1].record(stream)
        torch.cuda.synchronize()
        return evs[0].elapsed_time(evs[1]) / args.pass_launches

    t_dens = time_pass(1)
    t_force_e = time_pass(2)  # force pass with energies (logged steps)
    t_force = time_pass(3)    # force pass as run on the other steps
    # a plain elementwise kernel that reads and writes 512 MiB each: its
    # measured bandwidth is the practical HBM ceiling the force pass is also
    # reported against, and (--copy-calibration) the HBM byte counters of a
    # profiler run are scaled by what they read for one launch of it
    src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    copy_gbs = None
    if args.copy_calibration:
        log(f"[bench] calibration kernel: {src.numel() * 8} bytes read and written")
    else:
        cst = torch.cuda.current_stream()
        ce = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ce[0].record(cst)
        for _ in range(10):
            torch.mul(src, 2.0, out=dst)
        ce[1].record(cst)
        torch.cuda.synchronize()
        copy_gbs = 2 * src.numel() * 8 / (ce[0].elapsed_time(ce[1]) / 10 * 1e-3) / 1e9
        log(f"[bench] plain elementwise kernel: {copy_gbs:.0f} GB/s")
    del src, dst
    # bytes each kernel must move per launch (per real atom), with kp the mean
    # length of the (pruned) lists the passes read:
    #  density: length 4 + row 4 kp + own position 16 + g 4
    #  force:   length 4 + row 4 kp + own position and g 16 + force 12
    #           (+ energy 4 on logged steps)
    # (neighbour positions are staged per block and counted once per atom in
    # the own-position term)
    kact = b.mean_active_pairs()
    kfull, kp = b.list_lengths()
    bytes_force = n_real * (4.0 * kp + 32.0)
    bytes_force_e = n_real * (4.0 * kp + 36.0)
    bytes_dens = n_real * (4.0 * kp + 24.0)
    gbs_force = bytes_force / (t_force * 1e-3) / 1e9
    gbs_force_e = bytes_force_e / (t_force_e * 1e-3) / 1e9
    gbs_dens = bytes_dens / (t_dens * 1e-3) / 1e9
    log(f"[bench] mean listed neighbours {kbar:.2f} (pruned lists {kp:.2f}), active pairs {kact:.2f}; density {t_dens * 1e3:.1f} us "
        f"({gbs_dens:.0f} GB/s), force {t_force * 1e3:.1f} us ({gbs_force:.0f} GB/s), "
        f"force with energies {t_force_e * 1e3:.1f} us")

    # ---- plain path: the same kind of replicas, one replica per launch ----------------
    pr = prg = None
    if not args.no_per_replica:
        idx = np.linspace(0, b.R - 1, min(args.per_replica, b.R)).round().astype(int)
        atoms_steps = 0.0
        t_tot = 0.0
        t_graph = 0.0
        for r in idx:
            s1 = WireBatch([wl.replicas[r]], wl.precision, n_log=100, strain_max=strain_max,
                           qbits=b.qbits, skin=wl.skin, gamma=wl.gamma, k_cap=wl.k_cap)
            s1.prepare()
            s1.step(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s1.step(args.per_replica_steps)
            torch.cuda.synchronize()
            t_tot += time.perf_counter() - t0
            s1.run_batch(args.per_replica_steps, args.per_replica_steps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s1.run_batch(args.per_replica_steps, args.per_replica_steps)
            torch.cuda.synchronize()
            t_graph += time.perf_counter() - t0
            atoms_steps += int(s1.n_atoms[0]) * args.per_replica_steps
            del s1
        pr = atoms_steps / t_tot
        prg = atoms_steps / t_graph
        log(f"[bench] one replica per launch ({len(idx)} replicas): {pr:.4e} atom-steps/s; "
            f"with a graph per replica {prg:.4e}; batched/plain = {value / pr:.1f}x")

    # ---- the paper's protocols on the same replicas -------------------------------------
    # (not the headline: the workload's thermostat is Langevin with continuous pulling)
    cfg = {"replicas": b.R, "skin_A": b.skin, "r_cut_A": b.pot.r_cut, "prune_A": b.prune}
    protocols = None
    if not args.no_protocols:
        del b
        torch.cuda.empty_cache()
        protocols = {}
        K2 = args.steps
        for name, kw in (
                ("elongation: Nose-Hoover (tau 0.1 ps), grips moved 0.05 A per 20 ps, "
                 "ring notch 3 planes x 4.08 A",
                 dict(gamma=0.0, nh_tau=0.1, grip_step=0.05, grip_hold=10000,
                      notch=(3, W.A_LAT))),
                ("equilibration: Nose-Hoover on a 0.01 K -> T ramp over 400 ps, axial "
                 "barostat on the grip separation (W 1e4 amu, 1/ps friction)",
                 dict(gamma=0.0, nh_tau=0.1, T_start=0.01, ramp_begin=0, ramp_steps=200000,
                      baro_mass=1.0e4, baro_damp=1.0))):
            pb = WireBatch(wl.replicas, wl.precision, n_log=100, strain_max=strain_max,
                           skin=skin, prune=prune, k_cap=wl.k_cap, **kw)
            pb.prepare()
            pb.run_batch(args.warmup, S)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            pb.run_batch(K2, S)
            e1.record(stream)
            torch.cuda.synchronize()
            pms = e0.elapsed_time(e1)
            pn = int(pb.n_atoms.sum())
            protocols[name] = {"atoms": pn, "steps": K2, "ms_per_step": pms / K2,
                               "atom_timesteps_per_s": pn * K2 / (pms * 1e-3),
                               "bad_replicas": int(np.count_nonzero(
                                   pb.status() & (A.ST_NONFINITE | A.ST_OVERFLOW)))}
            log(f"[bench] {name}: {protocols[name]}")
            del pb
            torch.cuda.empty_cache()

    # ---- CPU baseline: the FP64 oracle on a bounded sample, this host's cores ---------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        rp = wl.replicas[0]
        x, y, z, f = oracle.build_wire(W.A_LAT, rp.D, rp.L, rp.n_grip)
        stt = oracle.State(x, y, z, f)
        zlo = z[f == 1].max()
        zhi = z[f == 2].min()
        md = oracle.MD(dt=W.DT, gamma=wl.gamma, T=rp.T, v_pull=rp.v_pull, z_lo=zlo, z_hi=zhi,
                       seed=rp.seed, rep_id=rp.rep_id)
        pot = oracle.Pot()
        oracle.init_state(md, stt, rp.jitter)
        oracle.compute_forces(pot, stt, 1)
        t0 = time.perf_counter()
        oracle.run(pot, md, stt, 1, 1)
        t1 = time.perf_counter() - t0
        k = max(1, int(args.cpu_seconds / max(t1, 1e-6)))
        t0 = time.perf_counter()
        oracle.run(pot, md, stt, k, 1)
        tc = time.perf_counter() - t0
        cpu_model = None
        try:
            with open("/proc/cpuinfo") as fh:
                cpu_model = next((ln.split(":", 1)[1].strip() for ln in fh
                                  if ln.startswith("model name")), None)
        except OSError:
            pass
        cpu = {"value": x.size * k / tc, "unit": "atom-timesteps/s",
               "cores": oracle.num_threads(), "kind": "oracle", "cpu_model": cpu_model,
               "sample": f"replica 0 of the workload ({x.size} atoms, D {rp.D / 10:.1f} nm x "
                         f"L {rp.L / 10:.2f} nm), {k} FP64 steps, cell-list mode, OpenMP"}
        log(f"[bench] oracle: {cpu['value']:.4e} atom-steps/s on {cpu['cores']} threads")

    drift = None
    if args.drift_steps > 0:
        drift = {}
        for name, rp, prec in (("fp64 D1.5xL3nm", W.wire_d1p5_l3_fp64().replicas[0], "fp64"),
                               ("mixed D1.5xL3nm", W.wire_d1p5_l3_fp64().replicas[0], "mixed"),
                               ("fp64 D3xL20nm", W.wire_d3_l20_mixed().replicas[0], "fp64"),
                               ("mixed D3xL20nm", W.wire_d3_l20_mixed().replicas[0], "mixed")):
            rp = W.Replica(rp.D, rp.L, rp.T, 0.0, rp.seed, rp.rep_id, jitter=rp.jitter)
            n_log = max(1, args.drift_steps // 100)
            nb = WireBatch([rp], prec, n_log=n_log, n_slots=100, gamma=0.0)
            nb.prepare()
            nb.run_batch(args.drift_steps, n_log)
            torch.cuda.synchronize()
            ob = nb.obs()[:, 0, :]
            ob = ob[np.argsort(ob[:, A.OBS_STEP])]
            t_ps = ob[:, A.OBS_STEP] * nb.dt
            etot = ob[:, A.OBS_EPOT] + ob[:, A.OBS_KE]
            na = int(nb.n_atoms[0])
            slope = np.polyfit(t_ps, etot, 1)[0]  # eV/ps
            drift[name] = {"steps": args.drift_steps, "atoms": na,
                           "drift_meV_per_atom_per_ns": slope * 1e3 * 1e3 / na,
                           "rms_fluct_meV_per_atom": float(np.std(etot)) * 1e3 / na,
                           "T_mean_K": float(ob[:, A.OBS_T].mean())}
            log(f"[bench] NVE {name}: {drift[name]}")

    oracle_other = None
    if args.oracle_workloads and not args.no_cpu_baseline:
        import oracle
        oracle_other = {}
        for name, w in (("D1.5xL3nm", W.wire_d1p5_l3_fp64()), ("D3xL20nm", W.wire_d3_l20_mixed()),
                        ("D10xL100nm", W.wire_d10_l100())):
            rp = w.replicas[0]
            x, y, z, f = oracle.build_wire(W.A_LAT, rp.D, rp.L, rp.n_grip)
            stt = oracle.State(x, y, z, f)
            md = oracle.MD(dt=W.DT, gamma=w.gamma, T=rp.T, v_pull=rp.v_pull,
                           z_lo=z[f == 1].max(), z_hi=z[f == 2].min(), seed=rp.seed,
                           rep_id=rp.rep_id)
            pot = oracle.Pot()
            oracle.init_state(md, stt, rp.jitter)
            oracle.compute_forces(pot, stt, 1)
            t0 = time.perf_counter()
            oracle.run(pot, md, stt, 1, 1)
            t1 = time.perf_counter() - t0
            k = max(1, int(args.cpu_seconds / 3 / max(t1, 1e-6)))
            t0 = time.perf_counter()
            oracle.run(pot, md, stt, k, 1)
            tc = time.perf_counter() - t0
            oracle_other[name] = {"atoms": int(x.size), "steps": k,
                                  "atom_timesteps_per_s": x.size * k / tc,
                                  "cores": oracle.num_threads()}
            log(f"[bench] oracle {name}: {oracle_other[name]}")

    force_rec = counter_record("k_force_mixed", wl.name)
    line = {
        "metric": "atom-timesteps/s, batched vs per-replica TB-SMA NVT; force-kernel % HBM peak",
        "value": value,
        "unit": "atom-timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "replicas": cfg["replicas"], "atoms": n_real,
                   "precision": "f32 pair math, f64 integration and sums",
                   "steps_per_graph": S, "skin_A": cfg["skin_A"], "r_cut_A": cfg["r_cut_A"],
                   "prune_A": cfg["prune_A"],
                   "thermalized_steps": args.thermalize,
                   "launch_shapes": tuned["names"] if tuned else "default (4 tiles/block, "
                                                                  "stage 1536)",
                   "parallelism": "replica batch, 1 GPU"},
        "window": window,
        "roofline": {"bound": "hbm", "achieved": gbs_force, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": gbs_force / HBM_PEAK_GBS,
                     "traffic": counter_traffic(force_rec),
                     # counter-measured HBM bytes per launch over the launch time,
                     # against the same 8 TB/s
                     "traffic_frac": (counter_traffic(force_rec) / (t_force * 1e-3) / 1e9
                                      / HBM_PEAK_GBS if force_rec else None),
                     "valu_issue": valu_issue(force_rec, t_force * 1e-3),
                     "copy_kernel_GBs": copy_gbs,
                     "frac_of_copy": gbs_force / copy_gbs if copy_gbs else None,
                     "traffic_frac_of_copy": (counter_traffic(force_rec) / (t_force * 1e-3) / 1e9
                                              / copy_gbs if copy_gbs and force_rec else None),
                     "kernel": "k_force_mixed",
                     "algorithmic_bytes_per_launch": bytes_force,
                     "avg_launch_us": t_force * 1e3,
                     "mean_listed_neighbours": kbar,
                     "mean_pruned_list": kp,
                     "mean_active_pairs": kact},
        "kernels": {"density": {"avg_launch_us": t_dens * 1e3, "GB/s": gbs_dens,
                                "frac": gbs_dens / HBM_PEAK_GBS},
                    "force_with_energies": {"avg_launch_us": t_force_e * 1e3,
                                            "GB/s": gbs_force_e,
                                            "frac": gbs_force_e / HBM_PEAK_GBS},
                    # both passes of a step: (8 kbar + 56) bytes per atom
                    "density_plus_force": {
                        "avg_us": (t_dens + t_force) * 1e3,
                        "GB/s": (bytes_dens + bytes_force) / ((t_dens + t_force) * 1e-3) / 1e9,
                        "frac": (bytes_dens + bytes_force) / ((t_dens + t_force) * 1e-3) / 1e9
                        / HBM_PEAK_GBS}},
        "per_replica_value": pr,
        "per_replica_graph_value": prg,
        "batched_over_per_replica": (value / pr) if pr else None,
        "bad_replicas": bad,
        "cpu_baseline": cpu,
    }
    if args.paper_table:
        line["paper_table"] = paper_table(args.paper_table_steps, 200, 50)
    if untuned_value is not None:
        line["untuned_value"] = untuned_value
    if protocols is not None:
        line["protocols"] = protocols
    if drift is not None:
        line["nve_drift"] = drift
    if oracle_other is not None:
        line["oracle_other_workloads"] = oracle_other
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
