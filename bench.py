"""Throughput of the DMTS-NC hot path on one MI355X.

Default workload: 4,096 rigid-geometry waters (12,288 atoms) in a 49.6 A
periodic box, conservative model 3 layers x 128 (FP32), distilled NC model
1 x 32 (FP32), DMTS-NC with a 4 fs outer step and 8 inner steps of 0.5 fs,
Langevin 300 K, gamma 1 ps^-1.  One "step" is one outer step of Algorithm 1:
neighbour maintenance, 8 NC force evaluations with 8 BAOA half-steps and
kicks, one conservative energy + hand-written-reverse force evaluation and
the outer kicks.

Prints one JSON line.  `value` is DMTS-NC ns/day with all inputs resident
in HBM, outer steps replayed from the recorded graph (the production
configuration).  Beside it, on the same system: single time stepping
(BAOAB 0.5 fs, conservative model alone), DMTS-NC with BF16 perceptrons,
and DMTS-NC with the rewind procedure armed (never tripping); each path's
force relative RMSE against the FP64 oracle.  `roofline` covers the dominant
kernel (the conservative message reverse) with its average launch duration
from HIP events on its own stream over a further timed region of the same
run in which only that kernel's launches are timed (launch timers on, so
outer steps are launched directly there); `kernels` lists the other message
kernels, the NC evaluation and the dense products the same way, a region
per group of launch sites.  `chain` is the
solvated-chain workload (BF16, HMR + HHF, 10 fs x 10), `serving` the
256-replica continuous-batching workload at 0.8 of the measured saturated
rate, and `cpu_baseline` the FP64 oracle timed on the host (all cores and
one thread) on a bounded sample.
"""

import argparse
import ctypes as C
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ns/day DMTS-NC vs 1-step at force RMSE vs FP64; p50/p99 replica step latency"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3


_T0 = time.perf_counter()


def _progress(msg):
    """One line per finished leg on stderr (stdout carries only the JSON line)."""
    print(f"bench [{time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def _ns_per_day(dt_fs, steps, seconds):
    return dt_fs * steps / seconds * 86400.0 * 1e-6


def message_counts(F, K, n_atoms, n_edges, reverse):
    """Algorithmic work of one conservative message launch (one layer), the
    counts the roofline uses: the per-edge radial filter (K -> 3F) is a
    dense contraction of 6KF flops per edge in the forward and twice that in
    the reverse (the filter and its radial derivative); the compulsory HBM
    traffic is 8F (forward) or 12F (reverse) float32 values per atom (the
    features and adjoints in and out) plus one 4-byte neighbour index per
    edge."""
    flops = (12 if reverse else 6) * K * F * n_edges
    nbytes = (12 if reverse else 8) * F * 4 * n_atoms + 4 * n_edges
    return flops, nbytes


# launch-timer groups, one timed region each: a site's launches are timed
# while the other launches of the step run untimed, so that the host keeps
# ahead of the device as in production (the dominant kernel alone first)
TIMER_GROUPS = (("message_bwd",), ("message_fwd",), ("message_fwd_first", "message_bwd_first"),
                ("nc_message_fwd", "nc_update", "head_fwd", "baoa"), ("gemm",))


def run_gpu(args):
    import torch

    import synth
    from paper_2602_14975_amd import _abi, nnp

    torch.cuda.set_device(0)
    s = synth.water_config(1)
    cw = synth.random_weights(synth.CONS_CFG1, 2001)
    nw = synth.random_weights(synth.NC_CFG1, 3001)
    models = {p: (nnp.Model.from_spec(synth.CONS_CFG1, cw, precision=p),
                  nnp.Model.from_spec(synth.NC_CFG1, nw, precision=p)) for p in (_abi.NNP_FP32, _abi.NNP_BF16)}
    m = s.standard_masses()
    gamma = np.ones(s.n)
    v0 = synth.maxwell_boltzmann(m, 300.0, 5001)
    lib = nnp.lib()

    def forces_at(pos, prec):
        cons, nc = models[prec]
        system = nnp.DeviceSystem(pos, s.species, s.box)
        nl = nnp.NeighborList(system.n, 5.0, 900000)
        ws = nnp.workspace(cons, nc, system.n, 1, nl.capacity)
        nnp.nnp_neighbors(system, nl, ws)
        e, fc = nnp.nnp_cons_energy_forces(cons, system, nl, ws)
        fn = nnp.nnp_nc_forces(nc, system, nl, ws)
        return (float(e.cpu()[0]), fc.cpu().numpy().T.astype(np.float64), fn.cpu().numpy().T.astype(np.float64),
                int(nl.n_edges))

    def timed(prec, mode, dt, n_inner, steps, warmup, sites=(), **kw):
        cons, nc = models[prec]
        system = nnp.DeviceSystem(s.pos, s.species, s.box)
        prm = nnp.respa_params(dt, n_inner, 300.0, seed=4001, mode=mode, skin=args.skin,
                               check_every=kw.pop("check_every", args.check_every), **kw)
        traj = nnp.Trajectory(cons, nc if mode == "dmts_nc" else None, system, v0, m, gamma, prm)
        traj.respa_step(max(1, warmup))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        traj.respa_step(steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        kt = {}
        for group in sites:
            # further timed regions of the same trajectory, one per group of
            # launch sites: every launch of a site in the group is bracketed
            # by HIP events on its own stream (outer steps are then launched
            # directly, not replayed)
            tot, cnt = C.c_double(), C.c_int64()
            for site in group:
                lib.nnp_timer_enable(site.encode(), 1)
                lib.nnp_timer_read(site.encode(), C.byref(tot), C.byref(cnt), 1)
            t0 = time.perf_counter()
            traj.respa_step(args.kernel_steps)
            torch.cuda.synchronize()
            kt.setdefault("region_ms_per_step", []).append((time.perf_counter() - t0) / args.kernel_steps * 1e3)
            for site in group:
                lib.nnp_timer_read(site.encode(), C.byref(tot), C.byref(cnt), 1)
                lib.nnp_timer_enable(site.encode(), 0)
                kt[site] = (tot.value, cnt.value)
        return t, traj, kt

    fp32, bf16 = _abi.NNP_FP32, _abi.NNP_BF16
    start = {fp32: forces_at(s.pos, fp32), bf16: forces_at(s.pos, bf16)}
    _progress("start-frame forces (fp32, bf16) done")
    t_dmts, traj, kt = timed(fp32, "dmts_nc", 4.0, 8, args.steps, args.warmup, sites=TIMER_GROUPS)
    _progress(f"fp32 DMTS-NC: {t_dmts / args.steps * 1e3:.3f} ms per outer step")
    x_end = traj.positions()
    end = forces_at(x_end, fp32)
    v_end = traj.velocities()
    kb = 8.31446261815324 / 4184.0  # kcal/mol/K
    ke_end = 0.5 * float((m[:, None] * v_end * v_end).sum()) / 4.184e-4  # amu A^2/fs^2 -> kcal/mol
    t_end = 2.0 * ke_end / (3 * s.n * kb)
    rebuilds = traj.n_rebuilds
    del traj
    t_bf16, _, _ = timed(bf16, "dmts_nc", 4.0, 8, args.steps, args.warmup)
    _progress(f"bf16 DMTS-NC: {t_bf16 / args.steps * 1e3:.3f} ms per outer step")
    t_rewind, tr, _ = timed(fp32, "dmts_nc", 4.0, 8, args.steps, args.warmup, rewind_threshold=1.0e6,
                            save_every=args.check_every, sts_after_rewind=8)
    rewinds = tr.n_rewinds
    _progress(f"rewind-armed DMTS-NC: {t_rewind / args.steps * 1e3:.3f} ms per outer step")
    del tr
    sts_steps = max(8, args.steps)
    t_sts, _, _ = timed(fp32, "sts", 0.5, 1, sts_steps, args.warmup)
    _progress(f"fp32 STS 0.5 fs: {t_sts / sts_steps * 1e3:.3f} ms per step")
    return {
        "t_dmts": t_dmts, "t_bf16": t_bf16, "t_rewind": t_rewind, "rewinds": rewinds, "t_sts": t_sts,
        "sts_steps": sts_steps, "kernel_timer": kt, "n_edges5": start[fp32][3], "rebuilds": rebuilds,
        "start": start, "end": end, "system": s, "cw": cw, "nw": nw, "t_end": t_end, "x_end": x_end,
        "gpu_name": torch.cuda.get_device_name(0),
    }


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_oracle(s, cw, nw, pos=None, threads=None):
    """FP64 oracle on the host: one conservative and one NC evaluation (at
    the starting configuration, or at `pos`), on `threads` threads (all the
    process may use when None)."""
    import torch

    import synth
    from oracle import models as om
    from oracle import neighbors as onb

    x = s.pos if pos is None else pos
    before = torch.get_num_threads()
    if threads is not None:
        torch.set_num_threads(threads)
    used = torch.get_num_threads()
    try:
        t0 = time.perf_counter()
        off5, nbr5 = onb.pairs_cell_list(x, s.box, 5.0)
        t_nb = time.perf_counter() - t0
        t0 = time.perf_counter()
        E, F = om.cons_energy_forces(synth.CONS_CFG1, cw, x, s.species, s.box, off5, nbr5)
        t_cons = time.perf_counter() - t0
        off35, nbr35 = onb.pairs_bruteforce(x, s.box, 3.5)
        t0 = time.perf_counter()
        Fn = om.nc_forces(synth.NC_CFG1, nw, x, s.species, s.box, off35, nbr35)
        t_nc = time.perf_counter() - t0
    finally:
        torch.set_num_threads(before)
    return {"E": E, "F": F, "Fn": Fn, "t_cons": t_cons, "t_nc": t_nc, "t_nb": t_nb, "threads": used}


def measured_traffic():
    """HBM bytes per message_bwd launch from the committed counter summary
    (two rocprofv3 --pmc passes, calibrated on a plain copy), or None when
    the kernel sources changed after the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "message_bwd_mx_water12288_traffic.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    keys = ("traffic_bytes_per_launch", "sources", "sources_sha256")
    fields = dict(line.strip().split(": ", 1) for line in text.splitlines()
                  if ": " in line and line.strip().split(": ", 1)[0] in keys)
    if len(fields) != 3:
        return None
    h = hashlib.sha256()
    for f in fields["sources"].split():
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return int(fields["traffic_bytes_per_launch"]) if h.hexdigest() == fields["sources_sha256"] else None


def run_serving(n_replicas=256, n_steps=500, load=0.8, budget_frac=0.04, seed=30000, max_slots=256,
                sat_steps=100, steps_per_call=2):
    """Continuous batching of replicas of 300-6,000 atoms (30% with a chain),
    DMTS-NC 4 fs x 8 with BF16 perceptrons.  The HBM budget is budget_frac of
    the summed footprints of all replicas (about ten replicas of the mean
    size: throughput stops growing with the resident atoms beyond about
    12,000, so at 0.8 load a larger budget would never bind).  The
    saturated rate is measured first, closed loop: every replica submitted
    at once with sat_steps outer steps, the same budget, atom-steps per
    second while some still wait for admission; Poisson arrivals then come
    at `load` times that rate expressed in replicas of the mix's mean size
    running n_steps outer steps."""
    import torch

    import synth
    from paper_2602_14975_amd import _abi, nnp, serve

    reps = synth.replica_mix(n_replicas=n_replicas)
    cons = nnp.Model.from_spec(synth.CONS_CFG1, synth.random_weights(synth.CONS_CFG1, 2004), precision=_abi.NNP_BF16)
    nc = nnp.Model.from_spec(synth.NC_CFG1, synth.random_weights(synth.NC_CFG1, 3004), precision=_abi.NNP_BF16)
    prm = nnp.respa_params(4.0, 8, 300.0, seed=4004, skin=1.0)
    probe = serve.Server(cons, nc, prm, 64 << 20, 1)
    sizes = [probe.replica_bytes(r.n, r.box) for r in reps]
    probe.close()
    budget = max(int(budget_frac * sum(sizes)), 2 * max(sizes))
    srv = serve.Server(cons, nc, prm, budget, max_slots)
    torch.cuda.synchronize()
    _progress(f"serving: budget {budget >> 20} MiB of {int(sum(sizes)) >> 20} MiB total footprint")
    sat_atom_steps, sat_wall = serve.saturated_rate(srv, reps, sat_steps, steps_per_call=4, vel_seed_base=7000)
    srv.close()
    mean_atoms = float(np.mean([r.n for r in reps]))
    sat_rate = sat_atom_steps / (mean_atoms * n_steps)
    rate = load * sat_rate
    arrivals = synth.systems.poisson_arrivals(n_replicas, rate, seed)
    srv = serve.Server(cons, nc, prm, budget, max_slots)
    torch.cuda.synchronize()
    _progress(f"serving: saturated {sat_atom_steps:.3g} atom-steps/s; arrivals at {rate:.3f}/s")
    rep = serve.run(srv, reps, arrivals, n_steps, 4.0, steps_per_call=steps_per_call, log=_progress)
    srv.close()
    rep.update({"steps_per_replica": n_steps, "saturated_atom_steps_per_s": round(sat_atom_steps, 1),
                "saturated_sample": (f"{n_replicas} replicas x {sat_steps} outer steps submitted at once, measured "
                                     f"while the queue was not empty ({sat_wall:.1f} s)"),
                "saturated_rate_per_s": round(sat_rate, 4), "load": load, "arrival_rate_per_s": round(rate, 4),
                "hbm_budget_MiB": budget >> 20, "budget_frac_of_total": budget_frac,
                "footprint_total_MiB": int(sum(sizes)) >> 20, "max_slots": max_slots,
                "atoms_total": int(sum(r.n for r in reps)), "steps_per_progress_call": steps_per_call,
                "latency_clock": "device wall clock, per replica between consecutive outer-step completions",
                "precision": "bf16 perceptrons, fp32 edge filter and forces, fp64 integration"})
    for k in ("latency_p50_ms", "latency_p99_ms", "aggregate_ns_per_day", "wall_s", "queue_delay_mean_s",
              "queue_delay_p99_s", "resident_mean"):
        rep[k] = round(rep[k], 4)
    return rep


def run_chain(args):
    """Solvated 600-heavy-atom chain + 30,000 waters (~92k atoms), HMR (H set
    to 3 amu) and high hydrogen friction (100 ps^-1 on H, 1 elsewhere),
    DMTS-NC 10 fs x 10, BF16 perceptrons.  Also reports the BF16-vs-FP32
    force error at the starting configuration."""
    import torch

    import synth
    from paper_2602_14975_amd import _abi, nnp

    s = synth.solvated_chain(600, 30000, seed=1002)
    cw = synth.random_weights(synth.CONS_CFG1, 2002)
    nw = synth.random_weights(synth.NC_CFG1, 3002)
    out = {}
    forces = {}
    for prec in (_abi.NNP_FP32, _abi.NNP_BF16):
        cons = nnp.Model.from_spec(synth.CONS_CFG1, cw, precision=prec)
        nc = nnp.Model.from_spec(synth.NC_CFG1, nw, precision=prec)
        system = nnp.DeviceSystem(s.pos, s.species, s.box)
        nl = nnp.NeighborList(system.n, 5.0, int(system.n * 60))
        ws = nnp.workspace(cons, nc, system.n, 1, nl.capacity)
        nnp.nnp_neighbors(system, nl, ws)
        _, fc = nnp.nnp_cons_energy_forces(cons, system, nl, ws)
        fn = nnp.nnp_nc_forces(nc, system, nl, ws)
        forces[prec] = (fc.double(), fn.double())
    rel = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    out["bf16_vs_fp32_force_rel_rmse"] = {"cons": rel(forces[1][0], forces[0][0]),
                                          "nc": rel(forces[1][1], forces[0][1])}
    m = nnp.nnp_hmr_masses(s.bonded_heavy, s.standard_masses(), 3.0, "set")
    gamma = np.where(s.species == 0, 100.0, 1.0)
    v0 = synth.maxwell_boltzmann(m, 300.0, 5002)
    cons = nnp.Model.from_spec(synth.CONS_CFG1, cw, precision=_abi.NNP_BF16)
    nc = nnp.Model.from_spec(synth.NC_CFG1, nw, precision=_abi.NNP_BF16)
    system = nnp.DeviceSystem(s.pos, s.species, s.box)
    prm = nnp.respa_params(10.0, 10, 300.0, seed=4002, skin=1.0, check_every=args.check_every)
    traj = nnp.Trajectory(cons, nc, system, v0, m, gamma, prm)
    traj.respa_step(max(1, args.warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ke = torch.zeros(args.steps, 1, dtype=torch.float64, device="cuda")
    traj.respa_step(args.steps, ke)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    T = 2 * ke.cpu().numpy()[:, 0] / (3 * s.n * 8.31446261815324 / 4184.0)
    out.update({"atoms": int(s.n), "box_A": round(s.box, 3), "ns_per_day": round(_ns_per_day(10.0, args.steps, t), 3),
                "ms_per_step": round(t / args.steps * 1e3, 3), "temperature_mean_K": round(float(T.mean()), 2),
                "list_rebuilds": traj.n_rebuilds})
    return out


def run_copy(mib=512, reps=5):
    """A plain device copy of known size (torch's copy kernel), the
    calibration point for the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    return {"bytes_read_per_copy": src.numel() * 4, "bytes_written_per_copy": src.numel() * 4,
            "copies": reps, "GBps": round(2 * src.numel() * 4 / t / 1e9, 1)}


def run_distill(args):
    """Distillation of the NC model (1 x 32) onto the conservative model
    (3 x 128) on the 1,536-atom box: 2,000 frames from a 0.5 fs NVT run
    in 20 independent runs (0.1 ps equilibration each, then one frame per
    5 fs), 1,800 training / 200 validation frames, batch 16, FP32 Adam
    lr 1e-3.  The randomly initialised teacher heats up beyond a few ps, so
    the frames come from several short runs."""
    import torch

    import synth
    from paper_2602_14975_amd import distill, nnp

    s = synth.water_config(3)
    cons = nnp.Model.from_spec(synth.CONS_CFG1, synth.random_weights(synth.CONS_CFG1, 2003))
    nw = synth.random_weights(synth.NC_CFG1, 3003)
    nc = nnp.Model.from_spec(synth.NC_CFG1, nw)
    t0 = time.perf_counter()
    pos, frc = distill.generate_frames(cons, s, s.standard_masses(), np.ones(s.n), n_frames=args.frames,
                                       equil_steps=200, every=10, n_traj=20)
    torch.cuda.synchronize()
    t_frames = time.perf_counter() - t0
    t0 = time.perf_counter()
    d, hist = distill.train(nc, nw, pos, frc, s.species, s.box, s.n, steps=args.train_steps,
                            n_val=max(1, args.frames // 10), batch=16, lr=1e-3, log_every=max(1, args.train_steps // 20))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    fref = frc.double()
    label_rms = float(torch.sqrt((fref * fref).mean()))
    label_max = float(fref.abs().max())
    return {"frames": args.frames, "frame_generation_s": round(t_frames, 2), "train_steps": args.train_steps,
            "train_s": round(t_train, 2), "ms_per_train_step": round(t_train / args.train_steps * 1e3, 3),
            "label_force_rms": round(label_rms, 4), "label_force_max": round(label_max, 3),
            "val_force_rmse_history": [(int(k), round(v, 5)) for k, v in hist]}


def run_diffusion(args):
    """Self-diffusion of water oxygens under DMTS-NC (4 fs x 8) with a
    Langevin thermostat at gamma = 1 and 10 ps^-1 and with fast-forward
    Langevin at 10 ps^-1 (the paper's thermostat comparison), on the 1,536-atom
    box: 4 independent runs per case, 0.1 ps equilibration, then positions and
    velocities every outer step for 0.8 ps; D from the MSD slope over
    0.1-0.4 ps and from the velocity autocorrelation integrated to 0.2 ps.
    The models are randomly initialised, so only the comparison between
    thermostats carries meaning."""
    import torch

    import synth
    from paper_2602_14975_amd import nnp, observables as ob

    s = synth.water_config(3)
    cons = nnp.Model.from_spec(synth.CONS_CFG1, synth.random_weights(synth.CONS_CFG1, 2003))
    nc = nnp.Model.from_spec(synth.NC_CFG1, synth.random_weights(synth.NC_CFG1, 3003))
    m = s.standard_masses()
    oxy = s.species == 3
    dt_outer, n_runs, n_equil, n_samples = 4.0, 4, 25, 200
    out = {}
    t0 = time.perf_counter()
    for thermo, gamma in (("langevin", 1.0), ("langevin", 10.0), ("ffl", 10.0)):
        xs, vs = [], []
        for run in range(n_runs):
            system = nnp.DeviceSystem(s.pos, s.species, s.box)
            v0 = synth.maxwell_boltzmann(m, 300.0, 5003 + run)
            prm = nnp.respa_params(dt_outer, 8, 300.0, seed=4003 + run, thermostat=thermo, skin=1.0, check_every=10)
            traj = nnp.Trajectory(cons, nc, system, v0, m, np.full(s.n, gamma), prm)
            traj.respa_step(n_equil)
            x, v = [], []
            for _ in range(n_samples):
                traj.respa_step(1)
                x.append(traj.positions())
                v.append(traj.velocities())
            xs.append(np.stack(x))
            vs.append(np.stack(v))
        msd = np.mean([ob.msd(x, select=oxy, max_lag=100) for x in xs], axis=0)
        c = np.mean([ob.vacf(v, select=oxy, max_lag=50) for v in vs], axis=0)
        to_cm2s = 0.1 * 1e5  # A^2/fs -> 1e-5 cm^2/s
        out[f"{thermo}_gamma{gamma:g}"] = {
            "D_einstein_1e-5cm2_s": round(ob.diffusion_einstein(msd, dt_outer, 25, 100) * to_cm2s, 4),
            "D_green_kubo_1e-5cm2_s": round(ob.diffusion_green_kubo(c, dt_outer) * to_cm2s, 4)}
    torch.cuda.synchronize()
    return {"cases": out, "wall_s": round(time.perf_counter() - t0, 2), "atoms": int(s.n),
            "runs_per_case": n_runs, "sampled_ps": n_samples * dt_outer * 1e-3}


def roofline_entry(name, tot_ms, launches, flops, nbytes, traffic=None):
    """Compute and HBM axes of a kernel from its average launch duration;
    the binding one (the larger lower bound on the time) comes first."""
    avg_s = tot_ms / launches * 1e-3
    tflops = flops / avg_s / 1e12
    gbs = nbytes / avg_s / 1e9
    compute = {"bound": "mfma", "achieved": round(tflops, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": round(tflops / FP32_PEAK_TFLOPS, 4)}
    hbm = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4)}
    first, second = (compute, hbm) if flops / (FP32_PEAK_TFLOPS * 1e12) >= nbytes / (HBM_PEAK_GBS * 1e9) \
        else (hbm, compute)
    out = dict(first)
    out.update({"traffic": traffic, "kernel": name, "avg_launch_us": round(avg_s * 1e6, 1), "launches": launches,
                "algorithmic_flops_per_launch": int(flops), "algorithmic_bytes_per_launch": int(nbytes),
                "other_axis": second})
    if traffic:
        out["traffic_over_algorithmic_bytes"] = round(traffic / nbytes, 2)
        out["measured_traffic_GBps"] = round(traffic / avg_s / 1e9, 1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--skin", type=float, default=1.0, help="Verlet skin of both lists (A) in the 12,288-atom legs")
    ap.add_argument("--kernel-steps", type=int, default=20, help="outer steps of the kernel-timing region")
    ap.add_argument("--no-oracle", action="store_true", help="skip the host oracle leg")
    ap.add_argument("--workload", default="water",
                    choices=["water", "serve", "chain", "copy", "distill", "diffusion"])
    ap.add_argument("--frames", type=int, default=2000)
    ap.add_argument("--train-steps", type=int, default=10000)
    ap.add_argument("--serve-replicas", type=int, default=256)
    ap.add_argument("--serve-steps", type=int, default=500)
    ap.add_argument("--chain-steps", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this implementation has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "serve":
        rep = run_serving(args.serve_replicas, args.serve_steps)
        print(json.dumps({"metric": "p50/p99 replica step latency; aggregate ns/day",
                          "workload": f"serving_{args.serve_replicas}x{args.serve_steps}", **rep}), flush=True)
        return
    if args.workload == "copy":
        print(json.dumps({"workload": "device_copy_512MiB", **run_copy()}), flush=True)
        return
    if args.workload == "diffusion":
        print(json.dumps({"metric": "O self-diffusion, Langevin vs FFL", "workload": "diffusion_water1536",
                          **run_diffusion(args)}), flush=True)
        return
    if args.workload == "distill":
        print(json.dumps({"metric": "distillation force RMSE vs steps", "workload": "distill_water1536",
                          **run_distill(args)}), flush=True)
        return
    if args.workload == "chain":
        args.steps = args.chain_steps
        print(json.dumps({"metric": "ns/day DMTS-NC (BF16), solvated chain", "workload": "chain92k_hmr_hhf_10fs_x10",
                          **run_chain(args)}), flush=True)
        return

    from paper_2602_14975_amd import _abi
    g = run_gpu(args)
    s = g["system"]
    dt = 4.0
    value = _ns_per_day(dt, args.steps, g["t_dmts"])
    sts = _ns_per_day(0.5, g["sts_steps"], g["t_sts"])
    bf16 = _ns_per_day(dt, args.steps, g["t_bf16"])
    rewind = _ns_per_day(dt, args.steps, g["t_rewind"])

    F, K = 128, 16
    kt = g["kernel_timer"]
    roof, kernels = None, {}
    if kt.get("message_bwd", (0, 0))[1] > 0:
        flops, nbytes = message_counts(F, K, s.n, g["n_edges5"], reverse=True)
        roof = roofline_entry("k_message_bwd_mx (conservative message reverse, layers 2-3, F=128, K=16, "
                              "cosine cutoff)",
                              *kt["message_bwd"], flops, nbytes, measured_traffic())
    if kt.get("message_fwd", (0, 0))[1] > 0:
        flops, nbytes = message_counts(F, K, s.n, g["n_edges5"], reverse=False)
        kernels["message_fwd"] = roofline_entry("k_message_fwd_mx (conservative message forward, layers 2-3)",
                                                *kt["message_fwd"], flops, nbytes)
    for site in ("message_fwd_first", "message_bwd_first", "nc_message_fwd", "nc_update", "head_fwd", "baoa", "gemm"):
        if kt.get(site, (0, 0))[1] > 0:
            tot, cnt = kt[site]
            kernels[site] = {"avg_launch_us": round(tot / cnt * 1e3, 2), "launches": cnt,
                             "us_per_outer_step": round(tot * 1e3 / args.kernel_steps, 1)}
    kernels["timing_region"] = {"outer_steps": args.kernel_steps,
                                "ms_per_step": [round(x, 4) for x in kt.get("region_ms_per_step", [])],
                                "groups": [list(g) for g in TIMER_GROUPS],
                                "launches": "direct (launch timers on)"}

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "ns/day", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(g["t_dmts"] / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": "water12288_dmts_nc_4fs_x8_fp32", "atoms": int(s.n), "box_A": s.box,
                   "cons_model": "3x128 l<=1 equivariant MP, 16 Bessel, 5 A", "nc_model": "1x32, 3.5 A",
                   "outer_dt_fs": dt, "n_inner": 8, "sts_dt_fs": 0.5, "check_every": args.check_every,
                   "launches": "recorded outer step replayed as a HIP graph"},
        "sts_ns_per_day": round(sts, 3), "speedup_vs_sts": round(value / sts, 3),
        "bf16_dmts_nc_ns_per_day": round(bf16, 3), "bf16_speedup_vs_fp32_sts": round(bf16 / sts, 3),
        "rewind_armed_ns_per_day": round(rewind, 3), "rewind_armed_rewinds": g["rewinds"],
        "rewind_armed_setup": f"threshold 1e6 kcal/mol/A (never trips), frames every {args.check_every} outer steps",
        "list_rebuilds": g["rebuilds"], "temperature_end_K": round(g["t_end"], 1), "gpu": g["gpu_name"],
        "roofline": roof, "kernels": kernels,
    }
    if args.chain_steps > 0:
        cargs = argparse.Namespace(**vars(args))
        cargs.steps = args.chain_steps
        out["chain"] = run_chain(cargs)
        _progress(f"chain: {out['chain']['ns_per_day']} ns/day")
    if args.serve_replicas > 0:
        out["serving"] = run_serving(args.serve_replicas, args.serve_steps)
        _progress(f"serving: p50 {out['serving']['latency_p50_ms']} ms, p99 {out['serving']['latency_p99_ms']} ms")
    if not args.no_oracle:
        o = run_oracle(s, g["cw"], g["nw"])
        _progress("oracle start frame done")
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        o1 = run_oracle(s, g["cw"], g["nw"], pos=g["x_end"])
        fp, bf = g["start"][_abi.NNP_FP32], g["start"][_abi.NNP_BF16]
        e1, f1, fn1, _ = g["end"]
        out["force_rel_rmse"] = {
            "frames": "fp32: start and end of the timed DMTS-NC run; bf16 and sts: start",
            "cons_fp32": [rel(fp[1], o["F"]), rel(f1, o1["F"])], "nc_fp32": [rel(fp[2], o["Fn"]), rel(fn1, o1["Fn"])],
            "cons_bf16": rel(bf[1], o["F"]), "nc_bf16": rel(bf[2], o["Fn"]),
            "energy_rel_fp32": [abs(fp[0] - o["E"]) / abs(o["E"]), abs(e1 - o1["E"]) / abs(o1["E"])],
            "sts_path": "the fp32 conservative forces above (the same kernels)"}
        _progress("oracle end frame done")
        o_single = run_oracle(s, g["cw"], g["nw"], threads=1)
        _progress("oracle single-thread sample done")
        step_s = o["t_cons"] + 8 * o["t_nc"]
        step_1 = o_single["t_cons"] + 8 * o_single["t_nc"]
        out["cpu_baseline"] = {
            "value": round(_ns_per_day(dt, 1, step_s), 6), "unit": "ns/day", "cores": o["threads"],
            "kind": "oracle", "cpu": cpu_model(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "single_thread_value": round(_ns_per_day(dt, 1, step_1), 6),
            "sample": (f"one FP64 conservative energy+force ({o['t_cons']:.2f} s) and one NC force "
                       f"({o['t_nc']:.2f} s) evaluation of the 12,288-atom box on {o['threads']} threads "
                       f"({o_single['t_cons']:.2f} s and {o_single['t_nc']:.2f} s on one thread); "
                       "outer step = cons + 8 NC.  The oracle is the plain FP64 PyTorch/numpy checker, "
                       "not a tuned CPU code"),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
