"""Throughput of the DMTS-NC hot path on one MI355X.

Default workload: 4,096 rigid-geometry waters (12,288 atoms) in a 49.6 A
periodic box, conservative model 3 layers x 128 (FP32), distilled NC model
1 x 32 (FP32), DMTS-NC with a 4 fs outer step and 8 inner steps of 0.5 fs,
Langevin 300 K, gamma 1 ps^-1.  One "step" is one outer step of Algorithm 1:
neighbour maintenance, 8 NC force evaluations with 8 BAOA half-steps and
kicks, one conservative energy + hand-written-reverse force evaluation and
the outer kicks.  The single-time-step (BAOAB, 0.5 fs, conservative model
alone) path is timed on the same system for comparison.

Prints one JSON line.  `value` is DMTS-NC ns/day on the device with all
inputs resident in HBM; `roofline` covers the dominant kernel (the
conservative message-passing reverse), timed with HIP events on its own
stream inside the timed region; `cpu_baseline` is the FP64 oracle timed on
the host on a bounded sample (one conservative and one NC evaluation of the
same box), which also supplies the reference forces of `force_rel_rmse`.
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
FP32_VECTOR_PEAK_TFLOPS = 157.3


def _ns_per_day(dt_fs, steps, seconds):
    return dt_fs * steps / seconds * 86400.0 * 1e-6


def message_bwd_flops_per_edge(F, K):
    """Algorithmic FP32 flops of the conservative message reverse per
    directed edge within the cutoff (one layer): the filter w = Wr e f + br f
    and its radial derivative (2 x 3F x K multiply-adds = 12 F K flops) and
    the adjoint products of both messages of the pair (about 40 multiply-adds
    per feature = 80 F flops)."""
    return 12 * F * K + 80 * F


def run_gpu(args):
    import torch

    import synth
    from paper_2602_14975_amd import nnp

    torch.cuda.set_device(0)
    s = synth.water_config(1)
    cw = synth.random_weights(synth.CONS_CFG1, 2001)
    nw = synth.random_weights(synth.NC_CFG1, 3001)
    cons = nnp.Model.from_spec(synth.CONS_CFG1, cw)
    nc = nnp.Model.from_spec(synth.NC_CFG1, nw)
    m = s.standard_masses()
    gamma = np.ones(s.n)
    v0 = synth.maxwell_boltzmann(m, 300.0, 5001)
    lib = nnp.lib()

    # forces at the starting configuration (for the accuracy report)
    sys0 = nnp.DeviceSystem(s.pos, s.species, s.box)
    nl = nnp.NeighborList(sys0.n, 5.0, 900000)
    ws = nnp.workspace(cons, nc, sys0.n, 1, nl.capacity)
    nnp.nnp_neighbors(sys0, nl, ws)
    e0, f_cons0 = nnp.nnp_cons_energy_forces(cons, sys0, nl, ws)
    f_nc0 = nnp.nnp_nc_forces(nc, sys0, nl, ws)
    n_edges5 = int(nl.n_edges)
    gpu_forces = (float(e0.cpu()[0]), f_cons0.cpu().numpy().T.astype(np.float64),
                  f_nc0.cpu().numpy().T.astype(np.float64))
    del ws

    def timed(mode, dt, n_inner, steps, warmup, timer_site=None):
        system = nnp.DeviceSystem(s.pos, s.species, s.box)
        prm = nnp.respa_params(dt, n_inner, 300.0, seed=4001, mode=mode, skin=1.0, check_every=args.check_every)
        traj = nnp.Trajectory(cons, nc if mode == "dmts_nc" else None, system, v0, m, gamma, prm)
        traj.respa_step(max(1, warmup))
        torch.cuda.synchronize()
        if timer_site:
            # the kernel's durations over the timed region itself, from HIP
            # events that its launches timestamp (no host-side records in
            # between); with timers on, outer steps are launched directly
            # rather than replayed from a recorded graph
            lib.nnp_timer_enable(timer_site.encode(), 1)
            tot, cnt = C.c_double(), C.c_int64()
            lib.nnp_timer_read(timer_site.encode(), C.byref(tot), C.byref(cnt), 1)
        t0 = time.perf_counter()
        traj.respa_step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kt = None
        if timer_site:
            tot, cnt = C.c_double(), C.c_int64()
            lib.nnp_timer_read(timer_site.encode(), C.byref(tot), C.byref(cnt), 1)
            lib.nnp_timer_enable(timer_site.encode(), 0)
            kt = (tot.value, cnt.value)
        return t1 - t0, traj, kt

    t_dmts, traj, kt = timed("dmts_nc", 4.0, 8, args.steps, args.warmup, timer_site="message_bwd")
    # forces at the configuration the timed run ended in (second accuracy frame)
    x_end = traj.positions()
    sys1 = nnp.DeviceSystem(x_end, s.species, s.box)
    nl1 = nnp.NeighborList(sys1.n, 5.0, 900000)
    ws1 = nnp.workspace(cons, nc, sys1.n, 1, nl1.capacity)
    nnp.nnp_neighbors(sys1, nl1, ws1)
    e1, f_cons1 = nnp.nnp_cons_energy_forces(cons, sys1, nl1, ws1)
    f_nc1 = nnp.nnp_nc_forces(nc, sys1, nl1, ws1)
    gpu_forces_end = (float(e1.cpu()[0]), f_cons1.cpu().numpy().T.astype(np.float64),
                      f_nc1.cpu().numpy().T.astype(np.float64))
    del ws1
    v_end = traj.velocities()
    kb = 8.31446261815324 / 4184.0  # kcal/mol/K
    ke_end = 0.5 * float((m[:, None] * v_end * v_end).sum()) / 4.184e-4  # amu A^2/fs^2 -> kcal/mol
    t_end = 2.0 * ke_end / (3 * s.n * kb)
    sts_steps = max(8, args.steps)
    t_sts, _, _ = timed("sts", 0.5, 1, sts_steps, args.warmup)
    return {
        "t_dmts": t_dmts, "t_sts": t_sts, "sts_steps": sts_steps, "kernel_timer": kt, "n_edges5": n_edges5,
        "rebuilds": traj.n_rebuilds, "gpu_forces": gpu_forces, "system": s, "cw": cw, "nw": nw, "t_end": t_end,
        "gpu_forces_end": gpu_forces_end, "x_end": x_end,
        "gpu_name": torch.cuda.get_device_name(0),
    }


def run_oracle(s, cw, nw, pos=None):
    """FP64 oracle on the host: one conservative and one NC evaluation (at
    the starting configuration, or at `pos`)."""
    import torch

    import synth
    from oracle import models as om
    from oracle import neighbors as onb

    x = s.pos if pos is None else pos
    threads = torch.get_num_threads()
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
    return {"E": E, "F": F, "Fn": Fn, "t_cons": t_cons, "t_nc": t_nc, "t_nb": t_nb, "threads": threads}


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


def run_serving(n_replicas, n_steps, per_atom_step_s, load=0.8, budget_frac=0.25, seed=30000, max_slots=64):
    """Continuous batching of replicas of 300-6,000 atoms (30% with a chain),
    DMTS-NC 4 fs x 8 with BF16 perceptrons, Poisson arrivals at `load` times
    the estimated saturated rate, HBM budget = budget_frac of the summed
    footprints."""
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
    budget = max(int(budget_frac * sum(sizes)), max(sizes) + (16 << 20))
    mean_atoms = float(np.mean([r.n for r in reps]))
    rate = load / (mean_atoms * n_steps * per_atom_step_s)
    arrivals = synth.systems.poisson_arrivals(n_replicas, rate, seed)
    srv = serve.Server(cons, nc, prm, budget, max_slots)
    torch.cuda.synchronize()
    rep = serve.run(srv, reps, arrivals, n_steps, 4.0)
    srv.close()
    rep.update({"steps_per_replica": n_steps, "arrival_rate_per_s": round(rate, 3), "hbm_budget_MiB": budget >> 20,
                "budget_frac_of_total": budget_frac, "max_slots": max_slots, "atoms_total": int(sum(r.n for r in reps)),
                "precision": "bf16 perceptrons, fp32 edge filter and forces, fp64 integration"})
    for k in ("latency_p50_ms", "latency_p99_ms", "aggregate_ns_per_day", "wall_s", "queue_delay_mean_s",
              "queue_delay_p99_s"):
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--no-oracle", action="store_true", help="skip the host oracle leg")
    ap.add_argument("--workload", default="water",
                    choices=["water", "serve", "chain", "copy", "distill", "diffusion"])
    ap.add_argument("--frames", type=int, default=2000)
    ap.add_argument("--train-steps", type=int, default=10000)
    ap.add_argument("--serve-replicas", type=int, default=32)
    ap.add_argument("--serve-steps", type=int, default=50)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "serve":
        rep = run_serving(256, 500, per_atom_step_s=0.5e-6)
        print(json.dumps({"metric": "p50/p99 replica step latency; aggregate ns/day", "workload": "serving_256x500",
                          **rep}), flush=True)
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
        print(json.dumps({"metric": "ns/day DMTS-NC (BF16), solvated chain", "workload": "chain92k_hmr_hhf_10fs_x10",
                          **run_chain(args)}), flush=True)
        return

    g = run_gpu(args)
    s = g["system"]
    dt = 4.0
    value = _ns_per_day(dt, args.steps, g["t_dmts"])
    sts = _ns_per_day(0.5, g["sts_steps"], g["t_sts"])

    F, K = 128, 16
    roof = None
    if g["kernel_timer"] and g["kernel_timer"][1] > 0:
        tot_ms, launches = g["kernel_timer"]
        avg_s = tot_ms / launches * 1e-3
        flops = message_bwd_flops_per_edge(F, K) * g["n_edges5"]
        achieved = flops / avg_s / 1e12
        roof = {"bound": "alu", "kernel": "k_message_bwd_mx (F=128, K=16, cosine cutoff)", "achieved": round(achieved, 2),
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": measured_traffic(), "avg_launch_us": round(avg_s * 1e6, 1), "launches": launches,
                "edges_per_launch": g["n_edges5"]}

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "ns/day", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(g["t_dmts"] / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": "water12288_dmts_nc_4fs_x8_fp32", "atoms": int(s.n), "box_A": s.box,
                   "cons_model": "3x128 l<=1 equivariant MP, 16 Bessel, 5 A", "nc_model": "1x32, 3.5 A",
                   "outer_dt_fs": dt, "n_inner": 8, "sts_dt_fs": 0.5, "check_every": args.check_every},
        "sts_ns_per_day": round(sts, 3), "speedup_vs_sts": round(value / sts, 3),
        "list_rebuilds": g["rebuilds"], "temperature_end_K": round(g["t_end"], 1), "gpu": g["gpu_name"],
        "roofline": roof,
    }
    if args.serve_replicas > 0:
        per_atom = g["t_dmts"] / args.steps / s.n
        out["serving"] = run_serving(args.serve_replicas, args.serve_steps, per_atom)
    if not args.no_oracle:
        o = run_oracle(s, g["cw"], g["nw"])
        e_gpu, f_gpu, fn_gpu = g["gpu_forces"]
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        o1 = run_oracle(s, g["cw"], g["nw"], pos=g["x_end"])
        e1, f1, fn1 = g["gpu_forces_end"]
        out["force_rel_rmse"] = {
            "frames": "start and end of the timed DMTS-NC run",
            "cons": [rel(f_gpu, o["F"]), rel(f1, o1["F"])], "nc": [rel(fn_gpu, o["Fn"]), rel(fn1, o1["Fn"])],
            "energy_rel": [abs(e_gpu - o["E"]) / abs(o["E"]), abs(e1 - o1["E"]) / abs(o1["E"])]}
        step_s = o["t_cons"] + 8 * o["t_nc"]
        out["cpu_baseline"] = {
            "value": round(_ns_per_day(dt, 1, step_s), 6), "unit": "ns/day", "cores": o["threads"],
            "kind": "oracle",
            "sample": (f"one FP64 conservative energy+force ({o['t_cons']:.2f} s) and one NC force "
                       f"({o['t_nc']:.2f} s) evaluation of the 12,288-atom box; outer step = cons + 8 NC"),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
