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
    sts_steps = max(8, args.steps)
    t_sts, _, _ = timed("sts", 0.5, 1, sts_steps, args.warmup)
    return {
        "t_dmts": t_dmts, "t_sts": t_sts, "sts_steps": sts_steps, "kernel_timer": kt, "n_edges5": n_edges5,
        "rebuilds": traj.n_rebuilds, "gpu_forces": gpu_forces, "system": s, "cw": cw, "nw": nw,
        "gpu_name": torch.cuda.get_device_name(0),
    }


def run_oracle(s, cw, nw):
    """FP64 oracle on the host: one conservative and one NC evaluation."""
    import torch

    import synth
    from oracle import models as om
    from oracle import neighbors as onb

    threads = torch.get_num_threads()
    t0 = time.perf_counter()
    off5, nbr5 = onb.pairs_cell_list(s.pos, s.box, 5.0)
    t_nb = time.perf_counter() - t0
    t0 = time.perf_counter()
    E, F = om.cons_energy_forces(synth.CONS_CFG1, cw, s.pos, s.species, s.box, off5, nbr5)
    t_cons = time.perf_counter() - t0
    off35, nbr35 = onb.pairs_bruteforce(s.pos, s.box, 3.5)
    t0 = time.perf_counter()
    Fn = om.nc_forces(synth.NC_CFG1, nw, s.pos, s.species, s.box, off35, nbr35)
    t_nc = time.perf_counter() - t0
    return {"E": E, "F": F, "Fn": Fn, "t_cons": t_cons, "t_nc": t_nc, "t_nb": t_nb, "threads": threads}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--no-oracle", action="store_true", help="skip the host oracle leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

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
        roof = {"bound": "alu", "kernel": "k_message_bwd<128,16,cos>", "achieved": round(achieved, 2),
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": None, "avg_launch_us": round(avg_s * 1e6, 1), "launches": launches,
                "edges_per_launch": g["n_edges5"]}

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "ns/day", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(g["t_dmts"] / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": "water12288_dmts_nc_4fs_x8_fp32", "atoms": int(s.n), "box_A": s.box,
                   "cons_model": "3x128 l<=1 equivariant MP, 16 Bessel, 5 A", "nc_model": "1x32, 3.5 A",
                   "outer_dt_fs": dt, "n_inner": 8, "sts_dt_fs": 0.5, "check_every": args.check_every},
        "sts_ns_per_day": round(sts, 3), "speedup_vs_sts": round(value / sts, 3),
        "list_rebuilds": g["rebuilds"], "gpu": g["gpu_name"],
        "roofline": roof,
    }
    if not args.no_oracle:
        o = run_oracle(s, g["cw"], g["nw"])
        e_gpu, f_gpu, fn_gpu = g["gpu_forces"]
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        out["force_rel_rmse"] = {"cons": rel(f_gpu, o["F"]), "nc": rel(fn_gpu, o["Fn"]),
                                 "energy_rel": abs(e_gpu - o["E"]) / abs(o["E"])}
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
