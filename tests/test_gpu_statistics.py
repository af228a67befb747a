"""Statistical parity of the GPU DMTS-NC path with the oracle on the
192-atom water workload (paper, Results "Bulk water": the instantaneous
temperature follows (T/d) chi^2(d), and the O-O radial distribution).

The oracle side is tests/golden/water192_dmts_nc_statistics.json, written by
tests/golden/make_water192_statistics.py from oracle trajectories (replicas
r = 0..31).  The GPU runs 64 independent replicas of the same recipe with
r = 100..163 packed into one system (replica i uses Philox stream 100 + i),
so the two ensembles are independent samples of the same law, and every
comparison is a two-sample test at significance about 1e-3:
  * temperature after 0.2 ps: ensemble mean equal to the oracle's (z <= 3.5
    with standard errors from independent replicas), spread across replicas
    within 12 % of the chi^2 law's 300 sqrt(2/3N) = 17.7 K;
  * O-O pair counts per frame in 0.1 A bins: chi-square over the bins with
    at least 20 counts on both sides, p > 1e-3, every |z| <= 4.5.
With a friction of 1/ps the ensemble mean is still relaxing from the
lattice start during that 1 ps (288 K at 0.25 ps, 296 K at 1 ps in the
oracle), so the equilibrium law of the mean is tested by a second GPU run
of the same replicas at 10/ps: mean 300 K within 3.5 standard errors or
1 %, whichever is larger, spread within 10 % of 17.7 K, after 0.3 ps.
"""

import json
import os

import numpy as np
import pytest
import torch

import synth
from tests._statistics import binned_chi2, chi2_temperature_spread, replica_mean_se

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "water192_dmts_nc_statistics.json")
KB = 8.31446261815324 / 4184.0
FIRST_GPU_REPLICA, N_GPU_REPLICAS = 100, 64


def _oo_counts(x, box, oxygen, bin_width, n_bins):
    o = x[oxygen]
    d = o[None, :, :] - o[:, None, :]
    d = d - box * np.round(d / box)
    r = np.sqrt((d * d).sum(-1))[np.triu_indices(o.shape[0], 1)]
    idx = np.floor(r / bin_width).astype(np.int64)
    return np.bincount(idx[idx < n_bins], minlength=n_bins)[:n_bins]


def _gpu_ensemble(nnp, rec, gamma_ps=None, histograms=True):
    systems = [synth.water_box(4, 12.42, 1100 + r) for r in range(FIRST_GPU_REPLICA,
                                                                  FIRST_GPU_REPLICA + N_GPU_REPLICAS)]
    n = systems[0].n
    masses = np.concatenate([s.standard_masses() for s in systems])
    vel = np.concatenate([synth.maxwell_boltzmann(s.standard_masses(), rec["temperature_K"], 5100 + r)
                          for r, s in zip(range(FIRST_GPU_REPLICA, FIRST_GPU_REPLICA + N_GPU_REPLICAS), systems)])
    cons = nnp.Model.from_spec(synth.CONS_CFG0, synth.random_weights(synth.CONS_CFG0, rec["cons_weights_seed"]))
    nc = nnp.Model.from_spec(synth.NC_CFG0, synth.random_weights(synth.NC_CFG0, rec["nc_weights_seed"]))
    system = nnp.DeviceSystem([s.pos for s in systems], [s.species for s in systems], [s.box for s in systems])
    prm = nnp.respa_params(rec["dt_outer_fs"], rec["n_inner"], rec["temperature_K"], seed=rec["philox_seed"],
                           stream_id=FIRST_GPU_REPLICA)
    gamma = rec["gamma_ps"] if gamma_ps is None else gamma_ps
    traj = nnp.Trajectory(cons, nc, system, vel, masses, np.full(system.n, gamma), prm)
    every = rec["t_every"]
    assert rec["rdf_every"] == every and rec["rdf_first"] % every == 0
    ke = torch.zeros(every, N_GPU_REPLICAS, dtype=torch.float64, device="cuda")
    temps = np.zeros((N_GPU_REPLICAS, rec["n_outer"] // every))
    hist = np.zeros((N_GPU_REPLICAS, rec["rdf_bins"]))
    oxygen = systems[0].species == 3
    for k in range(rec["n_outer"] // every):
        traj.respa_step(every, ke)
        temps[:, k] = ke[-1].cpu().numpy() * 2.0 / (3 * n * KB)
        step = (k + 1) * every
        if histograms and step >= rec["rdf_first"]:
            x = traj.positions()
            for i, s in enumerate(systems):
                hist[i] += _oo_counts(x[i * n:(i + 1) * n], s.box, oxygen, rec["rdf_bin"], rec["rdf_bins"])
    assert traj.step_count == rec["n_outer"] * rec["n_inner"]
    return temps, hist, n


def test_temperature_and_oo_rdf_within_statistical_error(gpu_lib):
    with open(GOLDEN) as f:
        ref = json.load(f)
    rec = ref["recipe"]
    print(f"case statistics water192 x {N_GPU_REPLICAS} replicas, {rec['n_outer']} outer steps", flush=True)
    t_gpu, h_gpu, n = _gpu_ensemble(gpu_lib, rec)
    t_ora = np.asarray(ref["temperature"])
    h_ora = np.asarray(ref["oo_counts"], dtype=np.float64)
    burn = rec["rdf_first"] // rec["t_every"] - 1          # first sample at 0.2 ps
    n_frames = (rec["n_outer"] - rec["rdf_first"]) // rec["rdf_every"] + 1
    sigma = chi2_temperature_spread(n)
    mg, sg = replica_mean_se(t_gpu[:, burn:].mean(1))
    mo, so = replica_mean_se(t_ora[:, burn:].mean(1))
    spread_g = float(np.sqrt(np.mean(t_gpu[:, burn:].var(0, ddof=1))))
    chi2, dof, p, zmax = binned_chi2(h_gpu / n_frames, h_ora / n_frames)
    print(f"T: GPU {mg:.1f} +- {sg:.1f} K, oracle {mo:.1f} +- {so:.1f} K; spread GPU {spread_g:.1f} K "
          f"(chi2 law {sigma:.1f}); O-O bins: chi2 {chi2:.1f} / {dof}, p {p:.3g}, max |z| {zmax:.2f}", flush=True)
    assert abs(mg - mo) <= 3.5 * np.hypot(sg, so)
    assert abs(spread_g / sigma - 1) <= 0.12
    assert dof >= 30
    assert p > 1e-3 and zmax <= 4.5


def test_temperature_follows_chi_square_law(gpu_lib):
    with open(GOLDEN) as f:
        rec = json.load(f)["recipe"]
    print(f"case chi2 temperature law water192 x {N_GPU_REPLICAS} replicas, friction 10/ps", flush=True)
    t, _, n = _gpu_ensemble(gpu_lib, rec, gamma_ps=10.0, histograms=False)
    burn = 300 // rec["t_every"] - 1
    mean, se = replica_mean_se(t[:, burn:].mean(1))
    spread = float(np.sqrt(np.mean(t[:, burn:].var(0, ddof=1))))
    sigma = chi2_temperature_spread(n)
    print(f"T at 10/ps: {mean:.1f} +- {se:.1f} K, spread {spread:.1f} K (law 300, {sigma:.1f})", flush=True)
    assert abs(mean - 300.0) <= max(3.5 * se, 0.01 * 300.0) and se < 3.0
    assert abs(spread / sigma - 1) <= 0.10
