"""Writes water192_dmts_nc_statistics.json: temperature series and O-O pair
histograms of oracle DMTS-NC trajectories of the 192-atom water workload,
the reference side of the statistical parity test (paper, Results "Bulk
water": the temperature law (T/d) chi^2(d) and the O-O radial distribution).

It calls only ``oracle`` and ``synth``; run it from the repository root:
    python tests/golden/make_water192_statistics.py [n_replicas] [n_workers]

Recipe (stored in the file, and read from there by the GPU test): replica r
is water_box(4, 12.42 A, seed 1100 + r) with standard masses,
Maxwell-Boltzmann velocities at 300 K (seed 5100 + r), the 192-atom
workload's models (conservative width 32 x 2 layers, weights seed 2000; NC
width 16, seed 3000), DMTS-NC with an outer step of 2 fs and 4 inner steps,
300 K, friction 1 / ps on every atom, Philox seed 4000 and stream r, for 500
outer steps (1 ps).  The temperature is recorded every 10 outer steps; the
O-O pair distances (minimum image) are histogrammed in 0.1 A bins up to
6.2 A at outer steps 100, 110, ..., 500 and summed over those frames.
"""

import json
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

RECIPE = {
    "system": "water_box(4, 12.42, 1100 + r)", "velocity_seed": "5100 + r", "cons_weights_seed": 2000,
    "nc_weights_seed": 3000, "dt_outer_fs": 2.0, "n_inner": 4, "temperature_K": 300.0, "gamma_ps": 1.0,
    "philox_seed": 4000, "philox_stream": "r", "n_outer": 500, "t_every": 10, "rdf_first": 100, "rdf_every": 10,
    "rdf_bin": 0.1, "rdf_bins": 62,
}


def oo_counts(x, box, oxygen, bin_width, n_bins):
    """Histogram of unordered O-O pair distances under the minimum image."""
    import numpy as np
    o = x[oxygen]
    d = o[None, :, :] - o[:, None, :]
    d = d - box * np.round(d / box)
    r = np.sqrt((d * d).sum(-1))[np.triu_indices(o.shape[0], 1)]
    idx = np.floor(r / bin_width).astype(np.int64)
    return np.bincount(idx[idx < n_bins], minlength=n_bins)[:n_bins]


def run_replica(r):
    import numpy as np
    import torch
    torch.set_num_threads(1)
    import synth
    from oracle import integrator as oi
    from oracle import models as om
    from oracle import neighbors as onb
    R = RECIPE
    s = synth.water_box(4, 12.42, 1100 + r)
    cw = synth.random_weights(synth.CONS_CFG0, R["cons_weights_seed"])
    nw = synth.random_weights(synth.NC_CFG0, R["nc_weights_seed"])
    m = s.standard_masses()
    st = oi.State(s.pos.copy(), synth.maxwell_boltzmann(m, R["temperature_K"], 5100 + r), m.copy())
    prm = oi.LangevinParams(R["dt_outer_fs"], R["n_inner"], R["temperature_K"], np.full(s.n, R["gamma_ps"]),
                            seed=R["philox_seed"], stream=r)

    def cons(x):
        return om.cons_energy_forces(synth.CONS_CFG0, cw, x, s.species, s.box,
                                     *onb.pairs_bruteforce(x, s.box, synth.CONS_CFG0.cutoff))[1]

    def nc(x):
        return om.nc_forces(synth.NC_CFG0, nw, x, s.species, s.box,
                            *onb.pairs_bruteforce(x, s.box, synth.NC_CFG0.cutoff))

    temps, hist = [], np.zeros(R["rdf_bins"], dtype=np.int64)
    oxygen = s.species == 3
    for k in range(1, R["n_outer"] + 1):
        oi.dmts_nc_step(st, cons, nc, prm)
        if k % R["t_every"] == 0:
            temps.append(oi.temperature(st.v, st.m))
        if k >= R["rdf_first"] and (k - R["rdf_first"]) % R["rdf_every"] == 0:
            hist += oo_counts(st.x, s.box, oxygen, R["rdf_bin"], R["rdf_bins"])
    print(f"replica {r}: mean T {np.mean(temps):.1f} K", flush=True)
    return [float(t) for t in temps], [int(c) for c in hist]


def main():
    n_rep = int(sys.argv[1]) if len(sys.argv) > 1 else 32
    workers = int(sys.argv[2]) if len(sys.argv) > 2 else min(8, os.cpu_count() or 1)
    with Pool(workers) as pool:
        res = pool.map(run_replica, range(n_rep))
    out = {"recipe": RECIPE, "n_replicas": n_rep, "temperature": [t for t, _ in res],
           "oo_counts": [h for _, h in res]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "water192_dmts_nc_statistics.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"wrote {path}")


if __name__ == "__main__":
    main()
