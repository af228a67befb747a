"""Observables used by the statistical checks (oracle, float64 numpy).

* Instantaneous temperature T = 2 KE / (d k_B), d = 3N (paper, "Bulk water":
  the equilibrium law of T is (T/d) chi^2(d)); hence mean T and standard
  deviation T sqrt(2/d).
* O-O radial distribution g(r): pair histogram under the minimum image with
  bins of width dr up to L/2, normalised by the ideal-gas count
  N_O (N_O - 1) / V * 4/3 pi (r_hi^3 - r_lo^3) / 2 per unordered pair set.
* Relative RMSE ||F - F_ref||_2 / ||F_ref||_2 over all atoms and components.

Pins: uniform random points give g(r) = 1 within noise; a simple cubic
lattice puts exactly 6 neighbours in the first shell.
"""

import math

import numpy as np


def chi2_temperature_moments(t0, n_atoms):
    d = 3 * n_atoms
    return t0, t0 * math.sqrt(2.0 / d)


def rdf(pos, box, select, dr=0.05, r_max=None):
    """g(r) over atoms where ``select`` is True.  Returns (r_centres, g)."""
    x = np.asarray(pos, dtype=np.float64)[np.asarray(select)]
    n = x.shape[0]
    r_max = box / 2.0 if r_max is None else r_max
    nb = int(math.floor(r_max / dr))
    hist = np.zeros(nb, dtype=np.float64)
    for a in range(n - 1):
        d = x[a + 1:] - x[a]
        d = d - box * np.round(d / box)
        r = np.sqrt(np.sum(d * d, axis=1))
        r = r[r < nb * dr]
        hist += np.bincount((r / dr).astype(np.int64), minlength=nb)[:nb]
    edges = dr * np.arange(nb + 1)
    shell = 4.0 / 3.0 * math.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    ideal = 0.5 * n * (n - 1) / box ** 3 * shell
    return 0.5 * (edges[1:] + edges[:-1]), hist / ideal


def rel_rmse(f, f_ref):
    f = np.asarray(f, dtype=np.float64)
    f_ref = np.asarray(f_ref, dtype=np.float64)
    return float(np.linalg.norm(f - f_ref) / np.linalg.norm(f_ref))
