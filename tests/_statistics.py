"""Two-sample statistics shared by the statistical parity tests (no method
arithmetic): ensemble means with standard errors from independent
replicas, and a chi-square comparison of binned means."""

import math

import numpy as np
from scipy import stats

T_CHI2_K = 300.0


def replica_mean_se(per_replica):
    """Mean over replicas and its standard error (replicas independent)."""
    a = np.asarray(per_replica, dtype=np.float64)
    return float(a.mean()), float(a.std(ddof=1) / math.sqrt(a.shape[0]))


def binned_chi2(a, b, min_total=20):
    """a, b: (replicas, bins) per-replica values from two independent
    ensembles.  Returns (chi2, dof, p, max |z|) over the bins whose pooled
    count reaches ``min_total`` on both sides, with z_b the difference of the
    bin means over the combined standard error."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    ma, mb = a.mean(0), b.mean(0)
    va = a.var(0, ddof=1) / a.shape[0]
    vb = b.var(0, ddof=1) / b.shape[0]
    use = (a.sum(0) >= min_total) & (b.sum(0) >= min_total) & (va + vb > 0)
    z = (ma[use] - mb[use]) / np.sqrt(va[use] + vb[use])
    chi2 = float(np.sum(z * z))
    dof = int(use.sum())
    return chi2, dof, float(stats.chi2.sf(chi2, dof)), float(np.max(np.abs(z))) if dof else 0.0


def chi2_temperature_spread(n_atoms, temperature=T_CHI2_K):
    """Standard deviation of the instantaneous temperature under the
    equilibrium law (T/d) chi^2(d), d = 3N (no constraints)."""
    return temperature * math.sqrt(2.0 / (3 * n_atoms))
