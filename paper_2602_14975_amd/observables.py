"""Transport observables from sampled trajectories (host-side numpy).

The paper compares thermostats by the self-diffusion they leave intact
(Methods, fast-forward Langevin; the diffusion table of the water results).
These estimators work on positions or velocities sampled every `dt_fs`:

* mean-squared displacement MSD(tau) = < |x_i(t + tau) - x_i(t)|^2 >, averaged
  over atoms and over every time origin t (positions must be unwrapped);
* velocity autocorrelation C(tau) = < v_i(t) . v_i(t + tau) >, likewise;
* D from the Einstein relation, MSD = 6 D tau + c, by a least-squares line
  over a window of lags; and from Green-Kubo, D = (1/3) integral C(tau) dtau
  (trapezoid rule) up to a cut-off lag.

Units follow the library: Angstrom, fs; D in Angstrom^2/fs (1 A^2/fs =
0.1 cm^2/s).
"""

import numpy as np


def _frames(a, select):
    a = np.asarray(a, dtype=np.float64)
    if a.ndim != 3 or a.shape[2] != 3:
        raise ValueError("expected samples shaped [frames][atoms][3]")
    return a if select is None else a[:, np.asarray(select), :]


def msd(positions, select=None, max_lag=None):
    """MSD for lags 0..max_lag (frames); returns an array of length max_lag + 1."""
    x = _frames(positions, select)
    t = x.shape[0]
    max_lag = t - 1 if max_lag is None else min(int(max_lag), t - 1)
    out = np.zeros(max_lag + 1)
    for lag in range(1, max_lag + 1):
        d = x[lag:] - x[:-lag]
        out[lag] = float(np.mean(np.sum(d * d, axis=2)))
    return out


def vacf(velocities, select=None, max_lag=None):
    """Velocity autocorrelation for lags 0..max_lag (frames)."""
    v = _frames(velocities, select)
    t = v.shape[0]
    max_lag = t - 1 if max_lag is None else min(int(max_lag), t - 1)
    out = np.zeros(max_lag + 1)
    for lag in range(max_lag + 1):
        out[lag] = float(np.mean(np.sum(v[: t - lag] * v[lag:], axis=2)))
    return out


def diffusion_einstein(msd_values, dt_fs, lag_lo, lag_hi):
    """D (A^2/fs) from the slope of MSD over lags [lag_lo, lag_hi]."""
    lags = np.arange(lag_lo, lag_hi + 1)
    slope, _ = np.polyfit(lags * dt_fs, np.asarray(msd_values)[lags], 1)
    return float(slope / 6.0)


def diffusion_green_kubo(vacf_values, dt_fs, lag_hi=None):
    """D (A^2/fs) = (1/3) * integral of the VACF up to lag_hi (trapezoid)."""
    c = np.asarray(vacf_values, dtype=np.float64)
    c = c if lag_hi is None else c[: int(lag_hi) + 1]
    return float(np.trapezoid(c, dx=dt_fs) / 3.0)
