"""CPU pins of the transport estimators (paper_2602_14975_amd.observables):
closed forms for ballistic motion and for an Ornstein-Uhlenbeck velocity
process, whose diffusion coefficient is s^2 / gamma."""

import numpy as np

from paper_2602_14975_amd import observables as ob


def test_ballistic_motion():
    rng = np.random.default_rng(1)
    v = rng.normal(size=(50, 3))
    dt = 2.0
    t = np.arange(40) * dt
    x = v[None, :, :] * t[:, None, None] + rng.uniform(0, 10, size=(1, 50, 3))
    m = ob.msd(x, max_lag=10)
    v2 = float(np.mean(np.sum(v * v, axis=1)))
    np.testing.assert_allclose(m, v2 * (np.arange(11) * dt) ** 2, rtol=1e-12, atol=1e-12)
    c = ob.vacf(np.repeat(v[None], 40, axis=0), max_lag=10)
    np.testing.assert_allclose(c, v2, rtol=1e-12)


def test_selection_and_lag_zero():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(6, 8, 3))
    sel = np.array([True, False] * 4)
    assert ob.msd(x)[0] == 0.0
    np.testing.assert_allclose(ob.msd(x, select=sel), ob.msd(x[:, sel]))


def test_ornstein_uhlenbeck_diffusion():
    """Exact OU updates v <- c v + sqrt(1 - c^2) s G with c = exp(-gamma dt);
    x integrated with the trapezoid rule.  Einstein and Green-Kubo both give
    D = s^2 / gamma within sampling error."""
    rng = np.random.default_rng(3)
    n, steps, dt, gamma, s = 300, 3000, 1.0, 0.05, 0.7
    c = np.exp(-gamma * dt)
    v = rng.normal(scale=s, size=(n, 3))
    x = np.zeros((n, 3))
    xs = np.empty((steps, n, 3))
    vs = np.empty((steps, n, 3))
    for k in range(steps):
        v_new = c * v + np.sqrt(1.0 - c * c) * s * rng.normal(size=(n, 3))
        x = x + 0.5 * dt * (v + v_new)
        v = v_new
        xs[k] = x
        vs[k] = v
    d_exact = s * s / gamma
    m = ob.msd(xs[::10], max_lag=60)
    d_e = ob.diffusion_einstein(m, 10 * dt, 20, 60)
    d_g = ob.diffusion_green_kubo(ob.vacf(vs[::2], max_lag=150), 2 * dt)
    assert abs(d_e - d_exact) < 0.08 * d_exact
    assert abs(d_g - d_exact) < 0.08 * d_exact
