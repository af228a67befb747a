"""Pins for the oracle's random numbers, integrators, HMR and observables."""

import copy

import numpy as np
import pytest
from scipy import stats

import synth
from oracle import analysis as oa
from oracle import integrator as oi


# ------------------------------------------------------------------ Philox --

def test_philox_known_answer():
    # Random123 known-answer vector for philox4x64-10 with zero counter and key.
    assert oi.philox4x64_scalar([0, 0, 0, 0], [0, 0]) == [
        0x16554D9ECA36314C, 0xDB20FE9D672D0FDC, 0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_philox_matches_numpy_bit_generator(seed):
    rng = np.random.default_rng(seed)
    for _ in range(5):
        key = [int(x) for x in rng.integers(0, 2 ** 63, size=2, dtype=np.uint64)]
        ctr = [int(x) for x in rng.integers(1, 2 ** 63, size=4, dtype=np.uint64)]
        # numpy's Philox increments its counter before producing a block.
        start = np.array([ctr[0] - 1, ctr[1], ctr[2], ctr[3]], dtype=np.uint64)
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=start)
        assert [int(x) for x in bg.random_raw(4)] == oi.philox4x64_scalar(ctr, key)


def test_philox_vectorised_equals_scalar():
    atoms = np.arange(50, dtype=np.uint64)
    w = oi.philox4x64(atoms, np.uint64(123456789), 0, 0, 42, 7)
    for a in (0, 1, 17, 49):
        assert [int(x[a]) for x in w] == oi.philox4x64_scalar([a, 123456789, 0, 0], [42, 7])


def test_normals_are_standard_gaussian():
    g = np.concatenate([oi.langevin_normals(5, 3, step, 20000) for step in range(10)])
    for c in range(3):
        assert stats.kstest(g[:, c], "norm").pvalue > 1e-4
    assert abs(g.mean()) < 5 / np.sqrt(g.size)
    assert abs(g.var() - 1) < 0.01
    # distinct steps and streams decorrelate
    a = oi.langevin_normals(5, 3, 0, 20000)[:, 0]
    b = oi.langevin_normals(5, 4, 0, 20000)[:, 0]
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.03


def test_box_muller_at_chosen_uniforms():
    """u0 = u2 = exp(-1/2) gives radius 1; the angles 2 pi u1 and 2 pi u3 at
    u = 0, 1/8, 1/4, 1/2 put the normals at known points of the unit circle."""
    r = np.exp(-0.5)
    u1 = np.array([0.0, 0.125, 0.25, 0.5])
    u3 = np.array([0.5, 0.0, 0.125, 0.25])
    g = oi.box_muller(np.full(4, r), u1, np.full(4, r * r), u3)   # second radius sqrt(2)
    h = np.sqrt(0.5)
    expect = np.array([[1.0, 0.0, -np.sqrt(2)], [h, h, np.sqrt(2)], [0.0, 1.0, 1.0], [-1.0, 0.0, 0.0]])
    np.testing.assert_allclose(g, expect, atol=1e-15)


def test_uniform_mapping_endpoints():
    u = oi.uniforms_from_bits(np.array([0, 2 ** 64 - 1], dtype=np.uint64))
    assert u[0] == 0.5 * 2.0 ** -53 and u[1] == 1.0 - 0.5 * 2.0 ** -53


# ------------------------------------------------------------ integrators --

def _harmonic(k):
    return lambda x: -k * x


def _state(n, seed, m=1.0):
    rng = np.random.default_rng(seed)
    x = rng.normal(scale=0.1, size=(n, 3))
    mass = np.full(n, m)
    v = synth.maxwell_boltzmann(mass, 300.0, seed + 1)
    return oi.State(x, v, mass)


def test_respa_one_inner_step_is_baoab():
    k = 50.0
    fs = _harmonic(k)
    fnc = lambda x: -0.3 * k * x + 0.01 * np.sin(x)  # any fast force
    st_a = _state(30, 1)
    st_b = copy.deepcopy(st_a)
    prm = oi.LangevinParams(1.0, 1, 300.0, np.full(30, 5.0), seed=9, stream=2)
    for _ in range(100):
        oi.dmts_nc_step(st_a, fs, fnc, prm)
        oi.baoab_step(st_b, fs, prm)
    assert np.max(np.abs(st_a.x - st_b.x)) <= 1e-12 * np.max(np.abs(st_b.x))
    assert np.max(np.abs(st_a.v - st_b.v)) <= 1e-12 * np.max(np.abs(st_b.v))


def test_respa_with_equal_models_is_n_baoab_steps():
    fs = _harmonic(80.0)
    st_a = _state(25, 2)
    st_b = copy.deepcopy(st_a)
    prm_a = oi.LangevinParams(4.0, 4, 300.0, np.full(25, 2.0), seed=3)
    prm_b = oi.LangevinParams(1.0, 1, 300.0, np.full(25, 2.0), seed=3)
    for _ in range(20):
        oi.dmts_nc_step(st_a, fs, fs, prm_a)
    for _ in range(80):
        oi.baoab_step(st_b, fs, prm_b)
    assert np.array_equal(st_a.x, st_b.x) and np.array_equal(st_a.v, st_b.v)
    assert st_a.step == st_b.step == 80


def test_rewind_never_tripping_is_plain_dmts_nc():
    fs, fnc = _harmonic(60.0), lambda x: -50.0 * x
    a = _state(20, 31)
    b = copy.deepcopy(a)
    prm = oi.LangevinParams(2.0, 4, 300.0, np.full(20, 5.0), seed=7)
    rewinds, seen = oi.dmts_nc_run_rewind(a, fs, fnc, prm, 9, threshold=1e9, save_every=2, sts_after=3)
    for _ in range(9):
        oi.dmts_nc_step(b, fs, fnc, prm)
    assert rewinds == 0 and len(seen) == 9
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v) and a.step == b.step == 36


def test_rewind_returns_to_the_last_saved_frame():
    """Methods, "Preventing rare model disagreements": when the models
    disagree, the run goes back to the last saved frame, takes single time
    steps with the reference force for a while and then multiple time steps
    again.  The fast force here disagrees only during its calls 14-17 (the
    fourth outer step; call 1 is the initial evaluation); frames are saved
    every two outer steps, so the run must equal: two outer steps, (frame)
    two outer steps that the rewind undoes, sts_after BAOAB steps of d from
    the frame with the O-step counter of that frame, a fresh F_NC, then the
    four remaining outer steps."""
    k = 60.0
    fs = _harmonic(k)
    calls = {"n": 0}

    def fnc(x, bad=range(14, 18)):
        calls["n"] += 1
        return -0.8 * k * x + (500.0 if calls["n"] in bad else 0.0)

    prm = oi.LangevinParams(2.0, 4, 300.0, np.full(20, 5.0), seed=11)
    a = _state(20, 32)
    b = copy.deepcopy(a)
    calls["n"] = 0
    rewinds, seen = oi.dmts_nc_run_rewind(a, fs, fnc, prm, 6, threshold=100.0, save_every=2, sts_after=3)
    assert rewinds == 1 and len(seen) == 8 and seen[3] > 100.0 and max(seen[:3] + seen[4:]) < 100.0

    plain = lambda x: -0.8 * k * x
    for _ in range(2):
        oi.dmts_nc_step(b, fs, plain, prm)
    frame = copy.deepcopy(b)
    for _ in range(2):
        oi.dmts_nc_step(b, fs, plain, prm)        # undone by the rewind
    b = frame
    sts = oi.LangevinParams(0.5, 1, 300.0, np.full(20, 5.0), seed=11)
    for _ in range(3):
        oi.baoab_step(b, fs, sts)
    b.f_nc = plain(b.x)
    for _ in range(4):
        oi.dmts_nc_step(b, fs, plain, prm)
    assert b.step == 2 * 4 + 3 + 4 * 4 == a.step
    np.testing.assert_allclose(a.x, b.x, rtol=0, atol=1e-13)
    np.testing.assert_allclose(a.v, b.v, rtol=0, atol=1e-13)


def test_rewind_gives_up_on_a_model_that_always_disagrees():
    fs, fnc = _harmonic(60.0), lambda x: np.full_like(x, 1e3)
    st = _state(10, 33)
    prm = oi.LangevinParams(2.0, 4, 300.0, np.full(10, 5.0), seed=7)
    with pytest.raises(RuntimeError, match="rewind limit"):
        oi.dmts_nc_run_rewind(st, fs, fnc, prm, 3, threshold=1.0, save_every=1, sts_after=2, max_rewinds=5)


def test_baoab_harmonic_configurational_variance():
    """BAOAB samples the exact configurational law of a harmonic oscillator
    for any stable step: <x^2> = k_B T / k per component."""
    n, k, T = 4000, 215.0, 300.0
    st = _state(n, 3)
    st.x = np.zeros((n, 3))
    prm = oi.LangevinParams(2.0, 1, T, np.full(n, 50.0), seed=4)
    fs = _harmonic(k)
    for _ in range(150):
        oi.baoab_step(st, fs, prm)
    acc = []
    for _ in range(200):
        oi.baoab_step(st, fs, prm)
        acc.append(np.mean(st.x ** 2))
    assert abs(np.mean(acc) / (oi.KB * T / k) - 1) < 0.02


def test_temperature_follows_chi_square():
    n, T = 64, 300.0
    st = _state(n, 5)
    st.x = np.zeros((n, 3))
    prm = oi.LangevinParams(2.0, 1, T, np.full(n, 200.0), seed=6)
    zero = lambda x: np.zeros_like(x)
    temps = []
    for step in range(3000):
        oi.baoab_step(st, zero, prm)
        if step >= 100 and step % 3 == 0:
            temps.append(oi.temperature(st.v, st.m))
    mean, sd = oa.chi2_temperature_moments(T, n)
    assert abs(np.mean(temps) - mean) < 0.02 * mean
    assert abs(np.std(temps) / sd - 1) < 0.1


def test_ffl_keeps_direction():
    st = _state(10, 7)
    v0 = st.v.copy()
    prm = oi.LangevinParams(1.0, 1, 300.0, np.full(10, 10.0), seed=1, thermostat="ffl")
    oi._o_step(st, prm, 1.0)
    cos = np.sum(st.v * v0, 1) / np.linalg.norm(st.v, axis=1) / np.linalg.norm(v0, axis=1)
    np.testing.assert_allclose(cos, 1.0, atol=1e-12)


def test_ffl_keeps_maxwell_boltzmann():
    """Fast-Forward Langevin (Methods, "High Hydrogen Friction": the O step
    takes the norm of the Langevin update and the direction of v) leaves the
    Maxwell-Boltzmann law invariant: with zero force, velocities started at
    four times the target temperature relax to T = 300 K with the
    (T/d) chi^2(d) spread, and the reduced speeds |v| sqrt(m / k_B T) follow
    the Maxwell (chi, 3 degrees of freedom) law."""
    n, T = 400, 300.0
    rng = np.random.default_rng(17)
    m = rng.choice([1.008, 3.0, 12.011, 15.999], size=n)
    st = oi.State(np.zeros((n, 3)), 2.0 * synth.maxwell_boltzmann(m, T, 18), m)
    prm = oi.LangevinParams(2.0, 1, T, rng.choice([10.0, 40.0], size=n), seed=19, thermostat="ffl")
    zero = lambda x: np.zeros_like(x)
    temps, speeds = [], []
    for step in range(2400):
        oi.baoab_step(st, zero, prm)
        if step >= 400 and step % 4 == 0:
            temps.append(oi.temperature(st.v, st.m))
        if step >= 400 and step % 50 == 0:
            speeds.append(np.linalg.norm(st.v, axis=1) * np.sqrt(m / (oi.KB * T * oi.ACC)))
    mean, sd = oa.chi2_temperature_moments(T, n)
    assert abs(np.mean(temps) - mean) < 0.01 * mean
    assert abs(np.std(temps) / sd - 1) < 0.1
    assert stats.kstest(np.concatenate(speeds), stats.chi(3).cdf).pvalue > 1e-3


def test_nve_energy_error_is_second_order():
    """Without friction BAOAB is velocity Verlet: with the conservative model
    the total energy fluctuates by O(dt^2) (the O(t^3) local error of the
    Strang splitting, Methods "Multi-time-step integrator"), so halving the
    step divides the fluctuation by about four."""
    from oracle import models as om
    from oracle import neighbors as nb
    spec = synth.ModelSpec("cons", 8, 2, 16, 5.0)
    th = synth.random_weights(spec, 51)
    rng = np.random.default_rng(52)
    n, box = 27, 11.0
    species = rng.integers(0, 4, size=n).astype(np.int32)
    g = np.stack(np.meshgrid(*[np.arange(3)] * 3, indexing="ij"), -1).reshape(-1, 3)
    pos = (g + 0.5) * (box / 3) + rng.normal(scale=0.2, size=(n, 3))
    m = np.full(n, 16.0)   # heavy atoms keep the 80 fs window free of close encounters
    v0 = synth.maxwell_boltzmann(m, 300.0, 53)
    energy = {}

    def force(x):
        e, f = om.cons_energy_forces(spec, th, x, species, box, *nb.pairs_bruteforce(x, box, spec.cutoff))
        energy["e"] = e
        return f

    def fluctuation(dt, steps):
        st = oi.State(pos.copy(), v0.copy(), m.copy())
        prm = oi.LangevinParams(dt, 1, 300.0, np.zeros(n), seed=1)
        h = []
        for _ in range(steps):
            oi.baoab_step(st, force, prm)
            h.append(energy["e"] + oi.kinetic_energy(st.v, st.m))
        h = np.array(h)
        return np.sqrt(np.mean((h - h.mean()) ** 2))

    f = [fluctuation(2.0, 40), fluctuation(1.0, 80), fluctuation(0.5, 160)]
    assert 3.0 < f[0] / f[1] < 5.0 and 3.0 < f[1] / f[2] < 5.0


def test_cell_rescaling_samples_ideal_gas_volume_law():
    """Stochastic cell rescaling with the Langevin thermostat on an ideal gas
    (zero force, W = 0) samples the isothermal-isobaric law
    p(V) ~ V^N exp(-P V / k_B T): <V> = (N + 1) k_B T / P_0 and
    var(V) = (N + 1) (k_B T / P_0)^2.  With N = 4 a k_B T / V drift term in
    d eps would shift <V> by a quarter and a wrong velocity scaling by more."""
    n, T = 4, 300.0
    kT = oi.KB * T
    bp = oi.BarostatParams(1000.0, 4.5e-4, 20.0, 2.0, T, seed=21)
    unit = kT / (bp.pressure_bar * oi.BAR)
    m = np.full(n, 16.0)
    st = oi.State(np.zeros((n, 3)), synth.maxwell_boltzmann(m, T, 22), m)
    prm = oi.LangevinParams(2.0, 1, T, np.full(n, 20.0), seed=23)
    zero = lambda x: np.zeros_like(x)
    box, vols = ((n + 1) * unit) ** (1.0 / 3.0), []
    for step in range(20000):
        oi.baoab_step(st, zero, prm)
        box = oi.scr_barostat_step(st, box, 0.0, bp, step)
        if step >= 500:
            vols.append(box ** 3 / unit)
    vols = np.array(vols)
    assert abs(vols.mean() / (n + 1) - 1) < 0.05
    assert abs(vols.var() / (n + 1) - 1) < 0.2


def test_cell_rescaling_scales_positions_and_velocities_oppositely():
    st = _state(6, 41)
    x0, v0 = st.x.copy(), st.v.copy()
    bp = oi.BarostatParams(1.0, 4.5e-5, 100.0, 4.0, 300.0, seed=5)
    box = oi.scr_barostat_step(st, 20.0, -35.0, bp, 3)
    mu = box / 20.0
    assert mu != 1.0 and st.first_step
    np.testing.assert_allclose(st.x, x0 * mu, rtol=1e-15)
    np.testing.assert_allclose(st.v, v0 / mu, rtol=1e-15)


# -------------------------------------------------------------- HMR/friction --

def test_hmr_keeps_molecule_mass():
    s = synth.solvated_chain(30, 50, seed=5)
    m0 = s.standard_masses()
    m = oi.hmr_masses(s.species, s.bonded_heavy, m0, 3.0, "set")
    for mol in np.unique(s.molecule):
        sel = s.molecule == mol
        assert abs(m[sel].sum() - m0[sel].sum()) < 1e-12
    assert np.all(m[s.species == 0] == 3.0)
    w = synth.water_config(0)
    mw = oi.hmr_masses(w.species, w.bonded_heavy, w.standard_masses(), 3.0, "set")
    np.testing.assert_allclose(mw[w.species == 3], 15.999 - 2 * (3.0 - 1.008), rtol=0, atol=1e-12)
    ma = oi.hmr_masses(w.species, w.bonded_heavy, w.standard_masses(), 3.0, "add")
    np.testing.assert_allclose(ma[w.species == 0], 4.008, atol=1e-12)


def test_friction_table():
    g = oi.friction_per_atom(np.array([0, 3, 1, 0]), [100.0, 1.0, 1.0, 1.0])
    assert list(g) == [100.0, 1.0, 1.0, 100.0]


# ------------------------------------------------------------------- RDF ----

def test_rdf_ideal_gas_is_one():
    rng = np.random.default_rng(0)
    box = 20.0
    pos = rng.uniform(0, box, size=(3000, 3))
    r, g = oa.rdf(pos, box, np.ones(3000, bool), dr=0.5)
    sel = r > 2.0
    assert abs(g[sel].mean() - 1) < 0.01
    assert np.all(np.abs(g[sel] - 1) < 0.1)


def test_rdf_simple_cubic_first_shell():
    a, m = 3.0, 6
    idx = np.arange(m)
    gx, gy, gz = np.meshgrid(idx, idx, idx, indexing="ij")
    pos = a * np.stack([gx.ravel(), gy.ravel(), gz.ravel()], 1).astype(float)
    box = a * m
    n = pos.shape[0]
    dr = 0.05
    r, g = oa.rdf(pos, box, np.ones(n, bool), dr=dr)
    shell = np.abs(r - a) < dr
    edges_lo = r[shell] - dr / 2
    edges_hi = r[shell] + dr / 2
    count = g[shell] * (n - 1) / box ** 3 * 4 / 3 * np.pi * (edges_hi ** 3 - edges_lo ** 3)
    assert abs(count.sum() - 6.0) < 1e-9
