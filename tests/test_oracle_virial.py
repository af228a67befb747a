"""Pins of the oracle's NPT virials (paper, Methods "Computation of the
virial term in NPT"): W = -sum_i F_i . q_i for the conservative model
against finite differences of the energy under uniform scaling and against
-sum_i F_i . q_i on an isolated cluster; the NC proxy sum_ij F_ij . r_ij
against -sum_i F_i . q_i on an isolated cluster (the paper's identity); the
outer-step estimator's reductions (one inner step; equal models)."""

import copy

import numpy as np
import pytest

import synth
from synth.weights import ModelSpec
from oracle import integrator as oi
from oracle import models as om
from oracle import neighbors as nb

SMALL_CONS = ModelSpec("cons", 8, 2, 16, 5.0)
SMALL_NC = ModelSpec("nc", 8, 1, 8, 3.5)


def _lists(pos, box, rc):
    return nb.pairs_bruteforce(pos, box, rc)


def _isolated(seed, n=18, spread=3.0, box=60.0):
    """Atoms within a few A of the centre of a large box: no pair crosses a
    periodic boundary, so q_i is unambiguous."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-spread, spread, size=(n, 3)) + box / 2
    species = rng.integers(0, 4, size=n).astype(np.int32)
    return pos, species, box


def test_cons_virial_is_scaling_derivative_of_energy():
    s = synth.water_config(0)
    th = synth.random_weights(SMALL_CONS, 31)
    off, nbr = _lists(s.pos, s.box, SMALL_CONS.cutoff)
    W = om.cons_virial(SMALL_CONS, th, s.pos, s.species, s.box, off, nbr)
    h = 1e-5
    ep = om.cons_energy(SMALL_CONS, th, s.pos * (1 + h), s.species, s.box * (1 + h), off, nbr)
    em = om.cons_energy(SMALL_CONS, th, s.pos * (1 - h), s.species, s.box * (1 - h), off, nbr)
    fd = (ep - em) / (2 * h)
    assert abs(W - fd) <= 1e-7 * max(abs(W), 1.0)
    assert abs(W) > 1.0  # not trivially zero


def test_cons_virial_equals_minus_q_dot_f_on_isolated_cluster():
    pos, species, box = _isolated(5)
    th = synth.random_weights(SMALL_CONS, 32)
    off, nbr = _lists(pos, box, SMALL_CONS.cutoff)
    _, F = om.cons_energy_forces(SMALL_CONS, th, pos, species, box, off, nbr)
    W = om.cons_virial(SMALL_CONS, th, pos, species, box, off, nbr)
    ref = -float((F * pos).sum())
    assert abs(W - ref) <= 1e-10 * np.abs(F * pos).sum()


def test_nc_proxy_equals_minus_q_dot_f_on_isolated_cluster():
    pos, species, box = _isolated(6, n=24, spread=2.5)
    th = synth.random_weights(SMALL_NC, 33)
    off, nbr = _lists(pos, box, SMALL_NC.cutoff)
    F = om.nc_forces(SMALL_NC, th, pos, species, box, off, nbr)
    W = om.nc_virial_proxy(SMALL_NC, th, pos, species, box, off, nbr)
    ref = -float((F * pos).sum())
    assert abs(W - ref) <= 1e-10 * np.abs(F * pos).sum()
    assert abs(W) > 1e-6


def test_nc_proxy_is_translation_invariant():
    s = synth.water_config(0)
    th = synth.random_weights(SMALL_NC, 34)
    off, nbr = _lists(s.pos, s.box, SMALL_NC.cutoff)
    W0 = om.nc_virial_proxy(SMALL_NC, th, s.pos, s.species, s.box, off, nbr)
    shifted = (s.pos + np.array([1.3, -2.1, 0.7])) % s.box
    off1, nbr1 = _lists(shifted, s.box, SMALL_NC.cutoff)
    W1 = om.nc_virial_proxy(SMALL_NC, th, shifted, s.species, s.box, off1, nbr1)
    assert abs(W1 - W0) <= 1e-10 * abs(W0)


def _harmonic(k):
    return lambda x: -k * x


def _harmonic_virial(k):
    return lambda x: float(k * (x * x).sum())  # -sum F.q with F = -k q


def _state(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(scale=0.1, size=(n, 3))
    mass = np.ones(n)
    v = synth.maxwell_boltzmann(mass, 300.0, seed + 1)
    return oi.State(x, v, mass)


def test_estimator_with_one_inner_step_is_the_end_virial():
    fs, ws = _harmonic(50.0), _harmonic_virial(50.0)
    fnc = lambda x: -20.0 * x
    wnc = _harmonic_virial(20.0)
    st = _state(20, 3)
    prm = oi.LangevinParams(1.0, 1, 300.0, np.full(20, 5.0), seed=9)
    for _ in range(5):
        st, W = oi.dmts_nc_step_virial(st, fs, fnc, prm, ws, wnc)
        assert abs(W - ws(st.x)) <= 1e-12 * abs(W)


def test_estimator_with_equal_models_is_the_inner_average():
    fs, ws = _harmonic(80.0), _harmonic_virial(80.0)
    st_a = _state(25, 4)
    st_b = copy.deepcopy(st_a)
    prm_a = oi.LangevinParams(4.0, 4, 300.0, np.full(25, 2.0), seed=3)
    prm_b = oi.LangevinParams(1.0, 1, 300.0, np.full(25, 2.0), seed=3)
    for _ in range(3):
        st_a, W = oi.dmts_nc_step_virial(st_a, fs, fs, prm_a, ws, ws)
        inner = []
        for _ in range(4):
            oi.baoab_step(st_b, fs, prm_b)
            inner.append(ws(st_b.x))
        assert np.array_equal(st_a.x, st_b.x)
        assert abs(W - sum(inner) / 4) <= 1e-12 * abs(W)
