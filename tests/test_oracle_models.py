"""Pins for the oracle's force models (see oracle/models.py for the list)."""

import math
from dataclasses import replace

import numpy as np
import pytest
import torch
import torch.nn.functional as tF

import synth
from synth.weights import ModelSpec
from oracle import models as om
from oracle import neighbors as nb

SMALL_CONS = ModelSpec("cons", 8, 2, 16, 5.0)
SMALL_NC = ModelSpec("nc", 8, 1, 8, 3.5)


def _cluster(seed, n=24, box=12.0):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, box, size=(n, 3))
    species = rng.integers(0, 4, size=n).astype(np.int32)
    return pos, species, box


def _energy(spec, th, pos, species, box):
    off, nbr = nb.pairs_bruteforce(pos, box, spec.cutoff)
    return om.cons_energy(spec, th, pos, species, box, off, nbr)


def _ef(spec, th, pos, species, box):
    off, nbr = nb.pairs_bruteforce(pos, box, spec.cutoff)
    return om.cons_energy_forces(spec, th, pos, species, box, off, nbr)


def _ncf(spec, th, pos, species, box):
    off, nbr = nb.pairs_bruteforce(pos, box, spec.cutoff)
    return om.nc_forces(spec, th, pos, species, box, off, nbr)


# ------------------------------------------------------------ radial parts --

def test_bessel_closed_form():
    rc = 5.0
    r = torch.tensor([rc / 2], dtype=torch.float64)
    e = om.bessel(r, 16, rc)[0].numpy()
    k = np.arange(1, 17)
    np.testing.assert_allclose(e, math.sqrt(2 / rc) * np.sin(k * math.pi / 2) / (rc / 2), rtol=0, atol=1e-15)
    # small-r limit: sqrt(2/rc) k pi / rc
    e0 = om.bessel(torch.tensor([1e-9], dtype=torch.float64), 4, rc)[0].numpy()
    np.testing.assert_allclose(e0, math.sqrt(2 / rc) * np.arange(1, 5) * math.pi / rc, rtol=1e-12)


@pytest.mark.parametrize("p", [5, 6, 8])
def test_polynomial_envelope(p):
    rc = 3.5
    assert float(om.poly_envelope(torch.tensor([0.0], dtype=torch.float64), rc, p)) == 1.0
    assert float(om.poly_envelope(torch.tensor([rc], dtype=torch.float64), rc, p)) == 0.0
    # derivative in d = r/rc: -p(p+1)(p+2)/2 d^(p-1) (1-d)^2 (zero value, slope, curvature at d=1)
    d = torch.linspace(0.05, 1.0, 40, dtype=torch.float64, requires_grad=True)
    u = om.poly_envelope(d * rc, rc, p)
    (g,) = torch.autograd.grad(u.sum(), d, create_graph=True)
    closed = -p * (p + 1) * (p + 2) / 2 * d.detach() ** (p - 1) * (1 - d.detach()) ** 2
    np.testing.assert_allclose(g.detach().numpy(), closed.numpy(), atol=1e-10)
    (g2,) = torch.autograd.grad(g[-1], d)
    assert abs(float(g2[-1])) < 1e-9


def test_polynomial_envelope_factored_form():
    """The GPU's float32 NC edge values evaluate the p = 5 envelope as
    (1 - d)^3 (1 + 3d + 6d^2 + 10d^3 + 15d^4): the same polynomial as the
    oracle's expanded form (coefficients compared exactly), and in float32
    it keeps its relative precision as d approaches 1."""
    rc = 3.5
    expanded = np.polynomial.Polynomial([1, 0, 0, 0, 0, -21, 35, -15])
    factored = np.polynomial.Polynomial([1, -1]) ** 3 * np.polynomial.Polynomial([1, 3, 6, 10, 15])
    np.testing.assert_array_equal(factored.coef, expanded.coef)
    d = np.linspace(0.0, 1.0, 257)
    u = om.poly_envelope(torch.tensor(d * rc, dtype=torch.float64), rc, 5).numpy()
    np.testing.assert_allclose(factored(d), u, rtol=1e-12, atol=1e-14)  # the expanded form cancels near d = 1
    d32 = np.float32(1.0) - np.float32(2.0) ** -np.arange(2, 20, dtype=np.float32)  # d close to 1
    e = np.float32(1.0) - d32
    q = ((((np.float32(15) * d32 + 10) * d32 + 6) * d32 + 3) * d32 + 1).astype(np.float32)
    f32 = (e * e * e * q).astype(np.float64)
    d64 = d32.astype(np.float64)
    exact = (1.0 - d64) ** 3 * (1 + 3 * d64 + 6 * d64**2 + 10 * d64**3 + 15 * d64**4)  # factored, in float64
    assert np.all(np.abs(f32 / exact - 1) < 1e-6)


def test_cosine_cutoff():
    rc = 5.0
    r = torch.tensor([0.0, rc / 2, rc, rc + 1], dtype=torch.float64, requires_grad=True)
    f = om.cosine_cutoff(r, rc)
    np.testing.assert_allclose(f.detach().numpy(), [1.0, 0.5, 0.0, 0.0], atol=1e-15)
    (g,) = torch.autograd.grad(f.sum(), r)
    assert abs(float(g[2])) < 1e-15


# ----------------------------------------------------------- conservative --

def test_forces_match_finite_differences():
    pos, species, box = _cluster(1)
    th = synth.random_weights(SMALL_CONS, 11)
    _, F = _ef(SMALL_CONS, th, pos, species, box)
    h = 1e-4
    Ffd = np.zeros_like(F)
    for a in range(pos.shape[0]):
        for c in range(3):
            xp = pos.copy(); xp[a, c] += h
            xm = pos.copy(); xm[a, c] -= h
            Ffd[a, c] = -(_energy(SMALL_CONS, th, xp, species, box)
                          - _energy(SMALL_CONS, th, xm, species, box)) / (2 * h)
    assert np.max(np.abs(F - Ffd)) <= 1e-6 * np.max(np.abs(F))


def test_translation_and_net_force():
    pos, species, box = _cluster(2)
    th = synth.random_weights(SMALL_CONS, 12)
    e0, F = _ef(SMALL_CONS, th, pos, species, box)
    e1, F1 = _ef(SMALL_CONS, th, pos + np.array([0.37, -5.1, 13.2]), species, box)
    assert abs(e1 - e0) <= 1e-11 * abs(e0)
    np.testing.assert_allclose(F1, F, atol=1e-10)
    assert np.linalg.norm(F.sum(0)) <= 1e-12 * np.abs(F).sum()


@pytest.mark.parametrize("perm,signs", [((1, 0, 2), (1, 1, 1)), ((2, 0, 1), (-1, 1, -1)),
                                        ((0, 1, 2), (-1, -1, -1))])
def test_cubic_symmetry(perm, signs):
    pos, species, box = _cluster(3)
    th = synth.random_weights(SMALL_CONS, 13)
    e0, F = _ef(SMALL_CONS, th, pos, species, box)
    R = np.zeros((3, 3))
    for a, (b, sg) in enumerate(zip(perm, signs)):
        R[a, b] = sg
    e1, F1 = _ef(SMALL_CONS, th, pos @ R.T, species, box)
    assert abs(e1 - e0) <= 1e-11 * abs(e0)
    np.testing.assert_allclose(F1, F @ R.T, atol=1e-10)


def test_same_species_permutation():
    pos, species, box = _cluster(4)
    th = synth.random_weights(SMALL_CONS, 14)
    e0, F = _ef(SMALL_CONS, th, pos, species, box)
    perm = np.random.default_rng(0).permutation(pos.shape[0])
    e1, F1 = _ef(SMALL_CONS, th, pos[perm], species[perm], box)
    assert abs(e1 - e0) <= 1e-11 * abs(e0)
    np.testing.assert_allclose(F1, F[perm], atol=1e-10)


def _rotation(seed):
    q = np.random.default_rng(seed).normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def test_rotation_of_isolated_cluster():
    rng = np.random.default_rng(5)
    box = 80.0
    pos = rng.uniform(-3, 3, size=(16, 3))
    species = rng.integers(0, 4, size=16).astype(np.int32)
    th = synth.random_weights(SMALL_CONS, 15)
    e0, F = _ef(SMALL_CONS, th, pos + box / 2, species, box)
    R = _rotation(6)
    e1, F1 = _ef(SMALL_CONS, th, pos @ R.T + box / 2, species, box)
    assert abs(e1 - e0) <= 1e-11 * abs(e0)
    np.testing.assert_allclose(F1, F @ R.T, atol=1e-10)


def test_additive_over_distant_clusters():
    s = synth.cluster_pair(7, gap=2 * 5.0 + 1.0)  # > rc apart, no image within rc
    th = synth.random_weights(SMALL_CONS, 16)
    a = s.molecule == 0
    eab = _energy(SMALL_CONS, th, s.pos, s.species, s.box)
    ea = _energy(SMALL_CONS, th, s.pos[a], s.species[a], s.box)
    eb = _energy(SMALL_CONS, th, s.pos[~a], s.species[~a], s.box)
    assert abs(eab - (ea + eb)) <= 1e-11 * abs(eab)


def test_energy_continuous_at_cutoff():
    th = synth.random_weights(SMALL_CONS, 17)
    species = np.array([3, 0], np.int32)
    box = 40.0
    far = _energy(SMALL_CONS, th, np.array([[10.0, 10, 10], [10.0 + 5.5, 10, 10]]), species, box)
    at = _energy(SMALL_CONS, th, np.array([[10.0, 10, 10], [15.0 - 1e-6, 10, 10]]), species, box)
    assert abs(at - far) < 1e-9


def _set(spec, th, name, value):
    p = om.unpack(spec, torch.as_tensor(th.copy()))
    p[name].copy_(torch.as_tensor(value, dtype=torch.float64))
    return torch.cat([p[k].reshape(-1) for k, _ in om.layout(spec)]).numpy()


def test_no_message_reduces_to_perceptrons():
    """Zero radial filter: E_i is the readout of the update-block perceptron
    applied to the species embedding, evaluated with library linear layers."""
    spec = replace(SMALL_CONS, n_layers=1)
    th = synth.random_weights(spec, 18)
    F = spec.width
    th = _set(spec, th, "l0.Wr", np.zeros((3 * F, 16)))
    th = _set(spec, th, "l0.br", np.zeros(3 * F))
    pos, species, box = _cluster(8)
    E = _energy(spec, th, pos, species, box)
    p = om.unpack(spec, torch.as_tensor(th))
    s = p["emb"][torch.as_tensor(species.astype(np.int64))]
    n = torch.full_like(s, 1e-4)
    h = tF.linear(tF.silu(tF.linear(torch.cat([s, n], 1), p["l0.M1"], p["l0.m1"])), p["l0.M2"], p["l0.m2"])
    s = s + h[:, :F]
    Ei = tF.linear(tF.silu(tF.linear(s, p["Wo"], p["bo"])), p["wo"])[:, 0] + p["beta"][torch.as_tensor(species.astype(np.int64))]
    assert abs(E - float(Ei.sum())) <= 1e-12 * abs(E)


def test_dimer_scalar_and_vector_messages():
    """Two atoms of different species, one layer, constant filter bias only:
    the message terms evaluated with library layers."""
    spec = replace(SMALL_CONS, n_layers=1)
    F = spec.width
    th = synth.random_weights(spec, 19)
    th = _set(spec, th, "l0.Wr", np.zeros((3 * F, 16)))
    rng = np.random.default_rng(3)
    br = rng.normal(size=3 * F)
    th = _set(spec, th, "l0.br", br)
    r = 3.1
    pos = np.array([[10.0, 10.0, 10.0], [10.0 + r * 0.6, 10.0 - r * 0.8, 10.0]])
    species = np.array([3, 0], np.int32)
    E = _energy(spec, th, pos, species, 40.0)
    p = om.unpack(spec, torch.as_tensor(th))
    sp = torch.as_tensor(species.astype(np.int64))
    s0 = p["emb"][sp]
    phi = tF.linear(tF.silu(tF.linear(s0, p["l0.W1"], p["l0.b1"])), p["l0.W2"], p["l0.b2"])
    fc = 0.5 * (math.cos(math.pi * r / 5.0) + 1)
    w = torch.as_tensor(br) * fc
    u = torch.tensor([[0.6, -0.8, 0.0], [-0.6, 0.8, 0.0]], dtype=torch.float64)
    s = s0 + torch.stack([phi[1, :F] * w[:F], phi[0, :F] * w[:F]])
    v = torch.stack([u[0][:, None] * (phi[1, 2 * F:] * w[2 * F:])[None, :],
                     u[1][:, None] * (phi[0, 2 * F:] * w[2 * F:])[None, :]])
    Uv = tF.linear(v, p["l0.U"])
    Vv = tF.linear(v, p["l0.V"])
    n = torch.sqrt((Vv ** 2).sum(1) + 1e-8)
    h = tF.linear(tF.silu(tF.linear(torch.cat([s, n], 1), p["l0.M1"], p["l0.m1"])), p["l0.M2"], p["l0.m2"])
    s = s + h[:, :F] + h[:, F:2 * F] * (Uv * Vv).sum(1)
    Ei = tF.linear(tF.silu(tF.linear(s, p["Wo"], p["bo"])), p["wo"])[:, 0] + p["beta"][sp]
    assert abs(E - float(Ei.sum())) <= 1e-12 * abs(E)


# -------------------------------------------------------- non-conservative --

def test_nc_net_force_per_component():
    s = synth.cluster_pair(9, gap=4.0)  # 4 A > 3.5 A: two components
    th = synth.random_weights(SMALL_NC, 21)
    F = _ncf(SMALL_NC, th, s.pos, s.species, s.box)
    for mol in (0, 1):
        sel = s.molecule == mol
        assert np.linalg.norm(F[sel].sum(0)) <= 1e-12 * np.abs(F).sum()
    assert np.abs(F).max() > 1e-3


def test_nc_rotation_equivariance_and_translation():
    rng = np.random.default_rng(10)
    box = 60.0
    pos = rng.uniform(-2.5, 2.5, size=(20, 3))
    species = rng.integers(0, 4, size=20).astype(np.int32)
    th = synth.random_weights(SMALL_NC, 22)
    F = _ncf(SMALL_NC, th, pos + box / 2, species, box)
    R = _rotation(11)
    F1 = _ncf(SMALL_NC, th, pos @ R.T + box / 2, species, box)
    np.testing.assert_allclose(F1, F @ R.T, atol=1e-11)
    F2 = _ncf(SMALL_NC, th, pos + box / 2 + np.array([7.3, -1.1, 33.0]), species, box)
    np.testing.assert_allclose(F2, F, atol=1e-11)


def test_nc_without_vector_heads_is_central():
    """n_l = 0: F_i = sum_j w_ij u_ij with w_ij = (S_ij + S_ji) f_c symmetric."""
    spec = replace(SMALL_NC, n_l=0)
    th = synth.random_weights(spec, 23)
    pos, species, box = _cluster(12, n=20, box=9.0)
    off, nbr = nb.pairs_bruteforce(pos, box, spec.cutoff)
    F = om.nc_forces(spec, th, pos, species, box, off, nbr)
    p = om.unpack(spec, torch.as_tensor(th))
    x = torch.as_tensor(pos)
    s, _, (i, j, r, unit) = om.embed(spec, p, x, species, box, off, nbr)
    q = torch.einsum("hcf,nf->nhc", p["Wq"], s)
    k = torch.einsum("hcf,nf->nhc", p["Wk"], s)
    S_ij = ((q[i] * k[j]).sum(2) / math.sqrt(spec.n_c) * om.bessel(r, spec.n_s, spec.cutoff)).sum(1)
    S_ji = ((q[j] * k[i]).sum(2) / math.sqrt(spec.n_c) * om.bessel(r, spec.n_s, spec.cutoff)).sum(1)
    w = (S_ij + S_ji) * om.poly_envelope(r, spec.cutoff, spec.poly_p)
    expect = torch.zeros(pos.shape[0], 3, dtype=torch.float64).index_add(0, i, w[:, None] * unit)
    np.testing.assert_allclose(F, expect.numpy(), atol=1e-12)


def test_nc_zero_queries_give_zero_force():
    th = synth.random_weights(SMALL_NC, 24)
    H = SMALL_NC.n_s + SMALL_NC.n_l
    th = _set(SMALL_NC, th, "Wq", np.zeros((H, SMALL_NC.n_c, SMALL_NC.width)))
    pos, species, box = _cluster(13, n=20, box=9.0)
    assert np.abs(_ncf(SMALL_NC, th, pos, species, box)).max() == 0.0


def test_nc_weight_gradient_finite_differences():
    pos, species, box = _cluster(14, n=24, box=9.0)
    th = synth.random_weights(SMALL_NC, 25)
    off, nbr = nb.pairs_bruteforce(pos, box, SMALL_NC.cutoff)
    g = np.random.default_rng(1).normal(size=(24, 3))
    grad = om.nc_weight_grad(SMALL_NC, th, pos, species, box, off, nbr, g)

    def L(t):
        return float(np.sum(om.nc_forces(SMALL_NC, t, pos, species, box, off, nbr) * g))

    rng = np.random.default_rng(2)
    h = 1e-6
    for idx in rng.choice(th.size, size=25, replace=False):
        tp = th.copy(); tp[idx] += h
        tm = th.copy(); tm[idx] -= h
        fd = (L(tp) - L(tm)) / (2 * h)
        assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(grad[idx]))
    d = rng.normal(size=th.size)
    fd = (L(th + h * d) - L(th - h * d)) / (2 * h)
    assert abs(fd - grad @ d) <= 1e-6 * max(1.0, abs(fd))


def _pack(spec, named):
    """Flat weight vector in manifest order from a dict of named arrays."""
    return np.concatenate([np.asarray(named[name], dtype=np.float64).reshape(-1)
                           for name, _, _ in synth.weights.manifest(spec)])


def _silu(x):
    return x / (1.0 + np.exp(-x))


def test_nc_dimer_closed_form():
    """Two atoms of different species, hand-set weights (Methods, "Model
    architecture": the equations for q_ih, k_ih, c_ijh, F_ij and F_i).

    With W1 = I, b1 = b2 = 0, Wr = 0 and the update perceptron switched off
    (M1 = 0, m1 = m2 = 0), the embedding after the layer is
        s_i = emb[t_i] + phi_a(j) * br_a u,   v_i = u_ij (phi_c(j) * br_c u)
    with phi(j) = W2 silu(emb[t_j]) and u the p = 5 envelope at d = r/rc.
    Every vector lies on the axis e = u_01, so V_0h = e g0_h and V_1h = -e g1_h
    with g0_h = WV[h] . (phi_c(1) br_c u), g1_h = WV[h] . (phi_c(0) br_c u),
    and the force on atom 0 is, along e,
        u [S_01 (1 + sum_h c_01(ns+h) g0_h) + S_10 (1 + sum_h c_10(ns+h) g1_h)].
    The weights are chosen so that the two plausible misreadings (the
    neighbour's vector heads V_jh in F_ij; c_ijh from q_jh . k_ih) change that
    value, which the test checks as well."""
    spec = SMALL_NC
    F, K, H, nc, ns, nl = spec.width, spec.n_rbf, spec.n_s + spec.n_l, spec.n_c, spec.n_s, spec.n_l
    rng = np.random.default_rng(41)
    w = {name: np.zeros(shape) for name, shape, _ in synth.weights.manifest(spec)}
    w["emb"] = rng.normal(size=(4, F))
    w["l0.W1"] = np.eye(F)
    w["l0.W2"] = rng.normal(size=(3 * F, F)) * 0.5
    w["l0.br"] = rng.normal(size=3 * F)
    w["l0.U"] = rng.normal(size=(F, F))      # unused: the update perceptron is off
    w["l0.V"] = rng.normal(size=(F, F))
    w["l0.M2"] = rng.normal(size=(3 * F, F))
    w["Wq"] = rng.normal(size=(H, nc, F)) * 0.5
    w["Wk"] = rng.normal(size=(H, nc, F)) * 0.5
    w["WV"] = rng.normal(size=(nl, F))
    th = _pack(spec, w)

    r, rc = 2.3, spec.cutoff
    e = np.array([0.6, -0.8, 0.0])
    pos = np.array([[10.0, 10.0, 10.0], 10.0 + r * e])
    species = np.array([3, 0], np.int32)
    Fo = _ncf(spec, th, pos, species, 40.0)

    d = r / rc
    u = 1 - 21 * d**5 + 35 * d**6 - 15 * d**7
    phi = [w["l0.W2"] @ _silu(w["emb"][t]) for t in species]
    wf = w["l0.br"] * u
    s = [w["emb"][species[0]] + phi[1][:F] * wf[:F], w["emb"][species[1]] + phi[0][:F] * wf[:F]]
    vc = [phi[1][2 * F:] * wf[2 * F:], phi[0][2 * F:] * wf[2 * F:]]    # v_0 = e vc0, v_1 = -e vc1
    q = [np.einsum("hcf,f->hc", w["Wq"], si) for si in s]
    k = [np.einsum("hcf,f->hc", w["Wk"], si) for si in s]
    g = [w["WV"] @ vc[0], w["WV"] @ vc[1]]
    c01 = (q[0] * k[1]).sum(1) / math.sqrt(nc)
    c10 = (q[1] * k[0]).sum(1) / math.sqrt(nc)
    B = math.sqrt(2 / rc) * np.sin(np.arange(1, ns + 1) * math.pi * r / rc) / r
    S01, S10 = c01[:ns] @ B, c10[:ns] @ B

    def along(S01, S10, C01, C10, g0, g1):
        return u * (S01 * (1 + C01[ns:] @ g0) + S10 * (1 + C10[ns:] @ g1))

    expect = along(S01, S10, c01, c10, g[0], g[1])
    np.testing.assert_allclose(Fo[0], expect * e, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(Fo[1], -expect * e, rtol=1e-12, atol=1e-14)
    # the configuration tells both misreadings apart from the paper's form
    swapped_v = u * (S01 * (1 - c01[ns:] @ g[1]) + S10 * (1 - c10[ns:] @ g[0]))
    swapped_qk = along(S10, S01, c10, c01, g[0], g[1])
    for alt in (swapped_v, swapped_qk):
        assert abs(alt - expect) > 1e-2 * abs(expect)
