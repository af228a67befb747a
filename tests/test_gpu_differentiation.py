"""Differentiation: autograd wrappers over the hand-written reverse passes,
the force-MSE loss kernel, finite differences on the 1,536-atom box, and a
short distillation run."""

import numpy as np
import pytest
import torch

import synth
from oracle import models as om
from oracle import neighbors as onb
from tests._helpers import FP32_TOL, gpu_list, rel_rmse

pytestmark = pytest.mark.gpu


def test_cons_energy_autograd_equals_minus_forces(gpu_lib):
    from paper_2602_14975_amd.autograd import ConsEnergy
    s = synth.water_config(0)
    w = synth.random_weights(synth.CONS_CFG0, 2000)
    m = gpu_lib.Model.from_spec(synth.CONS_CFG0, w)
    system = gpu_lib.DeviceSystem(s.pos, s.species, s.box)
    nl = gpu_list(gpu_lib, system, 5.0)
    ws = gpu_lib.workspace(m, None, system.n, 1, nl.capacity)
    pos = system.pos.clone().requires_grad_(True)
    e = ConsEnergy.apply(pos, m, system, nl, ws)
    (3.0 * e.sum()).backward()
    _, f = gpu_lib.nnp_cons_energy_forces(m, system, nl, ws)
    assert torch.equal(pos.grad, -3.0 * f.double())
    off, nbr = onb.pairs_bruteforce(s.pos, s.box, 5.0)
    _, F = om.cons_energy_forces(synth.CONS_CFG0, w, s.pos, s.species, s.box, off, nbr)
    assert rel_rmse(-pos.grad.cpu().numpy().T / 3.0, F) <= FP32_TOL


def test_cons_forces_finite_differences_1536(gpu_lib):
    """Hand-written reverse on the 1,536-atom box at full width against
    central differences (h = 1e-4 A) of the FP64 oracle energy on sampled
    atoms, and against the oracle gradient on all atoms."""
    s = synth.water_config(3)
    spec = synth.CONS_CFG1
    w = synth.random_weights(spec, 2003)
    m = gpu_lib.Model.from_spec(spec, w)
    system = gpu_lib.DeviceSystem(s.pos, s.species, s.box)
    nl = gpu_list(gpu_lib, system, 5.0)
    ws = gpu_lib.workspace(m, None, system.n, 1, nl.capacity)
    _, f = gpu_lib.nnp_cons_energy_forces(m, system, nl, ws)
    f = f.cpu().numpy().T.astype(np.float64)
    off, nbr = onb.pairs_bruteforce(s.pos, s.box, 5.0)
    _, F = om.cons_energy_forces(spec, w, s.pos, s.species, s.box, off, nbr)
    assert rel_rmse(f, F) <= FP32_TOL
    h = 1e-4
    for a in (0, 1, 700):
        for c in range(3):
            xp = s.pos.copy(); xp[a, c] += h
            xm = s.pos.copy(); xm[a, c] -= h
            ep = om.cons_energy(spec, w, xp, s.species, s.box, *onb.pairs_cell_list(xp, s.box, 5.0))
            em = om.cons_energy(spec, w, xm, s.species, s.box, *onb.pairs_cell_list(xm, s.box, 5.0))
            fd = -(ep - em) / (2 * h)
            assert abs(f[a, c] - fd) <= 1e-4 * max(1.0, abs(fd))


def test_nc_forces_autograd_weight_gradient(gpu_lib):
    from paper_2602_14975_amd.autograd import NCForces
    spec = synth.NC_CFG1
    s = synth.water_config(0)
    w = synth.random_weights(spec, 41)
    m = gpu_lib.Model.from_spec(spec, w)
    system = gpu_lib.DeviceSystem(s.pos, s.species, s.box)
    nl = gpu_list(gpu_lib, system, 3.5)
    ws = gpu_lib.workspace(None, m, system.n, 1, nl.capacity)
    theta = torch.as_tensor(w.astype(np.float32), device="cuda").requires_grad_(True)
    G = np.random.default_rng(7).normal(size=(3, system.n)).astype(np.float32)
    f = NCForces.apply(theta, system.pos, m, system, nl, ws)
    (f * torch.as_tensor(G, device="cuda")).sum().backward()
    off, nbr = onb.pairs_bruteforce(s.pos, s.box, 3.5)
    want = om.nc_weight_grad(spec, w, s.pos, s.species, s.box, off, nbr, G.T.astype(np.float64))
    assert rel_rmse(theta.grad.cpu().numpy(), want) <= 1e-4


def test_force_mse_kernel(gpu_lib):
    torch.manual_seed(1)
    f = torch.randn(3, 1001, device="cuda")
    r = torch.randn(3, 1001, device="cuda")
    ws = torch.empty(8192, dtype=torch.uint8, device="cuda")
    g = torch.empty_like(f)
    loss, _ = gpu_lib.nnp_force_mse(f, r, ws, grad=g)
    d = (f - r).double()
    assert abs(loss.item() - float((d * d).mean())) <= 1e-12 * float((d * d).mean())
    assert torch.allclose(g, (2 * (f - r) / f.numel()), rtol=1e-6, atol=1e-9)


def test_short_distillation_lowers_rmse(gpu_lib):
    from paper_2602_14975_amd import distill
    s = synth.water_config(3)
    cons = gpu_lib.Model.from_spec(synth.CONS_CFG0, synth.random_weights(synth.CONS_CFG0, 2003))
    nw = synth.random_weights(synth.NC_CFG1, 3003)
    nc = gpu_lib.Model.from_spec(synth.NC_CFG1, nw)
    m = s.standard_masses()
    pos, frc = distill.generate_frames(cons, s, m, np.ones(s.n), n_frames=24, equil_steps=40, every=10)
    assert torch.isfinite(pos).all() and torch.isfinite(frc).all()
    d, hist = distill.train(nc, nw, pos, frc, s.species, s.box, s.n, steps=150, n_val=8, batch=4, lr=1e-3,
                            log_every=50)
    print("distillation rmse history", hist)
    assert hist[-1][1] < 0.9 * hist[0][1]
