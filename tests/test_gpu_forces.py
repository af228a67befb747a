"""GPU parity of the force models against the FP64 oracle (float32 path):
conservative energy and hand-written-reverse forces, NC forces, the NC
weight gradient and the Adam step."""

import numpy as np
import pytest
import torch

import synth
from synth.weights import ModelSpec
from oracle import models as om
from tests._helpers import FP32_TOL, gpu_list, oracle_list, rel_rmse, small_box

pytestmark = pytest.mark.gpu


def _models(nnp, cons_spec, nc_spec, seed):
    cw = synth.random_weights(cons_spec, 2000 + seed)
    nw = synth.random_weights(nc_spec, 3000 + seed)
    return (nnp.Model.from_spec(cons_spec, cw), cw, nnp.Model.from_spec(nc_spec, nw), nw)


def _cons_case(nnp, spec, seed, pos, species, box, list_rc=None):
    from paper_2602_14975_amd.nnp import DeviceSystem, workspace
    w = synth.random_weights(spec, seed)
    m = nnp.Model.from_spec(spec, w)
    system = DeviceSystem(pos, species, box)
    nl = gpu_list(nnp, system, list_rc or spec.cutoff)
    ws = workspace(m, None, system.n, 1, nl.capacity)
    e, f = nnp.nnp_cons_energy_forces(m, system, nl, ws)
    off, nbr = oracle_list(pos, box, spec.cutoff)
    E, F = om.cons_energy_forces(spec, w, pos, species, box, off, nbr)
    return float(e.cpu()[0]), f.cpu().numpy().T.astype(np.float64), E, F


@pytest.mark.parametrize("which,spec", [(0, synth.CONS_CFG0), (3, synth.CONS_CFG1)])
def test_cons_energy_forces_water(gpu_lib, which, spec):
    s = synth.water_config(which)
    print(f"case cons water{which} width={spec.width}", flush=True)
    e, f, E, F = _cons_case(gpu_lib, spec, 2000 + which, s.pos, s.species, s.box)
    assert abs(e - E) <= 1e-6 * abs(E) + 1e-4
    assert rel_rmse(f, F) <= FP32_TOL
    assert np.linalg.norm(f.sum(0)) <= 1e-5 * np.abs(f).sum()


@pytest.mark.parametrize("width", [8, 16, 64])
def test_cons_other_widths_ragged(gpu_lib, width):
    spec = ModelSpec("cons", width, 2, 16, 5.0)
    pos, species, box = small_box(5 + width, n=101, box=11.5)
    e, f, E, F = _cons_case(gpu_lib, spec, 77 + width, pos, species, box)
    assert abs(e - E) <= 1e-6 * abs(E) + 1e-4
    assert rel_rmse(f, F) <= FP32_TOL


def test_cons_verlet_radius_does_not_change_result(gpu_lib):
    from paper_2602_14975_amd.nnp import DeviceSystem, workspace
    s = synth.water_config(3)
    m = gpu_lib.Model.from_spec(synth.CONS_CFG1, synth.random_weights(synth.CONS_CFG1, 5))
    system = DeviceSystem(s.pos, s.species, s.box)
    outs = []
    for rc in (5.0, 6.2):
        nl = gpu_list(gpu_lib, system, rc)
        ws = workspace(m, None, system.n, 1, nl.capacity)
        e, f = gpu_lib.nnp_cons_energy_forces(m, system, nl, ws)
        outs.append((e.cpu().numpy(), f.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_cons_packed_replicas_equal_alone(gpu_lib):
    from paper_2602_14975_amd.nnp import DeviceSystem, workspace
    reps = synth.replica_mix(n_replicas=3, n_min=300, n_max=900)
    spec = synth.CONS_CFG1
    m = gpu_lib.Model.from_spec(spec, synth.random_weights(spec, 9))
    packed = DeviceSystem([r.pos for r in reps], [r.species for r in reps], [r.box for r in reps])
    nl = gpu_list(gpu_lib, packed, 6.0)
    ws = workspace(m, None, packed.n, packed.n_rep, nl.capacity)
    e, f = gpu_lib.nnp_cons_energy_forces(m, packed, nl, ws)
    e, f = e.cpu().numpy(), f.cpu().numpy()
    for k, r in enumerate(reps):
        alone = DeviceSystem(r.pos, r.species, r.box)
        nl1 = gpu_list(gpu_lib, alone, 5.0)
        ws1 = workspace(m, None, alone.n, 1, nl1.capacity)
        e1, f1 = gpu_lib.nnp_cons_energy_forces(m, alone, nl1, ws1)
        a0, a1 = packed.rep_start[k], packed.rep_start[k + 1]
        assert np.array_equal(f[:, a0:a1], f1.cpu().numpy())
        assert e[k] == float(e1.cpu()[0])


def test_cons_full_size_properties(gpu_lib):
    """12,288-atom box at full width: net force, cubic-symmetry equivariance
    and sampled oracle comparison of the energy."""
    from paper_2602_14975_amd.nnp import DeviceSystem, workspace
    s = synth.water_config(1)
    spec = synth.CONS_CFG1
    w = synth.random_weights(spec, 2001)
    m = gpu_lib.Model.from_spec(spec, w)
    res = []
    for perm in ((0, 1, 2), (2, 0, 1)):
        pos = s.pos[:, perm]
        system = DeviceSystem(pos, s.species, s.box)
        nl = gpu_list(gpu_lib, system, 6.0)
        ws = workspace(m, None, system.n, 1, nl.capacity)
        e, f = gpu_lib.nnp_cons_energy_forces(m, system, nl, ws)
        res.append((float(e.cpu()[0]), f.cpu().numpy().T.astype(np.float64)))
    (e0, f0), (e1, f1) = res
    assert abs(e1 - e0) <= 1e-6 * abs(e0)
    assert rel_rmse(f1, f0[:, (2, 0, 1)]) <= FP32_TOL
    assert np.linalg.norm(f0.sum(0)) <= 1e-5 * np.abs(f0).sum()
    off, nbr = oracle_list(s.pos, s.box, spec.cutoff)
    E = om.cons_energy(spec, w, s.pos, s.species, s.box, off, nbr)
    assert abs(e0 - E) <= 1e-6 * abs(E)


@pytest.mark.parametrize("which,spec", [(0, synth.NC_CFG0), (1, synth.NC_CFG1)])
def test_nc_forces_water(gpu_lib, which, spec):
    from paper_2602_14975_amd.nnp import DeviceSystem, workspace
    s = synth.water_config(which)
    print(f"case nc water{which} width={spec.width}", flush=True)
    w = synth.random_weights(spec, 3000 + which)
    m = gpu_lib.Model.from_spec(spec, w)
    system = DeviceSystem(s.pos, s.species, s.box)
    nl = gpu_list(gpu_lib, system, 5.0)  # a larger list: the kernels filter at 3.5 A
    ws = workspace(None, m, system.n, 1, nl.capacity)
    f = gpu_lib.nnp_nc_forces(m, system, nl, ws).cpu().numpy().T.astype(np.float64)
    off, nbr = oracle_list(s.pos, s.box, spec.cutoff)
    F = om.nc_forces(spec, w, s.pos, s.species, s.box, off, nbr)
    assert rel_rmse(f, F) <= FP32_TOL
    assert np.linalg.norm(f.sum(0)) <= 1e-5 * np.abs(f).sum()


@pytest.mark.parametrize("width", [8, 16, 32, 64])
def test_nc_other_widths_ragged(gpu_lib, width):
    """Widths 8, 16 and 32 take the fused update/projection kernel (101
    atoms: a partial last pass of 64, 32 or 16 atoms per block), width 64
    the general GEMM sequence."""
    from paper_2602_14975_amd.nnp import DeviceSystem, workspace
    spec = ModelSpec("nc", width, 1, 8, 3.5)
    pos, species, box = small_box(11 + width, n=101, box=11.5)
    w = synth.random_weights(spec, 300 + width)
    m = gpu_lib.Model.from_spec(spec, w)
    system = DeviceSystem(pos, species, box)
    nl = gpu_list(gpu_lib, system, 3.5)
    ws = workspace(None, m, system.n, 1, nl.capacity)
    f = gpu_lib.nnp_nc_forces(m, system, nl, ws).cpu().numpy().T.astype(np.float64)
    off, nbr = oracle_list(pos, box, spec.cutoff)
    F = om.nc_forces(spec, w, pos, species, box, off, nbr)
    assert rel_rmse(f, F) <= FP32_TOL


def test_nc_weight_gradient(gpu_lib):
    from paper_2602_14975_amd.nnp import DeviceSystem, workspace
    spec = synth.NC_CFG1
    s = synth.water_config(0)
    w = synth.random_weights(spec, 31)
    m = gpu_lib.Model.from_spec(spec, w)
    system = DeviceSystem(s.pos, s.species, s.box)
    nl = gpu_list(gpu_lib, system, 3.5)
    ws = workspace(None, m, system.n, 1, nl.capacity)
    g = np.random.default_rng(4).normal(size=(system.n, 3))
    dl = torch.as_tensor(np.ascontiguousarray(g.T), dtype=torch.float32, device="cuda")
    got = gpu_lib.nnp_nc_weight_grad(m, system, nl, dl, ws).cpu().numpy().astype(np.float64)
    off, nbr = oracle_list(s.pos, s.box, spec.cutoff)
    want = om.nc_weight_grad(spec, w, s.pos, s.species, s.box, off, nbr, g.astype(np.float32).astype(np.float64))
    assert rel_rmse(got, want) <= 1e-4
    # every tensor of the manifest gets its own gradient
    k = 0
    for name, shape in om.layout(spec):
        size = int(np.prod(shape))
        seg_g, seg_w = got[k:k + size], want[k:k + size]
        assert np.linalg.norm(seg_g - seg_w) <= 1e-3 * np.linalg.norm(seg_w) + 1e-6, name
        k += size


def test_adam_matches_torch(gpu_lib):
    torch.manual_seed(0)
    p = torch.randn(1000, device="cuda")
    ref = p.clone().requires_grad_(True)
    opt = torch.optim.Adam([ref], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    for t in range(1, 6):
        g = torch.randn(1000, device="cuda")
        gpu_lib.nnp_adam_step(p, g, m, v, t)
        ref.grad = g.clone()
        opt.step()
    assert torch.allclose(p, ref.detach(), rtol=0, atol=1e-6)


BF16_TOL = 1e-2  # force relative RMSE bound for BF16 perceptrons


@pytest.mark.parametrize("which", ["water", "chain"])
def test_bf16_forces_within_bound(gpu_lib, which):
    from paper_2602_14975_amd import _abi
    from paper_2602_14975_amd.nnp import DeviceSystem, workspace
    if which == "water":
        s = synth.water_config(3)
    else:
        s = synth.solvated_chain(40, 700, seed=77)
    print(f"case bf16 {which} n={s.n}", flush=True)
    cw = synth.random_weights(synth.CONS_CFG1, 2010)
    nw = synth.random_weights(synth.NC_CFG1, 3010)
    cons = gpu_lib.Model.from_spec(synth.CONS_CFG1, cw, precision=_abi.NNP_BF16)
    nc = gpu_lib.Model.from_spec(synth.NC_CFG1, nw, precision=_abi.NNP_BF16)
    system = DeviceSystem(s.pos, s.species, s.box)
    nl = gpu_list(gpu_lib, system, 5.0)
    ws = workspace(cons, nc, system.n, 1, nl.capacity)
    e, f = gpu_lib.nnp_cons_energy_forces(cons, system, nl, ws)
    fn = gpu_lib.nnp_nc_forces(nc, system, nl, ws)
    off, nbr = oracle_list(s.pos, s.box, 5.0)
    E, F = om.cons_energy_forces(synth.CONS_CFG1, cw, s.pos, s.species, s.box, off, nbr)
    off3, nbr3 = oracle_list(s.pos, s.box, 3.5)
    Fn = om.nc_forces(synth.NC_CFG1, nw, s.pos, s.species, s.box, off3, nbr3)
    err_c = rel_rmse(f.cpu().numpy().T, F)
    err_n = rel_rmse(fn.cpu().numpy().T, Fn)
    print(f"bf16 force rel RMSE cons {err_c:.2e} nc {err_n:.2e}", flush=True)
    assert err_c <= BF16_TOL and err_n <= BF16_TOL
    assert err_c > 1e-6  # the BF16 path is really taken
    f64 = f.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(f64.sum(1)) <= 1e-5 * np.abs(f64).sum()


def test_chain_workload_forces_fp32_and_bf16(gpu_lib):
    """The 600-heavy-atom chain of the solvated-chain workload (its seed and
    composition) in 3,500 waters (12,043 atoms; the workload has 30,000):
    FP32 and BF16 conservative and NC forces against the oracle, with the
    workload's model widths."""
    from paper_2602_14975_amd import _abi
    from paper_2602_14975_amd.nnp import DeviceSystem, workspace
    s = synth.solvated_chain(600, 3500, seed=1002)
    print(f"case chain workload n={s.n}", flush=True)
    cw = synth.random_weights(synth.CONS_CFG1, 2004)
    nw = synth.random_weights(synth.NC_CFG1, 3004)
    off, nbr = oracle_list(s.pos, s.box, 5.0)
    E, F = om.cons_energy_forces(synth.CONS_CFG1, cw, s.pos, s.species, s.box, off, nbr)
    off3, nbr3 = oracle_list(s.pos, s.box, 3.5)
    Fn = om.nc_forces(synth.NC_CFG1, nw, s.pos, s.species, s.box, off3, nbr3)
    system = DeviceSystem(s.pos, s.species, s.box)
    nl = gpu_list(gpu_lib, system, 5.0)
    for prec, tol in ((_abi.NNP_FP32, FP32_TOL), (_abi.NNP_BF16, BF16_TOL)):
        cons = gpu_lib.Model.from_spec(synth.CONS_CFG1, cw, precision=prec)
        nc = gpu_lib.Model.from_spec(synth.NC_CFG1, nw, precision=prec)
        ws = workspace(cons, nc, system.n, 1, nl.capacity)
        e, f = gpu_lib.nnp_cons_energy_forces(cons, system, nl, ws)
        fn = gpu_lib.nnp_nc_forces(nc, system, nl, ws)
        err_c = rel_rmse(f.cpu().numpy().T, F)
        err_n = rel_rmse(fn.cpu().numpy().T, Fn)
        print(f"chain workload precision {prec}: force rel RMSE cons {err_c:.2e} nc {err_n:.2e}", flush=True)
        assert err_c <= tol and err_n <= tol
