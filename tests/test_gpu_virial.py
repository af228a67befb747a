"""GPU parity of the NPT virials (paper, Methods "Computation of the virial
term in NPT") against the oracle: the conservative virial from the
hand-written reverse pass (vector and matrix-core message kernels), the NC
pair proxy, packed replicas against each alone, and the outer-step
estimator of respa_step along a short DMTS-NC trajectory and for a single
time step."""

import numpy as np
import pytest
import torch

import synth
from oracle import integrator as oi
from oracle import models as om
from oracle import neighbors as onb
from tests._helpers import gpu_list, oracle_list

pytestmark = pytest.mark.gpu

VIR_TOL = 2e-5  # relative, float32 path


def _set_kernels(nnp, mode):
    from paper_2602_14975_amd import _abi
    _abi.check(nnp.lib().nnp_set_message_kernels(mode))


def _cons_virial(nnp, spec, w, s, list_rc):
    from paper_2602_14975_amd.nnp import DeviceSystem, workspace
    m = nnp.Model.from_spec(spec, w)
    system = DeviceSystem(s.pos, s.species, s.box)
    nl = gpu_list(nnp, system, list_rc)
    ws = workspace(m, None, system.n, 1, nl.capacity)
    e, f, W = nnp.nnp_cons_virial(m, system, nl, ws)
    e0, f0 = nnp.nnp_cons_energy_forces(m, system, nl, ws)
    assert torch.equal(f, f0) and torch.equal(e, e0)  # the virial changes nothing else
    return float(W.cpu()[0])


@pytest.mark.parametrize("which,spec,mode", [(0, synth.CONS_CFG0, 0), (3, synth.CONS_CFG1, 0),
                                             (3, synth.CONS_CFG1, 1)])
def test_cons_virial_matches_oracle(gpu_lib, which, spec, mode):
    s = synth.water_config(which)
    w = synth.random_weights(spec, 5100 + which)
    print(f"case water{which} width={spec.width} kernels={mode}", flush=True)
    try:
        _set_kernels(gpu_lib, mode)
        W = _cons_virial(gpu_lib, spec, w, s, spec.cutoff + 1.0)
    finally:
        _set_kernels(gpu_lib, 0)
    off, nbr = oracle_list(s.pos, s.box, spec.cutoff)
    ref = om.cons_virial(spec, w, s.pos, s.species, s.box, off, nbr)
    print(f"W gpu {W:.8g} oracle {ref:.8g}", flush=True)
    assert abs(W - ref) <= VIR_TOL * abs(ref)


@pytest.mark.parametrize("which,spec", [(0, synth.NC_CFG0), (3, synth.NC_CFG1)])
def test_nc_virial_matches_oracle(gpu_lib, which, spec):
    from paper_2602_14975_amd.nnp import DeviceSystem, workspace
    s = synth.water_config(which)
    w = synth.random_weights(spec, 5200 + which)
    m = gpu_lib.Model.from_spec(spec, w)
    system = DeviceSystem(s.pos, s.species, s.box)
    nl = gpu_list(gpu_lib, system, spec.cutoff + 1.0)
    ws = workspace(None, m, system.n, 1, nl.capacity)
    f, W = gpu_lib.nnp_nc_virial(m, system, nl, ws)
    f0 = gpu_lib.nnp_nc_forces(m, system, nl, ws)
    assert torch.equal(f, f0)
    off, nbr = oracle_list(s.pos, s.box, spec.cutoff)
    ref = om.nc_virial_proxy(spec, w, s.pos, s.species, s.box, off, nbr)
    W = float(W.cpu()[0])
    print(f"case water{which} W gpu {W:.8g} oracle {ref:.8g}", flush=True)
    assert abs(W - ref) <= VIR_TOL * abs(ref)


def test_packed_replica_virials_equal_alone(gpu_lib):
    from paper_2602_14975_amd.nnp import DeviceSystem, workspace
    reps = synth.replica_mix(n_replicas=3, n_min=300, n_max=900)
    spec = synth.CONS_CFG1
    m = gpu_lib.Model.from_spec(spec, synth.random_weights(spec, 5300))
    packed = DeviceSystem([r.pos for r in reps], [r.species for r in reps], [r.box for r in reps])
    nl = gpu_list(gpu_lib, packed, 6.0)
    ws = workspace(m, None, packed.n, packed.n_rep, nl.capacity)
    _, _, W = gpu_lib.nnp_cons_virial(m, packed, nl, ws)
    W = W.cpu().numpy()
    for k, r in enumerate(reps):
        alone = DeviceSystem(r.pos, r.species, r.box)
        nl1 = gpu_list(gpu_lib, alone, 5.0)
        ws1 = workspace(m, None, alone.n, 1, nl1.capacity)
        _, _, W1 = gpu_lib.nnp_cons_virial(m, alone, nl1, ws1)
        assert W[k] == float(W1.cpu()[0])


def _estimator_pair(nnp, mode, dt, n_inner, n_outer):
    s = synth.water_config(0)
    masses = s.standard_masses()
    gamma = np.ones(s.n)
    cons_spec, nc_spec = synth.CONS_CFG0, synth.NC_CFG0
    cw = synth.random_weights(cons_spec, 2000)
    nw = synth.random_weights(nc_spec, 3000)
    cons = nnp.Model.from_spec(cons_spec, cw)
    nc = nnp.Model.from_spec(nc_spec, nw)
    v0 = synth.maxwell_boltzmann(masses, 300.0, 5000)
    system = nnp.DeviceSystem(s.pos, s.species, s.box)
    prm = nnp.respa_params(dt, n_inner, 300.0, seed=4000, stream_id=0, mode=mode)
    traj = nnp.Trajectory(cons, nc if mode == "dmts_nc" else None, system, v0, masses, gamma, prm, virial=True)
    traj.respa_step(n_outer)
    W_gpu = float(traj.virial.cpu()[0])

    def cons_fn(x):
        off, nbr = onb.pairs_bruteforce(x, s.box, cons_spec.cutoff)
        return om.cons_energy_forces(cons_spec, cw, x, s.species, s.box, off, nbr)[1]

    def nc_fn(x):
        off, nbr = onb.pairs_bruteforce(x, s.box, nc_spec.cutoff)
        return om.nc_forces(nc_spec, nw, x, s.species, s.box, off, nbr)

    def cons_vir(x):
        off, nbr = onb.pairs_bruteforce(x, s.box, cons_spec.cutoff)
        return om.cons_virial(cons_spec, cw, x, s.species, s.box, off, nbr)

    def nc_vir(x):
        off, nbr = onb.pairs_bruteforce(x, s.box, nc_spec.cutoff)
        return om.nc_virial_proxy(nc_spec, nw, x, s.species, s.box, off, nbr)

    st = oi.State(s.pos.copy(), v0.copy(), masses.copy())
    p = oi.LangevinParams(dt, n_inner if mode == "dmts_nc" else 1, 300.0, gamma, seed=4000, stream=0)
    W_ref = None
    for _ in range(n_outer):
        if mode == "dmts_nc":
            st, W_ref = oi.dmts_nc_step_virial(st, cons_fn, nc_fn, p, cons_vir, nc_vir)
        else:
            oi.baoab_step(st, cons_fn, p)
            W_ref = cons_vir(st.x)
    assert np.max(np.abs(traj.positions() - st.x)) <= 2e-6
    return W_gpu, W_ref


def test_respa_virial_estimator_dmts_nc(gpu_lib):
    W, ref = _estimator_pair(gpu_lib, "dmts_nc", 2.0, 4, 3)
    print(f"estimator gpu {W:.8g} oracle {ref:.8g}", flush=True)
    assert abs(W - ref) <= 1e-4 * abs(ref)


def test_respa_virial_estimator_sts(gpu_lib):
    W, ref = _estimator_pair(gpu_lib, "sts", 0.5, 1, 4)
    print(f"estimator gpu {W:.8g} oracle {ref:.8g}", flush=True)
    assert abs(W - ref) <= 1e-4 * abs(ref)


def test_npt_barostat_matches_oracle(gpu_lib):
    """Stochastic cell rescaling fed by the outer step's virial estimator
    (Methods, "Computation of the virial term in NPT"): six barostat steps,
    each after two DMTS-NC outer steps, on the 192-atom workload.  Box edges
    follow the oracle's within 1e-9 relative, positions within 2e-6 A."""
    nnp = gpu_lib
    s = synth.water_config(0)
    masses = s.standard_masses()
    gamma = np.ones(s.n)
    cons_spec, nc_spec = synth.CONS_CFG0, synth.NC_CFG0
    cw = synth.random_weights(cons_spec, 2000)
    nw = synth.random_weights(nc_spec, 3000)
    v0 = synth.maxwell_boltzmann(masses, 300.0, 5000)
    system = nnp.DeviceSystem(s.pos, s.species, s.box)
    prm = nnp.respa_params(2.0, 4, 300.0, seed=4000)
    traj = nnp.Trajectory(nnp.Model.from_spec(cons_spec, cw), nnp.Model.from_spec(nc_spec, nw), system, v0,
                          masses, gamma, prm, virial=True)
    bp_gpu = nnp.barostat_params(1.0, 4.5e-5, 100.0, 4.0, 300.0, seed=6000)
    boxes_gpu = []
    for k in range(6):
        traj.respa_step(2)
        boxes_gpu.append(float(traj.barostat(bp_gpu, k)[0]))

    box = {"L": s.box}

    def lists(x, rc):
        return onb.pairs_bruteforce(x, box["L"], rc)

    def cons_fn(x):
        return om.cons_energy_forces(cons_spec, cw, x, s.species, box["L"], *lists(x, cons_spec.cutoff))[1]

    def nc_fn(x):
        return om.nc_forces(nc_spec, nw, x, s.species, box["L"], *lists(x, nc_spec.cutoff))

    def cons_vir(x):
        return om.cons_virial(cons_spec, cw, x, s.species, box["L"], *lists(x, cons_spec.cutoff))

    def nc_vir(x):
        return om.nc_virial_proxy(nc_spec, nw, x, s.species, box["L"], *lists(x, nc_spec.cutoff))

    st = oi.State(s.pos.copy(), v0.copy(), masses.copy())
    p = oi.LangevinParams(2.0, 4, 300.0, gamma, seed=4000)
    bp = oi.BarostatParams(1.0, 4.5e-5, 100.0, 4.0, 300.0, seed=6000)
    boxes = []
    for k in range(6):
        for _ in range(2):
            st, W = oi.dmts_nc_step_virial(st, cons_fn, nc_fn, p, cons_vir, nc_vir)
        box["L"] = oi.scr_barostat_step(st, box["L"], W, bp, k)
        boxes.append(box["L"])
    print("boxes gpu", boxes_gpu, "oracle", boxes, flush=True)
    assert abs(boxes[-1] / s.box - 1) > 1e-4          # the cell moved
    np.testing.assert_allclose(boxes_gpu, boxes, rtol=1e-9, atol=0)
    assert np.max(np.abs(traj.positions() - st.x)) <= 2e-6
    assert np.max(np.abs(traj.velocities() - st.v)) <= 1e-5 * np.max(np.abs(st.v))
