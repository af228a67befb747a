"""Serving: continuous batching gives each replica the same result alone and
in a mix (replicas admitted while others run, retired mid-run, resident ones
moved device to device), a served replica follows the oracle integrator,
admission is bounded by the HBM budget, and latencies are recorded per
replica step."""

import ctypes as C

import numpy as np
import pytest

import synth
from oracle import integrator as oi
from oracle import models as om
from oracle import neighbors as onb

pytestmark = pytest.mark.gpu


def _server(nnp, budget, slots, precision=None, cons_seed=2004, nc_seed=3004):
    from paper_2602_14975_amd import _abi
    kw = {} if precision is None else {"precision": precision}
    cons = nnp.Model.from_spec(synth.CONS_CFG0, synth.random_weights(synth.CONS_CFG0, cons_seed), **kw)
    nc = nnp.Model.from_spec(synth.NC_CFG0, synth.random_weights(synth.NC_CFG0, nc_seed), **kw)
    prm = nnp.respa_params(2.0, 4, 300.0, seed=7, skin=1.0)
    h = C.c_void_p()
    _abi.check(nnp.lib().nnp_server_create(cons.handle, nc.handle, C.byref(prm), int(budget), int(slots),
                                           C.byref(h)))
    return h, (cons, nc)


def _submit(nnp, h, rep, n_steps, seed):
    from paper_2602_14975_amd import _abi
    pos = np.ascontiguousarray(rep.pos, dtype=np.float64)
    m = rep.standard_masses()
    vel = np.ascontiguousarray(synth.maxwell_boltzmann(m, 300.0, seed))
    gamma = np.ones(rep.n)
    sp = np.ascontiguousarray(rep.species, dtype=np.int32)
    d = _abi.ReplicaDesc(rep.n, pos.ctypes.data_as(C.POINTER(C.c_double)), vel.ctypes.data_as(C.POINTER(C.c_double)),
                         m.ctypes.data_as(C.POINTER(C.c_double)), gamma.ctypes.data_as(C.POINTER(C.c_double)),
                         sp.ctypes.data_as(C.POINTER(C.c_int32)), rep.box, seed, seed + 1, n_steps)
    t = C.c_uint64()
    _abi.check(nnp.lib().replica_submit(h, C.byref(d), C.byref(t)))
    return t.value


def _progress(nnp, h, steps):
    from paper_2602_14975_amd import _abi
    nres = C.c_int32()
    _abi.check(nnp.lib().nnp_server_progress(h, int(steps), C.byref(nres)))
    return nres.value


def _drain(nnp, h, steps=8):
    for _ in range(100000):
        if _progress(nnp, h, steps) == 0:
            break


def _result(nnp, h, ticket, n):
    from paper_2602_14975_amd import _abi
    st = _abi.ReplicaStatus()
    pos = np.zeros((n, 3))
    vel = np.zeros((n, 3))
    _abi.check(nnp.lib().replica_poll(h, ticket, C.byref(st), pos.ctypes.data_as(C.POINTER(C.c_double)),
                                      vel.ctypes.data_as(C.POINTER(C.c_double))))
    return st, pos, vel


def _n_latencies(nnp, h):
    n = C.c_int64()
    nnp.lib().nnp_server_step_latencies(h, None, 0, C.byref(n))
    return n.value


def test_alone_equals_mixed(gpu_lib):
    """Replicas 0 and 1 start together; 2 and 3 arrive after two steps, while
    0 and 1 run, and are admitted with 0 and 1 resident; 0 retires after the
    next step (a device repack moves the rest).  Every final state equals
    that of the replica run alone, bit for bit."""
    reps = synth.replica_mix(n_replicas=4, n_min=300, n_max=700)
    steps = [3, 7, 4, 5]
    alone = []
    h, keep = _server(gpu_lib, 2 << 30, 1)
    for k, r in enumerate(reps):
        t = _submit(gpu_lib, h, r, steps[k], 100 + k)
        _drain(gpu_lib, h)
        alone.append(_result(gpu_lib, h, t, r.n))
    gpu_lib.lib().nnp_server_destroy(h)
    h, keep = _server(gpu_lib, 2 << 30, 4)
    tickets = [_submit(gpu_lib, h, r, steps[k], 100 + k) for k, r in enumerate(reps[:2])]
    assert _progress(gpu_lib, h, 2) == 2
    tickets += [_submit(gpu_lib, h, r, steps[k + 2], 102 + k) for k, r in enumerate(reps[2:])]
    assert _progress(gpu_lib, h, 1) == 3          # 0 ran its three steps and left
    _drain(gpu_lib, h, 3)
    for k, (r, t) in enumerate(zip(reps, tickets)):
        st, pos, vel = _result(gpu_lib, h, t, r.n)
        assert st.state == 2 and st.steps_done == steps[k]
        assert np.array_equal(pos, alone[k][1]) and np.array_equal(vel, alone[k][2])
        assert not np.array_equal(pos, r.pos)
    assert _n_latencies(gpu_lib, h) == sum(steps)
    gpu_lib.lib().nnp_server_destroy(h)


def test_budget_binds_residency(gpu_lib):
    """A budget of 2.5 single-replica footprints holds exactly two of three
    equal replicas; the third waits in the queue until one retires."""
    from paper_2602_14975_amd import _abi
    base = synth.replica_mix(n_replicas=1, n_min=500, n_max=501, chain_frac=0.0)[0]
    probe, keep = _server(gpu_lib, 2 << 30, 8)
    b = C.c_size_t()
    _abi.check(gpu_lib.lib().nnp_server_replica_bytes(probe, base.n, base.box, C.byref(b)))
    gpu_lib.lib().nnp_server_destroy(probe)
    h, keep = _server(gpu_lib, int(2.5 * b.value), 8)
    steps = [2, 6, 3]
    tickets = [_submit(gpu_lib, h, base, steps[k], 300 + k) for k in range(3)]
    assert _progress(gpu_lib, h, 1) == 2
    st2, _, _ = _result(gpu_lib, h, tickets[2], base.n)
    assert st2.state == 0
    _drain(gpu_lib, h, 1)
    sts = [_result(gpu_lib, h, t, base.n)[0] for t in tickets]
    assert all(s.state == 2 for s in sts) and [s.steps_done for s in sts] == steps
    assert sts[2].t_admit >= sts[0].t_done > sts[0].t_admit
    assert sts[2].t_admit > sts[2].t_submit
    gpu_lib.lib().nnp_server_destroy(h)


def _oracle_replica(rep, cw, nw, seed, n_outer):
    m = rep.standard_masses()
    st = oi.State(rep.pos.copy(), synth.maxwell_boltzmann(m, 300.0, seed), m.copy())

    def cons_fn(x):
        return om.cons_energy_forces(synth.CONS_CFG0, cw, x, rep.species, rep.box,
                                     *onb.pairs_bruteforce(x, rep.box, synth.CONS_CFG0.cutoff))[1]

    def nc_fn(x):
        return om.nc_forces(synth.NC_CFG0, nw, x, rep.species, rep.box,
                            *onb.pairs_bruteforce(x, rep.box, synth.NC_CFG0.cutoff))

    prm = oi.LangevinParams(2.0, 4, 300.0, np.ones(rep.n), seed=seed, stream=seed + 1)
    for _ in range(n_outer):
        oi.dmts_nc_step(st, cons_fn, nc_fn, prm)
    return st


@pytest.mark.parametrize("bf16", [False, True])
def test_served_replica_matches_oracle(gpu_lib, bf16):
    """A replica with a solvated chain, admitted while two others run and
    served in the mix for three outer steps, against the oracle's DMTS-NC
    integrator with its Philox stream: within 2e-6 A with FP32 models; with
    BF16 perceptrons (force error about 5e-3 relative) within 2e-4 A."""
    from paper_2602_14975_amd import _abi
    reps = synth.replica_mix(n_replicas=3, seed_base=20000, n_min=300, n_max=450, chain_frac=1.0)
    target = reps[0]
    cw = synth.random_weights(synth.CONS_CFG0, 2004)
    nw = synth.random_weights(synth.NC_CFG0, 3004)
    h, keep = _server(gpu_lib, 2 << 30, 3, precision=_abi.NNP_BF16 if bf16 else None)
    others = [_submit(gpu_lib, h, r, 6, 500 + k) for k, r in enumerate(reps[1:])]
    assert _progress(gpu_lib, h, 1) == 2
    t = _submit(gpu_lib, h, target, 3, 400)
    _drain(gpu_lib, h, 2)
    st, pos, vel = _result(gpu_lib, h, t, target.n)
    assert st.state == 2 and st.steps_done == 3
    assert all(_result(gpu_lib, h, o, r.n)[0].state == 2 for o, r in zip(others, reps[1:]))
    ref = _oracle_replica(target, cw, nw, 400, 3)
    dx = float(np.max(np.abs(pos - ref.x)))
    print(f"served replica ({'BF16' if bf16 else 'FP32'}) vs oracle: max |dx| {dx:.2e} A", flush=True)
    assert dx <= (2e-4 if bf16 else 2e-6)
    if not bf16:
        assert np.max(np.abs(vel - ref.v)) <= 1e-5 * np.max(np.abs(ref.v))
    gpu_lib.lib().nnp_server_destroy(h)


def test_rejects_replica_larger_than_budget(gpu_lib):
    from paper_2602_14975_amd import _abi
    reps = synth.replica_mix(n_replicas=1, n_min=3000, n_max=3001)
    h, keep = _server(gpu_lib, 2 << 20, 2)
    with pytest.raises(_abi.NnpError) as e:
        _submit(gpu_lib, h, reps[0], 2, 1)
    assert e.value.code == _abi.NNP_ENOMEM
    gpu_lib.lib().nnp_server_destroy(h)
