"""Serving: continuous batching gives each replica the same result alone and
in a mix, admission respects slots and the HBM budget, and latencies are
recorded per replica step."""

import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _server(nnp, budget, slots):
    from paper_2602_14975_amd import _abi
    cons = nnp.Model.from_spec(synth.CONS_CFG0, synth.random_weights(synth.CONS_CFG0, 2004))
    nc = nnp.Model.from_spec(synth.NC_CFG0, synth.random_weights(synth.NC_CFG0, 3004))
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


def _drain(nnp, h):
    from paper_2602_14975_amd import _abi
    nres = C.c_int32()
    for _ in range(100000):
        _abi.check(nnp.lib().nnp_server_progress(h, 8, C.byref(nres)))
        if nres.value == 0:
            break


def _result(nnp, h, ticket, n):
    from paper_2602_14975_amd import _abi
    st = _abi.ReplicaStatus()
    pos = np.zeros((n, 3))
    vel = np.zeros((n, 3))
    _abi.check(nnp.lib().replica_poll(h, ticket, C.byref(st), pos.ctypes.data_as(C.POINTER(C.c_double)),
                                      vel.ctypes.data_as(C.POINTER(C.c_double))))
    return st, pos, vel


def test_alone_equals_mixed(gpu_lib):
    reps = synth.replica_mix(n_replicas=4, n_min=300, n_max=700)
    steps = [3, 5, 2, 4]
    alone = []
    h, keep = _server(gpu_lib, 2 << 30, 1)
    for k, r in enumerate(reps):
        t = _submit(gpu_lib, h, r, steps[k], 100 + k)
        _drain(gpu_lib, h)
        alone.append(_result(gpu_lib, h, t, r.n))
    gpu_lib.lib().nnp_server_destroy(h)
    h, keep = _server(gpu_lib, 2 << 30, 4)
    tickets = [_submit(gpu_lib, h, r, steps[k], 100 + k) for k, r in enumerate(reps)]
    _drain(gpu_lib, h)
    for k, (r, t) in enumerate(zip(reps, tickets)):
        st, pos, vel = _result(gpu_lib, h, t, r.n)
        assert st.state == 2 and st.steps_done == steps[k]
        assert np.array_equal(pos, alone[k][1]) and np.array_equal(vel, alone[k][2])
        assert not np.array_equal(pos, r.pos)
    n = C.c_int64()
    gpu_lib.lib().nnp_server_step_latencies(h, None, 0, C.byref(n))
    assert n.value == sum(steps)
    gpu_lib.lib().nnp_server_destroy(h)


def test_budget_limits_residency(gpu_lib):
    reps = synth.replica_mix(n_replicas=3, n_min=400, n_max=500)
    h, keep = _server(gpu_lib, 512 << 20, 8)
    tickets = [_submit(gpu_lib, h, r, 2, 200 + k) for k, r in enumerate(reps)]
    from paper_2602_14975_amd import _abi
    nres = C.c_int32()
    _abi.check(gpu_lib.lib().nnp_server_progress(h, 1, C.byref(nres)))
    assert 1 <= nres.value <= 3
    _drain(gpu_lib, h)
    for t, r in zip(tickets, reps):
        st, _, _ = _result(gpu_lib, h, t, r.n)
        assert st.state == 2 and st.t_admit >= st.t_submit and st.t_done >= st.t_admit
    gpu_lib.lib().nnp_server_destroy(h)


def test_rejects_replica_larger_than_budget(gpu_lib):
    from paper_2602_14975_amd import _abi
    reps = synth.replica_mix(n_replicas=1, n_min=3000, n_max=3001)
    h, keep = _server(gpu_lib, 2 << 20, 2)
    with pytest.raises(_abi.NnpError) as e:
        _submit(gpu_lib, h, reps[0], 2, 1)
    assert e.value.code == _abi.NNP_ENOMEM
    gpu_lib.lib().nnp_server_destroy(h)
