"""GPU parity of the cell-list neighbour build against the oracle's brute
force: bit-exact pair sets and row order."""

import math

import numpy as np
import pytest

import synth
from tests._helpers import gpu_list, oracle_list, small_box

pytestmark = pytest.mark.gpu


def _same(nl, off, nbr):
    g_off, g_nbr = nl.rows()
    assert np.array_equal(g_off.astype(np.int64), off)
    assert np.array_equal(g_nbr.astype(np.int64), nbr)


@pytest.mark.parametrize("which", [0, 3, 1])
@pytest.mark.parametrize("rc", [5.0, 3.5, 6.0])
def test_water_boxes_bit_exact(gpu_lib, which, rc):
    from paper_2602_14975_amd.nnp import DeviceSystem
    s = synth.water_config(which)
    print(f"case water{which} rc={rc}", flush=True)
    system = DeviceSystem(s.pos, s.species, s.box)
    nl = gpu_list(gpu_lib, system, rc)
    off, nbr = oracle_list(s.pos, s.box, rc)
    _same(nl, off, nbr)


def test_reverse_index(gpu_lib):
    from paper_2602_14975_amd.nnp import DeviceSystem
    s = synth.water_config(3)
    system = DeviceSystem(s.pos, s.species, s.box)
    nl = gpu_list(gpu_lib, system, 5.0)
    off, nbr = nl.rows()
    rev = nl.rev.cpu().numpy()[: off[-1]]
    rows = np.repeat(np.arange(system.n), np.diff(off))
    assert np.array_equal(nbr[rev], rows) and np.array_equal(rows[rev], nbr)


def test_boundary_cases(gpu_lib):
    from paper_2602_14975_amd.nnp import DeviceSystem
    rc = 5.0
    box = 30.0
    below = math.nextafter(rc, 0.0)
    pos = np.array([[0.0, 0.0, 0.0], [rc, 0.0, 0.0],            # exactly rc: excluded
                    [10.0, 10.0, 10.0], [10.0, 10.0, 10.0 + below],  # one ulp below: included
                    [0.1, 20.0, 20.0], [box - 0.2, 20.0, 20.0],      # across a face
                    [0.05, 0.05, 29.9], [29.95, 29.95, 0.02],        # across a corner
                    [15.0, 25.0, 5.0 + 7 * box],                     # far outside, alone
                    [15.0 - 3 * box, 25.0, 5.0 + 7 * box + 4.0]])    # its neighbour via images
    species = np.zeros(len(pos), np.int32)
    system = DeviceSystem(pos, species, box)
    nl = gpu_list(gpu_lib, system, rc)
    off, nbr = oracle_list(pos, box, rc)
    _same(nl, off, nbr)


@pytest.mark.parametrize("seed", [0, 1])
def test_random_unwrapped_and_dense(gpu_lib, seed):
    from paper_2602_14975_amd.nnp import DeviceSystem
    pos, species, box = small_box(seed, n=700, box=16.0, lo=-40.0)
    system = DeviceSystem(pos, species, box)
    for rc in (3.5, 5.0, 7.9):
        nl = gpu_list(gpu_lib, system, rc)
        off, nbr = oracle_list(pos, box, rc)
        _same(nl, off, nbr)


def test_packed_replicas(gpu_lib):
    from paper_2602_14975_amd.nnp import DeviceSystem
    reps = synth.replica_mix(n_replicas=5, n_min=300, n_max=2500)
    system = DeviceSystem([r.pos for r in reps], [r.species for r in reps], [r.box for r in reps])
    nl = gpu_list(gpu_lib, system, 6.0)
    g_off, g_nbr = nl.rows()
    for k, r in enumerate(reps):
        a0, a1 = system.rep_start[k], system.rep_start[k + 1]
        off, nbr = oracle_list(r.pos, r.box, 6.0)
        rows = g_off[a0:a1 + 1] - g_off[a0]
        assert np.array_equal(rows, off)
        assert np.array_equal(g_nbr[g_off[a0]:g_off[a1]] - a0, nbr)


def test_packed_replicas_beyond_one_scan_tile(gpu_lib):
    """More than 16,384 atoms: the row offsets come from a scan over several
    tiles (the carry between tiles)."""
    from paper_2602_14975_amd.nnp import DeviceSystem
    reps = synth.replica_mix(n_replicas=12, seed_base=770, n_min=1500, n_max=2500, chain_frac=0.0)
    system = DeviceSystem([r.pos for r in reps], [r.species for r in reps], [r.box for r in reps])
    print(f"case {system.n} atoms in {len(reps)} replicas", flush=True)
    assert system.n > 16384
    nl = gpu_list(gpu_lib, system, 3.5)
    g_off, g_nbr = nl.rows()
    for k, r in enumerate(reps):
        a0, a1 = system.rep_start[k], system.rep_start[k + 1]
        off, nbr = oracle_list(r.pos, r.box, 3.5)
        assert np.array_equal(g_off[a0:a1 + 1] - g_off[a0], off)
        assert np.array_equal(g_nbr[g_off[a0]:g_off[a1]] - a0, nbr)


def test_minimal_and_isolated(gpu_lib):
    from paper_2602_14975_amd.nnp import DeviceSystem
    system = DeviceSystem(np.array([[1.0, 1.0, 1.0], [9.0, 9.0, 9.0]]), np.zeros(2, np.int32), 20.0)
    nl = gpu_list(gpu_lib, system, 5.0)
    off, nbr = nl.rows()
    assert list(off) == [0, 0, 0] and nbr.size == 0


def test_capacity_overflow_reports_size(gpu_lib):
    import ctypes as C
    from paper_2602_14975_amd import _abi
    from paper_2602_14975_amd.nnp import DeviceSystem, NeighborList, lib, workspace, _ptr, _stream
    s = synth.water_config(0)
    system = DeviceSystem(s.pos, s.species, s.box)
    nl = NeighborList(system.n, 5.0, 100)
    sentinel = nl.nbr.clone()
    ws = workspace(None, None, system.n, 1, 1)
    cl = nl.c()
    code = lib().nnp_neighbors(C.byref(system.c()), C.byref(cl), _ptr(ws), ws.numel(), _stream())
    assert code == _abi.NNP_ECAPACITY
    off, nbr = oracle_list(s.pos, s.box, 5.0)
    assert cl.n_edges == nbr.size
    assert bool((nl.nbr == sentinel).all())


def test_row_limit_has_its_own_status(gpu_lib):
    """2,400 atoms in a 10.5 A box give about 1,090 neighbours per atom at
    5 A, beyond the builder's 1,024-entry rows: NNP_EROWLIMIT (not the
    growable NNP_ECAPACITY) with the buffers untouched, and the binding
    raises instead of growing."""
    import ctypes as C
    from paper_2602_14975_amd import _abi
    from paper_2602_14975_amd.nnp import DeviceSystem, NeighborList, lib, workspace, _ptr, _stream
    rng = np.random.default_rng(77)
    n = 2400
    system = DeviceSystem(rng.uniform(0.0, 10.5, (n, 3)), np.zeros(n, np.int32), 10.5)
    nl = NeighborList(n, 5.0, 4 << 20)
    sentinel = nl.nbr[:4096].clone()
    ws = workspace(None, None, n, 1, 1)
    cl = nl.c()
    code = lib().nnp_neighbors(C.byref(system.c()), C.byref(cl), _ptr(ws), ws.numel(), _stream())
    assert code == _abi.NNP_EROWLIMIT
    assert bool((nl.nbr[:4096] == sentinel).all())
    with pytest.raises(_abi.NnpError) as e:
        gpu_lib.nnp_neighbors(system, nl, ws)
    assert e.value.code == _abi.NNP_EROWLIMIT and nl.capacity == 4 << 20


def test_rejects_cutoff_above_half_box(gpu_lib):
    from paper_2602_14975_amd import _abi
    from paper_2602_14975_amd.nnp import DeviceSystem, NeighborList, workspace
    s = synth.water_config(0)
    system = DeviceSystem(s.pos, s.species, s.box)
    nl = NeighborList(system.n, 6.3, 100000)
    ws = workspace(None, None, system.n, 1, 1)
    with pytest.raises(_abi.NnpError) as e:
        gpu_lib.nnp_neighbors(system, nl, ws)
    assert e.value.code == _abi.NNP_EINVAL
