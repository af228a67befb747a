"""Dense products of FP32 models on split-bfloat16 matrix cores: parity with
the FP64 oracle and with the float32-operand kernels, ragged row counts (the
row tiles hold 128 atoms) and sparse neighbourhoods, backward and forward
products alike (forces need both)."""

import numpy as np
import pytest

import synth
from synth.weights import ModelSpec
from oracle import models as om
from tests._helpers import FP32_TOL, gpu_list, oracle_list, rel_rmse, small_box

pytestmark = pytest.mark.gpu

SPEC2 = ModelSpec("cons", 128, 2, 16, 5.0)


def _set_dense(nnp, mode):
    from paper_2602_14975_amd import _abi
    _abi.check(nnp.lib().nnp_set_dense_kernels(mode))


def _forces(nnp, spec, w, pos, species, box, list_rc):
    from paper_2602_14975_amd.nnp import DeviceSystem, workspace
    m = nnp.Model.from_spec(spec, w)
    system = DeviceSystem(pos, species, box)
    nl = gpu_list(nnp, system, list_rc)
    ws = workspace(m, None, system.n, 1, nl.capacity)
    e, f = nnp.nnp_cons_energy_forces(m, system, nl, ws)
    return float(e.cpu()[0]), f.cpu().numpy().T.astype(np.float64)


def _oracle(spec, w, pos, species, box):
    off, nbr = oracle_list(pos, box, spec.cutoff)
    return om.cons_energy_forces(spec, w, pos, species, box, off, nbr)


def test_split_bf16_and_fp32_dense_kernels_agree(gpu_lib):
    s = synth.water_config(3)
    spec = synth.CONS_CFG1
    w = synth.random_weights(spec, 5100)
    print(f"case water3 n={s.n} width={spec.width}", flush=True)
    try:
        _set_dense(gpu_lib, 1)
        e32, f32 = _forces(gpu_lib, spec, w, s.pos, s.species, s.box, 6.0)
        _set_dense(gpu_lib, 0)
        ex, fx = _forces(gpu_lib, spec, w, s.pos, s.species, s.box, 6.0)
    finally:
        _set_dense(gpu_lib, 0)
    E, F = _oracle(spec, w, s.pos, s.species, s.box)
    assert rel_rmse(fx, F) <= FP32_TOL and rel_rmse(f32, F) <= FP32_TOL
    assert rel_rmse(fx, f32) <= 2e-6
    assert not np.array_equal(fx, f32)  # the switch selects other kernels
    assert abs(ex - E) <= 1e-6 * abs(E) + 1e-4
    assert abs(ex - e32) <= 1e-6 * abs(E) + 1e-4


def test_dense_mode_rejects_unknown_value(gpu_lib):
    assert gpu_lib.lib().nnp_set_dense_kernels(5) != 0


@pytest.mark.parametrize("n,box", [(40, 30.0), (101, 11.5), (257, 11.5)])
def test_ragged_row_tiles(gpu_lib, n, box):
    """40 atoms: one partial row tile, most rows of it past the end; 101 and
    257: partial last tiles (257 = 2 x 128 + 1)."""
    pos, species, b = small_box(190 + n, n=n, box=box)
    w = synth.random_weights(SPEC2, 5200 + n)
    print(f"case n={n} box={box}", flush=True)
    e, f = _forces(gpu_lib, SPEC2, w, pos, species, b, min(6.0, 0.49 * box))
    E, F = _oracle(SPEC2, w, pos, species, b)
    assert abs(e - E) <= 1e-6 * abs(E) + 1e-4
    assert rel_rmse(f, F) <= FP32_TOL


def test_bf16_models_on_the_same_kernels(gpu_lib):
    """BF16 models: the one-piece products (operands rounded to bfloat16,
    float32 accumulation) against the older BF16 kernels (the same rounding,
    another summation order) and the FP64 oracle."""
    from paper_2602_14975_amd import _abi
    from paper_2602_14975_amd.nnp import DeviceSystem, workspace
    s = synth.water_config(3)
    spec = synth.CONS_CFG1
    w = synth.random_weights(spec, 5300)
    print(f"case bf16 water3 n={s.n}", flush=True)
    out = {}
    try:
        for mode in (1, 0):
            _set_dense(gpu_lib, mode)
            m = gpu_lib.Model.from_spec(spec, w, precision=_abi.NNP_BF16)
            system = DeviceSystem(s.pos, s.species, s.box)
            nl = gpu_list(gpu_lib, system, 6.0)
            ws = workspace(m, None, system.n, 1, nl.capacity)
            e, f = gpu_lib.nnp_cons_energy_forces(m, system, nl, ws)
            out[mode] = f.cpu().numpy().T.astype(np.float64)
    finally:
        _set_dense(gpu_lib, 0)
    E, F = _oracle(spec, w, s.pos, s.species, s.box)
    assert rel_rmse(out[0], F) <= 1e-2 and rel_rmse(out[1], F) <= 1e-2
    assert rel_rmse(out[0], out[1]) <= 2e-3  # roundings to bfloat16 may differ in rare elements
    assert not np.array_equal(out[0], out[1])
