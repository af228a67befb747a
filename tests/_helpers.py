"""Shared setup for the GPU parity tests: seeded inputs for both sides."""

import numpy as np

import synth
from oracle import neighbors as onb

FP32_TOL = 1e-5  # force relative RMSE bound for the float32 path


def rel_rmse(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_list(pos, box, rc):
    return onb.pairs_bruteforce(pos, box, rc)


def gpu_list(nnp, system, rc, capacity=None, with_rev=True):
    from paper_2602_14975_amd.nnp import NeighborList, workspace
    cap = capacity if capacity is not None else int(system.n * 4.0 / 3.0 * np.pi * rc ** 3 * 0.2) + 4096
    nl = NeighborList(system.n, rc, cap, with_rev=with_rev)
    ws = workspace(None, None, system.n, system.n_rep, 1)
    nnp.nnp_neighbors(system, nl, ws)
    return nl


def small_box(seed, n=60, box=11.0, lo=0.0):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(lo, lo + box, size=(n, 3))
    species = rng.integers(0, 4, size=n).astype(np.int32)
    return pos, species, box
