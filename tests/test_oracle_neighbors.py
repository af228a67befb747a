"""Pins for the oracle's neighbour rule (brute force on tiny boxes, exact
boundary cases, symmetry, cell list == brute force)."""

import math

import numpy as np
import pytest

import synth
from oracle import neighbors as nb


def _python_pairs(pos, box, rc):
    """Independent pure-Python double loop (math only, float64)."""
    inv = 1.0 / box
    rows = []
    for i in range(len(pos)):
        row = []
        for j in range(len(pos)):
            if i == j:
                continue
            d = []
            for a in range(3):
                t = pos[j][a] - pos[i][a]
                t = t - box * round(t * inv)  # round(): half to even
                d.append(t)
            r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
            if r2 < rc * rc:
                row.append(j)
        rows.append(row)
    return rows


def _rows(offsets, nbr):
    return [list(nbr[offsets[i]:offsets[i + 1]]) for i in range(len(offsets) - 1)]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bruteforce_matches_python_loop(seed):
    rng = np.random.default_rng(seed)
    box = 11.0
    pos = rng.uniform(-box, 2 * box, size=(40, 3))  # unwrapped on purpose
    off, nbr = nb.pairs_bruteforce(pos, box, 5.0)
    assert _rows(off, nbr) == _python_pairs(pos.tolist(), box, 5.0)


def test_exact_cutoff_boundary():
    rc = 5.0
    below = math.nextafter(rc, 0.0)
    pos = np.array([[0.0, 0.0, 0.0], [rc, 0.0, 0.0],          # r == rc: excluded
                    [0.0, 20.0, 0.0], [0.0, 20.0 + 0.0, below]])  # one ulp below: included
    pos[3] = [0.0, 20.0, below]
    off, nbr = nb.pairs_bruteforce(pos, 50.0, rc)
    rows = _rows(off, nbr)
    assert rows[0] == [] and rows[1] == []
    assert rows[2] == [3] and rows[3] == [2]


def test_faces_and_corners():
    box = 12.0
    pos = np.array([[0.1, 6.0, 6.0], [box - 0.2, 6.0, 6.0],       # across the x face
                    [0.1, 0.1, 0.1], [box - 0.1, box - 0.1, box - 0.1],  # across a corner
                    [6.0, 6.0, 6.0 + 3 * box]])                   # far image, same place
    off, nbr = nb.pairs_bruteforce(pos, box, 1.0)
    rows = _rows(off, nbr)
    assert rows[0] == [1] and rows[1] == [0]
    assert rows[2] == [3] and rows[3] == [2]
    off, nbr = nb.pairs_bruteforce(np.array([[6.0, 6.0, 6.0], [6.0, 6.0, 6.5 + 3 * box]]), box, 1.0)
    assert _rows(off, nbr) == [[1], [0]]


def test_symmetric_and_sorted():
    s = synth.water_config(0)
    off, nbr = nb.pairs_bruteforce(s.pos, s.box, 5.0)
    rows = _rows(off, nbr)
    for i, r in enumerate(rows):
        assert r == sorted(r) and i not in r
        for j in r:
            assert i in rows[j]


@pytest.mark.parametrize("which,rc", [(0, 5.0), (0, 3.5), (3, 5.0), (3, 3.5)])
def test_cell_list_equals_bruteforce(which, rc):
    s = synth.water_config(which)
    a = nb.pairs_bruteforce(s.pos, s.box, rc)
    b = nb.pairs_cell_list(s.pos, s.box, rc)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_rejects_large_cutoff():
    with pytest.raises(ValueError):
        nb.pairs_bruteforce(np.zeros((2, 3)), 9.0, 4.5)
