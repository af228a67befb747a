"""Neighbour pairs under periodic boundary conditions (oracle).

The neighbour set N(i) of the paper (Methods, "Model architecture": every
atom j != i within the cutoff) is taken under the minimum-image convention in
a cubic box of edge L.  The decision is made in float64 exactly as follows,
for every ordered pair i != j:

    d     = x_j - x_i                      (per component)
    d     = d - L * rint(d * invL)         invL = 1.0 / L, rint = half-to-even
    r2    = (dx*dx + dy*dy) + dz*dz        left to right, no fused multiply-add
    pair  iff r2 < rc*rc

The set is symmetric (the paper's NPT paragraph relies on this) and each CSR
row lists j in ascending order.  ``pairs_bruteforce`` is the definition;
``pairs_cell_list`` is an independent O(N) construction pinned against it.

Pins (tests/test_oracle_neighbors.py): a pure-Python double loop on tiny
boxes, pairs at exactly rc (excluded) and one ulp below (included), pairs
across every face and corner, symmetry, cell list == brute force.
"""

import math

import numpy as np
import torch


def _decide(xi, xj, box, cutoff):
    """Float64 pair rule on broadcastable torch tensors (..., 3)."""
    inv = 1.0 / box
    d = xj - xi
    d = d - box * torch.round(d * inv)
    dx, dy, dz = d[..., 0], d[..., 1], d[..., 2]
    r2 = (dx * dx + dy * dy) + dz * dz
    return r2 < cutoff * cutoff


def pairs_bruteforce(pos, box, cutoff, row_block=1024):
    """CSR (offsets int64 [N+1], nbr int64 [E]) of all j != i with the rule
    above.  O(N^2) in float64."""
    x = torch.as_tensor(np.asarray(pos, dtype=np.float64))
    n = x.shape[0]
    if not (cutoff < box / 2):
        raise ValueError("cutoff must be below half the box edge")
    counts = np.zeros(n, dtype=np.int64)
    cols = []
    for r0 in range(0, n, row_block):
        r1 = min(n, r0 + row_block)
        m = _decide(x[r0:r1, None, :], x[None, :, :], box, cutoff)
        ar = torch.arange(r0, r1)
        m[ar - r0, ar] = False
        ii, jj = torch.nonzero(m, as_tuple=True)  # row-major: j ascending per row
        counts[r0:r1] = torch.bincount(ii, minlength=r1 - r0).numpy()
        cols.append(jj.numpy().astype(np.int64))
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    nbr = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    return offsets, nbr


def pairs_cell_list(pos, box, cutoff):
    """Same set as ``pairs_bruteforce`` from a cell list: atoms are binned
    into m^3 cells of edge L/m >= cutoff (m >= 3; otherwise every atom is a
    candidate) and only the 27 surrounding cells are tested with the same
    float64 rule."""
    x = np.asarray(pos, dtype=np.float64)
    n = x.shape[0]
    if not (cutoff < box / 2):
        raise ValueError("cutoff must be below half the box edge")
    m = int(math.floor(box / cutoff))
    while m >= 3 and box / m < cutoff * (1.0 + 1e-12):
        m -= 1
    if m < 3:
        return pairs_bruteforce(pos, box, cutoff)
    w = x - box * np.floor(x / box)
    c = np.minimum((w * (m / box)).astype(np.int64), m - 1)
    cid = (c[:, 0] * m + c[:, 1]) * m + c[:, 2]
    members = [[] for _ in range(m ** 3)]
    for a in range(n):
        members[cid[a]].append(a)
    members = [np.array(v, dtype=np.int64) for v in members]
    xt = torch.as_tensor(x)
    rows = []
    for i in range(n):
        cand = []
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    cx, cy, cz = (c[i, 0] + dx) % m, (c[i, 1] + dy) % m, (c[i, 2] + dz) % m
                    cand.append(members[(cx * m + cy) * m + cz])
        cand = np.unique(np.concatenate(cand))
        cand = cand[cand != i]
        ok = _decide(xt[i][None, :], xt[torch.as_tensor(cand)], box, cutoff).numpy()
        rows.append(cand[ok])
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum([r.size for r in rows], out=offsets[1:])
    nbr = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    return offsets, nbr


def edge_index(offsets, nbr):
    """Directed edge endpoints (i, j) for a CSR list."""
    offsets = np.asarray(offsets)
    counts = np.diff(offsets)
    i = np.repeat(np.arange(counts.size, dtype=np.int64), counts)
    return i, np.asarray(nbr, dtype=np.int64)
