"""Seeded synthetic atomic systems.

Every builder takes an explicit seed and returns a :class:`System` whose arrays
are plain numpy (positions float64 (N, 3) in Angstrom, unwrapped; species int32
with H=0, C=1, N=2, O=3).  The systems stand in for the paper's bulk-water
boxes (Table 1) and solvated proteins (Table 2), which are not available:

* ``water_box``: rigid waters (O-H 0.96 A, H-O-H 104.5 deg), uniformly random
  orientations, oxygens on a simple-cubic lattice with a per-molecule Gaussian
  jitter (the molecule is translated as a whole, so its geometry stays rigid).
* ``solvated_chain``: a self-avoiding random walk of C/N/O heavy atoms (bond
  1.5 A, bond angle uniform in 109.5 +- 10 deg, uniform dihedral, no heavy atom
  closer than 3 A to an earlier non-adjacent one), hydrogens filling the
  remaining valences at 1.09 A along tetrahedral directions, and waters on a
  lattice with sites closer than 2.6 A to the chain removed.
* ``replica_mix``: the serving workload, replicas with log-uniform sizes.

The ``bonded_heavy`` array gives, for every hydrogen, the index of the heavy
atom it is bonded to (-1 for heavy atoms); hydrogen mass repartitioning needs
it.  ``molecule`` numbers the molecules (the chain is one molecule).
"""

from dataclasses import dataclass, field
import math

import numpy as np

SPECIES = ("H", "C", "N", "O")
SPECIES_INDEX = {s: i for i, s in enumerate(SPECIES)}
# IUPAC standard atomic weights (amu), indexed by species.
MASS_AMU = np.array([1.008, 12.011, 14.007, 15.999], dtype=np.float64)

WATER_DENSITY = 0.1003  # atoms per cubic Angstrom for water at 1 g/cm^3

_KB_KCAL = 8.31446261815324 / 4184.0  # kcal/mol/K
_ACC = 4.184e-4                        # (kcal/mol/A/amu) -> A/fs^2


@dataclass
class System:
    pos: np.ndarray            # (N, 3) float64, unwrapped
    species: np.ndarray        # (N,) int32
    box: float                 # cubic edge, Angstrom
    bonded_heavy: np.ndarray   # (N,) int32, -1 for heavy atoms
    molecule: np.ndarray       # (N,) int32
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.pos.shape[0])

    def standard_masses(self):
        return MASS_AMU[self.species]


def _random_rotations(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _water_template():
    half = math.radians(104.5 / 2.0)
    d = 0.96
    return np.array([[0.0, 0.0, 0.0],
                     [d * math.sin(half), d * math.cos(half), 0.0],
                     [-d * math.sin(half), d * math.cos(half), 0.0]])


def _place_waters(rng, centers, jitter):
    """Rigid waters (O, H, H) at ``centers`` with random rotations and a
    per-molecule jitter."""
    nw = centers.shape[0]
    R = _random_rotations(rng, nw)
    shift = rng.normal(scale=jitter, size=(nw, 3)) if jitter > 0 else np.zeros((nw, 3))
    tmpl = _water_template()
    pos = centers[:, None, :] + shift[:, None, :] + np.einsum("nab,kb->nka", R, tmpl)
    return pos.reshape(-1, 3)


def water_box(n_per_dim, box, seed, jitter=0.1, name=""):
    """``n_per_dim**3`` waters on a simple-cubic lattice in a cubic box."""
    rng = np.random.default_rng(seed)
    a = box / n_per_dim
    idx = np.arange(n_per_dim)
    gi, gj, gk = np.meshgrid(idx, idx, idx, indexing="ij")
    centers = (np.stack([gi.ravel(), gj.ravel(), gk.ravel()], axis=1) + 0.5) * a
    pos = _place_waters(rng, centers, jitter)
    nw = centers.shape[0]
    species = np.tile(np.array([3, 0, 0], dtype=np.int32), nw)
    first = 3 * np.arange(nw, dtype=np.int32)
    bonded = np.stack([np.full(nw, -1, np.int32), first, first], axis=1).ravel()
    molecule = np.repeat(np.arange(nw, dtype=np.int32), 3)
    return System(pos, species, float(box), bonded.astype(np.int32), molecule,
                  name=name or f"water{3 * nw}", meta={"n_waters": nw, "seed": seed})


def water_config(k):
    """The water boxes used by the named workloads (k = 0, 1, 3)."""
    if k == 0:
        return water_box(4, 12.42, 1000, name="water192")
    if k == 1:
        return water_box(16, 49.6, 1001, name="water12288")
    if k == 3:
        return water_box(8, 24.834, 1003, name="water1536")
    raise ValueError(k)


def _mic(d, box):
    return d - box * np.round(d / box)


def _unit(v):
    return v / np.linalg.norm(v)


def _perp_basis(u):
    a = np.array([1.0, 0.0, 0.0]) if abs(u[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    p = _unit(np.cross(u, a))
    q = np.cross(u, p)
    return p, q


def _nerf(a, b, c, bond, angle, dihedral):
    """Place d so that |cd| = bond, angle(b, c, d) = angle, dihedral(a,b,c,d)."""
    bc = _unit(c - b)
    n = np.cross(b - a, bc)
    nn = np.linalg.norm(n)
    if nn < 1e-8:
        p, _ = _perp_basis(bc)
        n = p
    else:
        n = n / nn
    m = np.cross(n, bc)
    d2 = np.array([-bond * math.cos(angle),
                   bond * math.sin(angle) * math.cos(dihedral),
                   bond * math.sin(angle) * math.sin(dihedral)])
    return c + d2[0] * bc + d2[1] * m + d2[2] * n


def _random_walk(rng, n_heavy, box, start):
    bond = 1.5
    pts = [np.array(start, dtype=np.float64)]
    trials_left = 200000

    def ok(p, k):
        if k <= 2:
            return True
        prev = np.array(pts[: k - 2])
        d = _mic(prev - p, box)
        return bool(np.all(np.einsum("ij,ij->i", d, d) >= 9.0))

    while len(pts) < n_heavy:
        k = len(pts)
        placed = False
        for _ in range(100):
            trials_left -= 1
            if trials_left <= 0:
                raise RuntimeError("random walk could not be completed")
            if k == 1:
                p = pts[0] + bond * _unit(rng.normal(size=3))
            else:
                ang = math.radians(rng.uniform(99.5, 119.5))
                dih = rng.uniform(0.0, 2 * math.pi)
                if k == 2:
                    u = _unit(pts[1] - pts[0])
                    pp, qq = _perp_basis(u)
                    a = pts[0] - (pp * math.cos(dih) + qq * math.sin(dih))
                else:
                    a = pts[k - 3]
                p = _nerf(a, pts[k - 2], pts[k - 1], bond, ang, dih)
            if ok(p, k):
                pts.append(p)
                placed = True
                break
        if not placed and len(pts) > 1:
            pts.pop()  # backtrack one atom
    return np.array(pts)


_VALENCE = {1: 4, 2: 3, 3: 2}
_TET = math.acos(-1.0 / 3.0)  # 109.47 deg


def _hydrogens(heavy_pos, heavy_species, rng):
    nh = heavy_pos.shape[0]
    hpos, hbond = [], []
    for a in range(nh):
        nbrs = [b for b in (a - 1, a + 1) if 0 <= b < nh]
        n_h = _VALENCE[int(heavy_species[a])] - len(nbrs)
        if n_h <= 0:
            continue
        us = [_unit(heavy_pos[b] - heavy_pos[a]) for b in nbrs]
        dirs = []
        if len(us) == 2:
            d = -(us[0] + us[1])
            dn = np.linalg.norm(d)
            d = d / dn if dn > 1e-8 else _perp_basis(us[0])[0]
            nrm = np.cross(us[0], us[1])
            nn = np.linalg.norm(nrm)
            nrm = nrm / nn if nn > 1e-8 else _perp_basis(d)[0]
            half = _TET / 2.0
            if n_h == 1:
                dirs = [d]
            else:
                dirs = [d * math.cos(half) + nrm * math.sin(half),
                        d * math.cos(half) - nrm * math.sin(half)]
        else:
            u = us[0]
            p, q = _perp_basis(u)
            phi0 = rng.uniform(0.0, 2 * math.pi)
            for kk in range(n_h):
                phi = phi0 + 2 * math.pi * kk / 3.0
                dirs.append(u * math.cos(_TET) + math.sin(_TET) * (p * math.cos(phi) + q * math.sin(phi)))
        for d in dirs[:n_h]:
            hpos.append(heavy_pos[a] + 1.09 * d)
            hbond.append(a)
    if not hpos:
        return np.zeros((0, 3)), np.zeros(0, np.int32)
    return np.array(hpos), np.array(hbond, dtype=np.int32)


def solvated_chain(n_heavy, n_waters, seed, box=None, name="", jitter=0.1):
    """A random-walk C/N/O chain with hydrogens, solvated by ``n_waters``."""
    rng = np.random.default_rng(seed)
    heavy_species = rng.choice(np.array([1, 2, 3], dtype=np.int32), size=n_heavy,
                               p=[0.70, 0.15, 0.15]).astype(np.int32)
    n_bonds = np.full(n_heavy, 2)
    n_bonds[0] -= 1
    n_bonds[-1] -= 1
    n_hyd = int(sum(max(_VALENCE[int(s)] - int(b), 0) for s, b in zip(heavy_species, n_bonds)))
    n_total = n_heavy + n_hyd + 3 * n_waters
    if box is None:
        box = (n_total / WATER_DENSITY) ** (1.0 / 3.0)
    heavy = _random_walk(rng, n_heavy, box, start=np.full(3, box / 2.0))
    hpos, hbond = _hydrogens(heavy, heavy_species, rng)
    chain_pos = np.concatenate([heavy, hpos], axis=0)
    n_chain = chain_pos.shape[0]

    m = int(math.ceil((1.1 * n_waters) ** (1.0 / 3.0)))
    while True:
        a = box / m
        idx = np.arange(m)
        gi, gj, gk = np.meshgrid(idx, idx, idx, indexing="ij")
        sites = (np.stack([gi.ravel(), gj.ravel(), gk.ravel()], axis=1) + 0.5) * a
        keep = np.ones(sites.shape[0], dtype=bool)
        for c0 in range(0, n_chain, 256):
            blk = chain_pos[c0:c0 + 256]
            d = _mic(sites[:, None, :] - blk[None, :, :], box)
            keep &= np.all(np.einsum("sci,sci->sc", d, d) >= 2.6 ** 2, axis=1)
        surv = np.nonzero(keep)[0]
        if surv.size >= n_waters:
            break
        m += 1
    chosen = np.sort(rng.permutation(surv)[:n_waters])
    wpos = _place_waters(rng, sites[chosen], jitter)

    pos = np.concatenate([chain_pos, wpos], axis=0)
    species = np.concatenate([heavy_species, np.zeros(hpos.shape[0], np.int32),
                              np.tile(np.array([3, 0, 0], np.int32), n_waters)])
    wfirst = n_chain + 3 * np.arange(n_waters, dtype=np.int32)
    bonded = np.concatenate([np.full(n_heavy, -1, np.int32), hbond,
                             np.stack([np.full(n_waters, -1, np.int32), wfirst, wfirst], axis=1).ravel()])
    molecule = np.concatenate([np.zeros(n_chain, np.int32),
                               np.repeat(1 + np.arange(n_waters, dtype=np.int32), 3)])
    return System(pos, species.astype(np.int32), float(box), bonded.astype(np.int32), molecule,
                  name=name or f"chain{n_heavy}_water{n_waters}",
                  meta={"n_heavy": n_heavy, "n_chain_h": int(hpos.shape[0]), "n_waters": n_waters,
                        "seed": seed})


def replica_mix(n_replicas=256, seed_base=10000, n_min=300, n_max=6000, chain_frac=0.3):
    """Serving replicas: sizes log-uniform on [n_min, n_max], a fraction with a
    20-100 heavy-atom chain, waters filling the rest, water density box."""
    out = []
    for r in range(n_replicas):
        rng = np.random.default_rng(seed_base + r)
        n_target = float(np.exp(rng.uniform(math.log(n_min), math.log(n_max))))
        if rng.uniform() < chain_frac:
            n_heavy = int(rng.integers(20, 101))
            n_heavy = max(20, min(n_heavy, int(n_target) // 8))
            n_w = max(int(round((n_target - 2.2 * n_heavy) / 3.0)), 20)
            sysr = solvated_chain(n_heavy, n_w, seed_base + 5000 + r, name=f"replica{r}")
        else:
            n_w = max(int(round(n_target / 3.0)), 20)
            m = int(math.ceil(n_w ** (1.0 / 3.0)))
            box = (3 * n_w / WATER_DENSITY) ** (1.0 / 3.0)
            full = water_box(m, box, seed_base + 5000 + r)
            # keep the first n_w waters of the lattice
            keep = 3 * n_w
            sysr = System(full.pos[:keep].copy(), full.species[:keep].copy(), float(box),
                          full.bonded_heavy[:keep].copy(), full.molecule[:keep].copy(),
                          name=f"replica{r}", meta={"n_waters": n_w})
        sysr.meta["replica"] = r
        out.append(sysr)
    return out


def cluster_pair(seed, n_each=6, gap=6.0, box=60.0):
    """Two small random clusters separated by ``gap`` Angstrom (for checks that
    need disconnected interaction graphs)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 2.2, size=(n_each, 3)) + box / 2 - 4.0
    b = rng.uniform(0.0, 2.2, size=(n_each, 3)) + box / 2 - 4.0
    b[:, 0] += 2.2 + gap
    pos = np.concatenate([a, b])
    species = rng.integers(0, 4, size=2 * n_each).astype(np.int32)
    return System(pos, species, float(box), np.full(2 * n_each, -1, np.int32),
                  np.repeat(np.arange(2, dtype=np.int32), n_each), name="cluster_pair")


def maxwell_boltzmann(masses, temperature, seed):
    """Velocities (N, 3) in A/fs drawn from the Maxwell-Boltzmann law."""
    rng = np.random.default_rng(seed)
    z = rng.normal(size=(masses.shape[0], 3))
    return z * np.sqrt(_KB_KCAL * temperature * _ACC / masses)[:, None]


def poisson_arrivals(n, rate_per_s, seed):
    """Arrival times (s) of a Poisson stream."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
