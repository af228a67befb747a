"""Langevin integrators (oracle, float64 numpy).

Units: Angstrom, fs, amu, kcal/mol, K.  Accelerations are ACC * F / m with
ACC = 4.184e-4 (kcal/mol/A/amu -> A/fs^2); kinetic energies are
0.5 sum m v^2 / ACC; k_B = 8.31446261815324 / 4184 kcal/mol/K.  Frictions
are given in ps^-1 and used as 1e-3 fs^-1.

* BAOAB (paper, Methods "Multi-time-step integrator", the Strang splitting
  e^{tL} ~ B A O A B): half kick, half drift, Ornstein-Uhlenbeck step, half
  drift, force evaluation, half kick.
* DMTS-NC (Algorithm 1): with a cached pair (F, F_NC),
      v += (D/2) M^-1 (F - F_NC)
      n times: v += (d/2) M^-1 F_NC; x += (d/2) v; v <- O(v, d);
               x += (d/2) v; F_NC <- NC(x); v += (d/2) M^-1 F_NC
      F <- CONS(x); v += (D/2) M^-1 (F - F_NC)
  with d = D / n.  The sign of the outer kick is "+" as in Algorithm 1 (the
  enumerated list before it writes "-", but F_L = -grad U - F_S is a force).
  The thermostat of Algorithm 1 is the Ornstein-Uhlenbeck step
      v <- c1 v + sqrt((1 - c1^2) k_B T ACC / m) G,  c1 = exp(-gamma d)
  (the inner expression of the Fast-Forward Langevin update of the paper).
* The Fast-Forward Langevin variant replaces that step by
      v <- |c1 v + sigma G| v / |v|   per atom (3-vector norm).
* Rewind procedure (Methods, "Preventing rare model disagreements"): a
  frame (x, v, cached forces, O-step counter) is saved every ``save_every``
  kept outer steps; after each outer step the disagreement of the two force
  models at the step's end, sqrt(mean_i |F_i - F_NC,i|^2), is compared with
  a threshold, and when it is exceeded (or is not finite) the state returns
  to the saved frame, ``sts_after`` BAOAB steps of size d = D/n with the
  conservative force follow, F_NC is evaluated again and multiple time
  stepping resumes with a new frame.  Steps undone by a rewind do not count:
  a run of n_outer outer steps ends after n_outer kept ones.
* Barostat (Methods, "Computation of the virial term in NPT", which runs
  NPT with Bussi's stochastic barostat and the virial estimator below;
  the paper gives no barostat equations).  Isotropic stochastic cell
  rescaling in eps = ln V, one Euler-Maruyama step of length dt_b:
      P_int = (2K - W) / (3V)
      d eps = -(beta_T / tau_p)(P_0 - P_int) dt_b
              + sqrt(2 k_B T beta_T dt_b / (V tau_p)) R
  positions scaled by mu = exp(d eps / 3), velocities by 1/mu, box by mu;
  W is the outer step's virial estimator and K the kinetic energy after it.
  With the velocities rescaled with the cell no k_B T / V drift term is
  needed: the ideal gas then samples <V> = (N + 1) k_B T / P_0, the
  isothermal-isobaric law (pinned).  R is the first Box-Muller normal of the
  Philox block with key (seed, stream) and counter (0, barostat step, 1, 0)
  (word 2 = 1 keeps it apart from the O-step normals).
* Hydrogen mass repartitioning: each hydrogen's mass is raised (set to a
  value, or increased by an amount) and the difference is removed from the
  heavy atom it is bonded to, so each molecule keeps its mass.
* High hydrogen friction: a per-species friction table (diagonal Gamma).
* NPT virial estimator of one outer step (paper, Methods "Computation of the
  virial term in NPT"; the reading is that the final estimator is the virial
  of the slow force F_L = F - F_S at the end of the outer step and the
  correction is the average, over the inner loop, of the fast force's proxy):
      W = [W_cons(x_end) - W_S(x_end)] + (1/n) sum_m W_S(x_m)
  with x_m the positions after inner step m (x_n = x_end).  For a single
  time step it is W_cons(x_end).

Random numbers: Philox-4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) with key
(seed, stream) and counter (atom, step, 0, 0); the four 64-bit words give
uniforms u = ((w >> 11) + 0.5) 2^-53 and Box-Muller normals
    g0 = sqrt(-2 ln u0) cos(2 pi u1), g1 = sqrt(-2 ln u0) sin(2 pi u1),
    g2 = sqrt(-2 ln u2) cos(2 pi u3)
for the x, y, z noise of that atom at that O-step.  ``step`` counts O-steps
from the start of the trajectory.

Pins (tests/test_oracle_integrator.py): Philox known-answer vectors and
numpy's Philox bit generator; Box-Muller at chosen uniforms (closed-form
angles and radii); RESPA with n = 1 equal to BAOAB; RESPA with NC equal to
the conservative force equal to n BAOAB steps of size d; BAOAB on harmonic
oscillators giving <x^2> = kT/k; temperatures following (T/d) chi^2(d), for
the Langevin O step and for the Fast-Forward Langevin step (which keeps the
Maxwell-Boltzmann law: zero-force runs started far from it relax to 300 K
with the chi^2 spread, and the reduced speeds follow the Maxwell law);
energy conservation without friction (the energy fluctuation of BAOAB with
the conservative model shrinks four-fold when the step is halved, the
second-order error of the Strang splitting); molecule masses kept by HMR.
"""

import math
from dataclasses import dataclass

import numpy as np

ACC = 4.184e-4
KB = 8.31446261815324 / 4184.0

_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B
_MASK = (1 << 64) - 1


# ------------------------------------------------------------------ Philox --

def philox4x64_scalar(counter, key, rounds=10):
    """One Philox-4x64 block with Python integers (reference form)."""
    c0, c1, c2, c3 = (int(x) & _MASK for x in counter)
    k0, k1 = (int(x) & _MASK for x in key)
    for _ in range(rounds):
        p0 = _M0 * c0
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0) & _MASK, p1 & _MASK, ((p0 >> 64) ^ c3 ^ k1) & _MASK, p0 & _MASK
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return [c0, c1, c2, c3]


def _mulhilo(a, b):
    """64x64 -> (hi, lo) on uint64 numpy arrays via 32-bit halves."""
    lo32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a_lo, a_hi = a & lo32, a >> s32
    b_lo, b_hi = b & lo32, b >> s32
    ll = a_lo * b_lo
    hl = a_hi * b_lo
    lh = a_lo * b_hi
    hh = a_hi * b_hi
    cross = (ll >> s32) + (hl & lo32) + (lh & lo32)
    hi = hh + (hl >> s32) + (lh >> s32) + (cross >> s32)
    lo = a * b
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds=10):
    """Vectorised Philox-4x64 over uint64 arrays (broadcast)."""
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3))
        c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
        c0, c1, c2, c3 = c0.copy(), c1.copy(), c2.copy(), c3.copy()
        k0 = np.uint64(k0)
        k1 = np.uint64(k1)
        m0, m1 = np.uint64(_M0), np.uint64(_M1)
        w0, w1 = np.uint64(_W0), np.uint64(_W1)
        for _ in range(rounds):
            hi0, lo0 = _mulhilo(m0, c0)
            hi1, lo1 = _mulhilo(m1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
            k0 = k0 + w0
            k1 = k1 + w1
    return c0, c1, c2, c3


def uniforms_from_bits(w):
    return ((np.asarray(w, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53


def box_muller(u0, u1, u2, u3):
    """(..., 3) normals from four uniforms in (0, 1): the first pair gives
    the x and y components, the second pair the z component."""
    r0 = np.sqrt(-2.0 * np.log(u0))
    r1 = np.sqrt(-2.0 * np.log(u2))
    return np.stack([r0 * np.cos(2.0 * math.pi * u1),
                     r0 * np.sin(2.0 * math.pi * u1),
                     r1 * np.cos(2.0 * math.pi * u3)], axis=-1)


def langevin_normals(seed, stream, step, n_atoms):
    """(N, 3) standard normals for O-step ``step`` of stream ``stream``."""
    atoms = np.arange(n_atoms, dtype=np.uint64)
    w = philox4x64(atoms, np.uint64(step), 0, 0, seed, stream)
    return box_muller(*(uniforms_from_bits(x) for x in w))


# ----------------------------------------------------- masses and friction --

def hmr_masses(species, bonded_heavy, masses, h_mass=3.0, mode="set"):
    """Hydrogen mass repartitioning: hydrogens get ``h_mass`` ('set') or
    their mass plus ``h_mass`` ('add'); the bonded heavy atom loses the
    difference."""
    m = np.array(masses, dtype=np.float64, copy=True)
    for a in range(m.shape[0]):
        h = int(bonded_heavy[a])
        if h < 0:
            continue
        new = h_mass if mode == "set" else masses[a] + h_mass
        delta = new - masses[a]
        m[a] = new
        m[h] = m[h] - delta
    return m


def friction_per_atom(species, gamma_per_species_ps):
    return np.asarray(gamma_per_species_ps, dtype=np.float64)[np.asarray(species)]


# -------------------------------------------------------------- integrators --

@dataclass
class LangevinParams:
    dt_outer: float          # fs (Delta); for BAOAB the step size
    n_inner: int             # n (1 for BAOAB)
    temperature: float       # K
    gamma_ps: np.ndarray     # (N,) ps^-1
    seed: int
    stream: int = 0
    thermostat: str = "langevin"   # or "ffl"


@dataclass
class State:
    x: np.ndarray            # (N, 3)
    v: np.ndarray            # (N, 3)
    m: np.ndarray            # (N,)
    f: np.ndarray = None     # cached conservative force
    f_nc: np.ndarray = None  # cached fast force
    step: int = 0            # O-steps done
    first_step: bool = True


def kinetic_energy(v, m):
    return 0.5 * float(np.sum(m[:, None] * v * v)) / ACC


def temperature(v, m):
    return 2.0 * kinetic_energy(v, m) / (3 * v.shape[0] * KB)


def _o_step(st, prm, dt):
    g = np.asarray(prm.gamma_ps, dtype=np.float64) * 1e-3
    c1 = np.exp(-g * dt)
    sigma = np.sqrt((1.0 - c1 * c1) * KB * prm.temperature * ACC / st.m)
    G = langevin_normals(prm.seed, prm.stream, st.step, st.x.shape[0])
    new = c1[:, None] * st.v + sigma[:, None] * G
    if prm.thermostat == "ffl":
        nv = np.linalg.norm(st.v, axis=1)
        nn = np.linalg.norm(new, axis=1)
        scale = np.where(nv > 0, nn / np.where(nv > 0, nv, 1.0), 0.0)
        new = np.where(nv[:, None] > 0, st.v * scale[:, None], new)
    st.v = new
    st.step += 1


def _kick(st, f, dt):
    st.v = st.v + (0.5 * dt) * ACC * f / st.m[:, None]


def baoab_step(st, force_fn, prm):
    """One BAOAB step of size prm.dt_outer with force ``force_fn(x)``."""
    dt = prm.dt_outer
    if st.first_step or st.f is None:
        st.f = force_fn(st.x)
        st.first_step = False
    _kick(st, st.f, dt)
    st.x = st.x + 0.5 * dt * st.v
    _o_step(st, prm, dt)
    st.x = st.x + 0.5 * dt * st.v
    st.f = force_fn(st.x)
    _kick(st, st.f, dt)
    return st


def dmts_nc_step(st, cons_fn, nc_fn, prm):
    """One outer step of Algorithm 1 (BAOAB-RESPA with F_S = F_NC and
    F_L = F - F_NC)."""
    D, n = prm.dt_outer, prm.n_inner
    d = D / n
    if st.first_step or st.f is None or st.f_nc is None:
        st.f_nc = nc_fn(st.x)
        st.f = cons_fn(st.x)
        st.first_step = False
    st.v = st.v + (0.5 * D) * ACC * (st.f - st.f_nc) / st.m[:, None]
    for _ in range(n):
        _kick(st, st.f_nc, d)
        st.x = st.x + 0.5 * d * st.v
        _o_step(st, prm, d)
        st.x = st.x + 0.5 * d * st.v
        st.f_nc = nc_fn(st.x)
        _kick(st, st.f_nc, d)
    st.f = cons_fn(st.x)
    st.v = st.v + (0.5 * D) * ACC * (st.f - st.f_nc) / st.m[:, None]
    return st


def dmts_nc_step_virial(st, cons_fn, nc_fn, prm, cons_vir, fast_vir):
    """dmts_nc_step that also returns the step's NPT virial estimator;
    ``cons_vir(x)`` and ``fast_vir(x)`` give W = -sum_i F_i . q_i of the
    conservative and the fast force at x."""
    D, n = prm.dt_outer, prm.n_inner
    d = D / n
    if st.first_step or st.f is None or st.f_nc is None:
        st.f_nc = nc_fn(st.x)
        st.f = cons_fn(st.x)
        st.first_step = False
    st.v = st.v + (0.5 * D) * ACC * (st.f - st.f_nc) / st.m[:, None]
    inner = []
    for _ in range(n):
        _kick(st, st.f_nc, d)
        st.x = st.x + 0.5 * d * st.v
        _o_step(st, prm, d)
        st.x = st.x + 0.5 * d * st.v
        st.f_nc = nc_fn(st.x)
        inner.append(fast_vir(st.x))
        _kick(st, st.f_nc, d)
    st.f = cons_fn(st.x)
    st.v = st.v + (0.5 * D) * ACC * (st.f - st.f_nc) / st.m[:, None]
    return st, (cons_vir(st.x) - inner[-1]) + sum(inner) / n


def disagreement(f, f_nc):
    """sqrt(mean over atoms of |F_i - F_NC,i|^2) (kcal/mol/A)."""
    d = np.asarray(f, dtype=np.float64) - np.asarray(f_nc, dtype=np.float64)
    return float(np.sqrt(np.sum(d * d) / d.shape[0]))


def dmts_nc_run_rewind(st, cons_fn, nc_fn, prm, n_outer, threshold, save_every, sts_after, max_rewinds=None):
    """n_outer kept outer steps of Algorithm 1 under the rewind procedure.
    Returns (rewinds, disagreements) with the disagreement measured after
    every outer step taken, kept or undone."""
    frame, since_save, kept, rewinds, seen = None, 0, 0, 0, []
    limit = max(16, n_outer) if max_rewinds is None else max_rewinds
    sts = LangevinParams(prm.dt_outer / prm.n_inner, 1, prm.temperature, prm.gamma_ps, prm.seed, prm.stream,
                         prm.thermostat)
    while kept < n_outer:
        if since_save % save_every == 0:
            frame = (st.x.copy(), st.v.copy(), None if st.f is None else st.f.copy(),
                     None if st.f_nc is None else st.f_nc.copy(), st.step, st.first_step, kept)
            since_save = 0
        dmts_nc_step(st, cons_fn, nc_fn, prm)
        kept += 1
        since_save += 1
        dis = disagreement(st.f, st.f_nc) if np.all(np.isfinite(st.x)) and np.all(np.isfinite(st.v)) else math.inf
        seen.append(dis)
        if not dis <= threshold:
            rewinds += 1
            if rewinds > limit:
                raise RuntimeError("the fast model keeps disagreeing: rewind limit reached")
            x, v, f, f_nc, step, first, kept = frame
            st.x, st.v, st.f, st.f_nc, st.step, st.first_step = x.copy(), v.copy(), f, f_nc, step, first
            for _ in range(sts_after):
                baoab_step(st, cons_fn, sts)
            st.f_nc = nc_fn(st.x)
            since_save = 0
    return rewinds, seen


BAR = 1e5 * 6.02214076e23 * 1e-30 / 4184.0      # one bar in kcal/mol/A^3


@dataclass
class BarostatParams:
    pressure_bar: float
    compressibility_per_bar: float   # beta_T
    tau_fs: float                    # tau_p
    dt_fs: float                     # time between barostat steps
    temperature: float               # K
    seed: int
    stream: int = 0


def barostat_normal(seed, stream, step):
    w = philox4x64_scalar([0, step, 1, 0], [seed, stream])
    u0, u1 = (uniforms_from_bits(np.uint64(x)) for x in w[:2])
    return float(math.sqrt(-2.0 * math.log(u0)) * math.cos(2.0 * math.pi * u1))


def scr_barostat_step(st, box, virial, prm, step):
    """One stochastic cell rescaling step; returns the new box edge.  The
    cached forces no longer belong to the scaled positions: the state is
    marked for a fresh evaluation."""
    V = box ** 3
    K = kinetic_energy(st.v, st.m)
    p_int = (2.0 * K - virial) / (3.0 * V)
    beta = prm.compressibility_per_bar / BAR
    kT = KB * prm.temperature
    g = barostat_normal(prm.seed, prm.stream, step)
    de = (-(beta / prm.tau_fs) * (prm.pressure_bar * BAR - p_int) * prm.dt_fs
          + math.sqrt(2.0 * kT * beta * prm.dt_fs / (V * prm.tau_fs)) * g)
    mu = math.exp(de / 3.0)
    st.x = st.x * mu
    st.v = st.v / mu
    st.first_step = True
    return box * mu
