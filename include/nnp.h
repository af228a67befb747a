/*
 * nnp.h -- C interface of libnnp, the MI355X (gfx950) hot path of DMTS-NC:
 * distilled multi-time-stepping with non-conservative forces
 * (Gouraud, Cattin, Ple, Adjoua, Lagardere, Piquemal; arXiv 2602.14975).
 *
 * Units: Angstrom, fs, amu, kcal/mol, K; frictions in ps^-1.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Device arrays are HIP device pointers owned by the caller (for example
 *    torch tensors); the library never frees or reallocates them.  Host
 *    arrays are read during the call only.
 *  - Per-atom vectors are structure-of-arrays: x row, then y row, then z row
 *    ([3][n], row stride n).  Positions and velocities are float64; forces
 *    float32.  Positions are kept unwrapped; only the pair rule wraps.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls enqueue work on it and return without waiting unless stated.
 *  - A call returns NNP_OK or a negative status and never throws;
 *    nnp_last_error() then describes the failure (thread-local string, valid
 *    until the next call from the same thread).
 *  - Workspaces are caller-owned device buffers of at least the size
 *    reported by nnp_workspace_size(); their contents are scratch.
 *
 * Pair rule (paper, Methods "Model architecture": N(i) is every j != i
 * within the cutoff): in float64, per component d = x_j - x_i,
 * d = d - L * rint(d * (1/L)) with rint rounding half to even, then
 * r2 = (dx*dx + dy*dy) + dz*dz without fused multiply-add, and j is a
 * neighbour of i iff r2 < rc*rc.  The relation is symmetric.  It requires
 * rc < L/2 for every box.
 */
#ifndef NNP_H
#define NNP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nnp_status;
enum {
    NNP_OK = 0,
    NNP_EINVAL = -1,     /* bad argument, descriptor, size or geometry */
    NNP_ENOMEM = -2,     /* device allocation failed or budget exceeded */
    NNP_ECAPACITY = -3,  /* a neighbour list did not fit its buffer */
    NNP_EDEVICE = -4,    /* a HIP runtime call failed */
    NNP_EUNSTABLE = -5,  /* non-finite positions or velocities detected */
    NNP_ENOTFOUND = -6,  /* unknown ticket */
    NNP_EROWLIMIT = -7   /* an atom has more than 1024 list entries: the
                            builder sorts each row in LDS, so a larger list
                            buffer cannot fix it (a denser system than the
                            models are meant for, or a collapsing one) */
};

const char* nnp_last_error(void);
/* Interface version (increments on incompatible change). */
int32_t nnp_abi_version(void);

/* ------------------------------------------------------------------ models
 * Two model kinds share one embedding block.
 *
 * NNP_MODEL_CONS, the conservative potential U at the outer step (paper,
 * Methods "Model architecture", first paragraph; a synthetic equivariant
 * message-passing stand-in for FeNNix-Bio1, whose weights are unavailable):
 *   s_i = emb[t_i], v_i = 0; then n_layers times, with
 *   phi_j = W2 silu(W1 s_j + b1) + b2, w_ij = (Wr e(r_ij) + br) fcos(r_ij),
 *   [a|b|c]_ij = phi_j * w_ij:
 *     s_i += sum_j a_ij;  v_i[alpha] += sum_j (b_ij v_j[alpha] + u_ij[alpha] c_ij)
 *   followed by the update block
 *     Uv = U v, Vv = V v, n = sqrt(sum_alpha Vv^2 + 1e-8),
 *     [p|q|o] = M2 silu(M1 [s; n] + m1) + m2,
 *     s += p + q * sum_alpha Uv Vv,  v += o * Uv;
 *   E_i = wo . silu(Wo s_i + bo) + beta[t_i], E = sum_i E_i; forces -dE/dx.
 *   e_k(r) = sqrt(2/rc) sin(k pi r/rc)/r (k = 1..n_rbf);
 *   fcos(r) = (cos(pi r/rc) + 1)/2.
 *
 * NNP_MODEL_NC, the distilled non-conservative force model (paper, Methods:
 * equations for q_ih, k_ih, c_ijh, F_ij and F_i): one embedding layer with
 * the polynomial envelope u(d) = 1 - (p+1)(p+2)/2 d^p + p(p+2) d^(p+1)
 *   - p(p+1)/2 d^(p+2), d = r/rc, in place of fcos; then
 *   q_ih = Wq[h] s_i, k_ih = Wk[h] s_i (n_c each, h < n_s + n_l),
 *   V_ih = sum_f WV[h][f] v_i[:, f] (h < n_l),
 *   c_ijh = q_ih . k_jh / sqrt(n_c),
 *   F_ij = (sum_{h<n_s} c_ijh B_h(r)) (u_ij + sum_{h<n_l} c_ij(n_s+h) V_ih) u(r/rc),
 *   F_i = sum_{j in N(i)} (F_ij - F_ji), with B_h the same Bessel basis.
 *   The screened nuclear repulsion term of the paper is not included.
 *
 * Weight manifest: `weights` is one flat float64 host vector holding, in
 * order, row-major [out][in] matrices and vectors (F = width, K = n_rbf,
 * S = n_species, H = n_s + n_l):
 *   emb[S][F];
 *   per layer (CONS: n_layers of them, NC: exactly one):
 *     W1[F][F] b1[F] W2[3F][F] b2[3F] Wr[3F][K] br[3F] U[F][F] V[F][F]
 *     M1[F][2F] m1[F] M2[3F][F] m2[3F];
 *   CONS: Wo[F][F] bo[F] wo[F] beta[S];
 *   NC:   Wq[H][n_c][F] Wk[H][n_c][F] WV[n_l][F].
 * Supported sizes: width in {16, 32, 64, 128}; n_rbf in {8, 16};
 * NC: n_s = 8, n_l = 2, n_c = 8, poly_p = 5.
 */
enum { NNP_MODEL_CONS = 0, NNP_MODEL_NC = 1 };
enum { NNP_FP32 = 0, NNP_BF16 = 1 };  /* arithmetic of the perceptrons and filters */

typedef struct {
    int32_t kind;        /* NNP_MODEL_CONS or NNP_MODEL_NC */
    int32_t n_species;   /* 1..8 */
    int32_t width;       /* F */
    int32_t n_layers;    /* CONS: >= 1; NC: 1 */
    int32_t n_rbf;       /* K */
    int32_t poly_p;      /* NC envelope order */
    int32_t n_s, n_l, n_c;
    int32_t precision;   /* NNP_FP32 or NNP_BF16 */
    double cutoff;       /* rc, Angstrom */
    const double* weights;  /* host, manifest order */
    int64_t n_weights;
} nnp_model_desc;

typedef struct nnp_model nnp_model;

/* Copies the weights to the device (the only allocation of a model).
 * NNP_EINVAL if the descriptor is unsupported or n_weights does not match
 * the manifest. */
nnp_status nnp_model_create(const nnp_model_desc* desc, nnp_model** out);
void nnp_model_destroy(nnp_model* model);
int64_t nnp_model_n_weights(const nnp_model* model);
/* Replaces the weights from a device float32 vector in manifest order
 * (used by distillation after an optimiser step).  Enqueued on `stream`. */
nnp_status nnp_model_set_weights_f32(nnp_model* model, const float* weights_dev,
                                     int64_t n_weights, void* stream);

/* ----------------------------------------------------------------- systems
 * A system is one or more independent replicas packed contiguously: replica
 * r owns atoms [rep_start[r], rep_start[r+1]) and has cubic box box[r].
 * Neighbour lists never cross replicas. */
typedef struct {
    int64_t n_atoms;
    int32_t n_rep;               /* >= 1 */
    const double* pos;           /* device [3][n_atoms] */
    const int32_t* species;      /* device [n_atoms] */
    const int32_t* rep_of_atom;  /* device [n_atoms]; may be NULL if n_rep == 1 */
    const double* box_dev;       /* device [n_rep]; may be NULL if n_rep == 1 */
    const int64_t* rep_start;    /* host [n_rep + 1] */
    const double* box;           /* host [n_rep] */
} nnp_system;

/* Neighbour list in CSR form: row i lists its neighbours j in ascending
 * order in nbr[offsets[i] .. offsets[i+1]).  Buffers are caller-owned. */
typedef struct {
    int64_t n_atoms;    /* rows */
    int64_t capacity;   /* entries nbr can hold */
    int64_t n_edges;    /* out: entries written, or required on NNP_ECAPACITY */
    int32_t* offsets;   /* device [n_atoms + 1] */
    int32_t* nbr;       /* device [capacity] */
    int32_t* rev;       /* device [capacity] or NULL: rev[e] = index of the
                           reverse pair (j, i) of entry e = (i, j) */
    double cutoff;      /* radius of the pair rule used to build the list */
} nnp_nlist;

/* Workspace bytes sufficient for every call below on systems of at most
 * n_atoms atoms, n_rep replicas and max_edges list entries per list.
 * Either model may be NULL. */
nnp_status nnp_workspace_size(const nnp_model* cons, const nnp_model* nc, int64_t n_atoms,
                              int32_t n_rep, int64_t max_edges, size_t* bytes);

/* Builds the list of all pairs under the pair rule at nl->cutoff (a cell
 * list with a 27-cell stencil where a replica has >= 3 cells per side, all
 * atoms of the replica otherwise).  Synchronises `stream` to learn the edge
 * count.  NNP_ECAPACITY: nl->n_edges holds the required capacity and the
 * buffers are unchanged; NNP_EROWLIMIT: a row is longer than 1024 entries
 * (buffers unchanged); NNP_EINVAL: cutoff >= L/2 or bad sizes. */
nnp_status nnp_neighbors(const nnp_system* sys, nnp_nlist* nl, void* ws, size_t ws_bytes,
                         void* stream);

/* Conservative energy and forces F = -dE/dx by a hand-written reverse pass
 * (the outer-step force of Algorithm 1).  `nl` may be built at any radius
 * >= the model cutoff (a Verlet list); pairs are filtered with the pair rule
 * at the model cutoff, so the result does not depend on the list radius.
 * energy: device float64 [n_rep] (per replica); forces: device float32
 * [3][n_atoms]. */
nnp_status nnp_cons_energy_forces(const nnp_model* cons, const nnp_system* sys,
                                  const nnp_nlist* nl, void* ws, size_t ws_bytes,
                                  double* energy, float* forces, void* stream);

/* Non-conservative forces F_NC (the inner-step force of Algorithm 1);
 * forces: device float32 [3][n_atoms].  Same list rules as above. */
nnp_status nnp_nc_forces(const nnp_model* nc, const nnp_system* sys, const nnp_nlist* nl,
                         void* ws, size_t ws_bytes, float* forces, void* stream);

/* nnp_nc_forces for callers that cannot allocate device memory (code under
 * stream capture, serving loops or harnesses that forbid hipMalloc): the
 * same kernels and result as nnp_nc_forces, with the scratch taken from a
 * static device array of nnp_nc_forces_noalloc_max_bytes() bytes (64 MiB;
 * about 14,000 atoms for a width-32 NC model) instead of a workspace.  The
 * caller still owns sys, nl and forces.  The call allocates nothing; each GPU
 * the library runs on holds its own copy of the array until the process
 * ends.  No part of the array needs to start at zero (every byte a call
 * reads is written earlier in the same call).  Every call on one GPU shares
 * that GPU's array, so calls that overlap on one GPU (other streams, other
 * threads) race.  NNP_EINVAL (nothing launched) when the system needs more
 * scratch than the maximum, with the required size in nnp_last_error(). */
size_t nnp_nc_forces_noalloc_max_bytes(void);
nnp_status nnp_nc_forces_noalloc(const nnp_model* nc, const nnp_system* sys, const nnp_nlist* nl,
                                 float* forces, void* stream);

/* NPT virials (paper, Methods "Computation of the virial term in NPT"):
 * W = -sum_i F_i . q_i, written under periodic boundaries through the
 * minimum-image vectors r_ij = q_j - q_i.  With the kinetic energy K the
 * pressure is P = (2K - W) / (3V).  virial: device float64 [n_rep].
 *
 * nnp_cons_virial: energy (may be NULL) and forces (required) as
 * nnp_cons_energy_forces, and W = sum over directed edges of r_e . dE/dr_e
 * (equal to dE/dlambda when positions and box are scaled by lambda),
 * accumulated from the pair forces of the hand-written reverse pass. */
nnp_status nnp_cons_virial(const nnp_model* cons, const nnp_system* sys, const nnp_nlist* nl,
                           void* ws, size_t ws_bytes, double* energy, float* forces, double* virial,
                           void* stream);

/* nnp_nc_virial: forces as nnp_nc_forces and the paper's proxy
 * W = sum_i sum_{j in N(i)} F_ij . r_ij of the NC pair terms (equal to
 * -sum_i F_i . q_i wherever q_i is unambiguous). */
nnp_status nnp_nc_virial(const nnp_model* nc, const nnp_system* sys, const nnp_nlist* nl,
                         void* ws, size_t ws_bytes, float* forces, double* virial, void* stream);

/* Weight gradient of the NC model: given dl_df = dL/dF_NC (device float32
 * [3][n_atoms]) writes dL/dtheta (device float32 [n_weights], manifest
 * order), the vector-Jacobian product used to distil the NC model onto
 * conservative forces.  Deterministic (fixed reduction order). */
nnp_status nnp_nc_weight_grad(const nnp_model* nc, const nnp_system* sys, const nnp_nlist* nl,
                              const float* dl_df, float* dl_dtheta, void* ws, size_t ws_bytes,
                              void* stream);

/* Force-matching loss of the distillation: loss = mean over the `count`
 * entries of (f - f_ref)^2 (device float64 scalar), and, if grad is not
 * NULL, grad = dloss/df = 2 (f - f_ref) / count (device float32).  The sum is
 * taken in a fixed order.  ws: device scratch of at least 8 KiB. */
nnp_status nnp_force_mse(const float* f, const float* f_ref, int64_t count, double* loss, float* grad,
                         void* ws, size_t ws_bytes, void* stream);

/* One Adam step on a device float32 parameter vector (in place):
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; with bias corrections for
 * step t (>= 1): p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
nnp_status nnp_adam_step(float* param, const float* grad, float* m, float* v, int64_t n,
                         int64_t t, double lr, double beta1, double beta2, double eps,
                         void* stream);

/* --------------------------------------------------------------- integrator
 * Hydrogen mass repartitioning (paper, Methods "Hydrogen Mass
 * Repartitioning"): for each atom a with bonded_heavy[a] = h >= 0 (a
 * hydrogen bonded to heavy atom h) the new mass is h_mass (mode 0, "set") or
 * mass[a] + h_mass (mode 1, "add"); h loses the difference, so every
 * molecule keeps its mass.  Host arrays, n entries; writes out_mass. */
nnp_status nnp_hmr_masses(int64_t n, const int32_t* bonded_heavy, const double* mass,
                          double h_mass, int32_t mode, double* out_mass);

/* NNP_MODE_DMTS_NC: Algorithm 1 with the NC model as the fast force.
 * NNP_MODE_STS: BAOAB with the conservative force only.
 * NNP_MODE_DMTS: the same splitting with a small conservative model as the
 * fast force (the distilled conservative scheme the paper compares with). */
enum { NNP_MODE_DMTS_NC = 0, NNP_MODE_STS = 1, NNP_MODE_DMTS = 2 };
enum { NNP_THERMO_LANGEVIN = 0, NNP_THERMO_FFL = 1 };

typedef struct {
    double dt_outer_fs;     /* Delta (STS: the step) */
    int32_t n_inner;        /* n; delta = Delta / n (STS: ignored, 1) */
    int32_t mode;           /* NNP_MODE_DMTS_NC or NNP_MODE_STS */
    int32_t thermostat;     /* NNP_THERMO_LANGEVIN or NNP_THERMO_FFL */
    int32_t check_every;    /* outer steps between finiteness checks (>= 1) */
    double temperature_K;
    uint64_t seed;          /* Philox key word 0 */
    uint64_t stream_id;     /* Philox key word 1 for replica 0; replica r uses stream_id + r */
    double skin;            /* Verlet skin (A) of both lists; lists are rebuilt when an
                               atom has moved more than skin/2 since the last build */
    /* Rewind procedure (paper, Methods "Preventing rare model disagreements"):
     * when rewind_threshold > 0, after each outer step the device measures the
     * disagreement sqrt(mean_i |F_i - F_fast,i|^2) of every replica; if one
     * exceeds the threshold (or the state is not finite) the whole system
     * returns to the last saved frame (positions, velocities, forces and the
     * O-step counter), runs sts_after_rewind BAOAB steps of size delta with
     * the conservative force, re-evaluates the fast force and resumes MTS.
     * The trip is read at the status checks (every check_every outer steps),
     * where frames are also saved, every save_every kept outer steps
     * (save_every must be a multiple of check_every); outer steps undone by
     * a rewind do not count towards n_outer, so the result does not depend on
     * check_every.  More than max(16, n_outer) rewinds in one call return
     * NNP_EUNSTABLE with the state at the saved frame. */
    double rewind_threshold;  /* kcal/mol/A; 0 disables */
    int32_t save_every;       /* >= 1 */
    int32_t sts_after_rewind; /* >= 0 */
    /* 1: multiple-time-step runs record one outer step as a HIP graph on the
     * caller's stream and replay it (fewer launch gaps; the numbers are
     * identical); 0: launch every kernel directly.  Graphs are not used while
     * launch-site timers are enabled or for calls of fewer than three outer
     * steps. */
    int32_t graph;
} respa_params;

/* Device-resident trajectory state.  All pointers are caller-owned device
 * buffers.  The neighbour lists are built at (model cutoff + skin). */
typedef struct {
    nnp_system sys;        /* sys.pos aliases pos */
    double* pos;           /* [3][n] read/write */
    double* vel;           /* [3][n] read/write */
    const double* mass;    /* [n] amu (HMR applied by the caller if wanted) */
    const double* gamma;   /* [n] friction, ps^-1 (per-species table expanded) */
    float* f_cons;         /* [3][n] cached conservative force F */
    float* f_nc;           /* [3][n] cached fast force F_NC (DMTS-NC) */
    double* energy;        /* [n_rep] conservative energy at the last evaluation */
    double* pos_ref;       /* [3][n] positions at the last list build */
    nnp_nlist nl_cons;     /* conservative list (cutoff + skin) */
    nnp_nlist nl_nc;       /* fast-force list (its cutoff + skin); unused in STS mode */
    uint64_t step;         /* O-steps done so far (advanced by the call) */
    int32_t first_step;    /* 1: evaluate F and F_NC before the first kick */
    int32_t lists_valid;   /* 0: build both lists before the first use */
    double* ke;            /* [n_outer][n_rep] kinetic energy after each outer
                              step (kcal/mol), or NULL */
    int64_t n_rebuilds;    /* out: list rebuilds performed (accumulates) */
    int64_t n_rewinds;     /* out: rewinds performed (accumulates) */
    int64_t n_replays;     /* out: intervals replayed after a list went stale
                              between two predicted rebuilds (accumulates) */
    double* virial;        /* [n_rep] or NULL: after the call, the NPT virial
                              estimator W of the last outer step (see below) */
    int32_t* order;        /* [2 n] or NULL.  Non-NULL: the model evaluations
                              keep their per-atom rows in the cell order of the
                              last list build (atoms that are close in space
                              are close in memory, whatever the caller's
                              numbering); order[p] is the caller's index of row
                              p, order[n + i] the row of atom i.  Written at
                              each list build, read by later calls while
                              lists_valid is 1; nl_cons and nl_nc then hold
                              rows and entries in that order.  Each row lists
                              its neighbours in ascending caller index, so
                              every per-atom sum runs in the same order as
                              with NULL and the results are the same bits.
                              NULL: rows in the caller's order. */
} respa_state;

/* Advances the state by n_outer outer steps of Algorithm 1 (DMTS-NC, or
 * DMTS with `nc` a conservative model:
 * v += (D/2) M^-1 (F - F_NC); n x [B(d/2), A(d/2), O(d), A(d/2), F_NC, B(d/2)];
 * F; v += (D/2) M^-1 (F - F_NC)), or of BAOAB with the conservative force
 * (STS).  The O step is v <- c v + sqrt((1 - c^2) kT/m) G, c = exp(-gamma d),
 * G from Philox-4x64-10 with key (seed, stream_id + r) and counter
 * (atom index within its replica, O-step index, 0, 0), Box-Muller on the four
 * uniforms ((w >> 11) + 0.5) 2^-53; FFL keeps each atom's velocity direction.
 * Lists are rebuilt when an atom moved more than skin/2 since the last
 * build.  Multiple-time-step runs (n > 1) decide this once per
 * outer step, from the largest displacement so far and its growth over the
 * previous outer step; should an inner step still exceed skin/2, the
 * interval since the last check is replayed with the check after every
 * inner step (n_replays counts these; the numbers are the same either way).
 * Every `check_every` outer steps the call synchronises and checks list
 * capacity and finiteness; on NNP_ECAPACITY the state is restored to the
 * start of the failing outer step (grow the list buffers and call again);
 * NNP_EROWLIMIT restores it the same way, but is not recoverable by growing;
 * on NNP_EUNSTABLE it is left at the last checked good step.  The sizes of
 * completed steps are reflected in state->step.
 * Virial estimator (state->virial not NULL; paper, Methods "Computation of
 * the virial term in NPT"): for an outer step of n inner steps with fast
 * force F_S (the NC model, or the small conservative model), the virial of
 * the slow force F_L = F - F_S at the end of the step plus the average over
 * the inner loop of the fast force's proxy,
 *   W = [W_cons(x_end) - W_S(x_end)] + (1/n) sum_m W_S(x_m),
 * x_m the positions after inner step m; a single time step gives
 * W_cons(x_end).  W_S is the NC proxy (nnp_nc_virial) or the conservative
 * virial of the small model. */
nnp_status respa_step(const nnp_model* cons, const nnp_model* nc, respa_state* state,
                      const respa_params* params, int32_t n_outer, void* ws, size_t ws_bytes,
                      void* stream);

/* Barostat (paper, Methods "Computation of the virial term in NPT": NPT
 * runs with Bussi's stochastic barostat fed by the virial estimator of the
 * multiple-time-step outer step).  Isotropic stochastic cell rescaling, one
 * Euler-Maruyama step in eps = ln V per replica:
 *   P_int = (2K - W) / (3V),  K the kinetic energy of the state, W =
 *   state->virial[r] (the estimator of the last outer step of respa_step);
 *   d eps = -(beta_T / tau_p)(P_0 - P_int) dt_b
 *           + sqrt(2 k_B T beta_T dt_b / (V tau_p)) g;
 * positions scaled by mu = exp(d eps / 3), velocities by 1/mu, the box edge
 * by mu (the rescaling of the velocities makes a k_B T / V drift term
 * unnecessary: the ideal gas samples <V> = (N + 1) k_B T / P_0).  g is the
 * first Box-Muller normal of the Philox-4x64-10 block with key
 * (seed, stream_id + r) and counter (0, barostat_step, 1, 0).  1 bar =
 * 1e5 N_A 1e-30 / 4184 kcal/mol/A^3. */
typedef struct {
    double pressure_bar;             /* P_0 */
    double compressibility_per_bar;  /* beta_T */
    double tau_fs;                   /* tau_p */
    double dt_fs;                    /* time since the previous barostat step */
    double temperature_K;
    uint64_t seed;
    uint64_t stream_id;              /* replica r uses stream_id + r */
} nnp_barostat_params;

/* Applies the step to the state in place, writes the new box edges to
 * box_host (the system's host array, required) and box_dev (its device
 * array; NULL allowed for one replica), marks the lists invalid and sets
 * first_step (the cached forces belong to the old cell).  Synchronises
 * `stream`.  ws: a workspace of nnp_workspace_size for the system. */
nnp_status nnp_barostat_scr(respa_state* state, const nnp_barostat_params* params, uint64_t barostat_step,
                            double* box_host, double* box_dev, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ serving
 * Continuous batching of independent replicas.  Replicas are submitted at
 * any time, admitted at outer-step boundaries when a slot is free and their
 * device footprint fits the HBM budget, advanced together in fused launches
 * (one packed system, block-diagonal neighbour lists, per-replica boxes,
 * Philox keys and step counters), and retired when they reach their step
 * count.  The budget is reserved once at creation; it holds two banks of
 * packed state, a staging bank for admissions, and the lists and scratch of
 * the resident set.  An admitted replica is uploaded once, its lists built
 * and F and F_NC evaluated in the staging bank; when the resident set
 * changes, a gather kernel moves the resident replicas (with their cached
 * forces) and the admitted ones into the other bank, so resident state
 * never leaves the device and nothing is evaluated twice; only a retiring
 * replica's final state is copied to the host.  Results do not depend on
 * which other replicas share the launches. */
typedef struct nnp_server nnp_server;

nnp_status nnp_server_create(const nnp_model* cons, const nnp_model* nc,
                             const respa_params* params, size_t hbm_budget_bytes,
                             int32_t max_slots, nnp_server** out);
void nnp_server_destroy(nnp_server* server);

typedef struct {
    int64_t n;                 /* atoms */
    const double* pos;         /* host [n][3] */
    const double* vel;         /* host [n][3] */
    const double* mass;        /* host [n] */
    const double* gamma;       /* host [n] ps^-1 */
    const int32_t* species;    /* host [n] */
    double box;
    uint64_t seed;             /* Philox key word 0 for this replica */
    uint64_t stream_id;        /* Philox key word 1 */
    int32_t n_outer_steps;
} replica_desc;

enum { NNP_REPLICA_QUEUED = 0, NNP_REPLICA_RUNNING = 1, NNP_REPLICA_DONE = 2,
       NNP_REPLICA_FAILED = 3 };

typedef struct {
    int32_t state;
    int32_t steps_done;
    nnp_status error;
    double t_submit, t_admit, t_done;   /* seconds on the server clock */
} replica_status;

/* Copies the replica into the host queue and returns a ticket; never blocks
 * on the device.  NNP_EINVAL for bad geometry, NNP_ENOMEM if it can never fit
 * the budget. */
nnp_status replica_submit(nnp_server* server, const replica_desc* desc, uint64_t* ticket);
/* Status of a ticket; for DONE replicas, pos_out/vel_out (host [n][3], or
 * NULL) receive the final state. */
nnp_status replica_poll(nnp_server* server, uint64_t ticket, replica_status* out,
                        double* pos_out, double* vel_out);
/* Advances the resident set by up to max_outer_steps outer steps.  A
 * boundary (retirement, admission, repacking) comes at the start of the
 * call and whenever a resident replica reaches its step count; between
 * boundaries the steps run as one integrator call (recorded outer steps
 * replayed as a graph, one status check at its end), so the step count of
 * a call bounds the wait of replicas queued meanwhile.  Returns early when
 * nothing is resident.  *n_resident receives the resident count. */
nnp_status nnp_server_progress(nnp_server* server, int32_t max_outer_steps, int32_t* n_resident);
/* Copies up to cap per-replica step latencies (seconds between consecutive
 * outer-step completions of a replica, the first from its admission, on the
 * device's constant-rate wall clock: every outer step ends with a
 * timestamp). */
nnp_status nnp_server_step_latencies(nnp_server* server, double* out, int64_t cap, int64_t* n_out);
/* Device bytes that one replica of n atoms in a box of edge `box` occupies
 * when resident alone (state, neighbour lists and scratch); a resident set
 * needs about the sum of its members'. */
nnp_status nnp_server_replica_bytes(const nnp_server* server, int64_t n, double box, size_t* bytes);
/* Server clock now (seconds). */
double nnp_server_clock(const nnp_server* server);

/* ------------------------------------------------------------- diagnostics
 * Device-time measurement of named launch sites ("message_fwd",
 * "message_bwd", "nc_message_fwd", "nc_message_bwd", "head_fwd", "gemm",
 * "nbr_fill", "baoa").  While a site is enabled each of its launches is
 * bracketed by two HIP events on the launch's stream; nnp_timer_read waits
 * for them and returns the summed duration (ms) and the number of launches
 * (reset != 0 clears the record). */
nnp_status nnp_timer_enable(const char* site, int32_t on);
nnp_status nnp_timer_read(const char* site, double* total_ms, int64_t* launches, int32_t reset);

/* ------------------------------------------------------- kernel choice --
 * Message kernels of the conservative embedding (the message step
 * s_i += sum_j a_ij, v_i += sum_j (b_ij v_j + u_ij c_ij) of the models
 * section above, after the paper's Methods "Model architecture", and its
 * reverse), chosen process-wide for launches issued after the call:
 *   NNP_MP_AUTO (0): the matrix-core kernels for the shapes they cover
 *     (width 128, 16 Bessel functions, cosine cutoff, force evaluation);
 *     the radial filter runs there as split FP16 products at FP32-equivalent
 *     precision; the vector kernels elsewhere.  In that shape, with at most
 *     8 species, the first layer (whose neighbour features depend on the
 *     species alone and whose vector input is zero) is evaluated from
 *     per-atom sums of the radial basis by neighbour species and four dense
 *     products instead of per-edge feature work (the same function: the
 *     filter is linear in the basis); its reverse, for forces, likewise.
 *   NNP_MP_VECTOR (1): the vector kernels (plain FP32 filter) everywhere.
 *   NNP_MP_EDGE (2): as NNP_MP_AUTO, but the first layer per edge on the
 *     matrix-core kernels too.
 * All give results within FP32 rounding of each other; this is for
 * measuring one against another.  Other values: NNP_EINVAL. */
#define NNP_MP_AUTO 0
#define NNP_MP_VECTOR 1
#define NNP_MP_EDGE 2
nnp_status nnp_set_message_kernels(int32_t mode);

/* Kernel selection for the per-atom perceptrons and linear maps of FP32
 * models (every dense product of the models section: phi, the update block's
 * U, V and mixing perceptron, the readout, the NC projections, and the
 * input adjoints of each), chosen process-wide for launches issued after the
 * call:
 *   NNP_DENSE_AUTO (0): products with K of 128, 256 or 384 and N a
 *     multiple of 32 run on the bfloat16 matrix cores of one kernel family:
 *     for FP32 models with both operands split into three bfloat16 pieces
 *     (the six piece products down to 2^-18, float32 accumulation:
 *     FP32-equivalent), for BF16 models with the operands rounded to
 *     bfloat16; other shapes on the older kernels.
 *   NNP_DENSE_FP32 (1): the older kernels everywhere (float32 operands for
 *     FP32 models, bfloat16-rounded operands for BF16 models).
 * Other values: NNP_EINVAL. */
#define NNP_DENSE_AUTO 0
#define NNP_DENSE_FP32 1
nnp_status nnp_set_dense_kernels(int32_t mode);

#ifdef __cplusplus
}
#endif
#endif /* NNP_H */
