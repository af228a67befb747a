// Argument blocks of the message kernels (internal): the edge geometry and
// the forward and reverse message-step operands.
#pragma once

#include "common.h"

namespace nnp {

// One edge within the cutoff, as prepared for the matrix-core message
// kernels (list order within each atom's row).
struct EdgeRec {
    int j, t;       // neighbour, its species (clamped)
    float fc, dfc;  // f(r), f'(r)
    float u[3];     // r_ij / r
    float ir;       // 1 / r
};

// One NC edge within the cutoff as the NC message step leaves it for the
// pair head (list order within each owner's row): neighbour, r, unit vector
// and the envelope-weighted Bessel values B_h(r) u(r / rc), float32.
struct NcEdge {
    int j;
    float r;
    float u[3];
    float pad[3];
    float ef[8];
};

struct MpGeom {
    int n;
    const double* pos;
    const int* species;
    int n_species;  // species indices are clamped to [0, n_species) before any table lookup
    RepGeom geom;
    const int* off;
    const int* nbr;
    double rc, rc2, bessel_norm, pi_over_rc, inv_rc;
    // Prepared edges (launch_edge_prep), or nullptr: per atom i, ecnt[i]
    // edges within the cutoff at list positions off[i] .. off[i] + ecnt[i],
    // with records erec[p] and the radial values as FP16 pairs ehalf[p][8]
    // (e_k f hi, e_k f lo, d/dr hi, d/dr lo; 16 values each).
    const int* ecnt;
    const EdgeRec* erec;
    const uint4* ehalf;
    // Rows in a working order (or nullptr: the caller's): the caller's index
    // of row i, under which the per-atom outputs (forces, energies, virial
    // shares) are stored.
    const int* perm;
};

struct MpFwd {
    const float *s_in, *v_in, *phi, *Wr, *br;
    float *s_out, *v_out;
    // first layer: inputs are s = emb[t], v = 0, and phi = phi_tab[t] per species
    const int* species;
    const float* phi_tab;  // [S][3F] or nullptr
    const float* emb;      // [S][F]
    const float* mx_scale;  // [2] filter-weight scale and its inverse for the matrix-core kernels, or nullptr
    // [n][3][F] products phi_b * v_in per atom (phi_b: the second third of
    // phi, which gates the neighbour's vector features): written by the
    // matrix-core forward of layers past the first, read there and by the
    // reverse in place of phi_b and v_in; ignored elsewhere
    float* pv;
    // NC forward (vector kernel, F <= 64): when set, the edges within the
    // cutoff are also written as records at off[i] + rank (rank among the
    // atom's edges within the cutoff), with their count per atom
    NcEdge* edge_out;
    int* edge_cnt;
};

struct MpBwd {
    const float *v_in, *phi, *gsm, *gvm, *Wr, *br;
    float *gphi, *gv_in;
    const int* species;
    const float* phi_tab;  // first layer: phi = phi_tab[t], v_in = 0 (gv_in is not written)
    int want_gphi;         // write the phi adjoints
    float* force;       // [3][n] forces -dE/dx (GEO): written, or added to with accum_force
    int accum_force;
    float* wgrad_part;  // [blocks][3F][K + 1] filter weight adjoints (WGRAD)
    // [n] or nullptr (GEO): per owner atom i, 1/2 sum_j r_ij . f_ij of its pair
    // forces f_ij (its share of the virial -sum F . q), written or added to
    // with accum_force
    float* vir;
    const float* mx_scale;  // [2] filter-weight scale and its inverse for the matrix-core kernels, or nullptr
    const float* pv;        // phi_b * v_in as written by the matrix-core forward (layers past the first)
};

}  // namespace nnp
