// Launchers and argument blocks of the libnnp kernels (internal).
#pragma once

#include <cmath>
#include <string>
#include <vector>

#include "common.h"
#include "mp.h"

namespace nnp {

// Brackets one launch with HIP events when its site is enabled
// (nnp_timer_enable); otherwise costs one branch.
// With `by_launch`, the events are not recorded around the launch but handed
// to it (hipExtLaunchKernelGGL), which timestamps the kernel itself: the
// interval then excludes dispatch gaps and host-side delays.
struct ScopedTimer {
    const char* name;
    hipStream_t stream;
    hipEvent_t a = nullptr, b = nullptr;
    bool active = false;
    bool by_launch = false;
    ScopedTimer(const char* site, hipStream_t s, bool by_launch = false);
    ~ScopedTimer();
};

// ---------------------------------------------------------------- neighbours
struct CellPlan {
    std::vector<int> m;     // cells per side per replica (1 = whole replica)
    std::vector<int> base;  // first global cell of each replica
    int n_cells = 0;
    // Cell numbering: the cell at lexicographic position l ((cx m + cy) m + cz)
    // of replica r is number code[base_r + l]; lex is the inverse.  Within a
    // replica the numbers follow the Morton (bit-interleaved) order of the
    // cell coordinates, so consecutive cells, and the atoms the cell order
    // puts together, form compact blocks of space.
    std::vector<int> code, lex;
};

struct NbrScratch {
    int *grid_m, *grid_base, *cell_code, *cell_lex, *cell_of_atom, *slot_of_atom, *cell_count, *cell_start,
        *cell_atoms, *counts, *tmp_off, *status;
    double* cell_pos;  // [3][n] positions in cell order
};

CellPlan plan_cells(const nnp_system& sys, double radius);
int64_t max_cells(int64_t n_atoms, int32_t n_rep);
void carve_nbr_scratch(Arena& a, int64_t n, int32_t n_rep, NbrScratch& s);
void upload_cell_plan(const CellPlan& plan, NbrScratch& s, hipStream_t stream);
// cell_rows: rows and entries in the cell order of this list build (s.cell_atoms
// maps them to the caller's indices, s.cell_pos holds the positions in that
// order); each row still ascending in caller index.
void launch_build(int n, const double* pos, const RepGeom& geom, const CellPlan& plan, NbrScratch& s, const int* run,
                  double radius, int64_t capacity, int* offsets, int* nbr, int* rev, double* pos_ref,
                  hipStream_t stream, bool cell_rows = false);
// pos: the positions in the order of the input list's rows; key (or
// nullptr): caller's index of a row, for the reverse entries
// src_status (or nullptr): the input list's build status; a failed build
// leaves this list untouched
void launch_filter(int n, const double* pos, const RepGeom& geom, NbrScratch& s, const int* run, const int* off_in,
                   const int* nbr_in, double radius, int64_t capacity, int* offsets, int* nbr, int* rev, int* status,
                   hipStream_t stream, const int* key = nullptr, const int* src_status = nullptr);
// After a build into spare buffers that ran and succeeded (s.status): the
// spare list (and, with order_src, the order and row-ordered positions and
// species) copied over the ones in use.
void launch_adopt_lists(int n, const int* run, const NbrScratch& s, const int* off_src, const int* nbr_src,
                        int64_t capacity, int* off_dst, int* nbr_dst, const int* order_src, int* order_dst,
                        const double* pos_src, double* pos_dst, const int* sp_src, int* sp_dst, hipStream_t stream);
// After a cell-order build that succeeded: the permutation into order[2n]
// (row -> caller index, then caller index -> row), positions and species in
// row order.
void launch_commit_order(int n, const NbrScratch& s, const int* run, const int* species, int* order, double* pos_m,
                         int* species_m, hipStream_t stream);
// pos_m / species_m (or nullptr) in row order from the caller's arrays
void launch_gather_rows(int n, const int* order, const double* pos, const int* species, double* pos_m,
                        int* species_m, hipStream_t stream);
// The identity order into order[2n], with pos_m and species_m copied.
void launch_reset_rows(int n, int* order, const double* pos, const int* species, double* pos_m, int* species_m,
                       hipStream_t stream);
void launch_set_flag(int* flag, int value, hipStream_t stream);
void launch_disp_check(int n, const double* pos, const double* ref, double thr, int* flag, hipStream_t stream);
// Ends a (possibly skipped) rebuild: counts it, clears the trigger and, with
// `maxd2`, restarts the displacement record ([0] since the build, [1] at the
// previous decision).
void launch_finish_rebuild(int* flag, long long* n_rebuilds, unsigned* maxd2, hipStream_t stream);
// Per-outer-step decision: set `flag` when the largest displacement since
// the last build, extrapolated over one more outer step from its growth
// during the previous one, may reach `thr`.
void launch_predict_rebuild(unsigned* maxd2, double thr, int* flag, hipStream_t stream);

// --------------------------------------------------------------------- GEMM
enum { EPI_NONE = 0, EPI_SILU = 1, EPI_DSILU = 2 };

struct GemmArgs {
    int M, N, K;
    const float* A;
    int64_t sam, sak;
    const float* B;
    int64_t sbk, sbn;
    float* C;
    int64_t ldc;
    const float* bias;
    int epi;
    float* pre;
    int64_t ldp;
    int accum;
    int64_t chunk_rows;    // > 0: split the K range into chunks along grid.z
    int64_t chunk_stride;  // C offset between chunks
    int bf16;              // operands rounded to bfloat16 (float32 accumulation)
    // B(k, n) = B[n * sbn + k] also as three bfloat16 pieces (hi, mid, lo;
    // hi + mid + lo = B to within 2^-24 relative), piece p at Bx + p * bxs,
    // same [N][K] layout; lets FP32 products run on bfloat16 matrix cores
    const uint16_t* Bx;
    int64_t bxs;
    // float32 register-direct kernel only: rows from b_split on multiply by
    // B2 instead of B (same layout)
    const float* B2;
    int64_t b_split;
    // split-bfloat16 kernel: row tiles from b_split on (a multiple of 128)
    // take the pieces at Bx2 instead of Bx
    const uint16_t* Bx2;
};

void launch_gemm(const GemmArgs& g, hipStream_t s);
void gemm_xwt(int M, int N, int K, const float* X, int ldx, const float* W, const float* b, float* out, int ldo,
              int epi, float* pre, int ldp, bool accum, hipStream_t s, bool bf16 = false,
              const uint16_t* Wx = nullptr, int64_t wx_stride = 0);
// out = X W^T with float32 operands on the matrix cores, rows m >= m_split
// taking W2 (same [N][K] layout) instead of W; m_split a multiple of 32,
// N <= 160, K and the strides multiples of 4.
// The same on the split-bfloat16 kernel (FP32-equivalent): pieces Wx and Wx2
// (piece stride wx_stride), m_split a multiple of 128; false (nothing
// launched) where the kernel cannot take the shapes or the float32 kernels
// are selected.
bool gemm_x3_split(int M, int N, int K, const float* X, int ldx, const uint16_t* Wx, const uint16_t* Wx2,
                   int64_t wx_stride, int m_split, float* out, int ldo, hipStream_t s);
void gemm_xwt_f32_split(int M, int N, int K, const float* X, int ldx, const float* W, const float* W2, int m_split,
                        float* out, int ldo, hipStream_t s);
// dst[p * piece_stride + e] = piece p (hi, mid, lo) of src[e] as bfloat16
void launch_split3(const float* src, int64_t count, uint16_t* dst, int64_t piece_stride, hipStream_t s);
// 0: FP32 products on split-bfloat16 matrix cores where the shapes allow
// (default); 1: float32-operand kernels only
void set_dense_mode(int mode);
// dst[c][r] = src[r][c] for a rows x cols row-major matrix
void launch_transpose(int rows, int cols, const float* src, float* dst, hipStream_t s);
void gemm_gw(int M, int N, int K, const float* G, int ldg, const float* W, float* out, int ldo, int epi,
             const float* pre, int ldp, bool accum, hipStream_t s, bool bf16 = false);
void gemm_wgrad(int M, int N, int K, const float* G, int ldg, const float* X, int ldx, float* dW, float* scratch,
                int chunk, bool accum, hipStream_t s);
void colsum(int M, int N, const float* G, int ldg, float* db, float* scratch, int chunk, bool accum, hipStream_t s);

// ------------------------------------------------------------ edge kernels
// argument blocks: mp.h
int mp_blocks(int n, int F);
// matrix-core message kernels (F = 128, K = 16, cosine cutoff; forces, no weight adjoints)
bool message_mx_shape(int F, int K, int cut);
bool message_mx_active(int F, int K, int cut);  // shape covered and not switched off
bool species_sum_active();                       // first layer by neighbour species not switched off
// With Es, also the first conservative layer's edge sums by neighbour species
// (rows Es [n][ep], Ev [3n][ep]; S species, S <= 8; mp_species.hip).
void launch_edge_prep(const MpGeom& mg, int* ecnt, EdgeRec* erec, uint4* ehalf, hipStream_t s, float* Es = nullptr,
                      float* Ev = nullptr, int S = 0, int ep = 0);
// First layer of the conservative message step summed by neighbour species
// (mp_species.hip): row pitches (pp of the per-atom tables P, a multiple of
// 32; ep of the edge sums, 128 or 256), shapes covered, the weight tables
// T [2][F][ep] and TT [2][pp][F] (refreshed with the weights; the forward
// edge sums come from launch_edge_prep) and the reverse edge kernel from
// P0 [n][pp], P2 [3n][pp].
void species_sum_pitches(int n_species, int& pp, int& ep);
bool species_sum_shape(int F, int K, int cut, int n_species);
void launch_sp_tables(int F, int S, const float* Wr, const float* br, const float* phi, const float* emb, float* T,
                      float* TT, hipStream_t s);
void launch_sp_bwd(const MpGeom& mg, int S, const float* P0, const float* P2, float* force, bool accum, float* vir,
                   hipStream_t s);
void launch_message_fwd_mx(const MpGeom& mg, const MpFwd& a, hipStream_t s, const ScopedTimer& t);
void launch_message_bwd_mx(const MpGeom& mg, const MpBwd& a, hipStream_t s, const ScopedTimer& t);
void launch_filter_scale(int count, const float* Wr, float* out, hipStream_t s);
void launch_message_fwd(int F, int K, int cut, const MpGeom& mg, const MpFwd& a, hipStream_t s);
void launch_message_bwd(int F, int K, int cut, const MpGeom& mg, const MpBwd& a, bool geo, bool wgrad,
                        hipStream_t s);

// ----------------------------------------------------------- block kernels
void launch_embed(int n, int F, int S, const int* species, const float* emb, float* s, float* v, hipStream_t st);
void launch_build_x(int n, int F, const float* smid, const float* UV, float* X, hipStream_t st);
void launch_update_combine(int n, int F, const float* smid, const float* vmid, const float* UV, const float* pqo,
                           float* s_out, float* v_out, hipStream_t st);
void launch_update_combine_bwd(int n, int F, const float* UV, const float* pqo, const float* gs, const float* gv,
                               float* gpqo, float* gUV, hipStream_t st);
void launch_norm_bwd(int n, int F, const float* gs, const float* gX, const float* X, const float* UV, float* gsmid,
                     float* gUV, hipStream_t st);
// perm (or nullptr): E_i of row i stored at Ei[perm[i]]
void launch_readout(int n, int F, int S, const float* z, const float* wo, const float* beta, const int* species, float* Ei,
                    hipStream_t st, const int* perm = nullptr);
void launch_readout_bwd(int n, int F, const float* ao, const float* wo, float* gao, hipStream_t st);
void launch_rep_sum(int n_rep, const int64_t* rep_start, const float* x, double* out, hipStream_t st);
void launch_emb_grad(int n, int F, int S, const int* species, const float* gs0, float* gemb, hipStream_t st);
// vir_set / vir_add ([n] or nullptr): per owner i, sum_j F_ij . r_ij (its
// share of the NPT virial proxy), written / added to
void launch_head_fwd_rec(const MpGeom& mg, const int* cnt, const NcEdge* rec, const float* QK, const float* Vh,
                         float* F, bool accum, hipStream_t st, float* vir_set, float* vir_add);
void launch_head_fwd(const MpGeom& mg, const float* QK, const float* Vh, float* F, bool accum, hipStream_t st,
                     float* vir_set = nullptr, float* vir_add = nullptr);
void launch_head_bwd(const MpGeom& mg, const float* QK, const float* Vh, const float* gF, float* gQK, float* gVh,
                     hipStream_t st);

struct NcUpdateArgs {
    int n;
    const float *smid, *vmid;                          // message outputs [n][F], [n][3][F]
    const float *wt, *m1, *m2;                          // packed weights (pack_nc_weights), biases
    float *QK, *Vh;                                    // [n][2 H n_c], [n][3][n_l]
};
// Fused update block + q/k/V projections of the NC embedding (widths <= 32);
// returns false when the width is not supported by the fused kernel.
bool launch_nc_update_proj(const NcUpdateArgs& a, int F, bool bf16, hipStream_t st);
// LDS image of U|V, M1, M2, W_qk and W_V for k_nc_update_proj: one row per
// output, rows padded by four floats (rounded to bfloat16 when bf16);
// nc_image_count(F) floats
void pack_nc_weights(int F, const float* UV, const float* M1, const float* M2, const float* Wqk, const float* WV,
                     bool bf16, float* out, hipStream_t st);
int64_t nc_image_count(int F);

// -------------------------------------------------------------- integrator
struct BaoaArgs {
    int n;
    double* pos;
    double* vel;
    const double* mass;
    const double* gamma;
    const float* force;
    double dt;
    double temperature;
    const int32_t* rep_of_atom;
    const int64_t* rep_start;
    const uint64_t* seed;
    const uint64_t* stream;
    const uint64_t* step_base;
    uint64_t step_offset;
    const uint64_t* step_dev;  // optional device O-step counter added to step_offset
    int ffl;
    const double* pos_ref;
    double disp_thr2;
    int* flag;         // set when an atom moved more than sqrt(disp_thr2) since the last build
    unsigned* maxd2;   // optional: running maximum of the squared displacement (float bits)
    // 1: the opening kick is B(dt) instead of B(dt/2), standing for the
    // closing B(dt/2) of the previous step with the same force as well
    int full_kick;
    // optional: the new positions also into pos_rows[c * n + row[i]] (the
    // force evaluations' copy in their working row order)
    double* pos_rows;
    const int* row;
};

// v += half_dt * ACC * (Fa - Fb) / m; with `bump`, also advances that O-step
// counter by bump_by (read by the next k_baoa)
void launch_kick(int n, double* vel, const double* mass, const float* Fa, const float* Fb, double half_dt,
                 hipStream_t s, uint64_t* bump = nullptr, uint64_t bump_by = 1);
void launch_set_u64(uint64_t* p, uint64_t value, hipStream_t s);
void launch_disp_record(int n, const double* pos, const double* pos_ref, unsigned* maxd2, hipStream_t s);
// device wall-clock ticks (hipDeviceAttributeWallClockRate) written once the stream reaches it
void launch_stamp(uint64_t* out, hipStream_t s);
// zero fill as a kernel (safe inside recorded graphs); with `run`, only when *run != 0
void launch_zero(void* p, int64_t words, const int* run, hipStream_t s);
void launch_virial_combine(int n, const float* wc, const float* wl, const float* ws, float inv_n, float* out,
                           hipStream_t s);
void launch_add(int n, const float* x, float* y, hipStream_t s);  // y += x
bool timers_active();
void launch_baoa(const BaoaArgs& a, hipStream_t s);
// stochastic cell rescaling (pressures in kcal/mol/A^3, beta in their inverse)
struct ScrArgs {
    double p0, beta, tau, dt, temperature;
    uint64_t seed, stream, step;
};
void launch_scr(int n_rep, const double* ke, const double* virial, double* box, double* mu, const ScrArgs& a,
                hipStream_t s);
void launch_scale(int n, const int32_t* rep_of_atom, const double* mu, double* pos, double* vel, hipStream_t s);
// atoms per block of the chunked kinetic-energy reduction; part: scratch of
// n_rep * chunks doubles, chunks = the largest replica's atom count over
// kKeChunk, rounded up (without it, one block per replica)
constexpr int kKeChunk = 2048;
void launch_kinetic(int n_rep, const int64_t* rep_start, int n, const double* pos, const double* vel,
                    const double* mass, double* ke, int* bad, hipStream_t s,
                    const int32_t* rep_of_atom = nullptr, double* part = nullptr, int chunks = 0);

}  // namespace nnp
