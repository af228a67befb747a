// Device-side model object and the scratch layout of one force evaluation.
#pragma once

#include "common.h"
#include "kernels.h"

namespace nnp {

constexpr int kMaxLayers = 4;
constexpr int kChunk = 2048;  // rows per partial sum in weight adjoints

struct LayerOff {
    int64_t W1, b1, W2, b2, Wr, br, U, V, M1, m1, M2, m2;
};

// Weights live as one float32 device vector in manifest order; every tensor
// is addressed by its manifest offset (U and V are adjacent, so [U; V] is a
// single [2F][F] matrix; likewise [Wq; Wk] is one [2 H n_c][F] matrix).
struct Model {
    nnp_model_desc desc{};
    float* w = nullptr;
    int64_t n_weights = 0;
    int64_t off_emb = 0, off_Wo = 0, off_bo = 0, off_wo = 0, off_beta = 0, off_Wq = 0, off_Wk = 0, off_WV = 0;
    LayerOff loff[kMaxLayers]{};
    void layout();
    int n_layers() const { return desc.kind == NNP_MODEL_CONS ? desc.n_layers : 1; }
    const float* p(int64_t off) const { return w + off; }
    bool bf16() const { return desc.precision == NNP_BF16; }
    // First layer per species (functions of the weights only, refreshed when
    // the weights change): [S][F] pre-activation, [S][F] hidden, [S][3F] phi.
    float* tab = nullptr;
    float* h1_tab() const { return tab; }
    float* z_tab() const { return tab + int64_t(desc.n_species) * desc.width; }
    float* phi_tab() const { return tab + 2 * int64_t(desc.n_species) * desc.width; }
    // NC models of width <= 32: the update-block and projection weights
    // (UV, M1, M2, W_qk, W_V) as the LDS image of the fused update kernel
    // (pack_nc_weights), BF16-rounded for BF16 models; refreshed with the
    // tables.
    float* ncw = nullptr;
    // A mirror of the weight vector in which every matrix that input adjoints
    // multiply by (out = G W) is stored transposed at its own offset, so those
    // products run as X W^T with k contiguous in both operands.
    float* wT = nullptr;
    const float* pT(int64_t off) const { return wT + off; }
    // The matrices of both mirrors that X W^T products take as W, split into
    // three bfloat16 pieces (hi, mid, lo) for the matrix-core dense kernels
    // (BF16 models read only hi, the weights rounded to bfloat16).  Piece p of the matrix at offset off starts at element
    // 2 off of piece array p (16-byte aligned whenever off is a multiple of
    // 4); arrays of 2 n_weights elements (rounded up to 8), w's three then
    // wT's three.
    uint16_t* wx = nullptr;
    int64_t wx_stride() const { return (2 * n_weights + 7) / 8 * 8; }
    const uint16_t* px(int64_t off) const { return wx ? wx + 2 * off : nullptr; }
    const uint16_t* pxT(int64_t off) const { return wx ? wx + 3 * wx_stride() + 2 * off : nullptr; }
    // Per layer: the power-of-two scale of the filter weights used by the
    // matrix-core message kernels, and its inverse.
    float* mxs = nullptr;
    const float* mx_scale(int l) const { return mxs + 2 * l; }
    // Conservative models of the matrix-core message shape: the first
    // layer's tables by neighbour species (launch_sp_tables), T [2][F][ep]
    // then TT [2][pp][F] (species_sum_pitches), and the same split into
    // three bfloat16 pieces (piece stride sp_xs()) for the matrix-core
    // products.
    float* sp = nullptr;
    uint16_t* sp_x = nullptr;
    int sp_pp = 0, sp_ep = 0;
    int64_t sp_count() const { return 2 * int64_t(desc.width) * (sp_ep + sp_pp); }
    int64_t sp_xs() const { return (sp_count() + 7) / 8 * 8; }
    const float* sp_T(int c) const { return sp + int64_t(c) * desc.width * sp_ep; }
    const float* sp_TT(int c) const { return sp + 2 * int64_t(desc.width) * sp_ep + int64_t(c) * sp_pp * desc.width; }
    const uint16_t* sp_Tx(int c) const { return sp_x + int64_t(c) * desc.width * sp_ep; }
    const uint16_t* sp_TTx(int c) const {
        return sp_x + 2 * int64_t(desc.width) * sp_ep + int64_t(c) * sp_pp * desc.width;
    }
    void refresh_tables(hipStream_t s);
};

struct LayerBuf {
    float *h1, *zphi, *phi, *smid, *vmid, *UV, *X, *a1, *z, *pqo;
    float* pv = nullptr;  // phi_b * v_in (matrix-core message kernels, layers past the first)
};

struct ModelBuf {
    float* s[kMaxLayers + 1];
    float* v[kMaxLayers + 1];
    LayerBuf layer[kMaxLayers];
    float *ao = nullptr, *zo = nullptr, *Ei = nullptr;
    float *QK = nullptr, *Vh = nullptr, *gQK = nullptr, *gVh = nullptr;
    float *gs = nullptr, *gs2 = nullptr, *gv = nullptr, *gv2 = nullptr, *gpqo = nullptr, *ga1 = nullptr,
          *gX = nullptr, *gUV = nullptr, *gphi = nullptr, *gh1 = nullptr;
    float *chunk_part = nullptr, *mp_part = nullptr, *filt_sum = nullptr;
    // per-atom virial shares: of the last evaluation, and a running sum
    float *vir = nullptr, *vir_sum = nullptr;
    // first layer by neighbour species: the edge sums (forward) or the P
    // tables (reverse), [n][NS] then [3n][NS]; null when not carved
    float* sp = nullptr;
    // NC models: the edges within the cutoff as records for the pair head
    // (list capacity E), and their count per atom; null when not carved
    NcEdge* nc_edges = nullptr;
    int* nc_ecnt = nullptr;
    int64_t nc_edge_cap = 0;
    // prepared edges of the matrix-core message kernels (list capacity E)
    int* ecnt = nullptr;
    EdgeRec* erec = nullptr;
    uint4* ehalf = nullptr;
    // first layer per species: pre-activation, hidden, phi, and adjoints
    float *h1_tab = nullptr, *z_tab = nullptr, *phi_tab = nullptr, *gphi_tab = nullptr, *gh1_tab = nullptr;
};

struct SysTables {
    int64_t* rep_start;
    double *box, *inv_box;
    uint64_t *seed, *stream, *step_base;
    int* flags;
    int* rep_bad;
    long long* rebuilds;
    uint64_t* o_step;  // O-steps since the start of a respa call (read by k_baoa, advanced by the kicks)
};

struct RespaBuf {
    double *pos, *vel, *pos_ref, *energy;
    float *f_cons, *f_nc;
};

void launch_reverse(int n, const int* run, const int* status, const int* offsets, const int* nbr, int* rev,
                    hipStream_t s);
void launch_reduce_chunks(int64_t count, int nchunks, const float* part, int64_t stride, float* out, bool accum,
                          hipStream_t s);
struct CallScratch;
size_t call_scratch_bytes(const Model* cons, const Model* nc, int64_t n, int32_t n_rep, int64_t E);
void check_system(const nnp_system* sys);
nnp_status respa_run(const Model* cons, const Model* nc, respa_state* st, const respa_params* p, int32_t n_outer,
                     void* ws, size_t ws_bytes, hipStream_t s, const uint64_t* seeds, const uint64_t* streams,
                     const uint64_t* step_base, int* rep_bad, uint64_t* stamps = nullptr);
void launch_split_filter_grad(int rows, int K, const float* sum, float* dWr, float* dbr, hipStream_t s);

}  // namespace nnp
