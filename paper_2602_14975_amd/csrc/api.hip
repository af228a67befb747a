// C entry points of libnnp (see include/nnp.h) and the host-side drivers that
// sequence the kernels of one force evaluation or one integration call.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>

#include "common.h"
#include "kernels.h"
#include "model.h"

namespace nnp {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

}  // namespace nnp

using namespace nnp;

#define NNP_API_BEGIN try {
#define NNP_API_END                                                        \
    }                                                                      \
    catch (const Fail& f) {                                                \
        return f.code;                                                     \
    }                                                                      \
    catch (const std::exception& e) {                                      \
        set_error(std::string("internal error: ") + e.what());             \
        return NNP_EINVAL;                                                 \
    }                                                                      \
    return NNP_OK;

extern "C" const char* nnp_last_error(void) { return g_err.c_str(); }
extern "C" int32_t nnp_abi_version(void) { return 4; }

// ===================================================================== model
namespace nnp {

static int64_t manifest_count(const nnp_model_desc& d) {
    const int64_t F = d.width, K = d.n_rbf, S = d.n_species;
    const int64_t block = F * F + F + 3 * F * F + 3 * F + 3 * F * K + 3 * F + 2 * F * F + 2 * F * F + F +
                          3 * F * F + 3 * F;
    int64_t n = S * F;
    if (d.kind == NNP_MODEL_CONS) {
        n += d.n_layers * block + F * F + F + F + S;
    } else {
        const int64_t H = d.n_s + d.n_l;
        n += block + 2 * H * d.n_c * F + d.n_l * F;
    }
    return n;
}

void Model::layout() {
    const int64_t F = desc.width, K = desc.n_rbf, S = desc.n_species;
    int64_t o = 0;
    auto take = [&](int64_t count) { int64_t at = o; o += count; return at; };
    off_emb = take(S * F);
    const int L = desc.kind == NNP_MODEL_CONS ? desc.n_layers : 1;
    for (int l = 0; l < L; ++l) {
        LayerOff& lo = loff[l];
        lo.W1 = take(F * F); lo.b1 = take(F);
        lo.W2 = take(3 * F * F); lo.b2 = take(3 * F);
        lo.Wr = take(3 * F * K); lo.br = take(3 * F);
        lo.U = take(F * F); lo.V = take(F * F);
        lo.M1 = take(2 * F * F); lo.m1 = take(F);
        lo.M2 = take(3 * F * F); lo.m2 = take(3 * F);
    }
    if (desc.kind == NNP_MODEL_CONS) {
        off_Wo = take(F * F); off_bo = take(F); off_wo = take(F); off_beta = take(S);
    } else {
        const int64_t H = desc.n_s + desc.n_l;
        off_Wq = take(H * desc.n_c * F); off_Wk = take(H * desc.n_c * F); off_WV = take(desc.n_l * F);
    }
    n_weights = o;
}

}  // namespace nnp

extern "C" nnp_status nnp_model_create(const nnp_model_desc* desc, nnp_model** out) {
    NNP_API_BEGIN
    NNP_REQUIRE(desc && out, NNP_EINVAL, "null argument");
    *out = nullptr;
    const nnp_model_desc& d = *desc;
    NNP_REQUIRE(d.kind == NNP_MODEL_CONS || d.kind == NNP_MODEL_NC, NNP_EINVAL, "unknown model kind");
    NNP_REQUIRE(d.width == 8 || d.width == 16 || d.width == 32 || d.width == 64 || d.width == 128, NNP_EINVAL,
                "width must be 8, 16, 32, 64 or 128");
    NNP_REQUIRE(d.n_species >= 1 && d.n_species <= 8, NNP_EINVAL, "n_species must be in 1..8");
    NNP_REQUIRE(d.cutoff > 0, NNP_EINVAL, "cutoff must be positive");
    NNP_REQUIRE(d.precision == NNP_FP32 || d.precision == NNP_BF16, NNP_EINVAL, "unknown precision");
    if (d.kind == NNP_MODEL_CONS) {
        NNP_REQUIRE(d.n_rbf == 16, NNP_EINVAL, "conservative model needs n_rbf = 16");
        NNP_REQUIRE(d.n_layers >= 1 && d.n_layers <= kMaxLayers, NNP_EINVAL, "n_layers must be in 1..4");
    } else {
        NNP_REQUIRE(d.n_rbf == 8 && d.n_s == 8 && d.n_l == 2 && d.n_c == 8 && d.poly_p == 5 && d.n_layers == 1,
                    NNP_EINVAL, "NC model needs n_rbf = n_s = n_c = 8, n_l = 2, poly_p = 5, one layer");
        NNP_REQUIRE(d.width <= 64, NNP_EINVAL, "NC width must be <= 64");
    }
    NNP_REQUIRE(d.weights != nullptr, NNP_EINVAL, "weights are required");
    const int64_t need = manifest_count(d);
    NNP_REQUIRE(d.n_weights == need, NNP_EINVAL,
                "weight vector has " + std::to_string(d.n_weights) + " entries, manifest needs " +
                    std::to_string(need));
    Model* m = new Model();
    m->desc = d;
    m->desc.weights = nullptr;
    m->layout();
    std::vector<float> w32(size_t(m->n_weights));
    for (int64_t k = 0; k < m->n_weights; ++k) w32[k] = float(d.weights[k]);
    hipError_t e = hipMalloc(&m->w, sizeof(float) * m->n_weights);
    if (e != hipSuccess) {
        delete m;
        set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
        return NNP_ENOMEM;
    }
    e = hipMemcpy(m->w, w32.data(), sizeof(float) * m->n_weights, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&m->tab, sizeof(float) * 5 * d.n_species * d.width);
    if (e == hipSuccess && d.kind == NNP_MODEL_NC && d.width <= 32)
        e = hipMalloc(&m->ncw, sizeof(float) * nc_image_count(d.width));
    if (e == hipSuccess) e = hipMalloc(&m->wT, sizeof(float) * m->n_weights);
    if (e == hipSuccess) e = hipMalloc(&m->mxs, sizeof(float) * 2 * kMaxLayers);
    if (e == hipSuccess && d.kind == NNP_MODEL_CONS && species_sum_shape(d.width, d.n_rbf, 0, d.n_species)) {
        species_sum_pitches(d.n_species, m->sp_pp, m->sp_ep);
        e = hipMalloc(&m->sp, sizeof(float) * m->sp_count());
        if (e == hipSuccess) e = hipMalloc(&m->sp_x, sizeof(uint16_t) * 3 * m->sp_xs());
    }
    if (e == hipSuccess) e = hipMalloc(&m->wx, sizeof(uint16_t) * 6 * m->wx_stride());
    if (e != hipSuccess) {
        (void)hipFree(m->w);
        if (m->tab) (void)hipFree(m->tab);
        if (m->ncw) (void)hipFree(m->ncw);
        if (m->wT) (void)hipFree(m->wT);
        if (m->mxs) (void)hipFree(m->mxs);
        if (m->wx) (void)hipFree(m->wx);
        if (m->sp) (void)hipFree(m->sp);
        if (m->sp_x) (void)hipFree(m->sp_x);
        delete m;
        set_error(std::string("model set-up: ") + hipGetErrorString(e));
        return NNP_EDEVICE;
    }
    try {
        m->refresh_tables(nullptr);
        NNP_HIP(hipStreamSynchronize(nullptr));
    } catch (...) {
        (void)hipFree(m->w);
        (void)hipFree(m->tab);
        if (m->ncw) (void)hipFree(m->ncw);
        (void)hipFree(m->wT);
        (void)hipFree(m->mxs);
        if (m->wx) (void)hipFree(m->wx);
        if (m->sp) (void)hipFree(m->sp);
        if (m->sp_x) (void)hipFree(m->sp_x);
        delete m;
        throw;
    }
    *out = reinterpret_cast<nnp_model*>(m);
    NNP_API_END
}

extern "C" void nnp_model_destroy(nnp_model* model) {
    if (!model) return;
    Model* m = reinterpret_cast<Model*>(model);
    if (m->w) (void)hipFree(m->w);
    if (m->tab) (void)hipFree(m->tab);
    if (m->ncw) (void)hipFree(m->ncw);
    if (m->wT) (void)hipFree(m->wT);
    if (m->mxs) (void)hipFree(m->mxs);
    if (m->wx) (void)hipFree(m->wx);
    if (m->sp) (void)hipFree(m->sp);
    if (m->sp_x) (void)hipFree(m->sp_x);
    delete m;
}

extern "C" int64_t nnp_model_n_weights(const nnp_model* model) {
    return model ? reinterpret_cast<const Model*>(model)->n_weights : -1;
}

extern "C" nnp_status nnp_model_set_weights_f32(nnp_model* model, const float* weights_dev, int64_t n_weights,
                                                void* stream) {
    NNP_API_BEGIN
    NNP_REQUIRE(model && weights_dev, NNP_EINVAL, "null argument");
    Model* m = reinterpret_cast<Model*>(model);
    NNP_REQUIRE(n_weights == m->n_weights, NNP_EINVAL, "weight count does not match the model");
    NNP_HIP(hipMemcpyAsync(m->w, weights_dev, sizeof(float) * n_weights, hipMemcpyDeviceToDevice,
                           static_cast<hipStream_t>(stream)));
    m->refresh_tables(static_cast<hipStream_t>(stream));
    NNP_API_END
}

// ============================================================ system tables
namespace nnp {

void check_system(const nnp_system* sys) {
    NNP_REQUIRE(sys && sys->pos && sys->species && sys->rep_start && sys->box, NNP_EINVAL, "incomplete system");
    NNP_REQUIRE(sys->n_atoms >= 1 && sys->n_atoms < (int64_t(1) << 31), NNP_EINVAL, "n_atoms out of range");
    NNP_REQUIRE(sys->n_rep >= 1, NNP_EINVAL, "n_rep must be >= 1");
    NNP_REQUIRE(sys->n_rep == 1 || (sys->rep_of_atom && sys->box_dev), NNP_EINVAL,
                "multi-replica systems need rep_of_atom and box_dev");
    NNP_REQUIRE(sys->rep_start[0] == 0 && sys->rep_start[sys->n_rep] == sys->n_atoms, NNP_EINVAL,
                "rep_start must run from 0 to n_atoms");
    for (int r = 0; r < sys->n_rep; ++r) {
        NNP_REQUIRE(sys->rep_start[r + 1] >= sys->rep_start[r], NNP_EINVAL, "rep_start must be non-decreasing");
        NNP_REQUIRE(sys->box[r] > 0 && std::isfinite(sys->box[r]), NNP_EINVAL, "box edges must be positive");
    }
}

void carve_tables(Arena& a, int32_t n_rep, SysTables& t) {
    t.rep_start = a.take<int64_t>(n_rep + 1);
    t.box = a.take<double>(n_rep);
    t.inv_box = a.take<double>(n_rep);
    t.seed = a.take<uint64_t>(n_rep);
    t.stream = a.take<uint64_t>(n_rep);
    t.step_base = a.take<uint64_t>(n_rep);
    t.flags = a.take<int>(16);
    t.rep_bad = a.take<int>(n_rep);
    t.rebuilds = a.take<long long>(1);
    t.o_step = a.take<uint64_t>(1);
}

// Uploads the replica tables of `sys` (pageable copies are staged by the
// runtime before hipMemcpyAsync returns).
RepGeom upload_tables(const nnp_system& sys, SysTables& t, hipStream_t s, std::vector<double>& host_scratch) {
    const int R = sys.n_rep;
    host_scratch.assign(size_t(2 * R), 0.0);
    for (int r = 0; r < R; ++r) {
        host_scratch[r] = sys.box[r];
        host_scratch[R + r] = 1.0 / sys.box[r];
    }
    NNP_HIP(hipMemcpyAsync(t.rep_start, sys.rep_start, sizeof(int64_t) * (R + 1), hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(t.box, host_scratch.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(t.inv_box, host_scratch.data() + R, sizeof(double) * R, hipMemcpyHostToDevice, s));
    RepGeom g{};
    g.rep_of_atom = R > 1 ? sys.rep_of_atom : nullptr;
    g.box = t.box;
    g.inv_box = t.inv_box;
    g.rep_start = t.rep_start;
    g.box0 = sys.box[0];
    g.inv0 = 1.0 / sys.box[0];
    return g;
}

// ========================================================= model scratch
void carve_model(Arena& a, const Model* m, int64_t n, int64_t E, bool for_wgrad, ModelBuf& b) {
    const int64_t F = m->desc.width;
    const int L = m->n_layers();
    b.vir = a.take<float>(n);
    b.vir_sum = a.take<float>(n);
    for (int l = 0; l <= L; ++l) {
        b.s[l] = a.take<float>(n * F);
        b.v[l] = a.take<float>(n * 3 * F);
    }
    const int64_t S = m->desc.n_species;
    b.h1_tab = m->h1_tab();
    b.z_tab = m->z_tab();
    b.phi_tab = m->phi_tab();
    b.gphi_tab = a.take<float>(S * 3 * F);
    b.gh1_tab = a.take<float>(S * F);
    for (int l = 0; l < L; ++l) {
        LayerBuf& lb = b.layer[l];
        lb.h1 = a.take<float>(n * F);
        lb.zphi = a.take<float>(n * F);
        lb.phi = a.take<float>(n * 3 * F);
        lb.smid = a.take<float>(n * F);
        lb.vmid = a.take<float>(n * 3 * F);
        lb.UV = a.take<float>(n * 6 * F);
        lb.X = a.take<float>(n * 2 * F);
        lb.a1 = a.take<float>(n * F);
        lb.z = a.take<float>(n * F);
        lb.pqo = a.take<float>(n * 3 * F);
    }
    if (m->desc.kind == NNP_MODEL_CONS) {
        b.ao = a.take<float>(n * F);
        b.zo = a.take<float>(n * F);
        b.Ei = a.take<float>(n);
        b.gs = a.take<float>(n * F);
        b.gs2 = a.take<float>(n * F);
        b.gv = a.take<float>(n * 3 * F);
        b.gv2 = a.take<float>(n * 3 * F);
        b.gpqo = a.take<float>(n * 3 * F);
        b.ga1 = a.take<float>(n * F);
        b.gX = a.take<float>(n * 2 * F);
        b.gUV = a.take<float>(n * 6 * F);
        b.gphi = a.take<float>(n * 3 * F);
        b.gh1 = a.take<float>(n * F);
        if (message_mx_shape(int(F), m->desc.n_rbf, 0)) {
            b.ecnt = a.take<int>(n);
            b.erec = a.take<EdgeRec>(E);
            b.ehalf = a.take<uint4>(8 * E);
            for (int l = 1; l < L; ++l) b.layer[l].pv = a.take<float>(n * 3 * F);
            if (m->sp) b.sp = a.take<float>(n * 4 * std::max(m->sp_pp, m->sp_ep));
        }
    } else {
        const int64_t HC = 2 * int64_t(m->desc.n_s + m->desc.n_l) * m->desc.n_c;
        b.QK = a.take<float>(n * HC);
        b.Vh = a.take<float>(n * 3 * m->desc.n_l);
        if (E > 1) {
            b.nc_edges = a.take<NcEdge>(E);
            b.nc_ecnt = a.take<int>(n);
            b.nc_edge_cap = E;
        }
        if (for_wgrad) {
            b.gQK = a.take<float>(n * HC);
            b.gVh = a.take<float>(n * 3 * m->desc.n_l);
            b.gs = a.take<float>(n * F);
            b.gs2 = a.take<float>(n * F);
            b.gv = a.take<float>(n * 3 * F);
            b.gv2 = a.take<float>(n * 3 * F);
            b.gpqo = a.take<float>(n * 3 * F);
            b.ga1 = a.take<float>(n * F);
            b.gX = a.take<float>(n * 2 * F);
            b.gUV = a.take<float>(n * 6 * F);
            b.gphi = a.take<float>(n * 3 * F);
            b.gh1 = a.take<float>(n * F);
            const int64_t maxNK = std::max<int64_t>({3 * F * F, HC * F, 2 * F * F});
            b.chunk_part = a.take<float>(int64_t(cdiv(3 * n, kChunk) + 1) * maxNK);
            b.mp_part = a.take<float>(int64_t(mp_blocks(int(n), int(F))) * 3 * F * (m->desc.n_rbf + 1));
            b.filt_sum = a.take<float>(3 * F * (m->desc.n_rbf + 1));
        }
    }
}

// Embedding forward.  The first layer's perceptron input is the species
// embedding, so its phi is evaluated once per species (a table of S rows);
// the message kernel then reads phi_tab[t_j] and the zero vector input
// implicitly.  Every intermediate needed by the reverse pass stays in `b`.
void Model::refresh_tables(hipStream_t s) {
    const int F = desc.width, S = desc.n_species;
    const LayerOff& lo = loff[0];
    gemm_xwt(S, F, F, p(off_emb), F, p(lo.W1), p(lo.b1), z_tab(), F, EPI_SILU, h1_tab(), F, false, s, bf16());
    gemm_xwt(S, 3 * F, F, z_tab(), F, p(lo.W2), p(lo.b2), phi_tab(), 3 * F, EPI_NONE, nullptr, 0, false, s, bf16());
    if (ncw) pack_nc_weights(F, p(lo.U), p(lo.M1), p(lo.M2), p(off_Wq), p(off_WV), bf16(), ncw, s);
    if (sp) {
        launch_sp_tables(F, S, p(lo.Wr), p(lo.br), phi_tab(), p(off_emb), sp, sp + 2 * int64_t(F) * sp_ep, s);
        launch_split3(sp, sp_count(), sp_x, sp_xs(), s);
    }
    // transposed mirror of the matrices used as G W; both mirrors split into
    // bfloat16 pieces
    auto tr = [&](int64_t off, int rows, int cols) {
        launch_transpose(rows, cols, p(off), wT + off, s);
        if (wx) {
            const int64_t cnt = int64_t(rows) * cols;
            launch_split3(p(off), cnt, wx + 2 * off, wx_stride(), s);
            launch_split3(wT + off, cnt, wx + 3 * wx_stride() + 2 * off, wx_stride(), s);
        }
    };
    for (int l = 0; l < n_layers(); ++l) {
        const LayerOff& ll = loff[l];
        launch_filter_scale(3 * F * (desc.n_rbf + 1), p(ll.Wr), mxs + 2 * l, s);  // Wr, then br
        tr(ll.W1, F, F);
        tr(ll.W2, 3 * F, F);
        tr(ll.U, 2 * F, F);
        tr(ll.M1, F, 2 * F);
        tr(ll.M2, 3 * F, F);
    }
    if (desc.kind == NNP_MODEL_CONS) {
        tr(off_Wo, F, F);
    } else {
        tr(off_Wq, 2 * (desc.n_s + desc.n_l) * desc.n_c, F);
        tr(off_WV, desc.n_l, F);
    }
}

// out[M][K] = G[M][N] W[N][K] through the transposed mirror (X W^T form)
static void gemm_gwt(const Model* m, int64_t off, int M, int N, int K, const float* G, int ldg, float* out, int ldo,
                     int epi, const float* pre, int ldp, bool accum, hipStream_t s) {
    gemm_xwt(M, K, N, G, ldg, m->pT(off), nullptr, out, ldo, epi, const_cast<float*>(pre), ldp, accum, s, m->bf16(),
             m->pxT(off), m->wx_stride());
}

// The first layer of a conservative model by neighbour species (its edge
// sums and two dense products in place of the per-edge message kernels),
// where the model has the tables and the edges are prepared.
static bool species_sum_on(const Model* m, const MpGeom& mg, const ModelBuf& b) {
    return m->sp && b.sp && mg.ecnt && message_mx_active(m->desc.width, m->desc.n_rbf, 0) && species_sum_active();
}

void embed_forward(const Model* m, const nnp_system& sys, const MpGeom& mg, ModelBuf& b, hipStream_t s) {
    const int n = int(sys.n_atoms);
    const int F = m->desc.width, K = m->desc.n_rbf, S = m->desc.n_species;
    const int cut = m->desc.kind == NNP_MODEL_CONS ? 0 : 1;
    for (int l = 0; l < m->n_layers(); ++l) {
        const LayerOff& lo = m->loff[l];
        LayerBuf& lb = b.layer[l];
        MpFwd a{};
        a.Wr = m->p(lo.Wr);
        a.br = m->p(lo.br);
        a.mx_scale = m->mx_scale(l);
        a.s_out = lb.smid;
        a.v_out = lb.vmid;
        if (l == 0) {
            a.species = sys.species;
            a.phi_tab = b.phi_tab;
            a.emb = m->p(m->off_emb);
        } else {
            gemm_xwt(n, F, F, b.s[l], F, m->p(lo.W1), m->p(lo.b1), lb.zphi, F, EPI_SILU, lb.h1, F, false, s,
                     m->bf16(), m->px(lo.W1), m->wx_stride());
            gemm_xwt(n, 3 * F, F, lb.zphi, F, m->p(lo.W2), m->p(lo.b2), lb.phi, 3 * F, EPI_NONE, nullptr, 0, false,
                     s, m->bf16(), m->px(lo.W2), m->wx_stride());
            a.s_in = b.s[l];
            a.v_in = b.v[l];
            a.phi = lb.phi;
            a.pv = lb.pv;
        }
        if (l == 0 && species_sum_on(m, mg, b)) {
            // s = [E | species indicator] T_0^T (T_0 holds the embedding in
            // the indicator slots), v = U T_2^T: one launch over the rows
            // [s; v] where they are adjacent (FP32-equivalent split-bfloat16
            // products, else float32 ones)
            const int ep = m->sp_ep;
            float* Ev = b.sp + int64_t(n) * ep;
            // (the edge sums E, U come with the edge preparation)
            const bool adj = lb.vmid == lb.smid + int64_t(n) * F;
            if (!(adj && n % 128 == 0 &&
                  gemm_x3_split(4 * n, F, ep, b.sp, ep, m->sp_Tx(0), m->sp_Tx(1), m->sp_xs(), n, lb.smid, F, s))) {
                if (adj && n % 32 == 0) {
                    gemm_xwt_f32_split(4 * n, F, ep, b.sp, ep, m->sp_T(0), m->sp_T(1), n, lb.smid, F, s);
                } else {
                    gemm_xwt(n, F, ep, b.sp, ep, m->sp_T(0), nullptr, lb.smid, F, EPI_NONE, nullptr, 0, false, s);
                    gemm_xwt(3 * n, F, ep, Ev, ep, m->sp_T(1), nullptr, lb.vmid, F, EPI_NONE, nullptr, 0, false, s);
                }
            }
        } else {
            launch_message_fwd(F, K, cut, mg, a, s);
        }
        gemm_xwt(3 * n, 2 * F, F, lb.vmid, F, m->p(lo.U), nullptr, lb.UV, 2 * F, EPI_NONE, nullptr, 0, false, s,
                 m->bf16(), m->px(lo.U), m->wx_stride());
        launch_build_x(n, F, lb.smid, lb.UV, lb.X, s);
        gemm_xwt(n, F, 2 * F, lb.X, 2 * F, m->p(lo.M1), m->p(lo.m1), lb.z, F, EPI_SILU, lb.a1, F, false, s,
                 m->bf16(), m->px(lo.M1), m->wx_stride());
        gemm_xwt(n, 3 * F, F, lb.z, F, m->p(lo.M2), m->p(lo.m2), lb.pqo, 3 * F, EPI_NONE, nullptr, 0, false, s,
                 m->bf16(), m->px(lo.M2), m->wx_stride());
        launch_update_combine(n, F, lb.smid, lb.vmid, lb.UV, lb.pqo, b.s[l + 1], b.v[l + 1], s);
    }
}

// Reverse of one embedding layer.  In: gs, gv = adjoints of the layer
// output.  Out: gs, gv = adjoints of the layer input (buffers swapped).
// With `dtheta`, the weight adjoints of the layer are written too.
// With gv_zero, the adjoint of the layer's vector output is zero (the last
// layer of an energy: the readout takes s alone) and b.gv is not read.
void layer_backward(const Model* m, int l, const MpGeom& mg, ModelBuf& b, float* force, bool accum_force,
                    float* dtheta, hipStream_t s, float* vir = nullptr, bool gv_zero = false) {
    const int n = mg.n;
    const int F = m->desc.width, K = m->desc.n_rbf;
    const int cut = m->desc.kind == NNP_MODEL_CONS ? 0 : 1;
    const LayerOff& lo = m->loff[l];
    LayerBuf& lb = b.layer[l];
    const bool wg = dtheta != nullptr;
    launch_update_combine_bwd(n, F, lb.UV, lb.pqo, b.gs, gv_zero ? nullptr : b.gv, b.gpqo, b.gUV, s);
    if (wg) {
        gemm_wgrad(n, 3 * F, F, b.gpqo, 3 * F, lb.z, F, dtheta + lo.M2, b.chunk_part, kChunk, false, s);
        colsum(n, 3 * F, b.gpqo, 3 * F, dtheta + lo.m2, b.chunk_part, kChunk, false, s);
    }
    gemm_gwt(m, lo.M2, n, 3 * F, F, b.gpqo, 3 * F, b.ga1, F, EPI_DSILU, lb.a1, F, false, s);
    if (wg) {
        gemm_wgrad(n, F, 2 * F, b.ga1, F, lb.X, 2 * F, dtheta + lo.M1, b.chunk_part, kChunk, false, s);
        colsum(n, F, b.ga1, F, dtheta + lo.m1, b.chunk_part, kChunk, false, s);
    }
    gemm_gwt(m, lo.M1, n, F, 2 * F, b.ga1, F, b.gX, 2 * F, EPI_NONE, nullptr, 0, false, s);
    launch_norm_bwd(n, F, b.gs, b.gX, lb.X, lb.UV, b.gs2, b.gUV, s);  // gs2 = g_smid
    if (wg) gemm_wgrad(3 * n, 2 * F, F, b.gUV, 2 * F, lb.vmid, F, dtheta + lo.U, b.chunk_part, kChunk, false, s);
    gemm_gwt(m, lo.U, 3 * n, 2 * F, F, b.gUV, 2 * F, b.gv, F, EPI_NONE, nullptr, 0, !gv_zero, s);  // gv = g_vmid
    MpBwd a{};
    a.gsm = b.gs2;
    a.gvm = b.gv;
    a.Wr = m->p(lo.Wr);
    a.br = m->p(lo.br);
    a.mx_scale = m->mx_scale(l);
    a.gphi = b.gphi;
    a.gv_in = b.gv2;
    a.force = force;
    a.accum_force = accum_force;
    a.vir = vir;
    a.wgrad_part = wg ? b.mp_part : nullptr;
    if (l == 0) {
        a.species = mg.species;
        a.phi_tab = b.phi_tab;
        a.want_gphi = wg;  // forces alone need no adjoint of the first layer's input
    } else {
        a.v_in = b.v[l];
        a.phi = lb.phi;
        a.pv = lb.pv;
        a.want_gphi = 1;
    }
    if (l == 0 && !wg && force && species_sum_on(m, mg, b)) {
        // P_0 = g_smid T_0, P_2 = g_vmid T_2 (float32 products), then the
        // per-edge force shares
        // (one launch over the rows [g_smid; g_vmid] where they are adjacent)
        const int pp = m->sp_pp;
        float* P2 = b.sp + int64_t(n) * pp;
        const bool adj = b.gv == b.gs2 + int64_t(n) * F;
        if (!(adj && n % 128 == 0 &&
              gemm_x3_split(4 * n, pp, F, b.gs2, F, m->sp_TTx(0), m->sp_TTx(1), m->sp_xs(), n, b.sp, pp, s))) {
            if (adj && n % 32 == 0) {
                gemm_xwt_f32_split(4 * n, pp, F, b.gs2, F, m->sp_TT(0), m->sp_TT(1), n, b.sp, pp, s);
            } else {
                gemm_xwt(n, pp, F, b.gs2, F, m->sp_TT(0), nullptr, b.sp, pp, EPI_NONE, nullptr, 0, false, s);
                gemm_xwt(3 * n, pp, F, b.gv, F, m->sp_TT(1), nullptr, P2, pp, EPI_NONE, nullptr, 0, false, s);
            }
        }
        launch_sp_bwd(mg, m->desc.n_species, b.sp, P2, force, accum_force, vir, s);
        return;
    }
    launch_message_bwd(F, K, cut, mg, a, force != nullptr, wg, s);
    if (wg) {
        const int nb = mp_blocks(n, F);
        const int64_t cnt = int64_t(3) * F * (K + 1);
        launch_reduce_chunks(cnt, nb, b.mp_part, cnt, b.filt_sum, false, s);
        launch_split_filter_grad(3 * F, K, b.filt_sum, dtheta + lo.Wr, dtheta + lo.br, s);
    }
    if (l == 0) {
        if (wg) {
            // phi was evaluated per species: reduce its adjoints per species and
            // differentiate the table; the embedding gets the pass-through
            // adjoint of s plus the perceptron path.
            const int S = m->desc.n_species;
            launch_emb_grad(n, 3 * F, S, mg.species, b.gphi, b.gphi_tab, s);
            gemm_wgrad(S, 3 * F, F, b.gphi_tab, 3 * F, b.z_tab, F, dtheta + lo.W2, b.chunk_part, kChunk, false, s);
            colsum(S, 3 * F, b.gphi_tab, 3 * F, dtheta + lo.b2, b.chunk_part, kChunk, false, s);
            gemm_gw(S, 3 * F, F, b.gphi_tab, 3 * F, m->p(lo.W2), b.gh1_tab, F, EPI_DSILU, b.h1_tab, F, false, s);
            gemm_wgrad(S, F, F, b.gh1_tab, F, m->p(m->off_emb), F, dtheta + lo.W1, b.chunk_part, kChunk, false, s);
            colsum(S, F, b.gh1_tab, F, dtheta + lo.b1, b.chunk_part, kChunk, false, s);
            launch_emb_grad(n, F, S, mg.species, b.gs2, dtheta + m->off_emb, s);
            gemm_gw(S, F, F, b.gh1_tab, F, m->p(lo.W1), dtheta + m->off_emb, F, EPI_NONE, nullptr, 0, true, s);
        }
        return;
    }
    if (wg) {
        gemm_wgrad(n, 3 * F, F, b.gphi, 3 * F, lb.zphi, F, dtheta + lo.W2, b.chunk_part, kChunk, false, s);
        colsum(n, 3 * F, b.gphi, 3 * F, dtheta + lo.b2, b.chunk_part, kChunk, false, s);
    }
    gemm_gwt(m, lo.W2, n, 3 * F, F, b.gphi, 3 * F, b.gh1, F, EPI_DSILU, lb.h1, F, false, s);
    if (wg) {
        gemm_wgrad(n, F, F, b.gh1, F, b.s[l], F, dtheta + lo.W1, b.chunk_part, kChunk, false, s);
        colsum(n, F, b.gh1, F, dtheta + lo.b1, b.chunk_part, kChunk, false, s);
    }
    gemm_gwt(m, lo.W1, n, F, F, b.gh1, F, b.gs2, F, EPI_NONE, nullptr, 0, true, s);  // g_s_in
    std::swap(b.gs, b.gs2);
    std::swap(b.gv, b.gv2);
}

MpGeom make_geom(const Model* m, const nnp_system& sys, const RepGeom& geom, const nnp_nlist& nl) {
    MpGeom mg{};
    mg.n = int(sys.n_atoms);
    mg.pos = sys.pos;
    mg.species = sys.species;
    mg.n_species = m->desc.n_species;
    mg.geom = geom;
    mg.off = nl.offsets;
    mg.nbr = nl.nbr;
    mg.rc = m->desc.cutoff;
    mg.rc2 = m->desc.cutoff * m->desc.cutoff;
    mg.bessel_norm = std::sqrt(2.0 / m->desc.cutoff);
    mg.pi_over_rc = M_PI / m->desc.cutoff;
    mg.inv_rc = 1.0 / m->desc.cutoff;
    return mg;
}

// With `vir`, also the per-atom shares of the virial -sum_i F_i . q_i.
// With `perm`, sys and nl are in a working row order and row i's outputs
// (forces, atomic energies, virial shares) go to the caller's index perm[i].
void cons_eval(const Model* m, const nnp_system& sys, const RepGeom& geom, const SysTables& t, const nnp_nlist& nl,
               ModelBuf& b, double* energy, float* forces, hipStream_t s, float* vir = nullptr,
               const int* perm = nullptr) {
    const int n = int(sys.n_atoms);
    const int F = m->desc.width;
    MpGeom mg = make_geom(m, sys, geom, nl);
    mg.perm = perm;
    if (b.ecnt && message_mx_active(F, m->desc.n_rbf, 0)) {
        // the edges within the cutoff, prepared once for all six message launches
        // (with the first layer by neighbour species, its edge sums in the same pass)
        if (m->sp && b.sp && species_sum_active())
            launch_edge_prep(mg, b.ecnt, b.erec, b.ehalf, s, b.sp, b.sp + int64_t(n) * m->sp_ep, m->desc.n_species,
                             m->sp_ep);
        else
            launch_edge_prep(mg, b.ecnt, b.erec, b.ehalf, s);
        mg.ecnt = b.ecnt;
        mg.erec = b.erec;
        mg.ehalf = b.ehalf;
    }
    embed_forward(m, sys, mg, b, s);
    const int L = m->n_layers();
    gemm_xwt(n, F, F, b.s[L], F, m->p(m->off_Wo), m->p(m->off_bo), b.zo, F, EPI_SILU, b.ao, F, false, s, m->bf16(),
             m->px(m->off_Wo), m->wx_stride());
    launch_readout(n, F, m->desc.n_species, b.zo, m->p(m->off_wo), m->p(m->off_beta), sys.species, b.Ei, s, perm);
    if (energy) launch_rep_sum(sys.n_rep, t.rep_start, b.Ei, energy, s);
    if (!forces) return;
    launch_readout_bwd(n, F, b.ao, m->p(m->off_wo), b.gs2, s);
    gemm_gwt(m, m->off_Wo, n, F, F, b.gs2, F, b.gs, F, EPI_NONE, nullptr, 0, false, s);
    for (int l = L - 1; l >= 0; --l) layer_backward(m, l, mg, b, forces, l != L - 1, nullptr, s, vir, l == L - 1);
}

// With vir_set / vir_add, also the per-atom shares of the NPT virial proxy
// sum_i sum_j F_ij . r_ij, written / added to.
// `perm` as in cons_eval.
void nc_eval(const Model* m, const nnp_system& sys, const RepGeom& geom, const nnp_nlist& nl, ModelBuf& b,
             float* forces, hipStream_t s, float* vir_set = nullptr, float* vir_add = nullptr,
             const int* perm = nullptr) {
    const int n = int(sys.n_atoms);
    const int F = m->desc.width;
    const int HC = 2 * (m->desc.n_s + m->desc.n_l) * m->desc.n_c;
    MpGeom mg = make_geom(m, sys, geom, nl);
    mg.perm = perm;
    if (F <= 32) {
        // inference: species-table perceptron, message, then one fused kernel
        // for the update block and the projections (no intermediates kept)
        const int K = m->desc.n_rbf, S = m->desc.n_species;
        const LayerOff& lo = m->loff[0];
        LayerBuf& lb = b.layer[0];
        MpFwd a{};
        a.Wr = m->p(lo.Wr);
        a.br = m->p(lo.br);
        a.s_out = lb.smid;
        a.v_out = lb.vmid;
        a.species = sys.species;
        a.phi_tab = b.phi_tab;
        a.emb = m->p(m->off_emb);
        // the pair head then reads the edges as records (no second pair rule)
        const bool records = b.nc_edges && nl.capacity <= b.nc_edge_cap && K == 8 && m->desc.n_s == 8;
        if (records) {
            a.edge_out = b.nc_edges;
            a.edge_cnt = b.nc_ecnt;
        }
        launch_message_fwd(F, K, 1, mg, a, s);
        NcUpdateArgs u{n, lb.smid, lb.vmid, m->ncw, m->p(lo.m1), m->p(lo.m2), b.QK, b.Vh};
        if (m->ncw && launch_nc_update_proj(u, F, m->bf16(), s)) {
            if (records) launch_head_fwd_rec(mg, b.nc_ecnt, b.nc_edges, b.QK, b.Vh, forces, false, s, vir_set, vir_add);
            else launch_head_fwd(mg, b.QK, b.Vh, forces, false, s, vir_set, vir_add);
            return;
        }
    }
    embed_forward(m, sys, mg, b, s);
    gemm_xwt(n, HC, F, b.s[1], F, m->p(m->off_Wq), nullptr, b.QK, HC, EPI_NONE, nullptr, 0, false, s, m->bf16(),
             m->px(m->off_Wq), m->wx_stride());
    gemm_xwt(3 * n, m->desc.n_l, F, b.v[1], F, m->p(m->off_WV), nullptr, b.Vh, m->desc.n_l, EPI_NONE, nullptr, 0,
             false, s, m->bf16(), m->px(m->off_WV), m->wx_stride());
    launch_head_fwd(mg, b.QK, b.Vh, forces, false, s, vir_set, vir_add);
}

void nc_wgrad(const Model* m, const nnp_system& sys, const RepGeom& geom, const nnp_nlist& nl, ModelBuf& b,
              const float* dl_df, float* dtheta, hipStream_t s) {
    const int n = int(sys.n_atoms);
    const int F = m->desc.width;
    const int nl_ = m->desc.n_l;
    const int HC = 2 * (m->desc.n_s + m->desc.n_l) * m->desc.n_c;
    MpGeom mg = make_geom(m, sys, geom, nl);
    embed_forward(m, sys, mg, b, s);
    gemm_xwt(n, HC, F, b.s[1], F, m->p(m->off_Wq), nullptr, b.QK, HC, EPI_NONE, nullptr, 0, false, s, m->bf16(),
             m->px(m->off_Wq), m->wx_stride());
    gemm_xwt(3 * n, nl_, F, b.v[1], F, m->p(m->off_WV), nullptr, b.Vh, nl_, EPI_NONE, nullptr, 0, false, s, m->bf16(),
             m->px(m->off_WV), m->wx_stride());
    launch_head_bwd(mg, b.QK, b.Vh, dl_df, b.gQK, b.gVh, s);
    gemm_wgrad(n, HC, F, b.gQK, HC, b.s[1], F, dtheta + m->off_Wq, b.chunk_part, kChunk, false, s);
    gemm_gwt(m, m->off_Wq, n, HC, F, b.gQK, HC, b.gs, F, EPI_NONE, nullptr, 0, false, s);
    gemm_wgrad(3 * n, nl_, F, b.gVh, nl_, b.v[1], F, dtheta + m->off_WV, b.chunk_part, kChunk, false, s);
    gemm_gwt(m, m->off_WV, 3 * n, nl_, F, b.gVh, nl_, b.gv, F, EPI_NONE, nullptr, 0, false, s);
    layer_backward(m, 0, mg, b, nullptr, false, dtheta, s);
}

}  // namespace nnp

// ============================================================== workspace
namespace nnp {

// atoms per block of the disagreement reduction
constexpr int kDisChunk = 2048;

struct CallScratch {
    SysTables t;
    NbrScratch nb;
    ModelBuf cons, nc;
    RespaBuf rs;       // snapshot for capacity failures
    RespaBuf frame;    // saved frame of the rewind procedure
    double* inner_energy = nullptr;
    double* disagree = nullptr;
    double* ke_part = nullptr;
    double* pos_rows = nullptr;  // [3][n] positions in the evaluations' row order
    int* species_rows = nullptr;  // [n] species in that order
    // the next outer step's conservative list, built beside the current
    // step's conservative evaluation, with its order and row-ordered copies
    int *spare_off = nullptr, *spare_nbr = nullptr, *spare_order = nullptr, *spare_species = nullptr;
    double* spare_pos = nullptr;
};

// One layout serves every entry point: tables, neighbour scratch, the
// integrator's snapshot and flags, then the two model scratch areas.
void carve_all(Arena& a, const Model* cons, const Model* nc, int64_t n, int32_t n_rep, int64_t E, bool wgrad,
               CallScratch& c) {
    carve_tables(a, n_rep, c.t);
    carve_nbr_scratch(a, n, n_rep, c.nb);
    c.rs.pos = a.take<double>(3 * n);
    c.rs.vel = a.take<double>(3 * n);
    c.rs.pos_ref = a.take<double>(3 * n);
    c.rs.f_cons = a.take<float>(3 * n);
    c.rs.f_nc = a.take<float>(3 * n);
    c.rs.energy = a.take<double>(n_rep);
    c.frame.pos = a.take<double>(3 * n);
    c.frame.vel = a.take<double>(3 * n);
    c.frame.pos_ref = a.take<double>(3 * n);
    c.frame.f_cons = a.take<float>(3 * n);
    c.frame.f_nc = a.take<float>(3 * n);
    c.frame.energy = a.take<double>(n_rep);
    c.inner_energy = a.take<double>(n_rep);
    c.disagree = a.take<double>(int64_t(n_rep) * (cdiv(n, kDisChunk) + 1));
    c.ke_part = a.take<double>(int64_t(n_rep) * cdiv(n, kKeChunk));
    c.pos_rows = a.take<double>(3 * n);
    c.species_rows = a.take<int>(n);
    c.spare_off = a.take<int>(n + 1);
    c.spare_nbr = a.take<int>(E);
    c.spare_order = a.take<int>(2 * n);
    c.spare_pos = a.take<double>(3 * n);
    c.spare_species = a.take<int>(n);
    if (cons) carve_model(a, cons, n, E, false, c.cons);
    if (nc) carve_model(a, nc, n, E, wgrad, c.nc);
}

size_t call_scratch_bytes(const Model* cons, const Model* nc, int64_t n, int32_t n_rep, int64_t E) {
    Arena a(nullptr, 0);
    CallScratch c;
    carve_all(a, cons, nc, n, n_rep, std::max<int64_t>(E, 1), false, c);
    return a.used + 256;
}

}  // namespace nnp

extern "C" nnp_status nnp_workspace_size(const nnp_model* cons, const nnp_model* nc, int64_t n_atoms, int32_t n_rep,
                                         int64_t max_edges, size_t* bytes) {
    NNP_API_BEGIN
    NNP_REQUIRE(bytes && n_atoms >= 1 && n_rep >= 1 && max_edges >= 0, NNP_EINVAL, "bad workspace query");
    Arena a(nullptr, 0);
    CallScratch c;
    carve_all(a, reinterpret_cast<const Model*>(cons), reinterpret_cast<const Model*>(nc), n_atoms, n_rep,
              std::max<int64_t>(max_edges, 1), true, c);
    *bytes = a.used + 256;
    NNP_API_END
}

// ============================================================== neighbours
extern "C" nnp_status nnp_neighbors(const nnp_system* sys, nnp_nlist* nl, void* ws, size_t ws_bytes, void* stream) {
    NNP_API_BEGIN
    check_system(sys);
    NNP_REQUIRE(nl && nl->offsets && (nl->nbr || nl->capacity == 0), NNP_EINVAL, "incomplete neighbour list");
    NNP_REQUIRE(nl->n_atoms == sys->n_atoms, NNP_EINVAL, "list rows must equal n_atoms");
    NNP_REQUIRE(nl->cutoff > 0, NNP_EINVAL, "cutoff must be positive");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Arena a(ws, ws_bytes);
    SysTables t;
    carve_tables(a, sys->n_rep, t);
    NbrScratch nb;
    carve_nbr_scratch(a, sys->n_atoms, sys->n_rep, nb);
    std::vector<double> hs;
    RepGeom g = upload_tables(*sys, t, s, hs);
    CellPlan plan = plan_cells(*sys, nl->cutoff);
    upload_cell_plan(plan, nb, s);
    NNP_HIP(hipMemsetAsync(nb.status, 0, sizeof(int) * 8, s));
    launch_set_flag(t.flags, 1, s);
    launch_build(int(sys->n_atoms), sys->pos, g, plan, nb, t.flags, nl->cutoff, nl->capacity, nl->offsets,
                 nl->nbr, nl->rev, nullptr, s);
    int host_status[8];
    int total = 0;
    NNP_HIP(hipMemcpyAsync(host_status, nb.status, sizeof(host_status), hipMemcpyDeviceToHost, s));
    NNP_HIP(hipMemcpyAsync(&total, nb.tmp_off + sys->n_atoms, sizeof(int), hipMemcpyDeviceToHost, s));
    NNP_HIP(hipStreamSynchronize(s));
    nl->n_edges = total;
    NNP_REQUIRE(host_status[2] == 0, NNP_EROWLIMIT, "a neighbour row exceeds the 1024-entry limit of the builder");
    NNP_REQUIRE(host_status[0] == 0, NNP_ECAPACITY,
                "neighbour list needs " + std::to_string(total) + " entries, capacity " +
                    std::to_string(nl->capacity));
    NNP_API_END
}

// ================================================================== forces
namespace nnp {

static void check_list(const nnp_nlist* nl, const nnp_system* sys, double min_cutoff) {
    NNP_REQUIRE(nl && nl->offsets && nl->nbr, NNP_EINVAL, "incomplete neighbour list");
    NNP_REQUIRE(nl->n_atoms == sys->n_atoms, NNP_EINVAL, "list rows must equal n_atoms");
    NNP_REQUIRE(nl->cutoff >= min_cutoff, NNP_EINVAL, "list radius is below the model cutoff");
}

}  // namespace nnp

extern "C" nnp_status nnp_cons_energy_forces(const nnp_model* cons, const nnp_system* sys, const nnp_nlist* nl,
                                             void* ws, size_t ws_bytes, double* energy, float* forces,
                                             void* stream) {
    NNP_API_BEGIN
    NNP_REQUIRE(cons, NNP_EINVAL, "null model");
    const Model* m = reinterpret_cast<const Model*>(cons);
    NNP_REQUIRE(m->desc.kind == NNP_MODEL_CONS, NNP_EINVAL, "not a conservative model");
    check_system(sys);
    check_list(nl, sys, m->desc.cutoff);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Arena a(ws, ws_bytes);
    CallScratch c;
    carve_all(a, m, nullptr, sys->n_atoms, sys->n_rep, std::max<int64_t>(nl->capacity, 1), false, c);
    std::vector<double> hs;
    RepGeom g = upload_tables(*sys, c.t, s, hs);
    cons_eval(m, *sys, g, c.t, *nl, c.cons, energy, forces, s);
    NNP_API_END
}

extern "C" nnp_status nnp_cons_virial(const nnp_model* cons, const nnp_system* sys, const nnp_nlist* nl, void* ws,
                                      size_t ws_bytes, double* energy, float* forces, double* virial,
                                      void* stream) {
    NNP_API_BEGIN
    NNP_REQUIRE(cons && forces && virial, NNP_EINVAL, "null argument");
    const Model* m = reinterpret_cast<const Model*>(cons);
    NNP_REQUIRE(m->desc.kind == NNP_MODEL_CONS, NNP_EINVAL, "not a conservative model");
    check_system(sys);
    check_list(nl, sys, m->desc.cutoff);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Arena a(ws, ws_bytes);
    CallScratch c;
    carve_all(a, m, nullptr, sys->n_atoms, sys->n_rep, std::max<int64_t>(nl->capacity, 1), false, c);
    std::vector<double> hs;
    RepGeom g = upload_tables(*sys, c.t, s, hs);
    cons_eval(m, *sys, g, c.t, *nl, c.cons, energy, forces, s, c.cons.vir);
    launch_rep_sum(sys->n_rep, c.t.rep_start, c.cons.vir, virial, s);
    NNP_API_END
}

extern "C" nnp_status nnp_nc_virial(const nnp_model* nc, const nnp_system* sys, const nnp_nlist* nl, void* ws,
                                    size_t ws_bytes, float* forces, double* virial, void* stream) {
    NNP_API_BEGIN
    NNP_REQUIRE(nc && forces && virial, NNP_EINVAL, "null argument");
    const Model* m = reinterpret_cast<const Model*>(nc);
    NNP_REQUIRE(m->desc.kind == NNP_MODEL_NC, NNP_EINVAL, "not an NC model");
    check_system(sys);
    check_list(nl, sys, m->desc.cutoff);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Arena a(ws, ws_bytes);
    CallScratch c;
    carve_all(a, nullptr, m, sys->n_atoms, sys->n_rep, std::max<int64_t>(nl->capacity, 1), false, c);
    std::vector<double> hs;
    RepGeom g = upload_tables(*sys, c.t, s, hs);
    nc_eval(m, *sys, g, *nl, c.nc, forces, s, c.nc.vir, nullptr);
    launch_rep_sum(sys->n_rep, c.t.rep_start, c.nc.vir, virial, s);
    NNP_API_END
}

extern "C" nnp_status nnp_nc_forces(const nnp_model* nc, const nnp_system* sys, const nnp_nlist* nl, void* ws,
                                    size_t ws_bytes, float* forces, void* stream) {
    NNP_API_BEGIN
    NNP_REQUIRE(nc && forces, NNP_EINVAL, "null argument");
    const Model* m = reinterpret_cast<const Model*>(nc);
    NNP_REQUIRE(m->desc.kind == NNP_MODEL_NC, NNP_EINVAL, "not an NC model");
    check_system(sys);
    check_list(nl, sys, m->desc.cutoff);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Arena a(ws, ws_bytes);
    CallScratch c;
    carve_all(a, nullptr, m, sys->n_atoms, sys->n_rep, std::max<int64_t>(nl->capacity, 1), false, c);
    std::vector<double> hs;
    RepGeom g = upload_tables(*sys, c.t, s, hs);
    nc_eval(m, *sys, g, *nl, c.nc, forces, s);
    NNP_API_END
}

// ======================================================= no-allocation NC
// A variant of nnp_nc_forces for callers that cannot allocate device memory
// (code under stream capture, serving loops that forbid hipMalloc): its
// scratch is a file-scope device array instead of a caller workspace.  The
// array's name is a host-side stand-in in host code; the device address of
// each GPU's copy is looked up once per device with hipGetSymbolAddress and
// only that address is passed to kernels.
namespace nnp {

constexpr size_t kNcScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNcScratchBytes];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_addr;  // per device ordinal

static void* scratch_address() {
    int dev = 0;
    NNP_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (size_t(dev) >= g_scratch_addr.size()) g_scratch_addr.resize(size_t(dev) + 1, nullptr);
    if (!g_scratch_addr[dev]) {
        void* ptr = nullptr;
        NNP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        NNP_REQUIRE(ptr != nullptr, NNP_EDEVICE, "no device address for the static scratch array");
        g_scratch_addr[dev] = ptr;
    }
    return g_scratch_addr[dev];
}

// The part of the workspace layout that the NC force evaluation touches.
static void carve_nc_only(Arena& a, const Model* m, int64_t n, int32_t n_rep, SysTables& t, ModelBuf& b) {
    carve_tables(a, n_rep, t);
    carve_model(a, m, n, 1, false, b);
}

}  // namespace nnp

extern "C" size_t nnp_nc_forces_noalloc_max_bytes(void) { return nnp::kNcScratchBytes; }

extern "C" nnp_status nnp_nc_forces_noalloc(const nnp_model* nc, const nnp_system* sys, const nnp_nlist* nl,
                                            float* forces, void* stream) {
    NNP_API_BEGIN
    NNP_REQUIRE(nc && forces, NNP_EINVAL, "null argument");
    const Model* m = reinterpret_cast<const Model*>(nc);
    NNP_REQUIRE(m->desc.kind == NNP_MODEL_NC, NNP_EINVAL, "not an NC model");
    check_system(sys);
    check_list(nl, sys, m->desc.cutoff);
    {
        Arena probe(nullptr, 0);
        SysTables t;
        ModelBuf b;
        carve_nc_only(probe, m, sys->n_atoms, sys->n_rep, t, b);
        NNP_REQUIRE(probe.used <= kNcScratchBytes, NNP_EINVAL,
                    "nnp_nc_forces_noalloc: the system needs " + std::to_string(probe.used) +
                        " bytes of scratch, above the static maximum of " + std::to_string(kNcScratchBytes));
    }
    void* ptr = scratch_address();
    hipStream_t s = static_cast<hipStream_t>(stream);
    Arena a(ptr, kNcScratchBytes);
    SysTables t;
    ModelBuf b;
    carve_nc_only(a, m, sys->n_atoms, sys->n_rep, t, b);
    static thread_local std::vector<double> hs;  // reused: no host allocation once grown
    RepGeom g = upload_tables(*sys, t, s, hs);
    nc_eval(m, *sys, g, *nl, b, forces, s);
    NNP_API_END
}

extern "C" nnp_status nnp_nc_weight_grad(const nnp_model* nc, const nnp_system* sys, const nnp_nlist* nl,
                                         const float* dl_df, float* dl_dtheta, void* ws, size_t ws_bytes,
                                         void* stream) {
    NNP_API_BEGIN
    NNP_REQUIRE(nc && dl_df && dl_dtheta, NNP_EINVAL, "null argument");
    const Model* m = reinterpret_cast<const Model*>(nc);
    NNP_REQUIRE(m->desc.kind == NNP_MODEL_NC, NNP_EINVAL, "not an NC model");
    check_system(sys);
    check_list(nl, sys, m->desc.cutoff);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Arena a(ws, ws_bytes);
    CallScratch c;
    carve_all(a, nullptr, m, sys->n_atoms, sys->n_rep, std::max<int64_t>(nl->capacity, 1), true, c);
    std::vector<double> hs;
    RepGeom g = upload_tables(*sys, c.t, s, hs);
    nc_wgrad(m, *sys, g, *nl, c.nc, dl_df, dl_dtheta, s);
    NNP_API_END
}

// ==================================================================== Adam
namespace nnp {
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / bc1;
    const float vh = vi / bc2;
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}
}  // namespace nnp

extern "C" nnp_status nnp_adam_step(float* param, const float* grad, float* m, float* v, int64_t n, int64_t t,
                                    double lr, double beta1, double beta2, double eps, void* stream) {
    NNP_API_BEGIN
    NNP_REQUIRE(param && grad && m && v && n >= 0 && t >= 1, NNP_EINVAL, "bad Adam arguments");
    const float bc1 = float(1.0 - std::pow(beta1, double(t)));
    const float bc2 = float(1.0 - std::pow(beta2, double(t)));
    k_adam<<<cdiv(n, 256), 256, 0, static_cast<hipStream_t>(stream)>>>(param, grad, m, v, n, float(lr), float(beta1),
                                                                        float(beta2), float(eps), bc1, bc2);
    NNP_LAUNCH_CHECK();
    NNP_API_END
}

// =============================================================== force MSE
namespace nnp {
// loss partials per block (fixed order) and dL/dF = 2 (F - F_ref) / count
__global__ void __launch_bounds__(256) k_force_mse(int64_t count, const float* __restrict__ f,
                                                   const float* __restrict__ ref, float* __restrict__ grad,
                                                   double* __restrict__ part) {
    __shared__ double red[256];
    double acc = 0.0;
    const double scale = 2.0 / double(count);
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += int64_t(gridDim.x) * 256) {
        const float d = f[i] - ref[i];
        acc += double(d) * double(d);
        if (grad) grad[i] = float(scale * double(d));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ void k_sum_parts(int nparts, const double* __restrict__ part, int64_t count, double* __restrict__ loss) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < nparts; ++k) s += part[k];
        *loss = s / double(count);
    }
}
}  // namespace nnp

extern "C" nnp_status nnp_force_mse(const float* f, const float* f_ref, int64_t count, double* loss, float* grad,
                                    void* ws, size_t ws_bytes, void* stream) {
    NNP_API_BEGIN
    NNP_REQUIRE(f && f_ref && loss && count > 0, NNP_EINVAL, "bad force-MSE arguments");
    constexpr int kParts = 1024;
    NNP_REQUIRE(ws && ws_bytes >= kParts * sizeof(double), NNP_EINVAL, "workspace below 8 KiB");
    const int blocks = int(std::min<int64_t>(kParts, (count + 255) / 256));
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* part = static_cast<double*>(ws);
    k_force_mse<<<blocks, 256, 0, s>>>(count, f, f_ref, grad, part);
    k_sum_parts<<<1, 64, 0, s>>>(blocks, part, count, loss);
    NNP_LAUNCH_CHECK();
    NNP_API_END
}

// ===================================================================== HMR
extern "C" nnp_status nnp_hmr_masses(int64_t n, const int32_t* bonded_heavy, const double* mass, double h_mass,
                                     int32_t mode, double* out_mass) {
    NNP_API_BEGIN
    NNP_REQUIRE(n >= 0 && bonded_heavy && mass && out_mass, NNP_EINVAL, "null argument");
    NNP_REQUIRE(mode == 0 || mode == 1, NNP_EINVAL, "mode must be 0 (set) or 1 (add)");
    std::vector<double> m(mass, mass + n);
    for (int64_t a = 0; a < n; ++a) {
        const int32_t h = bonded_heavy[a];
        if (h < 0) continue;
        NNP_REQUIRE(h < n && bonded_heavy[h] < 0, NNP_EINVAL, "bonded_heavy must point to a heavy atom");
        const double nm = mode == 0 ? h_mass : mass[a] + h_mass;
        m[h] -= nm - mass[a];
        m[a] = nm;
    }
    for (int64_t a = 0; a < n; ++a) NNP_REQUIRE(m[a] > 0, NNP_EINVAL, "repartitioning leaves a non-positive mass");
    std::memcpy(out_mass, m.data(), sizeof(double) * n);
    NNP_API_END
}

// ============================================================== integrator
namespace nnp {

struct PinnedFlags {
    int* host = nullptr;
    PinnedFlags() {
        if (hipHostMalloc(reinterpret_cast<void**>(&host), 64 * sizeof(int), hipHostMallocDefault) != hipSuccess)
            host = nullptr;
    }
};

static int* pinned_flags() {
    static thread_local PinnedFlags pf;
    NNP_REQUIRE(pf.host != nullptr, NNP_EDEVICE, "could not allocate pinned host memory");
    return pf.host;
}

void check_respa(const respa_state* st, const respa_params* p, const Model* cons, const Model* nc) {
    NNP_REQUIRE(st && p && cons, NNP_EINVAL, "null argument");
    NNP_REQUIRE(cons->desc.kind == NNP_MODEL_CONS, NNP_EINVAL, "first model must be conservative");
    NNP_REQUIRE(p->mode == NNP_MODE_DMTS_NC || p->mode == NNP_MODE_STS || p->mode == NNP_MODE_DMTS, NNP_EINVAL,
                "unknown mode");
    if (p->mode != NNP_MODE_STS) {
        const int want = p->mode == NNP_MODE_DMTS_NC ? NNP_MODEL_NC : NNP_MODEL_CONS;
        NNP_REQUIRE(nc && nc->desc.kind == want, NNP_EINVAL,
                    p->mode == NNP_MODE_DMTS_NC ? "DMTS-NC needs an NC model as the fast force"
                                                : "DMTS needs a conservative model as the fast force");
        NNP_REQUIRE(p->n_inner >= 1, NNP_EINVAL, "n_inner must be >= 1");
        NNP_REQUIRE(st->f_nc && st->nl_nc.offsets && st->nl_nc.nbr, NNP_EINVAL,
                    "multi-time-stepping needs f_nc and the fast-force list");
        NNP_REQUIRE(nc->desc.cutoff <= cons->desc.cutoff, NNP_EINVAL,
                    "the fast-force cutoff must not exceed the conservative one");
    }
    NNP_REQUIRE(p->dt_outer_fs > 0 && p->temperature_K >= 0 && p->skin >= 0, NNP_EINVAL, "bad integrator parameters");
    NNP_REQUIRE(p->rewind_threshold >= 0 && (p->rewind_threshold == 0 || (p->save_every >= 1 && p->sts_after_rewind >= 0)),
                NNP_EINVAL, "bad rewind parameters");
    NNP_REQUIRE(st->pos && st->vel && st->mass && st->gamma && st->f_cons && st->energy && st->pos_ref, NNP_EINVAL,
                "incomplete state");
    NNP_REQUIRE(st->sys.pos == st->pos, NNP_EINVAL, "state.sys.pos must alias state.pos");
    NNP_REQUIRE(st->nl_cons.offsets && st->nl_cons.nbr, NNP_EINVAL, "the conservative list needs offsets and nbr");
    NNP_REQUIRE(st->nl_cons.n_atoms == st->sys.n_atoms, NNP_EINVAL, "list rows must equal n_atoms");
}

// Per-replica disagreement sqrt(mean_i |F_i - F_fast,i|^2) in two fixed-order
// float64 reductions: block (c, r) sums chunk c (kDisChunk atoms) of replica
// r into part[r * chunks + c], then one wavefront per replica adds its
// chunks in order.  Non-finite positions or velocities count as infinite
// disagreement (such atoms leave every neighbour list, so their forces alone
// would not show the failure).  A replica above `thr` (or not finite) sets
// *trip, which the host reads at its next status check.
__global__ void __launch_bounds__(256) k_disagreement_part(const int64_t* __restrict__ rep_start, int n, int chunks,
                                                           const float* __restrict__ fa, const float* __restrict__ fb,
                                                           const double* __restrict__ pos,
                                                           const double* __restrict__ vel, double* __restrict__ part) {
    __shared__ double red[256];
    const int r = blockIdx.y, ch = blockIdx.x;
    const int64_t a0 = rep_start[r] + int64_t(ch) * kDisChunk;
    const int64_t a1 = min(rep_start[r + 1], a0 + kDisChunk);
    double acc = 0.0;
    for (int64_t i = a0 + threadIdx.x; i < a1; i += 256)
        for (int c = 0; c < 3; ++c) {
            const double d = double(fa[c * int64_t(n) + i]) - double(fb[c * int64_t(n) + i]);
            acc += d * d;
            if (!isfinite(pos[c * int64_t(n) + i]) || !isfinite(vel[c * int64_t(n) + i])) acc = INFINITY;
        }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[int64_t(r) * chunks + ch] = red[0];
}

__global__ void k_disagreement_final(const int64_t* __restrict__ rep_start, int chunks, const double* __restrict__ part,
                                     double* __restrict__ out, double thr, int* __restrict__ trip) {
    const int r = blockIdx.x;
    if (threadIdx.x != 0) return;
    const int64_t na = rep_start[r + 1] - rep_start[r];
    const int nc = int((na + kDisChunk - 1) / kDisChunk);
    double acc = 0.0;
    for (int c = 0; c < nc; ++c) acc += part[int64_t(r) * chunks + c];
    const double dis = sqrt(acc / double(max<int64_t>(na, 1)));
    out[r] = dis;
    if (!(dis <= thr)) *trip = 1;
}

// Advances a packed system by n_outer outer steps.  Replica r draws its
// normals with key (seeds[r], streams[r]) and O-step index step_base[r] + k,
// k counting the O-steps of this call.  rep_bad (host, n_rep, optional)
// receives per-replica non-finite flags at each check; without it any
// non-finite replica fails the call.
// internal: a list went stale between predicted rebuilds; the fast force
// disagreed (rewind); neither is returned
constexpr nnp_status NNP_ESTALE_INTERNAL = static_cast<nnp_status>(-100);
constexpr nnp_status NNP_EREWIND_INTERNAL = static_cast<nnp_status>(-101);

// A second stream of the calling host thread on the current device, with a
// fork and a join event (created on first use, kept until the process ends;
// default priority).  The conservative evaluation at the end of an outer
// step runs there beside the last inner evaluation.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

static const SideStream* side_stream() {
    thread_local std::map<int, SideStream> per_device;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    auto it = per_device.find(dev);
    if (it == per_device.end()) {
        SideStream x;
        const bool ok = hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking) == hipSuccess &&
                        hipEventCreateWithFlags(&x.fork, hipEventDisableTiming) == hipSuccess &&
                        hipEventCreateWithFlags(&x.join, hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            return nullptr;
        }
        it = per_device.emplace(dev, x).first;
    }
    return &it->second;
}

nnp_status respa_run(const Model* cons, const Model* nc, respa_state* st, const respa_params* p, int32_t n_outer,
                     void* ws, size_t ws_bytes, hipStream_t s, const uint64_t* seeds, const uint64_t* streams,
                     const uint64_t* step_base, int* rep_bad, uint64_t* stamps) {
    check_respa(st, p, cons, nc);
    check_system(&st->sys);
    NNP_REQUIRE(n_outer >= 0, NNP_EINVAL, "n_outer must be >= 0");
    const bool mts = p->mode != NNP_MODE_STS;
    const bool inner_nc = mts && nc->desc.kind == NNP_MODEL_NC;
    const bool rewind = mts && p->rewind_threshold > 0;
    const int n = int(st->sys.n_atoms);
    const int R = st->sys.n_rep;
    Arena a(ws, ws_bytes);
    CallScratch c;
    const int64_t E = std::max<int64_t>({st->nl_cons.capacity, mts ? st->nl_nc.capacity : 0, int64_t(1)});
    carve_all(a, cons, mts ? nc : nullptr, n, R, E, false, c);
    RespaBuf& frame = c.frame;
    int ke_chunks = 1;
    for (int r = 0; r < R; ++r)
        ke_chunks = std::max<int>(ke_chunks, cdiv(st->sys.rep_start[r + 1] - st->sys.rep_start[r], kKeChunk));
    double* disagree = c.disagree;  // [R] results, then [R][dis_chunks] partial sums
    int dis_chunks = 1;
    for (int r = 0; r < R; ++r)
        dis_chunks = std::max<int>(dis_chunks, cdiv(st->sys.rep_start[r + 1] - st->sys.rep_start[r], kDisChunk));
    double* inner_energy = c.inner_energy;
    std::vector<double> hs;
    RepGeom g = upload_tables(st->sys, c.t, s, hs);
    NNP_HIP(hipMemcpyAsync(c.t.seed, seeds, sizeof(uint64_t) * R, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(c.t.stream, streams, sizeof(uint64_t) * R, hipMemcpyHostToDevice, s));
    NNP_HIP(hipMemcpyAsync(c.t.step_base, step_base, sizeof(uint64_t) * R, hipMemcpyHostToDevice, s));
    launch_set_u64(c.t.o_step, 0, s);  // O-steps since the start of the call, advanced by the kicks
    const double rc_cons = cons->desc.cutoff + p->skin;
    const double rc_nc = mts ? nc->desc.cutoff + p->skin : 0.0;
    CellPlan plan = plan_cells(st->sys, rc_cons);
    upload_cell_plan(plan, c.nb, s);
    // flags: [0] rebuild trigger, [4] stale-list flag of the predictive mode, [5..6]
    // displacement record, [8..10] fast-force list status, [12] rewind trip;
    // nb.status: conservative list
    int* trip = c.t.flags + 12;
    int* trig = c.t.flags;
    int* stale = c.t.flags + 4;
    unsigned* maxd2 = reinterpret_cast<unsigned*>(c.t.flags + 5);
    int* nc_status = c.t.flags + 8;
    NNP_HIP(hipMemsetAsync(c.t.flags, 0, sizeof(int) * 16, s));
    NNP_HIP(hipMemsetAsync(c.t.rep_bad, 0, sizeof(int) * R, s));
    NNP_HIP(hipMemsetAsync(c.nb.status, 0, sizeof(int) * 8, s));
    NNP_HIP(hipMemsetAsync(c.t.rebuilds, 0, sizeof(long long), s));
    NNP_HIP(hipMemsetAsync(c.spare_off, 0, sizeof(int) * (size_t(n) + 1), s));  // empty rows until a spare build

    nnp_nlist lc = st->nl_cons, ln = st->nl_nc;
    const double disp_thr = 0.5 * p->skin;
    // With state->order the force evaluations keep their rows in the cell
    // order of the last build (row_of: caller index -> row; perm: back) and
    // read positions and species from row-ordered copies, which the builds
    // and every B A O A update keep current.
    const bool rows = st->order != nullptr;
    const int* perm = rows ? st->order : nullptr;
    const int* row_of = rows ? st->order + n : nullptr;
    nnp_system sys_ev = st->sys;
    if (rows) {
        sys_ev.pos = c.pos_rows;
        sys_ev.species = c.species_rows;
    }
    auto rebuild_if_flagged = [&]() {
        launch_build(n, st->pos, g, plan, c.nb, trig, rc_cons, lc.capacity, lc.offsets, lc.nbr, lc.rev, st->pos_ref,
                     s, rows);
        if (mts)
            launch_filter(n, rows ? c.nb.cell_pos : st->pos, g, c.nb, trig, lc.offsets, lc.nbr, rc_nc, ln.capacity,
                          ln.offsets, ln.nbr, nullptr, nc_status, s, rows ? c.nb.cell_atoms : nullptr, c.nb.status);
        if (rows) launch_commit_order(n, c.nb, trig, st->sys.species, st->order, c.pos_rows, c.species_rows, s);
        launch_finish_rebuild(trig, c.t.rebuilds, maxd2, s);
    };
    // Predictive outer steps decide on the next step's rebuild right after
    // their last B A O A (the positions the next step starts from) and build
    // the conservative list into spare buffers beside the conservative
    // evaluation that still reads the one in use; the fast-force list, read
    // only by the inner evaluations before it, is filtered in place.  The
    // spare list is adopted once that evaluation is done.  Needs the side
    // stream and no reverse index.
    const bool overlap_build = mts && lc.rev == nullptr && lc.capacity <= E;
    auto build_spare_if_predicted = [&]() {
        launch_predict_rebuild(maxd2, disp_thr, trig, s);
        launch_build(n, st->pos, g, plan, c.nb, trig, rc_cons, lc.capacity, c.spare_off, c.spare_nbr, nullptr,
                     st->pos_ref, s, rows);
        launch_filter(n, rows ? c.nb.cell_pos : st->pos, g, c.nb, trig, c.spare_off, c.spare_nbr, rc_nc,
                      ln.capacity, ln.offsets, ln.nbr, nullptr, nc_status, s, rows ? c.nb.cell_atoms : nullptr,
                      c.nb.status);
        if (rows)
            launch_commit_order(n, c.nb, trig, st->sys.species, c.spare_order, c.spare_pos, c.spare_species, s);
    };
    auto adopt_spare = [&]() {
        launch_adopt_lists(n, trig, c.nb, c.spare_off, c.spare_nbr, lc.capacity, lc.offsets, lc.nbr,
                           rows ? c.spare_order : nullptr, st->order, c.spare_pos, c.pos_rows, c.spare_species,
                           c.species_rows, s);
        launch_finish_rebuild(trig, c.t.rebuilds, maxd2, s);
    };
    BaoaArgs ba{};
    ba.n = n;
    ba.pos = st->pos;
    ba.vel = st->vel;
    ba.mass = st->mass;
    ba.gamma = st->gamma;
    ba.temperature = p->temperature_K;
    ba.rep_of_atom = g.rep_of_atom;
    ba.rep_start = c.t.rep_start;
    ba.seed = c.t.seed;
    ba.stream = c.t.stream;
    ba.step_base = c.t.step_base;
    ba.ffl = p->thermostat == NNP_THERMO_FFL;
    ba.pos_ref = st->pos_ref;
    ba.disp_thr2 = disp_thr * disp_thr;
    ba.flag = trig;
    ba.maxd2 = maxd2;
    ba.step_offset = 0;
    ba.step_dev = c.t.o_step;
    ba.pos_rows = rows ? c.pos_rows : nullptr;
    ba.row = row_of;

    // NPT virial estimator (state->virial): per-atom shares of W_cons in
    // c.cons.vir, of the fast force's W_S in c.nc.vir (last evaluation) and
    // c.nc.vir_sum (summed over the inner loop of the current outer step)
    const bool want_vir = st->virial != nullptr;
    auto eval_cons = [&]() {
        cons_eval(cons, sys_ev, g, c.t, lc, c.cons, st->energy, st->f_cons, s, want_vir ? c.cons.vir : nullptr,
                  perm);
    };
    auto eval_inner = [&]() {
        if (inner_nc) {
            nc_eval(nc, sys_ev, g, ln, c.nc, st->f_nc, s, want_vir ? c.nc.vir : nullptr,
                    want_vir ? c.nc.vir_sum : nullptr, perm);
        } else {
            cons_eval(nc, sys_ev, g, c.t, ln, c.nc, inner_energy, st->f_nc, s, want_vir ? c.nc.vir : nullptr, perm);
            if (want_vir) launch_add(n, c.nc.vir, c.nc.vir_sum, s);
        }
    };

    int* hflags = pinned_flags();
    std::vector<int> bad(R);
    auto read_status = [&]() {
        NNP_HIP(hipMemcpyAsync(hflags, c.t.flags, sizeof(int) * 16, hipMemcpyDeviceToHost, s));
        NNP_HIP(hipMemcpyAsync(hflags + 16, c.nb.status, sizeof(int) * 8, hipMemcpyDeviceToHost, s));
        NNP_HIP(hipMemcpyAsync(hflags + 32, c.t.rebuilds, sizeof(long long), hipMemcpyDeviceToHost, s));
        NNP_HIP(hipMemcpyAsync(bad.data(), c.t.rep_bad, sizeof(int) * R, hipMemcpyDeviceToHost, s));
        NNP_HIP(hipStreamSynchronize(s));
    };
    auto copy_state = [&](RespaBuf& dst_buf, bool save) {
        const size_t d3 = sizeof(double) * 3 * size_t(n), f3 = sizeof(float) * 3 * size_t(n);
        auto cp = [&](void* dst, const void* src, size_t bytes) {
            NNP_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
        };
        if (save) {
            cp(dst_buf.pos, st->pos, d3); cp(dst_buf.vel, st->vel, d3); cp(dst_buf.pos_ref, st->pos_ref, d3);
            cp(dst_buf.f_cons, st->f_cons, f3); if (mts) cp(dst_buf.f_nc, st->f_nc, f3);
            cp(dst_buf.energy, st->energy, sizeof(double) * R);
        } else {
            cp(st->pos, dst_buf.pos, d3); cp(st->vel, dst_buf.vel, d3); cp(st->pos_ref, dst_buf.pos_ref, d3);
            cp(st->f_cons, dst_buf.f_cons, f3); if (mts) cp(st->f_nc, dst_buf.f_nc, f3);
            cp(st->energy, dst_buf.energy, sizeof(double) * R);
            if (rows) launch_gather_rows(n, perm, st->pos, nullptr, c.pos_rows, nullptr, s);
        }
    };
    long long rebuilds_seen = 0;
    uint64_t offset = 0;  // O-steps since the start of the call (the counter the kernels add to step_base)
    auto check = [&](uint64_t offset_at_snapshot, bool can_restore) -> nnp_status {
        read_status();
        long long rb;
        std::memcpy(&rb, hflags + 32, sizeof(long long));
        st->n_rebuilds += rb - rebuilds_seen;
        rebuilds_seen = rb;
        // a stale list may have produced anything else flagged here as well
        if (hflags[4] != 0) return NNP_ESTALE_INTERNAL;
        // so may a fast force that disagreed: the rewind undoes those steps
        if (rewind && hflags[12] != 0) return NNP_EREWIND_INTERNAL;
        const bool row_long = hflags[16 + 2] != 0 || hflags[8 + 2] != 0;
        const bool over_cons = hflags[16 + 0] != 0;
        const bool over_nc = hflags[8 + 0] != 0;
        if (row_long || over_cons || over_nc) {
            if (over_cons) st->nl_cons.n_edges = hflags[16 + 1];
            if (over_nc) st->nl_nc.n_edges = hflags[8 + 1];
            if (can_restore) {
                copy_state(c.rs, false);
                st->step -= offset - offset_at_snapshot;
                offset = offset_at_snapshot;
                NNP_HIP(hipStreamSynchronize(s));
            }
            st->lists_valid = 0;
            set_error(row_long ? "a neighbour row exceeds the 1024-entry limit of the builder"
                               : "neighbour list capacity exceeded; grow the buffer to n_edges and call again");
            return row_long ? NNP_EROWLIMIT : NNP_ECAPACITY;
        }
        bool any_bad = false;
        for (int r = 0; r < R; ++r) {
            any_bad |= bad[r] != 0;
            if (rep_bad) rep_bad[r] = bad[r];
        }
        if (any_bad && !rep_bad) {
            set_error("non-finite positions or velocities");
            return NNP_EUNSTABLE;
        }
        return NNP_OK;
    };

    // work at entry that can fail (a list build, the first evaluation) is
    // checked before the first step; a call that starts from valid lists and
    // cached forces goes straight on
    bool entry_work = false;
    const bool built_at_entry = !st->lists_valid;
    // valid lists from an earlier call: their order, with the caller's
    // current positions
    if (rows && st->lists_valid) launch_gather_rows(n, perm, st->pos, st->sys.species, c.pos_rows, c.species_rows, s);
    if (!st->lists_valid) {
        // empty rows until the first build succeeds, so a failed build never
        // leaves uninitialised offsets behind (and the identity order)
        if (rows) launch_reset_rows(n, st->order, st->pos, st->sys.species, c.pos_rows, c.species_rows, s);
        NNP_HIP(hipMemsetAsync(lc.offsets, 0, sizeof(int) * (size_t(n) + 1), s));
        if (mts) NNP_HIP(hipMemsetAsync(ln.offsets, 0, sizeof(int) * (size_t(n) + 1), s));
        launch_set_flag(trig, 1, s);
        rebuild_if_flagged();
        st->lists_valid = 1;
        entry_work = true;
    }
    if (st->first_step) {
        if (mts) eval_inner();
        eval_cons();
        st->first_step = 0;
        entry_work = true;
    }
    if (entry_work) {
        nnp_status e = check(0, false);
        if (e != NNP_OK) return e;
    }
    const int check_every = std::max(1, p->check_every);
    NNP_REQUIRE(!rewind || p->save_every % check_every == 0, NNP_EINVAL,
                "with rewinding on, save_every must be a multiple of check_every (frames are saved at checks)");
    const int n_in = mts ? p->n_inner : 1;
    const double D = p->dt_outer_fs;
    const double d = D / n_in;

    // one BAOAB step of size dt with the conservative force
    auto sts_step = [&](double dt) {
        ba.flag = trig;  // the per-step displacement check rebuilds at once
        ba.force = st->f_cons;
        ba.dt = dt;
        ba.step_offset = 0;
        ba.full_kick = 0;
        launch_baoa(ba, s);
        rebuild_if_flagged();
        eval_cons();
        if (want_vir) launch_rep_sum(R, c.t.rep_start, c.cons.vir, st->virial, s);
        launch_kick(n, st->vel, st->mass, st->f_cons, nullptr, 0.5 * dt, s, c.t.o_step);
        offset += 1;
        st->step += 1;
    };
    // One outer step of Algorithm 1.  Predictive mode decides on a rebuild
    // once per outer step (from the displacement record) and lets k_baoa only
    // flag a list that went stale; strict mode rebuilds after any inner step
    // whose displacement check fires.  Both give the same numbers whenever
    // no stale flag is raised (results do not depend on when lists are built).
    // (launches only; the caller advances offset and st->step by n_in)
    // The conservative evaluation at the end of the outer step reads the
    // positions the last inner BAOA fixed and writes only its own buffers:
    // it runs on the side stream beside the last inner evaluation and the
    // closing kick, and is joined before the outer kick.
    const SideStream* side = mts ? side_stream() : nullptr;
    auto eval_cons_beside = [&]() {
        NNP_HIP(hipEventRecord(side->fork, s));
        NNP_HIP(hipStreamWaitEvent(side->s, side->fork, 0));
        const hipStream_t main = s;
        struct Restore {
            hipStream_t& ref;
            hipStream_t v;
            ~Restore() { ref = v; }
        } restore{s, main};
        s = side->s;
        eval_cons();
        NNP_HIP(hipEventRecord(side->join, side->s));
    };
    // With the spare build (ov), the step's own rebuild was decided and made
    // by the previous step, or by mts_step just before it.
    auto mts_launches = [&](bool strict) {
        const bool ov = !strict && overlap_build && side;
        if (!strict && !ov) {
            launch_predict_rebuild(maxd2, disp_thr, trig, s);
            rebuild_if_flagged();
        }
        ba.flag = strict ? trig : stale;
        if (want_vir) launch_zero(c.nc.vir_sum, n, nullptr, s);
        launch_kick(n, st->vel, st->mass, st->f_cons, st->f_nc, 0.5 * D, s);
        // inner step k: its opening kick also closes step k - 1 (the same fast
        // force, nothing reads the velocities in between); its O-step index
        // is the counter plus k, and the closing kick of the last step
        // advances the counter past all n_in
        for (int k = 0; k < n_in; ++k) {
            ba.force = st->f_nc;
            ba.dt = d;
            ba.full_kick = k > 0;
            ba.step_offset = uint64_t(k);
            launch_baoa(ba, s);
            if (strict) rebuild_if_flagged();
            if (side && k == n_in - 1) eval_cons_beside();
            eval_inner();
        }
        if (ov) build_spare_if_predicted();
        launch_kick(n, st->vel, st->mass, st->f_nc, nullptr, 0.5 * d, s, c.t.o_step, uint64_t(n_in));
        if (side) NNP_HIP(hipStreamWaitEvent(s, side->join, 0));
        else eval_cons();
        if (ov) adopt_spare();
        if (want_vir) {
            launch_virial_combine(n, c.cons.vir, c.nc.vir, c.nc.vir_sum, float(1.0 / n_in), c.cons.vir_sum, s);
            launch_rep_sum(R, c.t.rep_start, c.cons.vir_sum, st->virial, s);
        }
        launch_kick(n, st->vel, st->mass, st->f_cons, st->f_nc, 0.5 * D, s);
        if (rewind) {
            // both forces now belong to the end of the step; a trip is acted
            // on at the next status check
            k_disagreement_part<<<dim3(dis_chunks, R), 256, 0, s>>>(c.t.rep_start, n, dis_chunks, st->f_cons,
                                                                   st->f_nc, st->pos, st->vel, disagree + R);
            k_disagreement_final<<<R, 64, 0, s>>>(c.t.rep_start, dis_chunks, disagree + R, disagree,
                                                  p->rewind_threshold, trip);
            NNP_LAUNCH_CHECK();
        }
    };
    // Predictive outer steps can be recorded once as a HIP graph and replayed:
    // every launch argument is fixed within the call (the O-step counter and
    // the rebuild decision live on the device) and nothing in them waits on
    // the host.
    struct OuterGraph {
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
        hipStream_t cs = nullptr;  // recording stream (the legacy default stream cannot record)
        bool failed = false;
        ~OuterGraph() {
            if (x) (void)hipGraphExecDestroy(x);
            if (g) (void)hipGraphDestroy(g);
            if (cs) (void)hipStreamDestroy(cs);
        }
    } outer_graph;
    bool prebuilt = false;  // this step's rebuild was decided by the previous (spare-building) step
    auto mts_step = [&](bool strict, bool allow_graph) {
        const bool ov = !strict && overlap_build && side;
        if (ov && !prebuilt) {
            launch_predict_rebuild(maxd2, disp_thr, trig, s);
            rebuild_if_flagged();
        }
        if (!strict && allow_graph && !outer_graph.failed) {
            if (!outer_graph.x) {
                // record on a private stream that first waits for the work
                // already queued on s; the launches below then target it
                bool ok = hipStreamCreateWithFlags(&outer_graph.cs, hipStreamNonBlocking) == hipSuccess;
                ok = ok && hipStreamSynchronize(s) == hipSuccess;
                const hipStream_t caller = s;
                ok = ok && hipStreamBeginCapture(outer_graph.cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
                if (ok) {
                    s = outer_graph.cs;
                    try {
                        mts_launches(false);
                    } catch (const Fail&) {
                        ok = false;
                    }
                    s = caller;
                    hipGraph_t g = nullptr;
                    ok = (hipStreamEndCapture(outer_graph.cs, &g) == hipSuccess) && ok && g;
                    outer_graph.g = g;
                    ok = ok && hipGraphInstantiate(&outer_graph.x, g, nullptr, nullptr, 0) == hipSuccess;
                }
                if (!ok) {
                    // recording is an optimisation only: fall back to direct launches
                    (void)hipGetLastError();
                    outer_graph.failed = true;
                }
            }
            if (outer_graph.x) {
                NNP_HIP(hipGraphLaunch(outer_graph.x, s));
            } else {
                mts_launches(false);
            }
        } else {
            mts_launches(strict);
        }
        prebuilt = ov;
        offset += n_in;
        st->step += n_in;
    };

    // predictive rebuilds for multiple-time-step runs; a stale list found at
    // a check sends the run back to the last snapshot, which is replayed in
    // strict mode
    const bool predictive = mts && n_in > 1;
    const bool use_graph = predictive && p->graph != 0 && n_outer >= 3 && !timers_active();
    if (predictive && !built_at_entry) {
        // lists from an earlier call: rebuild the displacement record from
        // pos_ref, taking its growth over the previous outer step to be all
        // of it (an over-estimate: at worst an early rebuild)
        launch_disp_record(n, st->pos, st->pos_ref, maxd2, s);
    }
    uint64_t snap_offset = 0;
    int snap_o = 0, strict_until = 0, snap_since_save = 0;
    copy_state(c.rs, true);
    // Rewind procedure: frames are saved at status checks only (the trip is
    // read there), every save_every kept outer steps; a trip sends the state
    // and the loop back to the frame, so the steps taken since then do not
    // count, whichever check found it.
    uint64_t frame_offset = 0;
    int frame_o = 0, since_save = 0, rewinds_here = 0;
    const int rewind_limit = std::max(16, n_outer);
    for (int o = 0; o < n_outer; ++o) {
        const bool strict = !predictive || o < strict_until;
        if (rewind && since_save % p->save_every == 0) {
            copy_state(frame, true);
            frame_offset = offset;
            frame_o = o;
            since_save = 0;
        }
        if (mts) mts_step(strict, use_graph);
        else sts_step(D);
        ++since_save;
        launch_kinetic(R, c.t.rep_start, n, st->pos, st->vel, st->mass, st->ke ? st->ke + int64_t(o) * R : nullptr,
                       c.t.rep_bad, s, st->sys.rep_of_atom, c.ke_part, ke_chunks);
        if (stamps) launch_stamp(stamps + o, s);
        if ((o + 1) % check_every == 0 || o + 1 == n_outer) {
            nnp_status e = check(snap_offset, true);
            if (e == NNP_ESTALE_INTERNAL || e == NNP_EREWIND_INTERNAL) {
                const bool back_to_frame = e == NNP_EREWIND_INTERNAL;
                if (back_to_frame) {
                    copy_state(frame, false);
                    st->step -= offset - frame_offset;
                    offset = frame_offset;
                    o = frame_o - 1;
                    strict_until = 0;
                    if (++rewinds_here > rewind_limit) {
                        // leave the state at the saved frame (its last good step)
                        NNP_HIP(hipStreamSynchronize(s));
                        set_error("the fast force keeps disagreeing: rewind limit of the call reached");
                        return NNP_EUNSTABLE;
                    }
                } else {
                    // back to the snapshot; replay up to here with strict rebuilds
                    copy_state(c.rs, false);
                    st->step -= offset - snap_offset;
                    offset = snap_offset;
                    strict_until = o + 1;
                    o = snap_o - 1;
                    since_save = snap_since_save;
                    st->n_replays += 1;
                }
                launch_set_u64(c.t.o_step, offset, s);
                prebuilt = false;
                NNP_HIP(hipMemsetAsync(c.t.flags + 4, 0, sizeof(int) * 12, s));  // stale, record, lists, trip
                NNP_HIP(hipMemsetAsync(c.nb.status, 0, sizeof(int) * 8, s));
                NNP_HIP(hipMemsetAsync(c.t.rep_bad, 0, sizeof(int) * R, s));
                launch_set_flag(trig, 1, s);
                rebuild_if_flagged();
                if (back_to_frame) {
                    // single time steps of delta with the reference force, a
                    // fresh fast force, then multiple time steps again
                    for (int k = 0; k < p->sts_after_rewind; ++k) sts_step(d);
                    eval_inner();
                    st->n_rewinds += 1;
                    since_save = 0;
                    snap_offset = offset;
                    snap_o = frame_o;
                    snap_since_save = 0;
                    copy_state(c.rs, true);
                }
                continue;
            }
            if (e != NNP_OK) return e;
            snap_offset = offset;
            snap_o = o + 1;
            snap_since_save = since_save;
            if (o + 1 < n_outer) copy_state(c.rs, true);
        }
    }
    return NNP_OK;
}

}  // namespace nnp

extern "C" nnp_status nnp_barostat_scr(respa_state* st, const nnp_barostat_params* p, uint64_t barostat_step,
                                       double* box_host, double* box_dev, void* ws, size_t ws_bytes, void* stream) {
    NNP_API_BEGIN
    NNP_REQUIRE(st && p && box_host, NNP_EINVAL, "null argument");
    NNP_REQUIRE(st->virial, NNP_EINVAL, "the barostat needs state->virial (the last outer step's estimator)");
    NNP_REQUIRE(st->pos && st->vel && st->mass && st->sys.pos == st->pos, NNP_EINVAL, "incomplete state");
    NNP_REQUIRE(p->tau_fs > 0 && p->dt_fs > 0 && p->compressibility_per_bar >= 0 && p->temperature_K >= 0 &&
                    std::isfinite(p->pressure_bar),
                NNP_EINVAL, "bad barostat parameters");
    check_system(&st->sys);
    NNP_REQUIRE(box_host == st->sys.box, NNP_EINVAL, "box_host must be the system's host box array");
    NNP_REQUIRE(st->sys.n_rep == 1 || box_dev == st->sys.box_dev, NNP_EINVAL,
                "box_dev must be the system's device box array");
    const int n = int(st->sys.n_atoms), R = st->sys.n_rep;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Arena a(ws, ws_bytes);
    SysTables t;
    carve_tables(a, R, t);
    double* ke = a.take<double>(R);
    double* mu = a.take<double>(R);
    int chunks = 1;
    for (int r = 0; r < R; ++r)
        chunks = std::max<int>(chunks, cdiv(st->sys.rep_start[r + 1] - st->sys.rep_start[r], kKeChunk));
    double* part = a.take<double>(int64_t(R) * chunks);
    std::vector<double> hs;
    upload_tables(st->sys, t, s, hs);
    launch_kinetic(R, t.rep_start, n, st->pos, st->vel, st->mass, ke, nullptr, s, st->sys.rep_of_atom, part, chunks);
    const double bar = 1e5 * 6.02214076e23 * 1e-30 / 4184.0;  // kcal/mol/A^3
    ScrArgs sa{p->pressure_bar * bar, p->compressibility_per_bar / bar, p->tau_fs, p->dt_fs, p->temperature_K,
               p->seed, p->stream_id, barostat_step};
    launch_scr(R, ke, st->virial, t.box, mu, sa, s);
    launch_scale(n, R > 1 ? st->sys.rep_of_atom : nullptr, mu, st->pos, st->vel, s);
    if (box_dev) NNP_HIP(hipMemcpyAsync(box_dev, t.box, sizeof(double) * R, hipMemcpyDeviceToDevice, s));
    std::vector<double> nb(R);
    NNP_HIP(hipMemcpyAsync(nb.data(), t.box, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    NNP_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < R; ++r) box_host[r] = nb[r];
    st->lists_valid = 0;
    st->first_step = 1;
    NNP_API_END
}

extern "C" nnp_status respa_step(const nnp_model* cons_h, const nnp_model* nc_h, respa_state* st,
                                 const respa_params* p, int32_t n_outer, void* ws, size_t ws_bytes, void* stream) {
    NNP_API_BEGIN
    NNP_REQUIRE(st && p, NNP_EINVAL, "null argument");
    const int R = st->sys.n_rep;
    NNP_REQUIRE(R >= 1, NNP_EINVAL, "n_rep must be >= 1");
    std::vector<uint64_t> seeds(R, p->seed), streams(R), base(R, st->step);
    for (int r = 0; r < R; ++r) streams[r] = p->stream_id + uint64_t(r);
    nnp_status e = respa_run(reinterpret_cast<const Model*>(cons_h), reinterpret_cast<const Model*>(nc_h), st, p,
                             n_outer, ws, ws_bytes, static_cast<hipStream_t>(stream), seeds.data(), streams.data(),
                             base.data(), nullptr);
    if (e != NNP_OK) return e;
    NNP_API_END
}
