// Edge kernels of the embedding block: the message step and its reverse.
//
// Layout: one feature column per lane.  An atom is handled by WPA = F / 64
// wavefronts when F > 64 (each owns 64 consecutive columns), otherwise by a
// group of G = F lanes (64 / G atoms per wavefront); a neighbour's row is
// read with unit stride across the lanes.  Splitting wide rows over two
// wavefronts halves the filter weights each lane keeps in registers.
// Per-atom rows are [n][F] (s), [n][3][F] (v) and [n][3F] (phi = [a|b|c]).
//
// Edge geometry is formed once per edge and batch: the group's lanes take
// one CSR entry each, apply the float64 pair rule at the model cutoff (this
// also filters Verlet lists built at a larger radius), compact the surviving
// edges with a wavefront ballot and stage r, u = r_ij / r and the radial
// values e_k(r) f(r) (and their r-derivatives for the reverse pass) in LDS.
// The per-edge filter w = (Wr e + br) f is then a K-term dot product per
// feature against Wr rows held in registers.
//
// Forward (per layer, synchronous: every term reads the layer input):
//   s_i += sum_j phi_a[j] w_a;  v_i[al] += sum_j (phi_b[j] w_b v_j[al] + u[al] phi_c[j] w_c)
//
// Reverse, owner-computes (atom o gathers everything that reaches it; no
// atomics; fixed order per atom).  For each neighbour n of o, with the layer
// adjoints gs = dL/ds_mid and gv = dL/dv_mid of both atoms:
//   (B) o as sender of the message o -> n: adjoints of phi_o and v_o;
//   (A) o as receiver of n -> o and (A') o as sender of o -> n: the filter
//       adjoints g_w of both messages share w(r) and dw/dr, so the pair's
//       contribution to the force on o,
//         -dE/dx_o (pair) = (d_A + d_A') u + (P(g_uA) - P(g_uA')) / r,
//         d = sum_f g_w . dw/dr,  P = 1 - u u^T,
//       is linear in per-lane partial sums; each lane accumulates its share
//       over all edges and the group is reduced once per atom.
//   With weight adjoints requested (NC distillation), the filter weight
//   adjoints of the message n -> o are accumulated as well (each directed
//   message is counted by its receiver).
#include <hip/hip_ext.h>

#include <atomic>

#include "common.h"
#include "kernels.h"
#include "mp_edge.h"

namespace nnp {

constexpr int kMpWaves = 4;

// Stages one batch of edges of atom i (lane l of its group takes entry e)
// into LDS; returns the number of surviving edges of this group.
template <int G, int K, int CUT, bool DERIV>
__device__ __forceinline__ int stage_batch(const MpGeom& mg, bool active, int e, int e_end, int l, int g, double xi,
                                           double yi, double zi, double L, double inv, EdgeSlot<K>* slots,
                                           const int* species) {
    bool ok = false;
    double dx = 0, dy = 0, dz = 0;
    int j = -1;
    if (active && e < e_end) {
        j = mg.nbr[e];
        const int n = mg.n;
        ok = pair_rule(xi, yi, zi, mg.pos[j], mg.pos[n + j], mg.pos[2 * n + j], L, inv, mg.rc2, dx, dy, dz);
    }
    const uint64_t bal = __ballot(ok);
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (g * G));
    const uint64_t mine = bal & gmask;
    const int pre = __popcll(mine & ((1ull << (g * G + l)) - 1ull));
    if (ok) {
        EdgeSlot<K>& s = slots[pre];
        if constexpr (CUT == 1 && !DERIV) {
            // NC forward: radial values in float32
            const float r = sqrtf(float((dx * dx + dy * dy) + dz * dz));
            const float ir = 1.f / r;
            radial_poly_f32<K>(r * float(mg.inv_rc), float(mg.bessel_norm) * ir, s.ef, s.fc);
            s.dfc = 0.f;
            s.u[0] = float(dx) * ir;
            s.u[1] = float(dy) * ir;
            s.u[2] = float(dz) * ir;
            s.ir = ir;
            s.r = r;
        } else if constexpr (CUT == 0) {
            // conservative model: radial values in float32
            const double r = sqrt((dx * dx + dy * dy) + dz * dz);
            const double ir = 1.0 / r;
            radial_cos_f32<K>(float(r), mg, s.ef, s.def, s.fc, s.dfc);
            s.u[0] = float(dx * ir);
            s.u[1] = float(dy * ir);
            s.u[2] = float(dz * ir);
            s.ir = float(ir);
        } else {
            const double r = sqrt((dx * dx + dy * dy) + dz * dz);
            const double ir = 1.0 / r;
            radial<K, CUT, DERIV>(r, mg, s.ef, s.def, s.fc, s.dfc);
            s.u[0] = float(dx * ir);
            s.u[1] = float(dy * ir);
            s.u[2] = float(dz * ir);
            s.ir = float(ir);
        }
        s.j = j;
        s.t = species ? min(max(species[j], 0), mg.n_species - 1) : 0;
    }
    wave_sync_lds();
    return __popcll(mine);
}

template <int FPL>
struct Vec {
    float x[FPL];
};

template <int FPL>
__device__ __forceinline__ Vec<FPL> ldv(const float* p) {
    Vec<FPL> r;
    if constexpr (FPL == 2) {
        const float2 t = *reinterpret_cast<const float2*>(p);
        r.x[0] = t.x;
        r.x[1] = t.y;
    } else if constexpr (FPL == 4) {
        const float4 t = *reinterpret_cast<const float4*>(p);
        r.x[0] = t.x; r.x[1] = t.y; r.x[2] = t.z; r.x[3] = t.w;
    } else {
#pragma unroll
        for (int q = 0; q < FPL; ++q) r.x[q] = p[q];
    }
    return r;
}

template <int FPL>
__device__ __forceinline__ void stv(float* p, const float* v) {
    if constexpr (FPL == 2) {
        *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
    } else {
#pragma unroll
        for (int q = 0; q < FPL; ++q) p[q] = v[q];
    }
}

template <int F>
struct MpShape {
    static constexpr int G = F >= 64 ? 64 : F;         // lanes per atom within a wavefront
    static constexpr int WPA = F / G;                  // wavefronts per atom
    static constexpr int APW = 64 / G;                 // atoms per wavefront
    static constexpr int APB = kMpWaves / WPA * APW;   // atoms per block
    // With several wavefronts per atom, the first one stages each batch of
    // edges for all of them (block barriers around the batch): the edge
    // geometry is computed once per atom and the slots take less LDS.
    static constexpr bool SHARED = WPA > 1;
    static constexpr int SLOT_SETS = SHARED ? kMpWaves / WPA : kMpWaves;
};

template <int F, int K, int CUT, bool L0>
__global__ void __launch_bounds__(64 * kMpWaves)
k_message_fwd(MpGeom mg, MpFwd a) {
    using S = MpShape<F>;
    constexpr int G = S::G, APW = S::APW, WPA = S::WPA, FPL = 1;
    __shared__ EdgeSlot<K> slots_all[S::SLOT_SETS][APW][G];
    __shared__ int batch_cnt[S::SLOT_SETS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane / G, l = lane % G;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int i = blk * S::APB + (w / WPA) * APW + g;
    const bool active = i < mg.n;
    const int n = mg.n;
    const int f0 = (w % WPA) * 64 + l;
    EdgeSlot<K>* slots = slots_all[S::SHARED ? w / WPA : w][g];

    float wr[3][FPL][K], bb[3][FPL];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < FPL; ++q) {
            const int row = p * F + f0 + q;
#pragma unroll
            for (int k = 0; k < K; ++k) wr[p][q][k] = a.Wr[row * K + k];
            bb[p][q] = a.br[row];
        }
    float sacc[FPL] = {}, vacc[3][FPL] = {};
    int start = 0, end = 0, emitted = 0;
    double xi = 0, yi = 0, zi = 0, L = 1, inv = 1;
    if (active) {
        start = mg.off[i];
        end = mg.off[i + 1];
        mg.geom.get(i, L, inv);
        xi = mg.pos[i]; yi = mg.pos[n + i]; zi = mg.pos[2 * n + i];
    }
    for (int base = 0; S::SHARED ? __syncthreads_or(start + base < end) != 0
                                 : __ballot(start + base < end) != 0ull;
         base += G) {
        int cnt;
        if constexpr (S::SHARED) {
            if (w % WPA == 0) {
                const int c = stage_batch<G, K, CUT, false>(mg, active, start + base + l, end, l, g, xi, yi, zi, L,
                                                          inv, slots, L0 ? a.species : nullptr);
                if (lane == 0) batch_cnt[w / WPA] = c;
            }
            __syncthreads();
            cnt = __builtin_amdgcn_readfirstlane(batch_cnt[w / WPA]);  // wavefront-uniform
        } else {
            cnt = stage_batch<G, K, CUT, false>(mg, active, start + base + l, end, l, g, xi, yi, zi, L, inv, slots,
                                              L0 ? a.species : nullptr);
            if constexpr (CUT == 1 && K == 8) {
                // the NC pair head reads the same edges as records
                if (a.edge_out && l < cnt) {
                    const EdgeSlot<K>& s = slots[l];
                    NcEdge rec;
                    rec.j = s.j;
                    rec.r = s.r;
                    rec.u[0] = s.u[0];
                    rec.u[1] = s.u[1];
                    rec.u[2] = s.u[2];
                    rec.pad[0] = rec.pad[1] = rec.pad[2] = 0.f;
#pragma unroll
                    for (int k = 0; k < K; ++k) rec.ef[k] = s.ef[k];
                    a.edge_out[start + emitted + l] = rec;
                }
                emitted += cnt;
            }
        }
#pragma unroll 1
        for (int t = 0; t < cnt; ++t) {
            const EdgeSlot<K>& s = slots[t];
            const float* phj = L0 ? a.phi_tab + s.t * 3 * F + f0 : a.phi + int64_t(s.j) * 3 * F + f0;
            const Vec<FPL> pa = ldv<FPL>(phj), pb = ldv<FPL>(phj + F), pc = ldv<FPL>(phj + 2 * F);
            Vec<FPL> v0{}, v1{}, v2{};
            if (!L0) {  // the first layer's vector input is zero
                const float* vj = a.v_in + int64_t(s.j) * 3 * F + f0;
                v0 = ldv<FPL>(vj);
                v1 = ldv<FPL>(vj + F);
                v2 = ldv<FPL>(vj + 2 * F);
            }
#pragma unroll
            for (int q = 0; q < FPL; ++q) {
                float wa = bb[0][q] * s.fc, wb = bb[1][q] * s.fc, wc = bb[2][q] * s.fc;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    wa = fmaf(wr[0][q][k], s.ef[k], wa);
                    if (!L0) wb = fmaf(wr[1][q][k], s.ef[k], wb);
                    wc = fmaf(wr[2][q][k], s.ef[k], wc);
                }
                const float c = pc.x[q] * wc;
                sacc[q] = fmaf(pa.x[q], wa, sacc[q]);
                if (L0) {
                    vacc[0][q] += s.u[0] * c;
                    vacc[1][q] += s.u[1] * c;
                    vacc[2][q] += s.u[2] * c;
                } else {
                    const float b = pb.x[q] * wb;
                    vacc[0][q] += b * v0.x[q] + s.u[0] * c;
                    vacc[1][q] += b * v1.x[q] + s.u[1] * c;
                    vacc[2][q] += b * v2.x[q] + s.u[2] * c;
                }
            }
        }
        if constexpr (S::SHARED) __syncthreads();  // the slots are restaged next
        else wave_sync_lds();
    }
    if constexpr (CUT == 1 && K == 8 && !S::SHARED) {
        if (a.edge_cnt && active && l == 0) a.edge_cnt[i] = emitted;
    }
    if (active) {
        float out[FPL];
        const int ti = L0 ? min(max(a.species[i], 0), mg.n_species - 1) : 0;
        const Vec<FPL> si = ldv<FPL>(L0 ? a.emb + ti * F + f0 : a.s_in + int64_t(i) * F + f0);
#pragma unroll
        for (int q = 0; q < FPL; ++q) out[q] = si.x[q] + sacc[q];
        stv<FPL>(a.s_out + int64_t(i) * F + f0, out);
#pragma unroll
        for (int al = 0; al < 3; ++al) {
            const int64_t idx = (int64_t(i) * 3 + al) * F + f0;
            Vec<FPL> vi{};
            if (!L0) vi = ldv<FPL>(a.v_in + idx);
#pragma unroll
            for (int q = 0; q < FPL; ++q) out[q] = vi.x[q] + vacc[al][q];
            stv<FPL>(a.v_out + idx, out);
        }
    }
}

template <int F, int K, int CUT, bool GEO, bool WGRAD, bool L0>
__global__ void __launch_bounds__(64 * kMpWaves, 2)
k_message_bwd(MpGeom mg, MpBwd a) {
    using S = MpShape<F>;
    constexpr int G = S::G, APW = S::APW, WPA = S::WPA, FPL = 1;
    static_assert(!WGRAD || WPA == 1, "filter weight adjoints need one wavefront per atom");
    __shared__ EdgeSlot<K> slots_all[S::SLOT_SETS][APW][G];
    __shared__ int batch_cnt[S::SLOT_SETS];
    __shared__ float fpart[kMpWaves][APW][4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane / G, l = lane % G;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int i = blk * S::APB + (w / WPA) * APW + g;
    const bool active = i < mg.n;
    const int n = mg.n;
    const int f0 = (w % WPA) * 64 + l;
    EdgeSlot<K>* slots = slots_all[S::SHARED ? w / WPA : w][g];

    float wr[3][FPL][K], bb[3][FPL];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < FPL; ++q) {
            const int row = p * F + f0 + q;
#pragma unroll
            for (int k = 0; k < K; ++k) wr[p][q][k] = a.Wr[row * K + k];
            bb[p][q] = a.br[row];
        }
    // own rows of the owner atom o = i
    float ph_o[3][FPL] = {}, v_o[3][FPL] = {}, gs_o[FPL] = {}, gv_o[3][FPL] = {};
    float gph[3][FPL] = {}, gvacc[3][FPL] = {};
    float fx = 0.f, fy = 0.f, fz = 0.f;  // per-lane share of the force on o
    float vr = 0.f;                      // and of sum_j r_oj . f_oj
    float gwr[WGRAD ? 3 : 1][WGRAD ? FPL : 1][WGRAD ? K : 1] = {};
    float gbr[WGRAD ? 3 : 1][WGRAD ? FPL : 1] = {};
    int start = 0, end = 0;
    double xi = 0, yi = 0, zi = 0, L = 1, inv = 1;
    if (active) {
        start = mg.off[i];
        end = mg.off[i + 1];
        mg.geom.get(i, L, inv);
        xi = mg.pos[i]; yi = mg.pos[n + i]; zi = mg.pos[2 * n + i];
        const int ti = L0 ? min(max(a.species[i], 0), mg.n_species - 1) : 0;
        const float* pho = L0 ? a.phi_tab + ti * 3 * F + f0 : a.phi + int64_t(i) * 3 * F + f0;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            const Vec<FPL> t = ldv<FPL>(pho + p * F);
#pragma unroll
            for (int q = 0; q < FPL; ++q) ph_o[p][q] = t.x[q];
        }
#pragma unroll
        for (int al = 0; al < 3; ++al) {
            Vec<FPL> tv{};
            if (!L0) tv = ldv<FPL>(a.v_in + (int64_t(i) * 3 + al) * F + f0);
            const Vec<FPL> tg = ldv<FPL>(a.gvm + (int64_t(i) * 3 + al) * F + f0);
#pragma unroll
            for (int q = 0; q < FPL; ++q) {
                v_o[al][q] = tv.x[q];
                gv_o[al][q] = tg.x[q];
            }
        }
        const Vec<FPL> tg = ldv<FPL>(a.gsm + int64_t(i) * F + f0);
#pragma unroll
        for (int q = 0; q < FPL; ++q) gs_o[q] = tg.x[q];
    }
    for (int base = 0; S::SHARED ? __syncthreads_or(start + base < end) != 0
                                 : __ballot(start + base < end) != 0ull;
         base += G) {
        int cnt;
        if constexpr (S::SHARED) {
            if (w % WPA == 0) {
                const int c = stage_batch<G, K, CUT, GEO>(mg, active, start + base + l, end, l, g, xi, yi, zi, L,
                                                          inv, slots, L0 ? a.species : nullptr);
                if (lane == 0) batch_cnt[w / WPA] = c;
            }
            __syncthreads();
            cnt = __builtin_amdgcn_readfirstlane(batch_cnt[w / WPA]);  // wavefront-uniform
        } else {
            cnt = stage_batch<G, K, CUT, GEO>(mg, active, start + base + l, end, l, g, xi, yi, zi, L, inv, slots,
                                              L0 ? a.species : nullptr);
        }
#pragma unroll 1
        for (int t = 0; t < cnt; ++t) {
            const EdgeSlot<K>& s = slots[t];
            const int j = s.j;
            const float* phj = L0 ? a.phi_tab + s.t * 3 * F + f0 : a.phi + int64_t(j) * 3 * F + f0;
            const float* gvj = a.gvm + int64_t(j) * 3 * F + f0;
            const Vec<FPL> pa = ldv<FPL>(phj), pb = ldv<FPL>(phj + F), pc = ldv<FPL>(phj + 2 * F);
            Vec<FPL> vj0{}, vj1{}, vj2{};
            if (!L0) {  // the first layer's vector input is zero
                const float* vj = a.v_in + int64_t(j) * 3 * F + f0;
                vj0 = ldv<FPL>(vj);
                vj1 = ldv<FPL>(vj + F);
                vj2 = ldv<FPL>(vj + 2 * F);
            }
            const Vec<FPL> g0 = ldv<FPL>(gvj), g1 = ldv<FPL>(gvj + F), g2 = ldv<FPL>(gvj + 2 * F);
            const Vec<FPL> gsn = ldv<FPL>(a.gsm + int64_t(j) * F + f0);
            const float u0 = s.u[0], u1 = s.u[1], u2 = s.u[2];
            float dr = 0.f, gu0 = 0.f, gu1 = 0.f, gu2 = 0.f;
#pragma unroll
            for (int q = 0; q < FPL; ++q) {
                float w[3], dw[3];
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    w[p] = bb[p][q] * s.fc;
                    dw[p] = bb[p][q] * s.dfc;
                }
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int p = 0; p < 3; ++p) {
                        w[p] = fmaf(wr[p][q][k], s.ef[k], w[p]);
                        if (GEO) dw[p] = fmaf(wr[p][q][k], s.def[k], dw[p]);
                    }
                // projections shared by several terms
                const float gvo_vn = gv_o[0][q] * vj0.x[q] + gv_o[1][q] * vj1.x[q] + gv_o[2][q] * vj2.x[q];
                const float gvo_u = gv_o[0][q] * u0 + gv_o[1][q] * u1 + gv_o[2][q] * u2;
                const float gvn_vo = g0.x[q] * v_o[0][q] + g1.x[q] * v_o[1][q] + g2.x[q] * v_o[2][q];
                const float gvn_u = g0.x[q] * u0 + g1.x[q] * u1 + g2.x[q] * u2;
                // (A) message n -> o: filter adjoints
                const float gwa = gs_o[q] * pa.x[q];
                const float gwb = pb.x[q] * gvo_vn;
                const float gwc = pc.x[q] * gvo_u;
                if (GEO) {
                    // (A') message o -> n (unit vector -u): filter adjoints
                    const float gwa2 = gsn.x[q] * ph_o[0][q];
                    const float gwb2 = ph_o[1][q] * gvn_vo;
                    const float gwc2 = -ph_o[2][q] * gvn_u;
                    dr += (gwa + gwa2) * dw[0] + (gwb + gwb2) * dw[1] + (gwc + gwc2) * dw[2];
                    // g_uA - g_uA': adjoints of the unit vector of each message
                    const float cA = pc.x[q] * w[2], cB = ph_o[2][q] * w[2];
                    gu0 += gv_o[0][q] * cA - g0.x[q] * cB;
                    gu1 += gv_o[1][q] * cA - g1.x[q] * cB;
                    gu2 += gv_o[2][q] * cA - g2.x[q] * cB;
                }
                if (WGRAD) {
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        gwr[0][q][k] = fmaf(gwa, s.ef[k], gwr[0][q][k]);
                        gwr[1][q][k] = fmaf(gwb, s.ef[k], gwr[1][q][k]);
                        gwr[2][q][k] = fmaf(gwc, s.ef[k], gwr[2][q][k]);
                    }
                    gbr[0][q] = fmaf(gwa, s.fc, gbr[0][q]);
                    gbr[1][q] = fmaf(gwb, s.fc, gbr[1][q]);
                    gbr[2][q] = fmaf(gwc, s.fc, gbr[2][q]);
                }
                // (B) o sends to n (unit vector of that message is -u)
                gph[0][q] = fmaf(gsn.x[q], w[0], gph[0][q]);
                gph[1][q] = fmaf(w[1], gvn_vo, gph[1][q]);
                gph[2][q] = fmaf(-w[2], gvn_u, gph[2][q]);
                const float wbp = w[1] * ph_o[1][q];
                gvacc[0][q] = fmaf(g0.x[q], wbp, gvacc[0][q]);
                gvacc[1][q] = fmaf(g1.x[q], wbp, gvacc[1][q]);
                gvacc[2][q] = fmaf(g2.x[q], wbp, gvacc[2][q]);
            }
            if (GEO) {
                // this lane's share of (d_A + d_A') u + P(g_uA - g_uA') / r
                const float ud = gu0 * u0 + gu1 * u1 + gu2 * u2;
                fx += dr * u0 + (gu0 - ud * u0) * s.ir;
                fy += dr * u1 + (gu1 - ud * u1) * s.ir;
                fz += dr * u2 + (gu2 - ud * u2) * s.ir;
                if (a.vir) vr += __fdividef(dr, s.ir);  // the projected term is normal to u
            }
        }
        if constexpr (S::SHARED) __syncthreads();  // the slots are restaged next
        else wave_sync_lds();
    }
    if (GEO) {
        fx = group_sum<G>(fx);
        fy = group_sum<G>(fy);
        fz = group_sum<G>(fz);
        vr = group_sum<G>(vr);
        if (WPA > 1) {
            // combine the wavefronts of the atom in a fixed order
            if (l == 0) {
                fpart[w][g][0] = fx;
                fpart[w][g][1] = fy;
                fpart[w][g][2] = fz;
                fpart[w][g][3] = vr;
            }
            __syncthreads();
            if (w % WPA == 0) {
                fx = fy = fz = vr = 0.f;
                for (int k = 0; k < WPA; ++k) {
                    fx += fpart[w + k][g][0];
                    fy += fpart[w + k][g][1];
                    fz += fpart[w + k][g][2];
                    vr += fpart[w + k][g][3];
                }
            }
        }
        if (active && l == 0 && w % WPA == 0) {
            const int io = mg.perm ? min(max(mg.perm[i], 0), n - 1) : i;
            if (a.accum_force) {
                a.force[io] += fx; a.force[n + io] += fy; a.force[2 * n + io] += fz;
            } else {
                a.force[io] = fx; a.force[n + io] = fy; a.force[2 * n + io] = fz;
            }
            if (a.vir) {  // each pair is seen by both of its atoms
                if (a.accum_force) a.vir[io] += 0.5f * vr;
                else a.vir[io] = 0.5f * vr;
            }
        }
    }
    if (active) {
        float out[FPL];
        if (a.want_gphi) {
#pragma unroll
            for (int p = 0; p < 3; ++p) stv<FPL>(a.gphi + int64_t(i) * 3 * F + p * F + f0, gph[p]);
        }
        if (!L0) {
#pragma unroll
            for (int al = 0; al < 3; ++al) {
#pragma unroll
                for (int q = 0; q < FPL; ++q) out[q] = gv_o[al][q] + gvacc[al][q];
                stv<FPL>(a.gv_in + (int64_t(i) * 3 + al) * F + f0, out);
            }
        }
    }
    if (WGRAD) {
        // per-block partial sums of the filter weight adjoints, reduced over
        // the groups and wavefronts of the block in a fixed order
        __shared__ float red[kMpWaves * APW][3 * F * (K + 1)];
        const int slot = w * APW + g;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < FPL; ++q) {
                const int row = p * F + f0 + q;
#pragma unroll
                for (int k = 0; k < K; ++k) red[slot][row * (K + 1) + k] = gwr[p][q][k];
                red[slot][row * (K + 1) + K] = gbr[p][q];
            }
        __syncthreads();
        for (int t = threadIdx.x; t < 3 * F * (K + 1); t += blockDim.x) {
            float sum = 0.f;
            for (int sl = 0; sl < kMpWaves * APW; ++sl) sum += red[sl][t];
            a.wgrad_part[int64_t(blk) * 3 * F * (K + 1) + t] = sum;
        }
    }
}

// ------------------------------------------------------------------- host --

// launches `kern`, timestamped by the launch itself when the site is timed
template <typename Kern, typename... Args>
static void launch_k(const ScopedTimer& t, Kern kern, dim3 grid, hipStream_t s, Args... args) {
    if (t.active && t.by_launch) hipExtLaunchKernelGGL(kern, grid, dim3(64 * kMpWaves), 0, s, t.a, t.b, 0, args...);
    else kern<<<grid, 64 * kMpWaves, 0, s>>>(args...);
}

template <int F, int K, int CUT>
static void fwd_inst(const MpGeom& mg, const MpFwd& a, hipStream_t s, const ScopedTimer& t) {
    const dim3 grid(cdiv(mg.n, MpShape<F>::APB));
    if (a.phi_tab) launch_k(t, k_message_fwd<F, K, CUT, true>, grid, s, mg, a);
    else launch_k(t, k_message_fwd<F, K, CUT, false>, grid, s, mg, a);
}

template <int F, int K, int CUT, bool L0>
static void bwd_inst_l(const MpGeom& mg, const MpBwd& a, bool geo, bool wgrad, hipStream_t s,
                       const ScopedTimer& t) {
    dim3 grid(cdiv(mg.n, MpShape<F>::APB));
    if constexpr (CUT == 1 && F <= 64) {
        // filter weight adjoints exist for the NC embedding only
        if (wgrad) {
            if (geo) launch_k(t, k_message_bwd<F, K, CUT, true, true, L0>, grid, s, mg, a);
            else launch_k(t, k_message_bwd<F, K, CUT, false, true, L0>, grid, s, mg, a);
            return;
        }
    } else {
        if (wgrad) {
            set_error("filter weight adjoints are only available for the NC embedding");
            throw Fail{NNP_EINVAL};
        }
    }
    if (geo) launch_k(t, k_message_bwd<F, K, CUT, true, false, L0>, grid, s, mg, a);
    else launch_k(t, k_message_bwd<F, K, CUT, false, false, L0>, grid, s, mg, a);
}

template <int F, int K, int CUT>
static void bwd_inst(const MpGeom& mg, const MpBwd& a, bool geo, bool wgrad, hipStream_t s, const ScopedTimer& t) {
    if (a.phi_tab) bwd_inst_l<F, K, CUT, true>(mg, a, geo, wgrad, s, t);
    else bwd_inst_l<F, K, CUT, false>(mg, a, geo, wgrad, s, t);
}

int mp_blocks(int n, int F) {
    const int G = F >= 64 ? 64 : F;
    return cdiv(n, kMpWaves / (F / G) * (64 / G));
}

// The matrix-core kernels serve the shapes they cover unless the vector
// kernels were selected (nnp_set_message_kernels).
static std::atomic<int> g_mp_mode{NNP_MP_AUTO};
static bool mx_enabled() { return g_mp_mode.load(std::memory_order_relaxed) != NNP_MP_VECTOR; }
bool message_mx_active(int F, int K, int cut) { return message_mx_shape(F, K, cut) && mx_enabled(); }
bool species_sum_active() { return g_mp_mode.load(std::memory_order_relaxed) == NNP_MP_AUTO; }

#define NNP_DISPATCH_MP(F_, K_, CUT_, CALL)                                          \
    if (F == F_ && K == K_ && cut == CUT_) { CALL; NNP_LAUNCH_CHECK(); return; }

void launch_message_fwd(int F, int K, int cut, const MpGeom& mg, const MpFwd& a, hipStream_t s) {
    if (mg.n <= 0) return;
    ScopedTimer timer(cut == 0 ? "message_fwd" : "nc_message_fwd", s, true);
    if (mg.ecnt && a.mx_scale && message_mx_active(F, K, cut)) {
        launch_message_fwd_mx(mg, a, s, timer);
        NNP_LAUNCH_CHECK();
        return;
    }
    NNP_DISPATCH_MP(128, 16, 0, (fwd_inst<128, 16, 0>(mg, a, s, timer)));
    NNP_DISPATCH_MP(64, 16, 0, (fwd_inst<64, 16, 0>(mg, a, s, timer)));
    NNP_DISPATCH_MP(32, 16, 0, (fwd_inst<32, 16, 0>(mg, a, s, timer)));
    NNP_DISPATCH_MP(16, 16, 0, (fwd_inst<16, 16, 0>(mg, a, s, timer)));
    NNP_DISPATCH_MP(32, 8, 1, (fwd_inst<32, 8, 1>(mg, a, s, timer)));
    NNP_DISPATCH_MP(16, 8, 1, (fwd_inst<16, 8, 1>(mg, a, s, timer)));
    NNP_DISPATCH_MP(64, 8, 1, (fwd_inst<64, 8, 1>(mg, a, s, timer)));
    NNP_DISPATCH_MP(8, 16, 0, (fwd_inst<8, 16, 0>(mg, a, s, timer)));
    NNP_DISPATCH_MP(8, 8, 1, (fwd_inst<8, 8, 1>(mg, a, s, timer)));
    set_error("unsupported message-passing shape");
    throw Fail{NNP_EINVAL};
}

void launch_message_bwd(int F, int K, int cut, const MpGeom& mg, const MpBwd& a, bool geo, bool wgrad,
                        hipStream_t s) {
    if (mg.n <= 0) return;
    ScopedTimer timer(cut == 0 ? "message_bwd" : "nc_message_bwd", s, true);
    if (geo && !wgrad && mg.ecnt && a.mx_scale && message_mx_active(F, K, cut)) {
        launch_message_bwd_mx(mg, a, s, timer);
        NNP_LAUNCH_CHECK();
        return;
    }
    NNP_DISPATCH_MP(128, 16, 0, (bwd_inst<128, 16, 0>(mg, a, geo, wgrad, s, timer)));
    NNP_DISPATCH_MP(64, 16, 0, (bwd_inst<64, 16, 0>(mg, a, geo, wgrad, s, timer)));
    NNP_DISPATCH_MP(32, 16, 0, (bwd_inst<32, 16, 0>(mg, a, geo, wgrad, s, timer)));
    NNP_DISPATCH_MP(16, 16, 0, (bwd_inst<16, 16, 0>(mg, a, geo, wgrad, s, timer)));
    NNP_DISPATCH_MP(32, 8, 1, (bwd_inst<32, 8, 1>(mg, a, geo, wgrad, s, timer)));
    NNP_DISPATCH_MP(16, 8, 1, (bwd_inst<16, 8, 1>(mg, a, geo, wgrad, s, timer)));
    NNP_DISPATCH_MP(64, 8, 1, (bwd_inst<64, 8, 1>(mg, a, geo, wgrad, s, timer)));
    NNP_DISPATCH_MP(8, 16, 0, (bwd_inst<8, 16, 0>(mg, a, geo, wgrad, s, timer)));
    NNP_DISPATCH_MP(8, 8, 1, (bwd_inst<8, 8, 1>(mg, a, geo, wgrad, s, timer)));
    set_error("unsupported message-passing shape");
    throw Fail{NNP_EINVAL};
}


}  // namespace nnp

extern "C" nnp_status nnp_set_message_kernels(int32_t mode) {
    if (mode != NNP_MP_AUTO && mode != NNP_MP_VECTOR && mode != NNP_MP_EDGE) return NNP_EINVAL;
    nnp::g_mp_mode.store(mode, std::memory_order_relaxed);
    return NNP_OK;
}
