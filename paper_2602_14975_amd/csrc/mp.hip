// Edge kernels of the embedding block: the message step and its reverse.
//
// Layout: one atom per group of G = min(F, 64) lanes (64 / G atoms per
// wavefront), each lane owning F / G feature columns.  Per-atom feature rows
// are [n][F] (s), [n][3][F] (v) and [n][3F] (phi = [a|b|c] channels), so the
// lanes of a group read a neighbour's row with unit stride.
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
// Reverse, owner-computes (atom o gathers everything that reaches it, no
// atomics, fixed order): for each neighbour n of o,
//   (A) o receives from n: g_w = dL/dw of the message n -> o, which gives the
//       edge's position gradient dL/dr_on = d u + (g_u - (g_u.u) u) / r,
//       d = sum_f g_w . dw/dr, and (NC only) the filter weight adjoints;
//   (B) o sends to n: the adjoints of phi_o and v_o from n's message adjoints.
// Forces are assembled afterwards as F_o = sum_e (g_e - g_rev(e)).
#include "common.h"
#include "kernels.h"

namespace nnp {

constexpr int kMpWaves = 4;

template <int K>
struct EdgeSlot {
    float ef[K];    // e_k(r) f(r)
    float def[K];   // d/dr [e_k(r) f(r)]
    float fc, dfc;  // f(r), f'(r)
    float u[3];
    float r;
    int j, e;
};

// Radial values of one edge (float64 Chebyshev recurrence for sin(k theta)).
template <int K, int CUT, bool DERIV>
__device__ __forceinline__ void radial(double r, const MpGeom& mg, float* ef, float* def, float& fc, float& dfc) {
    const double rc = mg.rc;
    const double theta = M_PI * r / rc;
    double sn, cs;
    sincos(theta, &sn, &cs);
    double f, df;
    if (CUT == 0) {
        f = 0.5 * (cs + 1.0);
        df = -0.5 * sn * M_PI / rc;
    } else {
        const double d = r / rc;
        const double d2 = d * d, d4 = d2 * d2, d5 = d4 * d;
        f = 1.0 - 21.0 * d5 + 35.0 * d5 * d - 15.0 * d5 * d2;
        df = (-105.0 * d4 + 210.0 * d5 - 105.0 * d5 * d) / rc;  // -p(p+1)(p+2)/2 d^4 (1-d)^2 / rc
    }
    const double norm = mg.bessel_norm;
    const double inv_r = 1.0 / r;
    double s_prev = 0.0, s_cur = sn;                 // sin(0), sin(theta)
    double c_prev = 1.0, c_cur = cs;                 // cos(0), cos(theta)
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        const double ek = norm * s_cur * inv_r;
        ef[k - 1] = float(ek * f);
        if (DERIV) {
            // d/dr [sin(k pi r/rc)/r] = (k pi/rc) cos(k theta)/r - sin(k theta)/r^2
            const double dek = norm * ((double(k) * M_PI / rc) * c_cur * inv_r - s_cur * inv_r * inv_r);
            def[k - 1] = float(dek * f + ek * df);
        }
        const double s_next = 2.0 * cs * s_cur - s_prev;
        const double c_next = 2.0 * cs * c_cur - c_prev;
        s_prev = s_cur; s_cur = s_next;
        c_prev = c_cur; c_cur = c_next;
    }
    fc = float(f);
    dfc = float(df);
}

// Stages one batch of edges of atom i (lanes l of its group) into LDS.
// Returns the number of surviving edges of this group in `cnt`.
template <int G, int K, int CUT, bool DERIV>
__device__ __forceinline__ int stage_batch(const MpGeom& mg, int i, bool active, int e, int e_end, int l, int g,
                                           double xi, double yi, double zi, double L, double inv,
                                           EdgeSlot<K>* slots) {
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
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        const double r = sqrt(r2);
        EdgeSlot<K>& s = slots[pre];
        radial<K, CUT, DERIV>(r, mg, s.ef, s.def, s.fc, s.dfc);
        s.u[0] = float(dx / r);
        s.u[1] = float(dy / r);
        s.u[2] = float(dz / r);
        s.r = float(r);
        s.j = j;
        s.e = e;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return __popcll(mine);
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <int F, int K, int CUT>
__global__ void __launch_bounds__(64 * kMpWaves)
k_message_fwd(MpGeom mg, MpFwd a) {
    constexpr int G = F >= 64 ? 64 : F;
    constexpr int FPL = F / G;
    constexpr int APW = 64 / G;
    __shared__ EdgeSlot<K> slots_all[kMpWaves][APW][G];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane / G, l = lane % G;
    const int i = (blockIdx.x * kMpWaves + w) * APW + g;
    const bool active = i < mg.n;
    const int n = mg.n;
    EdgeSlot<K>* slots = slots_all[w][g];

    float wr[3][FPL][K], bb[3][FPL];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < FPL; ++q) {
            const int row = p * F + l + q * G;
#pragma unroll
            for (int k = 0; k < K; ++k) wr[p][q][k] = a.Wr[row * K + k];
            bb[p][q] = a.br[row];
        }
    float sacc[FPL] = {}, vacc[3][FPL] = {};
    int start = 0, end = 0;
    double xi = 0, yi = 0, zi = 0, L = 1, inv = 1;
    if (active) {
        start = mg.off[i];
        end = mg.off[i + 1];
        mg.geom.get(i, L, inv);
        xi = mg.pos[i]; yi = mg.pos[n + i]; zi = mg.pos[2 * n + i];
    }
    for (int base = 0; __ballot(start + base < end) != 0ull; base += G) {
        const int cnt = stage_batch<G, K, CUT, false>(mg, i, active, start + base + l, end, l, g, xi, yi, zi, L,
                                                       inv, slots);
        for (int t = 0; t < cnt; ++t) {
            const EdgeSlot<K>& s = slots[t];
            const int j = s.j;
            const float* phj = a.phi + int64_t(j) * 3 * F;
            const float* vj = a.v_in + int64_t(j) * 3 * F;
#pragma unroll
            for (int q = 0; q < FPL; ++q) {
                const int f = l + q * G;
                float wa = bb[0][q] * s.fc, wb = bb[1][q] * s.fc, wc = bb[2][q] * s.fc;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    wa = fmaf(wr[0][q][k], s.ef[k], wa);
                    wb = fmaf(wr[1][q][k], s.ef[k], wb);
                    wc = fmaf(wr[2][q][k], s.ef[k], wc);
                }
                const float pa = phj[f], pb = phj[F + f] * wb, pc = phj[2 * F + f] * wc;
                sacc[q] = fmaf(pa, wa, sacc[q]);
#pragma unroll
                for (int al = 0; al < 3; ++al) vacc[al][q] += pb * vj[al * F + f] + s.u[al] * pc;
            }
        }
        wave_sync_lds();
    }
    if (active) {
#pragma unroll
        for (int q = 0; q < FPL; ++q) {
            const int f = l + q * G;
            a.s_out[int64_t(i) * F + f] = a.s_in[int64_t(i) * F + f] + sacc[q];
#pragma unroll
            for (int al = 0; al < 3; ++al) {
                const int64_t idx = (int64_t(i) * 3 + al) * F + f;
                a.v_out[idx] = a.v_in[idx] + vacc[al][q];
            }
        }
    }
}

template <int F, int K, int CUT, bool GEO, bool WGRAD>
__global__ void __launch_bounds__(64 * kMpWaves)
k_message_bwd(MpGeom mg, MpBwd a) {
    constexpr int G = F >= 64 ? 64 : F;
    constexpr int FPL = F / G;
    constexpr int APW = 64 / G;
    __shared__ EdgeSlot<K> slots_all[kMpWaves][APW][G];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane / G, l = lane % G;
    const int i = (blockIdx.x * kMpWaves + w) * APW + g;
    const bool active = i < mg.n;
    const int n = mg.n;
    EdgeSlot<K>* slots = slots_all[w][g];

    float wr[3][FPL][K], bb[3][FPL];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < FPL; ++q) {
            const int row = p * F + l + q * G;
#pragma unroll
            for (int k = 0; k < K; ++k) wr[p][q][k] = a.Wr[row * K + k];
            bb[p][q] = a.br[row];
        }
    // own data of atom i (owner)
    float ph_o[3][FPL] = {}, v_o[3][FPL] = {}, gs_o[FPL] = {}, gv_o[3][FPL] = {};
    float gph[3][FPL] = {}, gvacc[3][FPL] = {};
    float gwr[WGRAD ? 3 : 1][WGRAD ? FPL : 1][WGRAD ? K : 1] = {};
    float gbr[WGRAD ? 3 : 1][WGRAD ? FPL : 1] = {};
    int start = 0, end = 0;
    double xi = 0, yi = 0, zi = 0, L = 1, inv = 1;
    if (active) {
        start = mg.off[i];
        end = mg.off[i + 1];
        mg.geom.get(i, L, inv);
        xi = mg.pos[i]; yi = mg.pos[n + i]; zi = mg.pos[2 * n + i];
#pragma unroll
        for (int q = 0; q < FPL; ++q) {
            const int f = l + q * G;
#pragma unroll
            for (int p = 0; p < 3; ++p) ph_o[p][q] = a.phi[int64_t(i) * 3 * F + p * F + f];
#pragma unroll
            for (int al = 0; al < 3; ++al) {
                v_o[al][q] = a.v_in[(int64_t(i) * 3 + al) * F + f];
                gv_o[al][q] = a.gvm[(int64_t(i) * 3 + al) * F + f];
            }
            gs_o[q] = a.gsm[int64_t(i) * F + f];
        }
    }
    for (int base = 0; __ballot(start + base < end) != 0ull; base += G) {
        const int cnt = stage_batch<G, K, CUT, GEO>(mg, i, active, start + base + l, end, l, g, xi, yi, zi, L,
                                                     inv, slots);
        for (int t = 0; t < cnt; ++t) {
            const EdgeSlot<K>& s = slots[t];
            const int j = s.j;
            const float* phj = a.phi + int64_t(j) * 3 * F;
            const float* vj = a.v_in + int64_t(j) * 3 * F;
            const float* gvj = a.gvm + int64_t(j) * 3 * F;
            const float gsj_dummy = 0.f;
            (void)gsj_dummy;
            float dr = 0.f, gu0 = 0.f, gu1 = 0.f, gu2 = 0.f;
#pragma unroll
            for (int q = 0; q < FPL; ++q) {
                const int f = l + q * G;
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
                const float pa = phj[f], pb = phj[F + f], pc = phj[2 * F + f];
                const float vj0 = vj[f], vj1 = vj[F + f], vj2 = vj[2 * F + f];
                const float gvj0 = gvj[f], gvj1 = gvj[F + f], gvj2 = gvj[2 * F + f];
                const float gsj = a.gsm[int64_t(j) * F + f];
                // (A) o receives from j
                const float gva = gv_o[0][q] * vj0 + gv_o[1][q] * vj1 + gv_o[2][q] * vj2;
                const float gvu = gv_o[0][q] * s.u[0] + gv_o[1][q] * s.u[1] + gv_o[2][q] * s.u[2];
                const float gwa = gs_o[q] * pa;
                const float gwb = pb * gva;
                const float gwc = pc * gvu;
                if (GEO) {
                    dr += gwa * dw[0] + gwb * dw[1] + gwc * dw[2];
                    const float pcw = pc * w[2];
                    gu0 = fmaf(gv_o[0][q], pcw, gu0);
                    gu1 = fmaf(gv_o[1][q], pcw, gu1);
                    gu2 = fmaf(gv_o[2][q], pcw, gu2);
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
                // (B) o sends to j (unit vector of that edge is -u)
                gph[0][q] = fmaf(gsj, w[0], gph[0][q]);
                gph[1][q] = fmaf(w[1], gvj0 * v_o[0][q] + gvj1 * v_o[1][q] + gvj2 * v_o[2][q], gph[1][q]);
                gph[2][q] = fmaf(-w[2], gvj0 * s.u[0] + gvj1 * s.u[1] + gvj2 * s.u[2], gph[2][q]);
                const float wbp = w[1] * ph_o[1][q];
                gvacc[0][q] = fmaf(gvj0, wbp, gvacc[0][q]);
                gvacc[1][q] = fmaf(gvj1, wbp, gvacc[1][q]);
                gvacc[2][q] = fmaf(gvj2, wbp, gvacc[2][q]);
            }
            if (GEO) {
                dr = group_sum<G>(dr);
                gu0 = group_sum<G>(gu0);
                gu1 = group_sum<G>(gu1);
                gu2 = group_sum<G>(gu2);
                if (l == 0) {
                    const float ud = gu0 * s.u[0] + gu1 * s.u[1] + gu2 * s.u[2];
                    const float ir = 1.0f / s.r;
                    float* ge = a.edge_g + int64_t(s.e) * 3;
                    ge[0] += dr * s.u[0] + (gu0 - ud * s.u[0]) * ir;
                    ge[1] += dr * s.u[1] + (gu1 - ud * s.u[1]) * ir;
                    ge[2] += dr * s.u[2] + (gu2 - ud * s.u[2]) * ir;
                }
            }
        }
        wave_sync_lds();
    }
    if (active) {
#pragma unroll
        for (int q = 0; q < FPL; ++q) {
            const int f = l + q * G;
#pragma unroll
            for (int p = 0; p < 3; ++p) a.gphi[int64_t(i) * 3 * F + p * F + f] = gph[p][q];
#pragma unroll
            for (int al = 0; al < 3; ++al) {
                const int64_t idx = (int64_t(i) * 3 + al) * F + f;
                a.gv_in[idx] = gv_o[al][q] + gvacc[al][q];
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
                const int row = p * F + l + q * G;
#pragma unroll
                for (int k = 0; k < K; ++k) red[slot][row * (K + 1) + k] = gwr[p][q][k];
                red[slot][row * (K + 1) + K] = gbr[p][q];
            }
        __syncthreads();
        for (int t = threadIdx.x; t < 3 * F * (K + 1); t += blockDim.x) {
            float sum = 0.f;
            for (int sl = 0; sl < kMpWaves * APW; ++sl) sum += red[sl][t];
            a.wgrad_part[int64_t(blockIdx.x) * 3 * F * (K + 1) + t] = sum;
        }
    }
}

// Forces from per-edge position gradients: F_o = sum_e (g_e - g_rev(e)).
__global__ void k_assemble_forces(int n, const int* __restrict__ off, const int* __restrict__ rev,
                                  const float* __restrict__ g, float* __restrict__ F, int accum) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float fx = 0.f, fy = 0.f, fz = 0.f;
    for (int e = off[i]; e < off[i + 1]; ++e) {
        const int r = rev[e];
        fx += g[3 * e] - g[3 * r];
        fy += g[3 * e + 1] - g[3 * r + 1];
        fz += g[3 * e + 2] - g[3 * r + 2];
    }
    if (accum) {
        F[i] += fx; F[n + i] += fy; F[2 * n + i] += fz;
    } else {
        F[i] = fx; F[n + i] = fy; F[2 * n + i] = fz;
    }
}

// ------------------------------------------------------------------- host --

template <int F, int K, int CUT>
static void fwd_inst(const MpGeom& mg, const MpFwd& a, hipStream_t s) {
    constexpr int APW = 64 / (F >= 64 ? 64 : F);
    int atoms_per_block = kMpWaves * APW;
    k_message_fwd<F, K, CUT><<<cdiv(mg.n, atoms_per_block), 64 * kMpWaves, 0, s>>>(mg, a);
}

template <int F, int K, int CUT>
static void bwd_inst(const MpGeom& mg, const MpBwd& a, bool geo, bool wgrad, hipStream_t s) {
    constexpr int APW = 64 / (F >= 64 ? 64 : F);
    int atoms_per_block = kMpWaves * APW;
    dim3 grid(cdiv(mg.n, atoms_per_block));
    if constexpr (CUT == 1) {
        // filter weight adjoints exist for the NC embedding only
        if (wgrad) {
            if (geo) k_message_bwd<F, K, CUT, true, true><<<grid, 64 * kMpWaves, 0, s>>>(mg, a);
            else k_message_bwd<F, K, CUT, false, true><<<grid, 64 * kMpWaves, 0, s>>>(mg, a);
            return;
        }
    } else {
        if (wgrad) {
            set_error("filter weight adjoints are only available for the NC embedding");
            throw Fail{NNP_EINVAL};
        }
    }
    if (geo) k_message_bwd<F, K, CUT, true, false><<<grid, 64 * kMpWaves, 0, s>>>(mg, a);
    else k_message_bwd<F, K, CUT, false, false><<<grid, 64 * kMpWaves, 0, s>>>(mg, a);
}

int mp_blocks(int n, int F) {
    int G = F >= 64 ? 64 : F;
    return cdiv(n, kMpWaves * (64 / G));
}

#define NNP_DISPATCH_MP(F_, K_, CUT_, CALL)                                          \
    if (F == F_ && K == K_ && cut == CUT_) { CALL; NNP_LAUNCH_CHECK(); return; }

void launch_message_fwd(int F, int K, int cut, const MpGeom& mg, const MpFwd& a, hipStream_t s) {
    if (mg.n <= 0) return;
    ScopedTimer timer(cut == 0 ? "message_fwd" : "nc_message_fwd", s);
    NNP_DISPATCH_MP(128, 16, 0, (fwd_inst<128, 16, 0>(mg, a, s)));
    NNP_DISPATCH_MP(64, 16, 0, (fwd_inst<64, 16, 0>(mg, a, s)));
    NNP_DISPATCH_MP(32, 16, 0, (fwd_inst<32, 16, 0>(mg, a, s)));
    NNP_DISPATCH_MP(16, 16, 0, (fwd_inst<16, 16, 0>(mg, a, s)));
    NNP_DISPATCH_MP(32, 8, 1, (fwd_inst<32, 8, 1>(mg, a, s)));
    NNP_DISPATCH_MP(16, 8, 1, (fwd_inst<16, 8, 1>(mg, a, s)));
    NNP_DISPATCH_MP(64, 8, 1, (fwd_inst<64, 8, 1>(mg, a, s)));
    NNP_DISPATCH_MP(8, 16, 0, (fwd_inst<8, 16, 0>(mg, a, s)));
    NNP_DISPATCH_MP(8, 8, 1, (fwd_inst<8, 8, 1>(mg, a, s)));
    set_error("unsupported message-passing shape");
    throw Fail{NNP_EINVAL};
}

void launch_message_bwd(int F, int K, int cut, const MpGeom& mg, const MpBwd& a, bool geo, bool wgrad,
                        hipStream_t s) {
    if (mg.n <= 0) return;
    ScopedTimer timer(cut == 0 ? "message_bwd" : "nc_message_bwd", s);
    NNP_DISPATCH_MP(128, 16, 0, (bwd_inst<128, 16, 0>(mg, a, geo, wgrad, s)));
    NNP_DISPATCH_MP(64, 16, 0, (bwd_inst<64, 16, 0>(mg, a, geo, wgrad, s)));
    NNP_DISPATCH_MP(32, 16, 0, (bwd_inst<32, 16, 0>(mg, a, geo, wgrad, s)));
    NNP_DISPATCH_MP(16, 16, 0, (bwd_inst<16, 16, 0>(mg, a, geo, wgrad, s)));
    NNP_DISPATCH_MP(32, 8, 1, (bwd_inst<32, 8, 1>(mg, a, geo, wgrad, s)));
    NNP_DISPATCH_MP(16, 8, 1, (bwd_inst<16, 8, 1>(mg, a, geo, wgrad, s)));
    NNP_DISPATCH_MP(64, 8, 1, (bwd_inst<64, 8, 1>(mg, a, geo, wgrad, s)));
    NNP_DISPATCH_MP(8, 16, 0, (bwd_inst<8, 16, 0>(mg, a, geo, wgrad, s)));
    NNP_DISPATCH_MP(8, 8, 1, (bwd_inst<8, 8, 1>(mg, a, geo, wgrad, s)));
    set_error("unsupported message-passing shape");
    throw Fail{NNP_EINVAL};
}

void launch_assemble_forces(int n, const int* off, const int* rev, const float* g, float* F, bool accum,
                            hipStream_t s) {
    k_assemble_forces<<<cdiv(n, 256), 256, 0, s>>>(n, off, rev, g, F, accum);
    NNP_LAUNCH_CHECK();
}

}  // namespace nnp
