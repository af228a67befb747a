// First layer of the conservative message step, summed by neighbour species.
//
// In the first layer a neighbour enters only through the features of its
// species, phi_p[t_j] (the species table of the first perceptron), the
// vector input is zero, and the radial filter is linear in the basis
// B(r) = (e_0 f, ..., e_{K-1} f, f): w_p(r)[f] = sum_k W'_p[f][k] B_k(r), with
// W'_p = [Wr_p | br_p] (paper, Methods: message and radial filter).  So the
// messages of atom i depend on its edges only through per-species sums of
// the basis,
//   E_i[S][k] = sum_{j: t_j = S} B_k(r_ij),   U_i[S][a][k] = sum_{j: t_j = S} u_ij[a] B_k(r_ij),
//   s_i = emb[t_i] + sum_{S,k} T_0[:, (S, k)] E_i[S][k],   v_i[a] = sum_{S,k} T_2[:, (S, k)] U_i[S][a][k],
// with the tables T_p[f][(S, k)] = phi_p[S][f] W'_p[f][k] (functions of the
// weights only).  In reverse, every feature sum of the per-edge adjoint
// turns into a sum over k, with per-atom tables
//   P_0[x][(S, k)] = sum_f gs_x[f] T_0[f][(S, k)],   P_2[x][a][(S, k)] = sum_f gv_x[a][f] T_2[f][(S, k)],
// and the force share of edge (o, n) on its owner o (both messages of the
// pair, n -> o and o -> n, depend on r_on; the unit vector of the vector
// message contributes the term normal to u):
//   dr  = sum_k (P_0[o][t_n] + P_0[n][t_o])_k B'_k + sum_a u_a sum_k (P_2[o][a][t_n] - P_2[n][a][t_o])_k B'_k,
//   Q_a = sum_k (P_2[o][a][t_n] - P_2[n][a][t_o])_k B_k,
//   F_o += dr u + (Q - (Q . u) u) / r.
// Per edge this reads 4 (K + 1) numbers of the neighbour instead of 4 F
// feature values, and the per-feature work moves into four dense products
// per evaluation (two launches: [s; v] and [P_0; P_2] each take one, the
// row tiles past n multiplying by the second table).  The edges are those of the edge preparation (records and
// split radial values, see mp_mx.hip), which also forms the forward sums E
// and U in the same pass; this file holds the tables and the reverse.
//
// Slot layout of a species: KP = K + 4 numbers, k < K the basis, K the
// cutoff (bias column), K + 1 the species indicator (forward: T_0 holds the
// embedding there, so the product also adds emb[t_i]), the rest zero.  Rows
// of the edge sums have ep slots (128 or 256, the depth of the dense
// product that reads them), rows of P have pp (S KP rounded up to 32, its
// width); the slots past S KP are zero.
#include <hip/hip_ext.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace nnp {

namespace {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));

constexpr int kSpK = 16;             // basis functions (the matrix-core message shape)
constexpr int kSpKP = kSpK + 4;      // slots per species
constexpr int kSpMaxSpecies = 8;
constexpr int kSpWaves = 4;          // wavefronts (atoms) per block

// the 16 radial values (or derivatives) of an edge from its FP16 pieces
__device__ __forceinline__ void unsplit16(const uint4* hi, const uint4* lo, float* x) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const half8_t h = __builtin_bit_cast(half8_t, hi[q]), l = __builtin_bit_cast(half8_t, lo[q]);
#pragma unroll
        for (int e = 0; e < 8; ++e) x[8 * q + e] = static_cast<float>(h[e]) + static_cast<float>(l[e]);
    }
}

// Entry (c, f, slot) of the tables: T_c for c = 0 (scalar channel, phi_0)
// and c = 1 (vector channel, phi_2); with `indicator`, emb in the indicator
// slots of T_0.
__device__ __forceinline__ float sp_entry(int F, int S, int c, int f, int slot, bool indicator,
                                          const float* __restrict__ Wr, const float* __restrict__ br,
                                          const float* __restrict__ phi, const float* __restrict__ emb) {
    constexpr int K = kSpK, KP = kSpKP;
    if (slot >= S * KP) return 0.f;
    const int sp = slot / KP, k = slot % KP;
    const int p = c == 0 ? 0 : 2;
    if (k == K + 1) return (indicator && c == 0) ? emb[sp * F + f] : 0.f;
    if (k > K + 1) return 0.f;
    const float ph = phi[sp * 3 * F + p * F + f];
    return k < K ? ph * Wr[(p * F + f) * K + k] : ph * br[p * F + f];
}

// T[c][f][ep] (forward products, with the embedding) and TT[c][pp][f]
// (reverse products).
__global__ void k_sp_tables(int F, int S, int pp, int ep, const float* __restrict__ Wr, const float* __restrict__ br,
                            const float* __restrict__ phi, const float* __restrict__ emb, float* __restrict__ T,
                            float* __restrict__ TT) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nT = int64_t(2) * F * ep, nTT = int64_t(2) * pp * F;
    if (t < nT) {
        const int c = int(t / (int64_t(F) * ep));
        const int rem = int(t % (int64_t(F) * ep));
        T[t] = sp_entry(F, S, c, rem / ep, rem % ep, true, Wr, br, phi, emb);
    }
    if (t < nTT) {
        const int c = int(t / (int64_t(pp) * F));
        const int rem = int(t % (int64_t(pp) * F));
        TT[t] = sp_entry(F, S, c, rem % F, rem / F, false, Wr, br, phi, emb);
    }
}

// Reverse: one wavefront per owner atom, one lane per edge (64 at a time);
// the owner's P rows in LDS, the neighbour's rows of the owner's species
// gathered as 16-byte pieces.  The owner's force share (and, with VIR, the
// virial share r . F_pair / 2) is summed over the lanes in a fixed order.
template <bool VIR>
__global__ void __launch_bounds__(64 * kSpWaves) k_sp_bwd(MpGeom mg, int S, int pp, const float* __restrict__ P0,
                                                        const float* __restrict__ P2, float* __restrict__ force,
                                                        int accum, float* __restrict__ vir) {
    constexpr int K = kSpK, KP = kSpKP, NQ = KP / 4;
    __shared__ __align__(16) float po[kSpWaves][4 * kSpMaxSpecies * KP];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = xcd_block(blockIdx.x, gridDim.x) * kSpWaves + w;
    if (i >= mg.n) return;  // whole wavefronts; no block barriers below
    const int n = mg.n, NS = S * KP;
    const int start = mg.off[i], cnt = mg.ecnt[i];
    // the first 64 edges' records and radial pieces, requested before the
    // owner's rows are staged
    EdgeRec rec0{};
    uint4 pc0[8];
    if (lane < cnt) {
        rec0 = mg.erec[start + lane];
        const uint4* hp = mg.ehalf + int64_t(start + lane) * 8;
#pragma unroll
        for (int q = 0; q < 8; ++q) pc0[q] = hp[q];
    }
    float* own = po[w];
    {
        // rows P_0[i], then P_2[3 i], P_2[3 i + 1], P_2[3 i + 2] (contiguous),
        // as 16-byte pieces, every load issued before the first store
        constexpr int U = (kSpMaxSpecies * KP + 63) / 64;  // pieces per lane (4 NS / 4 <= 64 U)
        // (the used S KP slots of each row, NS / 4 pieces)
        const int NQ4 = NS / 4, PQ = pp / 4;
        const float4* s0 = reinterpret_cast<const float4*>(P0 + int64_t(i) * pp);
        const float4* s2 = reinterpret_cast<const float4*>(P2 + int64_t(i) * 3 * pp);
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = lane + 64 * u;
            const int r = t / NQ4, q = t % NQ4;
            v[u] = t < NQ4 ? s0[q] : t < 4 * NQ4 ? s2[(r - 1) * PQ + q] : float4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = lane + 64 * u;
            if (t < 4 * NQ4) reinterpret_cast<float4*>(own)[t] = v[u];
        }
    }
    wave_sync_lds();
    const int to = min(max(mg.species[i], 0), S - 1);
    float fx = 0.f, fy = 0.f, fz = 0.f, vr = 0.f;
    for (int base = 0; base < cnt; base += 64) {
        const int e = base + lane;
        if (e >= cnt) continue;
        const int p = start + e;
        EdgeRec rec;
        uint4 pc[8];
        if (base == 0) {
            rec = rec0;
#pragma unroll
            for (int q = 0; q < 8; ++q) pc[q] = pc0[q];
        } else {
            rec = mg.erec[p];
            const uint4* hp = mg.ehalf + int64_t(p) * 8;
#pragma unroll
            for (int q = 0; q < 8; ++q) pc[q] = hp[q];
        }
        const float4* nb0 = reinterpret_cast<const float4*>(P0 + int64_t(rec.j) * pp + to * KP);
        const float4* nb2 = reinterpret_cast<const float4*>(P2 + int64_t(rec.j) * 3 * pp + to * KP);
        float4 pn[4][NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) pn[0][q] = nb0[q];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int q = 0; q < NQ; ++q) pn[1 + a][q] = nb2[a * (pp / 4) + q];
        const uint4 bh[2] = {pc[0], pc[1]}, bl[2] = {pc[2], pc[3]}, dh[2] = {pc[4], pc[5]}, dl[2] = {pc[6], pc[7]};
        float B[K + 1], D[K + 1];
        unsplit16(bh, bl, B);
        unsplit16(dh, dl, D);
        B[K] = rec.fc;
        D[K] = rec.dfc;
        const int tn = min(max(rec.t, 0), S - 1);
        const float* o0 = own + tn * KP;
        const float u[3] = {rec.u[0], rec.u[1], rec.u[2]};
        float dr = 0.f;
        {
            const float* pn0 = reinterpret_cast<const float*>(pn[0]);
#pragma unroll
            for (int k = 0; k <= K; ++k) dr = fmaf(o0[k] + pn0[k], D[k], dr);
        }
        float Q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float* o2 = own + (1 + a) * NS + tn * KP;
            const float* pn2 = reinterpret_cast<const float*>(pn[1 + a]);
            float g = 0.f, q = 0.f;
#pragma unroll
            for (int k = 0; k <= K; ++k) {
                const float cc = o2[k] - pn2[k];
                g = fmaf(cc, D[k], g);
                q = fmaf(cc, B[k], q);
            }
            dr = fmaf(u[a], g, dr);
            Q[a] = q;
        }
        const float qu = fmaf(Q[2], u[2], fmaf(Q[1], u[1], Q[0] * u[0]));
        const float ir = rec.ir;
        fx += fmaf(dr, u[0], fmaf(-qu, u[0], Q[0]) * ir);
        fy += fmaf(dr, u[1], fmaf(-qu, u[1], Q[1]) * ir);
        fz += fmaf(dr, u[2], fmaf(-qu, u[2], Q[2]) * ir);
        if constexpr (VIR) vr += __fdividef(dr, ir);
    }
    fx = wave_sum(fx);
    fy = wave_sum(fy);
    fz = wave_sum(fz);
    if constexpr (VIR) vr = wave_sum(vr);
    if (lane == 0) {
        const int io = mg.perm ? min(max(mg.perm[i], 0), n - 1) : i;
        float* F3[3] = {force + io, force + n + io, force + 2 * n + io};
        const float fv[3] = {fx, fy, fz};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (accum) *F3[a] += fv[a];
            else *F3[a] = fv[a];
        }
        if constexpr (VIR) {
            if (accum) vir[io] += 0.5f * vr;
            else vir[io] = 0.5f * vr;
        }
    }
}

}  // namespace

void species_sum_pitches(int n_species, int& pp, int& ep) {
    const int used = n_species * kSpKP;
    pp = (used + 31) / 32 * 32;
    ep = used <= 128 ? 128 : 256;
}

bool species_sum_shape(int F, int K, int cut, int n_species) {
    return message_mx_shape(F, K, cut) && K == kSpK && n_species >= 1 && n_species <= kSpMaxSpecies;
}

void launch_sp_tables(int F, int S, const float* Wr, const float* br, const float* phi, const float* emb, float* T,
                      float* TT, hipStream_t s) {
    int pp, ep;
    species_sum_pitches(S, pp, ep);
    const int64_t total = int64_t(2) * F * std::max(pp, ep);
    k_sp_tables<<<cdiv(total, 256), 256, 0, s>>>(F, S, pp, ep, Wr, br, phi, emb, T, TT);
    NNP_LAUNCH_CHECK();
}

void launch_sp_bwd(const MpGeom& mg, int S, const float* P0, const float* P2, float* force, bool accum, float* vir,
                   hipStream_t s) {
    if (mg.n <= 0) return;
    int pp, ep;
    species_sum_pitches(S, pp, ep);
    ScopedTimer t("message_bwd_first", s, true);
    const dim3 grid(cdiv(mg.n, kSpWaves)), block(64 * kSpWaves);
    auto go = [&](auto kern) {
        if (t.active && t.by_launch)
            hipExtLaunchKernelGGL(kern, grid, block, 0, s, t.a, t.b, 0, mg, S, pp, P0, P2, force, int(accum), vir);
        else kern<<<grid, block, 0, s>>>(mg, S, pp, P0, P2, force, int(accum), vir);
    };
    if (vir) go(k_sp_bwd<true>);
    else go(k_sp_bwd<false>);
    NNP_LAUNCH_CHECK();
}

}  // namespace nnp
