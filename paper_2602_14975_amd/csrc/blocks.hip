// Per-atom elementwise pieces of the embedding block and the readout, and
// the non-conservative pair head (paper, Methods: q_ih, k_ih, c_ijh, F_ij,
// F_i = sum_j (F_ij - F_ji)).  The dense contractions around them run in
// gemm.hip; the edge loops of the embedding in mp.hip.
#include <algorithm>
#include <atomic>

#include "common.h"
#include "kernels.h"
#include "mp_edge.h"

namespace nnp {

// s0[i] = emb[t_i]; v0[i] = 0
__global__ void k_embed(int n, int F, int S, const int* __restrict__ species, const float* __restrict__ emb,
                        float* __restrict__ s, float* __restrict__ v) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n) * F) return;
    int i = int(t / F), f = int(t % F);
    const int sp = min(max(species[i], 0), S - 1);  // out-of-range species read row 0 or S-1, never past the table
    s[t] = emb[sp * F + f];
    v[(int64_t(i) * 3 + 0) * F + f] = 0.f;
    v[(int64_t(i) * 3 + 1) * F + f] = 0.f;
    v[(int64_t(i) * 3 + 2) * F + f] = 0.f;
}

// X[i] = [smid_i ; sqrt(sum_al Vv[i][al]^2 + 1e-8)], UV rows [Uv (F) | Vv (F)] per component.
__global__ void k_build_x(int n, int F, const float* __restrict__ smid, const float* __restrict__ UV,
                          float* __restrict__ X) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n) * F) return;
    int i = int(t / F), f = int(t % F);
    float acc = 1e-8f;
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        float vv = UV[(int64_t(i) * 3 + al) * 2 * F + F + f];
        acc = fmaf(vv, vv, acc);
    }
    X[int64_t(i) * 2 * F + f] = smid[t];
    X[int64_t(i) * 2 * F + F + f] = sqrtf(acc);
}

// s_out = smid + p + q * sum_al Uv Vv ; v_out = vmid + o * Uv
__global__ void k_update_combine(int n, int F, const float* __restrict__ smid, const float* __restrict__ vmid,
                                 const float* __restrict__ UV, const float* __restrict__ pqo,
                                 float* __restrict__ s_out, float* __restrict__ v_out) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n) * F) return;
    int i = int(t / F), f = int(t % F);
    const float* h = pqo + int64_t(i) * 3 * F;
    float dot = 0.f, uv[3];
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const float* row = UV + (int64_t(i) * 3 + al) * 2 * F;
        uv[al] = row[f];
        dot = fmaf(row[f], row[F + f], dot);
    }
    s_out[t] = smid[t] + h[f] + h[F + f] * dot;
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        int64_t idx = (int64_t(i) * 3 + al) * F + f;
        v_out[idx] = vmid[idx] + h[2 * F + f] * uv[al];
    }
}

// Reverse of k_update_combine: g_pqo and the Uv/Vv adjoints (the norm path
// of Vv is added by k_norm_bwd).
__global__ void k_update_combine_bwd(int n, int F, const float* __restrict__ UV, const float* __restrict__ pqo,
                                     const float* __restrict__ gs, const float* __restrict__ gv,
                                     float* __restrict__ gpqo, float* __restrict__ gUV) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n) * F) return;
    int i = int(t / F), f = int(t % F);
    const float* h = pqo + int64_t(i) * 3 * F;
    const float q = h[F + f], o = h[2 * F + f];
    const float g = gs[t];
    float dot = 0.f, go = 0.f;
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const float* row = UV + (int64_t(i) * 3 + al) * 2 * F;
        const float u = row[f], vv = row[F + f];
        const float gva = gv ? gv[(int64_t(i) * 3 + al) * F + f] : 0.f;  // nullptr: zero adjoint
        dot = fmaf(u, vv, dot);
        go = fmaf(gva, u, go);
        float* grow = gUV + (int64_t(i) * 3 + al) * 2 * F;
        grow[f] = g * q * vv + gva * o;
        grow[F + f] = g * q * u;
    }
    float* gh = gpqo + int64_t(i) * 3 * F;
    gh[f] = g;
    gh[F + f] = g * dot;
    gh[2 * F + f] = go;
}

// g_smid = gs + gX[:, :F];  gVv[al] += gX[:, F:] * Vv[al] / nrm
__global__ void k_norm_bwd(int n, int F, const float* __restrict__ gs, const float* __restrict__ gX,
                           const float* __restrict__ X, const float* __restrict__ UV, float* __restrict__ gsmid,
                           float* __restrict__ gUV) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n) * F) return;
    int i = int(t / F), f = int(t % F);
    gsmid[t] = gs[t] + gX[int64_t(i) * 2 * F + f];
    const float gn = gX[int64_t(i) * 2 * F + F + f] / X[int64_t(i) * 2 * F + F + f];
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const int64_t idx = (int64_t(i) * 3 + al) * 2 * F + F + f;
        gUV[idx] = fmaf(gn, UV[idx], gUV[idx]);
    }
}

// E_i = wo . z_i + beta[t_i] (z = silu(Wo s + bo) from the GEMM epilogue)
__global__ void k_readout(int n, int F, int S, const float* __restrict__ z, const float* __restrict__ wo,
                          const float* __restrict__ beta, const int* __restrict__ species, float* __restrict__ Ei,
                          const int* __restrict__ perm) {
    int lane = threadIdx.x & 63;
    int i = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (i >= n) return;
    float acc = 0.f;
    for (int f = lane; f < F; f += 64) acc = fmaf(wo[f], z[int64_t(i) * F + f], acc);
    acc = wave_sum(acc);
    if (lane == 0) Ei[perm ? min(max(perm[i], 0), n - 1) : i] = acc + beta[min(max(species[i], 0), S - 1)];
}

// g_ao = wo * silu'(a_o)  (dE/dE_i = 1)
__global__ void k_readout_bwd(int n, int F, const float* __restrict__ ao, const float* __restrict__ wo,
                              float* __restrict__ gao) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n) * F) return;
    gao[t] = wo[t % F] * silu_grad(ao[t]);
}

// Per-replica float64 sums in a fixed order (one block per replica).
__global__ void __launch_bounds__(256) k_rep_sum(const int64_t* __restrict__ rep_start, const float* __restrict__ x,
                                                 double* __restrict__ out) {
    __shared__ double red[256];
    int r = blockIdx.x;
    int64_t a0 = rep_start[r], a1 = rep_start[r + 1];
    double s = 0.0;
    int64_t a = a0 + threadIdx.x;
    // eight loads in flight, added in the same order as one at a time
    for (; a + 7 * 256 < a1; a += 8 * 256) {
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = x[a + k * 256];
#pragma unroll
        for (int k = 0; k < 8; ++k) s += double(v[k]);
    }
    for (; a < a1; a += 256) s += double(x[a]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[r] = red[0];
}

// Per-species column sums: out[t][f] = sum over atoms of species t of x[i][f]
// (fixed order), for the adjoints of per-species tables.
__global__ void k_emb_grad(int n, int F, int S, const int* __restrict__ species, const float* __restrict__ gs0,
                           float* __restrict__ gemb) {
    const int t = blockIdx.x;  // species
    for (int f = threadIdx.x; f < F; f += blockDim.x) {
        float acc = 0.f;
        for (int i = 0; i < n; ++i)
            if (species[i] == t) acc += gs0[int64_t(i) * F + f];
        gemb[t * F + f] = acc;
    }
}

// ------------------------------------------------------------- NC head ----
// Per owner atom i (one wavefront), lanes over the CSR entries of its row.
// QK rows: [q (H x n_c) | k (H x n_c)]; Vh rows [n][3][n_l].
constexpr int kNs = 8, kNl = 2, kNc = 8, kH = kNs + kNl;

struct HeadEdge {
    float ef[kNs];  // B_h(r) u(r/rc)
    float u[3];
    float r;
    int j;
};

__device__ __forceinline__ bool head_edge(const MpGeom& mg, int i, int e, double xi, double yi, double zi,
                                          double L, double inv, HeadEdge& he) {
    const int n = mg.n;
    const int j = mg.nbr[e];
    double dx, dy, dz;
    if (!pair_rule(xi, yi, zi, mg.pos[j], mg.pos[n + j], mg.pos[2 * n + j], L, inv, mg.rc2, dx, dy, dz)) return false;
    // radial values in float32 (the pair rule above decides in float64)
    const float r = sqrtf(float((dx * dx + dy * dy) + dz * dz));
    const float ir = 1.f / r;
    float env;
    radial_poly_f32<kNs>(r * float(mg.inv_rc), float(mg.bessel_norm) * ir, he.ef, env);
    he.u[0] = float(dx) * ir;
    he.u[1] = float(dy) * ir;
    he.u[2] = float(dz) * ir;
    he.r = r;
    he.j = j;
    return true;
}

__device__ __forceinline__ void head_coeffs(const float* qa, const float* kb, float* c) {
    const float scale = 0.35355339059327373f;  // 1/sqrt(n_c), n_c = 8
#pragma unroll
    for (int h = 0; h < kH; ++h) {
        const float4 a0 = *reinterpret_cast<const float4*>(qa + h * kNc);
        const float4 a1 = *reinterpret_cast<const float4*>(qa + h * kNc + 4);
        const float4 b0 = *reinterpret_cast<const float4*>(kb + h * kNc);
        const float4 b1 = *reinterpret_cast<const float4*>(kb + h * kNc + 4);
        float acc = a0.x * b0.x;
        acc = fmaf(a0.y, b0.y, acc); acc = fmaf(a0.z, b0.z, acc); acc = fmaf(a0.w, b0.w, acc);
        acc = fmaf(a1.x, b1.x, acc); acc = fmaf(a1.y, b1.y, acc); acc = fmaf(a1.z, b1.z, acc);
        acc = fmaf(a1.w, b1.w, acc);
        c[h] = acc * scale;
    }
}

// S = sum_h c_h B_h(r) u(r/rc) over the n_s Bessel heads in one fixed
// order, ((p0 + p4) + (p2 + p6)) + ((p1 + p5) + (p3 + p7)) with rounded
// products p_h: the order a butterfly over eight lanes produces, so that
// the record kernel below, which spreads the heads over lanes, gives the
// same sums bit for bit.
__device__ __forceinline__ float head_sum(const float* c, const float* ef) {
#pragma clang fp contract(off)  // rounded products: no product may fuse into the sums
    float p[kNs];
#pragma unroll
    for (int h = 0; h < kNs; ++h) p[h] = c[h] * ef[h];
    return ((p[0] + p[4]) + (p[2] + p[6])) + ((p[1] + p[5]) + (p[3] + p[7]));
}

// The contribution of edge (i, j) to F_i: F_ij - F_ji = S_ij D_ij - S_ji D_ji
// with D_ij = u + c_ij,s V_i,0 + c_ij,s+1 V_i,1 and D_ji = -u + c_ji,s V_j,0 +
// c_ji,s+1 V_j,1 (s = n_s), and with VIR its share F_ij . r_ij of the virial
// proxy in out[3].  Vi, Vj: [n_l][3].  Explicit fused operations fix the
// rounding.
template <bool VIR>
__device__ __forceinline__ void head_pair(float Sij, float Sji, float ci8, float ci9, float cj8, float cj9,
                                          const float* u, float r, const float (*Vi)[3], const float (*Vj)[3],
                                          float* out) {
    float fu = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float Dij = fmaf(ci9, Vi[1][a], fmaf(ci8, Vi[0][a], u[a]));
        const float Dji = fmaf(cj9, Vj[1][a], fmaf(cj8, Vj[0][a], -u[a]));
        out[a] = fmaf(Sij, Dij, -(Sji * Dji));
        if (VIR) fu = fmaf(Sij * Dij, u[a], fu);
    }
    out[3] = VIR ? fu * r : 0.f;
}

// A group of G lanes per owner atom (64 / G atoms per wavefront); lanes take
// one CSR entry each.  The contributions of the entries that pass the pair
// rule are compacted (ballot) into LDS and added by the group's first lane
// in row order, so the sum does not depend on how many extra Verlet entries
// the row holds or where batch boundaries fall.
template <int G, bool VIR>
__global__ void __launch_bounds__(256) k_head_fwd(MpGeom mg, const float* __restrict__ QK,
                                                  const float* __restrict__ Vh, float* __restrict__ Fout, int accum,
                                                  float* __restrict__ vir_set, float* __restrict__ vir_add) {
    constexpr int APW = 64 / G;
    // force (and F_ij . r_ij) per staged edge, one 16-byte slot each
    __shared__ __align__(16) float contrib[4][APW][G][4];
    // the owner's q and k rows, read by every lane of its group: in LDS
    __shared__ __align__(16) float qk_s[4][APW][2 * kH * kNc];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int g = lane / G, l = lane % G;
    const int i = (xcd_block(blockIdx.x, gridDim.x) * 4 + w) * APW + g;
    const bool active = i < mg.n;
    const int n = mg.n;
    double L = 1, inv = 1, xi = 0, yi = 0, zi = 0;
    int e0 = 0, e1 = 0;
    float Vi[kNl][3] = {};
    if (active) {
        mg.geom.get(i, L, inv);
        xi = mg.pos[i]; yi = mg.pos[n + i]; zi = mg.pos[2 * n + i];
        e0 = mg.off[i];
        e1 = mg.off[i + 1];
#pragma unroll
        for (int t = l; t < 2 * kH * kNc; t += G) qk_s[w][g][t] = QK[int64_t(i) * 2 * kH * kNc + t];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int h = 0; h < kNl; ++h) Vi[h][a] = Vh[(int64_t(i) * 3 + a) * kNl + h];
    }
    wave_sync_lds();
    const float* qi = qk_s[w][g];
    const float* ki = qi + kH * kNc;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (g * G));
    float fx = 0.f, fy = 0.f, fz = 0.f, vr = 0.f;  // running sums (first lane of the group)
    for (int base = 0; __ballot(e0 + base < e1) != 0ull; base += G) {
        const int e = e0 + base + l;
        HeadEdge he;
        const bool ok = e < e1 && head_edge(mg, i, e, xi, yi, zi, L, inv, he);
        const uint64_t mine = __ballot(ok) & gmask;
        if (ok) {
            const int j = he.j;
            const float* qj = QK + int64_t(j) * 2 * kH * kNc;
            const float* kj = qj + kH * kNc;
            float cij[kH], cji[kH];
            head_coeffs(qi, kj, cij);
            head_coeffs(qj, ki, cji);
            float Vj[kNl][3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int h = 0; h < kNl; ++h) Vj[h][a] = Vh[(int64_t(j) * 3 + a) * kNl + h];
            const int pre = __popcll(mine & ((1ull << lane) - 1ull));
            float c[4];
            head_pair<VIR>(head_sum(cij, he.ef), head_sum(cji, he.ef), cij[kNs], cij[kNs + 1], cji[kNs],
                           cji[kNs + 1], he.u, he.r, Vi, Vj, c);
            *reinterpret_cast<float4*>(&contrib[w][g][pre][0]) = make_float4(c[0], c[1], c[2], c[3]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (l == 0) {
            const int cnt = __popcll(mine);
            for (int t = 0; t < cnt; ++t) {
                const float4 c = *reinterpret_cast<const float4*>(&contrib[w][g][t][0]);
                fx += c.x;
                fy += c.y;
                fz += c.z;
                if constexpr (VIR) vr += c.w;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    if (active && l == 0) {
        const int io = mg.perm ? min(max(mg.perm[i], 0), n - 1) : i;
        if (accum) {
            Fout[io] += fx; Fout[n + io] += fy; Fout[2 * n + io] += fz;
        } else {
            Fout[io] = fx; Fout[n + io] = fy; Fout[2 * n + io] = fz;
        }
        if constexpr (VIR) {
            if (vir_set) vir_set[io] = vr;
            if (vir_add) vir_add[io] += vr;
        }
    }
}

// The same head over the records the NC message step left (edges within the
// cutoff in list order, B_h u, u and r in float32): no pair rule or radial
// values here.  One wavefront per four owner atoms, lanes 16 e .. 16 e + 15
// for owner e, which they walk one edge at a time in record order: lane
// 16 e + h takes head h (h < 10), so that the neighbour's q and k rows are
// read as 32-byte pieces per lane, contiguous across the heads of an edge.
// Everything an edge needs is requested three edges ahead: lanes h < 8 read
// B_h u of the record, lane 8 its u and r and the neighbour's V rows (the
// first 32 neighbours of each owner are read up front, two per lane).  The
// head sums S come from a butterfly over lanes 0..7 (the order of
// head_sum), and lane 8 forms the pair contribution (head_pair) and adds it
// to the owner's sums: the result is the same, bit for bit, as that of the
// kernel above.
template <bool VIR>
__global__ void __launch_bounds__(256) k_head_fwd_rec(int n, const int* __restrict__ off,
                                                      const int* __restrict__ cnt_in, const NcEdge* __restrict__ rec,
                                                      const float* __restrict__ QK, const float* __restrict__ Vh,
                                                      float* __restrict__ Fout, int accum, float* __restrict__ vir_set,
                                                      float* __restrict__ vir_add, const int* __restrict__ perm) {
    constexpr int HC = 2 * kH * kNc;
    const int lane = threadIdx.x & 63;
    const int e = lane >> 4, h = lane & 15;
    const int iw = (xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6)) * 4;
    if (iw >= n) return;  // whole wavefronts
    const int i = iw + e;
    const bool own = i < n;
    const int e0 = own ? off[i] : 0, cnt = own ? cnt_in[i] : 0;
    const int hh = h < kH ? h : 0;
    float qi[kNc] = {}, ki[kNc] = {};
    float Vi[kNl][3] = {};
    if (own) {
        const float4* q4 = reinterpret_cast<const float4*>(QK + int64_t(i) * HC + hh * kNc);
        const float4* k4 = reinterpret_cast<const float4*>(QK + int64_t(i) * HC + (kH + hh) * kNc);
        const float4 a0 = q4[0], a1 = q4[1], b0 = k4[0], b1 = k4[1];
        qi[0] = a0.x; qi[1] = a0.y; qi[2] = a0.z; qi[3] = a0.w; qi[4] = a1.x; qi[5] = a1.y; qi[6] = a1.z; qi[7] = a1.w;
        ki[0] = b0.x; ki[1] = b0.y; ki[2] = b0.z; ki[3] = b0.w; ki[4] = b1.x; ki[5] = b1.y; ki[6] = b1.z; ki[7] = b1.w;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int l = 0; l < kNl; ++l) Vi[l][a] = Vh[(int64_t(i) * 3 + a) * kNl + l];
    }
    // the longest row of the four
    int steps = cnt;
#pragma unroll
    for (int m = 16; m <= 32; m <<= 1) steps = max(steps, __shfl_xor(steps, m, 64));
    const float scale = 0.35355339059327373f;  // 1/sqrt(n_c), n_c = 8
    // q_a . k_b over the channels in the order of head_coeffs
    auto dot8 = [](const float* a, const float4& b0, const float4& b1) {
        float acc = a[0] * b0.x;
        acc = fmaf(a[1], b0.y, acc); acc = fmaf(a[2], b0.z, acc); acc = fmaf(a[3], b0.w, acc);
        acc = fmaf(a[4], b1.x, acc); acc = fmaf(a[5], b1.y, acc); acc = fmaf(a[6], b1.z, acc);
        acc = fmaf(a[7], b1.w, acc);
        return acc;
    };
    auto dot8r = [](const float4& a0, const float4& a1, const float* b) {
        float acc = a0.x * b[0];
        acc = fmaf(a0.y, b[1], acc); acc = fmaf(a0.z, b[2], acc); acc = fmaf(a0.w, b[3], acc);
        acc = fmaf(a1.x, b[4], acc); acc = fmaf(a1.y, b[5], acc); acc = fmaf(a1.z, b[6], acc);
        acc = fmaf(a1.w, b[7], acc);
        return acc;
    };
    // what one lane holds of an edge: its head's q and k rows of the
    // neighbour; B_h u (h < 8); u, r and the neighbour's V (h = 8)
    struct Pre {
        float4 q0, q1, k0, k1;
        float ef, u[3], r;
        float2 vj[3];
    };
    // neighbours of the owner's first 32 edges: lane 16 e + h holds those of
    // edges h and 16 + h
    const int jl0 = h < cnt ? rec[e0 + h].j : 0;
    const int jl1 = 16 + h < cnt ? rec[e0 + 16 + h].j : 0;
    // edge t of this lane's owner (t < cnt); every lane takes part in the shuffles
    auto fetch = [&](int t, Pre& p) {
        const int tt = t & 15;
        const int a0 = __shfl(jl0, 16 * e + tt, 64), a1 = __shfl(jl1, 16 * e + tt, 64);
        if (t >= cnt) return;
        const int j = t < 16 ? a0 : t < 32 ? a1 : rec[e0 + t].j;
        const NcEdge* re = rec + e0 + t;
        if (h < kH) {
            const float4* q4 = reinterpret_cast<const float4*>(QK + int64_t(j) * HC + h * kNc);
            const float4* k4 = reinterpret_cast<const float4*>(QK + int64_t(j) * HC + (kH + h) * kNc);
            p.q0 = q4[0]; p.q1 = q4[1]; p.k0 = k4[0]; p.k1 = k4[1];
        }
        if (h < kNs) p.ef = re->ef[h];
        if (h == kNs) {
            p.u[0] = re->u[0]; p.u[1] = re->u[1]; p.u[2] = re->u[2];
            p.r = re->r;
#pragma unroll
            for (int a = 0; a < 3; ++a) p.vj[a] = *reinterpret_cast<const float2*>(Vh + (int64_t(j) * 3 + a) * kNl);
        }
    };
    float fx = 0.f, fy = 0.f, fz = 0.f, vr = 0.f;  // the owner's sums (lane 16 e + 8)
    // edge t with its operands in `cur`
    auto edge_step = [&](int t, const Pre& cur) {
        float cij = 0.f, cji = 0.f;
        if (h < kH) {
            cij = dot8(qi, cur.k0, cur.k1) * scale;   // q_i . k_j
            cji = dot8r(cur.q0, cur.q1, ki) * scale;  // q_j . k_i
        }
        // S over lanes 0..7 of the owner (butterfly 4, 2, 1; rounded products
        // as in head_sum)
        float pij, pji;
        {
#pragma clang fp contract(off)
            pij = h < kNs ? cij * cur.ef : 0.f;
            pji = h < kNs ? cji * cur.ef : 0.f;
#pragma unroll
            for (int m = 4; m >= 1; m >>= 1) {
                pij += __shfl_xor(pij, m, 64);
                pji += __shfl_xor(pji, m, 64);
            }
        }
        const float Sij = __shfl(pij, 16 * e, 64), Sji = __shfl(pji, 16 * e, 64);
        const float ci9 = __shfl(cij, 16 * e + kNs + 1, 64), cj9 = __shfl(cji, 16 * e + kNs + 1, 64);
        if (h == kNs && t < cnt) {
            const float Vj[kNl][3] = {{cur.vj[0].x, cur.vj[1].x, cur.vj[2].x}, {cur.vj[0].y, cur.vj[1].y, cur.vj[2].y}};
            float c[4];
            head_pair<VIR>(Sij, Sji, cij, ci9, cji, cj9, cur.u, cur.r, Vi, Vj, c);
            fx += c[0];
            fy += c[1];
            fz += c[2];
            if constexpr (VIR) vr += c[3];
        }
    };
    // three edges in flight: the operands of edge t + 3 are requested as
    // soon as edge t is done with its stage
    Pre p0{}, p1{}, p2{};
    fetch(0, p0);
    if (1 < steps) fetch(1, p1);
    if (2 < steps) fetch(2, p2);
    for (int t = 0; t < steps; t += 3) {
        edge_step(t, p0);
        if (t + 3 < steps) fetch(t + 3, p0);
        if (t + 1 < steps) {
            edge_step(t + 1, p1);
            if (t + 4 < steps) fetch(t + 4, p1);
        }
        if (t + 2 < steps) {
            edge_step(t + 2, p2);
            if (t + 5 < steps) fetch(t + 5, p2);
        }
    }
    if (own && h == kNs) {
        const int io = perm ? min(max(perm[i], 0), n - 1) : i;  // outputs under the caller's index
        if (accum) {
            Fout[io] += fx; Fout[n + io] += fy; Fout[2 * n + io] += fz;
        } else {
            Fout[io] = fx; Fout[n + io] = fy; Fout[2 * n + io] = fz;
        }
        if constexpr (VIR) {
            if (vir_set) vir_set[io] = vr;
            if (vir_add) vir_add[io] += vr;
        }
    }
}

// Reverse of the head for a loss with dL/dF_i = gF_i: each directed edge
// (i, j) carries a_ij = gF_i - gF_j as the adjoint of F_ij.  The owner i
// accumulates only its own adjoints, so no atomics are needed: q_i and V_i
// from its edges (i, j) (first sweep), k_i from the reverse edges (j, i)
// (second sweep).  In each sweep, phase 1 (lanes over edges) forms the
// coefficient adjoints dL/dc and stages them in LDS; phase 2 (lanes over the
// (head, channel) pairs) gathers the neighbour's k or q row.
__global__ void __launch_bounds__(64) k_head_bwd(MpGeom mg, const float* __restrict__ QK, const float* __restrict__ Vh,
                                                 const float* __restrict__ gF, float* __restrict__ gQK,
                                                 float* __restrict__ gVh) {
    __shared__ float gc[64][kH];
    __shared__ int jj[64];
    __shared__ float gvc[64][kNl * 3];  // per-entry V adjoint contributions (sweep 0)
    const int lane = threadIdx.x;
    const int i = xcd_block(blockIdx.x, gridDim.x);
    const int n = mg.n;
    double L, inv;
    mg.geom.get(i, L, inv);
    const double xi = mg.pos[i], yi = mg.pos[n + i], zi = mg.pos[2 * n + i];
    const float* qi = QK + int64_t(i) * 2 * kH * kNc;
    const float* ki = qi + kH * kNc;
    float Vi[kNl][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int h = 0; h < kNl; ++h) Vi[h][a] = Vh[(int64_t(i) * 3 + a) * kNl + h];
    const float gFi[3] = {gF[i], gF[n + i], gF[2 * n + i]};
    const float scale = 0.35355339059327373f;  // 1/sqrt(n_c)
    const int e0 = mg.off[i], e1 = mg.off[i + 1];
    float* gq = gQK + int64_t(i) * 2 * kH * kNc;
    float* gk = gq + kH * kNc;
    float gv_acc = 0.f;  // lane < 6: component (h, a) = (lane / 3, lane % 3)
    for (int sweep = 0; sweep < 2; ++sweep) {
        float acc0 = 0.f, acc1 = 0.f;  // (h, c) = lane and 64 + lane (lane < 16)
        for (int base = e0; base < e1; base += 64) {
            const int e = base + lane;
            HeadEdge he;
            const bool ok = e < e1 && head_edge(mg, i, e, xi, yi, zi, L, inv, he);
            if (ok) {
                const int j = he.j;
                const float* qj = QK + int64_t(j) * 2 * kH * kNc;
                const float* kj = qj + kH * kNc;
                float aij[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) aij[a] = gFi[a] - gF[a * n + j];
                float c[kH];
                if (sweep == 0) {
                    head_coeffs(qi, kj, c);  // c_ijh
                    float S = 0.f;
#pragma unroll
                    for (int h = 0; h < kNs; ++h) S = fmaf(c[h], he.ef[h], S);
                    float D[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) D[a] = he.u[a] + c[kNs] * Vi[0][a] + c[kNs + 1] * Vi[1][a];
                    const float gS = aij[0] * D[0] + aij[1] * D[1] + aij[2] * D[2];
#pragma unroll
                    for (int h = 0; h < kNs; ++h) gc[lane][h] = gS * he.ef[h];
#pragma unroll
                    for (int h = 0; h < kNl; ++h) {
                        gc[lane][kNs + h] = S * (aij[0] * Vi[h][0] + aij[1] * Vi[h][1] + aij[2] * Vi[h][2]);
#pragma unroll
                        for (int a = 0; a < 3; ++a) gvc[lane][h * 3 + a] = aij[a] * S * c[kNs + h];
                    }
                } else {
                    head_coeffs(qj, ki, c);  // c_jih
                    float Vj[kNl][3];
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int h = 0; h < kNl; ++h) Vj[h][a] = Vh[(int64_t(j) * 3 + a) * kNl + h];
                    float S = 0.f;
#pragma unroll
                    for (int h = 0; h < kNs; ++h) S = fmaf(c[h], he.ef[h], S);
                    float D[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) D[a] = -he.u[a] + c[kNs] * Vj[0][a] + c[kNs + 1] * Vj[1][a];
                    // the adjoint of F_ji is -aij
                    const float gS = -(aij[0] * D[0] + aij[1] * D[1] + aij[2] * D[2]);
#pragma unroll
                    for (int h = 0; h < kNs; ++h) gc[lane][h] = gS * he.ef[h];
#pragma unroll
                    for (int h = 0; h < kNl; ++h)
                        gc[lane][kNs + h] = -S * (aij[0] * Vj[h][0] + aij[1] * Vj[h][1] + aij[2] * Vj[h][2]);
                }
                jj[lane] = j;
            } else {
                jj[lane] = -1;
            }
            __syncthreads();
            const int cnt = min(64, e1 - base);
            for (int t = 0; t < cnt; ++t) {
                const int j = jj[t];
                if (j < 0) continue;
                // sweep 0 gathers k_j, sweep 1 gathers q_j
                const float* row = QK + int64_t(j) * 2 * kH * kNc + (sweep == 0 ? kH * kNc : 0);
                acc0 = fmaf(gc[t][lane / kNc] * scale, row[lane], acc0);
                if (lane < 16) acc1 = fmaf(gc[t][(64 + lane) / kNc] * scale, row[64 + lane], acc1);
                if (sweep == 0 && lane < kNl * 3) gv_acc += gvc[t][lane];
            }
            __syncthreads();
        }
        float* out = sweep == 0 ? gq : gk;
        out[lane] = acc0;
        if (lane < 16) out[64 + lane] = acc1;
    }
    if (lane < kNl * 3) {
        const int h = lane / 3, a = lane % 3;
        gVh[(int64_t(i) * 3 + a) * kNl + h] = gv_acc;
    }
}

// ------------------------------------------------- fused NC update block --
// Update block of the one-layer NC embedding followed by its q/k and vector
// projections, for widths F <= 32: one lane per feature column of two atoms
// (each weight read from LDS serves both).
// The model keeps an LDS image of these weights (pack_nc_weights: one row
// per output, rows padded by four floats, rounded for BF16 models), so
// staging is a straight 16-byte copy; a lane then reads four consecutive k
// of its output's row per 16-byte LDS read (the padding puts the rows of
// neighbouring lanes in different banks), the per-atom inputs as broadcast
// 16-byte reads, and the block walks over groups of atoms.  Every sum runs
// over k in increasing order.  With BF16, weights and every perceptron input
// are rounded to bfloat16 and products accumulate in float32, as in the MFMA
// GEMMs of the general path.
__device__ __forceinline__ float bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

// floats of the packed image: rows of U;V (2F), M2 (3F), W_qk (HC) and W_V
// (n_l) of pitch F + 4, rows of M1 (F) of pitch 2F + 4
// atoms per lane and block pass of k_nc_update_proj
constexpr int kNcAtomsPerLane = 2;

constexpr int64_t nc_image_floats(int F) {
    return int64_t(5 * F + 2 * kH * kNc + kNl) * (F + 4) + int64_t(F) * (2 * F + 4);
}

template <int F, bool BF16>
__global__ void __launch_bounds__(256) k_nc_update_proj(NcUpdateArgs a) {
    constexpr int HC = 2 * kH * kNc;  // q and k outputs
    constexpr int GPB = 256 / F;      // lane groups per block
    constexpr int NA = kNcAtomsPerLane;
    constexpr int APB = NA * GPB;     // atoms per block pass
    constexpr int QPL = HC / F;       // q/k outputs per lane
    static_assert(HC % F == 0, "q/k outputs split evenly over the lanes of an atom");
    constexpr int P1 = F + 4, P2 = 2 * F + 4;
    extern __shared__ float lds[];
    float* UV = lds;                   // [2F][P1]  outputs of U, then of V
    float* M1 = UV + 2 * F * P1;       // [F][P2]
    float* M2 = M1 + F * P2;           // [3F][P1]
    float* Q = M2 + 3 * F * P1;        // [HC][P1]
    float* WV = Q + HC * P1;           // [kNl][P1]
    float* m1 = WV + kNl * P1;         // [F]
    float* m2 = m1 + F;                // [3F]
    float* work = m2 + 3 * F;          // per atom: sm[F], vm[3F], x[2F], z[F], so[F], vo[3F]
    auto rnd = [](float x) { return BF16 ? bf16_round(x) : x; };
    auto ld4 = [](const float* p) { return *reinterpret_cast<const float4*>(p); };
    constexpr int NW = int(nc_image_floats(F));
    static_assert(NW % 4 == 0, "image of whole 16-byte units");
    {
        // every load issued before the first store: one round trip per block
        constexpr int U = (NW / 4 + 255) / 256;
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            v[u] = reinterpret_cast<const float4*>(a.wt)[min(int(threadIdx.x) + u * 256, NW / 4 - 1)];
        const float b1 = a.m1[threadIdx.x % F], b2 = a.m2[threadIdx.x % (3 * F)];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = threadIdx.x + u * 256;
            if (idx < NW / 4) reinterpret_cast<float4*>(lds)[idx] = v[u];
        }
        if (threadIdx.x < F) m1[threadIdx.x] = b1;
        if (threadIdx.x < 3 * F) m2[threadIdx.x] = b2;
    }
    // lane (g, f) takes feature f of atoms base + g + u GPB, u < NA: every
    // weight read from LDS serves NA atoms
    const int g = threadIdx.x / F, f = threadIdx.x % F;
    float *sm[NA], *vm[NA], *x[NA], *z[NA], *so[NA], *vo[NA];
#pragma unroll
    for (int u = 0; u < NA; ++u) {
        sm[u] = work + (g + u * GPB) * 11 * F;
        vm[u] = sm[u] + F;
        x[u] = vm[u] + 3 * F;
        z[u] = x[u] + 2 * F;
        so[u] = z[u] + F;
        vo[u] = so[u] + F;
    }
    const int n = a.n;
    for (int base = blockIdx.x * APB; base < n; base += gridDim.x * APB) {
        __syncthreads();  // weights staged / previous pass done with the work rows
        // the work rows hold perceptron inputs as the products read them
        // (rounded once here for BF16 models); the lane keeps its own
        // columns of s and v unrounded for the residual sums
        float s_own[NA], v_own[NA][3];
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int i = base + g + u * GPB;
            const bool act = i < n;
            s_own[u] = act ? a.smid[int64_t(i) * F + f] : 0.f;
            sm[u][f] = rnd(s_own[u]);
#pragma unroll
            for (int al = 0; al < 3; ++al) {
                v_own[u][al] = act ? a.vmid[(int64_t(i) * 3 + al) * F + f] : 0.f;
                vm[u][al * F + f] = rnd(v_own[u][al]);
            }
        }
        __syncthreads();
        float Uv[NA][3] = {}, Vv[NA][3] = {};
        {
            const float* ur = UV + f * P1;
            const float* vr = UV + (F + f) * P1;
#pragma unroll 2
            for (int k = 0; k < F; k += 4) {
                const float4 uw = ld4(ur + k);
                const float4 vw = ld4(vr + k);
#pragma unroll
                for (int u = 0; u < NA; ++u)
#pragma unroll
                    for (int al = 0; al < 3; ++al) {
                        const float4 vk = ld4(vm[u] + al * F + k);
                        Uv[u][al] = fmaf(uw.x, vk.x, Uv[u][al]);
                        Vv[u][al] = fmaf(vw.x, vk.x, Vv[u][al]);
                        Uv[u][al] = fmaf(uw.y, vk.y, Uv[u][al]);
                        Vv[u][al] = fmaf(vw.y, vk.y, Vv[u][al]);
                        Uv[u][al] = fmaf(uw.z, vk.z, Uv[u][al]);
                        Vv[u][al] = fmaf(vw.z, vk.z, Vv[u][al]);
                        Uv[u][al] = fmaf(uw.w, vk.w, Uv[u][al]);
                        Vv[u][al] = fmaf(vw.w, vk.w, Vv[u][al]);
                    }
            }
        }
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            float nn = 1e-8f;
#pragma unroll
            for (int al = 0; al < 3; ++al) nn = fmaf(Vv[u][al], Vv[u][al], nn);
            x[u][f] = sm[u][f];
            x[u][F + f] = rnd(sqrtf(nn));
        }
        __syncthreads();
        {
            float a1[NA];
#pragma unroll
            for (int u = 0; u < NA; ++u) a1[u] = m1[f];
            const float* wr = M1 + f * P2;
#pragma unroll 4
            for (int k = 0; k < 2 * F; k += 4) {
                const float4 w = ld4(wr + k);
#pragma unroll
                for (int u = 0; u < NA; ++u) {
                    const float4 xv = ld4(x[u] + k);
                    a1[u] = fmaf(w.x, xv.x, a1[u]);
                    a1[u] = fmaf(w.y, xv.y, a1[u]);
                    a1[u] = fmaf(w.z, xv.z, a1[u]);
                    a1[u] = fmaf(w.w, xv.w, a1[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < NA; ++u) z[u][f] = rnd(silu(a1[u]));
        }
        __syncthreads();
        float pq[NA][3];
#pragma unroll
        for (int u = 0; u < NA; ++u)
#pragma unroll
            for (int c = 0; c < 3; ++c) pq[u][c] = m2[c * F + f];
#pragma unroll 2
        for (int k = 0; k < F; k += 4) {
            float4 zk[NA];
#pragma unroll
            for (int u = 0; u < NA; ++u) zk[u] = ld4(z[u] + k);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float4 w = ld4(M2 + (c * F + f) * P1 + k);
#pragma unroll
                for (int u = 0; u < NA; ++u) {
                    pq[u][c] = fmaf(w.x, zk[u].x, pq[u][c]);
                    pq[u][c] = fmaf(w.y, zk[u].y, pq[u][c]);
                    pq[u][c] = fmaf(w.z, zk[u].z, pq[u][c]);
                    pq[u][c] = fmaf(w.w, zk[u].w, pq[u][c]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const float dot = Uv[u][0] * Vv[u][0] + Uv[u][1] * Vv[u][1] + Uv[u][2] * Vv[u][2];
            so[u][f] = rnd(s_own[u] + pq[u][0] + pq[u][1] * dot);
#pragma unroll
            for (int al = 0; al < 3; ++al) vo[u][al * F + f] = rnd(v_own[u][al] + pq[u][2] * Uv[u][al]);
        }
        __syncthreads();
        {
            // q/k outputs f + q F, q < QPL, of every atom of the lane: one
            // read of each input chunk serves all of them
            float acc[NA][QPL] = {};
#pragma unroll 2
            for (int k = 0; k < F; k += 4) {
                float4 sv[NA];
#pragma unroll
                for (int u = 0; u < NA; ++u) sv[u] = ld4(so[u] + k);
#pragma unroll
                for (int q = 0; q < QPL; ++q) {
                    const float4 w = ld4(Q + (f + q * F) * P1 + k);
#pragma unroll
                    for (int u = 0; u < NA; ++u) {
                        acc[u][q] = fmaf(w.x, sv[u].x, acc[u][q]);
                        acc[u][q] = fmaf(w.y, sv[u].y, acc[u][q]);
                        acc[u][q] = fmaf(w.z, sv[u].z, acc[u][q]);
                        acc[u][q] = fmaf(w.w, sv[u].w, acc[u][q]);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < NA; ++u) {
                const int i = base + g + u * GPB;
                if (i < n) {
#pragma unroll
                    for (int q = 0; q < QPL; ++q) a.QK[int64_t(i) * HC + f + q * F] = acc[u][q];
                }
            }
        }
        if (f < 3 * kNl) {
            const int h = f / 3, al = f % 3;
            const float* wr = WV + h * P1;
            float acc[NA] = {};
#pragma unroll 2
            for (int k = 0; k < F; k += 4) {
                const float4 w = ld4(wr + k);
#pragma unroll
                for (int u = 0; u < NA; ++u) {
                    const float4 vv = ld4(vo[u] + al * F + k);
                    acc[u] = fmaf(w.x, vv.x, acc[u]);
                    acc[u] = fmaf(w.y, vv.y, acc[u]);
                    acc[u] = fmaf(w.z, vv.z, acc[u]);
                    acc[u] = fmaf(w.w, vv.w, acc[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < NA; ++u) {
                const int i = base + g + u * GPB;
                if (i < n) a.Vh[(int64_t(i) * 3 + al) * kNl + h] = acc[u];
            }
        }
    }
}

// The LDS image of k_nc_update_proj, element (row o, column k) of each
// segment = W[o][k] (zero in the padding), rounded for BF16 models.
__global__ void k_pack_nc(int F, const float* __restrict__ UV, const float* __restrict__ M1,
                          const float* __restrict__ M2, const float* __restrict__ Wqk, const float* __restrict__ WV,
                          int bf16, float* __restrict__ out) {
    constexpr int HC = 2 * kH * kNc;
    const int P1 = F + 4, P2 = 2 * F + 4;
    const int64_t total = nc_image_floats(F);
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= total) return;
    int64_t r = t;
    float v = 0.f;
    if (r < 2 * F * P1) {
        const int o = int(r / P1), k = int(r % P1);
        if (k < F) v = UV[int64_t(o) * F + k];
    } else if ((r -= 2 * F * P1) < int64_t(F) * P2) {
        const int o = int(r / P2), k = int(r % P2);
        if (k < 2 * F) v = M1[int64_t(o) * 2 * F + k];
    } else if ((r -= int64_t(F) * P2) < 3 * F * P1) {
        const int o = int(r / P1), k = int(r % P1);
        if (k < F) v = M2[int64_t(o) * F + k];
    } else if ((r -= 3 * F * P1) < int64_t(HC) * P1) {
        const int o = int(r / P1), k = int(r % P1);
        if (k < F) v = Wqk[int64_t(o) * F + k];
    } else {
        r -= int64_t(HC) * P1;
        const int o = int(r / P1), k = int(r % P1);
        if (k < F) v = WV[int64_t(o) * F + k];
    }
    out[t] = bf16 ? bf16_round(v) : v;
}

void pack_nc_weights(int F, const float* UV, const float* M1, const float* M2, const float* Wqk, const float* WV,
                     bool bf16, float* out, hipStream_t st) {
    const int64_t total = nc_image_floats(F);
    k_pack_nc<<<cdiv(total, 256), 256, 0, st>>>(F, UV, M1, M2, Wqk, WV, bf16 ? 1 : 0, out);
    NNP_LAUNCH_CHECK();
}

size_t nc_update_lds_bytes(int F) {
    return sizeof(float) *
           (size_t(nc_image_floats(F)) + size_t(F + 3 * F) + size_t(kNcAtomsPerLane) * size_t(256 / F) * 11 * F);
}

int64_t nc_image_count(int F) { return nc_image_floats(F); }

bool launch_nc_update_proj(const NcUpdateArgs& a, int F, bool bf16, hipStream_t st) {
    if (a.n <= 0) return true;
    const size_t lds = nc_update_lds_bytes(F);
    const int blocks = std::min(cdiv(a.n, kNcAtomsPerLane * (256 / F)), 512);
    ScopedTimer timer("nc_update", st);
    // more than 64 KB of dynamic LDS at F = 32: raise each instance's limit
    // once (flag per width and precision)
    static std::atomic<bool> raised[6];
    const int slot = (F == 32 ? 0 : F == 16 ? 1 : 2) * 2 + (bf16 ? 1 : 0);
    auto launch = [&](void (*kernel)(NcUpdateArgs)) {
        if (!raised[slot].load()) {
            NNP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
            raised[slot].store(true);
        }
        kernel<<<blocks, 256, lds, st>>>(a);
    };
    if (F == 32) {
        if (bf16) launch(k_nc_update_proj<32, true>);
        else launch(k_nc_update_proj<32, false>);
    } else if (F == 16) {
        if (bf16) launch(k_nc_update_proj<16, true>);
        else launch(k_nc_update_proj<16, false>);
    } else if (F == 8) {
        if (bf16) launch(k_nc_update_proj<8, true>);
        else launch(k_nc_update_proj<8, false>);
    } else {
        return false;
    }
    NNP_LAUNCH_CHECK();
    return true;
}

// ------------------------------------------------------------------- host --
static int ew_blocks(int64_t count) { return cdiv(count, 256); }

void launch_embed(int n, int F, int S, const int* species, const float* emb, float* s, float* v, hipStream_t st) {
    k_embed<<<ew_blocks(int64_t(n) * F), 256, 0, st>>>(n, F, S, species, emb, s, v);
    NNP_LAUNCH_CHECK();
}
void launch_build_x(int n, int F, const float* smid, const float* UV, float* X, hipStream_t st) {
    k_build_x<<<ew_blocks(int64_t(n) * F), 256, 0, st>>>(n, F, smid, UV, X);
    NNP_LAUNCH_CHECK();
}
void launch_update_combine(int n, int F, const float* smid, const float* vmid, const float* UV, const float* pqo,
                           float* s_out, float* v_out, hipStream_t st) {
    k_update_combine<<<ew_blocks(int64_t(n) * F), 256, 0, st>>>(n, F, smid, vmid, UV, pqo, s_out, v_out);
    NNP_LAUNCH_CHECK();
}
void launch_update_combine_bwd(int n, int F, const float* UV, const float* pqo, const float* gs, const float* gv,
                               float* gpqo, float* gUV, hipStream_t st) {
    k_update_combine_bwd<<<ew_blocks(int64_t(n) * F), 256, 0, st>>>(n, F, UV, pqo, gs, gv, gpqo, gUV);
    NNP_LAUNCH_CHECK();
}
void launch_norm_bwd(int n, int F, const float* gs, const float* gX, const float* X, const float* UV, float* gsmid,
                     float* gUV, hipStream_t st) {
    k_norm_bwd<<<ew_blocks(int64_t(n) * F), 256, 0, st>>>(n, F, gs, gX, X, UV, gsmid, gUV);
    NNP_LAUNCH_CHECK();
}
void launch_readout(int n, int F, int S, const float* z, const float* wo, const float* beta, const int* species, float* Ei,
                    hipStream_t st, const int* perm) {
    k_readout<<<cdiv(n, 4), 256, 0, st>>>(n, F, S, z, wo, beta, species, Ei, perm);
    NNP_LAUNCH_CHECK();
}
void launch_readout_bwd(int n, int F, const float* ao, const float* wo, float* gao, hipStream_t st) {
    k_readout_bwd<<<ew_blocks(int64_t(n) * F), 256, 0, st>>>(n, F, ao, wo, gao);
    NNP_LAUNCH_CHECK();
}
void launch_rep_sum(int n_rep, const int64_t* rep_start, const float* x, double* out, hipStream_t st) {
    k_rep_sum<<<n_rep, 256, 0, st>>>(rep_start, x, out);
    NNP_LAUNCH_CHECK();
}
void launch_emb_grad(int n, int F, int S, const int* species, const float* gs0, float* gemb, hipStream_t st) {
    k_emb_grad<<<S, 128, 0, st>>>(n, F, S, species, gs0, gemb);
    NNP_LAUNCH_CHECK();
}
void launch_head_fwd(const MpGeom& mg, const float* QK, const float* Vh, float* F, bool accum, hipStream_t st,
                     float* vir_set, float* vir_add) {
    if (mg.n <= 0) return;
    ScopedTimer timer("head_fwd", st);
    // 16 lanes per atom: rows of the 3.5 A list hold about 40 candidates
    if (vir_set || vir_add) k_head_fwd<16, true><<<cdiv(mg.n, 16), 256, 0, st>>>(mg, QK, Vh, F, accum, vir_set, vir_add);
    else k_head_fwd<16, false><<<cdiv(mg.n, 16), 256, 0, st>>>(mg, QK, Vh, F, accum, nullptr, nullptr);
    NNP_LAUNCH_CHECK();
}
void launch_head_fwd_rec(const MpGeom& mg, const int* cnt, const NcEdge* rec, const float* QK, const float* Vh,
                         float* F, bool accum, hipStream_t st, float* vir_set, float* vir_add) {
    if (mg.n <= 0) return;
    ScopedTimer timer("head_fwd", st);
    // four owner atoms per wavefront
    if (vir_set || vir_add)
        k_head_fwd_rec<true><<<cdiv(mg.n, 16), 256, 0, st>>>(mg.n, mg.off, cnt, rec, QK, Vh, F, accum, vir_set, vir_add,
                                                             mg.perm);
    else
        k_head_fwd_rec<false><<<cdiv(mg.n, 16), 256, 0, st>>>(mg.n, mg.off, cnt, rec, QK, Vh, F, accum, nullptr,
                                                              nullptr, mg.perm);
    NNP_LAUNCH_CHECK();
}
void launch_head_bwd(const MpGeom& mg, const float* QK, const float* Vh, const float* gF, float* gQK, float* gVh,
                     hipStream_t st) {
    if (mg.n <= 0) return;
    k_head_bwd<<<mg.n, 64, 0, st>>>(mg, QK, Vh, gF, gQK, gVh);
    NNP_LAUNCH_CHECK();
}

}  // namespace nnp
