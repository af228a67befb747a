// Matrix-core message kernels for width-128 embeddings with 16 Bessel
// functions and the cosine cutoff (the message step and its reverse), and
// the edge preparation they share.
//
// The radial filter of a batch of edges is a product of the per-edge basis
// (edges x K) with the filter weights (K x 3F).  It runs on the FP16 matrix
// cores at FP32-equivalent precision: each FP32 operand x is split into
// x_hi = fp16(x) and x_lo = fp16(x - x_hi), which together carry 22
// significant bits, and the products lo*hi, hi*lo and hi*hi are accumulated
// in FP32 (lo*lo lies below FP32 rounding).  The weights enter scaled by a
// power of two that puts their largest magnitude in [2^13, 2^14), inside the
// FP16 range whatever the model; every sum that is linear in the filter is
// rescaled once per atom, which is exact.
//
// Edge preparation (once per force evaluation, shared by the three layers'
// forward and reverse launches): one wavefront per atom applies the float64
// pair rule at the model cutoff to the atom's list row, compacts the edges
// that pass in list order to the front of the row, and stores per edge a
// record (neighbour, species, f, f', unit vector, 1/r) and the radial values
// e_k(r) f(r) and their r-derivatives (float32) already split into FP16
// pairs.
//
// Message kernels: blocks take four atoms in turn with four wavefronts, one
// per block of 32 features; the wavefronts do not synchronise except once
// per block in the reverse, to add their force shares.  An atom's edges are
// consumed in batches of fixed size (32 forward, 16 reverse) in list order,
// so the batch an edge falls into depends only on its rank among the atom's
// edges within the cutoff: results do not depend on the list radius.
//
// In a 32x32x16 product the lane (c, h) = (lane % 32, lane / 32) holds output
// column c for rows 8j + 4h + i (j, i = 0..3): every lane owns one feature and
// accumulates over a fixed subset of each batch's edges; the two halves of the
// wavefront are added at the end of the atom.  Forward: the rows are 32 edges.
// Reverse: rows 0..15 hold e_k(r) f(r) and rows 16..31 their r-derivatives
// for the same 16 edges, so one product gives w and dw/dr of an edge in the
// same lane.  The per-edge work after the filter is that of the vector
// kernels (same formulas; see the message kernels of mp.hip).
#include <hip/hip_ext.h>

#include "common.h"
#include "kernels.h"
#include "mp_edge.h"

namespace nnp {

namespace {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float floatx16_t __attribute__((ext_vector_type(16)));

constexpr int kMxF = 128, kMxK = 16, kMxWaves = 4, kMxAtoms = 4;
// forward: edges of a lane whose loads are issued together (eight: 40
// loads in flight per lane, within three wavefronts per SIMD)
constexpr int kFwdGroup = 8;
// reverse: the same; small groups keep every variant within three
// wavefronts per SIMD (measured: more gathers in flight per wavefront at
// two wavefronts per SIMD are 7 % slower than fewer at three)
template <bool L0>
constexpr int kBwdGroup = L0 ? 4 : 2;

__device__ __forceinline__ void split8(const float* x, half8_t& hi, half8_t& lo) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const _Float16 t = static_cast<_Float16>(x[q]);
        hi[q] = t;
        lo[q] = static_cast<_Float16>(x[q] - static_cast<float>(t));
    }
}

// The bias product (rows ab, bias operand bb), then A (32 x 16) times
// B (16 x 32) from the split operands, small terms first
template <bool BIAS = true>
__device__ __forceinline__ floatx16_t mma3(const half4_t& ab, const half4_t& bb, const half8_t& ah,
                                           const half8_t& al, const half8_t& bh, const half8_t& bl) {
    floatx16_t c = {};
    if constexpr (BIAS) c = __builtin_amdgcn_mfma_f32_32x32x8f16(ab, bb, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, c, 0, 0, 0);
    return c;
}

__device__ __forceinline__ void load8(const float* p, float* x) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    const float4 b = *reinterpret_cast<const float4*>(p + 4);
    x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
    x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
}

// This lane's B fragments: rows 8h..8h+7 of column f of the scaled filter
// weights of each channel, split; and the bias operand of each channel (a
// 32x32x8 product): rows 0..2 of column f hold (b_hi, b_hi, b_lo) of the
// scaled bias, the other rows zero, so that with A rows (c_hi, c_lo, c_hi,
// 0, ...) of a per-edge factor c one product gives c b at FP32-equivalent
// precision.
__device__ __forceinline__ void load_filter(const float* Wr, const float* br, float sc, int f, int h, half8_t* bh,
                                            half8_t* bl, half4_t* bb) {
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        float x[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) x[q] = Wr[(p * kMxF + f) * kMxK + 8 * h + q] * sc;
        split8(x, bh[p], bl[p]);
        const float b = br[p * kMxF + f] * sc;
        const _Float16 b_hi = static_cast<_Float16>(b);
        const _Float16 b_lo = static_cast<_Float16>(b - static_cast<float>(b_hi));
        bb[p] = half4_t{};
        if (h == 0) {
            bb[p][0] = b_hi;
            bb[p][1] = b_hi;
            bb[p][2] = b_lo;
        }
    }
}

// The A operand of the bias product for a row whose per-edge factor is c
// (the cutoff f or its derivative): (c_hi, c_lo, c_hi, 0, ...) in the lanes
// of the first half, zero in the second.
__device__ __forceinline__ half4_t bias_rows(float c, int h) {
    half4_t a = {};
    if (h == 0) {
        const _Float16 c_hi = static_cast<_Float16>(c);
        a[0] = c_hi;
        a[1] = static_cast<_Float16>(c - static_cast<float>(c_hi));
        a[2] = c_hi;
    }
    return a;
}

__device__ __forceinline__ half8_t as_half8(const uint4& u) { return __builtin_bit_cast(half8_t, u); }

// A float at a 32-bit byte offset from a wavefront-uniform base: the
// neighbour-row gathers then take one 32-bit multiply-add per edge for
// their address, and the quantities of a row differ by immediate offsets.
__device__ __forceinline__ float ld_off(const float* base, uint32_t byte_off) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + byte_off);
}

// ---------------------------------------------------------- edge preparation

// With SM > 0 the same pass also forms the first conservative layer's edge
// sums by neighbour species (see mp_species.hip): the edges of each
// iteration are staged in LDS grouped by species, and lane (c, k) =
// (lane / 16, lane % 16) adds w_c e_k f (w_0 = 1, w_{1+a} = u_a) and w_c f
// over each species' segment; rows Es[i][ep] (c = 0) and Ev[3 i + a][ep],
// 20 slots per species (16 basis values, the cutoff, the species
// indicator, two zeros), zero past S species.
constexpr int kSpKP = kMxK + 4;

template <int SM>
__global__ void __launch_bounds__(256, 3) k_edge_prep(MpGeom mg, int* __restrict__ ecnt, EdgeRec* __restrict__ erec,
                                                   uint4* __restrict__ ehalf, float* __restrict__ Es,
                                                   float* __restrict__ Ev, int S, int ep) {
    constexpr int SP_PITCH = kMxK + 5;  // staged edge: e_k f, 1, u[3], f
    __shared__ float stage[SM > 0 ? 4 : 1][SM > 0 ? 64 : 1][SP_PITCH];
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= mg.n) return;  // whole wavefronts
    const int c = lane >> 4, kk = lane & 15;
    float acc[SM > 0 ? SM : 1] = {}, accf[SM > 0 ? SM : 1] = {};
    float(*st)[SP_PITCH] = stage[SM > 0 ? (threadIdx.x >> 6) : 0];
    const int n = mg.n;
    const int start = mg.off[i], end = mg.off[i + 1];
    double L, inv;
    mg.geom.get(i, L, inv);
    const double xi = mg.pos[i], yi = mg.pos[n + i], zi = mg.pos[2 * n + i];
    int cnt = 0;
    for (int base = start; base < end; base += 64) {
        const int e = base + lane;
        bool ok = false;
        double dx = 0, dy = 0, dz = 0;
        int j = -1;
        if (e < end) {
            j = mg.nbr[e];
            ok = pair_rule(xi, yi, zi, mg.pos[j], mg.pos[n + j], mg.pos[2 * n + j], L, inv, mg.rc2, dx, dy, dz);
        }
        const uint64_t bal = __ballot(ok);
        const int tj = ok && mg.species ? min(max(mg.species[j], 0), mg.n_species - 1) : 0;
        // this iteration's edges grouped by neighbour species (list order
        // within a species)
        int seg[SM + 1];
        seg[0] = 0;
        int slot = 0;  // staging row of this lane's edge
        if constexpr (SM > 0) {
            const int t = ok ? min(tj, S - 1) : SM;
#pragma unroll
            for (int sp = 0; sp < SM; ++sp) {
                const uint64_t m = __ballot(t == sp);
                if (t == sp) slot = seg[sp] + __popcll(m & ((1ull << lane) - 1ull));
                seg[sp + 1] = seg[sp] + __popcll(m);
            }
        }
        if (ok) {
            const int p = start + cnt + __popcll(bal & ((1ull << lane) - 1ull));
            const double r = sqrt((dx * dx + dy * dy) + dz * dz);
            const double ir = 1.0 / r;
            float ef[kMxK], def[kMxK], fc, dfc;
            radial_cos_f32<kMxK>(float(r), mg, ef, def, fc, dfc);
            EdgeRec rec;
            rec.j = j;
            rec.t = tj;
            rec.fc = fc;
            rec.dfc = dfc;
            rec.u[0] = float(dx * ir);
            rec.u[1] = float(dy * ir);
            rec.u[2] = float(dz * ir);
            rec.ir = float(ir);
            erec[p] = rec;
            uint4* dst = ehalf + int64_t(p) * 8;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                half8_t hi, lo;
                split8(ef + 8 * q, hi, lo);
                dst[q] = __builtin_bit_cast(uint4, hi);
                dst[2 + q] = __builtin_bit_cast(uint4, lo);
                split8(def + 8 * q, hi, lo);
                dst[4 + q] = __builtin_bit_cast(uint4, hi);
                dst[6 + q] = __builtin_bit_cast(uint4, lo);
            }
            if constexpr (SM > 0) {
#pragma unroll
                for (int q = 0; q < kMxK; ++q) st[slot][q] = ef[q];
                st[slot][kMxK] = 1.f;
                st[slot][kMxK + 1] = rec.u[0];
                st[slot][kMxK + 2] = rec.u[1];
                st[slot][kMxK + 3] = rec.u[2];
                st[slot][kMxK + 4] = fc;
            }
        }
        cnt += __popcll(bal);
        if constexpr (SM > 0) {
            wave_sync_lds();
            // each edge added to the running sums in list order (within its
            // species), so that the sums do not depend on where the list
            // rows split into iterations (list radius, replica packing)
#pragma unroll
            for (int sp = 0; sp < SM; ++sp) {
                for (int q = seg[sp]; q < seg[sp + 1]; ++q) {
                    const float wc = st[q][kMxK + c];
                    acc[sp] = fmaf(wc, st[q][kk], acc[sp]);
                    accf[sp] = fmaf(wc, st[q][kMxK + 4], accf[sp]);
                }
            }
            wave_sync_lds();  // the next iteration overwrites the staged edges
        }
    }
    if (lane == 0) ecnt[i] = cnt;
    if constexpr (SM > 0) {
        float* row = c == 0 ? Es + int64_t(i) * ep : Ev + (int64_t(i) * 3 + (c - 1)) * ep;
        const int ti = min(max(mg.species[i], 0), S - 1);
#pragma unroll
        for (int sp = 0; sp < SM; ++sp) {
            if (sp >= S) break;
            row[sp * kSpKP + kk] = acc[sp];
            if (kk == 0) row[sp * kSpKP + kMxK] = accf[sp];
            if (kk == 1) row[sp * kSpKP + kMxK + 1] = (c == 0 && sp == ti) ? 1.f : 0.f;
            if (kk >= 2 && kk < kSpKP - kMxK) row[sp * kSpKP + kMxK + kk] = 0.f;
        }
        for (int z = S * kSpKP + kk; z < ep; z += 16) row[z] = 0.f;
    }
}

// A batch's prepared edges are loaded once per block: thread t holds one
// 16-byte piece (radial pieces of the batch's edges, then its records) in a
// register while the previous batch is processed, and stores it into the
// batch's LDS buffer (two, alternating) after the barrier that ends that
// batch's predecessor.  The forward needs only the e_k f pieces of an edge.
template <int BATCH>
struct BatchBuf {
    static constexpr int AP = BATCH == 32 ? 4 : 8;  // radial pieces per edge
    static constexpr int NA = BATCH * AP, N = NA + 2 * BATCH;
    uint4 a[BATCH][AP];
    EdgeRec rec[BATCH];
};

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint4 load_nt(const uint4* p) {
    const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
    return make_uint4(v[0], v[1], v[2], v[3]);
}

template <int BATCH>
__device__ __forceinline__ uint4 fetch_piece(const MpGeom& mg, int p0, int nb) {
    using B = BatchBuf<BATCH>;
    const int t = threadIdx.x;
    uint4 v = make_uint4(0, 0, 0, 0);
    // read once per evaluation and layer: non-temporal, so that the streamed
    // edges do not displace the neighbour rows from L2
    if (t < B::NA) {
        const int e = t / B::AP, q = t % B::AP;
        if (e < nb) v = load_nt(mg.ehalf + int64_t(p0 + e) * 8 + q);
    } else if (t < B::N) {
        const int u = t - B::NA;
        if (u < 2 * nb) v = load_nt(reinterpret_cast<const uint4*>(mg.erec + p0) + u);
    }
    return v;
}

template <int BATCH>
__device__ __forceinline__ void store_piece(BatchBuf<BATCH>& b, const uint4& v) {
    if (threadIdx.x < BatchBuf<BATCH>::N) reinterpret_cast<uint4*>(&b)[threadIdx.x] = v;
}

// The block's batches in processing order: atoms i0 .. i0 + kMxAtoms - 1
// (those below n), each atom's edges in batches of BATCH.  Returns the list
// position and size of the batch after batch b0 of atom ai (ai = -1: the
// first batch), or nb = 0 when there is none.
struct NextBatch {
    int p0, nb;
};

template <int BATCH>
__device__ __forceinline__ NextBatch next_batch(const MpGeom& mg, int i0, int ai, int b0, int cnt) {
    if (ai >= 0 && b0 + BATCH < cnt) return {mg.off[i0 + ai] + b0 + BATCH, min(BATCH, cnt - b0 - BATCH)};
    for (int a2 = ai + 1; a2 < kMxAtoms && i0 + a2 < mg.n; ++a2) {
        const int c2 = mg.ecnt[i0 + a2];
        if (c2 > 0) return {mg.off[i0 + a2], min(BATCH, c2)};
    }
    return {0, 0};
}

// ------------------------------------------------------------- forward --

struct FwdAcc {
    float s, v[3];
};

// One batch of nb <= 32 edges.  The lane's 16 edges are taken kFwdGroup at
// a time, the loads of a group issued before its arithmetic (an invalid edge
// of a partial batch reads the batch's first edge and contributes nothing).
template <bool L0>
__device__ __forceinline__ void fwd_batch(const MpFwd& a, const float* ptab, const BatchBuf<32>& buf, int nb, int f,
                                          int h, const half8_t* bh, const half8_t* bl, const half4_t* bb,
                                          FwdAcc& acc) {
    constexpr int F = kMxF, E = 16;
    const EdgeRec* rec = buf.rec;
    const int r = threadIdx.x & 31;  // A row: edge r (zero past nb: staged as zeros)
    const half8_t ah = as_half8(buf.a[r][h]), al = as_half8(buf.a[r][2 + h]);
    const half4_t ab = bias_rows(rec[r].fc, h);
    // w = Wr (e f) + b f of every channel
    const floatx16_t wa = mma3(ab, bb[0], ah, al, bh[0], bl[0]);
    floatx16_t wb = {};
    if (!L0) wb = mma3(ab, bb[1], ah, al, bh[1], bl[1]);  // the first layer's vector input is zero
    const floatx16_t wc = mma3(ab, bb[2], ah, al, bh[2], bl[2]);
    const uint32_t fo = uint32_t(f) * 4u;
#pragma unroll
    for (int g0 = 0; g0 < E; g0 += kFwdGroup) {
        // the b channel enters only as phi_b v_j, read as one product; rows
        // of phi and pv are 3F floats: one byte offset per edge serves both
        float pa[kFwdGroup], pc[kFwdGroup], pv[kFwdGroup][3];
#pragma unroll
        for (int g = 0; g < kFwdGroup; ++g) {
            const int q = g0 + g;
            const int te = 8 * (q / 4) + 4 * h + q % 4;
            const EdgeRec& s = rec[te < nb ? te : 0];
            if (L0) {
                const float* phj = ptab + s.t * 3 * F + f;
                pa[g] = phj[0];
                pc[g] = phj[2 * F];
            } else {
                const uint32_t off = uint32_t(s.j) * (3u * F * 4u) + fo;
                pa[g] = ld_off(a.phi, off);
                pc[g] = ld_off(a.phi, off + 2 * F * 4);
                pv[g][0] = ld_off(a.pv, off);
                pv[g][1] = ld_off(a.pv, off + F * 4);
                pv[g][2] = ld_off(a.pv, off + 2 * F * 4);
            }
        }
#pragma unroll
        for (int g = 0; g < kFwdGroup; ++g) {
            const int q = g0 + g;
            const int te = 8 * (q / 4) + 4 * h + q % 4;
            if (te >= nb) continue;
            const EdgeRec& s = rec[te];
            const float w_a = wa[q];
            const float c = pc[g] * wc[q];
            acc.s = fmaf(pa[g], w_a, acc.s);
            if (L0) {
                acc.v[0] = fmaf(s.u[0], c, acc.v[0]);
                acc.v[1] = fmaf(s.u[1], c, acc.v[1]);
                acc.v[2] = fmaf(s.u[2], c, acc.v[2]);
            } else {
                const float b = wb[q];
                acc.v[0] = fmaf(s.u[0], c, fmaf(b, pv[g][0], acc.v[0]));
                acc.v[1] = fmaf(s.u[1], c, fmaf(b, pv[g][1], acc.v[1]));
                acc.v[2] = fmaf(s.u[2], c, fmaf(b, pv[g][2], acc.v[2]));
            }
        }
    }
}

template <bool L0>
__global__ void __launch_bounds__(64 * kMxWaves, 2) k_message_fwd_mx(MpGeom mg, MpFwd a) {
    constexpr int F = kMxF, BATCH = 32;
    __shared__ __align__(16) BatchBuf<BATCH> buf[2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int h = lane >> 5, f = w * 32 + (lane & 31);
    const int n = mg.n;
    // first layer: the species table of phi in LDS
    __shared__ float ptab_s[L0 ? 8 * 3 * kMxF : 1];
    if constexpr (L0) {
        for (int t = threadIdx.x; t < mg.n_species * 3 * F; t += blockDim.x) ptab_s[t] = a.phi_tab[t];
        __syncthreads();
    }
    const float sc = a.mx_scale[0], isc = a.mx_scale[1];
    half8_t bh[3], bl[3];
    half4_t bb[3];
    load_filter(a.Wr, a.br, sc, f, h, bh, bl, bb);
    const int i0 = xcd_block(blockIdx.x, gridDim.x) * kMxAtoms;
    NextBatch nx = next_batch<BATCH>(mg, i0, -1, 0, 0);
    uint4 piece = fetch_piece<BATCH>(mg, nx.p0, nx.nb);
    int k = 0;  // batches of the block so far (LDS buffer parity)
    for (int ai = 0; ai < kMxAtoms; ++ai) {
        const int i = i0 + ai;
        if (i >= n) break;
        const int cnt = mg.ecnt[i];
        FwdAcc acc{};
        for (int b0 = 0; b0 < cnt; b0 += BATCH, ++k) {
            BatchBuf<BATCH>& b = buf[k & 1];
            store_piece(b, piece);
            __syncthreads();  // the batch is staged; the other buffer's batch is done
            nx = next_batch<BATCH>(mg, i0, ai, b0, cnt);
            piece = fetch_piece<BATCH>(mg, nx.p0, nx.nb);
            fwd_batch<L0>(a, ptab_s, b, min(BATCH, cnt - b0), f, h, bh, bl, bb, acc);
        }
        // both halves of the wavefront hold partial sums of feature f
        acc.s += __shfl_xor(acc.s, 32, 64);
#pragma unroll
        for (int al = 0; al < 3; ++al) acc.v[al] += __shfl_xor(acc.v[al], 32, 64);
        if (h == 0) {
            const int ti = L0 ? min(max(a.species[i], 0), mg.n_species - 1) : 0;
            const float si = L0 ? a.emb[ti * F + f] : a.s_in[int64_t(i) * F + f];
            a.s_out[int64_t(i) * F + f] = si + acc.s * isc;
#pragma unroll
            for (int al = 0; al < 3; ++al) {
                const int64_t idx = (int64_t(i) * 3 + al) * F + f;
                const float vi = L0 ? 0.f : a.v_in[idx];
                a.v_out[idx] = vi + acc.v[al] * isc;
            }
        }
    }
}

// ------------------------------------------------------------- reverse --

struct Owner {
    float ph[3], v[3], gs, gv[3];
};

// Per-lane sums of the reverse over the lane's edges (feature f):
//   gph0 = sum gs_n w_a,  gph2 = -sum w_c (g_vn . u),  GV = sum w_b g_vn
//   (phi_b adjoint o.v . GV and v adjoint o.ph_b GV at the end),
// and the lane's share of the force on the owner,
//   sum_e [dr u + (g_u - (g_u . u) u) / r]
//     = S1 + o.gv T1 - o.ph_c T2,  g_u = pc w_c o.gv - o.ph_c w_c g_vn,
//   S1 = sum (dr - (g_u . u) / r) u,  T1 = sum pc w_c / r,  T2 = sum w_c g_vn / r,
// which keeps the owner's factors out of the per-edge work.
struct BwdAcc {
    float gph0, gph2, GV[3], S1[3], T1, T2[3], vir;
};

// The split filter operands of a lane in LDS: pieces bh[0..2], bl[0..2],
// then bb[0], bb[1] and bb[2] (8 bytes each) in pieces 6 and 7, each piece
// at stride 64 (one lane's) so that a wavefront reads 1 KB contiguously.
constexpr int kFiltPieces = 8;

__device__ __forceinline__ void store_filter(uint4* fl, const half8_t* bh, const half8_t* bl, const half4_t* bb) {
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        fl[p * 64] = __builtin_bit_cast(uint4, bh[p]);
        fl[(3 + p) * 64] = __builtin_bit_cast(uint4, bl[p]);
    }
    const uint2 b0 = __builtin_bit_cast(uint2, bb[0]), b1 = __builtin_bit_cast(uint2, bb[1]),
                b2 = __builtin_bit_cast(uint2, bb[2]);
    fl[6 * 64] = make_uint4(b0.x, b0.y, b1.x, b1.y);
    fl[7 * 64] = make_uint4(b2.x, b2.y, 0u, 0u);
}

__device__ __forceinline__ void load_channel(const uint4* fl, int p, half8_t& bh, half8_t& bl, half4_t& bb) {
    bh = as_half8(fl[p * 64]);
    bl = as_half8(fl[(3 + p) * 64]);
    const uint4 q = fl[(6 + p / 2) * 64];
    bb = __builtin_bit_cast(half4_t, p % 2 == 0 ? make_uint2(q.x, q.y) : make_uint2(q.z, q.w));
}

// The neighbour rows one group of edges needs (phi_b of the neighbour
// enters only as phi_b v_n, read as one product; phi, pv and the vector
// adjoints have rows of 3F floats, one byte offset per edge serves them,
// the scalar adjoints rows of F).
template <int G>
struct BwdGather {
    float pa[G], pc[G], pvn[G][3], gn[G][3], gsn[G];
};

// One batch of nb <= 16 edges.  The lane's eight edges are taken kBwdGroup
// at a time (an invalid edge of a partial batch reads the batch's first
// edge and contributes nothing).  Past the first layer the rows of the next
// group are requested before the current one is reduced, and the filter
// operands come from LDS (fl) for the products only, which keeps their
// registers free for the second group; the first layer, with fewer rows per
// edge and room for a fourth wavefront per SIMD, keeps its operands in
// registers (bhr, blr, bbr) and takes the groups one after the other.
template <bool L0, bool VIR>
__device__ __forceinline__ void bwd_batch(const MpBwd& a, const float* ptab, const BatchBuf<16>& buf, int nb, int f,
                                          int h, const uint4* fl, const half8_t* bhr, const half8_t* blr,
                                          const half4_t* bbr, const float* b0, const Owner& o, BwdAcc& acc) {
    constexpr int F = kMxF, E = 8, G = kBwdGroup<L0>;
    const EdgeRec* rec = buf.rec;
    // A rows 0..15: e_k f of edges 0..15, rows 16..31: their r-derivatives
    // (zero past nb: staged as zeros), and the bias rows f or f'
    const int r = threadIdx.x & 31, e = r & 15, part = 4 * (r >> 4);
    const half8_t ah = as_half8(buf.a[e][part + h]), al = as_half8(buf.a[e][part + 2 + h]);
    // the first layer adds the biases in the per-edge work instead: the
    // bias operands would cost it the registers of a fourth wavefront per SIMD
    const half4_t ab = L0 ? half4_t{} : bias_rows(part ? rec[e].dfc : rec[e].fc, h);
    floatx16_t m0, m1 = {}, m2;
    if constexpr (L0) {
        // the b channel gates v, zero in the first layer: nothing of it
        // reaches the forces there
        m0 = mma3<false>(ab, bbr[0], ah, al, bhr[0], blr[0]);
        m2 = mma3<false>(ab, bbr[2], ah, al, bhr[2], blr[2]);
    } else {
        half8_t bh, bl;
        half4_t bb;
        load_channel(fl, 0, bh, bl, bb);
        m0 = mma3(ab, bb, ah, al, bh, bl);
        load_channel(fl, 1, bh, bl, bb);
        m1 = mma3(ab, bb, ah, al, bh, bl);
        load_channel(fl, 2, bh, bl, bb);
        m2 = mma3(ab, bb, ah, al, bh, bl);
    }
    const uint32_t fo = uint32_t(f) * 4u;
    auto gather = [&](int g0, BwdGather<G>& d) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int q = g0 + g;
            const int te = 8 * (q / 4) + 4 * h + q % 4;
            const EdgeRec& s = rec[te < nb ? te : 0];
            const uint32_t j = uint32_t(s.j);
            const uint32_t off3 = j * (3u * F * 4u) + fo;
            if (L0) {
                const float* phj = ptab + s.t * 3 * F + f;
                d.pa[g] = phj[0];
                d.pc[g] = phj[2 * F];
            } else {
                d.pa[g] = ld_off(a.phi, off3);
                d.pc[g] = ld_off(a.phi, off3 + 2 * F * 4);
                d.pvn[g][0] = ld_off(a.pv, off3);
                d.pvn[g][1] = ld_off(a.pv, off3 + F * 4);
                d.pvn[g][2] = ld_off(a.pv, off3 + 2 * F * 4);
            }
            d.gn[g][0] = ld_off(a.gvm, off3);
            d.gn[g][1] = ld_off(a.gvm, off3 + F * 4);
            d.gn[g][2] = ld_off(a.gvm, off3 + 2 * F * 4);
            d.gsn[g] = ld_off(a.gsm, j * (F * 4u) + fo);
        }
    };
    auto reduce = [&](int g0, const BwdGather<G>& d) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int q = g0 + g;
            const int te = 8 * (q / 4) + 4 * h + q % 4;
            if (te >= nb) continue;
            const EdgeRec& s = rec[te];
            // w of edge te is row te, dw/dr row 16 + te: accumulator elements q and 8 + q
            const float ir = s.ir;
            float w0 = m0[q], w2 = m2[q], dw0 = m0[8 + q], dw2 = m2[8 + q];
            if constexpr (L0) {
                w0 = fmaf(b0[0], s.fc, w0);
                w2 = fmaf(b0[2], s.fc, w2);
                dw0 = fmaf(b0[0], s.dfc, dw0);
                dw2 = fmaf(b0[2], s.dfc, dw2);
            }
            const float u0 = s.u[0], u1 = s.u[1], u2 = s.u[2];
            const float g0v = d.gn[g][0], g1v = d.gn[g][1], g2v = d.gn[g][2];
            const float gvn_u = fmaf(g2v, u2, fmaf(g1v, u1, g0v * u0));
            const float gvo_u = fmaf(o.gv[2], u2, fmaf(o.gv[1], u1, o.gv[0] * u0));
            // filter adjoints of both messages of the pair (n -> o and o -> n),
            // contracted with dw/dr
            const float A = fmaf(o.gs, d.pa[g], o.ph[0] * d.gsn[g]);
            const float C = fmaf(d.pc[g], gvo_u, -(o.ph[2] * gvn_u));
            float dr;
            if constexpr (L0) {
                dr = fmaf(A, dw0, C * dw2);
            } else {
                const float w1 = m1[q], dw1 = m1[8 + q];
                const float gvn_vo = fmaf(g2v, o.v[2], fmaf(g1v, o.v[1], g0v * o.v[0]));
                const float gvo_pvn =
                    fmaf(o.gv[2], d.pvn[g][2], fmaf(o.gv[1], d.pvn[g][1], o.gv[0] * d.pvn[g][0]));
                const float B = fmaf(o.ph[1], gvn_vo, gvo_pvn);
                dr = fmaf(A, dw0, fmaf(B, dw1, C * dw2));
                acc.GV[0] = fmaf(w1, g0v, acc.GV[0]);
                acc.GV[1] = fmaf(w1, g1v, acc.GV[1]);
                acc.GV[2] = fmaf(w1, g2v, acc.GV[2]);
            }
            // g_u . u of the unit-vector adjoints is w2 C (the projections
            // above), so its share of the radial term is C w2 / r
            const float w2ir = w2 * ir;
            const float sv = fmaf(-C, w2ir, dr);
            acc.S1[0] = fmaf(sv, u0, acc.S1[0]);
            acc.S1[1] = fmaf(sv, u1, acc.S1[1]);
            acc.S1[2] = fmaf(sv, u2, acc.S1[2]);
            acc.T1 = fmaf(d.pc[g], w2ir, acc.T1);
            acc.T2[0] = fmaf(w2ir, g0v, acc.T2[0]);
            acc.T2[1] = fmaf(w2ir, g1v, acc.T2[1]);
            acc.T2[2] = fmaf(w2ir, g2v, acc.T2[2]);
            // o as the sender of the message o -> n
            acc.gph0 = fmaf(d.gsn[g], w0, acc.gph0);
            acc.gph2 = fmaf(-w2, gvn_u, acc.gph2);
            // r_ij . (pair force share): the projected term is normal to u
            if constexpr (VIR) acc.vir += __fdividef(dr, ir);
        }
    };
    if constexpr (L0) {
#pragma unroll
        for (int g0 = 0; g0 < E; g0 += G) {
            BwdGather<G> d;
            gather(g0, d);
            reduce(g0, d);
        }
    } else {
        BwdGather<G> d0, d1;
        gather(0, d0);
#pragma unroll
        for (int g0 = 0; g0 < E; g0 += 2 * G) {
            if (g0 + G < E) gather(g0 + G, d1);
            reduce(g0, d0);
            if (g0 + G < E) {
                if (g0 + 2 * G < E) gather(g0 + 2 * G, d0);
                reduce(g0 + G, d1);
            }
        }
    }
}

template <bool L0, bool VIR>
__global__ void __launch_bounds__(64 * kMxWaves, 3) k_message_bwd_mx(MpGeom mg, MpBwd a) {
    constexpr int F = kMxF, BATCH = 16;
    __shared__ __align__(16) BatchBuf<BATCH> buf[2];
    __shared__ float fpart[kMxAtoms][kMxWaves][4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int h = lane >> 5, f = w * 32 + (lane & 31);
    const int n = mg.n;
    // first layer: the species table of phi in LDS
    __shared__ float ptab_s[L0 ? 8 * 3 * kMxF : 1];
    if constexpr (L0) {
        for (int t = threadIdx.x; t < mg.n_species * 3 * F; t += blockDim.x) ptab_s[t] = a.phi_tab[t];
        __syncthreads();
    }
    const float sc = a.mx_scale[0], isc = a.mx_scale[1];
    // this lane's split filter operands: past the first layer kept in LDS
    // between the batches, in the first layer in registers
    __shared__ __align__(16) uint4 filt_s[L0 ? 1 : kMxWaves][L0 ? 1 : kFiltPieces][64];
    uint4* fl = L0 ? nullptr : &filt_s[L0 ? 0 : w][0][lane];
    half8_t bh[3], bl[3];
    half4_t bb[3];
    load_filter(a.Wr, a.br, sc, f, h, bh, bl, bb);
    if constexpr (!L0) {
        store_filter(fl, bh, bl, bb);
        wave_sync_lds();
    }
    float bf[3] = {};  // the scaled biases, for the first layer's per-edge work
    if constexpr (L0) {
#pragma unroll
        for (int p = 0; p < 3; ++p) bf[p] = a.br[p * F + f] * sc;
    }
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int i0 = blk * kMxAtoms;
    NextBatch nx = next_batch<BATCH>(mg, i0, -1, 0, 0);
    uint4 piece = fetch_piece<BATCH>(mg, nx.p0, nx.nb);
    int k = 0;  // batches of the block so far (LDS buffer parity)
    for (int ai = 0; ai < kMxAtoms; ++ai) {
        const int i = i0 + ai;
        if (i >= n) break;
        const int cnt = mg.ecnt[i];
        Owner o{};
        {
            const int ti = L0 ? min(max(a.species[i], 0), mg.n_species - 1) : 0;
            const float* pho = L0 ? ptab_s + ti * 3 * F + f : a.phi + int64_t(i) * 3 * F + f;
#pragma unroll
            for (int p = 0; p < 3; ++p) o.ph[p] = pho[p * F];
#pragma unroll
            for (int al = 0; al < 3; ++al) {
                const int64_t idx = (int64_t(i) * 3 + al) * F + f;
                if (!L0) o.v[al] = a.v_in[idx];
                o.gv[al] = a.gvm[idx];
            }
            o.gs = a.gsm[int64_t(i) * F + f];
        }
        BwdAcc acc{};
        for (int b0 = 0; b0 < cnt; b0 += BATCH, ++k) {
            BatchBuf<BATCH>& b = buf[k & 1];
            store_piece(b, piece);
            __syncthreads();  // the batch is staged; the other buffer's batch is done
            nx = next_batch<BATCH>(mg, i0, ai, b0, cnt);
            piece = fetch_piece<BATCH>(mg, nx.p0, nx.nb);
            bwd_batch<L0, VIR>(a, ptab_s, b, min(BATCH, cnt - b0), f, h, fl, bh, bl, bb, bf, o, acc);
        }
        // the lane's force share, then both halves of the wavefront (partial
        // sums of feature f) and the features of the wavefront
        float fs[3];
#pragma unroll
        for (int al = 0; al < 3; ++al) fs[al] = fmaf(o.gv[al], acc.T1, fmaf(-o.ph[2], acc.T2[al], acc.S1[al]));
        acc.gph0 += __shfl_xor(acc.gph0, 32, 64);
        acc.gph2 += __shfl_xor(acc.gph2, 32, 64);
#pragma unroll
        for (int p = 0; p < 3; ++p) acc.GV[p] += __shfl_xor(acc.GV[p], 32, 64);
        const float gph[3] = {acc.gph0, fmaf(o.v[2], acc.GV[2], fmaf(o.v[1], acc.GV[1], o.v[0] * acc.GV[0])),
                              acc.gph2};
        const float fx = group_sum<64>(fs[0]), fy = group_sum<64>(fs[1]), fz = group_sum<64>(fs[2]);
        const float vr = VIR ? group_sum<64>(acc.vir) : 0.f;
        if (lane == 0) {
            fpart[ai][w][0] = fx;
            fpart[ai][w][1] = fy;
            fpart[ai][w][2] = fz;
            fpart[ai][w][3] = vr;
        }
        if (h == 0) {
            if (a.want_gphi) {
#pragma unroll
                for (int p = 0; p < 3; ++p) a.gphi[int64_t(i) * 3 * F + p * F + f] = gph[p] * isc;
            }
            if (!L0) {
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                    const int64_t idx = (int64_t(i) * 3 + al) * F + f;
                    a.gv_in[idx] = o.gv[al] + (o.ph[1] * acc.GV[al]) * isc;
                }
            }
        }
    }
    __syncthreads();
    // the force (and virial share) of each atom of the block: the feature
    // blocks' shares in a fixed order
    const int t = threadIdx.x;
    if (t < 4 * kMxAtoms) {
        const int ai = t / 4, c = t % 4;
        const int i = i0 + ai;
        if (i < n && (c < 3 || VIR)) {
            float sum = 0.f;
            for (int k = 0; k < kMxWaves; ++k) sum += fpart[ai][k][c];
            sum *= isc;
            const int io = mg.perm ? min(max(mg.perm[i], 0), n - 1) : i;
            float* fo = c < 3 ? a.force + int64_t(c) * n + io : a.vir + io;
            if (c == 3) sum *= 0.5f;  // each pair is seen by both of its atoms
            if (a.accum_force) *fo += sum;
            else *fo = sum;
        }
    }
}

// Scale of the filter weights and biases of one layer for the split
// products: a power of two s with max(|Wr|, |br|) s in [2^13, 2^14) (s = 1
// when all are zero), and 1 / s.  Wr and br are contiguous in the weights.
__global__ void __launch_bounds__(256) k_filter_scale(int count, const float* Wr, float* out) {
    __shared__ float part[256];
    float m = 0.f;
    for (int k = threadIdx.x; k < count; k += blockDim.x) m = fmaxf(m, fabsf(Wr[k]));
    part[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) part[threadIdx.x] = fmaxf(part[threadIdx.x], part[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float mx = part[0];
        int e = 0;
        if (mx > 0.f && isfinite(mx)) (void)frexpf(mx, &e);  // mx < 2^e
        e = min(max(e, -100), 100);
        out[0] = ldexpf(1.f, 14 - e);
        out[1] = ldexpf(1.f, e - 14);
    }
}

// pv[i][al][f] = phi[i][F + f] * v[i][al][f]: one thread per four features
// of an atom.
__global__ void __launch_bounds__(256) k_phib_v(int n, const float* __restrict__ phi, const float* __restrict__ v,
                                                float* __restrict__ pv) {
    constexpr int F = kMxF, C = F / 4;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n) * C) return;
    const int64_t i = t / C;
    const int c = int(t % C);
    const float4 b = reinterpret_cast<const float4*>(phi + i * 3 * F + F)[c];
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const int64_t row = (i * 3 + al) * F;
        const float4 x = reinterpret_cast<const float4*>(v + row)[c];
        reinterpret_cast<float4*>(pv + row)[c] = make_float4(b.x * x.x, b.y * x.y, b.z * x.z, b.w * x.w);
    }
}

template <typename Kern, typename Args>
void launch_mx(const ScopedTimer& t, Kern kern, int n, hipStream_t s, const MpGeom& mg, const Args& a) {
    const dim3 grid(cdiv(n, kMxAtoms));
    if (t.active && t.by_launch) hipExtLaunchKernelGGL(kern, grid, dim3(64 * kMxWaves), 0, s, t.a, t.b, 0, mg, a);
    else kern<<<grid, 64 * kMxWaves, 0, s>>>(mg, a);
}

}  // namespace

bool message_mx_shape(int F, int K, int cut) { return F == kMxF && K == kMxK && cut == 0; }

void launch_message_fwd_mx(const MpGeom& mg, const MpFwd& a, hipStream_t s, const ScopedTimer& t) {
    if (a.phi_tab) {
        launch_mx(t, k_message_fwd_mx<true>, mg.n, s, mg, a);
        return;
    }
    if (!a.pv) {
        set_error("matrix-core message step: no phi_b * v buffer");
        throw Fail{NNP_EINVAL};
    }
    k_phib_v<<<cdiv(int64_t(mg.n) * (kMxF / 4), 256), 256, 0, s>>>(mg.n, a.phi, a.v_in, a.pv);
    launch_mx(t, k_message_fwd_mx<false>, mg.n, s, mg, a);
}

void launch_message_bwd_mx(const MpGeom& mg, const MpBwd& a, hipStream_t s, const ScopedTimer& t) {
    if (!a.phi_tab && !a.pv) {
        set_error("matrix-core message reverse: no phi_b * v buffer");
        throw Fail{NNP_EINVAL};
    }
    if (a.vir) {
        if (a.phi_tab) launch_mx(t, k_message_bwd_mx<true, true>, mg.n, s, mg, a);
        else launch_mx(t, k_message_bwd_mx<false, true>, mg.n, s, mg, a);
    } else {
        if (a.phi_tab) launch_mx(t, k_message_bwd_mx<true, false>, mg.n, s, mg, a);
        else launch_mx(t, k_message_bwd_mx<false, false>, mg.n, s, mg, a);
    }
}

void launch_edge_prep(const MpGeom& mg, int* ecnt, EdgeRec* erec, uint4* ehalf, hipStream_t s, float* Es, float* Ev,
                      int S, int ep) {
    if (mg.n <= 0) return;
    const dim3 grid(cdiv(mg.n, 4));
    if (!Es) k_edge_prep<0><<<grid, 256, 0, s>>>(mg, ecnt, erec, ehalf, nullptr, nullptr, 0, 0);
    else if (S <= 2) k_edge_prep<2><<<grid, 256, 0, s>>>(mg, ecnt, erec, ehalf, Es, Ev, S, ep);
    else if (S <= 4) k_edge_prep<4><<<grid, 256, 0, s>>>(mg, ecnt, erec, ehalf, Es, Ev, S, ep);
    else k_edge_prep<8><<<grid, 256, 0, s>>>(mg, ecnt, erec, ehalf, Es, Ev, S, ep);
    NNP_LAUNCH_CHECK();
}

void launch_filter_scale(int count, const float* Wr, float* out, hipStream_t s) {
    k_filter_scale<<<1, 256, 0, s>>>(count, Wr, out);
    NNP_LAUNCH_CHECK();
}

}  // namespace nnp
