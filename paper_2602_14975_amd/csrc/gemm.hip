// Dense per-atom contractions (the perceptrons of both models).
//
// C(m, n) = epi( sum_k A(m, k) B(k, n) + bias(n) ) with strided operands.
// Two kernel families:
//  * k_gemm_x3 (the products X W^T of the force evaluation, K of 128, 256 or
//    384): bfloat16 matrix cores, FP32 models through operands split into
//    three bfloat16 pieces, BF16 models through rounded operands;
//  * k_gemm / k_gemm_rk (other shapes, the weight adjoints G^T X by chunks
//    of rows, and everything when the older kernels are selected): float32
//    (or bfloat16-rounded) operands on the matrix cores, LDS-staged 64 x 64
//    tiles or register-direct 32-wide strips.
//
// Epilogues: SILU stores the pre-activation (for the reverse pass) and
// writes silu(y); DSILU multiplies by silu'(pre(m, n)); ACCUM adds into C.
#include <atomic>

#include "common.h"
#include "kernels.h"
#include "model.h"

namespace nnp {

constexpr int TM = 64, TN = 64;

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef short short4_t __attribute__((ext_vector_type(4)));

// float32 -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ short bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return short(u >> 16);
}

// One 64 x 64 output tile per block of four wavefronts; wavefront w owns the
// 32 x 32 sub-tile (w / 2, w % 2) and accumulates it with MFMA in float32:
// v_mfma_f32_32x32x2f32 (operands float32) or v_mfma_f32_32x32x8bf16_1k
// (operands rounded to bfloat16).  Operand lane layout of the 32 x 32 x k
// instructions: lane l supplies row (col) l % 32 and k-group l / 32; the
// accumulator holds column l % 32, rows 8 (r / 4) + 4 (l / 32) + r % 4.
template <bool BF16>
__global__ void __launch_bounds__(256)
k_gemm(GemmArgs g) {
    constexpr int TK = 32;
    constexpr int PER = TM * TK / 256;  // staged elements per thread and operand
    __shared__ float As[TK][TM + 4];
    __shared__ float Bs[TK][TN + 4];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    // 1-D launches (no row chunks) number tiles so that each XCD gets a
    // contiguous run, column tile fastest: the A rows of a run stay in its L2.
    int bm = blockIdx.x, bn = blockIdx.y;
    if (g.chunk_rows == 0) {
        const int NT = (g.N + TN - 1) / TN;
        const int L = xcd_block(blockIdx.x, gridDim.x);
        bm = L / NT;
        bn = L % NT;
    }
    const int m0 = bm * TM, n0 = bn * TN;
    int kbeg = 0, kend = g.K;
    if (g.chunk_rows > 0) {
        kbeg = int(int64_t(blockIdx.z) * g.chunk_rows);
        kend = min(g.K, int(int64_t(blockIdx.z) * g.chunk_rows + g.chunk_rows));
    }
    // Element t of a staged tile: along k when that is the contiguous
    // dimension of the operand (coalesced), along m / n otherwise.
    float ra[PER], rb[PER];
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int t = tid + u * 256;
            int mm, kk;
            if (g.sak == 1) { mm = t / TK; kk = t % TK; } else { kk = t / TM; mm = t % TM; }
            const int m = m0 + mm, k = k0 + kk;
            ra[u] = (m < g.M && k < kend) ? g.A[int64_t(m) * g.sam + int64_t(k) * g.sak] : 0.f;
            int nn, kb;
            if (g.sbk == 1) { nn = t / TK; kb = t % TK; } else { kb = t / TN; nn = t % TN; }
            const int nc = n0 + nn, kc = k0 + kb;
            rb[u] = (nc < g.N && kc < kend) ? g.B[int64_t(kc) * g.sbk + int64_t(nc) * g.sbn] : 0.f;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int t = tid + u * 256;
            int mm, kk;
            if (g.sak == 1) { mm = t / TK; kk = t % TK; } else { kk = t / TM; mm = t % TM; }
            As[kk][mm] = ra[u];
            int nn, kb;
            if (g.sbk == 1) { nn = t / TK; kb = t % TK; } else { kb = t / TN; nn = t % TN; }
            Bs[kb][nn] = rb[u];
        }
    };
    floatx16 acc = {};
    const int row = lane & 31, grp = lane >> 5;
    if (kbeg < kend) load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
        store();
        __syncthreads();
        if (k0 + TK < kend) load(k0 + TK);  // next tile in flight during the MFMAs
        if constexpr (BF16) {
#pragma unroll
            for (int kk = 0; kk < TK; kk += 8) {
                short4_t a, b;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    a[q] = bf16_bits(As[kk + 4 * grp + q][wr + row]);
                    b[q] = bf16_bits(Bs[kk + 4 * grp + q][wc + row]);
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < TK; kk += 2)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(As[kk + grp][wr + row], Bs[kk + grp][wc + row], acc, 0,
                                                           0, 0);
        }
        __syncthreads();
    }
    float* C = g.C + int64_t(blockIdx.z) * g.chunk_stride;
    const int col = n0 + wc + (lane & 31);
    if (col >= g.N) return;
    const float bias = g.bias ? g.bias[col] : 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = m0 + wr + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        if (m >= g.M) continue;
        float y = acc[r] + bias;
        const int64_t idx = int64_t(m) * g.ldc + col;
        if (g.epi == EPI_SILU) {
            if (g.pre) g.pre[int64_t(m) * g.ldp + col] = y;
            y = silu(y);
        } else if (g.epi == EPI_DSILU) {
            y *= silu_grad(g.pre[int64_t(m) * g.ldp + col]);
        }
        if (g.accum) y += C[idx];
        C[idx] = y;
    }
}

// Register-direct variant for operands whose k index is contiguous in both
// A (A(m, k) = A[m * sam + k]) and B (B(k, n) = B[n * sbn + k]): no LDS
// staging and no barriers in the k loop.  Within each 32-deep slice the
// MFMA k slots are permuted so that every lane reads 16 consecutive k values
// of its own row with four float4 loads; A and B use the same permutation,
// so each product term A(m, k) B(k, n) appears exactly once.  A block of S
// wavefronts shares one 32 x 32T output strip: wavefront w takes slices
// w, w + S, ... and the partial sums are added in wavefront order (fixed,
// so results are reproducible).
template <int T, int S, bool BF16>
__global__ void __launch_bounds__(64 * S) k_gemm_rk(GemmArgs g) {
    __shared__ float red[S > 1 ? S - 1 : 1][T][16][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 31, h = lane >> 5;
    const int NT = (g.N + 32 * T - 1) / (32 * T);
    const int L = xcd_block(blockIdx.x, gridDim.x);  // column strip fastest within an XCD's run
    const int m0 = (L / NT) * 32, n0 = (L % NT) * (32 * T);
    const bool mok = m0 + r < g.M;
    const float* arow = g.A + (mok ? int64_t(m0 + r) * g.sam : 0);
    const float* brow[T];
    bool nok[T];
    // rows from b_split on take the second operand (b_split a multiple of 32)
    const float* B = (g.B2 && m0 >= g.b_split) ? g.B2 : g.B;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        nok[t] = n0 + 32 * t + r < g.N;
        brow[t] = B + (nok[t] ? int64_t(n0 + 32 * t + r) * g.sbn : 0);
    }
    floatx16 acc[T];
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = floatx16{};
    const int nsl = (g.K + 31) / 32;
    float4 a[4], b[T][4];
    auto load = [&](int c, float4* pa, float4 (*pb)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = c * 32 + 16 * h + 4 * q;
            const bool kok = k < g.K;  // K % 4 == 0: a float4 is wholly in or out
            pa[q] = (mok && kok) ? *reinterpret_cast<const float4*>(arow + k) : float4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < T; ++t)
                pb[t][q] = (nok[t] && kok) ? *reinterpret_cast<const float4*>(brow[t] + k)
                                           : float4{0.f, 0.f, 0.f, 0.f};
        }
    };
    auto slice = [&](const float4* pa, const float4 (*pb)[4]) {
        if constexpr (BF16) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                short4_t av = {bf16_bits(pa[q].x), bf16_bits(pa[q].y), bf16_bits(pa[q].z), bf16_bits(pa[q].w)};
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    short4_t bv = {bf16_bits(pb[t][q].x), bf16_bits(pb[t][q].y), bf16_bits(pb[t][q].z),
                                   bf16_bits(pb[t][q].w)};
                    acc[t] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc[t], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float av[4] = {pa[q].x, pa[q].y, pa[q].z, pa[q].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
#pragma unroll
                    for (int t = 0; t < T; ++t) {
                        const float bv[4] = {pb[t][q].x, pb[t][q].y, pb[t][q].z, pb[t][q].w};
                        acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[e], bv[e], acc[t], 0, 0, 0);
                    }
                }
            }
        }
    };
    int c = wave;
    if (c < nsl) load(c, a, b);
    for (; c < nsl; c += S) {
        float4 an[4], bn[T][4];
        const bool more = c + S < nsl;
        if (more) load(c + S, an, bn);  // next slice in flight during the MFMAs
        slice(a, b);
        if (more) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = an[q];
#pragma unroll
                for (int t = 0; t < T; ++t) b[t][q] = bn[t][q];
            }
        }
    }
    if constexpr (S > 1) {
        if (wave > 0) {
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int i = 0; i < 16; ++i) red[wave - 1][t][i][lane] = acc[t][i];
        }
        __syncthreads();
        if (wave > 0) return;
#pragma unroll
        for (int w = 0; w < S - 1; ++w)
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[t][i] += red[w][t][i][lane];
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int col = n0 + 32 * t + r;
        if (col >= g.N) continue;
        const float bias = g.bias ? g.bias[col] : 0.f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = m0 + (i >> 2) * 8 + h * 4 + (i & 3);
            if (m >= g.M) continue;
            float y = acc[t][i] + bias;
            const int64_t idx = int64_t(m) * g.ldc + col;
            if (g.epi == EPI_SILU) {
                if (g.pre) g.pre[int64_t(m) * g.ldp + col] = y;
                y = silu(y);
            } else if (g.epi == EPI_DSILU) {
                y *= silu_grad(g.pre[int64_t(m) * g.ldp + col]);
            }
            if (g.accum) y += g.C[idx];
            g.C[idx] = y;
        }
    }
}


// FP32 products on bfloat16 matrix cores.  Each operand is split into three
// bfloat16 pieces, x = x_h + x_m + x_l (each piece the round-to-nearest of
// what the previous ones leave), so that x_h carries 8 significant bits,
// x_h + x_m 16 and x_h + x_m + x_l 24.  Of the nine piece products the six
// of order >= 2^-18 are accumulated in float32 (hh, hm, mh, hl, lh, mm); the
// dropped ones are below 2^-26 relative, under float32 rounding itself.
// The right operand (weights, [N][K]) is split once when the weights change;
// the left one (activations) on the fly from float32.  BF16 models take the
// first piece alone (the operands rounded to bfloat16, one product).
//
// One block of four wavefronts computes 128 rows x 32T columns over the
// whole K.  The weight pieces of its columns (3 x 32T rows of K bfloat16)
// are staged in LDS once, all loads issued together; after that single
// barrier each wavefront streams its own 32 activation rows in 32-deep
// chunks straight into registers (a lane reads 16 consecutive k of its
// row), RING - 1 chunks in flight ahead of the one being multiplied.  MFMA
// v_mfma_f32_32x32x16_bf16; operand slot i of k-step j in lane half h holds
// k = 16h + 8j + i of the chunk, for both operands alike, so every product
// term appears once.  Accumulator layout as in k_gemm.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_v __attribute__((ext_vector_type(4)));

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Two floats rounded to nearest bfloat16, packed (element 0 in the low half).
__device__ __forceinline__ uint32_t pack_bf16(f32x2_t x) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(x, bf16x2_t));
}

// The float values of a packed pair: a bfloat16 is the high half of its float.
__device__ __forceinline__ f32x2_t unpack_bf16(uint32_t p) {
    return f32x2_t{__uint_as_float(p << 16), __uint_as_float(p & 0xFFFF0000u)};
}

// Pairs of elements are rounded with one packed conversion and taken back
// apart with a shift and a mask, so each piece costs half a conversion, one
// bit operation and one subtraction per element.
__device__ __forceinline__ void split3(const float (&x)[8], bf16x8_t& h, bf16x8_t& m, bf16x8_t& l) {
    u32x4_v hw, mw, lw;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const f32x2_t a{x[2 * p], x[2 * p + 1]};
        const uint32_t ph = pack_bf16(a);
        const f32x2_t r1 = a - unpack_bf16(ph);  // exact
        const uint32_t pm = pack_bf16(r1);
        const f32x2_t r2 = r1 - unpack_bf16(pm);  // exact
        hw[p] = ph;
        mw[p] = pm;
        lw[p] = pack_bf16(r2);
    }
    h = __builtin_bit_cast(bf16x8_t, hw);
    m = __builtin_bit_cast(bf16x8_t, mw);
    l = __builtin_bit_cast(bf16x8_t, lw);
}

// The piece products of one 32-deep chunk: activations av (this lane's 16 k
// values) against the staged weight pieces; B points at this lane's column
// (r) and k offset (16 h) of the chunk in piece 0.  NP = 3: the six products
// of the split operands (FP32 models); NP = 1: the product of the operands
// rounded to bfloat16 (BF16 models).
template <int T, int J, int PITCH, int NP>
__device__ __forceinline__ void x3_products(floatx16 (&acc)[J][T], const f32x4_t (&av)[4], const uint16_t* B) {
    constexpr int PIECE = 32 * T * PITCH;
#pragma unroll
    for (int j0 = 0; j0 < 2; j0 += J) {
        bf16x8_t ah[J], am[J], al[J], bh[J][T], bm[J][T], bl[J][T];
#pragma unroll
        for (int jj = 0; jj < J; ++jj) {
            const int j = j0 + jj;
            const float x[8] = {av[2 * j].x,     av[2 * j].y,     av[2 * j].z,     av[2 * j].w,
                                av[2 * j + 1].x, av[2 * j + 1].y, av[2 * j + 1].z, av[2 * j + 1].w};
            if constexpr (NP == 3) {
                split3(x, ah[jj], am[jj], al[jj]);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) ah[jj][i] = __bf16(x[i]);
            }
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const uint16_t* b = B + 32 * t * PITCH + 8 * j;
                bh[jj][t] = *reinterpret_cast<const bf16x8_t*>(b);
                if constexpr (NP == 3) {
                    bm[jj][t] = *reinterpret_cast<const bf16x8_t*>(b + PIECE);
                    bl[jj][t] = *reinterpret_cast<const bf16x8_t*>(b + 2 * PIECE);
                }
            }
        }
        // smallest terms first; independent accumulators between dependent ones
#define NNP_X3_TERM(AX, BX)                                                                                    \
    _Pragma("unroll") for (int jj = 0; jj < J; ++jj) _Pragma("unroll") for (int t = 0; t < T; ++t) acc[jj][t] = \
        __builtin_amdgcn_mfma_f32_32x32x16_bf16(AX[jj], BX[jj][t], acc[jj][t], 0, 0, 0);
        if constexpr (NP == 3) {
            NNP_X3_TERM(al, bh)
            NNP_X3_TERM(ah, bl)
            NNP_X3_TERM(am, bm)
            NNP_X3_TERM(am, bh)
            NNP_X3_TERM(ah, bm)
        }
        NNP_X3_TERM(ah, bh)
#undef NNP_X3_TERM
    }
}

template <int T, int KK, int RING, int NP>
__global__ void __launch_bounds__(256) k_gemm_x3(GemmArgs g) {
    constexpr int BN = 32 * T;
    constexpr int PITCH = KK + 8;   // bfloat16 per staged row: 4-bank shift per row, conflict-free 16-byte reads
    constexpr int NCH = KK / 32;    // chunks
    constexpr int RU = KK / 8;      // 16-byte units per staged row
    constexpr int UNITS = NP * BN * RU;
    constexpr int UPT = UNITS / 256;
    constexpr int J = T == 1 ? 2 : 1;  // k-steps issued together (independent accumulators for T = 1)
    static_assert(NCH % RING == 0 && UNITS % 256 == 0, "shape");
    __shared__ __align__(16) uint16_t Bs[NP * BN * PITCH];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 31, h = lane >> 5;
    const int NT = g.N / BN;
    const int L = xcd_block(blockIdx.x, gridDim.x);  // column tiles of a row tile stay on one XCD
    const int m0 = (L / NT) * 128 + wave * 32, n0 = (L % NT) * BN;
    // rows past M read row M - 1 (unconditional loads keep the waits exact)
    // and are never stored
    const float* arow = g.A + int64_t(min(m0 + r, g.M - 1)) * g.sam + 16 * h;
    // row tiles from b_split on take the second set of pieces
    const uint16_t* Bx = (g.Bx2 && (L / NT) * 128 >= g.b_split) ? g.Bx2 : g.Bx;

#define NNP_X3_LOAD_A(DST, C) \
    _Pragma("unroll") for (int q = 0; q < 4; ++q) DST[q] = *reinterpret_cast<const f32x4_t*>(arow + (C) * 32 + 4 * q);
    f32x4_t ring[RING][4];
#pragma unroll
    for (int s = 0; s < RING - 1; ++s) NNP_X3_LOAD_A(ring[s], s)
    {
        // weight pieces of the block's columns, all of K: unit idx is piece
        // idx / (BN RU), column (idx / RU) % BN, k 8 (idx % RU)
        u32x4_v tmp[UPT];
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            const int idx = u * 256 + tid;
            const int p = idx / (BN * RU), col = (idx / RU) % BN, q = idx % RU;
            tmp[u] = *reinterpret_cast<const u32x4_v*>(Bx + p * g.bxs + int64_t(n0 + col) * KK + 8 * q);
        }
#pragma unroll
        for (int u = 0; u < UPT; ++u) {
            const int idx = u * 256 + tid;
            const int p = idx / (BN * RU), col = (idx / RU) % BN, q = idx % RU;
            *reinterpret_cast<u32x4_v*>(&Bs[(p * BN + col) * PITCH + 8 * q]) = tmp[u];
        }
    }
    __syncthreads();

    floatx16 acc[J][T];
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
        for (int t = 0; t < T; ++t) acc[j][t] = floatx16{};
    const uint16_t* Bl = Bs + r * PITCH + 16 * h;
    // register sets in rotation: each step loads the chunk RING - 1 ahead
    // (past the end: the last chunk again, never used) and multiplies one
    for (int c = 0; c < NCH; c += RING) {
#pragma unroll
        for (int s = 0; s < RING; ++s) {
            NNP_X3_LOAD_A(ring[(s + RING - 1) % RING], min(c + s + RING - 1, NCH - 1))
            __builtin_amdgcn_sched_barrier(0);
            x3_products<T, J, PITCH, NP>(acc, ring[s], Bl + (c + s) * 32);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#undef NNP_X3_LOAD_A
    if constexpr (J == 2) {
#pragma unroll
        for (int t = 0; t < T; ++t) acc[0][t] += acc[1][t];
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int col = n0 + 32 * t + r;
        const float bias = g.bias ? g.bias[col] : 0.f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = m0 + (i >> 2) * 8 + h * 4 + (i & 3);
            if (m >= g.M) continue;
            float y = acc[0][t][i] + bias;
            const int64_t idx = int64_t(m) * g.ldc + col;
            // streaming stores: the outputs are not read again by this kernel
            if (g.epi == EPI_SILU) {
                if (g.pre) __builtin_nontemporal_store(y, &g.pre[int64_t(m) * g.ldp + col]);
                y = silu(y);
            } else if (g.epi == EPI_DSILU) {
                y *= silu_grad(g.pre[int64_t(m) * g.ldp + col]);
            }
            if (g.accum) y += g.C[idx];
            __builtin_nontemporal_store(y, &g.C[idx]);
        }
    }
}

// Shapes and alignment the split-bfloat16 kernel assumes: k contiguous in A
// with 16-byte aligned rows, K one of 128, 256, 384, N a multiple of 32, the
// weight pieces present and 16-byte aligned (for BF16 models only the
// first piece, the rounded weights, is read).
static bool x3_ok(const GemmArgs& g) {
    return g.Bx && g.chunk_rows == 0 && g.sak == 1 && g.sam % 4 == 0 &&
           (g.K == 128 || g.K == 256 || g.K == 384) && g.N % 32 == 0 && g.bxs % 8 == 0 &&
           (reinterpret_cast<uintptr_t>(g.A) & 15) == 0 && (reinterpret_cast<uintptr_t>(g.Bx) & 15) == 0;
}

static int x3_blocks(const GemmArgs& g, int T) { return cdiv(g.M, 128) * (g.N / (32 * T)); }

static void x3_launch(const GemmArgs& g, hipStream_t stream) {
    // 64 columns per block where K = 128 (52 KB of staged weights) and that
    // still gives two blocks per compute unit; 32 otherwise
    const bool wide = g.K == 128 && g.N % 64 == 0 && x3_blocks(g, 2) >= 512;
    const dim3 grid(x3_blocks(g, wide ? 2 : 1));
    if (g.bf16) {  // BF16 models: the rounded operands, one product
        if (wide) k_gemm_x3<2, 128, 4, 1><<<grid, 256, 0, stream>>>(g);
        else if (g.K == 128) k_gemm_x3<1, 128, 4, 1><<<grid, 256, 0, stream>>>(g);
        else if (g.K == 256) k_gemm_x3<1, 256, 4, 1><<<grid, 256, 0, stream>>>(g);
        else k_gemm_x3<1, 384, 4, 1><<<grid, 256, 0, stream>>>(g);
    } else {
        if (wide) k_gemm_x3<2, 128, 4, 3><<<grid, 256, 0, stream>>>(g);
        else if (g.K == 128) k_gemm_x3<1, 128, 4, 3><<<grid, 256, 0, stream>>>(g);
        else if (g.K == 256) k_gemm_x3<1, 256, 4, 3><<<grid, 256, 0, stream>>>(g);
        else k_gemm_x3<1, 384, 4, 3><<<grid, 256, 0, stream>>>(g);
    }
}

__global__ void k_split3(const float* __restrict__ src, int64_t count, __bf16* __restrict__ dst, int64_t ps) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const float x = src[e];
    const __bf16 a = __bf16(x);
    const float r1 = x - float(a);
    const __bf16 b = __bf16(r1);
    dst[e] = a;
    dst[ps + e] = b;
    dst[2 * ps + e] = __bf16(r1 - float(b));
}

void launch_split3(const float* src, int64_t count, uint16_t* dst, int64_t piece_stride, hipStream_t s) {
    if (count <= 0) return;
    k_split3<<<cdiv(count, 256), 256, 0, s>>>(src, count, reinterpret_cast<__bf16*>(dst), piece_stride);
    NNP_LAUNCH_CHECK();
}

static std::atomic<int> g_dense_mode{0};
void set_dense_mode(int mode) { g_dense_mode.store(mode); }

// Operands qualify for k_gemm_rk when k is contiguous in both, K and the row
// strides are multiples of 4 and the bases 16-byte aligned.
static bool rk_ok(const GemmArgs& g) {
    return g.sak == 1 && g.sbk == 1 && g.K % 4 == 0 && g.sam % 4 == 0 && g.sbn % 4 == 0 &&
           (reinterpret_cast<uintptr_t>(g.A) & 15) == 0 && (reinterpret_cast<uintptr_t>(g.B) & 15) == 0 &&
           g.chunk_rows == 0;
}

template <int T, int S>
static void rk_launch(const GemmArgs& g, hipStream_t stream) {
    dim3 grid(cdiv(g.M, 32) * cdiv(g.N, 32 * T));
    if (g.bf16) k_gemm_rk<T, S, true><<<grid, 64 * S, 0, stream>>>(g);
    else k_gemm_rk<T, S, false><<<grid, 64 * S, 0, stream>>>(g);
}

static void gemm_dispatch(const GemmArgs& g, dim3 grid, hipStream_t stream) {
    if (g.bf16) k_gemm<true><<<grid, 256, 0, stream>>>(g);
    else k_gemm<false><<<grid, 256, 0, stream>>>(g);
}

void launch_gemm(const GemmArgs& g, hipStream_t stream) {
    if (g.M <= 0 || g.N <= 0) return;
    ScopedTimer timer("gemm", stream);
    if (g_dense_mode.load() == 0 && x3_ok(g)) {
        x3_launch(g, stream);
    } else if (g.N <= 160 && rk_ok(g)) {
        // narrow outputs: more, smaller tiles and k split over the block's
        // wavefronts fill the chip better than 64 x 64 tiles
        if (g.K >= 128) rk_launch<1, 4>(g, stream);
        else rk_launch<1, 1>(g, stream);
    } else {
        dim3 grid(cdiv(g.M, TM) * cdiv(g.N, TN), 1, 1);
        gemm_dispatch(g, grid, stream);
    }
    NNP_LAUNCH_CHECK();
}

// out = X W^T + b (X [M][K] row-major, W [N][K]), optional SiLU (saving pre).
void gemm_xwt(int M, int N, int K, const float* X, int ldx, const float* W, const float* b, float* out,
              int ldo, int epi, float* pre, int ldp, bool accum, hipStream_t s, bool bf16, const uint16_t* Wx,
              int64_t wx_stride) {
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K;
    g.A = X; g.sam = ldx; g.sak = 1;
    g.B = W; g.sbk = 1; g.sbn = K;
    g.C = out; g.ldc = ldo; g.bias = b; g.epi = epi; g.pre = pre; g.ldp = ldp; g.accum = accum;
    g.bf16 = bf16;
    g.Bx = Wx; g.bxs = wx_stride;
    launch_gemm(g, s);
}

bool gemm_x3_split(int M, int N, int K, const float* X, int ldx, const uint16_t* Wx, const uint16_t* Wx2,
                   int64_t wx_stride, int m_split, float* out, int ldo, hipStream_t s) {
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K;
    g.A = X; g.sam = ldx; g.sak = 1;
    g.sbk = 1; g.sbn = K;
    g.C = out; g.ldc = ldo; g.epi = EPI_NONE;
    g.Bx = Wx; g.bxs = wx_stride;
    g.Bx2 = Wx2; g.b_split = m_split;
    if (g_dense_mode.load() != 0 || m_split % 128 != 0 || !Wx2 || (reinterpret_cast<uintptr_t>(Wx2) & 15) != 0 ||
        !x3_ok(g))
        return false;
    if (M <= 0) return true;
    ScopedTimer timer("gemm", s);
    x3_launch(g, s);
    NNP_LAUNCH_CHECK();
    return true;
}

void gemm_xwt_f32_split(int M, int N, int K, const float* X, int ldx, const float* W, const float* W2, int m_split,
                        float* out, int ldo, hipStream_t s) {
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K;
    g.A = X; g.sam = ldx; g.sak = 1;
    g.B = W; g.sbk = 1; g.sbn = K;
    g.B2 = W2; g.b_split = m_split;
    g.C = out; g.ldc = ldo; g.epi = EPI_NONE;
    if (M <= 0 || N <= 0) return;
    if (m_split % 32 != 0 || !rk_ok(g) || N > 160) {
        set_error("gemm_xwt_f32_split: unsupported shape");
        throw Fail{NNP_EINVAL};
    }
    ScopedTimer timer("gemm", s);
    // one block per 32 rows and all N columns (N = 128: one wavefront over
    // all of K; N <= 160 with K >= 128: K split over four wavefronts);
    // otherwise one 32-column strip per block
    const int T = cdiv(N, 32);
    if (T == 4) rk_launch<4, 1>(g, s);
    else if (K >= 128 && T <= 2) rk_launch<2, 4>(g, s);
    else if (K >= 128 && T == 3) rk_launch<3, 4>(g, s);
    else if (K >= 128) rk_launch<5, 4>(g, s);
    else rk_launch<1, 1>(g, s);
    NNP_LAUNCH_CHECK();
}

// out = G W (G [M][N] row-major, W [N][K]) -> [M][K]; optional silu'(pre) factor.
void gemm_gw(int M, int N, int K, const float* G, int ldg, const float* W, float* out, int ldo, int epi,
             const float* pre, int ldp, bool accum, hipStream_t s, bool bf16) {
    GemmArgs g{};
    g.M = M; g.N = K; g.K = N;
    g.A = G; g.sam = ldg; g.sak = 1;
    g.B = W; g.sbk = K; g.sbn = 1;
    g.C = out; g.ldc = ldo; g.epi = epi; g.pre = const_cast<float*>(pre); g.ldp = ldp; g.accum = accum;
    g.bf16 = bf16;
    launch_gemm(g, s);
}

__global__ void k_transpose(int rows, int cols, const float* __restrict__ src, float* __restrict__ dst) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(rows) * cols) return;
    const int c = int(t / rows), r = int(t % rows);  // dst index t = c * rows + r
    dst[t] = src[int64_t(r) * cols + c];
}

void launch_transpose(int rows, int cols, const float* src, float* dst, hipStream_t s) {
    const int64_t total = int64_t(rows) * cols;
    if (total <= 0) return;
    k_transpose<<<cdiv(total, 256), 256, 0, s>>>(rows, cols, src, dst);
    NNP_LAUNCH_CHECK();
}

// Weight adjoint dW[N][K] += sum_m G[m][n] X[m][k], deterministic: chunks of
// rows write partials that k_reduce_chunks adds in chunk order.
__global__ void k_reduce_chunks(int64_t count, int nchunks, const float* __restrict__ part, int64_t stride,
                                float* __restrict__ out, int accum) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= count) return;
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += part[int64_t(c) * stride + t];
    out[t] = accum ? out[t] + s : s;
}

void gemm_wgrad(int M, int N, int K, const float* G, int ldg, const float* X, int ldx, float* dW, float* scratch,
                int chunk, bool accum, hipStream_t s) {
    if (M <= 0) return;
    int nch = cdiv(M, chunk);
    GemmArgs g{};
    g.M = N; g.N = K; g.K = M;
    g.A = G; g.sam = 1; g.sak = ldg;   // A(n, m) = G[m][n]
    g.B = X; g.sbk = ldx; g.sbn = 1;   // B(m, k) = X[m][k]
    g.C = scratch; g.ldc = K; g.chunk_rows = chunk; g.chunk_stride = int64_t(N) * K;
    dim3 grid(cdiv(N, TM), cdiv(K, TN), nch);
    gemm_dispatch(g, grid, s);
    int64_t cnt = int64_t(N) * K;
    k_reduce_chunks<<<cdiv(cnt, 256), 256, 0, s>>>(cnt, nch, scratch, cnt, dW, accum);
    NNP_LAUNCH_CHECK();
}

// Column sums db[n] (+)= sum_m G[m][n] in fixed order (chunks of rows).
__global__ void k_colsum_partial(int M, int N, const float* __restrict__ G, int ldg, int chunk,
                                 float* __restrict__ part) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    int c = blockIdx.y;
    if (n >= N) return;
    int m0 = c * chunk, m1 = min(M, m0 + chunk);
    float s = 0.f;
    for (int m = m0; m < m1; ++m) s += G[int64_t(m) * ldg + n];
    part[int64_t(c) * N + n] = s;
}

void colsum(int M, int N, const float* G, int ldg, float* db, float* scratch, int chunk, bool accum,
            hipStream_t s) {
    if (M <= 0) return;
    int nch = cdiv(M, chunk);
    k_colsum_partial<<<dim3(cdiv(N, 64), nch), 64, 0, s>>>(M, N, G, ldg, chunk, scratch);
    k_reduce_chunks<<<cdiv(N, 256), 256, 0, s>>>(N, nch, scratch, N, db, accum);
    NNP_LAUNCH_CHECK();
}

}  // namespace nnp

namespace nnp {
void launch_reduce_chunks(int64_t count, int nchunks, const float* part, int64_t stride, float* out, bool accum,
                          hipStream_t s) {
    k_reduce_chunks<<<cdiv(count, 256), 256, 0, s>>>(count, nchunks, part, stride, out, accum);
    NNP_LAUNCH_CHECK();
}

// [rows][K + 1] (filter weights then bias per row) -> Wr [rows][K], br [rows]
__global__ void k_split_filter_grad(int rows, int K, const float* __restrict__ sum, float* __restrict__ dWr,
                                    float* __restrict__ dbr) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * (K + 1)) return;
    int r = t / (K + 1), k = t % (K + 1);
    if (k < K) dWr[r * K + k] = sum[t];
    else dbr[r] = sum[t];
}

void launch_split_filter_grad(int rows, int K, const float* sum, float* dWr, float* dbr, hipStream_t s) {
    k_split_filter_grad<<<cdiv(rows * (K + 1), 256), 256, 0, s>>>(rows, K, sum, dWr, dbr);
    NNP_LAUNCH_CHECK();
}
}  // namespace nnp

extern "C" nnp_status nnp_set_dense_kernels(int32_t mode) {
    if (mode != NNP_DENSE_AUTO && mode != NNP_DENSE_FP32) return NNP_EINVAL;
    nnp::set_dense_mode(mode);
    return NNP_OK;
}
