// Internal helpers shared by the libnnp translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/nnp.h"

namespace nnp {

// ----------------------------------------------------------------- errors --
void set_error(const std::string& msg);

struct Fail {
    nnp_status code;
};

#define NNP_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::nnp::set_error(std::string(#call) + ": " + hipGetErrorString(e_));   \
            throw ::nnp::Fail{NNP_EDEVICE};                                        \
        }                                                                          \
    } while (0)

#define NNP_REQUIRE(cond, code, msg)                                               \
    do {                                                                           \
        if (!(cond)) {                                                             \
            ::nnp::set_error(msg);                                                 \
            throw ::nnp::Fail{code};                                               \
        }                                                                          \
    } while (0)

#define NNP_LAUNCH_CHECK() NNP_HIP(hipGetLastError())

// --------------------------------------------------------------- workspace --
// Bump allocator over a caller-provided buffer.  With base == nullptr it only
// measures, which is how nnp_workspace_size() is computed: every entry point
// carves its scratch with the same sequence of take() calls.
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    Arena(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
    template <class T>
    T* take(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        size_t bytes = count * sizeof(T);
        used = off + bytes;
        if (base == nullptr) return nullptr;
        if (used > cap) {
            set_error("workspace too small: need at least " + std::to_string(used) + " bytes");
            throw Fail{NNP_EINVAL};
        }
        return reinterpret_cast<T*>(base + off);
    }
};

inline int cdiv(int64_t a, int64_t b) { return int((a + b - 1) / b); }

// ------------------------------------------------------------- pair rule ---
// The float64 minimum-image pair rule, evaluated exactly as documented in
// nnp.h: no fused multiply-add, rint half to even, left-to-right sum.
__device__ __forceinline__ bool pair_rule(double xi, double yi, double zi, double xj, double yj,
                                          double zj, double L, double invL, double rc2,
                                          double& dx, double& dy, double& dz) {
#pragma clang fp contract(off)
    dx = xj - xi;
    dy = yj - yi;
    dz = zj - zi;
    dx = dx - L * __builtin_rint(dx * invL);
    dy = dy - L * __builtin_rint(dy * invL);
    dz = dz - L * __builtin_rint(dz * invL);
    double r2 = (dx * dx + dy * dy) + dz * dz;
    return r2 < rc2;
}

// Per-replica geometry table used by every kernel that forms displacements.
struct RepGeom {
    const int32_t* rep_of_atom;  // nullptr: single replica
    const double* box;           // [n_rep] L
    const double* inv_box;       // [n_rep] 1/L
    const int64_t* rep_start;    // [n_rep + 1]
    double box0, inv0;           // replica 0 (used when rep_of_atom == nullptr)
    __device__ __forceinline__ void get(int i, double& L, double& inv) const {
        if (rep_of_atom) {
            int r = rep_of_atom[i];
            L = box[r];
            inv = inv_box[r];
        } else {
            L = box0;
            inv = inv0;
        }
    }
};

// ------------------------------------------------------------- wave utils --
// Workgroups of one launch are dealt out to the 8 XCDs in turn (hardware id b
// runs on XCD b % 8).  This bijection of [0, G) hands each XCD one contiguous
// range of logical ids instead, so that rows of spatially ordered atoms (and
// the neighbours they gather) stay within one XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int G) {
    constexpr int X = 8;
    const int x = b % X, local = b / X;
    const int per = G / X, rem = G % X;
    return x < rem ? x * (per + 1) + local : rem * (per + 1) + (x - rem) * per + local;
}

// LDS written by some lanes of a wavefront, then read by others of the same one
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
template <int W>
__device__ __forceinline__ float group_sum(float x) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ float silu(float x) { return x / (1.0f + __expf(-x)); }
__device__ __forceinline__ float silu_grad(float x) {
    float s = 1.0f / (1.0f + __expf(-x));
    return s * (1.0f + x * (1.0f - s));
}

}  // namespace nnp
