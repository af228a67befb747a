// Float64 Langevin integration on the device (paper, Methods
// "Multi-time-step integrator", Algorithm 1, "High Hydrogen Friction", and
// the Fast-Forward Langevin update).  Positions and velocities are [3][n]
// float64; forces are float32 and promoted before use.
//
// Random numbers: Philox-4x64-10 (Salmon et al., SC'11) keyed by
// (seed_r, stream_r) of the atom's replica with counter (local atom index,
// O-step index, 0, 0); the four words map to uniforms ((w >> 11) + 0.5) 2^-53
// and Box-Muller gives the x, y, z normals.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace nnp {

constexpr double kAcc = 4.184e-4;                        // kcal/mol/A/amu -> A/fs^2
constexpr double kKb = 8.31446261815324 / 4184.0;        // kcal/mol/K

__device__ __forceinline__ void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2, uint64_t& c3, uint64_t k0,
                                              uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
}

__device__ __forceinline__ double u01(uint64_t w) { return (double(w >> 11) + 0.5) * 0x1p-53; }

__device__ __forceinline__ void normals3(uint64_t atom, uint64_t step, uint64_t k0, uint64_t k1, double g[3]) {
    uint64_t c0 = atom, c1 = step, c2 = 0, c3 = 0;
    philox4x64_10(c0, c1, c2, c3, k0, k1);
    const double u0 = u01(c0), u1 = u01(c1), u2 = u01(c2), u3 = u01(c3);
    const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
    g[0] = r0 * cos(2.0 * M_PI * u1);
    g[1] = r0 * sin(2.0 * M_PI * u1);
    g[2] = r1 * cos(2.0 * M_PI * u3);
}

// v += coef * (Fa - Fb) / m   (Fb may be null)
__global__ void k_kick(int n, double* __restrict__ vel, const double* __restrict__ mass, const float* __restrict__ Fa,
                       const float* __restrict__ Fb, double coef, uint64_t* bump, uint64_t bump_by) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (bump && i == 0) *bump += bump_by;
    if (i >= n) return;
    const double im = 1.0 / mass[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double f = double(Fa[a * n + i]);
        if (Fb) f -= double(Fb[a * n + i]);
        vel[a * n + i] += coef * f * im;
    }
}

// Fused B(d/2) A(d/2) O(d) A(d/2) with the displacement trigger of the
// Verlet lists (flag set when an atom moved more than the threshold since
// the last build, or is not finite).  With full_kick the opening kick is
// B(d): the previous step's closing B(d/2) with the same force folded in.
__global__ void k_baoa(BaoaArgs a) {
    const int n = a.n;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool over = false;
    float dmax = 0.f;
    if (i < n) {
        const int r = a.rep_of_atom ? a.rep_of_atom[i] : 0;
        const double m = a.mass[i];
        const double im = 1.0 / m;
        const double hd = 0.5 * a.dt;
        const double kd = a.full_kick ? a.dt : hd;
        double x[3], v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[c] = a.pos[c * n + i];
            v[c] = a.vel[c * n + i];
            v[c] += kd * kAcc * double(a.force[c * n + i]) * im;
            x[c] += hd * v[c];
        }
        // O step
        const double gamma = a.gamma[i] * 1e-3;  // ps^-1 -> fs^-1
        const double c1 = exp(-gamma * a.dt);
        const double sigma = sqrt((1.0 - c1 * c1) * kKb * a.temperature * kAcc * im);
        const uint64_t local = uint64_t(i - a.rep_start[r]);
        const uint64_t step = a.step_base[r] + a.step_offset + (a.step_dev ? *a.step_dev : 0ull);
        double g[3];
        normals3(local, step, a.seed[r], a.stream[r], g);
        double nv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) nv[c] = c1 * v[c] + sigma * g[c];
        if (a.ffl) {
            const double n_old = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            const double n_new = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
            if (n_old > 0.0) {
                const double s = n_new / n_old;
#pragma unroll
                for (int c = 0; c < 3; ++c) nv[c] = v[c] * s;
            }
        }
        double d2 = 0.0;
        const int ri = a.pos_rows ? min(max(a.row[i], 0), n - 1) : 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[c] += hd * nv[c];
            a.pos[c * n + i] = x[c];
            if (a.pos_rows) a.pos_rows[c * n + ri] = x[c];
            a.vel[c * n + i] = nv[c];
            if (a.pos_ref) {
                const double d = x[c] - a.pos_ref[c * n + i];
                d2 += d * d;
            }
        }
        over = a.pos_ref && !(d2 <= a.disp_thr2);
        dmax = over && !(d2 <= 3.0e38) ? 3.0e38f : float(d2);  // finite bits for the record
    }
    if (a.flag && __ballot(over) != 0ull && (threadIdx.x & 63) == 0) atomicOr(a.flag, 1);
    if (a.maxd2) {
        for (int o = 32; o > 0; o >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, o));
        if ((threadIdx.x & 63) == 0) atomicMax(a.maxd2, __float_as_uint(dmax));
    }
}

// Largest squared displacement since the last list build, into the record
// that k_baoa keeps (for calls that start with valid lists).
__global__ void k_disp_record(int n, const double* __restrict__ pos, const double* __restrict__ pos_ref,
                              unsigned* __restrict__ maxd2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float dmax = 0.f;
    if (i < n) {
        double d2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double d = pos[c * n + i] - pos_ref[c * n + i];
            d2 += d * d;
        }
        dmax = !(d2 <= 3.0e38) ? 3.0e38f : float(d2);
    }
    for (int o = 32; o > 0; o >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, o));
    if ((threadIdx.x & 63) == 0) atomicMax(maxd2, __float_as_uint(dmax));
}

__global__ void k_stamp(uint64_t* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = uint64_t(wall_clock64());
}

void launch_disp_record(int n, const double* pos, const double* pos_ref, unsigned* maxd2, hipStream_t s) {
    if (n > 0) k_disp_record<<<cdiv(n, 256), 256, 0, s>>>(n, pos, pos_ref, maxd2);
    NNP_LAUNCH_CHECK();
}

void launch_stamp(uint64_t* out, hipStream_t s) {
    k_stamp<<<1, 64, 0, s>>>(out);
    NNP_LAUNCH_CHECK();
}

// Per-replica kinetic energy (fixed-order float64 reduction, one block per
// replica) and a per-replica finiteness flag of positions and velocities.
__global__ void __launch_bounds__(256) k_kinetic(const int64_t* __restrict__ rep_start, int n,
                                                 const double* __restrict__ pos, const double* __restrict__ vel,
                                                 const double* __restrict__ mass, double* __restrict__ ke,
                                                 int* __restrict__ bad) {
    __shared__ double red[256];
    const int r = blockIdx.x;
    const int64_t a0 = rep_start[r], a1 = rep_start[r + 1];
    double s = 0.0;
    bool nonfinite = false;
    for (int64_t i = a0 + threadIdx.x; i < a1; i += 256) {
        double v2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = vel[c * int64_t(n) + i];
            const double x = pos[c * int64_t(n) + i];
            v2 += v * v;
            nonfinite |= !isfinite(v) || !isfinite(x);
        }
        s += mass[i] * v2;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && ke) ke[r] = 0.5 * red[0] / kAcc;
    if (nonfinite && bad) atomicOr(bad + r, 1);
}

// The same over chunks of kKeChunk atoms: block (c, r) writes the partial
// sum of chunk c of replica r to part[r * chunks + c], then one lane per
// replica adds its chunks in order.
__global__ void __launch_bounds__(256) k_kinetic_part(const int64_t* __restrict__ rep_start, int n, int chunks,
                                                      const double* __restrict__ pos, const double* __restrict__ vel,
                                                      const double* __restrict__ mass, double* __restrict__ part,
                                                      int* __restrict__ bad) {
    __shared__ double red[256];
    const int r = blockIdx.y, ch = blockIdx.x;
    const int64_t a0 = rep_start[r] + int64_t(ch) * kKeChunk;
    const int64_t a1 = min(rep_start[r + 1], a0 + kKeChunk);
    double s = 0.0;
    bool nonfinite = false;
    for (int64_t i = a0 + threadIdx.x; i < a1; i += 256) {
        double v2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = vel[c * int64_t(n) + i];
            const double x = pos[c * int64_t(n) + i];
            v2 += v * v;
            nonfinite |= !isfinite(v) || !isfinite(x);
        }
        s += mass[i] * v2;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[int64_t(r) * chunks + ch] = red[0];
    if (nonfinite && bad) atomicOr(bad + r, 1);
}

__global__ void k_kinetic_final(const int64_t* __restrict__ rep_start, int chunks, const double* __restrict__ part,
                                double* __restrict__ ke) {
    const int r = blockIdx.x;
    if (threadIdx.x != 0) return;
    const int64_t na = rep_start[r + 1] - rep_start[r];
    const int nc = int((na + kKeChunk - 1) / kKeChunk);
    double acc = 0.0;
    for (int c = 0; c < nc; ++c) acc += part[int64_t(r) * chunks + c];
    ke[r] = 0.5 * acc / kAcc;
}

// The finiteness flags alone (no kinetic energy requested): one thread per
// atom over the whole grid.
__global__ void __launch_bounds__(256) k_finite(int n, const int32_t* __restrict__ rep_of_atom,
                                                const double* __restrict__ pos, const double* __restrict__ vel,
                                                int* __restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool nonfinite = false;
#pragma unroll
    for (int c = 0; c < 3; ++c) nonfinite |= !isfinite(vel[c * int64_t(n) + i]) || !isfinite(pos[c * int64_t(n) + i]);
    if (nonfinite) atomicOr(bad + (rep_of_atom ? rep_of_atom[i] : 0), 1);
}

// ------------------------------------------------------------------- host --
void launch_kick(int n, double* vel, const double* mass, const float* Fa, const float* Fb, double half_dt,
                 hipStream_t s, uint64_t* bump, uint64_t bump_by) {
    k_kick<<<cdiv(n, 256), 256, 0, s>>>(n, vel, mass, Fa, Fb, half_dt * kAcc, bump, bump_by);
    NNP_LAUNCH_CHECK();
}

__global__ void k_set_u64(uint64_t* p, uint64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

void launch_set_u64(uint64_t* p, uint64_t value, hipStream_t s) {
    k_set_u64<<<1, 64, 0, s>>>(p, value);
    NNP_LAUNCH_CHECK();
}

__global__ void k_zero(uint32_t* __restrict__ p, int64_t words, const int* __restrict__ run) {
    if (run && *run == 0) return;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < words; t += int64_t(gridDim.x) * blockDim.x)
        p[t] = 0u;
}

void launch_zero(void* p, int64_t words, const int* run, hipStream_t s) {
    if (words <= 0) return;
    const int blocks = int(std::min<int64_t>(cdiv(words, 256), 2048));
    k_zero<<<blocks, 256, 0, s>>>(static_cast<uint32_t*>(p), words, run);
    NNP_LAUNCH_CHECK();
}

// NPT virial estimator of an outer step per atom (the per-atom shares of
// the virial of the slow force at the end of the step plus the inner-loop
// average of the fast force's proxy): out = w_cons - w_fast_last + inv_n w_fast_sum
__global__ void k_virial_combine(int n, const float* __restrict__ wc, const float* __restrict__ wl,
                                 const float* __restrict__ ws, float inv_n, float* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = (wc[t] - wl[t]) + ws[t] * inv_n;
}

void launch_virial_combine(int n, const float* wc, const float* wl, const float* ws, float inv_n, float* out,
                           hipStream_t s) {
    if (n <= 0) return;
    k_virial_combine<<<cdiv(n, 256), 256, 0, s>>>(n, wc, wl, ws, inv_n, out);
    NNP_LAUNCH_CHECK();
}

__global__ void k_add(int n, const float* __restrict__ x, float* __restrict__ y) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] += x[t];
}

void launch_add(int n, const float* x, float* y, hipStream_t s) {
    if (n <= 0) return;
    k_add<<<cdiv(n, 256), 256, 0, s>>>(n, x, y);
    NNP_LAUNCH_CHECK();
}

void launch_baoa(const BaoaArgs& a, hipStream_t s) {
    ScopedTimer timer("baoa", s);
    k_baoa<<<cdiv(a.n, 256), 256, 0, s>>>(a);
    NNP_LAUNCH_CHECK();
}

// Stochastic cell rescaling, one thread per replica: P = (2K - W) / (3V),
// d eps = -(beta/tau)(P0 - P) dt + sqrt(2 kT beta dt / (V tau)) g with g the
// first Box-Muller normal of the Philox block at counter (0, step, 1, 0);
// mu = exp(d eps / 3) and the box edge becomes L mu.
__global__ void k_scr(int n_rep, const double* __restrict__ ke, const double* __restrict__ virial,
                      double* __restrict__ box, double* __restrict__ mu, ScrArgs a) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rep) return;
    const double L = box[r];
    const double V = L * L * L;
    const double p_int = (2.0 * ke[r] - virial[r]) / (3.0 * V);
    uint64_t c0 = 0, c1 = a.step, c2 = 1, c3 = 0;
    philox4x64_10(c0, c1, c2, c3, a.seed, a.stream + uint64_t(r));
    const double g = sqrt(-2.0 * log(u01(c0))) * cos(2.0 * M_PI * u01(c1));
    const double kT = kKb * a.temperature;
    const double de = -(a.beta / a.tau) * (a.p0 - p_int) * a.dt + sqrt(2.0 * kT * a.beta * a.dt / (V * a.tau)) * g;
    const double m = exp(de / 3.0);
    mu[r] = m;
    box[r] = L * m;
}

__global__ void k_scale(int n, const int32_t* __restrict__ rep_of_atom, const double* __restrict__ mu,
                        double* __restrict__ pos, double* __restrict__ vel) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double m = mu[rep_of_atom ? rep_of_atom[i] : 0];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        pos[c * int64_t(n) + i] *= m;
        vel[c * int64_t(n) + i] /= m;
    }
}

void launch_scr(int n_rep, const double* ke, const double* virial, double* box, double* mu, const ScrArgs& a,
                hipStream_t s) {
    k_scr<<<cdiv(n_rep, 64), 64, 0, s>>>(n_rep, ke, virial, box, mu, a);
    NNP_LAUNCH_CHECK();
}

void launch_scale(int n, const int32_t* rep_of_atom, const double* mu, double* pos, double* vel, hipStream_t s) {
    if (n > 0) k_scale<<<cdiv(n, 256), 256, 0, s>>>(n, rep_of_atom, mu, pos, vel);
    NNP_LAUNCH_CHECK();
}

void launch_kinetic(int n_rep, const int64_t* rep_start, int n, const double* pos, const double* vel,
                    const double* mass, double* ke, int* bad, hipStream_t s, const int32_t* rep_of_atom,
                    double* part, int chunks) {
    if (!ke && bad && (n_rep == 1 || rep_of_atom)) {
        if (n > 0) k_finite<<<cdiv(n, 256), 256, 0, s>>>(n, rep_of_atom, pos, vel, bad);
    } else if (part && chunks > 1) {
        k_kinetic_part<<<dim3(chunks, n_rep), 256, 0, s>>>(rep_start, n, chunks, pos, vel, mass, part, bad);
        if (ke) k_kinetic_final<<<n_rep, 64, 0, s>>>(rep_start, chunks, part, ke);
    } else {
        k_kinetic<<<n_rep, 256, 0, s>>>(rep_start, n, pos, vel, mass, ke, bad);
    }
    NNP_LAUNCH_CHECK();
}

}  // namespace nnp
