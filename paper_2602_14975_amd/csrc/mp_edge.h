// Per-edge staging shared by the message kernels: the LDS slot of one edge
// and the radial values that fill it.
#pragma once

#include "common.h"
#include "kernels.h"

namespace nnp {

template <int K>
struct EdgeSlot {
    float ef[K];    // e_k(r) f(r)
    float def[K];   // d/dr [e_k(r) f(r)]
    float fc, dfc;  // f(r), f'(r)
    float u[3];
    float ir;       // 1 / r
    float r;        // NC forward only: r in float32
    int j, t;       // neighbour, neighbour species
};

// Radial values of one edge: float64 Chebyshev recurrence for sin(k theta)
// and cos(k theta), theta = pi r / rc.
template <int K, int CUT, bool DERIV>
__device__ __forceinline__ void radial(double r, const MpGeom& mg, float* ef, float* def, float& fc, float& dfc) {
    const double theta = mg.pi_over_rc * r;
    double sn, cs;
    sincos(theta, &sn, &cs);
    double f, df;
    if (CUT == 0) {
        f = 0.5 * (cs + 1.0);
        df = -0.5 * sn * mg.pi_over_rc;
    } else {
        const double d = r * mg.inv_rc;
        const double d2 = d * d, d4 = d2 * d2, d5 = d4 * d;
        f = 1.0 - 21.0 * d5 + 35.0 * d5 * d - 15.0 * d5 * d2;
        df = (-105.0 * d4 + 210.0 * d5 - 105.0 * d5 * d) * mg.inv_rc;  // -p(p+1)(p+2)/2 d^4 (1-d)^2 / rc
    }
    const double inv_r = 1.0 / r;
    const double nr = mg.bessel_norm * inv_r;
    double s_prev = 0.0, s_cur = sn;  // sin(0), sin(theta)
    double c_prev = 1.0, c_cur = cs;  // cos(0), cos(theta)
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        const double ek = nr * s_cur;
        ef[k - 1] = float(ek * f);
        if (DERIV) {
            // d/dr [sin(k pi r/rc)/r] = (k pi/rc) cos(k theta)/r - sin(k theta)/r^2
            const double dek = nr * (double(k) * mg.pi_over_rc * c_cur - s_cur * inv_r);
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

// Radial values of the cosine cutoff (the conservative model) in float32,
// with their r-derivatives; the pair rule and the displacement stay in
// float64 upstream.  sin(k theta) and cos(k theta), theta = pi r / rc, come
// from sincospi(r / rc) and the rotation by theta (angle addition), whose
// rounding errors grow only linearly with k.
template <int K>
__device__ __forceinline__ void radial_cos_f32(float r, const MpGeom& mg, float* ef, float* def, float& fc,
                                               float& dfc) {
    const float inv_rc = float(mg.inv_rc), k_pi = float(mg.pi_over_rc);
    float sn, cs;
    sincospif(r * inv_rc, &sn, &cs);
    const float f = 0.5f * (cs + 1.f);
    const float df = -0.5f * sn * k_pi;
    const float ir = 1.f / r;
    const float nr = float(mg.bessel_norm) * ir;
    float s = sn, c = cs;  // sin(k theta), cos(k theta) for k = 1
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        const float ek = nr * s;
        ef[k - 1] = ek * f;
        // d/dr [sin(k pi r/rc)/r] = (k pi/rc) cos(k theta)/r - sin(k theta)/r^2
        const float dek = nr * fmaf(float(k) * k_pi, c, -s * ir);
        def[k - 1] = fmaf(dek, f, ek * df);
        const float s_next = fmaf(s, cs, c * sn);
        const float c_next = fmaf(c, cs, -(s * sn));
        s = s_next;
        c = c_next;
    }
    fc = f;
    dfc = df;
}

// Forward radial values of the polynomial envelope (the NC model) in
// float32; the pair rule and the displacement stay in float64 upstream.
// d = r / rc, nr = bessel_norm / r.  sin(k pi d) follows the Chebyshev
// recurrence from sincospi(d); the envelope 1 - 21 d^5 + 35 d^6 - 15 d^7 is
// evaluated in its factored form (1 - d)^3 (1 + 3d + 6d^2 + 10d^3 + 15d^4),
// which keeps full relative precision as d approaches 1 (1 - d is exact for
// d >= 1/2).
template <int K>
__device__ __forceinline__ void radial_poly_f32(float d, float nr, float* ef, float& fc) {
    float sn, cs;
    sincospif(d, &sn, &cs);
    const float e = 1.f - d;
    const float q = fmaf(d, fmaf(d, fmaf(d, fmaf(d, 15.f, 10.f), 6.f), 3.f), 1.f);
    const float f = e * e * e * q;
    const float nf = nr * f;
    float s_prev = 0.f, s_cur = sn;
    const float c2 = 2.f * cs;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        ef[k] = nf * s_cur;
        const float s_next = fmaf(c2, s_cur, -s_prev);
        s_prev = s_cur;
        s_cur = s_next;
    }
    fc = f;
}

}  // namespace nnp
