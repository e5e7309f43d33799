// device_common.h -- device helpers: complex numbers, exactly reduced phases,
// J_0 at an exactly carried argument, constant tables.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.h"

namespace hank {

template <typename F>
struct cx {
    F x, y;
};

template <typename F>
__device__ __forceinline__ cx<F> mk(F a, F b) {
    cx<F> r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename F>
__device__ __forceinline__ cx<F> operator+(cx<F> a, cx<F> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename F>
__device__ __forceinline__ cx<F> operator-(cx<F> a, cx<F> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename F>
__device__ __forceinline__ cx<F> cmul(cx<F> a, cx<F> b) {
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename F>
__device__ __forceinline__ cx<F> cscale(cx<F> a, F s) { return mk(a.x * s, a.y * s); }

// Global-memory views.  A pointer read from a descriptor in memory is one the
// compiler cannot prove global, so it would be accessed with FLAT
// instructions, which also count against the LDS wait counter (every wait for
// an LDS exchange would then wait for the outstanding HBM loads and stores as
// well).  Through these views the accesses are global_* instructions.
template <typename T>
using glob = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ glob<T>* gview(T* p) {
    return (glob<T>*)p;
}
template <typename T>
__device__ __forceinline__ const glob<T>* gview(const T* p) {
    return (const glob<T>*)p;
}
// complex loads and stores through a global view (as one 2-vector)
template <typename F>
__device__ __forceinline__ cx<F> gload(const glob<cx<F>>* p) {
    typedef F v2 __attribute__((ext_vector_type(2)));
    const v2 t = *(const glob<v2>*)p;
    return mk(t.x, t.y);
}
template <typename F>
__device__ __forceinline__ void gstore(glob<cx<F>>* p, cx<F> v) {
    typedef F v2 __attribute__((ext_vector_type(2)));
    v2 t;
    t.x = v.x;
    t.y = v.y;
    *(glob<v2>*)p = t;
}

// Device copy of the host tables (see tables.cpp).
extern __device__ DeviceTables g_tab;

// sin and cos of pi*r/den for an integer 0 <= r < 2*den (den > 0), with the
// angle reduced exactly: 4r = o*den + rem fixes the octant o, the remaining
// fraction is below a quarter and goes through sincospi.
__device__ __forceinline__ void sincospi_ratio(int64_t r, int64_t den, double* s, double* c) {
    int64_t t = 4 * r;
    int64_t o = (int64_t)((double)t / (double)den); // estimate, then fix
    int64_t rem = t - o * den;
    while (rem < 0) {
        --o;
        rem += den;
    }
    while (rem >= den) {
        ++o;
        rem -= den;
    }
    double y;
    int q;
    bool neg;
    if (o & 1) {
        q = (int)((o + 1) >> 1);
        y = (double)(den - rem) / (double)(4 * den);
        neg = true;
    } else {
        q = (int)(o >> 1);
        y = (double)rem / (double)(4 * den);
        neg = false;
    }
    double sy, cy;
    sincospi(y, &sy, &cy);
    if (neg) sy = -sy;
    switch (q & 3) {
    case 0: *s = sy; *c = cy; break;
    case 1: *s = cy; *c = -sy; break;
    case 2: *s = -sy; *c = -cy; break;
    default: *s = -cy; *c = sy; break;
    }
}

// e^{i pi num/den}, num any int64 (reduced here), den > 0
__device__ __forceinline__ cx<double> expi_ratio(int64_t num, int64_t den) {
    int64_t m = num % (2 * den);
    if (m < 0) m += 2 * den;
    double s, c;
    sincospi_ratio(m, den, &s, &c);
    return mk(c, s);
}

// sin/cos of a small angle |d| <= 0.25 by Taylor polynomials (error < 1e-17)
__device__ __forceinline__ void sincos_small(double d, double* s, double* c) {
    double d2 = d * d;
    double sp = 1.0 + d2 * (-1.0 / 6 + d2 * (1.0 / 120 + d2 * (-1.0 / 5040 + d2 * (1.0 / 362880 + d2 * (-1.0 / 39916800 + d2 * (1.0 / 6227020800.0))))));
    double cp = 1.0 + d2 * (-0.5 + d2 * (1.0 / 24 + d2 * (-1.0 / 720 + d2 * (1.0 / 40320 + d2 * (-1.0 / 3628800 + d2 * (1.0 / 479001600.0 + d2 * (-1.0 / 87178291200.0)))))));
    *s = d * sp;
    *c = cp;
}

// J_0(z) for 0 <= z < 20 from the tables: series below 2, Taylor pieces above,
// each truncated to its first NT terms (NT = 8 keeps the error below 6.2e-10:
// 1/(8!)^2 for the series at z^2/4 < 1, 0.25^8/8! for a piece, |J_0^(8)| <= 1).
template <int NT = J0_TAYLOR_DEG>
__device__ __forceinline__ double j0_small(double z) {
    static_assert(NT <= J0_TAYLOR_DEG && NT <= J0_SERIES_TERMS, "table size");
    if (z < J0_TAYLOR_Z0) {
        double w = 0.25 * z * z;
        double p = g_tab.ser[NT - 1];
#pragma unroll
        for (int k = NT - 2; k >= 0; --k) p = fma(p, w, g_tab.ser[k]);
        return p;
    }
    int i = (int)((z - J0_TAYLOR_Z0) * (1.0 / J0_TAYLOR_H));
    i = i < 0 ? 0 : (i >= J0_TAYLOR_INTERVALS ? J0_TAYLOR_INTERVALS - 1 : i);
    double dz = z - (J0_TAYLOR_Z0 + (i + 0.5) * J0_TAYLOR_H);
    const double* t = g_tab.tay[i];
    double p = t[NT - 1];
#pragma unroll
    for (int u = NT - 2; u >= 0; --u) p = fma(p, dz, t[u]);
    return p;
}

// J_0(z), 0 <= z < 20 (and up to a rounding above), from the first NT
// coefficients of the Taylor pieces about 0.25, 0.75, ..., 19.75 held in
// `tl` (LD doubles per piece, pieces 0-3 on [0, 2)): no series branch, and
// the truncation error is that of the pieces above 2 (NT = 8: below
// 0.25^8/8! < 3.8e-10, |J_0^(8)| <= 1)
template <int NT, int LD>
__device__ __forceinline__ double j0_small_tab(double z, const double* tl) {
    static_assert(NT <= LD && NT <= J0_TAYLOR_DEG, "table size");
    constexpr int NP = J0_TAYLOR0_PIECES + J0_TAYLOR_INTERVALS;
    const int i = min((int)(z * (1.0 / J0_TAYLOR_H)), NP - 1);
    const double dz = z - fma((double)i, J0_TAYLOR_H, 0.5 * J0_TAYLOR_H);
    const double* t = tl + i * LD;
    double p = t[NT - 1];
#pragma unroll
    for (int u = NT - 2; u >= 0; --u) p = fma(p, dz, t[u]);
    return p;
}

// Hankel P_nu, Q_nu (Sec. 3.1) with M = mterms pairs, at zi = 1/z.
__device__ __forceinline__ void hankel_pq(int nu, double zi, int mterms, double* P, double* Q) {
    double zi2 = zi * zi;
    const double* a = g_tab.hank[nu];
    double p = 0.0, q = 0.0;
    for (int m = mterms - 1; m >= 0; --m) {
        double sg = (m & 1) ? -1.0 : 1.0;
        p = fma(p, zi2, sg * a[2 * m]);
        q = fma(q, zi2, sg * a[2 * m + 1]);
    }
    *P = p;
    *Q = q * zi;
}

// pairs of Hankel terms that keep the remainder (errorBound) below 1e-17
__device__ __forceinline__ int hankel_terms_for(double z) {
    return z < 28.0 ? 12 : z < 44.0 ? 8 : z < 65.0 ? 6 : z < 123.0 ? 5 : z < 376.0 ? 4 : 3;
}

// J_0(z) for z = pi*I/D + delta >= 20, phase reduced exactly: ir = I mod 2D.
__device__ __forceinline__ double j0_asy(int64_t ir, int64_t D, double delta, double z) {
    // chi = pi*(4 ir - D)/(4D) + delta
    int64_t num = 4 * ir - D;
    if (num < 0) num += 8 * D;
    double s0, c0, sd, cd;
    sincospi_ratio(num, 4 * D, &s0, &c0);
    sincos_small(delta, &sd, &cd);
    double s = s0 * cd + c0 * sd, c = c0 * cd - s0 * sd;
    double zi = 1.0 / z;
    double P, Q;
    hankel_pq(0, zi, hankel_terms_for(z), &P, &Q);
    return 0.79788456080286535588 * sqrt(zi) * (c * P - s * Q); // sqrt(2/pi)
}

// J_0 at a plain argument (used for tests and roots)
__device__ __forceinline__ double j0_plain(double z) {
    z = fabs(z);
    if (z < J0_ASY_Z) return j0_small(z);
    double s, c;
    sincos(z - 0.78539816339744830962, &s, &c);
    double zi = 1.0 / z, P, Q;
    hankel_pq(0, zi, hankel_terms_for(z), &P, &Q);
    return 0.79788456080286535588 * sqrt(zi) * (c * P - s * Q);
}

} // namespace hank
