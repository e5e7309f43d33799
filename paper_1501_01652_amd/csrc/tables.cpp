// tables.cpp -- host-side constant tables for the device kernels (long double).
//
// * J_0 on [2, 20): Taylor polynomials about the centres 2.25, 2.75, ..., 19.75
//   (half-width 1/4, degree 13, truncation < 1e-19).  The derivatives come from
//   J_0^(u) = 2^-u sum_j (-1)^j C(u,j) J_{2j-u} (DLMF 10.6.1 applied u times),
//   with J_m(x) by Miller's backward recurrence (DLMF 3.6(vi)), the method the
//   paper names for direct summation (Sec. 2.1), normalised by
//   J_0 + 2 sum J_{2k} = 1.
// * J_0 on [0, 2): the Taylor series (Sec. 3.2) coefficients (-1)^t/(t!)^2,
//   and Taylor polynomials about 0.25, 0.75, 1.25, 1.75 like those above (the
//   near field's 8-term step uses pieces on all of [0, 20)).
// * Hankel coefficients a_m(0), a_m(1) (Sec. 3.1) for the large-argument branch
//   and the root iteration.
// * FFT twiddles e^{-2 pi i t/2^13} and the two-level table of e^{-2 pi i t/2^23}.
#include "tables.h"

#include <cmath>

namespace hank {

// J_0 .. J_mmax at x by Miller's algorithm (mmax < 64).
static void miller(long double x, int mmax, long double* J) {
    int start = 2 * (int(x) + 40 + mmax / 2);
    long double jp1 = 0.0L, j = 1e-40L;
    long double norm = 0.0L;
    long double tmp[400];
    for (int m = start; m >= 1; --m) {
        long double jm1 = (2.0L * m / x) * j - jp1;
        jp1 = j;
        j = jm1;
        if (m - 1 < 400) tmp[m - 1] = j;
        if (((m - 1) % 2) == 0 && m - 1 > 0) norm += 2.0L * j;
    }
    norm += tmp[0];
    for (int m = 0; m <= mmax; ++m) J[m] = tmp[m] / norm;
}

static long double lbinom(int n, int k) {
    long double r = 1.0L;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// Taylor coefficients J_nu^(u)(x)/u!, u < J0_TAYLOR_DEG, from
// J_nu^(u) = 2^-u sum_j (-1)^j C(u,j) J_{nu-u+2j} (DLMF 10.6.1 applied u times)
// and J_{-m} = (-1)^m J_m
static void taylor_coeffs(int nu, long double x, double* out) {
    long double J[64];
    miller(x, nu + J0_TAYLOR_DEG + 2, J);
    long double fact = 1.0L;
    for (int u = 0; u < J0_TAYLOR_DEG; ++u) {
        if (u > 0) fact *= u;
        long double d = 0.0L;
        for (int j = 0; j <= u; ++j) {
            int mu = nu - u + 2 * j;
            long double Jm = J[std::abs(mu)];
            if (mu < 0 && (std::abs(mu) & 1)) Jm = -Jm;
            d += ((j & 1) ? -1.0L : 1.0L) * lbinom(u, j) * Jm;
        }
        out[u] = double(std::ldexp(d, -u) / fact);
    }
}

void build_nu_table(int nu, double* out) {
    long double a = 1.0L; // a_m(nu)
    for (int m = 0; m < 2 * NU_HANKEL_PAIRS; ++m) {
        if (m > 0) a *= (4.0L * nu * nu - (long double)(2 * m - 1) * (2 * m - 1)) / (8.0L * m);
        const long double sg = ((m / 2) & 1) ? -1.0L : 1.0L;
        out[(m & 1 ? NU_TAB_Q : NU_TAB_P) + m / 2] = double(sg * a);
    }
    long double f = 1.0L, g = 1.0L; // t!, (t+nu)!
    for (int i = 1; i <= nu; ++i) g *= i;
    for (int t = 0; t < NU_SERIES_TERMS; ++t) {
        if (t > 0) {
            f *= t;
            g *= t + nu;
        }
        out[NU_TAB_SER + t] = double(((t & 1) ? -1.0L : 1.0L) / (f * g));
    }
    for (int i = 0; i < NU_TAYLOR_INTERVALS; ++i)
        taylor_coeffs(nu, J0_TAYLOR_Z0 + (i + 0.5L) * J0_TAYLOR_H, out + NU_TAB_TAY + J0_TAYLOR_DEG * i);
}

void build_tables(DeviceTables& t) {
    // series on [0, 2)
    long double f = 1.0L;
    for (int k = 0; k < J0_SERIES_TERMS; ++k) {
        if (k > 0) f *= (long double)k * (long double)k;
        t.ser[k] = double(((k & 1) ? -1.0L : 1.0L) / f);
    }
    // Taylor tables on [2, 20)
    for (int i = 0; i < J0_TAYLOR_INTERVALS; ++i) {
        long double xc = J0_TAYLOR_Z0 + (i + 0.5L) * J0_TAYLOR_H;
        long double J[64];
        miller(xc, 40, J);
        long double fact = 1.0L;
        for (int u = 0; u < J0_TAYLOR_DEG; ++u) {
            if (u > 0) fact *= u;
            long double d = 0.0L;
            for (int j = 0; j <= u; ++j) {
                int mu = 2 * j - u;
                long double Jm = J[std::abs(mu)];
                if (mu < 0 && (std::abs(mu) & 1)) Jm = -Jm; // J_{-m} = (-1)^m J_m
                d += ((j & 1) ? -1.0L : 1.0L) * lbinom(u, j) * Jm;
            }
            d = std::ldexp(d, -u);
            t.tay[i][u] = double(d / fact);
        }
    }
    // Taylor pieces on [0, 2)
    for (int i = 0; i < J0_TAYLOR0_PIECES; ++i) taylor_coeffs(0, (i + 0.5L) * J0_TAYLOR_H, t.tay0[i]);
    // Hankel coefficients
    for (int nu = 0; nu < 2; ++nu) {
        long double a = 1.0L;
        for (int m = 0; m < HANKEL_TERMS; ++m) {
            if (m > 0) a *= (4.0L * nu * nu - (long double)(2 * m - 1) * (2 * m - 1)) / (8.0L * m);
            t.hank[nu][m] = double(a);
        }
    }
    // twiddles
    const long double twopi = 6.283185307179586476925286766559L;
    for (int k = 0; k < TW_SMALL; ++k) {
        long double a = -twopi * k / TW_SMALL;
        t.tw_small[k][0] = double(cosl(a));
        t.tw_small[k][1] = double(sinl(a));
    }
    for (int k = 0; k < TW_HI; ++k) { // e^{-2 pi i k * TW_LO / 2^23}
        long double a = -twopi * (long double)k * TW_LO / (long double)TW_BIG;
        t.tw_hi[k][0] = double(cosl(a));
        t.tw_hi[k][1] = double(sinl(a));
    }
    for (int k = 0; k < TW_LO; ++k) { // e^{-2 pi i k / 2^23}
        long double a = -twopi * (long double)k / (long double)TW_BIG;
        t.tw_lo[k][0] = double(cosl(a));
        t.tw_lo[k][1] = double(sinl(a));
    }
}

} // namespace hank
