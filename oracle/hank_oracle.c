/*
 * hank_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, CPU-only reference for the sums
 *
 *     f_k = sum_{n=1}^{N} c_n J_0(r_k w_n),   1 <= k <= N            (Sec. 1, eq. (2))
 *
 * for the three tasks of Townsend, "A fast analysis-based discrete Hankel
 * transform using asymptotic expansions":
 *
 *   task 0  Schlomilch       w_n = n*pi,      r_k = (k-1)/(N-1)     (Sec. 4, eq. (Schlomilch))
 *   task 1  Fourier-Bessel   w_n = j_{0,n},   r_k = (k-1)/(N-1)     (Sec. 5, eq. (FourierBessel))
 *   task 2  DHT of order 0   w_n = j_{0,n},   r_k = j_{0,k}/j_{0,N+1}  (Sec. 6, eq. (DHT))
 *   task 3  Schlomilch on the paper's own grid r_k = k/N
 *   task 4  Fourier-Bessel on the paper's own grid r_k = k/N
 *
 * The fast method of the paper reaches this same vector up to O(eps*sum|c_n|)
 * (Sec. 1), so the oracle is the definition written out: every J_0(r_k w_n) is
 * evaluated and the products are summed.  Nothing of the fast method (no
 * partition, no DCT/DST, no Neumann or Taylor perturbation) appears here.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header, table or constant generator
 * with the GPU library; neither includes or links the other.
 *
 * J_0 (and, for the Wronskian check only, J_1, Y_0, Y_1) come from:
 *   - the convergent Taylor series (Sec. 3.2, eq. (TaylorSeriesInfinite)),
 *     summed in double-double arithmetic for z < 20 so that the cancellation
 *     between its terms (largest term ~1e7 at z = 20) costs nothing;
 *   - the Hankel asymptotic expansion (Sec. 3.1, eq. (HankelExpansion)) for
 *     z >= 20, with up to 2*12 terms; by the remainder bound (eq. (errorBound))
 *     the truncation error there is below 1e-17.
 * The trigonometric phase of the asymptotic expansion is reduced exactly: every
 * argument is carried as z = pi*I/D + delta with integers I, D and a small
 * double-double correction delta, and I is reduced modulo 2D in integer
 * arithmetic before any floating-point work.
 *
 * The roots j_{0,n} are found with the oracle's own J_0 by bracketed
 * regula falsi (Illinois variant) inside the interval of Lemma 3.2:
 *     j_{0,n} = (n - 1/4)*pi + b_n,   0 <= b_n <= 1/(8 (n - 1/4) pi).
 *
 * Sums over n use Neumaier (compensated) summation, n ascending.
 *
 * The Schlomilch and Fourier-Bessel sums may also be of order nu > 0,
 * f_k = sum_n c_n J_nu(r_k w_n) (Sec. 4, eq. (FourierBessel): still at the roots
 * of J_0), and the Schlomilch ones with w_n = (n + shift) pi (Remark 4.1); J_nu
 * comes from the same two expansions (series below z = 20 + nu/2).
 *
 * The inverse DHT of Sec. 6 (eq. (inverseTest)), c = (1/j_{0,N+1}^2) D_v J D_v f
 * with v_n = 2/J_1(j_{0,n})^2, is this same direct sum between two diagonal
 * scalings (or_dht_weights gives v).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------ */
/* double-double arithmetic                                            */
/* ------------------------------------------------------------------ */
typedef struct { double hi, lo; } dd;

static dd two_sum(double a, double b) {
    double s = a + b, bb = s - a;
    return (dd){s, (a - (s - bb)) + (b - bb)};
}
static dd quick_two_sum(double a, double b) {
    double s = a + b;
    return (dd){s, b - (s - a)};
}
static dd two_prod(double a, double b) {
    double p = a * b;
    return (dd){p, fma(a, b, -p)};
}
static dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi), t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
static dd dd_neg(dd a) { return (dd){-a.hi, -a.lo}; }
static dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
static dd dd_mul(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}
static dd dd_mul_d(dd a, double b) {
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}
static dd dd_div_d(dd a, double b) {
    double q1 = a.hi / b;
    dd p = two_prod(q1, b);
    dd r = dd_sub(a, p);
    double q2 = r.hi / b;
    return quick_two_sum(q1, q2);
}
static dd dd_div(dd a, dd b) {
    double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul_d(b, q1));
    double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul_d(b, q2));
    double q3 = r.hi / b.hi;
    dd q = quick_two_sum(q1, q2);
    return dd_add(q, (dd){q3, 0.0});
}
static dd dd_from(double a) { return (dd){a, 0.0}; }

/* pi to double-double precision */
static const dd DD_PI = {3.141592653589793116, 1.2246467991473532e-16};

/* ------------------------------------------------------------------ */
/* Taylor series (Sec. 3.2), double-double                             */
/* ------------------------------------------------------------------ */
/* J_nu(z) = sum_t (-1)^t (z/2)^(2t+nu) / (t! (t+nu)!), integer nu >= 0. */
static dd series_jn(int nu, dd z) {
    dd h = dd_mul_d(z, 0.5);
    dd w = dd_mul(h, h);              /* z^2/4 */
    dd term = dd_from(1.0);           /* t = 0 term: (z/2)^nu / nu! */
    for (int i = 1; i <= nu; ++i) term = dd_div_d(dd_mul(term, h), (double)i);
    dd sum = term;
    for (int t = 1; t < 200; ++t) {
        term = dd_mul(term, w);
        term = dd_div_d(term, -(double)t * (double)(t + nu));
        sum = dd_add(sum, term);
        if (fabs(term.hi) < 1e-34 * (1.0 + fabs(sum.hi)) && t > 2) break;
    }
    return sum;
}

/* ------------------------------------------------------------------ */
/* Hankel asymptotic expansion (Sec. 3.1, eq. (HankelExpansion))        */
/* ------------------------------------------------------------------ */
#define ASY_MMAX 12 /* at most 2*ASY_MMAX terms */

/* a_m(nu) = prod_{i=1..m} (4nu^2 - (2i-1)^2) / (m! 8^m) */
static void hankel_coeffs(int nu, double* a, int count) {
    a[0] = 1.0;
    for (int m = 1; m < count; ++m) {
        double f = 4.0 * nu * nu - (double)(2 * m - 1) * (double)(2 * m - 1);
        a[m] = a[m - 1] * f / (8.0 * m);
    }
}

/* P = sum_{m<M} (-1)^m a_{2m}/z^{2m},  Q = sum_{m<M} (-1)^m a_{2m+1}/z^{2m+1};
 * stops once the next pair of terms is below 1e-20, which by (errorBound)
 * bounds the neglected remainder. */
static void hankel_pq(int nu, double z, double* P, double* Q) {
    double a[2 * ASY_MMAX + 2];
    hankel_coeffs(nu, a, 2 * ASY_MMAX + 2);
    double p = 0.0, q = 0.0, zinv = 1.0 / z, zp = 1.0; /* zp = z^-(2m) */
    for (int m = 0; m < ASY_MMAX; ++m) {
        double sgn = (m & 1) ? -1.0 : 1.0;
        double t0 = sgn * a[2 * m] * zp;
        double t1 = sgn * a[2 * m + 1] * zp * zinv;
        p += t0;
        q += t1;
        zp *= zinv * zinv;
        double nxt = fabs(a[2 * m + 2] * zp) + fabs(a[2 * m + 3] * zp * zinv);
        if (nxt < 1e-20) break;
    }
    *P = p;
    *Q = q;
}

/* The first 2M terms of (HankelExpansion) for J_0 at a plain argument, with no
 * early stop: used only by the pin on the remainder R_{0,M} (Sec. 3.1). */
double or_hankel_j0(double z, int M) {
    double a[64];
    if (M < 1 || 2 * M + 2 > 64) return NAN;
    hankel_coeffs(0, a, 2 * M + 2);
    double p = 0.0, q = 0.0, zinv = 1.0 / z, zp = 1.0;
    for (int m = 0; m < M; ++m) {
        double sgn = (m & 1) ? -1.0 : 1.0;
        p += sgn * a[2 * m] * zp;
        q += sgn * a[2 * m + 1] * zp * zinv;
        zp *= zinv * zinv;
    }
    double s = sin(z - M_PI / 4), c = cos(z - M_PI / 4);
    return sqrt(2.0 / (M_PI * z)) * (c * p - s * q);
}

/* cos and sin of a double-double angle */
static void dd_sincos(dd x, double* s, double* c) {
    double sh = sin(x.hi), ch = cos(x.hi);
    *s = sh + ch * x.lo;
    *c = ch - sh * x.lo;
}

/* Argument carried exactly: z = pi*I/D + delta. */
typedef struct {
    int64_t I, D; /* D > 0, I >= 0 */
    dd delta;
} arg_t;

static dd arg_value(const arg_t* a) {
    dd z = dd_div_d(dd_mul_d(DD_PI, (double)a->I), (double)a->D);
    return dd_add(z, a->delta);
}

/* chi = z - (2nu+1)*pi/4, reduced: pi*(I mod 2D)/D - (2nu+1)pi/4 + delta */
static dd arg_phase(const arg_t* a, int nu) {
    int64_t r = a->I % (2 * a->D);
    dd th = dd_div_d(dd_mul_d(DD_PI, (double)r), (double)a->D);
    th = dd_sub(th, dd_mul_d(DD_PI, (2.0 * nu + 1.0) / 4.0));
    return dd_add(th, a->delta);
}

#define SERIES_ZMAX 20.0

/* Series below z = 20 + nu/2, Hankel above: with 2*12 terms the remainder
 * bound of (errorBound) is below 1e-17 from z = 19.9 (nu = 0) to 22.2 (nu = 8)
 * and 25.5 (nu = 12); the largest series term there is below 1e8, so the
 * double-double sum keeps 1e-23. */
static double series_zmax(int nu) { return SERIES_ZMAX + 0.5 * nu; }

static double jn_arg(int nu, const arg_t* a) {
    dd z = arg_value(a);
    if (z.hi < series_zmax(nu)) return series_jn(nu, z).hi;
    double P, Q, s, c;
    hankel_pq(nu, z.hi, &P, &Q);
    dd_sincos(arg_phase(a, nu), &s, &c);
    return sqrt(2.0 / (M_PI * z.hi)) * (c * P - s * Q);
}

static double j0_arg(const arg_t* a) { return jn_arg(0, a); }

/* an arbitrary double z as an exact argument: I/D = 0, delta = z */
static arg_t arg_plain(double z) {
    arg_t a = {0, 1, {z, 0.0}};
    return a;
}

/* Plain-argument special functions (exported for the pins). */
double or_j0(double z) {
    z = fabs(z);
    arg_t a = arg_plain(z);
    return j0_arg(&a);
}

/* J_nu at a plain argument, integer 0 <= nu <= 12 */
double or_jn(int nu, double z) {
    if (nu < 0 || nu > 12) return NAN;
    z = fabs(z);
    arg_t a = arg_plain(z);
    return jn_arg(nu, &a);
}

double or_j0_phase(int64_t I, int64_t D, double dhi, double dlo) {
    arg_t a = {I, D, {dhi, dlo}};
    return j0_arg(&a);
}

double or_j1(double z) {
    if (z < SERIES_ZMAX) return series_jn(1, dd_from(z)).hi;
    double P, Q;
    hankel_pq(1, z, &P, &Q);
    /* mu = z - 3pi/4 */
    dd chi = dd_sub(dd_from(z), dd_mul_d(DD_PI, 0.75));
    double s, c;
    dd_sincos(chi, &s, &c);
    return sqrt(2.0 / (M_PI * z)) * (c * P - s * Q);
}

static const double EULER_GAMMA = 0.57721566490153286061;

/* Y_0 by its ascending series (DLMF 10.8.2) for z < 20, Hankel otherwise.
 * Used only by the Wronskian pin of J_0/J_1. */
double or_y0(double z) {
    if (z < SERIES_ZMAX) {
        dd zz = dd_from(z);
        dd j0 = series_jn(0, zz);
        dd h = dd_mul_d(zz, 0.5);
        dd w = dd_mul(h, h);
        dd term = dd_from(1.0), sum = dd_from(0.0), harm = dd_from(0.0);
        for (int t = 1; t < 200; ++t) {
            term = dd_mul(term, w);
            term = dd_div_d(term, (double)t * (double)t); /* (z^2/4)^t/(t!)^2 */
            harm = dd_add(harm, dd_div_d(dd_from(1.0), (double)t));
            dd tt = dd_mul(term, harm);
            sum = (t & 1) ? dd_add(sum, tt) : dd_sub(sum, tt);
            if (fabs(tt.hi) < 1e-34 * (1.0 + fabs(sum.hi)) && t > 2) break;
        }
        double lg = log(z / 2.0) + EULER_GAMMA;
        dd r = dd_add(dd_mul_d(j0, lg), sum);
        return r.hi * (2.0 / M_PI) + r.lo * (2.0 / M_PI);
    }
    double P, Q, s, c;
    hankel_pq(0, z, &P, &Q);
    dd_sincos(dd_sub(dd_from(z), dd_mul_d(DD_PI, 0.25)), &s, &c);
    return sqrt(2.0 / (M_PI * z)) * (s * P + c * Q);
}

/* Y_1 by DLMF 10.8.1 (n = 1) for z < 20, Hankel otherwise. */
double or_y1(double z) {
    if (z < SERIES_ZMAX) {
        dd zz = dd_from(z);
        dd j1 = series_jn(1, zz);
        dd h = dd_mul_d(zz, 0.5);
        dd w = dd_mul(h, h);
        /* sum_k (psi(k+1) + psi(k+2)) (-w)^k / (k! (k+1)!) */
        dd term = dd_from(1.0), sum = dd_from(0.0);
        dd hk = dd_from(0.0); /* H_k */
        for (int k = 0; k < 200; ++k) {
            if (k > 0) {
                term = dd_mul(term, w);
                term = dd_div_d(term, -(double)k * (double)(k + 1));
                hk = dd_add(hk, dd_div_d(dd_from(1.0), (double)k));
            }
            /* psi(k+1) + psi(k+2) = -2 gamma + 2 H_k + 1/(k+1) */
            dd ps = dd_add(dd_mul_d(hk, 2.0), dd_div_d(dd_from(1.0), (double)(k + 1)));
            ps = dd_sub(ps, dd_from(2.0 * EULER_GAMMA));
            dd tt = dd_mul(term, ps);
            sum = dd_add(sum, tt);
            if (k > 2 && fabs(tt.hi) < 1e-34 * (1.0 + fabs(sum.hi))) break;
        }
        dd r = dd_mul_d(j1, (2.0 / M_PI) * log(z / 2.0));
        r = dd_sub(r, dd_mul_d(dd_mul(h, sum), 1.0 / M_PI));
        r = dd_sub(r, dd_from(2.0 / (M_PI * z)));
        return r.hi + r.lo;
    }
    double P, Q, s, c;
    hankel_pq(1, z, &P, &Q);
    dd_sincos(dd_sub(dd_from(z), dd_mul_d(DD_PI, 0.75)), &s, &c);
    return sqrt(2.0 / (M_PI * z)) * (s * P + c * Q);
}

/* ------------------------------------------------------------------ */
/* Roots j_{0,n} = (n - 1/4) pi + b_n  (Lemma 3.2)                       */
/* ------------------------------------------------------------------ */
/* (n - 1/4) pi as double-double */
static dd beta_dd(int64_t n) { return dd_mul_d(DD_PI, (double)n - 0.25); }

/* A function with the sign of (-1)^n J_0((n - 1/4) pi + b) (up to a positive
 * factor) on the Lemma 3.2 bracket.  For large arguments the Hankel form
 * J_0 ~ sqrt(2/(pi z)) (-1)^n (P sin b + Q cos b) is used, which follows from
 * (HankelExpansion) with chi = (n - 1/2) pi + b and needs no phase reduction. */
static double root_fn(int64_t n, double b) {
    dd z = dd_add(beta_dd(n), dd_from(b));
    if (z.hi < SERIES_ZMAX + 5.0) {
        double j = series_jn(0, z).hi;
        return (n & 1) ? -j : j;
    }
    double P, Q;
    hankel_pq(0, z.hi, &P, &Q);
    return P * sin(b) + Q * cos(b);
}

static double root_offset(int64_t n) {
    double lo = 0.0, hi = 1.0 / (8.0 * ((double)n - 0.25) * M_PI);
    double flo = root_fn(n, lo), fhi = root_fn(n, hi);
    if (flo == 0.0) return lo;
    if (fhi == 0.0) return hi;
    /* The bracket of Lemma 3.2 must change sign. */
    if ((flo > 0) == (fhi > 0)) return NAN;
    int side = 0;
    for (int it = 0; it < 200; ++it) {
        double x = (lo * fhi - hi * flo) / (fhi - flo);
        if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
        double fx = root_fn(n, x);
        if (fx == 0.0) return x;
        if ((fx > 0) == (fhi > 0)) {
            hi = x;
            fhi = fx;
            if (side == 1) flo *= 0.5;
            side = 1;
        } else {
            lo = x;
            flo = fx;
            if (side == -1) fhi *= 0.5;
            side = -1;
        }
        if (hi - lo <= 4e-17 * hi) break;
    }
    return 0.5 * (lo + hi);
}

/* b[n-1] = j_{0,n} - (n - 1/4) pi for 1 <= n <= nmax; returns the number of
 * failures (0 on success). */
int64_t or_root_offsets(int64_t nmax, double* b) {
    int64_t bad = 0;
    for (int64_t n = 1; n <= nmax; ++n) {
        b[n - 1] = root_offset(n);
        if (!(b[n - 1] >= 0.0)) ++bad;
    }
    return bad;
}

/* Weights of the self-inverse relation of the DHT (Sec. 6, eq. (selfinverse)):
 * v[n-1] = 2 / J_1(j_{0,n})^2 for 1 <= n <= N, from the root offsets b.
 * At z = j_{0,n} = (n - 1/4) pi + b_n the Hankel phase z - 3pi/4 is
 * (n - 1) pi + b_n, reduced exactly; below z = 20 the series in double-double. */
void or_dht_weights(int64_t N, const double* b, double* v) {
    for (int64_t n = 1; n <= N; ++n) {
        const double bn = b[n - 1];
        dd z = dd_add(beta_dd(n), dd_from(bn));
        double j1;
        if (z.hi < SERIES_ZMAX) {
            j1 = series_jn(1, z).hi;
        } else {
            double P, Q;
            hankel_pq(1, z.hi, &P, &Q);
            const double sg = ((n - 1) & 1) ? -1.0 : 1.0;
            j1 = sg * sqrt(2.0 / (M_PI * z.hi)) * (cos(bn) * P - sin(bn) * Q);
        }
        v[n - 1] = 2.0 / (j1 * j1);
    }
}

/* ------------------------------------------------------------------ */
/* The direct sum                                                       */
/* ------------------------------------------------------------------ */
enum { T_SCHL = 0, T_FB = 1, T_DHT = 2, T_SCHL_PG = 3, T_FB_PG = 4 };

typedef struct {
    int task;
    int nu;        /* Bessel order (Schlomilch tasks; 0 otherwise) */
    int64_t shift; /* w_n = (n + shift) pi (Schlomilch tasks) */
    int64_t N;
    const double* c;
    const double* b; /* root offsets b_1..b_{N+1} (tasks 1, 2, 4) */
    const int64_t* rows;
    const int64_t* nz; /* 1-based columns with c_n != 0, ascending */
    int64_t nnz;
    double* out;
    int64_t nrows;
    int64_t next; /* shared work counter */
    pthread_mutex_t mu;
} job_t;

/* z_{kn} = r_k w_n as an exact argument */
static arg_t make_arg(const job_t* J, int64_t k, int64_t n) {
    int64_t N = J->N;
    arg_t a;
    switch (J->task) {
    case T_SCHL: /* (k-1) (n + shift) pi / (N-1) */
        a.I = (k - 1) * (n + J->shift);
        a.D = N - 1;
        a.delta = dd_from(0.0);
        break;
    case T_SCHL_PG: /* k (n + shift) pi / N */
        a.I = k * (n + J->shift);
        a.D = N;
        a.delta = dd_from(0.0);
        break;
    case T_FB: /* (k-1)/(N-1) * ((n - 1/4) pi + b_n) */
        a.I = (k - 1) * (4 * n - 1);
        a.D = 4 * (N - 1);
        a.delta = dd_div_d(two_prod((double)(k - 1), J->b[n - 1]), (double)(N - 1));
        break;
    case T_FB_PG: /* k/N * ((n - 1/4) pi + b_n) */
        a.I = k * (4 * n - 1);
        a.D = 4 * N;
        a.delta = dd_div_d(two_prod((double)k, J->b[n - 1]), (double)N);
        break;
    default: { /* T_DHT: j_k j_n / j_{N+1} */
        dd jk = dd_add(beta_dd(k), dd_from(J->b[k - 1]));
        dd jn = dd_add(beta_dd(n), dd_from(J->b[n - 1]));
        dd jN = dd_add(beta_dd(N + 1), dd_from(J->b[N]));
        dd z = dd_div(dd_mul(jk, jn), jN);
        a.I = (4 * k - 1) * (4 * n - 1);
        a.D = 4 * (4 * N + 3);
        dd zt = dd_div_d(dd_mul_d(DD_PI, (double)a.I), (double)a.D);
        a.delta = dd_sub(z, zt);
        break;
    }
    }
    return a;
}

static double row_sum(const job_t* J, int64_t k) {
    double s = 0.0, comp = 0.0; /* Neumaier */
    for (int64_t i = 0; i < J->nnz; ++i) { /* columns with c_n = 0 add nothing */
        int64_t n = J->nz[i];
        double cn = J->c[n - 1];
        arg_t a = make_arg(J, k, n);
        double t = cn * jn_arg(J->nu, &a);
        double u = s + t;
        if (fabs(s) >= fabs(t))
            comp += (s - u) + t;
        else
            comp += (t - u) + s;
        s = u;
    }
    return s + comp;
}

static void* worker(void* p) {
    job_t* J = (job_t*)p;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        int64_t i = J->next++;
        pthread_mutex_unlock(&J->mu);
        if (i >= J->nrows) break;
        J->out[i] = row_sum(J, J->rows[i]);
    }
    return NULL;
}

int or_default_threads(void) {
    long n = sysconf(_SC_NPROCESSORS_ONLN);
    return n > 0 ? (int)n : 1;
}

/* f_k for the 1-based rows[i], written to out[i], with J_nu in place of J_0
 * and w_n = (n + shift) pi for the Schlomilch tasks (Sec. 4 and Remark 4.1;
 * nu = shift = 0 for the others).  b holds b_1..b_{N+1} (ignored by the
 * Schlomilch tasks, may be NULL there).  Returns 0, or -1 on bad arguments. */
int or_eval_rows_nu(int task, int nu, int64_t shift, int64_t N, const double* c, const double* b,
                    int64_t nrows, const int64_t* rows, double* out, int nthreads) {
    if (N < 1 || !c || !rows || !out || nrows < 0) return -1;
    if (nu < 0 || nu > 12 || shift < 0 || shift > 1024) return -1;
    if (nu && task == T_DHT) return -1;                         /* order nu: Sec. 4 and 5 */
    if (shift && task != T_SCHL && task != T_SCHL_PG) return -1; /* Remark 4.1 */
    if ((task == T_SCHL || task == T_FB) && N < 2) return -1;
    if (task != T_SCHL && task != T_SCHL_PG && !b) return -1;
    if (task < 0 || task > 4) return -1;
    for (int64_t i = 0; i < nrows; ++i)
        if (rows[i] < 1 || rows[i] > N) return -1;
    job_t J;
    int64_t* nz = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    if (!nz) return -1;
    int64_t nnz = 0;
    for (int64_t n = 1; n <= N; ++n)
        if (c[n - 1] != 0.0) nz[nnz++] = n;
    J.nz = nz;
    J.nnz = nnz;
    J.task = task;
    J.nu = nu;
    J.shift = shift;
    J.N = N;
    J.c = c;
    J.b = b;
    J.rows = rows;
    J.out = out;
    J.nrows = nrows;
    J.next = 0;
    pthread_mutex_init(&J.mu, NULL);
    if (nthreads <= 0) nthreads = or_default_threads();
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, worker, &J);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.mu);
    free(nz);
    return 0;
}

int or_eval_rows(int task, int64_t N, const double* c, const double* b, int64_t nrows,
                 const int64_t* rows, double* out, int nthreads) {
    return or_eval_rows_nu(task, 0, 0, N, c, b, nrows, rows, out, nthreads);
}

/* J_nu(r_k w_n) for one entry (used by the one-hot pins). */
double or_entry_nu(int task, int nu, int64_t shift, int64_t N, const double* b, int64_t k, int64_t n) {
    job_t J;
    memset(&J, 0, sizeof J);
    J.task = task;
    J.nu = nu;
    J.shift = shift;
    J.N = N;
    J.b = b;
    arg_t a = make_arg(&J, k, n);
    return jn_arg(nu, &a);
}

double or_entry(int task, int64_t N, const double* b, int64_t k, int64_t n) {
    return or_entry_nu(task, 0, 0, N, b, k, n);
}
