// kernels.hip -- gfx950 kernels of the fast Bessel-sum library.
//
//   roots        b_n = j_{0,n} - (n - 1/4) pi  (Lemma 3.2) by McMahon + Newton
//   dht_e        e_k = j_{0,k}/j_{0,N+1} - (4k-1)/(4N+3)  (Lemma 3.2, proof)
//   near         direct sum over the near field (J^EVAL of eq. (StableMatrixDecomposition)
//                and the first columns/rows of Sec. 5.1 / 6), FP64
//   near_reduce  fixed-order sum of the near-field partials into f
//   pass_a/b/c   one far-field block as a chirp-z transform: the DCT-I/DST-I sums
//                of eq. (AsymptoticDecomposition) on a shifted equispaced grid
//                (Remark 4.1) evaluated by Bluestein's convolution on a
//                four-step power-of-two FFT; pass A generates the block's
//                term inputs and runs the column FFTs, pass B the row FFT,
//                chirp-spectrum product and inverse row FFT, pass C the
//                inverse column FFTs and the epilogue that adds the block's
//                contribution to f.
#include "kernels.h"

#include "fft_device.h"

namespace hank {

__device__ DeviceTables g_tab;

// ---------------------------------------------------------------------------
// Roots
// ---------------------------------------------------------------------------
// J_0 and J_0' from Taylor piece i at offset dz from its centre
__device__ __forceinline__ void j0_taylor_piece(int i, double dz, double* J, double* dJ) {
    const double* t = g_tab.tay[i];
    double p = t[J0_TAYLOR_DEG - 1], d = (J0_TAYLOR_DEG - 1) * t[J0_TAYLOR_DEG - 1];
    for (int u = J0_TAYLOR_DEG - 2; u >= 1; --u) {
        p = fma(p, dz, t[u]);
        d = fma(d, dz, u * t[u]);
    }
    *J = fma(p, dz, t[0]);
    *dJ = d;
}

__global__ void k_roots(int64_t nmax, double* b) {
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (n > nmax) return;
    const double beta = ((double)n - 0.25) * M_PI;
    // McMahon's expansion for nu = 0 (DLMF 10.21.19): j ~ beta + 1/(8 beta) - 31/(384 beta^3)
    double bi = 1.0 / beta;
    double x = bi * (0.125 - (31.0 / 384.0) * bi * bi);
    if (beta < 21.0) {
        // Newton on b itself with (n - 1/4) pi = beta + beta_lo carried exactly, so
        // the Taylor offset dz = (beta - z_c) + (beta_lo + b) keeps b's precision
        const double pi_lo = 1.2246467991473532e-16;
        const double nq = (double)n - 0.25;
        const double beta_lo = fma(nq, M_PI, -beta) + nq * pi_lo;
        for (int it = 0; it < 10; ++it) {
            double z = beta + x;
            int i = (int)((z - J0_TAYLOR_Z0) * (1.0 / J0_TAYLOR_H));
            i = i < 0 ? 0 : (i >= J0_TAYLOR_INTERVALS ? J0_TAYLOR_INTERVALS - 1 : i);
            const double zc = J0_TAYLOR_Z0 + (i + 0.5) * J0_TAYLOR_H;
            const double dz = (beta - zc) + (beta_lo + x);
            double J, dJ;
            j0_taylor_piece(i, dz, &J, &dJ);
            x -= J / dJ;
        }
    } else {
        // J_0 ~ A(-1)^n (P0 sin b + Q0 cos b), J_1 ~ A(-1)^n (-P1 cos b + Q1 sin b)
        // (eq. (HankelExpansion) at z = (n-1/2)pi + b + pi/4); Newton: b += J_0/J_1
        for (int it = 0; it < 4; ++it) {
            double z = beta + x, zi = 1.0 / z;
            int m = hankel_terms_for(z);
            double P0, Q0, P1, Q1, s, c;
            hankel_pq(0, zi, m, &P0, &Q0);
            hankel_pq(1, zi, m, &P1, &Q1);
            sincos_small(x, &s, &c);
            x += (P0 * s + Q0 * c) / (-P1 * c + Q1 * s);
        }
    }
    b[n - 1] = x;
}

__global__ void k_dht_e(int64_t N, const double* b, double* e) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (k > N) return;
    const double Np = (double)N + 0.75, bN = b[N];
    e[k - 1] = (b[k - 1] * Np - bN * ((double)k - 0.25)) / ((Np * M_PI + bN) * Np);
}

__global__ void k_j0(const double* z, int64_t n, double* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = j0_plain(z[i]);
}

// ---------------------------------------------------------------------------
// Near field
// ---------------------------------------------------------------------------
// Hankel coefficients of J_0 (Sec. 3.1) folded with their signs:
// P = sum_m HP[m] z^-2m, Q = z^-1 sum_m HQ[m] z^-2m, HP[m] = (-1)^m a_2m(0), HQ[m] = (-1)^m a_2m+1(0).
struct Hankel0 {
    double p[12], q[12];
};
constexpr Hankel0 make_hankel0() {
    Hankel0 h{};
    double a = 1.0;
    for (int m = 0; m < 24; ++m) {
        if (m > 0) a *= -double(2 * m - 1) * double(2 * m - 1) / (8.0 * m);
        const double sg = ((m / 2) & 1) ? -1.0 : 1.0;
        if (m & 1)
            h.q[m / 2] = sg * a;
        else
            h.p[m / 2] = sg * a;
    }
    return h;
}

// z^{-1/2} to full precision: hardware estimate and two Newton steps
__device__ __forceinline__ double rsqrt_full(double z) {
    double y = __builtin_amdgcn_rsq(z);
    double h = 0.5 * z;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// Near-field sweep of one tile for a fixed number M of Hankel pairs.  SMALL:
// some entry may have z < 20 (Taylor tables); ASY: some entry has z >= 20.
template <int M, bool SMALL, bool ASY>
__device__ __forceinline__ double near_sweep(const GridArgs& G, const double* __restrict__ c,
                                             const double* __restrict__ bvec, int64_t n, int64_t n1,
                                             double Kd, double rk, double ek, int64_t ir, int64_t step) {
    constexpr Hankel0 H = make_hankel0();
    const int64_t D2 = 2 * G.D;
    double acc = 0.0;
    for (; n < n1; n += 4) {
        const double cn = c[n - 1];
        const double bn = G.col_pert ? bvec[n - 1] : 0.0;
        const double Nd = (double)(G.ac * n + G.bc);
        const double lam = fma(Nd, G.pi_Qc, bn);
        const double delta = fma(ek, lam, rk * bn);
        const double I = Kd * Nd; // exact: K_k N_n < 2^53
        const double pz = I * G.piD_hi;
        const double z = (pz + (fma(I, G.piD_hi, -pz) + I * G.piD_lo)) + delta;
        double J = 0.0;
        if (ASY) {
            // phase/pi = ir/D - 1/4 + delta/pi with ir = K_k N_n mod 2D exact
            const double phi = fma((double)ir, G.invD, -0.25) + delta * 0.31830988618379067154;
            double sn, cs;
            sincospi(phi, &sn, &cs);
            const double y = rsqrt_full(z), zi = y * y, zi2 = zi * zi;
            double P = H.p[M - 1], Q = H.q[M - 1];
#pragma unroll
            for (int m = M - 2; m >= 0; --m) {
                P = fma(P, zi2, H.p[m]);
                Q = fma(Q, zi2, H.q[m]);
            }
            J = 0.79788456080286535588 * y * fma(cs, P, -sn * (Q * zi));
        }
        if (SMALL) {
            if (!ASY || z < J0_ASY_Z) J = j0_small(z);
        }
        acc = fma(cn, J, acc);
        ir += step;
        if (ir >= D2) ir -= D2;
    }
    return acc;
}

// One workgroup = 64 rows (one per lane) x a column range; its 4 waves take
// every 4th column (wave-uniform, so the column data are scalar loads) and
// their sums are added in a fixed order.  The tile's flags (host-computed
// bounds on z over the tile) select the Hankel term count and the branches.
__global__ __launch_bounds__(256) void k_near(GridArgs G, const double* __restrict__ c,
                                              const double* __restrict__ bvec,
                                              const double* __restrict__ evec,
                                              const NearTile* __restrict__ tiles,
                                              double* __restrict__ partial) {
    __shared__ double red[4][64];
    const NearTile T = tiles[blockIdx.x];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool active = lane < T.nk;
    const int64_t k = T.k0 + (active ? lane : 0);
    const int64_t K = G.ar * k + G.br;
    const double rk = (double)K / (double)G.Dr;
    const double ek = G.row_pert ? evec[k - 1] : 0.0;
    const int64_t D2 = 2 * G.D;
    const int64_t n = T.n0 + wave;
    int64_t ir = 0, step = 0;
    if (n < T.n1) {
        ir = (K * (G.ac * n + G.bc)) % D2;
        step = (K * 4 * G.ac) % D2;
    }
    const double Kd = (double)K;
    const bool small = T.flags & 1, asy = T.flags & 2;
    const int M = T.flags >> 8;
    double acc = 0.0;
    if (!asy) {
        acc = near_sweep<3, true, false>(G, c, bvec, n, T.n1, Kd, rk, ek, ir, step);
    } else if (small) {
        acc = near_sweep<12, true, true>(G, c, bvec, n, T.n1, Kd, rk, ek, ir, step);
    } else {
        switch (M) {
        case 3: acc = near_sweep<3, false, true>(G, c, bvec, n, T.n1, Kd, rk, ek, ir, step); break;
        case 4: acc = near_sweep<4, false, true>(G, c, bvec, n, T.n1, Kd, rk, ek, ir, step); break;
        case 5: acc = near_sweep<5, false, true>(G, c, bvec, n, T.n1, Kd, rk, ek, ir, step); break;
        case 6: acc = near_sweep<6, false, true>(G, c, bvec, n, T.n1, Kd, rk, ek, ir, step); break;
        case 8: acc = near_sweep<8, false, true>(G, c, bvec, n, T.n1, Kd, rk, ek, ir, step); break;
        default: acc = near_sweep<12, false, true>(G, c, bvec, n, T.n1, Kd, rk, ek, ir, step); break;
        }
    }
    red[wave][lane] = active ? acc : 0.0;
    __syncthreads();
    if (wave == 0)
        partial[(int64_t)blockIdx.x * 64 + lane] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// f_k = sum of the row's tile partials; 4 waves take every 4th tile and their
// sums are combined in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_near_reduce(const RowTile* __restrict__ rt,
                                                     const double* __restrict__ partial, double* __restrict__ f) {
    __shared__ double red[4][64];
    const RowTile R = rt[blockIdx.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double s = 0.0;
    for (int64_t t = wave; t < R.ntiles; t += 4) s += partial[(R.tile0 + t) * 64 + lane];
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && lane < R.nk) f[R.k0 + lane - 1] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// ---------------------------------------------------------------------------
// Far field: chirp-z transform of one block
// ---------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ double ipow_d(double x, int e) {
    double r = 1.0;
    bool inv = e < 0;
    unsigned u = inv ? -e : e;
    while (u) {
        if (u & 1) r *= x;
        x *= x;
        u >>= 1;
    }
    return inv ? 1.0 / r : r;
}

// Pass A on the block's data: y_n' = q(n') c_n X_g(n), column FFTs over j2.
// Per column position the group-independent factors are kept:
//   base = c_n q(n') (w^_n/w0)^(-1/2),  iw = w0/w^_n,  x = (b_n/bref) iw,  la = lambda_n/lref
// and X_g = la^a (w^_n/w0)^e sum_b K_{g,b} x^b, with (w^_n/w0)^e updated
// incrementally over the groups (sorted by a, then e).
template <typename F, int L2, int W>
__global__ __launch_bounds__(W * L2 / 8) void k_pass_a(FarArgs A, const double* __restrict__ c,
                                                       const double* __restrict__ bvec,
                                                       cx<F>* __restrict__ buf) {
    constexpr int R = 8, NTC = L2 / R;
    __shared__ cx<F> sh[W * (L2 + L2 / 8)];
    const int t = threadIdx.x, w = t % W, tt = t / W;
    const int64_t j1 = (int64_t)blockIdx.x * W + w;
    cx<F>* my = sh + w * (L2 + L2 / 8);

    double vw[R], xb[R], la[R], pw[R];
    cx<double> base[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t j2 = tt + r * NTC;
        const int64_t np = j1 + (int64_t)A.L1 * j2;
        vw[r] = 1.0;
        xb[r] = la[r] = 0.0;
        base[r] = mk(0.0, 0.0);
        if (np < A.ncols) {
            const int64_t n = A.na + np;
            const int64_t Nn = A.ac * n + A.bc;
            const double wn = (double)Nn * A.pi_Qc;
            const double bn = A.col_pert ? bvec[n - 1] : 0.0;
            vw[r] = wn / A.w0;
            const double iw = 1.0 / vw[r];
            xb[r] = (bn / A.bref) * iw;
            la[r] = (wn + bn) / A.lref;
            const cx<double> q = expi_ratio(2 * A.Kka * A.ac * np + A.ar * A.ac * np * np, 2 * A.D);
            base[r] = cscale(q, c[n - 1] * sqrt(iw));
        }
    }
    int ecur = 0, acur = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) pw[r] = 1.0; // (w^_n/w0)^ecur * la^acur
    for (int g = A.g0; g < A.g1; ++g) {
        const GroupDev Gd = A.groups[g];
        if (Gd.a != acur || g == A.g0) { // restart the powers
#pragma unroll
            for (int r = 0; r < R; ++r)
                pw[r] = ipow_d<double>(vw[r], Gd.e) * (Gd.a ? ipow_d<double>(la[r], Gd.a) : 1.0);
        } else {
            for (; ecur < Gd.e; ++ecur) {
#pragma unroll
                for (int r = 0; r < R; ++r) pw[r] *= vw[r];
            }
            for (; ecur > Gd.e; --ecur) {
#pragma unroll
                for (int r = 0; r < R; ++r) pw[r] /= vw[r];
            }
        }
        ecur = Gd.e;
        acur = Gd.a;
        cx<F> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double xp = 1.0, Xr = 0.0, Xi = 0.0;
            int bcur = 0;
            const bool live = (j1 + (int64_t)A.L1 * (tt + r * NTC)) < A.ncols; // zero padding otherwise
            if (live)
                for (int ti = Gd.t0; ti < Gd.t1; ++ti) {
                const TermDev Td = A.terms[ti];
                while (bcur < Td.b) {
                    xp *= xb[r];
                    ++bcur;
                }
                Xr = fma(Td.kre, xp, Xr);
                Xi = fma(Td.kim, xp, Xi);
            }
            const cx<double> y = cmul(mk(Xr * pw[r], Xi * pw[r]), base[r]);
            v[r] = mk(F(y.x), F(y.y));
        }
        fft_reg<F, L2, R, -1>(v, my, tt);
        cx<F>* out = buf + (int64_t)(g - A.g0) * A.L;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t m2 = tt + r * NTC;
            out[m2 * A.L1 + j1] = cmul(v[r], tw_big<F>(j1 * m2, A.twshift));
        }
    }
}

// Pass A on the chirp kernel h(m) = e^{-i pi ar ac m^2 / (2D)}, m = k' - n',
// laid out for a circular convolution of length L (first FFT step of H^).
template <typename F, int L2, int W>
__global__ __launch_bounds__(W * L2 / 8) void k_pass_a_kernel(FarArgs A, cx<F>* __restrict__ buf) {
    constexpr int R = 8, NTC = L2 / R;
    __shared__ cx<F> sh[W * (L2 + L2 / 8)];
    const int t = threadIdx.x, w = t % W, tt = t / W;
    const int64_t j1 = (int64_t)blockIdx.x * W + w;
    cx<F>* my = sh + w * (L2 + L2 / 8);
    cx<F> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t j = j1 + (int64_t)A.L1 * (tt + r * NTC);
        int64_t m = 0;
        bool use = false;
        if (j < A.nrows) {
            m = j;
            use = true;
        } else if (j > A.L - A.ncols) {
            m = j - A.L;
            use = true;
        }
        v[r] = mk(F(0), F(0));
        if (use) {
            const cx<double> h = expi_ratio(-A.ar * A.ac * m * m, 2 * A.D);
            v[r] = mk(F(h.x), F(h.y));
        }
    }
    fft_reg<F, L2, R, -1>(v, my, tt);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t m2 = tt + r * NTC;
        buf[m2 * A.L1 + j1] = cmul(v[r], tw_big<F>(j1 * m2, A.twshift));
    }
}

// Pass B, forward only: H^[m2][m1] = (1/L) * row FFT (the chirp spectrum).
template <typename F, int L1, int ROWS>
__global__ __launch_bounds__(ROWS * L1 / 8) void k_pass_b_fwd(FarArgs A, const cx<F>* __restrict__ buf,
                                                               cx<F>* __restrict__ H) {
    constexpr int R = 8, NTR = L1 / R;
    __shared__ cx<F> sh[ROWS * (L1 + L1 / 8)];
    const int t = threadIdx.x, rl = t / NTR, tt = t % NTR;
    const int64_t row = (int64_t)blockIdx.x * ROWS + rl;
    const bool okrow = row < A.L2;
    cx<F> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = okrow ? buf[row * L1 + tt + r * NTR] : mk(F(0), F(0));
    fft_reg<F, L1, R, -1>(v, sh + rl * (L1 + L1 / 8), tt);
    const F s = F(1.0 / (double)A.L);
    if (okrow) {
#pragma unroll
        for (int r = 0; r < R; ++r) H[row * L1 + tt + r * NTR] = cscale(v[r], s);
    }
}

// Pass B: row FFT, product with H^, inverse row FFT, inverse twiddle; in place.
// HANK_PASSB_HREG 1: H^ and the inverse twiddles of the row are held in
// registers across the groups; 0: re-read per group (L2 hits), fewer registers.
#ifndef HANK_PASSB_HREG
#define HANK_PASSB_HREG 1
#endif
template <typename F, int L1, int ROWS>
__global__ __launch_bounds__(ROWS * L1 / 8) void k_pass_b(FarArgs A, cx<F>* __restrict__ buf,
                                                           const cx<F>* __restrict__ H) {
    constexpr int R = 8, NTR = L1 / R;
    __shared__ cx<F> sh[ROWS * (L1 + L1 / 8)];
    const int t = threadIdx.x, rl = t / NTR, tt = t % NTR;
    const int64_t row = (int64_t)blockIdx.x * ROWS + rl;
    const bool okrow = row < A.L2;
    const int64_t rowc = okrow ? row : 0;
    cx<F>* my = sh + rl * (L1 + L1 / 8);
    const cx<F>* hrow = H + rowc * L1;
#if HANK_PASSB_HREG
    cx<F> hv[R], tw[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        hv[r] = hrow[tt + r * NTR];
        const cx<F> w = tw_big<F>((int64_t)(tt + r * NTR) * rowc, A.twshift);
        tw[r] = mk(w.x, -w.y);
    }
#endif
    for (int g = A.g0; g < A.g1; ++g) {
        cx<F>* p = buf + (int64_t)(g - A.g0) * A.L + rowc * L1;
        cx<F> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = p[tt + r * NTR];
        fft_reg<F, L1, R, -1>(v, my, tt);
#pragma unroll
        for (int r = 0; r < R; ++r) {
#if HANK_PASSB_HREG
            v[r] = cmul(v[r], hv[r]);
#else
            v[r] = cmul(v[r], hrow[tt + r * NTR]);
#endif
        }
        fft_reg<F, L1, R, 1>(v, my, tt);
        if (okrow) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
#if HANK_PASSB_HREG
                p[tt + r * NTR] = cmul(v[r], tw[r]);
#else
                const cx<F> w = tw_big<F>((int64_t)(tt + r * NTR) * row, A.twshift);
                p[tt + r * NTR] = cmul(v[r], mk(w.x, -w.y)); // e^{+2 pi i j1 m2 / L}
#endif
            }
        }
    }
}

// Pass C: inverse column FFTs, then f_k += sum_g A_g(k) Re(p(k') conv_g(k')),
// A_g(k) = scale_g (e_k/eref)^a (r^_k/r0)^(e - 1/2) with the power of r^_k/r0
// updated incrementally over the groups.
template <typename F, int L2, int W>
__global__ __launch_bounds__(W * L2 / 8) void k_pass_c(FarArgs A, const cx<F>* __restrict__ buf,
                                                       const double* __restrict__ evec,
                                                       double* __restrict__ f) {
    constexpr int R = 8, NTC = L2 / R;
    __shared__ cx<F> sh[W * (L2 + L2 / 8)];
    const int t = threadIdx.x, w = t % W, tt = t / W;
    const int64_t j1 = (int64_t)blockIdx.x * W + w;
    cx<F>* my = sh + w * (L2 + L2 / 8);
    double rho[R], ek[R], acc[R], pw[R];
    cx<double> pk[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t kp = j1 + (int64_t)A.L1 * (tt + r * NTC);
        rho[r] = 1.0;
        ek[r] = 0.0;
        acc[r] = 0.0;
        pk[r] = mk(0.0, 0.0);
        if (kp < A.nrows) {
            const int64_t k = A.ka + kp;
            rho[r] = ((double)(A.ar * k + A.br) / (double)A.Dr) / A.r0;
            ek[r] = A.row_pert ? evec[k - 1] / A.eref : 0.0;
            pk[r] = cscale(expi_ratio(2 * A.Kka * A.Nna + 2 * A.ar * A.Nna * kp + A.ar * A.ac * kp * kp, 2 * A.D),
                           1.0 / sqrt(rho[r]));
        }
    }
    int ecur = 0, acur = 0;
    for (int g = A.g0; g < A.g1; ++g) {
        const GroupDev Gd = A.groups[g];
        if (Gd.a != acur || g == A.g0) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                pw[r] = ipow_d<double>(rho[r], Gd.e) * (Gd.a ? ipow_d<double>(ek[r], Gd.a) : 1.0);
        } else {
            for (; ecur < Gd.e; ++ecur) {
#pragma unroll
                for (int r = 0; r < R; ++r) pw[r] *= rho[r];
            }
            for (; ecur > Gd.e; --ecur) {
#pragma unroll
                for (int r = 0; r < R; ++r) pw[r] /= rho[r];
            }
        }
        ecur = Gd.e;
        acur = Gd.a;
        const cx<F>* p = buf + (int64_t)(g - A.g0) * A.L;
        cx<F> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = p[(int64_t)(tt + r * NTC) * A.L1 + j1];
        fft_reg<F, L2, R, 1>(v, my, tt);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (j1 + (int64_t)A.L1 * (tt + r * NTC) < A.nrows) { // rows past the block are discarded
                const double re = pk[r].x * (double)v[r].x - pk[r].y * (double)v[r].y;
                acc[r] = fma(Gd.scale * pw[r], re, acc[r]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t kp = j1 + (int64_t)A.L1 * (tt + r * NTC);
        if (kp < A.nrows) f[A.ka + kp - 1] += acc[r];
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t upload_tables(const DeviceTables& t) {
    return hipMemcpyToSymbol(HIP_SYMBOL(g_tab), &t, sizeof(DeviceTables), 0, hipMemcpyHostToDevice);
}

hipError_t launch_roots(int64_t nmax, double* b, hipStream_t s) {
    if (nmax <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_roots, dim3((unsigned)((nmax + 255) / 256)), dim3(256), 0, s, nmax, b);
    return hipGetLastError();
}

hipError_t launch_dht_e(int64_t N, const double* b, double* e, hipStream_t s) {
    hipLaunchKernelGGL(k_dht_e, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, b, e);
    return hipGetLastError();
}

hipError_t launch_j0(const double* z, int64_t n, double* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_j0, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, z, n, out);
    return hipGetLastError();
}

hipError_t launch_near(const GridArgs& G, const double* c, const double* b, const double* e,
                       const NearTile* tiles, int64_t ntiles, double* partial, hipStream_t s) {
    if (ntiles > 0) hipLaunchKernelGGL(k_near, dim3((unsigned)ntiles), dim3(256), 0, s, G, c, b, e, tiles, partial);
    return hipGetLastError();
}

hipError_t launch_near_reduce(const RowTile* rt, int64_t nrt, const double* partial, double* f, hipStream_t s) {
    if (nrt > 0) hipLaunchKernelGGL(k_near_reduce, dim3((unsigned)nrt), dim3(256), 0, s, rt, partial, f);
    return hipGetLastError();
}

template <typename F, int L2>
static void pass_ac_dispatch(int which, const FarArgs& A, const double* c, const double* b, const double* e,
                             void* buf, double* f, hipStream_t s) {
    constexpr int W = 8;
    dim3 grid((unsigned)(A.L1 / W)), block(W * L2 / 8);
    if (which == 0)
        hipLaunchKernelGGL((k_pass_a<F, L2, W>), grid, block, 0, s, A, c, b, (cx<F>*)buf);
    else if (which == 1)
        hipLaunchKernelGGL((k_pass_a_kernel<F, L2, W>), grid, block, 0, s, A, (cx<F>*)buf);
    else
        hipLaunchKernelGGL((k_pass_c<F, L2, W>), grid, block, 0, s, A, (const cx<F>*)buf, e, f);
}

template <typename F>
static hipError_t pass_ac(int which, const FarArgs& A, const double* c, const double* b, const double* e,
                          void* buf, double* f, hipStream_t s) {
    switch (A.L2) {
    case 8: pass_ac_dispatch<F, 8>(which, A, c, b, e, buf, f, s); break;
    case 16: pass_ac_dispatch<F, 16>(which, A, c, b, e, buf, f, s); break;
    case 32: pass_ac_dispatch<F, 32>(which, A, c, b, e, buf, f, s); break;
    case 64: pass_ac_dispatch<F, 64>(which, A, c, b, e, buf, f, s); break;
    case 128: pass_ac_dispatch<F, 128>(which, A, c, b, e, buf, f, s); break;
    case 256: pass_ac_dispatch<F, 256>(which, A, c, b, e, buf, f, s); break;
    case 512: pass_ac_dispatch<F, 512>(which, A, c, b, e, buf, f, s); break;
    case 1024: pass_ac_dispatch<F, 1024>(which, A, c, b, e, buf, f, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename F, int L1>
static void pass_b_dispatch(bool fwd_only, const FarArgs& A, void* buf, void* H, hipStream_t s) {
    constexpr int ROWS = (L1 >= 2048) ? 1 : 2048 / L1;
    dim3 grid((unsigned)((A.L2 + ROWS - 1) / ROWS)), block(ROWS * L1 / 8);
    if (fwd_only)
        hipLaunchKernelGGL((k_pass_b_fwd<F, L1, ROWS>), grid, block, 0, s, A, (const cx<F>*)buf, (cx<F>*)H);
    else
        hipLaunchKernelGGL((k_pass_b<F, L1, ROWS>), grid, block, 0, s, A, (cx<F>*)buf, (const cx<F>*)H);
}

template <typename F>
static hipError_t pass_b(bool fwd_only, const FarArgs& A, void* buf, void* H, hipStream_t s) {
    switch (A.L1) {
    case 8: pass_b_dispatch<F, 8>(fwd_only, A, buf, H, s); break;
    case 16: pass_b_dispatch<F, 16>(fwd_only, A, buf, H, s); break;
    case 32: pass_b_dispatch<F, 32>(fwd_only, A, buf, H, s); break;
    case 64: pass_b_dispatch<F, 64>(fwd_only, A, buf, H, s); break;
    case 128: pass_b_dispatch<F, 128>(fwd_only, A, buf, H, s); break;
    case 256: pass_b_dispatch<F, 256>(fwd_only, A, buf, H, s); break;
    case 512: pass_b_dispatch<F, 512>(fwd_only, A, buf, H, s); break;
    case 1024: pass_b_dispatch<F, 1024>(fwd_only, A, buf, H, s); break;
    case 2048: pass_b_dispatch<F, 2048>(fwd_only, A, buf, H, s); break;
    case 4096: pass_b_dispatch<F, 4096>(fwd_only, A, buf, H, s); break;
    case 8192: pass_b_dispatch<F, 8192>(fwd_only, A, buf, H, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_chirp_spectrum(const FarArgs& A, bool fp32, void* work, void* H, hipStream_t s) {
    hipError_t e = fp32 ? pass_ac<float>(1, A, nullptr, nullptr, nullptr, work, nullptr, s)
                        : pass_ac<double>(1, A, nullptr, nullptr, nullptr, work, nullptr, s);
    if (e != hipSuccess) return e;
    return fp32 ? pass_b<float>(true, A, work, H, s) : pass_b<double>(true, A, work, H, s);
}

hipError_t launch_far_pass(int which, const FarArgs& A, bool fp32, const double* c, const double* b,
                           const double* e, void* work, const void* H, double* f, hipStream_t s) {
    if (which == 1)
        return fp32 ? pass_b<float>(false, A, work, (void*)H, s) : pass_b<double>(false, A, work, (void*)H, s);
    const int w = (which == 0) ? 0 : 2;
    return fp32 ? pass_ac<float>(w, A, c, b, e, work, f, s) : pass_ac<double>(w, A, c, b, e, work, f, s);
}

} // namespace hank
