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

// J_0 at entry (k, n) of a near-field tile.  Row data per lane: Kd = K_k,
// rk = r^_k, ek = e_k; column data (uniform): Nd = N_n, bn = b_n; ir = K_k N_n
// mod 2D exactly.  M Hankel pairs; SMALL/ASY select the branches the tile needs.
template <int M, bool SMALL, bool ASY>
__device__ __forceinline__ double near_j0(const GridArgs& G, double Kd, double rk, double ek, double Nd,
                                          double bn, int64_t ir) {
    constexpr Hankel0 H = make_hankel0();
    const double lam = fma(Nd, G.pi_Qc, bn);
    const double delta = fma(ek, lam, rk * bn);
    const double I = Kd * Nd; // exact: K_k N_n < 2^53
    const double pz = I * G.piD_hi;
    const double z = (pz + (fma(I, G.piD_hi, -pz) + I * G.piD_lo)) + delta;
    double J = 0.0;
    if (ASY) {
        // phase/pi = ir/D - 1/4 + delta/pi
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
    return J;
}

// Near-field sweep of one tile (one right-hand side): columns n, n+4, ... < n1.
template <int M, bool SMALL, bool ASY>
__device__ __forceinline__ double near_sweep(const GridArgs& G, const double* __restrict__ c,
                                             const double* __restrict__ bvec, int64_t n, int64_t n1,
                                             double Kd, double rk, double ek, int64_t ir, int64_t step) {
    const int64_t D2 = 2 * G.D;
    double acc = 0.0;
    for (; n < n1; n += 4) {
        const double cn = c[n - 1];
        const double bn = G.col_pert ? bvec[n - 1] : 0.0;
        const double Nd = (double)(G.ac * n + G.bc);
        acc = fma(cn, near_j0<M, SMALL, ASY>(G, Kd, rk, ek, Nd, bn, ir), acc);
        ir += step;
        if (ir >= D2) ir -= D2;
    }
    return acc;
}

// Row state of a near-field tile for lane `lane` and the column start n.
struct NearRow {
    double Kd, rk, ek;
    int64_t ir, step;
    bool active;
};

__device__ __forceinline__ NearRow near_row(const GridArgs& G, const double* __restrict__ evec, const NearTile& T,
                                            int lane, int64_t n) {
    NearRow r;
    r.active = lane < T.nk;
    const int64_t k = T.k0 + (r.active ? lane : 0);
    const int64_t K = G.ar * k + G.br;
    r.Kd = (double)K;
    r.rk = (double)K / (double)G.Dr;
    r.ek = G.row_pert ? evec[k - 1] : 0.0;
    const int64_t D2 = 2 * G.D;
    r.ir = (K * (G.ac * n + G.bc)) % D2;
    r.step = (K * 4 * G.ac) % D2;
    return r;
}

// One workgroup = 64 rows (one per lane) x a column range; its 4 waves take
// every 4th column (wave-uniform, so the column data are scalar loads) and
// their sums are added in a fixed order.  The tile's flags (host-computed
// bounds on z over the tile) select the Hankel term count and the branches.
__global__ __launch_bounds__(256) void k_near(const NearProb* __restrict__ probs,
                                              const NearTile* __restrict__ tiles,
                                              double* __restrict__ partial) {
    __shared__ double red[4][64];
    const NearTile T = tiles[blockIdx.x];
    const GridArgs G = probs[T.prob].G; // by value: scalar registers, loaded once
    const double* c = probs[T.prob].c;
    const double* bvec = probs[T.prob].b;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t n = T.n0 + wave;
    const NearRow R = near_row(G, probs[T.prob].e, T, lane, n);
    const bool small = T.flags & 1, asy = T.flags & 2;
    const int M = T.flags >> 8;
    double acc = 0.0;
#define SWEEP(M_, S_, A_) near_sweep<M_, S_, A_>(G, c, bvec, n, T.n1, R.Kd, R.rk, R.ek, R.ir, R.step)
    if (!asy) {
        acc = SWEEP(3, true, false);
    } else if (small) {
        acc = SWEEP(12, true, true);
    } else {
        switch (M) {
        case 3: acc = SWEEP(3, false, true); break;
        case 4: acc = SWEEP(4, false, true); break;
        case 5: acc = SWEEP(5, false, true); break;
        case 6: acc = SWEEP(6, false, true); break;
        case 8: acc = SWEEP(8, false, true); break;
        default: acc = SWEEP(12, false, true); break;
        }
    }
#undef SWEEP
    red[wave][lane] = R.active ? acc : 0.0;
    __syncthreads();
    if (wave == 0)
        partial[T.pbase + lane] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Many right-hand sides: the tile's J_0 values are evaluated once, 64 columns
// at a time, into LDS, and applied to every right-hand side -- a
// (64 rows x 64 columns) by (64 columns x nrhs) product per step.  With MFMA
// (nrhs >= 16) wave w owns rows 16w..16w+15 and all right-hand-side blocks of
// 16 on v_mfma_f64_16x16x4f64; otherwise thread (row, wave) accumulates the
// right-hand sides j = wave, wave+4, wave+8, wave+12 with FMAs.
template <int M, bool SMALL, bool ASY, bool MFMA>
__device__ __forceinline__ void near_multi_body(const NearProb& P, const NearTile& T, double (*Js)[65],
                                                double (*Cs)[65], double* __restrict__ partial) {
    const GridArgs& G = P.G;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int nr = P.nrhs;
    NearRow R = near_row(G, P.e, T, lane, T.n0 + wave);
    const int64_t D2 = 2 * G.D;
    v4d accm[4];
    double acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        accm[i] = v4d{0.0, 0.0, 0.0, 0.0};
        acc[i] = 0.0;
    }
    for (int64_t nb = T.n0; nb < T.n1; nb += 64) {
        // J tile: wave w fills columns w, w+4, ..., w+60 for its lane's row
#pragma unroll 4
        for (int i = 0; i < 16; ++i) {
            const int col = wave + 4 * i;
            const int64_t n = nb + col;
            double J = 0.0;
            if (n < T.n1) {
                const double bn = G.col_pert ? P.b[n - 1] : 0.0;
                J = near_j0<M, SMALL, ASY>(G, R.Kd, R.rk, R.ek, (double)(G.ac * n + G.bc), bn, R.ir);
            }
            Js[col][lane] = R.active ? J : 0.0;
            R.ir += R.step;
            if (R.ir >= D2) R.ir -= D2;
        }
        // coefficient tile: Cs[col][j] = c_j[nb + col]
#pragma unroll 4
        for (int i = 0; i < 16; ++i) {
            const int j = (t >> 6) + 4 * i;
            const int64_t n = nb + lane;
            Cs[lane][j] = (j < nr && n < T.n1) ? P.c[(int64_t)j * P.ldc + n - 1] : 0.0;
        }
        __syncthreads();
        if (MFMA) {
            // A (16x4): lane -> row l%16, k l/16;  B (4x16): lane -> k l/16, column l%16
            const int ar = 16 * wave + (lane & 15), kq = lane >> 4;
            for (int kc = 0; kc < 16; ++kc) {
                const double a = Js[4 * kc + kq][ar];
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) {
                    if (16 * jb < nr) {
                        const double b = Cs[4 * kc + kq][16 * jb + (lane & 15)];
                        accm[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, accm[jb], 0, 0, 0);
                    }
                }
            }
        } else {
            for (int col = 0; col < 64; ++col) {
                const double J = Js[col][lane];
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[i] = fma(J, Cs[col][wave + 4 * i], acc[i]);
            }
        }
        __syncthreads();
    }
    if (MFMA) {
        // D (16x16): lane l, register r -> row l/16 + 4r, column l%16 (FP64 layout)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            const int j = 16 * jb + (lane & 15);
            if (j < nr) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    partial[T.pbase + (int64_t)j * 64 + 16 * wave + (lane >> 4) + 4 * r] = accm[jb][r];
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = wave + 4 * i;
            if (j < nr) partial[T.pbase + (int64_t)j * 64 + lane] = acc[i];
        }
    }
}

template <bool MFMA>
__global__ __launch_bounds__(256) void k_near_multi(const NearProb* __restrict__ probs,
                                                    const NearTile* __restrict__ tiles,
                                                    double* __restrict__ partial) {
    __shared__ double Js[64][65];
    __shared__ double Cs[64][65];
    const NearTile T = tiles[blockIdx.x];
    const NearProb P = probs[T.prob]; // by value: scalar registers, loaded once
    const bool small = T.flags & 1, asy = T.flags & 2;
    const int M = T.flags >> 8;
    if (!asy) {
        near_multi_body<3, true, false, MFMA>(P, T, Js, Cs, partial);
    } else if (small) {
        near_multi_body<12, true, true, MFMA>(P, T, Js, Cs, partial);
    } else {
        switch (M) {
        case 3: near_multi_body<3, false, true, MFMA>(P, T, Js, Cs, partial); break;
        case 4: near_multi_body<4, false, true, MFMA>(P, T, Js, Cs, partial); break;
        case 5: near_multi_body<5, false, true, MFMA>(P, T, Js, Cs, partial); break;
        case 6: near_multi_body<6, false, true, MFMA>(P, T, Js, Cs, partial); break;
        case 8: near_multi_body<8, false, true, MFMA>(P, T, Js, Cs, partial); break;
        default: near_multi_body<12, false, true, MFMA>(P, T, Js, Cs, partial); break;
        }
    }
}

// f_k = sum of the row's tile partials, per right-hand side; 4 waves take
// every 4th tile and their sums are combined in a fixed order.
__global__ __launch_bounds__(256) void k_near_reduce(const RowTile* __restrict__ rt,
                                                     const double* __restrict__ partial) {
    __shared__ double red[4][64];
    const RowTile R = rt[blockIdx.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t per_tile = (int64_t)R.nrhs * 64;
    for (int j = 0; j < R.nrhs; ++j) {
        double s = 0.0;
        for (int64_t t = wave; t < R.ntiles; t += 4) s += partial[R.pbase + t * per_tile + (int64_t)j * 64 + lane];
        red[wave][lane] = s;
        __syncthreads();
        if (wave == 0 && lane < R.nk)
            R.f[(int64_t)j * R.ldo + R.k0 + lane - 1] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        __syncthreads();
    }
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

// Pass A on a block's data: y_n' = q(n') c_n X_g(n), column FFTs over j2, for
// every right-hand side and group of the descriptor.  Per column position the
// group-independent factors are kept:
//   qb = q(n') (w^_n/w0)^(-1/2),  vw = w^_n/w0,  x = (b_n/bref)/vw,  la = lambda_n/lref
// and X_g = la^a vw^e sum_b K_{g,b} x^b, with vw^e updated incrementally over
// the groups (sorted by a, then e).
template <typename F, int L2, int W>
__global__ __launch_bounds__(W * L2 / 8) void k_pass_a(const FarDesc* __restrict__ descs,
                                                       const WgMap* __restrict__ wmap) {
    constexpr int R = 8, NTC = L2 / R;
    __shared__ cx<F> sh[W * (L2 + L2 / 8)];
    const WgMap mp = wmap[blockIdx.x];
    const FarDesc& D = descs[mp.desc];
    const FarArgs& A = D.A;
    const int t = threadIdx.x, w = t % W, tt = t / W;
    const int64_t j1 = (int64_t)mp.wg * W + w;
    cx<F>* my = sh + w * (L2 + L2 / 8);
    const int ng = A.g1 - A.g0;
    cx<F>* buf = (cx<F>*)D.buf;

    double vw[R], xb[R], la[R], pw[R];
    cx<double> qb[R];
    int32_t nidx[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t np = j1 + (int64_t)A.L1 * (tt + r * NTC);
        vw[r] = 1.0;
        xb[r] = la[r] = 0.0;
        qb[r] = mk(0.0, 0.0);
        nidx[r] = -1;
        if (np < A.ncols) {
            const int64_t n = A.na + np;
            const int64_t Nn = A.ac * n + A.bc;
            const double wn = (double)Nn * A.pi_Qc;
            const double bn = A.col_pert ? D.b[n - 1] : 0.0;
            vw[r] = wn / A.w0;
            const double iw = 1.0 / vw[r];
            xb[r] = (bn / A.bref) * iw;
            la[r] = (wn + bn) / A.lref;
            qb[r] = cscale(expi_ratio(2 * A.Kka * A.ac * np + A.ar * A.ac * np * np, 2 * A.D), sqrt(iw));
            nidx[r] = int32_t(n - 1);
        }
    }
    {
        const int j = mp.j;
        const int gs = A.g0 + mp.chunk * D.gchunk, ge = min(A.g1, gs + D.gchunk);
        const double* cj = D.c + (int64_t)j * D.ldc;
        double cv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) cv[r] = nidx[r] >= 0 ? cj[nidx[r]] : 0.0;
        int ecur = 0, acur = 0;
        for (int g = gs; g < ge; ++g) {
            const GroupDev Gd = A.groups[g];
            if (Gd.a != acur || g == gs) { // restart the powers
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
                if (nidx[r] >= 0) // zero padding otherwise
                    for (int ti = Gd.t0; ti < Gd.t1; ++ti) {
                        const TermDev Td = A.terms[ti];
                        while (bcur < Td.b) {
                            xp *= xb[r];
                            ++bcur;
                        }
                        Xr = fma(Td.kre, xp, Xr);
                        Xi = fma(Td.kim, xp, Xi);
                    }
                const double sc = pw[r] * cv[r];
                const cx<double> y = cmul(mk(Xr * sc, Xi * sc), qb[r]);
                v[r] = mk(F(y.x), F(y.y));
            }
            fft_reg<F, L2, R, -1>(v, my, tt);
            cx<F>* out = buf + ((int64_t)j * ng + (g - A.g0)) * A.L;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t m2 = tt + r * NTC;
                out[m2 * A.L1 + j1] = cmul(v[r], tw_big<F>(j1 * m2, A.twshift));
            }
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

// Pass B: row FFT, product with H^, inverse row FFT, inverse twiddle; in place,
// for every (right-hand side, group) of the descriptor.
// HANK_PASSB_HREG 1: H^ and the inverse twiddles of the row are held in
// registers across the groups; 0: re-read per group (L2 hits), fewer registers.
#ifndef HANK_PASSB_HREG
#define HANK_PASSB_HREG 1
#endif
template <typename F, int L1, int ROWS>
__global__ __launch_bounds__(ROWS * L1 / 8) void k_pass_b(const FarDesc* __restrict__ descs,
                                                           const WgMap* __restrict__ wmap) {
    constexpr int R = 8, NTR = L1 / R;
    __shared__ cx<F> sh[ROWS * (L1 + L1 / 8)];
    const WgMap mp = wmap[blockIdx.x];
    const FarDesc& D = descs[mp.desc];
    const FarArgs& A = D.A;
    const int t = threadIdx.x, rl = t / NTR, tt = t % NTR;
    const int64_t row = (int64_t)mp.wg * ROWS + rl;
    const bool okrow = row < A.L2;
    const int64_t rowc = okrow ? row : 0;
    cx<F>* my = sh + rl * (L1 + L1 / 8);
    const cx<F>* hrow = (const cx<F>*)D.H + rowc * L1;
    cx<F>* buf = (cx<F>*)D.buf;
#if HANK_PASSB_HREG
    cx<F> hv[R], tw[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        hv[r] = hrow[tt + r * NTR];
        const cx<F> w = tw_big<F>((int64_t)(tt + r * NTR) * rowc, A.twshift);
        tw[r] = mk(w.x, -w.y);
    }
#endif
    const int ng = A.g1 - A.g0;
    const int gs = mp.chunk * D.gchunk, ge = min(ng, gs + D.gchunk);
    for (int gq = gs; gq < ge; ++gq) {
        const int64_t q = (int64_t)mp.j * ng + gq;
        cx<F>* p = buf + q * A.L + rowc * L1;
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
// A_g(k) = scale_g (e_k/eref)^a (r^_k/r0)^(e - 1/2), per right-hand side, with
// the power of r^_k/r0 updated incrementally over the groups.
template <typename F, int L2, int W>
__global__ __launch_bounds__(W * L2 / 8) void k_pass_c(const FarDesc* __restrict__ descs,
                                                       const WgMap* __restrict__ wmap) {
    constexpr int R = 8, NTC = L2 / R;
    __shared__ cx<F> sh[W * (L2 + L2 / 8)];
    const WgMap mp = wmap[blockIdx.x];
    const FarDesc& D = descs[mp.desc];
    const FarArgs& A = D.A;
    const int t = threadIdx.x, w = t % W, tt = t / W;
    const int64_t j1 = (int64_t)mp.wg * W + w;
    cx<F>* my = sh + w * (L2 + L2 / 8);
    const int ng = A.g1 - A.g0;
    const cx<F>* buf = (const cx<F>*)D.buf;
    double rho[R], ek[R], acc[R], pw[R];
    cx<double> pk[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t kp = j1 + (int64_t)A.L1 * (tt + r * NTC);
        rho[r] = 1.0;
        ek[r] = 0.0;
        pk[r] = mk(0.0, 0.0);
        if (kp < A.nrows) {
            const int64_t k = A.ka + kp;
            rho[r] = ((double)(A.ar * k + A.br) / (double)A.Dr) / A.r0;
            ek[r] = A.row_pert ? D.e[k - 1] / A.eref : 0.0;
            pk[r] = cscale(expi_ratio(2 * A.Kka * A.Nna + 2 * A.ar * A.Nna * kp + A.ar * A.ac * kp * kp, 2 * A.D),
                           1.0 / sqrt(rho[r]));
        }
    }
    {
        const int j = mp.j;
        const int gs = A.g0 + mp.chunk * D.gchunk, ge = min(A.g1, gs + D.gchunk);
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        int ecur = 0, acur = 0;
        for (int g = gs; g < ge; ++g) {
            const GroupDev Gd = A.groups[g];
            if (Gd.a != acur || g == gs) {
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
            const cx<F>* p = buf + ((int64_t)j * ng + (g - A.g0)) * A.L;
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
        if (D.nchunk == 1) {
            double* fj = D.f + (int64_t)j * D.ldo;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t kp = j1 + (int64_t)A.L1 * (tt + r * NTC);
                if (kp < A.nrows) fj[A.ka + kp - 1] += acc[r];
            }
        } else {
            double* pj = D.part + ((int64_t)j * D.nchunk + mp.chunk) * A.nrows;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t kp = j1 + (int64_t)A.L1 * (tt + r * NTC);
                if (kp < A.nrows) pj[kp] = acc[r];
            }
        }
    }
}

// f += sum of the pass-C chunk sums, in chunk order (deterministic)
__global__ __launch_bounds__(256) void k_far_reduce(const FarDesc* __restrict__ descs,
                                                    const WgMap* __restrict__ wmap) {
    const WgMap mp = wmap[blockIdx.x];
    const FarDesc& D = descs[mp.desc];
    const int64_t kp = (int64_t)mp.wg * 256 + threadIdx.x;
    if (kp >= D.A.nrows) return;
    const double* pj = D.part + (int64_t)mp.j * D.nchunk * D.A.nrows + kp;
    double s = 0.0;
    for (int q = 0; q < D.nchunk; ++q) s += pj[(int64_t)q * D.A.nrows];
    D.f[(int64_t)mp.j * D.ldo + D.A.ka + kp - 1] += s;
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

hipError_t launch_near(const NearProb* probs, const NearTile* tiles, int64_t ntiles, double* partial,
                       hipStream_t s) {
    if (ntiles > 0) hipLaunchKernelGGL(k_near, dim3((unsigned)ntiles), dim3(256), 0, s, probs, tiles, partial);
    return hipGetLastError();
}

hipError_t launch_near_multi(const NearProb* probs, const NearTile* tiles, int64_t ntiles, bool mfma,
                             double* partial, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (mfma)
        hipLaunchKernelGGL(k_near_multi<true>, dim3((unsigned)ntiles), dim3(256), 0, s, probs, tiles, partial);
    else
        hipLaunchKernelGGL(k_near_multi<false>, dim3((unsigned)ntiles), dim3(256), 0, s, probs, tiles, partial);
    return hipGetLastError();
}

hipError_t launch_near_reduce(const RowTile* rt, int64_t nrt, const double* partial, hipStream_t s) {
    if (nrt > 0) hipLaunchKernelGGL(k_near_reduce, dim3((unsigned)nrt), dim3(256), 0, s, rt, partial);
    return hipGetLastError();
}

// column passes: which 0 = A on data, 1 = A on the chirp kernel, 2 = C
template <typename F, int L2>
static void pass_ac_dispatch(int which, const FarArgs* A, const FarDesc* descs, const WgMap* map, int64_t nwg,
                             void* buf, hipStream_t s) {
    constexpr int W = 8;
    dim3 block(W * L2 / 8);
    if (which == 0)
        hipLaunchKernelGGL((k_pass_a<F, L2, W>), dim3((unsigned)nwg), block, 0, s, descs, map);
    else if (which == 1)
        hipLaunchKernelGGL((k_pass_a_kernel<F, L2, W>), dim3((unsigned)(A->L1 / W)), block, 0, s, *A, (cx<F>*)buf);
    else
        hipLaunchKernelGGL((k_pass_c<F, L2, W>), dim3((unsigned)nwg), block, 0, s, descs, map);
}

template <typename F>
static hipError_t pass_ac(int which, int32_t L2, const FarArgs* A, const FarDesc* descs, const WgMap* map,
                          int64_t nwg, void* buf, hipStream_t s) {
    switch (L2) {
    case 8: pass_ac_dispatch<F, 8>(which, A, descs, map, nwg, buf, s); break;
    case 16: pass_ac_dispatch<F, 16>(which, A, descs, map, nwg, buf, s); break;
    case 32: pass_ac_dispatch<F, 32>(which, A, descs, map, nwg, buf, s); break;
    case 64: pass_ac_dispatch<F, 64>(which, A, descs, map, nwg, buf, s); break;
    case 128: pass_ac_dispatch<F, 128>(which, A, descs, map, nwg, buf, s); break;
    case 256: pass_ac_dispatch<F, 256>(which, A, descs, map, nwg, buf, s); break;
    case 512: pass_ac_dispatch<F, 512>(which, A, descs, map, nwg, buf, s); break;
    case 1024: pass_ac_dispatch<F, 1024>(which, A, descs, map, nwg, buf, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int L1>
constexpr int rows_per_wg() {
    return (L1 >= 2048) ? 1 : 2048 / L1;
}

// row passes: fwd_only = the chirp spectrum (one block by value), else pass B
template <typename F, int L1>
static void pass_b_dispatch(bool fwd_only, const FarArgs* A, const FarDesc* descs, const WgMap* map,
                            int64_t nwg, void* buf, void* H, hipStream_t s) {
    constexpr int ROWS = rows_per_wg<L1>();
    dim3 block(ROWS * L1 / 8);
    if (fwd_only)
        hipLaunchKernelGGL((k_pass_b_fwd<F, L1, ROWS>), dim3((unsigned)((A->L2 + ROWS - 1) / ROWS)), block, 0, s, *A,
                           (const cx<F>*)buf, (cx<F>*)H);
    else
        hipLaunchKernelGGL((k_pass_b<F, L1, ROWS>), dim3((unsigned)nwg), block, 0, s, descs, map);
}

template <typename F>
static hipError_t pass_b(bool fwd_only, int32_t L1, const FarArgs* A, const FarDesc* descs, const WgMap* map,
                         int64_t nwg, void* buf, void* H, hipStream_t s) {
    switch (L1) {
    case 8: pass_b_dispatch<F, 8>(fwd_only, A, descs, map, nwg, buf, H, s); break;
    case 16: pass_b_dispatch<F, 16>(fwd_only, A, descs, map, nwg, buf, H, s); break;
    case 32: pass_b_dispatch<F, 32>(fwd_only, A, descs, map, nwg, buf, H, s); break;
    case 64: pass_b_dispatch<F, 64>(fwd_only, A, descs, map, nwg, buf, H, s); break;
    case 128: pass_b_dispatch<F, 128>(fwd_only, A, descs, map, nwg, buf, H, s); break;
    case 256: pass_b_dispatch<F, 256>(fwd_only, A, descs, map, nwg, buf, H, s); break;
    case 512: pass_b_dispatch<F, 512>(fwd_only, A, descs, map, nwg, buf, H, s); break;
    case 1024: pass_b_dispatch<F, 1024>(fwd_only, A, descs, map, nwg, buf, H, s); break;
    case 2048: pass_b_dispatch<F, 2048>(fwd_only, A, descs, map, nwg, buf, H, s); break;
    case 4096: pass_b_dispatch<F, 4096>(fwd_only, A, descs, map, nwg, buf, H, s); break;
    case 8192: pass_b_dispatch<F, 8192>(fwd_only, A, descs, map, nwg, buf, H, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int32_t far_rows_per_wg(int32_t L1) { return L1 >= 2048 ? 1 : 2048 / L1; }

hipError_t launch_far_reduce(const FarDesc* descs, const WgMap* map, int64_t nwg, hipStream_t s) {
    if (nwg > 0) hipLaunchKernelGGL(k_far_reduce, dim3((unsigned)nwg), dim3(256), 0, s, descs, map);
    return hipGetLastError();
}

hipError_t launch_chirp_spectrum(const FarArgs& A, bool fp32, void* work, void* H, hipStream_t s) {
    hipError_t e = fp32 ? pass_ac<float>(1, A.L2, &A, nullptr, nullptr, 0, work, s)
                        : pass_ac<double>(1, A.L2, &A, nullptr, nullptr, 0, work, s);
    if (e != hipSuccess) return e;
    return fp32 ? pass_b<float>(true, A.L1, &A, nullptr, nullptr, 0, work, H, s)
                : pass_b<double>(true, A.L1, &A, nullptr, nullptr, 0, work, H, s);
}

hipError_t launch_far_pass(int which, bool fp32, int32_t L1, int32_t L2, const FarDesc* descs, const WgMap* map,
                           int64_t nwg, hipStream_t s) {
    if (nwg <= 0) return hipSuccess;
    if (which == 1)
        return fp32 ? pass_b<float>(false, L1, nullptr, descs, map, nwg, nullptr, nullptr, s)
                    : pass_b<double>(false, L1, nullptr, descs, map, nwg, nullptr, nullptr, s);
    const int w = (which == 0) ? 0 : 2;
    return fp32 ? pass_ac<float>(w, L2, nullptr, descs, map, nwg, nullptr, s)
                : pass_ac<double>(w, L2, nullptr, descs, map, nwg, nullptr, s);
}

} // namespace hank
