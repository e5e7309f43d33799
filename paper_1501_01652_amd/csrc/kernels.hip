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

#include <map>
#include <mutex>

#include "fft_device.h"

namespace hank {

__device__ DeviceTables g_tab;

// Workspace of the allocation-free entry point: a file-scope device array
// (each GPU holds its own copy, at its own address, until the process ends).
// Host code never passes its name to a kernel or a copy: it takes the address
// that noalloc_scratch returns for the current device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(void** ptr) {
    static std::mutex mu;
    static std::map<int, void*> addr; // device -> address of its copy of scratch
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        it = addr.emplace(dev, p).first;
    }
    *ptr = it->second;
    return hipSuccess;
}

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

// b[n-1] for n <= nmax (if b is given) and, for n <= nv, the weights
// v[n-1] = 2 / J_1(j_{0,n})^2 of the self-inverse relation of the DHT (Sec. 6):
// J_1 at the root is -J_0' there, the by-product of the last Newton step.
__global__ void k_roots(int64_t nmax, double* b, int64_t nv, double* v) {
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
        if (v && n <= nv) {
            const double z = beta + x;
            int i = (int)((z - J0_TAYLOR_Z0) * (1.0 / J0_TAYLOR_H));
            i = i < 0 ? 0 : (i >= J0_TAYLOR_INTERVALS ? J0_TAYLOR_INTERVALS - 1 : i);
            const double zc = J0_TAYLOR_Z0 + (i + 0.5) * J0_TAYLOR_H;
            double J, dJ;
            j0_taylor_piece(i, (beta - zc) + (beta_lo + x), &J, &dJ);
            v[n - 1] = 2.0 / (dJ * dJ);
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
        if (v && n <= nv) {
            // |J_1(z)| = sqrt(2/(pi z)) |P1 cos x - Q1 sin x| at z = (n - 1/4) pi + x
            const double z = beta + x, zi = 1.0 / z;
            double P1, Q1, s, c;
            hankel_pq(1, zi, hankel_terms_for(z), &P1, &Q1);
            sincos_small(x, &s, &c);
            const double a = P1 * c - Q1 * s;
            v[n - 1] = M_PI * z / (a * a);
        }
    }
    if (b) b[n - 1] = x;
}

// dst[i] = src[i] v[i] for i < N, times 1/j_{0,N+1}^2 (j_{0,N+1} = (N + 3/4) pi
// + b[N]) when final is set: the diagonal factors of the self-inverse relation
__global__ void k_dht_scale(int64_t N, const double* __restrict__ v, const double* b, const double* src,
                            double* dst, int final) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double w = v[i];
    if (final) {
        const double S = ((double)N + 0.75) * M_PI + b[N];
        w /= S * S;
    }
    dst[i] = src[i] * w;
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
// coefficients of P_0 and Q_0 (Sec. 3.1), times `scale`; for the scaled
// amplitude Y = S z^{-1/2} (S a power of two, so the scaling is exact) the
// j-th coefficient of P is divided by S^(4j+1) and that of Q by S^(4j+3):
// with Z = Y^2, W = Z^2, Y (cos P'(W) - sin Z Q'(W)) is the unscaled form
constexpr Hankel0 make_hankel0(double scale = 1.0, double S = 1.0) {
    Hankel0 h{};
    double a = scale, d = S; // d = S^(2m+1): 4j+1 for P (m = 2j), 4j+3 for Q (m = 2j+1)
    for (int m = 0; m < 24; ++m) {
        if (m > 0) a *= -double(2 * m - 1) * double(2 * m - 1) / (8.0 * m);
        const double sg = ((m / 2) & 1) ? -1.0 : 1.0;
        if (m & 1)
            h.q[m / 2] = sg * a / d;
        else
            h.p[m / 2] = sg * a / d;
        d *= S * S;
    }
    return h;
}

// z^{-1/2}: hardware estimate and Newton steps, two to full precision; one
// when lean (the estimate's relative error is about 2^-23, one step leaves
// about 1e-14)
__device__ __forceinline__ double rsqrt_nr(double z, bool lean) {
    double y = __builtin_amdgcn_rsq(z);
    const double h = 0.5 * z;
    y = y * fma(-h * y, y, 1.5);
    if (!lean) y = y * fma(-h * y, y, 1.5);
    return y;
}
__device__ __forceinline__ double rsqrt_full(double z) { return rsqrt_nr(z, false); }

// Y = S z^{-1/2} by the same Newton steps with the factor 1/2 left out
// (S = 2 after one step, 16 after two; make_hankel0 folds S into the
// coefficients): one multiplication per step fewer
__device__ __forceinline__ double rsqrt_scaled(double z, bool lean) {
    const double y = __builtin_amdgcn_rsq(z);
    const double Y = y * fma(-z * y, y, 3.0);
    if (lean) return Y;
    return Y * fma(-z * Y, Y, 12.0);
}
constexpr double rsqrt_scale(bool lean) { return lean ? 2.0 : 16.0; }

// sin and cos of a residual phase |x| < 0.06 (Taylor; the first omitted terms
// are below 1e-17; lean, the series to x^5 and x^4: below 6.5e-11)
__device__ __forceinline__ void sincos_tiny(double x, double* s, double* c, bool lean = false) {
    const double x2 = x * x;
    if (lean) {
        *s = x * fma(x2, fma(x2, 1.0 / 120.0, -1.0 / 6.0), 1.0);
        *c = fma(x2, fma(x2, 1.0 / 24.0, -0.5), 1.0);
        return;
    }
    *s = x * fma(x2, fma(x2, fma(x2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), 1.0);
    *c = fma(x2, fma(x2, fma(x2, fma(x2, 1.0 / 40320.0, -1.0 / 720.0), 1.0 / 24.0), -0.5), 1.0);
}

// Workgroup-uniform read-only records (a block's group and term tables, a
// near-field tile) read through the constant address space from a
// readfirstlane'd base: their fields then come through scalar loads into
// scalar registers, and the loops they drive are uniform branches instead of
// masked vector loops.
template <typename T>
__device__ __forceinline__ T scalar_entry(const T* p, int i) {
    static_assert(sizeof(T) % 4 == 0, "whole words");
    typedef const __attribute__((address_space(4))) uint32_t cword;
    const uint64_t a = reinterpret_cast<uint64_t>(p + i);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    cword* q = reinterpret_cast<cword*>(((uint64_t)hi << 32) | lo);
    uint32_t w[sizeof(T) / 4];
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) w[k] = q[k];
    T out;
    __builtin_memcpy(&out, w, sizeof(T));
    return out;
}

// Index of the last of n descriptors whose grid offset (member M) is <= bid:
// the descriptor of workgroup bid (offsets are non-decreasing; a descriptor
// with no workgroups is never the last one at or below a valid bid).
template <typename T, int64_t T::*M>
__device__ __forceinline__ int find_desc(const T* __restrict__ d, int n, int64_t bid) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].*M <= bid)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// State of one lane (one row k) sweeping the columns n, n+4, n+8, ... of a
// near-field tile.  With z = z~ + delta, z~ = pi K_k N_n / D (Lemma 3.2's
// split) the Hankel phase z - pi/4, in units of pi, is
//     L_n + rho_n / pi,   L_n = ir_n/D - 1/4 + e_k N_n / Qc,   rho_n = (e_k + r^_k) b_n,
// where ir_n = K_k N_n mod 2D is exact.  L_n grows by the same amount at every
// step, so u = e^{i pi L_n} is advanced by one complex rotation w and set
// afresh every 16 steps; e^{i rho_n} comes from sincos_tiny (b_n <= b_1 < 0.05).
// Integers (ir, N_n) are carried exactly in doubles.  For the amplitude and
// the P, Q series z is formed as al N_n + s_k b_n, al = pi K_k / D + pi e_k / Qc,
// s_k = e_k + r^_k (working precision, one FMA per column).
struct NearLane {
    double Kd, al, ek, sk;
    double ir, ir16, D2;
    double Nd, dNd;
    cx<double> u, w;
    bool active;
};

__device__ __forceinline__ NearLane near_lane(const GridArgs& G, const double* __restrict__ evec,
                                              const NearTile& T, int lane, int64_t n) {
    NearLane r;
    r.active = lane < T.nk;
    const int64_t k = T.k0 + (r.active ? lane : 0);
    const int64_t K = G.ar * k + G.br;
    const int64_t D2 = 2 * G.D;
    const int64_t Nn = G.ac * n + G.bc;
    const int64_t step = (K * 4 * G.ac) % D2;
    r.Kd = (double)K;
    const double rk = r.Kd / (double)G.Dr;
    r.ek = G.row_pert ? evec[k - 1] : 0.0;
    r.sk = r.ek + rk;
    r.al = fma(r.ek, G.pi_Qc, r.Kd * G.piD_hi);
    r.ir = (double)((K * Nn) % D2);
    r.ir16 = (double)((16 * step) % D2);
    r.D2 = (double)D2;
    r.Nd = (double)Nn;
    r.dNd = (double)(4 * G.ac);
    // w = e^{i pi step/D} (exactly reduced) times e^{i pi e_k 4 ac / Qc}
    double s0, c0, s1, c1;
    sincospi_ratio(step, G.D, &s0, &c0);
    sincos_tiny(M_PI * r.ek * r.dNd * G.invQc, &s1, &c1);
    r.w = cmul(mk(c0, s0), mk(c1, s1));
    r.u = mk(1.0, 0.0);
    return r;
}

// u = e^{i pi L_n} at the lane's current column
__device__ __forceinline__ void near_anchor(const GridArgs& G, NearLane& r) {
    double s, c;
    sincospi(fma(r.ir, G.invD, -0.25) + r.ek * r.Nd * G.invQc, &s, &c);
    r.u = mk(c, s);
}

// to the lane's column 16 steps on from the last anchor
__device__ __forceinline__ void near_skip16(NearLane& r) {
    r.ir += r.ir16;
    if (r.ir >= r.D2) r.ir -= r.D2;
}

// The first M coefficients of P and Q with sqrt(2/pi) folded in, held in
// scalar registers from the start of a block: as the addends of the Horner
// steps they are operands of three-address v_fma_f64 (constants the compiler
// keeps in vector registers are copied into the accumulator of v_fmac_f64 at
// every use instead).  The empty asm statements only pin the values to scalar
// registers once, outside the step loops.
template <int M>
struct HankelSet {
    double p[M], q[M];
};
template <int M, bool LEAN = false>
__device__ __forceinline__ HankelSet<M> hankel_set() {
    constexpr Hankel0 H = make_hankel0(0.79788456080286535588, rsqrt_scale(LEAN));
    HankelSet<M> h;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        double a = H.p[m], b = H.q[m];
        asm("" : "+s"(a));
        asm("" : "+s"(b));
        h.p[m] = a;
        h.q[m] = b;
    }
    return h;
}

// Hankel expansion (Sec. 3.1, M pairs of terms) at the lane's current column;
// bn = b_n (0 without column perturbations).  z only sets the amplitude and
// the P, Q series, so it is formed to working precision.
// LEAN (the plan's G.lean: per-entry budget of at least 1.25e-10): one Newton
// step for z^{-1/2} and the shorter residual sine and cosine.
// ROT1: the residual factor e^{i rho} to first order, 1 + i rho (blocks whose
// rho is small enough, chosen on the host).
template <int M, bool PERT, bool LEAN = false, bool ROT1 = false>
__device__ __forceinline__ double near_asy(const GridArgs& G, const NearLane& r, double bn,
                                           const HankelSet<M>& H) {
    // z = z~ + e_k (w^_n + b_n) + r^_k b_n = al N_n + rho, rho = s_k b_n
    const double x = PERT ? r.sk * bn : 0.0;
    const double z = PERT ? fma(r.al, r.Nd, x) : r.al * r.Nd;
    // H holds the coefficients for Y = S z^{-1/2}, Z = Y^2, W = Z^2
    const double Y = rsqrt_scaled(z, LEAN), Z = Y * Y, W = Z * Z;
    double P = H.p[M - 1], Q = H.q[M - 1];
#pragma unroll
    for (int m = M - 2; m >= 0; --m) {
        P = fma(P, W, H.p[m]);
        Q = fma(Q, W, H.q[m]);
    }
    double cs = r.u.x, sn = r.u.y;
    if (PERT && ROT1) {
        cs = fma(-r.u.y, x, r.u.x);
        sn = fma(r.u.x, x, r.u.y);
    } else if (PERT) {
        double s, c;
        sincos_tiny(x, &s, &c, LEAN);
        cs = fma(r.u.x, c, -r.u.y * s);
        sn = fma(r.u.y, c, r.u.x * s);
    }
    return Y * fma(cs, P, -sn * (Q * Z));
}

// z at the lane's current column with pi K N / D carried in two parts (the
// small-argument branch needs it to absolute accuracy)
__device__ __forceinline__ double near_z_at(const GridArgs& G, const NearLane& r, double Nd, double bn) {
    const double delta = fma(r.ek * Nd, G.pi_Qc, r.sk * bn);
    const double I = r.Kd * Nd; // exact: K_k N_n < 2^53
    const double pz = I * G.piD_hi;
    return (pz + (fma(I, G.piD_hi, -pz) + I * G.piD_lo)) + delta;
}
__device__ __forceinline__ double near_z_exact(const GridArgs& G, const NearLane& r, double bn) {
    return near_z_at(G, r, r.Nd, bn);
}

// The 8-term small-argument step of k_near (budgets from 1.25e-9 up): Taylor
// pieces on all of [0, 20) copied to LDS per workgroup, the first TAY_LDS_NT
// coefficients of each in rows of TAY_LDS_LD doubles (80 bytes: 16-byte
// aligned for 128-bit reads, and the rows of neighbouring pieces start in
// different banks), and z in the working-precision form al N_n + rho of the
// Hankel step (absolute error ~1e-14 below z = 20, far inside the budget),
// which the branch between the two then shares.  Build knob HANK_TAYLOR_LDS:
// 0 keeps the global table, the series below z = 2 and the compensated z.
#ifndef HANK_TAYLOR_LDS
#define HANK_TAYLOR_LDS 1
#endif
constexpr int TAY_LDS_NT = 8, TAY_LDS_LD = 10;
constexpr int TAY_LDS_PIECES = J0_TAYLOR0_PIECES + J0_TAYLOR_INTERVALS;

template <int NT, bool TL>
__device__ __forceinline__ double near_j0_small(double z, const double* tl) {
    if constexpr (TL)
        return j0_small_tab<NT, TAY_LDS_LD>(z, tl);
    else
        return j0_small<NT>(z);
}

// z for the branch at z = 20 and the small-argument step
template <bool PERT, bool TL>
__device__ __forceinline__ double near_z_small(const GridArgs& G, const NearLane& r, double Nd, double bn) {
    if constexpr (TL)
        return PERT ? fma(r.al, Nd, r.sk * bn) : r.al * Nd;
    else
        return near_z_at(G, r, Nd, bn);
}

// J_0 at the lane's current column, then one step on
// (both branches: each lane takes its own, so a wave pays for both only where
// its rows straddle z = 20).  TL: the small-argument step of the LDS pieces tl.
template <int M, bool SMALL, bool ASY, bool PERT, int NT = J0_TAYLOR_DEG, bool LEAN = false, bool ROT1 = false,
          bool TL = false>
__device__ __forceinline__ double near_step(const GridArgs& G, NearLane& r, double bn, const HankelSet<M>& H,
                                            const double* tl = nullptr) {
    double J;
    if (SMALL && ASY) {
        const double z = near_z_small<PERT, TL>(G, r, r.Nd, bn);
        if (z < J0_ASY_Z)
            J = near_j0_small<NT, TL>(z, tl);
        else
            J = near_asy<M, PERT, LEAN, ROT1>(G, r, bn, H);
    } else if (SMALL) {
        J = near_j0_small<NT, TL>(near_z_small<PERT, TL>(G, r, r.Nd, bn), tl);
    } else {
        J = near_asy<M, PERT, LEAN, ROT1>(G, r, bn, H);
    }
    if (ASY) r.u = cmul(r.u, r.w);
    r.Nd += r.dNd;
    return J;
}

// Build knobs (measured variants): unroll of the near-field column loop, and
// a lower bound on waves per SIMD for k_near (0: the compiler's choice).  With
// the Hankel coefficients in scalar registers the kernel fits 4 waves (at most
// 128 registers) without spilling, which measured 4% faster at N = 2^20 than
// 3 (slower by up to 10% on the small all-near Schlomilch N = 4096).
#ifndef HANK_NEAR_UNROLL
#define HANK_NEAR_UNROLL 4
#endif
#ifndef HANK_NEAR_PREFETCH
#define HANK_NEAR_PREFETCH 1
#endif
#ifndef HANK_NEAR_WPE
#define HANK_NEAR_WPE 4
#endif
#define HANK_STR2(x) #x
#define HANK_PRAGMA(x) _Pragma(HANK_STR2(x))

struct alignas(16) ColCB {
    double c, b;
};

// variant (NearVariant) of the 64-column block starting at column nb of a
// tile whose first column is n0; bv: the tile's bvar words, copied to LDS by
// the kernel (read with a uniform address; a per-lane copy of the tile would
// live in private memory)
__device__ __forceinline__ int tile_block_variant(const uint32_t* bv, int64_t n0, int64_t nb) {
    const int b = (int)((nb - n0) >> 6);
    return (int)((bv[b >> 3] >> (4 * (b & 7))) & 15u);
}

// One 64-column block of a sweep: the lane's columns p[0], p[4], ... (cnt of them)
template <int M, bool SMALL, bool ASY, bool PERT, int NT = J0_TAYLOR_DEG, bool LEAN = false, bool ROT1 = false>
__device__ __forceinline__ void near_block(const GridArgs& G, const ColCB* p, int cnt, NearLane& r, double& acc,
                                           const double* tl, bool anchor) {
    constexpr bool TL = HANK_TAYLOR_LDS && SMALL && NT <= TAY_LDS_NT;
    if (ASY && anchor) near_anchor(G, r);
    const HankelSet<M> H = hankel_set<M, LEAN>();
#if HANK_NEAR_PREFETCH
    // the next column's data read one step ahead (the read past the last
    // column lands in the 4 spare entries of cb)
    ColCB v = p[0];
    HANK_PRAGMA(unroll HANK_NEAR_UNROLL)
    for (int i = 0; i < cnt; ++i) {
        const ColCB vn = p[4 * (i + 1)];
        acc = fma(v.c, near_step<M, SMALL, ASY, PERT, NT, LEAN, ROT1, TL>(G, r, PERT ? v.b : 0.0, H, tl), acc);
        v = vn;
    }
#else
    HANK_PRAGMA(unroll HANK_NEAR_UNROLL)
    for (int i = 0; i < cnt; ++i) {
        const ColCB v = p[4 * i];
        acc = fma(v.c, near_step<M, SMALL, ASY, PERT, NT, LEAN, ROT1, TL>(G, r, PERT ? v.b : 0.0, H, tl), acc);
    }
#endif
}

// Internal code of the Hankel-only block with 6 pairs and the first-order
// residual factor (the Hankel side of NV_MIX6_8R; never stored in a tile).
constexpr int NV_M6R_WAVE = NV_COUNT;

// A block the host marked as taking both branches (NV_MIX*) may lie on one
// side of z = 20 for the 16 rows of this wave: z grows along a row, so the
// lanes' first and last columns decide.  Returns the variant that evaluates
// exactly the same branch for every entry of the wave: the small-argument or
// the Hankel code alone, or the mixed one.
// b0, b1: the root offsets of the lane's first and last column of the block
template <bool PERT, bool TL>
__device__ __forceinline__ int near_refine_mix(int v, const GridArgs& G, const NearLane& r, int cnt, double b0,
                                               double b1) {
    const bool small = near_z_small<PERT, TL>(G, r, r.Nd, b0) < J0_ASY_Z;
    const bool asy = !(near_z_small<PERT, TL>(G, r, fma(double(cnt - 1), r.dNd, r.Nd), b1) < J0_ASY_Z);
    const bool any_small = __ballot(small) != 0;
    const bool any_asy = __ballot(asy) != 0;
    if (any_small && any_asy) return v;
    const bool t8 = v == NV_MIX12_8 || v == NV_MIX6_8 || v == NV_MIX6_8R;
    if (!any_asy) return t8 ? NV_SMALL8 : NV_SMALL;
    return v == NV_MIX6_8R ? NV_M6R_WAVE : (v == NV_MIX12 || v == NV_MIX12_8) ? NV_M12 : NV_M6;
}

// Blocks of 64 columns (16 steps of a lane) between two settings of u from
// sincospi, where u was carried through the previous block: 1 with the full
// budget (the recurrence drifts by ~16 roundings per block), HANK_NEAR_ANCHOR
// with the lean one (64 steps drift by ~1e-14, far inside 1.25e-10).
#ifndef HANK_NEAR_ANCHOR
#define HANK_NEAR_ANCHOR 4
#endif

// Near-field sweep of one tile (one right-hand side) for the lane of column
// phase ph: columns T.n0 + ph, +4, ..., 16 per block of 64, coefficients and
// root offsets read from LDS (cb[i] is column T.n0 + i; the columns from T.n1
// to the next multiple of 4 carry c = 0, so that every lane of a block takes
// the same number of steps).  The variant is chosen per block (wave-uniform).
// A block of the small-argument step alone leaves u behind, so the next
// block sets it afresh.
template <bool PERT, bool LEAN>
__device__ __forceinline__ double near_sweep(const GridArgs& G, const ColCB* cb, const uint32_t* bv,
                                             const double* tl, const NearTile& T, int ph, NearLane& r) {
    double acc = 0.0;
    bool carried = false; // u is current at this block's first column
    int since = 0;        // blocks since u was set
    for (int64_t nb = T.n0; nb < T.n1; nb += 64) {
        const int cnt = ((int)min<int64_t>(64, T.n1 - nb) + 3) >> 2;
        const ColCB* p = cb + (nb - T.n0) + ph;
        int v = tile_block_variant(bv, T.n0, nb);
        if (v == NV_MIX12 || v == NV_MIX6)
            v = near_refine_mix<PERT, false>(v, G, r, cnt, p[0].b, p[4 * (cnt - 1)].b);
        else if (v == NV_MIX12_8 || v == NV_MIX6_8 || v == NV_MIX6_8R)
            v = near_refine_mix<PERT, HANK_TAYLOR_LDS != 0>(v, G, r, cnt, p[0].b, p[4 * (cnt - 1)].b);
        const bool anchor = !(LEAN && carried && since < HANK_NEAR_ANCHOR - 1);
        since = anchor ? 0 : since + 1;
        carried = !(v == NV_SMALL || v == NV_SMALL8);
#define BLOCK(M_, S_, A_) near_block<M_, S_, A_, PERT, J0_TAYLOR_DEG, LEAN>(G, p, cnt, r, acc, tl, anchor); break
#define BLOCK8(M_, A_) near_block<M_, true, A_, PERT, 8, LEAN>(G, p, cnt, r, acc, tl, anchor); break
#define BLOCKR(M_, S_, A_, NT_) near_block<M_, S_, A_, PERT, NT_, LEAN, PERT>(G, p, cnt, r, acc, tl, anchor); break
        switch (v) {
        case NV_M6R_WAVE: BLOCKR(6, false, true, J0_TAYLOR_DEG);
        case NV_M2R: BLOCKR(2, false, true, J0_TAYLOR_DEG);
        case NV_M3R: BLOCKR(3, false, true, J0_TAYLOR_DEG);
        case NV_M4R: BLOCKR(4, false, true, J0_TAYLOR_DEG);
        case NV_MIX6_8R: BLOCKR(6, true, true, 8);
        case NV_SMALL: BLOCK(3, true, false);
        case NV_MIX12: BLOCK(12, true, true);
        case NV_MIX6: BLOCK(6, true, true);
        case NV_SMALL8: BLOCK8(3, false);
        case NV_MIX12_8: BLOCK8(12, true);
        case NV_MIX6_8: BLOCK8(6, true);
        case NV_M2: BLOCK(2, false, true);
        case NV_M3: BLOCK(3, false, true);
        case NV_M4: BLOCK(4, false, true);
        case NV_M6: BLOCK(6, false, true);
        case NV_M8: BLOCK(8, false, true);
        default: BLOCK(12, false, true);
        }
#undef BLOCKR
#undef BLOCK8
#undef BLOCK
        near_skip16(r);
    }
    return acc;
}

// One workgroup = 64 rows x a column range of at most NEAR_TILE_COLS.  Wave w
// takes rows 16w .. 16w+15 of the tile (lane l: row 16w + l%16) and lane l
// every 4th column from phase l/16, so a wave's rows straddle z = 20 over
// fewer columns than 64 rows would; the four phase sums of a row are added in
// a fixed order, into the tile's partial slot or, for the only tile of its
// rows, into f.  One kernel serves every variant, so that tiles of all kinds
// share a launch and fill the chip together.
__global__ __launch_bounds__(256)
#if HANK_NEAR_WPE
__attribute__((amdgpu_waves_per_eu(HANK_NEAR_WPE)))
#endif
void k_near(const NearProb* __restrict__ probs, int nprob, double* __restrict__ partial) {
    __shared__ ColCB cb[NEAR_TILE_COLS + 4];
    __shared__ double red[4][64];
    __shared__ uint32_t sbv[4];
    __shared__ __align__(16) double tl[HANK_TAYLOR_LDS ? TAY_LDS_PIECES * TAY_LDS_LD : 2];
    const NearProb& P = probs[find_desc<NearProb, &NearProb::tile_start>(probs, nprob, blockIdx.x)];
    const NearTile T = scalar_entry(P.tiles, (int)(blockIdx.x - P.tile_start));
    if (threadIdx.x < 4) sbv[threadIdx.x] = P.tiles[blockIdx.x - P.tile_start].bvar[threadIdx.x];
    double* out = partial + P.pbase + T.slot * 64;
    const GridArgs G = P.G; // by value: scalar registers, loaded once
    const auto c = gview(P.c);
    const auto bvec = gview(P.b);
    const double* evec = P.e;
    const int ncol = (int)(T.n1 - T.n0);
    for (int i = threadIdx.x; i < ((ncol + 3) & ~3); i += 256) {
        ColCB v{0.0, 0.0};
        if (i < ncol) {
            v.c = c[T.n0 - 1 + i];
            v.b = G.col_pert ? bvec[T.n0 - 1 + i] : 0.0;
        }
        cb[i] = v;
    }
    if (HANK_TAYLOR_LDS)
        for (int i = threadIdx.x; i < TAY_LDS_PIECES * TAY_LDS_NT; i += 256) {
            const int pc = i / TAY_LDS_NT, u = i % TAY_LDS_NT;
            tl[pc * TAY_LDS_LD + u] =
                pc < J0_TAYLOR0_PIECES ? g_tab.tay0[pc][u] : g_tab.tay[pc - J0_TAYLOR0_PIECES][u];
        }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int row = 16 * wave + (lane & 15), ph = lane >> 4;
    NearLane R = near_lane(G, evec, T, row, T.n0 + ph);
    const double acc = G.col_pert ? (G.lean ? near_sweep<true, true>(G, cb, sbv, tl, T, ph, R)
                                            : near_sweep<true, false>(G, cb, sbv, tl, T, ph, R))
                                  : (G.lean ? near_sweep<false, true>(G, cb, sbv, tl, T, ph, R)
                                            : near_sweep<false, false>(G, cb, sbv, tl, T, ph, R));
    red[ph][row] = R.active ? acc : 0.0;
    __syncthreads();
    if (wave == 0) {
        const double v = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        if (!T.sole)
            out[lane] = v;
        else if (lane < T.nk)
            gview(P.f)[T.k0 + lane - 1] = v; // what the reduce would write: 0 + v
    }
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Several right-hand sides (nrhs <= 64): a (64 rows x columns) by
// (columns x nrhs) product on v_mfma_f64_16x16x4f64 whose A operand is J_0
// evaluated in place.  Wave w owns rows 16w..16w+15; in a step of 4 columns
// lane l evaluates J_0 for row 16w + l%16 and column l/16 -- exactly the A
// layout (lane -> row l%16, k l/16) -- so no lane needs another's J, and
// each lane sweeps its columns with stride 4 like k_near.  Per 64-column
// block a lane evaluates its 16 values (kept in its own slots of an LDS
// buffer, so that the unrolled evaluations overlap) and then feeds them to
// the MFMAs.  The coefficients of 64 columns at a time are staged in LDS as
// the B operand (lane -> k l/16, right-hand side l%16); several workgroups
// per compute unit hide the staging latency.
// the fields of a NearProb that the sweeps use, held in scalar registers
struct NearJob {
    GridArgs G;
    const double* c;
    const double* b;
    const double* e;
    int64_t ldc;
    int32_t nrhs;
};

__device__ __forceinline__ NearJob near_job(const NearProb& P) {
    NearJob J;
    J.G = P.G;
    J.c = P.c;
    J.b = P.b;
    J.e = P.e;
    J.ldc = P.ldc;
    J.nrhs = P.nrhs;
    return J;
}

constexpr int CS_LD = 80; // row stride of the coefficient tile (16 mod 32 banks)
#ifndef HANK_MULTI_UNROLL
#define HANK_MULTI_UNROLL 1
#endif

// 16 steps of 4 columns (one 64-column block) of the multi right-hand-side
// product.  With HANK_MULTI_STAGE the lane first evaluates its 16 values of J
// (steps unrolled like k_near, so that their chains overlap) into its wave's
// LDS slice Js and then feeds them to the MFMAs; otherwise each J goes
// straight into its MFMA.
#ifndef HANK_MULTI_STAGE
#define HANK_MULTI_STAGE 1
#endif
template <int M, bool SMALL, bool ASY, bool PERT, bool ROT1 = false, bool LEAN = false, int NT = J0_TAYLOR_DEG>
__device__ __forceinline__ void near_multi_block(const GridArgs& G, NearLane& R, const double (*Cs)[CS_LD],
                                                 const double* Bs, double* Js, int64_t nb, int64_t n1, int kq,
                                                 int lane, int nblk, v4d (&acc)[4], const double* tl, bool anchor) {
    constexpr bool TL = HANK_TAYLOR_LDS && SMALL && NT <= TAY_LDS_NT;
    if (ASY && anchor) near_anchor(G, R);
    const HankelSet<M> H = hankel_set<M, LEAN>();
#if HANK_MULTI_STAGE
    HANK_PRAGMA(unroll HANK_NEAR_UNROLL)
    for (int i = 0; i < 16; ++i) {
        const int col = 4 * i + kq;
        const double J =
            near_step<M, SMALL, ASY, PERT, NT, LEAN, ROT1, TL>(G, R, PERT ? Bs[col] : 0.0, H, tl);
        Js[64 * i + lane] = (R.active && nb + col < n1) ? J : 0.0;
    }
#pragma unroll 1
    for (int i = 0; i < 16; ++i) {
        const int col = 4 * i + kq;
        const double J = Js[64 * i + lane]; // written by this lane
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
            if (jb < nblk) acc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(J, Cs[col][16 * jb + (lane & 15)], acc[jb], 0, 0, 0);
    }
#else
    (void)Js;
    HANK_PRAGMA(unroll HANK_MULTI_UNROLL)
    for (int i = 0; i < 16; ++i) {
        const int col = 4 * i + kq;
        double J = near_step<M, SMALL, ASY, PERT, NT, LEAN, ROT1, TL>(G, R, PERT ? Bs[col] : 0.0, H, tl);
        J = (R.active && nb + col < n1) ? J : 0.0;
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
            if (jb < nblk) acc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(J, Cs[col][16 * jb + (lane & 15)], acc[jb], 0, 0, 0);
    }
#endif
}

template <bool PERT, bool LEAN>
__device__ __forceinline__ void near_multi_body(const NearJob& P, const NearTile& T, const uint32_t* bv,
                                                double (*Cs)[CS_LD], double* Bs, double* Js, const double* tl,
                                                double* __restrict__ out) {
    const GridArgs& G = P.G;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int nr = P.nrhs;
    const int nblk = (nr + 15) >> 4;
    const int row = 16 * wave + (lane & 15), kq = lane >> 4;
    NearLane R = near_lane(G, P.e, T, row, T.n0 + kq);
    v4d acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
    bool carried = false; // as in near_sweep
    int since = 0;
    for (int64_t nb = T.n0; nb < T.n1; nb += 64) {
        // stage: thread t carries column t%64 of right-hand sides t/64 + 4i
        {
            const int64_t n = nb + lane;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int j = (t >> 6) + 4 * i;
                Cs[lane][j] = (j < nr && n < T.n1) ? gview(P.c)[(int64_t)j * P.ldc + n - 1] : 0.0;
            }
            if (PERT && t < 64) Bs[t] = n < T.n1 ? gview(P.b)[n - 1] : 0.0;
        }
        __syncthreads();
        int var = tile_block_variant(bv, T.n0, nb);
        {
            const double b0 = PERT ? Bs[kq] : 0.0, b1 = PERT ? Bs[60 + kq] : 0.0;
            if (var == NV_MIX12 || var == NV_MIX6)
                var = near_refine_mix<PERT, false>(var, G, R, 16, b0, b1);
            else if (var == NV_MIX12_8 || var == NV_MIX6_8 || var == NV_MIX6_8R)
                var = near_refine_mix<PERT, HANK_TAYLOR_LDS != 0>(var, G, R, 16, b0, b1);
        }
        const bool anchor = !(LEAN && carried && since < HANK_NEAR_ANCHOR - 1);
        since = anchor ? 0 : since + 1;
        carried = !(var == NV_SMALL || var == NV_SMALL8);
#define BLOCK(M_, S_, A_) near_multi_block<M_, S_, A_, PERT, false, LEAN>(G, R, Cs, Bs, Js + 1024 * wave, nb, T.n1, kq, lane, nblk, acc, tl, anchor); break
#define BLOCK8(M_, A_) near_multi_block<M_, true, A_, PERT, false, LEAN, 8>(G, R, Cs, Bs, Js + 1024 * wave, nb, T.n1, kq, lane, nblk, acc, tl, anchor); break
#define BLOCKR(M_, S_, A_, NT_) near_multi_block<M_, S_, A_, PERT, PERT, LEAN, NT_>(G, R, Cs, Bs, Js + 1024 * wave, nb, T.n1, kq, lane, nblk, acc, tl, anchor); break
        switch (var) {
        case NV_M6R_WAVE: BLOCKR(6, false, true, J0_TAYLOR_DEG);
        case NV_M2R: BLOCKR(2, false, true, J0_TAYLOR_DEG);
        case NV_M3R: BLOCKR(3, false, true, J0_TAYLOR_DEG);
        case NV_M4R: BLOCKR(4, false, true, J0_TAYLOR_DEG);
        case NV_MIX6_8R: BLOCKR(6, true, true, 8);
        case NV_SMALL8: BLOCK8(3, false);
        case NV_MIX12_8: BLOCK8(12, true);
        case NV_MIX6_8: BLOCK8(6, true);
        case NV_SMALL: BLOCK(3, true, false);
        case NV_MIX12: BLOCK(12, true, true);
        case NV_MIX6: BLOCK(6, true, true);
        case NV_M2: BLOCK(2, false, true);
        case NV_M3: BLOCK(3, false, true);
        case NV_M4: BLOCK(4, false, true);
        case NV_M6: BLOCK(6, false, true);
        case NV_M8: BLOCK(8, false, true);
        default: BLOCK(12, false, true);
        }
#undef BLOCKR
#undef BLOCK8
#undef BLOCK
        near_skip16(R);
        __syncthreads();
    }
    // D (16x16): lane l, register r -> row l/16 + 4r, column l%16 (FP64 layout)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int j = 16 * jb + (lane & 15);
        if (j < nr) {
#pragma unroll
            for (int r = 0; r < 4; ++r) out[(int64_t)j * 64 + 16 * wave + (lane >> 4) + 4 * r] = acc[jb][r];
        }
    }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_near_multi(const NearProb* __restrict__ probs, int nprob,
                                                    double* __restrict__ partial) {
    __shared__ double Cs[64][CS_LD];
    __shared__ double Bs[64];
#if HANK_MULTI_STAGE
    __shared__ double Js[4 * 1024]; // per wave: J of its 16 steps x 64 lanes
#else
    double* Js = nullptr;
#endif
    __shared__ uint32_t sbv[4];
    __shared__ __align__(16) double tl[HANK_TAYLOR_LDS ? TAY_LDS_PIECES * TAY_LDS_LD : 2];
    const NearProb& Pr = probs[find_desc<NearProb, &NearProb::tile_start>(probs, nprob, blockIdx.x)];
    const NearTile T = Pr.tiles[blockIdx.x - Pr.tile_start];
    if (threadIdx.x < 4) sbv[threadIdx.x] = Pr.tiles[blockIdx.x - Pr.tile_start].bvar[threadIdx.x];
    if (HANK_TAYLOR_LDS)
        for (int i = threadIdx.x; i < TAY_LDS_PIECES * TAY_LDS_NT; i += 256) {
            const int pc = i / TAY_LDS_NT, u = i % TAY_LDS_NT;
            tl[pc * TAY_LDS_LD + u] =
                pc < J0_TAYLOR0_PIECES ? g_tab.tay0[pc][u] : g_tab.tay[pc - J0_TAYLOR0_PIECES][u];
        }
    const NearJob P = near_job(Pr); // by value: scalar registers, loaded once
    double* out = partial + Pr.pbase + T.slot * (int64_t)P.nrhs * 64;
    // (the body's first barrier orders the LDS copies above before their use)
    if (P.G.col_pert)
        P.G.lean ? near_multi_body<true, true>(P, T, sbv, Cs, Bs, Js, tl, out)
                 : near_multi_body<true, false>(P, T, sbv, Cs, Bs, Js, tl, out);
    else
        P.G.lean ? near_multi_body<false, true>(P, T, sbv, Cs, Bs, Js, tl, out)
                 : near_multi_body<false, false>(P, T, sbv, Cs, Bs, Js, tl, out);
}

// ---------------------------------------------------------------------------
// Near field of order nu > 0 (Schlomilch, Sec. 4; Fourier-Bessel, Sec. 5, whose
// z = z~ + r^_k b_n carries the root offset b_n): J_nu at each entry from the
// plan's table (tables.h).  Below z = 20 + nu/2 the series (z < 2) or the
// Taylor pieces, with z carried as hi + lo so that the offset from the
// piece's centre is exact; above it mnu Hankel pairs.  The Hankel phase
// z - (2nu+1)pi/4 = pi (i_n/D - (2nu+1)/4), i_n = K N_n mod 2D, grows by the
// same angle pi step/D at each of the wave's columns: the lane keeps
// u = e^{i phase}, advances it by one complex rotation and recomputes it from
// the exact integer i_n every 16 columns.  Same tiles, partial slots and
// reduction as k_near.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double jnu_small(const double* __restrict__ tab, int nu, double hi, double lo) {
    const double z = hi + lo;
    if (z < J0_TAYLOR_Z0) {
        const double h = 0.5 * z, w = h * h;
        double p = tab[NU_TAB_SER + NU_SERIES_TERMS - 1];
        for (int t = NU_SERIES_TERMS - 2; t >= 0; --t) p = fma(p, w, tab[NU_TAB_SER + t]);
        for (int i = 0; i < nu; ++i) p *= h;
        return p;
    }
    int i = (int)((z - J0_TAYLOR_Z0) * (1.0 / J0_TAYLOR_H));
    i = i < 0 ? 0 : (i >= NU_TAYLOR_INTERVALS ? NU_TAYLOR_INTERVALS - 1 : i);
    const double dz = (hi - (J0_TAYLOR_Z0 + (i + 0.5) * J0_TAYLOR_H)) + lo;
    const double* t = tab + NU_TAB_TAY + J0_TAYLOR_DEG * i;
    double p = t[J0_TAYLOR_DEG - 1];
#pragma unroll
    for (int u = J0_TAYLOR_DEG - 2; u >= 0; --u) p = fma(p, dz, t[u]);
    return p;
}

__global__ __launch_bounds__(256) void k_near_nu(const NearProb* __restrict__ probs, int nprob,
                                                 double* __restrict__ partial) {
    __shared__ double cs[NEAR_TILE_COLS], bs[NEAR_TILE_COLS];
    __shared__ double red[4][64];
    const NearProb& P = probs[find_desc<NearProb, &NearProb::tile_start>(probs, nprob, blockIdx.x)];
    const NearTile T = P.tiles[blockIdx.x - P.tile_start];
    double* out = partial + P.pbase + T.slot * 64;
    const GridArgs G = P.G;
    const double* tab = P.nutab;
    const int nu = P.nu, mnu = P.mnu;
    const bool pert = G.col_pert != 0;
    const int ncol = (int)(T.n1 - T.n0);
    for (int i = threadIdx.x; i < ncol; i += 256) {
        cs[i] = gview(P.c)[T.n0 - 1 + i];
        bs[i] = pert ? gview(P.b)[T.n0 - 1 + i] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool active = lane < T.nk;
    const int64_t k = T.k0 + (active ? lane : 0);
    const int64_t K = G.ar * k + G.br;
    const double rk = (double)K / (double)G.Dr; // r^_k
    const int64_t D2 = 2 * G.D;
    int64_t n = T.n0 + wave;
    int64_t Nn = G.ac * n + G.bc;
    int64_t ir = (K * Nn) % D2;
    const int64_t step = (K * 4 * G.ac) % D2, step16 = (16 * step) % D2;
    const double zsw = 20.0 + 0.5 * nu, ph0 = -0.25 * (2 * nu + 1);
    double hp[NU_HANKEL_PAIRS], hq[NU_HANKEL_PAIRS]; // wave-uniform: held in scalar registers
#pragma unroll
    for (int m = 0; m < NU_HANKEL_PAIRS; ++m) {
        hp[m] = tab[NU_TAB_P + m];
        hq[m] = tab[NU_TAB_Q + m];
    }
    double ws, wc;
    sincospi_ratio(step, G.D, &ws, &wc); // e^{i pi step / D}
    double acc = 0.0;
    while (n < T.n1) {
        // anchor: u = e^{i pi (i_n/D - (2nu+1)/4)} from the exact integer i_n
        double us, uc;
        sincospi(fma((double)ir, G.invD, ph0), &us, &uc);
        const int64_t nend = min(T.n1, n + 64);
        for (; n < nend; n += 4) {
            const double I = (double)K * (double)Nn; // exact: K N_n < 2^53
            const double hi = I * G.piD_hi;
            const double delta = rk * bs[n - T.n0]; // z - z~ (0 without root offsets)
            const double lo = (fma(I, G.piD_hi, -hi) + I * G.piD_lo) + delta;
            double J;
            if (hi + lo < zsw) {
                J = jnu_small(tab, nu, hi, lo);
            } else {
                const double z = hi + lo;
                double y = __builtin_amdgcn_rsq(z);
                const double h = 0.5 * z;
                y = y * fma(-h * y, y, 1.5);
                y = y * fma(-h * y, y, 1.5);
                const double zi = y * y, zi2 = zi * zi;
                double Pv = 0.0, Qv = 0.0;
#pragma unroll
                for (int m = NU_HANKEL_PAIRS - 1; m >= 0; --m) {
                    if (m < mnu) { // uniform: the plan's pair count
                        Pv = fma(Pv, zi2, hp[m]);
                        Qv = fma(Qv, zi2, hq[m]);
                    }
                }
                double cph = uc, sph = us;
                if (pert) { // the phase of z~ carried by u, plus delta
                    double sd, cd;
                    sincos_small(delta, &sd, &cd);
                    cph = fma(uc, cd, -us * sd);
                    sph = fma(us, cd, uc * sd);
                }
                J = (0.79788456080286535588 * y) * fma(cph, Pv, -sph * (Qv * zi)); // sqrt(2/pi)
            }
            acc = fma(cs[n - T.n0], J, acc);
            const double t = uc * ws;
            uc = fma(uc, wc, -us * ws);
            us = fma(us, wc, t);
            Nn += 4 * G.ac;
        }
        ir += step16;
        if (ir >= D2) ir -= D2;
    }
    red[wave][lane] = active ? acc : 0.0;
    __syncthreads();
    if (wave == 0) out[lane] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Row tiles of the single-right-hand-side problems (the first ones, row
// tiles [0, nrt1)), wpr waves each from wave wv_start of the problem on:
// wave sub of a row tile sums its tiles sub, sub + wpr, ... and with wpr = 4
// the four sums (one workgroup) are added in wave order.  Waves past a
// problem's last row tile (alignment padding) and past nwv write nothing.
__global__ __launch_bounds__(256) void k_near_reduce1(const NearProb* __restrict__ probs, int nprob, int64_t nwv,
                                                      int64_t nrt1, const double* __restrict__ partial) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t gw = (int64_t)blockIdx.x * 4 + wave;
    const int pi = find_desc<NearProb, &NearProb::wv_start>(probs, nprob, gw < nwv ? gw : 0);
    const NearProb& P = probs[pi];
    const int wpr = P.wpr;
    const int64_t local = gw - P.wv_start, rt_end = pi + 1 < nprob ? probs[pi + 1].rt_start : nrt1;
    const int64_t rt = P.rt_start + local / wpr;
    const int sub = (int)(local % wpr);
    const bool valid = gw < nwv && rt < rt_end;
    // wpr = 4 problems start at a multiple of 4 waves, so `four' is the same
    // for every wave of a workgroup
    const bool four = valid && wpr == 4;
    double s = 0.0;
    RowTile R{};
    if (valid) {
        R = P.rts[rt - P.rt_start];
        const double* q = partial + P.pbase + R.slot0 * 64 + lane;
        // four tiles per step, loads unconditional (clamped to the last tile)
        // so that they are in flight together; the sum stays in tile order
        const int64_t last = R.ntiles - 1;
        for (int64_t t = sub; t <= last; t += 4 * wpr) {
            double v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = q[min(t + i * wpr, last) * 64];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (t + i * wpr <= last) s += v[i];
        }
    }
    if (four) {
        red[wave][lane] = s;
        __syncthreads();
        if (wave == 0 && lane < R.nk)
            gview(P.f)[R.k0 + lane - 1] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    } else if (valid && lane < R.nk) {
        gview(P.f)[R.k0 + lane - 1] = s;
    }
}

// A row tile's sums for nrhs > 1: its partials are E = nrhs x 64 contiguous
// values per tile (right-hand side j, lane l at j*64 + l); thread i sums
// elements i, i + 256, ... (PER of them, PER*256 >= E) over the tiles in
// tile order.  The loads of one tile are unconditional (indices past E read
// element E-1, and those sums are dropped), so they are all in flight at once.
template <int PER>
__device__ __forceinline__ void near_reduce_multi(const NearProb& P, const RowTile& R, const double* __restrict__ base,
                                                  int E) {
    double s[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) s[i] = 0.0;
    for (int64_t t = 0; t < R.ntiles; ++t) {
        const double* q = base + t * E;
        double v[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) v[i] = q[min((int)threadIdx.x + 256 * i, E - 1)];
#pragma unroll
        for (int i = 0; i < PER; ++i) s[i] += v[i];
        // issue every load of the tile before the first add
        __builtin_amdgcn_sched_group_barrier(0x020, PER, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, PER, 0);
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = (int)threadIdx.x + 256 * i, l = e & 63;
        if (e < E && l < R.nk) gview(P.f)[(int64_t)(e >> 6) * P.ldo + R.k0 + l - 1] = s[i];
    }
}

// One workgroup per row tile of a problem with several right-hand sides (row
// tiles from rt0 on); up to 128 registers, so that 16 loads per thread fit
// in flight.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_near_reduce(const NearProb* __restrict__ probs, int nprob, int64_t rt0,
                                                     const double* __restrict__ partial) {
    const int64_t rt = rt0 + blockIdx.x;
    const NearProb& P = probs[find_desc<NearProb, &NearProb::rt_start>(probs, nprob, rt)];
    const RowTile R = P.rts[rt - P.rt_start];
    const int E = P.nrhs * 64; // nrhs <= 64
    const double* base = partial + P.pbase + R.slot0 * E;
    const int per = (E + 255) >> 8;
    if (per <= 1)
        near_reduce_multi<1>(P, R, base, E);
    else if (per <= 2)
        near_reduce_multi<2>(P, R, base, E);
    else if (per <= 4)
        near_reduce_multi<4>(P, R, base, E);
    else if (per <= 8)
        near_reduce_multi<8>(P, R, base, E);
    else
        near_reduce_multi<16>(P, R, base, E);
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

// LDS elements per column FFT buffer of the column passes: L2 + L2/8 made
// odd, so that the W columns of a workgroup start in different banks
template <int L2>
constexpr int col_stride() {
    return (L2 + L2 / 8) | 1;
}

// (descriptor, workgroup within its item, right-hand side, group chunk) of
// this workgroup.  which: 0 column passes (per workgroups per item), 1 pass B
// (per workgroups per item), 2 chunk reduction (ceil(nrows/256) per
// right-hand side).
struct FarItem {
    int desc, wg, j, chunk;
};

// split: pass B workgroups carry the descriptor's bsplit (k_pass_bw)
__device__ __forceinline__ FarItem far_item(const FarDesc* __restrict__ descs, int ndesc, int which, int per,
                                            bool split = false) {
    const int64_t bid = blockIdx.x;
    FarItem it;
    int64_t local;
    if (which == 0) {
        it.desc = find_desc<FarDesc, &FarDesc::wg_ac>(descs, ndesc, bid);
        local = bid - descs[it.desc].wg_ac;
    } else if (which == 1) {
        it.desc = find_desc<FarDesc, &FarDesc::wg_b>(descs, ndesc, bid);
        local = bid - descs[it.desc].wg_b;
        if (split) per *= max(1, descs[it.desc].bsplit);
    } else {
        it.desc = find_desc<FarDesc, &FarDesc::wg_r>(descs, ndesc, bid);
        local = bid - descs[it.desc].wg_r;
        per = (int)((descs[it.desc].A.nrows + 255) / 256);
    }
    const int item = (int)(local / per);
    it.wg = (int)(local % per);
    const int nch = which == 2 ? 1 : descs[it.desc].nchunk;
    it.j = item / nch;
    it.chunk = item % nch;
    return it;
}

// Pass A on a block's data: y_n' = q(n') c_n X_g(n), column FFTs over j2, for
// every right-hand side and group of the descriptor.  Per column position the
// group-independent factors are kept:
//   qb = q(n') (w^_n/w0)^(-1/2),  vw = w^_n/w0,  x = (b_n/bref)/vw,  la = lambda_n/lref
// and X_g = la^a vw^e sum_b K_{g,b} x^b, with vw^e updated incrementally over
// the groups (sorted by a, then e).
template <typename F, int L2, int W>
__global__ __launch_bounds__(W * L2 / 8) void k_pass_a(const FarDesc* __restrict__ descs, int ndesc) {
    constexpr int R = 8, NTC = L2 / R;
    __shared__ cx<F> sh[W * col_stride<L2>()];
    const FarItem mp = far_item(descs, ndesc, 0, descs[0].A.L1 / W);
    const FarDesc& D = descs[mp.desc];
    const FarArgs& A = D.A;
    const int t = threadIdx.x, w = t % W, tt = t / W;
    const int64_t j1 = (int64_t)mp.wg * W + w;
    if ((int64_t)mp.wg * W >= A.ncols) return; // columns past the block: zero input, not stored
    cx<F>* my = sh + w * col_stride<L2>();
    const int ng = A.g1 - A.g0;
    const auto buf = gview((cx<F>*)D.buf);

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
            const double bn = A.col_pert ? gview(D.b)[n - 1] : 0.0;
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
        const auto cj = gview(D.c) + (int64_t)j * D.ldc;
        double cv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) cv[r] = nidx[r] >= 0 ? cj[nidx[r]] : 0.0;
        // four-step twiddles e^{-2 pi i j1 m2 / L}, m2 = tt + r NTC, shared by
        // every group: w_r = w(j1 tt) w(j1 NTC)^r from two table entries
        const cx<double> tw0 = tw_big<double>(j1 * tt, A.twshift);
        const cx<double> tws = tw_big<double>(j1 * NTC, A.twshift);
        int ecur = 0, acur = 0;
        for (int g = gs; g < ge; ++g) {
            const GroupDev Gd = scalar_entry(A.groups, g);
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
                        const TermDev Td = scalar_entry(A.terms, ti);
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
            const auto out = buf + ((int64_t)j * ng + (g - A.g0)) * A.L;
            cx<double> tw = tw0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t m2 = tt + r * NTC;
                gstore(out + m2 * A.L1 + j1, cmul(v[r], mk(F(tw.x), F(tw.y))));
                if (r + 1 < R) tw = cmul(tw, tws);
            }
        }
    }
}

// Pass A on the chirp kernel h(m) = e^{-i pi ar ac m^2 / (2D)}, m = k' - n',
// laid out for a circular convolution of length L (first FFT step of H^).
template <typename F, int L2, int W>
__global__ __launch_bounds__(W * L2 / 8) void k_pass_a_kernel(FarArgs A, cx<F>* __restrict__ buf) {
    constexpr int R = 8, NTC = L2 / R;
    __shared__ cx<F> sh[W * col_stride<L2>()];
    const int t = threadIdx.x, w = t % W, tt = t / W;
    const int64_t j1 = (int64_t)blockIdx.x * W + w;
    cx<F>* my = sh + w * col_stride<L2>();
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
// Pass B: H^ and the inverse twiddles of the row are loaded once and held in
// registers across the groups.  (A variant that re-read them per group for the
// FP64 rows of 8192 points, to avoid spilling under the 128-register cap of
// 1024 threads, measured no faster and gave run-to-run differences in a few
// output columns; it was removed.)
template <typename F, int L1, int ROWS>
__global__ __launch_bounds__(ROWS * L1 / 8) void k_pass_b(const FarDesc* __restrict__ descs, int ndesc,
                                                           int per_b) {
    constexpr int R = 8, NTR = L1 / R;
    __shared__ cx<F> sh[ROWS * (L1 + L1 / 8)];
    const FarItem mp = far_item(descs, ndesc, 1, per_b);
    const FarDesc& D = descs[mp.desc];
    const FarArgs& A = D.A;
    const int t = threadIdx.x, rl = t / NTR, tt = t % NTR;
    const int64_t row = (int64_t)mp.wg * ROWS + rl;
    const bool okrow = row < A.L2;
    const int64_t rowc = okrow ? row : 0;
    cx<F>* my = sh + rl * (L1 + L1 / 8);
    const auto hrow = gview((const cx<F>*)D.H) + rowc * L1;
    const auto buf = gview((cx<F>*)D.buf);
    cx<F> hv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) hv[r] = gload(hrow + tt + r * NTR);
    // inverse four-step twiddles e^{+2 pi i j1 m2 / L}, j1 = tt + r NTR, formed
    // per group as t0 ts^r from two table entries (holding all eight across the
    // groups would cost 32 more registers)
    cx<double> t0 = tw_big<double>((int64_t)tt * rowc, A.twshift);
    cx<double> ts = tw_big<double>((int64_t)NTR * rowc, A.twshift);
    t0.y = -t0.y;
    ts.y = -ts.y;
    const int ng = A.g1 - A.g0;
    const int gs = mp.chunk * D.gchunk, ge = min(ng, gs + D.gchunk);
    for (int gq = gs; gq < ge; ++gq) {
        const int64_t q = (int64_t)mp.j * ng + gq;
        const auto p = buf + q * A.L + rowc * L1;
        cx<F> v[R];
        // columns j1 >= ncols hold zeros (pass A does not store them), and
        // columns j1 >= nrows feed no output row (pass C skips them)
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = tt + r * NTR < A.ncols ? gload(p + tt + r * NTR) : mk(F(0), F(0));
        fft_reg<F, L1, R, -1>(v, my, tt);
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = cmul(v[r], hv[r]);
        fft_reg<F, L1, R, 1>(v, my, tt);
        if (okrow) {
            cx<double> t = t0;
            asm volatile("" : "+v"(t.x), "+v"(t.y)); // formed here, not hoisted out of the group loop
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (tt + r * NTR < A.nrows) gstore(p + tt + r * NTR, cmul(v[r], mk(F(t.x), F(t.y))));
                if (r + 1 < R) t = cmul(t, ts);
            }
        }
    }
}

// Pass C: inverse column FFTs, then f_k += sum_g A_g(k) Re(p(k') conv_g(k')),
// A_g(k) = scale_g (e_k/eref)^a (r^_k/r0)^(e - 1/2), per right-hand side, with
// the power of r^_k/r0 updated incrementally over the groups.
template <typename F, int L2, int W>
__global__ __launch_bounds__(W * L2 / 8) void k_pass_c(const FarDesc* __restrict__ descs, int ndesc) {
    constexpr int R = 8, NTC = L2 / R;
    __shared__ cx<F> sh[W * col_stride<L2>()];
    const FarItem mp = far_item(descs, ndesc, 0, descs[0].A.L1 / W);
    const FarDesc& D = descs[mp.desc];
    const FarArgs& A = D.A;
    const int t = threadIdx.x, w = t % W, tt = t / W;
    const int64_t j1 = (int64_t)mp.wg * W + w;
    if ((int64_t)mp.wg * W >= A.nrows) return; // columns holding no output row
    cx<F>* my = sh + w * col_stride<L2>();
    const int ng = A.g1 - A.g0;
    const auto buf = gview((const cx<F>*)D.buf);
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
            ek[r] = A.row_pert ? gview(D.e)[k - 1] / A.eref : 0.0;
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
            const GroupDev Gd = scalar_entry(A.groups, g);
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
            const auto p = buf + ((int64_t)j * ng + (g - A.g0)) * A.L;
            cx<F> v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = gload(p + (int64_t)(tt + r * NTC) * A.L1 + j1);
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
            const auto fj = gview(D.f) + (int64_t)j * D.ldo;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t kp = j1 + (int64_t)A.L1 * (tt + r * NTC);
                if (kp < A.nrows) fj[A.ka + kp - 1] += acc[r];
            }
        } else {
            const auto pj = gview(D.part) + ((int64_t)j * D.nchunk + mp.chunk) * A.nrows;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t kp = j1 + (int64_t)A.L1 * (tt + r * NTC);
                if (kp < A.nrows) pj[kp] = acc[r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Column passes with one wave per column (L2 = 64 R points, W = 8 columns per
// workgroup of 8 waves).  The column FFT is wave-local: its stages exchange
// through the wave's own LDS region without a workgroup barrier.  The data
// cross between the coalesced global layout (thread t: column t % 8, rows
// t/8 + 64 r, so a wave instruction covers 8 rows x 128 bytes) and the
// wave-per-column layout through an LDS transposition; with two LDS buffers
// (L2 <= 256) one workgroup barrier per group suffices, with one buffer two.
// ---------------------------------------------------------------------------
// two workgroups per compute unit (at most 128 registers) for columns of 256
// points; one for 512 (eight points per lane)
#ifndef HANK_WAVE_COLS_WPE
#define HANK_WAVE_COLS_WPE __attribute__((amdgpu_waves_per_eu(L2 <= 256 ? 4 : 2)))
#endif
// LDS elements per column of the wave-per-column kernels (slots lds_swz):
// L2 + 2, so that the eight columns a wave instruction touches in the
// transposition (two rows each) fall into distinct groups of four banks
template <int L2>
constexpr int wave_col_stride() {
    return HANK_LDS_SWZ ? L2 + 2 : (L2 + L2 / 8) | 1;
}
// LDS buffers (groups alternate between them: one workgroup barrier per
// group with two, two with one).  At 512 points a workgroup already holds a
// compute unit by its registers, so its two buffers (148 KB) cost nothing.
#ifndef HANK_WAVE_COLS_BUFS512
#define HANK_WAVE_COLS_BUFS512 2
#endif
template <int L2>
constexpr int wave_col_bufs() {
    return L2 <= 256 ? 2 : HANK_WAVE_COLS_BUFS512;
}

// Pass A for a block of at most L1 columns: only row 0 (n' = j1) of each
// column input can be nonzero, so the column DFT is that value at every m2
// and the output is it times the four-step twiddle e^{-2 pi i j1 m2 / L}: no
// FFT and no LDS.  Thread t writes column jb + t % 8, rows t/8 + 64 r, as the
// transposed stores of the general path do.
template <typename F, int L2>
__device__ __forceinline__ void pass_aw_row0(const FarDesc& D, const FarItem& mp, int64_t jb) {
    constexpr int W = 8, R = L2 / 64;
    const FarArgs& A = D.A;
    const int t = threadIdx.x, cw = t % W, q = t / W;
    const int64_t j1 = jb + cw;
    const int ng = A.g1 - A.g0;
    const auto buf = gview((cx<F>*)D.buf);
    const auto x0 = gview((cx<F>*)D.x0); // (null: the full columns)
    const int j = mp.j;
    double vw = 1.0, xb = 0.0, la = 0.0;
    cx<double> qb = mk(0.0, 0.0);
    if (j1 < A.ncols) {
        const int64_t n = A.na + j1;
        const int64_t Nn = A.ac * n + A.bc;
        const double wn = (double)Nn * A.pi_Qc;
        const double bn = A.col_pert ? gview(D.b)[n - 1] : 0.0;
        vw = wn / A.w0;
        const double iw = 1.0 / vw;
        xb = (bn / A.bref) * iw;
        la = (wn + bn) / A.lref;
        qb = cscale(expi_ratio(2 * A.Kka * A.ac * j1 + A.ar * A.ac * j1 * j1, 2 * A.D),
                    sqrt(iw) * gview(D.c)[(int64_t)j * D.ldc + n - 1]);
    }
    cx<F> tw[R];
    if (!x0) {
        cx<double> w = tw_big<double>(j1 * q, A.twshift);
        const cx<double> ws = tw_big<double>(j1 * 64, A.twshift);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            tw[r] = mk(F(w.x), F(w.y));
            if (r + 1 < R) w = cmul(w, ws);
        }
    }
    const int gs = A.g0 + mp.chunk * D.gchunk, ge = min(A.g1, gs + D.gchunk);
    int ecur = 0, acur = 0;
    double pw = 1.0;
    for (int g = gs; g < ge; ++g) {
        const GroupDev Gd = scalar_entry(A.groups, g);
        if (Gd.a != acur || g == gs) {
            pw = ipow_d<double>(vw, Gd.e) * (Gd.a ? ipow_d<double>(la, Gd.a) : 1.0);
        } else {
            for (; ecur < Gd.e; ++ecur) pw *= vw;
            for (; ecur > Gd.e; --ecur) pw /= vw;
        }
        ecur = Gd.e;
        acur = Gd.a;
        double xp = 1.0, Xr = 0.0, Xi = 0.0;
        int bcur = 0;
        for (int ti = Gd.t0; ti < Gd.t1; ++ti) {
            const TermDev Td = scalar_entry(A.terms, ti);
            while (bcur < Td.b) {
                xp *= xb;
                ++bcur;
            }
            Xr = fma(Td.kre, xp, Xr);
            Xi = fma(Td.kim, xp, Xi);
        }
        const cx<double> y = cmul(mk(Xr * pw, Xi * pw), qb);
        const cx<F> yf = mk(F(y.x), F(y.y));
        if (x0) { // pass B forms the rows from this value
            if (q == 0 && j1 < A.ncols) gstore(x0 + ((int64_t)j * ng + (g - A.g0)) * A.ncols + j1, yf);
            continue;
        }
        const auto out = buf + ((int64_t)j * ng + (g - A.g0)) * A.L + jb + cw;
#pragma unroll
        for (int r = 0; r < R; ++r) gstore(out + (int64_t)(q + 64 * r) * A.L1, cmul(yf, tw[r]));
    }
}

// Pass A: the inputs of the lane's positions n' = j1 + L1 (lane + 64 r) of the
// wave's column j1 for every group (as k_pass_a), the column FFT, the
// four-step twiddle, and through LDS to buf[m2][j1].
// HALF: every position n' >= jb + L/2 is past the block's columns, so the
// lane's registers r >= R/2 hold zeros (not formed; the FFT's first stage
// knows them).
template <typename F, int L2, bool HALF>
__device__ __forceinline__ void pass_aw_main(const FarDesc& D, const FarItem& mp, int64_t jb,
                                             cx<F> (*sh)[8 * wave_col_stride<L2>()]) {
    constexpr int W = 8, R = L2 / 64, S = wave_col_stride<L2>(), NB = wave_col_bufs<L2>();
    constexpr int RH = HALF ? R / 2 : R; // registers that can be nonzero
    const FarArgs& A = D.A;
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int cw = t % W, q = t / W;
    const int64_t j1 = jb + wv;
    const int ng = A.g1 - A.g0;
    const auto buf = gview((cx<F>*)D.buf);

    double vw[RH], xb[RH], la[RH], pw[RH];
    cx<double> qb[RH]; // q(n') c_n (w^_n/w0)^(-1/2); zero past the block's columns
    const int j = mp.j;
    const auto cj = gview(D.c) + (int64_t)j * D.ldc;
#pragma unroll
    for (int r = 0; r < RH; ++r) {
        const int64_t np = j1 + (int64_t)A.L1 * (lane + 64 * r);
        vw[r] = 1.0;
        xb[r] = la[r] = 0.0;
        qb[r] = mk(0.0, 0.0);
        if (np < A.ncols) {
            const int64_t n = A.na + np;
            const int64_t Nn = A.ac * n + A.bc;
            const double wn = (double)Nn * A.pi_Qc;
            const double bn = A.col_pert ? gview(D.b)[n - 1] : 0.0;
            vw[r] = wn / A.w0;
            const double iw = 1.0 / vw[r];
            xb[r] = (bn / A.bref) * iw;
            la[r] = (wn + bn) / A.lref;
            qb[r] = cscale(expi_ratio(2 * A.Kka * A.ac * np + A.ar * A.ac * np * np, 2 * A.D), sqrt(iw) * cj[n - 1]);
        }
    }
    // four-step twiddles e^{-2 pi i j1 m2 / L} of the outputs m2 = lane + 64 r
    const cx<double> tw0 = tw_big<double>(j1 * lane, A.twshift);
    const cx<double> tws = tw_big<double>(j1 * 64, A.twshift);
    const int gs = A.g0 + mp.chunk * D.gchunk, ge = min(A.g1, gs + D.gchunk);
    int ecur = 0, acur = 0, b = 0;
    for (int g = gs; g < ge; ++g) {
        const GroupDev Gd = scalar_entry(A.groups, g);
        if (Gd.a != acur || g == gs) {
#pragma unroll
            for (int r = 0; r < RH; ++r)
                pw[r] = ipow_d<double>(vw[r], Gd.e) * (Gd.a ? ipow_d<double>(la[r], Gd.a) : 1.0);
        } else {
            for (; ecur < Gd.e; ++ecur) {
#pragma unroll
                for (int r = 0; r < RH; ++r) pw[r] *= vw[r];
            }
            for (; ecur > Gd.e; --ecur) {
#pragma unroll
                for (int r = 0; r < RH; ++r) pw[r] /= vw[r];
            }
        }
        ecur = Gd.e;
        acur = Gd.a;
        cx<F> v[R];
#pragma unroll
        for (int r = RH; r < R; ++r) v[r] = mk(F(0), F(0));
#pragma unroll
        for (int r = 0; r < RH; ++r) {
            double xp = 1.0, Xr = 0.0, Xi = 0.0;
            int bcur = 0;
            for (int ti = Gd.t0; ti < Gd.t1; ++ti) {
                const TermDev Td = scalar_entry(A.terms, ti);
                while (bcur < Td.b) {
                    xp *= xb[r];
                    ++bcur;
                }
                Xr = fma(Td.kre, xp, Xr);
                Xi = fma(Td.kim, xp, Xi);
            }
            const cx<double> y = cmul(mk(Xr * pw[r], Xi * pw[r]), qb[r]);
            v[r] = mk(F(y.x), F(y.y));
        }
        cx<F>* my = &sh[b][wv * S];
        fft_reg<F, L2, R, -1, true, HALF>(v, my, lane);
        cx<double> tw = tw0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            my[lds_swz(lane + 64 * r)] = cmul(v[r], mk(F(tw.x), F(tw.y)));
            if (r + 1 < R) tw = cmul(tw, tws);
        }
        __syncthreads();
        const auto out = buf + ((int64_t)j * ng + (g - A.g0)) * A.L;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int m2 = q + 64 * r;
            gstore(out + (int64_t)m2 * A.L1 + jb + cw, sh[b][cw * S + lds_swz(m2)]);
        }
        if constexpr (NB == 1)
            __syncthreads();
        else
            b ^= 1;
    }
}

template <typename F, int L2>
__global__ __launch_bounds__(512) HANK_WAVE_COLS_WPE void k_pass_aw(const FarDesc* __restrict__ descs, int ndesc) {
    constexpr int W = 8, S = wave_col_stride<L2>(), NB = wave_col_bufs<L2>();
    __shared__ cx<F> sh[NB][W * S];
    const FarItem mp = far_item(descs, ndesc, 0, descs[0].A.L1 / W);
    const FarDesc& D = descs[mp.desc];
    const FarArgs& A = D.A;
    const int64_t jb = (int64_t)mp.wg * W;
    if (jb >= A.ncols) return; // columns past the block: zero input, not stored
    // (uniform per workgroup)
    if (A.ncols <= A.L1)
        pass_aw_row0<F, L2>(D, mp, jb); // one input row
    else if (A.ncols <= jb + A.L / 2)
        pass_aw_main<F, L2, true>(D, mp, jb, sh);
    else
        pass_aw_main<F, L2, false>(D, mp, jb, sh);
}

// Pass C for a block of at most L1 rows: only row 0 (k' = j1) of each column
// is an output, and row 0 of the inverse column DFT is the plain sum of the
// column.  Thread t (column jb + t % 8, rows t/8 + 64 r) adds its values of
// every group with the group's weight at k' = j1; the 64 threads of a column
// are then summed in a fixed order, the 8 of each wave by lane shuffles and
// the 8 waves through LDS (red: 64 complex values).
template <typename F, int L2>
__device__ __forceinline__ void pass_cw_row0(const FarDesc& D, const FarItem& mp, int64_t jb, cx<double>* red) {
    constexpr int W = 8, R = L2 / 64;
    const FarArgs& A = D.A;
    const int t = threadIdx.x, cw = t % W, q = t / W;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t kp = jb + cw;
    const bool valid = kp < A.nrows;
    const int ng = A.g1 - A.g0;
    const auto buf = gview((const cx<F>*)D.buf);
    const int j = mp.j;
    double rho = 1.0, ek = 0.0;
    if (valid) {
        const int64_t k = A.ka + kp;
        rho = ((double)(A.ar * k + A.br) / (double)A.Dr) / A.r0;
        ek = A.row_pert ? gview(D.e)[k - 1] / A.eref : 0.0;
    }
    const int gs = A.g0 + mp.chunk * D.gchunk, ge = min(A.g1, gs + D.gchunk);
    int ecur = 0, acur = 0;
    double pw = 1.0;
    cx<double> acc = mk(0.0, 0.0);
    for (int g = gs; g < ge; ++g) {
        const GroupDev Gd = scalar_entry(A.groups, g);
        if (Gd.a != acur || g == gs) {
            pw = ipow_d<double>(rho, Gd.e) * (Gd.a ? ipow_d<double>(ek, Gd.a) : 1.0);
        } else {
            for (; ecur < Gd.e; ++ecur) pw *= rho;
            for (; ecur > Gd.e; --ecur) pw /= rho;
        }
        ecur = Gd.e;
        acur = Gd.a;
        if (valid) {
            const auto p = buf + ((int64_t)j * ng + (g - A.g0)) * A.L + jb + cw;
            double sx = 0.0, sy = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const cx<F> v = gload(p + (int64_t)(q + 64 * r) * A.L1);
                sx += (double)v.x;
                sy += (double)v.y;
            }
            const double wgt = Gd.scale * pw;
            acc.x = fma(wgt, sx, acc.x);
            acc.y = fma(wgt, sy, acc.y);
        }
    }
    // lanes cw + 8 i of a wave hold column cw: add over i (lane bits 3-5)
#pragma unroll
    for (int m = 8; m < 64; m <<= 1) {
        acc.x += __shfl_xor(acc.x, m);
        acc.y += __shfl_xor(acc.y, m);
    }
    if ((t & 63) < W) red[wv * W + cw] = acc;
    __syncthreads();
    if (t < W && valid) {
        cx<double> tot = red[cw];
#pragma unroll
        for (int w = 1; w < 8; ++w) tot = tot + red[w * W + cw];
        const cx<double> pk = cscale(
            expi_ratio(2 * A.Kka * A.Nna + 2 * A.ar * A.Nna * kp + A.ar * A.ac * kp * kp, 2 * A.D), 1.0 / sqrt(rho));
        const double val = pk.x * tot.x - pk.y * tot.y;
        if (D.nchunk == 1)
            gview(D.f)[(int64_t)j * D.ldo + A.ka - 1 + kp] += val;
        else
            gview(D.part)[((int64_t)j * D.nchunk + mp.chunk) * A.nrows + kp] = val;
    }
}

// Pass C: buf[m2][j1] through LDS to the wave of column j1, the inverse column
// FFT, and per output position k' = j1 + L1 (lane + 64 r) the complex sum
// acc = sum_g A_g(k) conv_g(k') over the groups (A_g real, so that the post-
// chirp p(k') is applied once at the end: f_k += Re(p(k') acc)).  The next
// group's data are loaded while the current one is transformed.
// HALF: every output position k' >= jb + L/2 is past the block's rows, so
// the lane's registers r >= R/2 are not used (nor, after the FFT, formed).
template <typename F, int L2, bool HALF>
__device__ __forceinline__ void pass_cw_main(const FarDesc& D, const FarItem& mp, int64_t jb,
                                             cx<F> (*sh)[8 * wave_col_stride<L2>()]) {
    constexpr int W = 8, R = L2 / 64, S = wave_col_stride<L2>(), NB = wave_col_bufs<L2>();
    constexpr int RH = HALF ? R / 2 : R; // registers holding output rows
    const FarArgs& A = D.A;
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int cw = t % W, q = t / W;
    const int64_t j1 = jb + wv;
    const int ng = A.g1 - A.g0;
    const auto buf = gview((const cx<F>*)D.buf);
    double rho[RH], ek[RH], pw[RH];
    cx<double> acc[RH];
#pragma unroll
    for (int r = 0; r < RH; ++r) {
        const int64_t kp = j1 + (int64_t)A.L1 * (lane + 64 * r);
        rho[r] = 1.0;
        ek[r] = 0.0;
        acc[r] = mk(0.0, 0.0);
        if (kp < A.nrows) {
            const int64_t k = A.ka + kp;
            rho[r] = ((double)(A.ar * k + A.br) / (double)A.Dr) / A.r0;
            ek[r] = A.row_pert ? gview(D.e)[k - 1] / A.eref : 0.0;
        }
    }
    const int j = mp.j;
    const int gs = A.g0 + mp.chunk * D.gchunk, ge = min(A.g1, gs + D.gchunk);
    auto load = [&](int g, cx<F>(&v)[R]) {
        const auto p = buf + ((int64_t)j * ng + (g - A.g0)) * A.L + jb + cw;
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = gload(p + (int64_t)(q + 64 * r) * A.L1);
    };
    cx<F> vn[R];
    load(gs, vn);
    int ecur = 0, acur = 0, b = 0;
    for (int g = gs; g < ge; ++g) {
        cx<F> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            v[r] = vn[r];
            sh[b][cw * S + lds_swz(q + 64 * r)] = v[r];
        }
        if (g + 1 < ge) load(g + 1, vn);
        __syncthreads();
        cx<F>* my = &sh[b][wv * S];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = my[lds_swz(lane + 64 * r)];
        wave_sync();
        fft_reg<F, L2, R, 1, true>(v, my, lane);
        const GroupDev Gd = scalar_entry(A.groups, g);
        if (Gd.a != acur || g == gs) {
#pragma unroll
            for (int r = 0; r < RH; ++r)
                pw[r] = ipow_d<double>(rho[r], Gd.e) * (Gd.a ? ipow_d<double>(ek[r], Gd.a) : 1.0);
        } else {
            for (; ecur < Gd.e; ++ecur) {
#pragma unroll
                for (int r = 0; r < RH; ++r) pw[r] *= rho[r];
            }
            for (; ecur > Gd.e; --ecur) {
#pragma unroll
                for (int r = 0; r < RH; ++r) pw[r] /= rho[r];
            }
        }
        ecur = Gd.e;
        acur = Gd.a;
#pragma unroll
        for (int r = 0; r < RH; ++r) {
            const double wgt = Gd.scale * pw[r];
            acc[r].x = fma(wgt, (double)v[r].x, acc[r].x);
            acc[r].y = fma(wgt, (double)v[r].y, acc[r].y);
        }
        if constexpr (NB == 1)
            __syncthreads();
        else
            b ^= 1;
    }
    const auto fj = gview(D.nchunk == 1 ? D.f + (int64_t)j * D.ldo + A.ka - 1
                                        : D.part + ((int64_t)j * D.nchunk + mp.chunk) * A.nrows);
#pragma unroll
    for (int r = 0; r < RH; ++r) {
        const int64_t kp = j1 + (int64_t)A.L1 * (lane + 64 * r);
        if (kp < A.nrows) { // rows past the block are discarded
            const cx<double> pk = cscale(
                expi_ratio(2 * A.Kka * A.Nna + 2 * A.ar * A.Nna * kp + A.ar * A.ac * kp * kp, 2 * A.D),
                1.0 / sqrt(rho[r]));
            const double val = pk.x * acc[r].x - pk.y * acc[r].y;
            if (D.nchunk == 1)
                fj[kp] += val;
            else
                fj[kp] = val;
        }
    }
}

template <typename F, int L2>
__global__ __launch_bounds__(512) HANK_WAVE_COLS_WPE void k_pass_cw(const FarDesc* __restrict__ descs, int ndesc) {
    constexpr int W = 8, S = wave_col_stride<L2>(), NB = wave_col_bufs<L2>();
    __shared__ cx<F> sh[NB][W * S];
    const FarItem mp = far_item(descs, ndesc, 0, descs[0].A.L1 / W);
    const FarDesc& D = descs[mp.desc];
    const FarArgs& A = D.A;
    const int64_t jb = (int64_t)mp.wg * W;
    if (jb >= A.nrows) return; // columns holding no output row
    // (uniform per workgroup)
    if (A.nrows <= A.L1)
        pass_cw_row0<F, L2>(D, mp, jb, reinterpret_cast<cx<double>*>(&sh[0][0])); // one output row
    else if (A.nrows <= jb + A.L / 2)
        pass_cw_main<F, L2, true>(D, mp, jb, sh);
    else
        pass_cw_main<F, L2, false>(D, mp, jb, sh);
}

// ---------------------------------------------------------------------------
// Row pass for rows of L1 = 8 x 512 points, 8 waves per row.  With j1 = b + 512 a
// and k = k1 + 8 k2 (a, k1 < 8; b, k2 < 512) the row DFT is
//     X[k1 + 8 k2] = sum_b W512^{b k2} W^{b k1} sum_a x[b + 512 a] W8^{a k1},
// W = e^{-2 pi i/L1}: thread b does the 8-point DFT over a in registers, one
// LDS exchange hands wave k1 the values of every b, and wave k1 does the
// 512-point DFT over b wave-locally.  The spectrum then sits in wave k1, lane
// l, register s as X[k1 + 8 (l + 64 s)] -- the layout in which the chirp
// spectrum of such rows is stored (k_pass_bw_fwd) -- and the inverse retraces
// the steps.  A group costs two workgroup barriers.
// ---------------------------------------------------------------------------
#ifndef HANK_WAVE_ROWS
#define HANK_WAVE_ROWS 1
#endif

template <typename F, int L1>
constexpr bool wave_rows() {
    return HANK_WAVE_ROWS && sizeof(F) == 8 && L1 == 4096;
}

// forward steps on v[a] = x[t + 512 a] of thread t; on return v[s] holds
// X[wv + 8 (lane + 64 s)] of the thread's wave wv.  sh: 8 regions of SR.
template <typename F, int SR>
__device__ __forceinline__ void row8x512_forward(cx<F> (&v)[8], cx<F>* sh, int t, int lane, int wv) {
    dft_small<F, 8, -1>(v);
    cx<double> w1 = tw_big<double>(t, 23 - 12); // W^t
    asm volatile("" : "+v"(w1.x), "+v"(w1.y));  // powers formed here, per group
    cx<double> w = w1;
    sh[lds_swz(t)] = v[0];
#pragma unroll
    for (int k1 = 1; k1 < 8; ++k1) {
        sh[k1 * SR + lds_swz(t)] = cmul(v[k1], mk(F(w.x), F(w.y)));
        if (k1 + 1 < 8) w = cmul(w, w1);
    }
    __syncthreads();
    cx<F>* my = sh + wv * SR;
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = my[lds_swz(lane + 64 * s)];
    wave_sync();
    fft_reg<F, 512, 8, -1, true>(v, my, lane);
}

template <typename F, int L1>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_pass_bw(
    const FarDesc* __restrict__ descs, int ndesc, int per_b) {
    static_assert(L1 == 4096, "rows of 8 x 512 points");
    constexpr int SR = wave_lds_len<512>();
    __shared__ cx<F> sh[8 * SR];
    const FarItem mp = far_item(descs, ndesc, 1, per_b, true);
    const FarDesc& D = descs[mp.desc];
    const FarArgs& A = D.A;
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    // one row per workgroup, and of the chunk's groups the share bs of bsplit
    const int64_t row = mp.wg % A.L2;
    const int bs = mp.wg / A.L2, nbs = max(1, D.bsplit);
    cx<F>* my = sh + wv * SR;
    // this wave's chirp spectrum (permuted layout)
    const auto hrow = gview((const cx<F>*)D.H) + row * L1 + wv * 512;
    cx<F> hv[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) hv[s] = gload(hrow + lane + 64 * s);
    const auto buf = gview((cx<F>*)D.buf);
    const int ng = A.g1 - A.g0;
    const int cs = mp.chunk * D.gchunk, ce = min(ng, cs + D.gchunk), share = (ce - cs + nbs - 1) / nbs;
    const int gs = cs + bs * share, ge = min(ce, gs + share);
    // columns j1 = t + 512 a >= ncols hold zeros (pass A does not store them),
    // and columns j1 >= nrows feed no output row (pass C skips them): the
    // loads and stores this thread makes, as bit masks over a
    uint32_t lmask = 0, smask = 0;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        lmask |= uint32_t(t + 512 * a < A.ncols) << a;
        smask |= uint32_t(t + 512 * a < A.nrows) << a;
    }
    const auto x0 = gview((const cx<F>*)D.x0);
    for (int gq = gs; gq < ge; ++gq) {
        const auto p = buf + ((int64_t)mp.j * ng + gq) * A.L + row * L1;
        cx<F> v[8];
        if (x0) {
            // a block of at most L1 columns: the row is x0(j1) e^{-2 pi i j1 row / L},
            // j1 = t + 512 a < ncols (what pass A would have stored)
            const auto xr = x0 + ((int64_t)mp.j * ng + gq) * A.ncols;
            cx<double> w = tw_big<double>((int64_t)t * row, A.twshift);
            const cx<double> ws = tw_big<double>((int64_t)512 * row, A.twshift);
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                v[a] = (lmask >> a) & 1 ? cmul(gload(xr + t + 512 * a), mk(F(w.x), F(w.y))) : mk(F(0), F(0));
                if (a + 1 < 8) w = cmul(w, ws);
            }
        } else {
#pragma unroll
            for (int a = 0; a < 8; ++a) v[a] = (lmask >> a) & 1 ? gload(p + t + 512 * a) : mk(F(0), F(0));
        }
        row8x512_forward<F, SR>(v, sh, t, lane, wv);
#pragma unroll
        for (int s = 0; s < 8; ++s) v[s] = cmul(v[s], hv[s]);
        fft_reg<F, 512, 8, 1, true>(v, my, lane);
        {
            // W^{-b wv} for b = lane + 64 s (base times step^s, from the table per group)
            const cx<double> i0 = tw_big<double>((int64_t)lane * wv, 23 - 12);
            cx<double> is = tw_big<double>((int64_t)64 * wv, 23 - 12);
            is.y = -is.y;
            cx<double> w = mk(i0.x, -i0.y);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                my[lds_swz(lane + 64 * s)] = cmul(v[s], mk(F(w.x), F(w.y)));
                if (s + 1 < 8) w = cmul(w, is);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) v[k1] = sh[k1 * SR + lds_swz(t)];
        dft_small<F, 8, 1>(v);
        // four-step twiddles e^{+2 pi i j1 row / L}, j1 = t + 512 a
        const cx<double> f0 = tw_big<double>((int64_t)t * row, A.twshift);
        cx<double> fs = tw_big<double>((int64_t)512 * row, A.twshift);
        fs.y = -fs.y;
        cx<double> w = mk(f0.x, -f0.y);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            if ((smask >> a) & 1) gstore(p + t + 512 * a, cmul(v[a], mk(F(w.x), F(w.y))));
            if (a + 1 < 8) w = cmul(w, fs);
        }
    }
}

// The chirp spectrum H^ = row FFT / L of such rows, stored in the permuted
// layout H'[row][k1 * 512 + k2] = H^[row][k1 + 8 k2].
template <typename F, int L1>
__global__ __launch_bounds__(512) void k_pass_bw_fwd(FarArgs A, const cx<F>* __restrict__ buf, cx<F>* __restrict__ H) {
    static_assert(L1 == 4096, "rows of 8 x 512 points");
    constexpr int SR = wave_lds_len<512>();
    __shared__ cx<F> sh[8 * SR];
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t row = blockIdx.x;
    cx<F> v[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) v[a] = buf[row * L1 + t + 512 * a];
    row8x512_forward<F, SR>(v, sh, t, lane, wv);
    const F sc = F(1.0 / (double)A.L);
#pragma unroll
    for (int s = 0; s < 8; ++s) H[row * L1 + wv * 512 + lane + 64 * s] = cscale(v[s], sc);
}

// f += sum of the pass-C chunk sums, in chunk order (deterministic)
__global__ __launch_bounds__(256) void k_far_reduce(const FarDesc* __restrict__ descs, int ndesc) {
    const FarItem mp = far_item(descs, ndesc, 2, 0);
    const FarDesc& D = descs[mp.desc];
    const int64_t kp = (int64_t)mp.wg * 256 + threadIdx.x;
    if (kp >= D.A.nrows) return;
    const auto pj = gview(D.part) + (int64_t)mp.j * D.nchunk * D.A.nrows + kp;
    double s = 0.0;
    for (int q = 0; q < D.nchunk; ++q) s += pj[(int64_t)q * D.A.nrows];
    gview(D.f)[(int64_t)mp.j * D.ldo + D.A.ka + kp - 1] += s;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t upload_tables(const DeviceTables& t) {
    return hipMemcpyToSymbol(HIP_SYMBOL(g_tab), &t, sizeof(DeviceTables), 0, hipMemcpyHostToDevice);
}

hipError_t launch_roots(int64_t nmax, double* b, int64_t nv, double* v, hipStream_t s) {
    if (nmax <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_roots, dim3((unsigned)((nmax + 255) / 256)), dim3(256), 0, s, nmax, b, nv, v);
    return hipGetLastError();
}

hipError_t launch_dht_scale(int64_t N, const double* v, const double* b, const double* src, double* dst,
                            bool final, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dht_scale, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, v, b, src, dst,
                       final ? 1 : 0);
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

hipError_t launch_near(const NearProb* probs, int32_t nprob, int64_t ntiles, double* partial, hipStream_t s) {
    if (ntiles > 0) hipLaunchKernelGGL(k_near, dim3((unsigned)ntiles), dim3(256), 0, s, probs, (int)nprob, partial);
    return hipGetLastError();
}

hipError_t launch_near_nu(const NearProb* probs, int32_t nprob, int64_t ntiles, double* partial, hipStream_t s) {
    if (ntiles > 0) hipLaunchKernelGGL(k_near_nu, dim3((unsigned)ntiles), dim3(256), 0, s, probs, (int)nprob, partial);
    return hipGetLastError();
}

hipError_t launch_near_multi(const NearProb* probs, int32_t nprob, int64_t ntiles, double* partial, hipStream_t s) {
    if (ntiles > 0)
        hipLaunchKernelGGL(k_near_multi, dim3((unsigned)ntiles), dim3(256), 0, s, probs, (int)nprob, partial);
    return hipGetLastError();
}

hipError_t launch_near_reduce(const NearProb* probs, int32_t nprob, int64_t nwv1, int64_t nrt1, int64_t nrt,
                              const double* partial, hipStream_t s) {
    if (nrt1 < 0 || nrt1 > nrt || nwv1 < nrt1) return hipErrorInvalidValue;
    if (nwv1 > 0)
        hipLaunchKernelGGL(k_near_reduce1, dim3((unsigned)((nwv1 + 3) / 4)), dim3(256), 0, s, probs, (int)nprob, nwv1,
                           nrt1, partial);
    if (nrt > nrt1)
        hipLaunchKernelGGL(k_near_reduce, dim3((unsigned)(nrt - nrt1)), dim3(256), 0, s, probs, (int)nprob, nrt1,
                           partial);
    return hipGetLastError();
}

// column passes: which 0 = A on data, 1 = A on the chirp kernel, 2 = C
#ifndef HANK_WAVE_COLS
#define HANK_WAVE_COLS 1
#endif
template <typename F, int L2>
static void pass_ac_dispatch(int which, const FarArgs* A, const FarDesc* descs, int ndesc, int64_t nwg, void* buf,
                             hipStream_t s) {
    constexpr int W = col_width(L2, sizeof(F) == 4);
    dim3 block(W * L2 / 8);
    // FP64 columns of 256 and 512 points: the one-wave-per-column kernels
    constexpr bool wave_cols = HANK_WAVE_COLS && sizeof(F) == 8 && (L2 == 256 || L2 == 512) && W == 8;
    if (which == 0) {
        if constexpr (wave_cols)
            hipLaunchKernelGGL((k_pass_aw<F, L2>), dim3((unsigned)nwg), dim3(512), 0, s, descs, ndesc);
        else
            hipLaunchKernelGGL((k_pass_a<F, L2, W>), dim3((unsigned)nwg), block, 0, s, descs, ndesc);
    } else if (which == 1) {
        hipLaunchKernelGGL((k_pass_a_kernel<F, L2, W>), dim3((unsigned)(A->L1 / W)), block, 0, s, *A, (cx<F>*)buf);
    } else {
        if constexpr (wave_cols)
            hipLaunchKernelGGL((k_pass_cw<F, L2>), dim3((unsigned)nwg), dim3(512), 0, s, descs, ndesc);
        else
            hipLaunchKernelGGL((k_pass_c<F, L2, W>), dim3((unsigned)nwg), block, 0, s, descs, ndesc);
    }
}

template <typename F>
static hipError_t pass_ac(int which, int32_t L2, const FarArgs* A, const FarDesc* descs, int ndesc, int64_t nwg,
                          void* buf, hipStream_t s) {
    switch (L2) {
    case 8: pass_ac_dispatch<F, 8>(which, A, descs, ndesc, nwg, buf, s); break;
    case 16: pass_ac_dispatch<F, 16>(which, A, descs, ndesc, nwg, buf, s); break;
    case 32: pass_ac_dispatch<F, 32>(which, A, descs, ndesc, nwg, buf, s); break;
    case 64: pass_ac_dispatch<F, 64>(which, A, descs, ndesc, nwg, buf, s); break;
    case 128: pass_ac_dispatch<F, 128>(which, A, descs, ndesc, nwg, buf, s); break;
    case 256: pass_ac_dispatch<F, 256>(which, A, descs, ndesc, nwg, buf, s); break;
    case 512: pass_ac_dispatch<F, 512>(which, A, descs, ndesc, nwg, buf, s); break;
    case 1024: pass_ac_dispatch<F, 1024>(which, A, descs, ndesc, nwg, buf, s); break;
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
static void pass_b_dispatch(bool fwd_only, const FarArgs* A, int32_t L2, const FarDesc* descs, int ndesc,
                            int64_t nwg, void* buf, void* H, hipStream_t s) {
    constexpr int ROWS = rows_per_wg<L1>();
    dim3 block(ROWS * L1 / 8);
    if constexpr (wave_rows<F, L1>()) { // one row per workgroup of 512 threads, as k_pass_b's
        static_assert(ROWS == 1, "one row per workgroup");
        if (fwd_only)
            hipLaunchKernelGGL((k_pass_bw_fwd<F, L1>), dim3((unsigned)A->L2), dim3(512), 0, s, *A, (const cx<F>*)buf,
                               (cx<F>*)H);
        else
            hipLaunchKernelGGL((k_pass_bw<F, L1>), dim3((unsigned)nwg), dim3(512), 0, s, descs, ndesc, (int)L2);
    } else if (fwd_only) {
        hipLaunchKernelGGL((k_pass_b_fwd<F, L1, ROWS>), dim3((unsigned)((A->L2 + ROWS - 1) / ROWS)), block, 0, s, *A,
                           (const cx<F>*)buf, (cx<F>*)H);
    } else {
        hipLaunchKernelGGL((k_pass_b<F, L1, ROWS>), dim3((unsigned)nwg), block, 0, s, descs, ndesc,
                           (int)((L2 + ROWS - 1) / ROWS));
    }
}

template <typename F>
static hipError_t pass_b(bool fwd_only, int32_t L1, const FarArgs* A, int32_t L2, const FarDesc* descs, int ndesc,
                         int64_t nwg, void* buf, void* H, hipStream_t s) {
    switch (L1) {
    case 8: pass_b_dispatch<F, 8>(fwd_only, A, L2, descs, ndesc, nwg, buf, H, s); break;
    case 16: pass_b_dispatch<F, 16>(fwd_only, A, L2, descs, ndesc, nwg, buf, H, s); break;
    case 32: pass_b_dispatch<F, 32>(fwd_only, A, L2, descs, ndesc, nwg, buf, H, s); break;
    case 64: pass_b_dispatch<F, 64>(fwd_only, A, L2, descs, ndesc, nwg, buf, H, s); break;
    case 128: pass_b_dispatch<F, 128>(fwd_only, A, L2, descs, ndesc, nwg, buf, H, s); break;
    case 256: pass_b_dispatch<F, 256>(fwd_only, A, L2, descs, ndesc, nwg, buf, H, s); break;
    case 512: pass_b_dispatch<F, 512>(fwd_only, A, L2, descs, ndesc, nwg, buf, H, s); break;
    case 1024: pass_b_dispatch<F, 1024>(fwd_only, A, L2, descs, ndesc, nwg, buf, H, s); break;
    case 2048: pass_b_dispatch<F, 2048>(fwd_only, A, L2, descs, ndesc, nwg, buf, H, s); break;
    case 4096: pass_b_dispatch<F, 4096>(fwd_only, A, L2, descs, ndesc, nwg, buf, H, s); break;
    case 8192: pass_b_dispatch<F, 8192>(fwd_only, A, L2, descs, ndesc, nwg, buf, H, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int32_t far_rows_per_wg(int32_t L1) { return L1 >= 2048 ? 1 : 2048 / L1; }

hipError_t launch_far_reduce(const FarDesc* descs, int32_t ndesc, int64_t nwg, hipStream_t s) {
    if (nwg > 0) hipLaunchKernelGGL(k_far_reduce, dim3((unsigned)nwg), dim3(256), 0, s, descs, (int)ndesc);
    return hipGetLastError();
}

hipError_t launch_chirp_spectrum(const FarArgs& A, bool fp32, void* work, void* H, hipStream_t s) {
    hipError_t e = fp32 ? pass_ac<float>(1, A.L2, &A, nullptr, 0, 0, work, s)
                        : pass_ac<double>(1, A.L2, &A, nullptr, 0, 0, work, s);
    if (e != hipSuccess) return e;
    return fp32 ? pass_b<float>(true, A.L1, &A, A.L2, nullptr, 0, 0, work, H, s)
                : pass_b<double>(true, A.L1, &A, A.L2, nullptr, 0, 0, work, H, s);
}

hipError_t launch_far_pass(int which, bool fp32, int32_t L1, int32_t L2, const FarDesc* descs, int32_t ndesc,
                           int64_t nwg, hipStream_t s) {
    if (nwg <= 0) return hipSuccess;
    if (which == 1)
        return fp32 ? pass_b<float>(false, L1, nullptr, L2, descs, ndesc, nwg, nullptr, nullptr, s)
                    : pass_b<double>(false, L1, nullptr, L2, descs, ndesc, nwg, nullptr, nullptr, s);
    const int w = (which == 0) ? 0 : 2;
    return fp32 ? pass_ac<float>(w, L2, nullptr, descs, ndesc, nwg, nullptr, s)
                : pass_ac<double>(w, L2, nullptr, descs, ndesc, nwg, nullptr, s);
}

} // namespace hank
