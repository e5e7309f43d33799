// fft_device.h -- power-of-two complex FFTs held in registers and exchanged
// through LDS (Stockham autosort, radix 8 with one radix-2/4 stage).
//
// A transform of length LEN is computed by NT = LEN/R threads; thread tt
// holds the R points x[tt + r*NT], r < R, before and after the call (natural
// order both ways).  SIGN = -1 is the forward DFT X_m = sum_j x_j e^{-2 pi i jm/LEN},
// SIGN = +1 the unnormalised inverse.  Every stage is one radix butterfly per
// register group, one LDS write and one LDS read, except the last, which
// leaves its outputs in the registers that hold them (its exchange would be
// the identity); `sh` must hold
// LEN + LEN/8 elements for this transform and every thread of the workgroup
// must call the function (it synchronises the workgroup).
#pragma once

#include "device_common.h"

// Build knobs (measured variants):
//   HANK_TW_DIRECT  1: each stage twiddle W^{kk s} is its own table load;
//                   0: one load and powers by complex multiplication
//   HANK_TW_OPAQUE  1: twiddle tables reached through an opaque pointer, so
//                   they are reloaded per group instead of hoisted into registers;
//                   2: only the base twiddle of each stage may be hoisted, its
//                   powers are formed at every use (pinned by an empty asm)
#ifndef HANK_TW_DIRECT
#define HANK_TW_DIRECT 0
#endif
#ifndef HANK_TW_OPAQUE
#define HANK_TW_OPAQUE 2
#endif

namespace hank {

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 3); }

// LDS slot of element i in the wave-local transforms: a permutation of the
// low six bits (each bit XORed with higher ones, so it is invertible and keeps
// i within its power-of-two block) under which the 16-byte elements that the
// radix-4 and radix-8 stages, and runs of 16 consecutive lanes, access
// together fall into distinct groups of four banks.
// (measured: the swizzle removes most bank conflicts of the wave-local
// stages but its index arithmetic costs registers and spills; the padded
// layout is faster, so it is the default)
#ifndef HANK_LDS_SWZ
#define HANK_LDS_SWZ 0
#endif
__device__ __forceinline__ int lds_swz(int i) {
#if HANK_LDS_SWZ
    return i ^ ((i >> 2) & 15) ^ ((i >> 3) & 15);
#else
    return lds_pad(i);
#endif
}
// LDS elements a wave-local transform of LEN points occupies
template <int LEN>
constexpr int wave_lds_len() {
    return HANK_LDS_SWZ ? LEN : LEN + LEN / 8;
}

template <typename F, int SIGN>
__device__ __forceinline__ cx<F> mul_si(cx<F> a) { // a * (SIGN i)
    return SIGN < 0 ? mk(a.y, -a.x) : mk(-a.y, a.x);
}

// HALF: a[RS/2 ..] are known to be zero (RS = 4, 8)
template <typename F, int RS, int SIGN, bool HALF = false>
__device__ __forceinline__ void dft_small(cx<F> (&a)[RS]) {
    static_assert(!HALF || RS >= 4, "half-zero inputs for radix 4 and 8");
    if constexpr (RS == 4 && HALF) {
        const cx<F> t = mul_si<F, SIGN>(a[1]);
        const cx<F> a0 = a[0], a1 = a[1];
        a[0] = a0 + a1;
        a[1] = a0 + t;
        a[2] = a0 - a1;
        a[3] = a0 - t;
    } else if constexpr (RS == 2) {
        cx<F> t = a[0];
        a[0] = t + a[1];
        a[1] = t - a[1];
    } else if constexpr (RS == 4) {
        cx<F> t0 = a[0] + a[2], t1 = a[0] - a[2], t2 = a[1] + a[3], t3 = mul_si<F, SIGN>(a[1] - a[3]);
        a[0] = t0 + t2;
        a[1] = t1 + t3;
        a[2] = t0 - t2;
        a[3] = t1 - t3;
    } else { // RS == 8: two DFT4 and the W8 twiddles
        const F c = F(0.70710678118654752440);
        cx<F> e[4] = {a[0], a[2], a[4], a[6]}, o[4] = {a[1], a[3], a[5], a[7]};
        dft_small<F, 4, SIGN, HALF>(e);
        dft_small<F, 4, SIGN, HALF>(o);
        cx<F> o1 = mk(c * (o[1].x - F(SIGN) * o[1].y), c * (F(SIGN) * o[1].x + o[1].y));
        cx<F> o2 = mul_si<F, SIGN>(o[2]);
        cx<F> o3 = mk(c * (-o[3].x - F(SIGN) * o[3].y), c * (F(SIGN) * o[3].x - o[3].y));
        a[0] = e[0] + o[0];
        a[4] = e[0] - o[0];
        a[1] = e[1] + o1;
        a[5] = e[1] - o1;
        a[2] = e[2] + o2;
        a[6] = e[2] - o2;
        a[3] = e[3] + o3;
        a[7] = e[3] - o3;
    }
}

// twiddle e^{SIGN 2 pi i t / TW_SMALL} from table `tw`
template <typename F, int SIGN>
__device__ __forceinline__ cx<F> tw_small(const double (*tw)[2], int t) {
    double c = tw[t][0], s = tw[t][1];
    return mk(F(c), F(SIGN < 0 ? s : -s));
}

// The twiddle table pointer passed through an empty asm statement: inside a
// loop over groups this stops the compiler from hoisting every stage's
// twiddles out of the loop (which would keep ~28 registers per stage alive).
__device__ __forceinline__ const double (*opaque_tw())[2] {
    const double(*p)[2] = g_tab.tw_small;
#if HANK_TW_OPAQUE == 1
    asm volatile("" : "+s"(p));
#endif
    return p;
}

// Synchronisation of LDS data that only one wave reads and writes: the LDS
// operations of a wave complete in issue order, so the fences only keep the
// compiler from moving them across this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// WAVE: the LEN/R threads of the transform are one wave (LEN = 64 R), whose
// exchanges need no workgroup barrier; its LDS slots are lds_swz(i) (LEN
// elements), otherwise lds_pad(i) (LEN + LEN/8).
// LAST: the final stage (Ns * RS = LEN).  Its butterfly q of thread tt
// produces the outputs tt + (q + s NB) NT -- exactly the positions that thread
// holds in registers v[q + s NB] afterwards -- so its LDS exchange is the
// identity and is skipped (the previous stage's synchronisation already
// orders every earlier LDS access before the caller's next one).
// HALFIN (first stage only, RS = R): the inputs v[R/2 ..] are zero.
template <typename F, int LEN, int R, int RS, int SIGN, bool WAVE = false, bool LAST = false, bool HALFIN = false>
__device__ __forceinline__ void fft_stage(cx<F> (&v)[R], cx<F>* sh, int tt, int Ns, const double (*tw)[2]) {
    static_assert(!HALFIN || RS == R, "half-zero input in a full-radix first stage");
    constexpr int NT = LEN / R;
    constexpr int NB = R / RS;
    auto slot = [](int i) { return WAVE ? lds_swz(i) : lds_pad(i); };
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int j = tt + q * NT;
        cx<F> a[RS];
#pragma unroll
        for (int s = 0; s < RS; ++s) a[s] = v[q + s * NB];
        const int kk = j & (Ns - 1);
        if (Ns > 1) {
            const int step = kk * (TW_SMALL / (Ns * RS));
#if HANK_TW_DIRECT
#pragma unroll
            for (int s = 1; s < RS; ++s) a[s] = cmul(a[s], tw_small<F, SIGN>(tw, s * step));
#else
            cx<F> w1 = tw_small<F, SIGN>(tw, step);
#if HANK_TW_OPAQUE == 2
            asm volatile("" : "+v"(w1.x), "+v"(w1.y));
#endif
            cx<F> w = w1;
#pragma unroll
            for (int s = 1; s < RS; ++s) {
                a[s] = cmul(a[s], w);
                if (s + 1 < RS) w = cmul(w, w1);
            }
#endif
        }
        dft_small<F, RS, SIGN, HALFIN>(a);
        if constexpr (LAST) {
#pragma unroll
            for (int s = 0; s < RS; ++s) v[q + s * NB] = a[s];
            continue;
        }
        const int base = (j - kk) * RS + kk;
#pragma unroll
        for (int s = 0; s < RS; ++s) sh[slot(base + s * Ns)] = a[s];
    }
    if constexpr (LAST) return;
    if constexpr (WAVE) wave_sync(); else __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = sh[slot(tt + r * NT)];
    if constexpr (WAVE) wave_sync(); else __syncthreads();
}

template <int N>
struct ilog2 {
    static constexpr int v = 1 + ilog2<N / 2>::v;
};
template <>
struct ilog2<1> {
    static constexpr int v = 0;
};

// HALFIN: the inputs x[LEN/2 ..] (registers v[R/2 ..]) are zero; needs
// LEN >= R * R, so that the first stage is a full-radix one
template <typename F, int LEN, int R, int SIGN, bool WAVE = false, bool HALFIN = false>
__device__ __forceinline__ void fft_reg(cx<F> (&v)[R], cx<F>* sh, int tt) {
    constexpr int LG = ilog2<LEN>::v, LR = ilog2<R>::v;
    static_assert((1 << LG) == LEN && (1 << LR) == R && LEN >= R, "power-of-two sizes");
    static_assert(!WAVE || LEN == 64 * R, "a wave-local transform has one point set per lane");
    constexpr int NST = LG / LR; // full-radix stages
    static_assert(!HALFIN || NST >= 2, "half-zero input: at least two full-radix stages");
    int Ns = 1;
#pragma unroll
    for (int st = 0; st < NST - 1; ++st) {
        if (HALFIN && st == 0)
            fft_stage<F, LEN, R, R, SIGN, WAVE, false, HALFIN>(v, sh, tt, Ns, opaque_tw());
        else
            fft_stage<F, LEN, R, R, SIGN, WAVE>(v, sh, tt, Ns, opaque_tw());
        Ns *= R;
    }
    if constexpr (LG % LR != 0) {
        if constexpr (NST > 0) {
            fft_stage<F, LEN, R, R, SIGN, WAVE>(v, sh, tt, Ns, opaque_tw());
            Ns *= R;
        }
        fft_stage<F, LEN, R, (1 << (LG % LR)), SIGN, WAVE, true>(v, sh, tt, Ns, opaque_tw());
    } else {
        fft_stage<F, LEN, R, R, SIGN, WAVE, true>(v, sh, tt, Ns, opaque_tw());
    }
}

// e^{-2 pi i e / L} for 0 <= e < L, L = 2^lg <= 2^23, from the two-level table
// (its base passed through an empty asm statement, as for opaque_tw)
template <typename F>
__device__ __forceinline__ cx<F> tw_big(int64_t e, int shift /* 23 - lg */) {
    int64_t E = e << shift;
    int hi = (int)(E >> 12), lo = (int)(E & (TW_LO - 1));
    const DeviceTables* T = &g_tab;
#if HANK_TW_OPAQUE == 1
    asm volatile("" : "+s"(T));
#endif
    cx<double> a = mk(T->tw_hi[hi][0], T->tw_hi[hi][1]);
    cx<double> b = mk(T->tw_lo[lo][0], T->tw_lo[lo][1]);
    cx<double> p = cmul(a, b);
    return mk(F(p.x), F(p.y));
}

} // namespace hank
