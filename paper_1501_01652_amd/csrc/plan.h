// plan.h -- host-side description of how one transform is computed.
//
// A plan splits the N x N matrix J_0(r w^T) of Sec. 1 into
//   * far-field blocks: rectangles on which every entry is replaced by the
//     Hankel expansion (Sec. 3.1) of J_0 at an equispaced reference argument,
//     corrected for the Bessel-root perturbations by a Taylor series in the
//     perturbation (the Neumann-addition/Taylor decomposition of Prop. 5.1 and
//     eq. (HankelSum), grouped by total perturbation degree as in Sec. 5.2);
//     each block costs one chirp-z transform per output group;
//   * the near field: everything else, summed directly (J^EVAL of
//     eq. (StableMatrixDecomposition) and the first columns/rows of Sec. 5.1/6).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace hank {

enum Task { T_SCHL = 0, T_FB = 1, T_DHT = 2, T_SCHL_PG = 3, T_FB_PG = 4 };

// The argument z_kn = r_k w_n written as  z~_kn + delta_kn  with the
// equispaced part z~_kn = r^_k w^_n = pi * K_k * N_n / D  exactly rational:
//   K_k = ar*k + br  (row integer),   r^_k = K_k / Dr
//   N_n = ac*n + bc  (column integer), w^_n = pi * N_n / Qc,   D = Dr*Qc
// and delta_kn = e_k * lambda_n + r^_k * b_n, where lambda_n = w^_n + b_n = j_{0,n}
// (Lemma 3.2: j_{0,n} = (n - 1/4) pi + b_n and j_{0,k}/j_{0,N+1} = r^_k + e_k).
// The Schlomilch and Fourier-Bessel tasks may be of integer order nu (J_nu in
// place of J_0; Fourier-Bessel still at the roots of J_0, eq. (FourierBessel)),
// and the Schlomilch ones have w_n = (n + shift) pi (Sec. 4, Remark 4.1):
// shift enters as N_n = n + shift.
constexpr int HANK_NU_MAX = 8;
constexpr int64_t HANK_SHIFT_MAX = 1024;
struct Grid {
    int task = 0;
    int nu = 0;
    int64_t shift = 0;
    int64_t N = 0;
    int64_t ar = 1, br = 0, ac = 1, bc = 0, Dr = 1, Qc = 1, D = 1;
    bool row_pert = false, col_pert = false;

    double rhat(int64_t k) const { return double(ar * k + br) / double(Dr); }
    double what(int64_t n) const;
    double ztilde(int64_t k, int64_t n) const;
};

Grid make_grid(int task, int64_t N, int nu = 0, int64_t shift = 0);

// Input-side term of a group: coefficient K times
//   (lambda_n/lref)^a (b_n/bref)^b (w^_n/w0)^(-m-1/2)
// where a is the group's row/column perturbation degree.
struct Term {
    int32_t b, m;
    double kre, kim;
};

// A group shares the output weight  (e_k/eref)^a (r^_k/r0)^(e-1/2) * scale.
struct Group {
    int32_t a, e;
    int32_t t0, t1; // terms [t0, t1)
    double scale;
};

struct Block {
    int64_t ka, kb, na, nb; // rows [ka,kb], columns [na,nb], 1-based inclusive
    int64_t L;              // FFT length, L >= (kb-ka+1) + (nb-na+1) - 1
    int32_t L1, L2;         // L = L1 * L2: row FFTs of length L1, column FFTs of L2
    double r0, w0, s0;      // r^_ka, w^_na, z~ at the block corner
    double eref, lref, bref;
    int32_t maxa, maxb, maxm; // largest exponents used by its terms
    int32_t g64 = 0;          // groups [0, g64) in FP64, [g64, end) in FP32
    std::vector<Group> groups;
    std::vector<Term> terms;
};

// Precision of a block's transforms: bulk 0 all FP64, 2 all FP32, 1 FP32 for
// the groups whose contribution is too small for FP32 rounding to matter
// (bound of every entry of the group's matrix relative to |c_n| times
// 4 log2(L) u_32 at most eps/(8 G)), provided the saving under cost model cm
// pays for a second set of launches; reorders the groups FP64 first.
struct CostModel;
void set_group_precision(const Grid& g, Block& b, double eps, int bulk, const CostModel& cm);

// Rows [k0, k1) sum columns [1, ncut) directly.
struct NearSeg {
    int64_t k0, k1, ncut;
};

struct Plan {
    Grid g;
    double eps = 0;
    int mode = 0; // 0 tuned, 1 paper
    bool fp32 = false;
    bool direct = false;
    int M = 0, K = 0, T = 0, P = 0;
    double s = 0, alpha = 0, beta = 0;
    int first_direct = 0;
    int64_t nrhs = 1; // right-hand sides the partition was balanced for
    std::vector<Block> blocks;
    std::vector<NearSeg> near;
    int64_t near_entries = 0;
    double cost = 0; // modelled seconds
};

// Cost-model constants (seconds); refined from measurements through the
// environment (HANK_COST_FFT, HANK_COST_NEAR, HANK_COST_BLOCK).
struct CostModel {
    double fft_pt_group64 = 1.8e-11; // per FFT point per group per right-hand side, FP64 (measured)
    double fft_pt_group32 = 1.5e-11; // same, FP32 (the passes move half the bytes but do the same
                                     // FFT work; measured FP32-bulk plans run barely faster)
    double near_entry = 1.2e-12;     // per directly summed entry, one right-hand side (measured)
    double near_plain_entry = 1.3e-12; // the same without root perturbations (Schlomilch, order 0)
    double near_nu_entry = 5.1e-12;  // the same for Schlomilch of order nu > 0 (k_near_nu, measured)
    double near_multi_entry = 5.5e-12; // per entry with several right-hand sides (J_0 once per entry;
                                       // set by the batched workload's throughput: 3.0e-12..7.0e-12
                                       // gave 4840..5036 transforms/s, best at 5.5e-12)
    double near_rhs = 4.5e-14;       // per entry and right-hand side of the product (FP64 MFMA)
    double block = 30e-6;            // fixed cost per block: three dependent launches and a reduce
                                     // (measured on single transforms, N = 3000..50000, as 50e-6;
                                     // 30e-6 after the kernel changes: batched workload 3% faster,
                                     // the single-transform configurations unchanged; 15e-6 cost
                                     // Schlomilch 4096 and Fourier-Bessel 2^16 at 1e-8 20-25%)
};

// ---- parameter formulas ----
double hankel_a(int m, int nu);                    // a_m(nu), Sec. 3.1
double param_s(int nu, int M, double eps);         // s_{nu,M}(eps), Sec. 3.1
double rem_bound(int nu, int M, double z);         // eq. (errorBound)
double param_t(int nu, int T, double eps);         // t_{nu,T}(eps), Sec. 3.2
double param_neumann(int K, double eps);           // eq. (NeumannInequality)
double param_pK(int K, double eps);                // eq. (pKe)
double param_qT(int T, double eps);                // eq. (qTe)
int paper_M(double eps);                           // Table 4
double paper_beta(int64_t N);                      // Table 4
int paper_P(double alpha, double beta, int64_t N); // Table 4

// bounds of Lemma 3.2
double bmax(int64_t n);
double emax(int64_t k, int64_t N);

// Build a plan.  Throws std::invalid_argument on bad input.
// nrhs: the number of right-hand sides the tuned partition is balanced for.
// mode: 0 tuned, 1 paper, 2 paper with P = 0 (single partition).
// Mpaper: M in modes 1 and 2 (0: Table 4's rule).  nu, shift: order and
// frequency shift of the Schlomilch tasks (0 for the others).
Plan make_plan(int task, int64_t N, double eps, int mode, int precision, bool direct,
               const CostModel& cm, int64_t nrhs = 1, int Mpaper = 0, int nu = 0, int64_t shift = 0);

// Fill terms/groups of a block; returns false if the truncation would exceed
// the supported term count.
bool build_block_terms(const Grid& g, Block& b, double eps, int mode, int Mpaper, int K, int T);

// Choose L1 x L2 for an FFT length: the autotuned split for log2(L) if one
// was installed (set_fft_split), else the default rule (default_fft_l2).
void fft_split(int64_t L, int32_t& L1, int32_t& L2);
int default_fft_l2(int lg);
void set_fft_split(int lg, int l2); // l2 = 0 restores the default
int tuned_fft_split(int lg);        // the installed l2 (0: none)
bool valid_fft_split(int lg, int l2); // a split the kernels support (L1 >= L2, L1 <= 8192)

CostModel cost_model_from_env();

} // namespace hank
