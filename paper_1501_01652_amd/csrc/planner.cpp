// planner.cpp -- parameter selection and partition (host, FP64, no GPU calls).
//
// Every parameter follows from eps and N through the paper's error bounds:
//   M, s_{nu,M}(eps), alpha, beta, P          Table 4 and Sec. 3.1 / 4.2
//   K, T, the first direct columns/rows       Sec. 5.1 (eqs. (pKe), (qTe)) and Sec. 6
// Three modes build the partition:
//   paper  the paper's rules verbatim (global K, T and M for every block);
//   single the paper's rules with P = 0: one far block (Sec. 3.3);
//   tuned  the same staircase of rectangular blocks, but the block shape is
//          chosen by a cost model of this GPU and each block keeps only the
//          perturbation and asymptotic terms its own error bound requires.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <map>
#include <mutex>
#include <stdexcept>
#include <tuple>

namespace hank {

using cplx = std::complex<double>;

double Grid::what(int64_t n) const { return M_PI * double(ac * n + bc) / double(Qc); }

double Grid::ztilde(int64_t k, int64_t n) const {
    // K_k * N_n < 2^53, so the product is exact in double
    return M_PI * (double(ar * k + br) * double(ac * n + bc)) / double(D);
}

Grid make_grid(int task, int64_t N, int nu, int64_t shift) {
    if (nu < 0 || nu > HANK_NU_MAX || shift < 0 || shift > HANK_SHIFT_MAX)
        throw std::invalid_argument("nu must lie in [0, 8] and shift in [0, 1024]");
    if (nu != 0 && task == T_DHT) throw std::invalid_argument("nu applies to the Schlomilch and Fourier-Bessel tasks");
    if (shift != 0 && task != T_SCHL && task != T_SCHL_PG)
        throw std::invalid_argument("shift applies to the Schlomilch tasks only");
    Grid g;
    g.task = task;
    g.nu = nu;
    g.shift = shift;
    g.N = N;
    switch (task) {
    case T_SCHL: // r_k = (k-1)/(N-1), w_n = (n + shift) pi
        g.ar = 1; g.br = -1; g.Dr = N - 1; g.ac = 1; g.bc = shift; g.Qc = 1;
        break;
    case T_FB: // r_k = (k-1)/(N-1), w_n = j_{0,n} = (n-1/4)pi + b_n
        g.ar = 1; g.br = -1; g.Dr = N - 1; g.ac = 4; g.bc = -1; g.Qc = 4;
        g.col_pert = true;
        break;
    case T_DHT: // r_k = j_{0,k}/j_{0,N+1} = (4k-1)/(4N+3) + e_k
        g.ar = 4; g.br = -1; g.Dr = 4 * N + 3; g.ac = 4; g.bc = -1; g.Qc = 4;
        g.row_pert = g.col_pert = true;
        break;
    case T_SCHL_PG: // r_k = k/N, w_n = (n + shift) pi
        g.ar = 1; g.br = 0; g.Dr = N; g.ac = 1; g.bc = shift; g.Qc = 1;
        break;
    case T_FB_PG: // r_k = k/N, w_n = j_{0,n}
        g.ar = 1; g.br = 0; g.Dr = N; g.ac = 4; g.bc = -1; g.Qc = 4;
        g.col_pert = true;
        break;
    default:
        throw std::invalid_argument("unknown task");
    }
    g.D = g.Dr * g.Qc;
    return g;
}

// ---------------------------------------------------------------------------
// Parameter formulas
// ---------------------------------------------------------------------------
double hankel_a(int m, int nu) {
    // a_m(nu) for the orders and term counts the planner uses, tabulated once
    static const int NUS = 48, MS = 64;
    struct Tab {
        double v[NUS][MS];
        Tab() {
            for (int n = 0; n < NUS; ++n) {
                v[n][0] = 1.0;
                for (int i = 1; i < MS; ++i)
                    v[n][i] = v[n][i - 1] * (4.0 * n * n - double(2 * i - 1) * double(2 * i - 1)) / (8.0 * i);
            }
        }
    };
    static const Tab tab; // thread-safe one-time initialisation
    if (nu >= 0 && nu < NUS && m >= 0 && m < MS) return tab.v[nu][m];
    double v = 1.0;
    for (int i = 1; i <= m; ++i) v *= (4.0 * nu * nu - double(2 * i - 1) * double(2 * i - 1)) / (8.0 * i);
    return v;
}

double param_s(int nu, int M, double eps) {
    // fixed-point iteration of Sec. 3.1, started at 1, four steps
    double a0 = std::fabs(hankel_a(2 * M, nu)), a1 = std::fabs(hankel_a(2 * M + 1, nu));
    double s = 1.0;
    for (int j = 0; j < 4; ++j)
        s = std::pow(std::sqrt(2.0) * (a0 + a1 / s) / (std::sqrt(M_PI) * eps), 1.0 / (2.0 * M + 0.5));
    return s;
}

double rem_bound(int nu, int M, double z) {
    return std::sqrt(2.0 / (M_PI * z)) *
           (std::fabs(hankel_a(2 * M, nu)) / std::pow(z, 2 * M) +
            std::fabs(hankel_a(2 * M + 1, nu)) / std::pow(z, 2 * M + 1));
}

static double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

double param_t(int nu, int T, double eps) {
    return std::pow(std::ldexp(1.0, 2 * T + nu) * factorial(T + nu) * factorial(T) * eps,
                    1.0 / (2 * T + nu));
}

double param_neumann(int K, double eps) { return 2.0 / M_E * std::pow(eps / 5.2, 1.0 / K); }

double param_pK(int K, double eps) { return M_E / (16.0 * M_PI) * std::pow(5.2 / eps, 1.0 / K) + 0.25; }

double param_qT(int T, double eps) {
    return std::pow(eps, -1.0 / (2.0 * T)) / (16.0 * M_PI * std::pow(factorial(T), 1.0 / T)) + 0.25;
}

int paper_M(double eps) { return std::max(int(std::floor(0.3 * std::log(1.0 / eps))), 3); }

double paper_beta(int64_t N) { return std::min(3.0 / std::log(double(N)), 1.0); }

int paper_P(double alpha, double beta, int64_t N) {
    if (beta >= 1.0) return 0;
    double x = std::log(30.0 / (alpha * std::sqrt(double(N)))) / std::log(beta);
    return std::max(0, int(std::ceil(x)));
}

double bmax(int64_t n) { return 1.0 / (8.0 * (double(n) - 0.25) * M_PI); }

double emax(int64_t k, int64_t N) {
    return 1.0 / (8.0 * (double(N) + 0.75) * (double(k) - 0.25) * M_PI * M_PI);
}

// l2 chosen by the autotuner per log2(L) (0: the default rule)
static int g_l2_tuned[32] = {0};

void set_fft_split(int lg, int l2) {
    if (lg >= 0 && lg < 32) g_l2_tuned[lg] = l2;
}

int tuned_fft_split(int lg) { return (lg >= 0 && lg < 32) ? g_l2_tuned[lg] : 0; }

bool valid_fft_split(int lg, int l2) { return lg >= 6 && lg <= 23 && l2 >= 3 && 2 * l2 <= lg && lg - l2 <= 13; }

int default_fft_l2(int lg);

void fft_split(int64_t L, int32_t& L1, int32_t& L2) {
    int lg = 0;
    while ((int64_t(1) << lg) < L) ++lg;
    if (lg < 32 && g_l2_tuned[lg] > 0 && valid_fft_split(lg, g_l2_tuned[lg])) {
        L2 = int32_t(1) << g_l2_tuned[lg];
        L1 = int32_t(1) << (lg - g_l2_tuned[lg]);
        return;
    }
    const int l2 = default_fft_l2(lg);
    L1 = int32_t(1) << (lg - l2);
    L2 = int32_t(1) << l2;
}

int default_fft_l2(int lg) {
    // columns (passes A and C) of 2^l2 <= 1024 points, rows (pass B) of
    // 2^l1 <= 2^l1max points; balanced below 2^16, columns of at least 256
    // above.  l1max = 12 up to 2^21 points (rows of 4096 points run on the
    // eight-wave four-step row pass, measured faster than rows of 8192 with
    // columns of 256), 13 above; HANK_FFT_L1MAX overrides
    static const int l1max_env = [] {
        const char* e = std::getenv("HANK_FFT_L1MAX");
        return e ? std::max(8, std::min(13, std::atoi(e))) : 0;
    }();
    const int l1max = l1max_env ? l1max_env : (lg <= 21 ? 12 : 13);
    return (lg <= 16) ? lg / 2 : std::min(10, std::max(8, lg - l1max));
}

CostModel cost_model_from_env() {
    CostModel cm;
    if (const char* v = std::getenv("HANK_COST_FFT")) cm.fft_pt_group64 = std::atof(v);
    if (const char* v = std::getenv("HANK_COST_FFT32")) cm.fft_pt_group32 = std::atof(v);
    if (const char* v = std::getenv("HANK_COST_NEAR")) cm.near_entry = std::atof(v);
    if (const char* v = std::getenv("HANK_COST_BLOCK")) cm.block = std::atof(v);
    if (const char* v = std::getenv("HANK_COST_NEAR_MULTI")) cm.near_multi_entry = std::atof(v);
    if (const char* v = std::getenv("HANK_COST_NEAR_RHS")) cm.near_rhs = std::atof(v);
    if (const char* v = std::getenv("HANK_COST_NEAR_NU")) cm.near_nu_entry = std::atof(v);
    if (const char* v = std::getenv("HANK_COST_NEAR_PLAIN")) cm.near_plain_entry = std::atof(v);
    return cm;
}

// ---------------------------------------------------------------------------
// Terms of a block
// ---------------------------------------------------------------------------
static double binom(int n, int k) { return factorial(n) / (factorial(k) * factorial(n - k)); }

// Paper's rearranged truncation (Sec. 5.2): for perturbation degree u the
// orders mu = 2j - u with min(j, u-j) <= T-1 and |u - 2j| <= K-1 are kept.
static bool paper_keep(int u, int j, int K, int T) {
    return std::min(j, u - j) <= T - 1 && std::abs(u - 2 * j) <= K - 1;
}

// d^a/dz^a d^b/dz^b J_0 = sum_mu w_mu J_mu  (J_mu' = (J_{mu-1} - J_{mu+1})/2,
// DLMF 10.6.1); in paper mode each level keeps only its paper orders.
static std::map<int, double> order_mix(int a, int b, bool paper, int K, int T) {
    std::map<int, double> w;
    for (int ja = 0; ja <= a; ++ja) {
        if (paper && a > 0 && !paper_keep(a, ja, K, T)) continue;
        double wa = std::ldexp(1.0, -a) * ((ja & 1) ? -1.0 : 1.0) * binom(a, ja);
        for (int jb = 0; jb <= b; ++jb) {
            if (paper && b > 0 && !paper_keep(b, jb, K, T)) continue;
            double wb = std::ldexp(1.0, -b) * ((jb & 1) ? -1.0 : 1.0) * binom(b, jb);
            w[(2 * ja - a) + (2 * jb - b)] += wa * wb;
        }
    }
    return w;
}

// the same mix for J_nu in place of J_0: every order mu becomes mu + nu
static std::map<int, double> shift_orders(const std::map<int, double>& w, int nu) {
    if (nu == 0) return w;
    std::map<int, double> out;
    for (auto& kv : w) out[kv.first + nu] = kv.second;
    return out;
}

static cplx ipow(int p) { // i^p
    switch (((p % 4) + 4) % 4) {
    case 0: return {1, 0};
    case 1: return {0, 1};
    case 2: return {-1, 0};
    default: return {0, -1};
    }
}

// J_mu(z) ~ sqrt(2/pi) Re[ e^{i(z - pi/4)} (-i)^mu sum_m i^m a_m(mu) z^{-m-1/2} ]
// (eq. (HankelExpansion) with mu = z - (2 mu + 1) pi/4), so a mix sum_mu w_mu J_mu
// has coefficient kappa_m = sqrt(2/pi) i^m sum_mu w_mu (-i)^mu a_m(|mu|).
static cplx kappa(const std::map<int, double>& w, int m) {
    cplx s = 0;
    for (auto& kv : w) s += kv.second * ipow(-kv.first) * hankel_a(m, std::abs(kv.first));
    return std::sqrt(2.0 / M_PI) * ipow(m) * s;
}

static int max_order(const std::map<int, double>& w) {
    int mx = 0;
    for (auto& kv : w)
        if (kv.second != 0.0) mx = std::max(mx, std::abs(kv.first));
    return mx;
}

static const int MAX_GROUPS = 512;
static const int MAX_TERMS = 8192;
static const int MAX_B = 24, MAX_A = 24, MAX_M = 60;

bool build_block_terms(const Grid& g, Block& bk, double eps, int mode, int Mpaper, int K, int T) {
    const int64_t N = g.N;
    bk.r0 = g.rhat(bk.ka);
    bk.w0 = g.what(bk.na);
    bk.s0 = bk.r0 * bk.w0;
    bk.lref = g.what(bk.nb) + (g.col_pert || g.row_pert ? bmax(bk.nb) : 0.0);
    bk.eref = g.row_pert ? emax(bk.ka, N) : 1.0;
    bk.bref = g.col_pert ? bmax(bk.na) : 1.0;
    const double dA = g.row_pert ? bk.eref * bk.lref : 0.0; // >= |e_k lambda_n|
    const double dB = g.col_pert ? g.rhat(bk.kb) * bk.bref : 0.0; // >= |r^_k b_n|
    const bool paper = (mode == 1);

    struct Pair {
        int a, b, M;
        double w;
        std::map<int, double> mix;
    };
    std::vector<Pair> pairs;

    if (paper) {
        int U = 2 * T + K - 2; // degrees 0 .. 2T+K-3 (Sec. 5.2)
        int amax = g.row_pert ? U - 1 : 0, bmx = g.col_pert ? U - 1 : 0;
        for (int a = 0; a <= amax; ++a)
            for (int b = 0; b <= bmx; ++b) {
                Pair p{a, b, Mpaper, 0.0, shift_orders(order_mix(a, b, true, K, T), g.nu)};
                bool any = false;
                for (auto& kv : p.mix) any |= kv.second != 0.0;
                if (any) pairs.push_back(p);
            }
    } else {
        // keep the largest Taylor weights dA^a dB^b/(a! b!) until the dropped
        // remainder (|J_0^(u)| <= 1) is below a quarter of eps
        const double eps_trunc = 0.25 * eps, eps_asy = 0.25 * eps;
        std::vector<std::pair<double, std::pair<int, int>>> all;
        int amax = dA > 0 ? 24 : 0, bmx = dB > 0 ? 24 : 0;
        for (int a = 0; a <= amax; ++a)
            for (int b = 0; b <= bmx; ++b) {
                double w = std::pow(dA, a) / factorial(a) * std::pow(dB, b) / factorial(b);
                if (a == 0 && b == 0) w = 1.0;
                all.push_back({w, {a, b}});
            }
        std::sort(all.begin(), all.end(), [](auto& x, auto& y) { return x.first > y.first; });
        std::vector<double> suffix(all.size() + 1, 0.0);
        for (size_t i = all.size(); i-- > 0;) suffix[i] = suffix[i + 1] + all[i].first;
        size_t keep = 1;
        while (keep < all.size() && suffix[keep] > eps_trunc) ++keep;
        for (size_t i = 0; i < keep; ++i) {
            Pair p{all[i].second.first, all[i].second.second, 0, all[i].first,
                   shift_orders(order_mix(all[i].second.first, all[i].second.second, false, 0, 0), g.nu)};
            pairs.push_back(p);
        }
        // fewest asymptotic terms per pair: w * E_u(M, zmin) <= eps_asy / |S|,
        // E_u = sum_mu |w_mu| R-bound_{mu,M}; the bound of (errorBound) needs
        // M >= mu/2 - 1/4 (DLMF 10.17(iii))
        const double share = eps_asy / double(pairs.size());
        for (auto& p : pairs) {
            int mo = max_order(p.mix);
            int Mlo = std::max(1, int(std::ceil(mo / 2.0 - 0.25)));
            int Mbest = -1;
            for (int M = Mlo; M <= 28; ++M) {
                double E = 0.0;
                for (auto& kv : p.mix) E += std::fabs(kv.second) * rem_bound(std::abs(kv.first), M, bk.s0);
                if (p.w * E <= share) {
                    Mbest = M;
                    break;
                }
            }
            if (Mbest < 0) return false;
            p.M = Mbest;
        }
    }

    // terms and groups by (a, e = b - m)
    std::map<std::pair<int, int>, std::vector<Term>> gm;
    const cplx rot = std::polar(1.0, -M_PI / 4); // e^{-i pi/4}
    for (auto& p : pairs) {
        double fac = std::pow(bk.eref * bk.lref, p.a) * std::pow(bk.r0 * bk.bref, p.b) /
                     (factorial(p.a) * factorial(p.b));
        for (int m = 0; m < 2 * p.M; ++m) {
            cplx kap = kappa(p.mix, m);
            if (kap == cplx(0, 0)) continue;
            cplx Kc = rot * kap * fac * std::pow(bk.s0, -m - 0.5);
            gm[{p.a, p.b - m}].push_back(Term{p.b, m, Kc.real(), Kc.imag()});
        }
    }
    bk.groups.clear();
    bk.terms.clear();
    bk.maxa = bk.maxb = bk.maxm = 0;
    for (auto& kv : gm) {
        Group G;
        G.a = kv.first.first;
        G.e = kv.first.second;
        G.t0 = int32_t(bk.terms.size());
        double sc = 0.0;
        for (auto& t : kv.second) sc = std::max(sc, std::hypot(t.kre, t.kim));
        if (sc == 0.0) continue;
        for (auto t : kv.second) {
            t.kre /= sc;
            t.kim /= sc;
            bk.terms.push_back(t);
            bk.maxb = std::max(bk.maxb, t.b);
            bk.maxm = std::max(bk.maxm, t.m);
        }
        G.t1 = int32_t(bk.terms.size());
        std::sort(bk.terms.begin() + G.t0, bk.terms.end(),
                  [](const Term& x, const Term& y) { return x.b < y.b; });
        G.scale = sc;
        bk.maxa = std::max(bk.maxa, G.a);
        bk.groups.push_back(G);
    }
    if (int(bk.groups.size()) > MAX_GROUPS || int(bk.terms.size()) > MAX_TERMS || bk.maxa > MAX_A ||
        bk.maxb > MAX_B || bk.maxm > MAX_M)
        return false;
    int64_t need = (bk.kb - bk.ka + 1) + (bk.nb - bk.na + 1) - 1;
    bk.L = 64;
    while (bk.L < need) bk.L *= 2;
    fft_split(bk.L, bk.L1, bk.L2);
    return true;
}

void set_group_precision(const Grid& g, Block& bk, double eps, int bulk, const CostModel& cm) {
    const int G = int(bk.groups.size());
    if (bulk != 1) {
        bk.g64 = bulk == 2 ? 0 : G;
        return;
    }
    int lg = 0;
    while ((int64_t(1) << lg) < bk.L) ++lg;
    const double u32 = 5.9604644775390625e-8; // 2^-24
    const double limit = eps / (8.0 * double(std::max(G, 1))) / (4.0 * double(lg) * u32);
    const double rmax = g.rhat(bk.kb);
    std::vector<Group> g64, g32;
    for (auto& G_ : bk.groups) {
        // |A_g(k) X_g(n)| <= scale (r^_k/r0)^(e-1/2) sum|K| |c_n|: the other ratios are <= 1
        double ksum = 0;
        for (int t = G_.t0; t < G_.t1; ++t) ksum += std::hypot(bk.terms[size_t(t)].kre, bk.terms[size_t(t)].kim);
        const double rowf = std::max(1.0, std::pow(rmax / bk.r0, double(G_.e) - 0.5));
        (G_.scale * rowf * ksum <= limit ? g32 : g64).push_back(G_);
    }
    const double saving = double(bk.L) * double(g32.size()) * (cm.fft_pt_group64 - cm.fft_pt_group32);
    if (g32.empty() || (!g64.empty() && saving < cm.block)) {
        bk.g64 = G;
        return;
    }
    bk.g64 = int32_t(g64.size());
    bk.groups = g64;
    bk.groups.insert(bk.groups.end(), g32.begin(), g32.end());
}

// ---------------------------------------------------------------------------
// Partition
// ---------------------------------------------------------------------------
static int64_t first_row_ge(const Grid& g, double r) { // smallest k with r^_k >= r
    if (r <= g.rhat(1)) return 1;
    double kk = (r * double(g.Dr) - double(g.br)) / double(g.ar);
    int64_t k = std::max<int64_t>(1, int64_t(std::ceil(kk)) - 1);
    while (k <= g.N && g.rhat(k) < r) ++k;
    while (k > 1 && g.rhat(k - 1) >= r) --k;
    return k;
}

static int64_t first_col_ge(const Grid& g, double w) { // smallest n with w^_n >= w
    if (w <= g.what(1)) return 1;
    double nn = (w * double(g.Qc) / M_PI - double(g.bc)) / double(g.ac);
    if (nn > double(g.N) + 2) return g.N + 1;
    int64_t n = std::max<int64_t>(1, int64_t(std::ceil(nn)) - 1);
    while (n <= g.N && g.what(n) < w) ++n;
    while (n > 1 && g.what(n - 1) >= w) --n;
    return n;
}

static int64_t n_min(const Grid& g, int64_t k, double s, int64_t nfloor) {
    double r = g.rhat(k);
    if (r <= 0) return g.N + 1;
    int64_t n = std::max(first_col_ge(g, s / r), nfloor);
    while (n <= g.N && g.ztilde(k, n) < s) ++n;
    return n;
}

static int64_t k_min(const Grid& g, int64_t n, double s, int64_t kfloor) {
    double w = g.what(n);
    int64_t k = std::max(first_row_ge(g, s / w), kfloor);
    while (k <= g.N && g.ztilde(k, n) < s) ++k;
    return k;
}

// Split blocks whose chirp-z convolution would exceed the largest FFT.
static const int64_t MAX_SPAN = int64_t(1) << 22;

static void push_block(std::vector<Block>& out, int64_t ka, int64_t kb, int64_t na, int64_t nb) {
    if (ka > kb || na > nb) return;
    for (int64_t r = ka; r <= kb; r += MAX_SPAN)
        for (int64_t c = na; c <= nb; c += MAX_SPAN) {
            Block b{};
            b.ka = r;
            b.kb = std::min(kb, r + MAX_SPAN - 1);
            b.na = c;
            b.nb = std::min(nb, c + MAX_SPAN - 1);
            out.push_back(b);
        }
}

// The staircase of Fig. 4: a square-ish block Q1 from (k0, n0) plus P row
// strips and P column strips, each strip's corner on the curve z~ = s.
// A block whose FFT would exceed MAX_FFT points (8192-point rows x
// 1024-point columns) is cut into f x f sub-blocks, rows and columns in f
// nearly equal parts, f the smallest power of two that fits.  The sub-blocks
// cover the same entries, each with its own corner and terms.
static const int64_t MAX_FFT = int64_t(1) << 23;
static void split_large(std::vector<Block>& v) {
    std::vector<Block> out;
    for (auto& b : v) {
        const int64_t R = b.kb - b.ka + 1, C = b.nb - b.na + 1;
        int64_t f = 1;
        while ((R + f - 1) / f + (C + f - 1) / f - 1 > MAX_FFT) f *= 2;
        for (int64_t i = 0; i < f; ++i)
            for (int64_t j = 0; j < f; ++j) {
                const int64_t ka = b.ka + i * R / f, kb = b.ka + (i + 1) * R / f - 1;
                const int64_t na = b.na + j * C / f, nb = b.na + (j + 1) * C / f - 1;
                if (ka <= kb && na <= nb) push_block(out, ka, kb, na, nb);
            }
    }
    v.swap(out);
}

static std::vector<Block> staircase(const Grid& g, double s, double R0, double beta, int P,
                                    int64_t kfloor, int64_t nfloor) {
    std::vector<Block> out;
    const int64_t N = g.N;
    int64_t k0 = std::max(first_row_ge(g, R0), kfloor);
    if (k0 > N) return out;
    int64_t n0 = n_min(g, k0, s, nfloor);
    if (n0 > N) return out;
    push_block(out, k0, N, n0, N);
    const double r0 = g.rhat(k0), w0 = g.what(n0);
    int64_t kprev = k0, nprev = n0;
    for (int p = 1; p <= P; ++p) { // row strips: rows below k0, long column range
        int64_t kp = std::max(first_row_ge(g, r0 * std::pow(beta, p)), kfloor);
        if (kp >= kprev) break;
        int64_t na = n_min(g, kp, s, nfloor);
        if (na <= N) push_block(out, kp, kprev - 1, na, N);
        kprev = kp;
    }
    for (int p = 1; p <= P; ++p) { // column strips
        int64_t np = std::max(first_col_ge(g, w0 * std::pow(beta, p)), nfloor);
        if (np >= nprev) break;
        int64_t ka = k_min(g, np, s, kfloor);
        if (ka <= N) push_block(out, ka, N, np, nprev - 1);
        nprev = np;
    }
    split_large(out);
    return out;
}

// Near field: per row k the far columns must be a suffix [ncut, N].
static bool near_segments(const Grid& g, const std::vector<Block>& blocks, std::vector<NearSeg>& segs,
                          int64_t& entries) {
    const int64_t N = g.N;
    std::vector<int64_t> cuts{1, N + 1};
    for (auto& b : blocks) {
        cuts.push_back(b.ka);
        cuts.push_back(b.kb + 1);
    }
    std::sort(cuts.begin(), cuts.end());
    cuts.erase(std::unique(cuts.begin(), cuts.end()), cuts.end());
    segs.clear();
    entries = 0;
    for (size_t i = 0; i + 1 < cuts.size(); ++i) {
        int64_t x = cuts[i], y = cuts[i + 1];
        if (x > N) break;
        int64_t nc = N + 1, cover = 0;
        for (auto& b : blocks)
            if (b.ka <= x && b.kb >= y - 1) {
                nc = std::min(nc, b.na);
                cover += b.nb - b.na + 1;
            }
        if (cover != N + 1 - nc) return false;
        if (!segs.empty() && segs.back().ncut == nc && segs.back().k1 == x)
            segs.back().k1 = y;
        else
            segs.push_back(NearSeg{x, y, nc});
        entries += (y - x) * (nc - 1);
    }
    return true;
}

static double plan_cost(const Plan& p, const CostModel& cm) {
    const double r = double(p.nrhs);
    const bool plain = !p.g.col_pert && !p.g.row_pert;
    double c = double(p.near_entries) *
               (p.g.nu > 0      ? r * cm.near_nu_entry
                : p.nrhs == 1   ? (plain ? cm.near_plain_entry : cm.near_entry)
                                : cm.near_multi_entry + r * cm.near_rhs);
    for (auto& b : p.blocks) {
        const double g64 = double(b.g64), g32 = double(b.groups.size()) - g64;
        // the passes skip the work-buffer columns without data (j1 >= ncols:
        // pass A and pass B's loads) or results (j1 >= nrows: pass B's stores
        // and pass C); with time shares of about 1/4, 1/2, 1/4 for passes A, B, C
        // and pass B's transforms always run in full, the relative cost is
        // 1/4 + 3/8 (fa + fc)
        const double L1 = double(b.L1), fa = std::min(double(b.nb - b.na + 1), L1) / L1,
                     fc = std::min(double(b.kb - b.ka + 1), L1) / L1;
        c += cm.block * ((g64 > 0 && g32 > 0) ? 2.0 : 1.0) +
             double(b.L) * (g64 * cm.fft_pt_group64 + g32 * cm.fft_pt_group32) * r * (0.25 + 0.375 * (fa + fc));
    }
    return c;
}

// Outcome of the tuned search at a grid size, per (task, N, eps, precision,
// nrhs, nu, shift), computed once (by a full make_plan there) and kept.
struct TunedParams {
    int M = 0;
    double beta = 0;
    int P = 0;
};
static thread_local TunedParams last_search_;
static bool tuned_params(int task, int64_t Ng, double eps, int precision, int64_t nrhs, int nu, int64_t shift,
                         const CostModel& cm, TunedParams& out) {
    typedef std::tuple<int, int64_t, double, int, int64_t, int, int64_t> K;
    static std::mutex mu;
    static std::map<K, TunedParams> cache;
    const K key{task, Ng, eps, precision, nrhs, nu, shift};
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            out = it->second;
            return true;
        }
    }
    try {
        (void)make_plan(task, Ng, eps, 0, precision, false, cm, nrhs, 0, nu, shift); // runs the full search
    } catch (const std::exception&) {
        return false;
    }
    out = last_search_;
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = out;
    return true;
}

Plan make_plan(int task, int64_t N, double eps, int mode, int precision, bool direct, const CostModel& cm,
               int64_t nrhs, int Mpaper, int nu, int64_t shift) {
    if (!(eps >= 1e-15 && eps < 1.0) || !std::isfinite(eps)) throw std::invalid_argument("eps out of range");
    if (mode < 0 || mode > 2) throw std::invalid_argument("plan_mode must be 0, 1 or 2");
    if (Mpaper < 0 || Mpaper > 20 || (Mpaper > 0 && mode == 0))
        throw std::invalid_argument("M must lie in [1, 20] and needs plan_mode 1 or 2");
    int64_t Nmin = (task == T_SCHL || task == T_FB) ? 2 : 1;
    if (N < Nmin || N > (int64_t(1) << 24)) throw std::invalid_argument("N out of range");
    Plan p;
    p.g = make_grid(task, N, nu, shift);
    p.eps = eps;
    p.mode = mode;
    p.direct = direct;
    p.fp32 = (precision == 2) || (precision == 0 && eps >= 1e-6);
    p.nrhs = std::max<int64_t>(1, nrhs);

    // paper parameters (reported in both modes)
    p.M = Mpaper > 0 ? Mpaper : paper_M(eps);
    int numax = nu; // Schlomilch of order nu: only J_nu
    if (p.g.col_pert || p.g.row_pert) {
        double f = (task == T_DHT) ? 1.01 : 1.0;
        p.K = 1;
        while (f * param_pK(p.K, eps) > 30.0) ++p.K;
        p.T = 1;
        while (f * param_qT(p.T, eps) > 30.0) ++p.T;
        p.first_direct = int(std::floor(f * std::max(param_pK(p.K, eps), param_qT(p.T, eps))));
        numax = (task == T_DHT) ? 2 * p.K - 2 : nu + p.K - 1; // orders nu -+ (K-1), Sec. 5.1
    }
    // the remainder bound of eq. (errorBound) holds for orders mu <= 2M + 1/2:
    // Table 4's M is raised to that where the orders need it (an explicit M is not)
    if (Mpaper == 0) p.M = std::max(p.M, int(std::ceil(numax / 2.0 - 0.25)));
    if (mode != 0 && 2 * p.M + 0.5 < numax)
        throw std::invalid_argument("M too small for the Bessel orders of this plan");
    p.s = param_s(numax, p.M, eps);
    p.alpha = std::sqrt(p.s / M_PI);
    // DHT: the footnote of Sec. 6 runs Fourier-Bessel on the padded size 4N+3
    int64_t Neff = (task == T_DHT) ? 4 * N + 3 : N;
    p.beta = paper_beta(Neff);
    p.P = mode == 2 ? 0 : paper_P(p.alpha, p.beta, Neff);

    auto finish = [&](Plan& q) -> bool {
        if (!near_segments(q.g, q.blocks, q.near, q.near_entries)) return false;
        q.cost = plan_cost(q, cm);
        return true;
    };

    if (direct) {
        finish(p);
        return p;
    }

    int64_t kfloor = 1, nfloor = 1;
    if (task == T_FB || task == T_FB_PG) nfloor = p.first_direct + 1;
    if (task == T_DHT) kfloor = p.first_direct + 1;

    if (mode != 0) {
        double R0 = p.alpha / std::sqrt(double(Neff));
        p.blocks = staircase(p.g, p.s, R0, p.beta, p.P, kfloor, nfloor);
        std::vector<Block> ok;
        for (auto& b : p.blocks) {
            if (!build_block_terms(p.g, b, eps, 1, p.M, p.K, p.T))
                throw std::runtime_error("paper plan exceeds supported term count");
            set_group_precision(p.g, b, eps, p.fp32 ? 2 : 0, cm);
            ok.push_back(b);
        }
        p.blocks = ok;
        if (!finish(p)) throw std::logic_error("partition is not a staircase");
        return p;
    }

    // tuned: search corner value s, refinement beta and strip count P;
    // candidates share many blocks, so block term tables are memoised
    struct Key {
        int64_t a, b, c, d;
        bool operator<(const Key& o) const {
            return a != o.a ? a < o.a : b != o.b ? b < o.b : c != o.c ? c < o.c : d < o.d;
        }
    };
    std::map<Key, std::pair<bool, Block>> memo;
    auto build = [&](Block& b) -> bool {
        Key key{b.ka, b.kb, b.na, b.nb};
        auto it = memo.find(key);
        if (it != memo.end()) {
            b = it->second.second;
            return it->second.first;
        }
        bool ok = build_block_terms(p.g, b, eps, 0, 0, 0, 0);
        if (ok) set_group_precision(p.g, b, eps, p.fp32 ? 2 : (precision == 0 ? 1 : 0), cm);
        memo[key] = {ok, b};
        return ok;
    };
    // the plain direct sum is a candidate too
    Plan best = p;
    finish(best);
    int best_M = 0; // 0: the direct sum
    // one candidate: corner value s_{nu,M}(eps/8), refinement beta, P strips;
    // returns false when it adds no strip over P - 1
    auto candidate = [&](int Mc, double beta, int P) -> bool {
        const double s = param_s(nu, Mc, eps / 8.0);
        if (s < 2.0) return true;
        const double R0 = std::sqrt(s / M_PI) / std::sqrt(double(N));
        Plan q = p;
        q.s = s;
        q.alpha = std::sqrt(s / M_PI);
        q.beta = beta;
        q.P = P;
        q.blocks = staircase(q.g, s, R0, beta, P, 1, 1);
        bool valid = true;
        for (auto& b : q.blocks)
            if (!build(b)) {
                valid = false;
                break;
            }
        if (valid && finish(q) && q.cost < best.cost) {
            best = q;
            best_M = Mc;
        }
        return !(P > 0 && q.blocks.size() <= size_t(1 + 2 * (P - 1)));
    };
    // The full search costs 5-60 ms of host time, and its outcome (M, beta, P)
    // changes slowly with N.  Off the grid N_j = round(2^(j/4)) the outcome of
    // the search at the grid point below is reused, so that planning an
    // unseen N costs one candidate; it depends on N alone (never on which
    // plans were built before), so the same N always gets the same plan.
    const bool default_cm = cm.near_entry == CostModel().near_entry && cm.fft_pt_group64 == CostModel().fft_pt_group64 &&
                            cm.block == CostModel().block && cm.near_multi_entry == CostModel().near_multi_entry;
    int jg = 0;
    while (std::llround(std::pow(2.0, (jg + 1) / 4.0)) <= N) ++jg;
    const int64_t Ng = std::llround(std::pow(2.0, jg / 4.0));
    TunedParams tp;
    if (default_cm && Ng != N && Ng >= 1024 && tuned_params(task, Ng, eps, precision, nrhs, nu, shift, cm, tp)) {
        if (tp.M > 0) candidate(tp.M, tp.beta, tp.P);
    } else {
        const double betas[] = {0.06, 0.1, 0.15, 0.22, 0.3, 0.4, 0.55};
        int bp = 0;
        double bbeta = 0;
        for (int Mc = 2; Mc <= 14; ++Mc) {
            if (2 * Mc + 0.5 < nu) continue; // the remainder bound needs M >= nu/2 - 1/4
            for (double beta : betas)
                for (int P = 0; P <= 10; ++P) {
                    const int before = best_M;
                    const double bcost = best.cost;
                    if (!candidate(Mc, beta, P)) break; // no new strip
                    if (best_M != before || best.cost != bcost) {
                        bp = P;
                        bbeta = beta;
                    }
                }
        }
        last_search_ = TunedParams{best_M, bbeta, bp};
    }
    // keep the paper's reported M, K, T alongside the tuned partition
    best.M = p.M;
    best.K = p.K;
    best.T = p.T;
    best.first_direct = p.first_direct;
    return best;
}

} // namespace hank
