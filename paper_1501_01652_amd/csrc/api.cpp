// api.cpp -- the C ABI (include/hank.h): argument checks, plan cache, device
// resources of a plan, and the launch sequence of one transform.
#include "../../include/hank.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <atomic>
#include <thread>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.h"
#include "plan.h"
#include "tables.h"

using namespace hank;

namespace {

thread_local std::string t_err;
std::recursive_mutex g_mu;

hank_status fail(hank_status s, const std::string& msg) {
    t_err = msg;
    return s;
}

#define HIP_TRY(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(e_ == hipErrorOutOfMemory ? HANK_ENOMEM : HANK_EDEVICE,                    \
                        std::string(#call) + ": " + hipGetErrorString(e_));                        \
    } while (0)

// Columns per near-field work item.  A tile's columns are a serial loop, so
// the widest tile bounds the launch: the width is the largest of 2048, 1024,
// ..., 64 whose 64-row tile holds no more than the average work of one of the
// 1024 workgroups the chip keeps resident (256 compute units x 4; occupancy of
// the near kernel).  Small problems then fill the chip with short tiles and
// large ones keep the per-row reduction short.  HANK_NEAR_COLS fixes it.
int64_t near_chunk(const std::vector<NearSeg>& segs) {
    static const int64_t fixed = [] {
        const char* e = std::getenv("HANK_NEAR_COLS");
        return e ? std::max<int64_t>(64, std::min<int64_t>(NEAR_TILE_COLS, std::atoll(e))) : int64_t(0);
    }();
    if (fixed) return fixed;
    double entries = 0;
    for (auto& seg : segs) entries += double(seg.k1 - seg.k0) * double(seg.ncut - 1);
    const double resident = 1024.0;
    int64_t chunk = NEAR_TILE_COLS;
    while (chunk > 64 && 64.0 * double(chunk) * resident > entries) chunk /= 2;
    return chunk;
}

struct DevBlock {
    Block hb;
    FarArgs args{};
    void* H = nullptr;   // chirp spectrum for the FP64 groups [0, g64)
    void* H32 = nullptr; // and for the FP32 groups [g64, ngroups)
    GroupDev* groups = nullptr;
    TermDev* terms = nullptr;
};

struct DevPlan {
    Plan plan;
    int device = 0;
    double* b = nullptr; // root offsets b_1..b_{N+1}
    double* e = nullptr; // DHT row perturbations e_1..e_N
    double* v = nullptr; // DHT: v_n = 2/J_1(j_{0,n})^2, n = 1..N (self-inverse weights)
    double* nutab = nullptr; // Schlomilch of order nu > 0: the J_nu table (build_nu_table)
    int32_t mnu = NU_HANKEL_PAIRS; // Hankel pairs of the order-nu near field
    std::vector<NearTile> tiles; // host copies of the near-field tiles and row tiles
    std::vector<RowTile> rts;
    std::vector<RowTile> rts_red; // the row tiles that do not have exactly one tile
    int64_t rt_max_tiles = 0;     // most tiles of one row tile
    NearTile* d_tiles = nullptr;  // the same on the device
    RowTile* d_rts = nullptr;
    RowTile* d_rts_red = nullptr;
    std::vector<DevBlock> blocks;
    void* work = nullptr; // chirp-spectrum scratch during the build
    size_t bytes = 0;
    GridArgs G{};
    // cache bookkeeping (under g_mu): pins by graphs and server requests,
    // last use for the LRU order, and the call that last fetched the plan
    int32_t pins = 0;
    uint64_t last_use = 0, call = 0;

    ~DevPlan() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        auto fr = [](void* p) {
            if (p) (void)hipFree(p);
        };
        fr(b);
        fr(e);
        fr(v);
        fr(nutab);
        fr(work);
        fr(d_tiles);
        fr(d_rts);
        fr(d_rts_red);
        for (auto& d : blocks) {
            fr(d.H);
            fr(d.H32);
            fr(d.groups);
            fr(d.terms);
        }
        (void)hipSetDevice(cur);
    }
};

using Key = std::tuple<int, int64_t, uint64_t, int, int, int, int>;
std::map<Key, std::unique_ptr<DevPlan>> g_cache;
std::set<int> g_tables_ready;
// Plan cache limit (hank_cache_limit): past it the least recently used plans
// that nothing pins and the current call did not fetch are freed.
int64_t g_cache_limit = int64_t(16) << 30;
uint64_t g_use_clock = 0; // advanced by every fetch
uint64_t g_call = 0;      // advanced by every call that fetches plans

int64_t cache_total() {
    int64_t t = 0;
    for (auto& kv : g_cache) t += int64_t(kv.second->bytes);
    return t;
}

// Free least recently used plans until the cache holds at most `target`
// bytes; plans pinned or fetched by the current call stay.  Freeing
// synchronises the device (hipFree), so a plan's enqueued work completes first.
void evict_to(int64_t target) {
    int64_t total = cache_total();
    while (total > target) {
        auto victim = g_cache.end();
        for (auto it = g_cache.begin(); it != g_cache.end(); ++it) {
            const DevPlan& d = *it->second;
            if (d.pins > 0 || d.call == g_call) continue;
            if (victim == g_cache.end() || d.last_use < victim->second->last_use) victim = it;
        }
        if (victim == g_cache.end()) return; // everything left is in use
        total -= int64_t(victim->second->bytes);
        g_cache.erase(victim);
    }
}

hank_status ensure_tables(int dev) {
    if (g_tables_ready.count(dev)) return HANK_OK;
    static DeviceTables* host = nullptr;
    if (!host) {
        host = new DeviceTables;
        build_tables(*host);
    }
    HIP_TRY(upload_tables(*host));
    g_tables_ready.insert(dev);
    return HANK_OK;
}

// Device allocation of the library.  For tests of the failure paths,
// HANK_TEST_FAIL_ALLOC=n makes the n-th allocation from then on (counted
// across the process) fail as out of memory.
hipError_t hank_malloc(void** p, size_t bytes) {
    static std::atomic<long> count{0};
    static std::string armed;
    const char* e = std::getenv("HANK_TEST_FAIL_ALLOC");
    if (e && *e) {
        static std::mutex mu;
        std::lock_guard<std::mutex> lk(mu);
        if (armed != e) { // a new setting restarts the count
            armed = e;
            count = 0;
        }
        if (++count == std::atol(e)) return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

template <typename T>
hank_status dev_alloc(T*& p, size_t count, size_t& total) {
    if (count == 0) count = 1;
    void* q = nullptr;
    hipError_t e = hank_malloc(&q, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? HANK_ENOMEM : HANK_EDEVICE,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    p = (T*)q;
    total += count * sizeof(T);
    return HANK_OK;
}

CostModel cost_model_for(const hank_options* o) {
    CostModel cm = cost_model_from_env();
    if (o && o->prefer_far) {
        cm.near_entry *= 1000.0;
        cm.near_multi_entry *= 1000.0;
        cm.near_rhs *= 1000.0;
        cm.near_nu_entry *= 1000.0;
        cm.near_plain_entry *= 1000.0;
        cm.block = 0.0;
    }
    return cm;
}

GridArgs grid_args(const Grid& g) {
    GridArgs a{};
    a.ar = g.ar;
    a.br = g.br;
    a.ac = g.ac;
    a.bc = g.bc;
    a.D = g.D;
    a.Dr = g.Dr;
    a.Qc = g.Qc;
    const long double PI = 3.141592653589793238462643383279502884L;
    a.pi_Qc = double(PI / (long double)g.Qc);
    long double pd = PI / (long double)g.D;
    a.piD_hi = double(pd);
    a.piD_lo = double(pd - (long double)a.piD_hi);
    a.invD = double(1.0L / (long double)g.D);
    a.invQc = double(1.0L / (long double)g.Qc);
    a.row_pert = g.row_pert;
    a.col_pert = g.col_pert;
    return a;
}

// Groups per launch of passes A-C.  A bounded batch keeps the work buffer
// (groups x L complex) small enough to stay in the Infinity Cache between the
// passes, but every launch repeats pass A's per-column set-up; measured on
// MI355X the single launch is faster, so the budget defaults to unlimited
// (HANK_GROUP_BATCH_MB caps it).
size_t group_batch(size_t bytes_per_group, size_t ngroups) {
    static const double budget = [] {
        const char* v = std::getenv("HANK_GROUP_BATCH_MB");
        return (v ? std::atof(v) : 1e12) * 1048576.0;
    }();
    size_t gb = size_t(budget / double(bytes_per_group));
    if (gb < 1) gb = 1;
    return std::min(gb, std::max<size_t>(1, ngroups));
}

// Per-block kernel variants of the near field.  The near field's share of the
// error budget is eps/8 per entry (the far blocks take eps/2), so a block
// whose smallest z is at least s_{0,M}(eps/8) (Sec. 3.1, eq. (errorBound))
// needs only M Hankel pairs; below z = 20 the tabulated Taylor pieces are
// used whatever eps.  Direct mode keeps the full-accuracy rule (1e-17).
struct NearRule {
    double zM[6]; // s_{0,M} for M = 2, 3, 4, 6, 8, 12
    bool mix6;    // 6 pairs suffice at z = 20
    bool small8;  // 8 terms of the small-argument pieces suffice (budget >= 1.25e-9)
    double rho1;  // residual phases up to this take the first-order factor (NV_*R)
};

NearRule near_rule(const Plan& p) {
    const double e = p.direct ? 1e-17 : p.eps / 8.0;
    const int Ms[6] = {2, 3, 4, 6, 8, 12};
    NearRule r{};
    for (int i = 0; i < 6; ++i) r.zM[i] = param_s(0, Ms[i], e);
    r.mix6 = r.zM[3] <= J0_ASY_Z;
    r.small8 = e >= 1.25e-9;
    // |e^{i rho} - (1 + i rho)| <= rho^2/2 times an amplitude <= 0.2 (z >= 20):
    // at most eps/64 per entry for rho <= sqrt(eps/6.4)
    r.rho1 = p.direct ? 0.0 : std::sqrt(p.eps / 6.4);
    return r;
}

// Bound on the residual phase rho = (e_k + r^_k) b_n over rows <= k1 and
// columns >= n0: r^_k grows with k; e_k <= b_k / (pi (N + 3/4)) < 0.02/N
// (Lemma 3.2's perturbation of the DHT rows, b_k < 0.05); b_n < 1/(8 pi (n - 1/4))
// (the leading term of McMahon's expansion, which the next, negative, term
// only lowers), with a margin of 0.1%.
double rho_bound(const Grid& g, int64_t k1, int64_t n0) {
    if (!g.col_pert) return 0.0;
    const double s = g.rhat(k1) + (g.row_pert ? 0.02 / double(g.N) : 0.0);
    return s * 1.001 / (8.0 * M_PI * (double(n0) - 0.25));
}

// Variant of the block of columns [n0, n1] of rows [k0, k1], from bounds on z
// over it: z >= z~ (the perturbations e_k, b_n are non-negative) and
// z <= z~ + 0.25.
int near_block_variant(const Grid& g, const NearRule& r, int64_t k0, int64_t k1, int64_t n0, int64_t n1) {
    const double zlo = g.ztilde(k0, n0), zhi = g.ztilde(k1, n1) + 0.25;
    const bool rot1 = g.col_pert && rho_bound(g, k1, n0) <= r.rho1;
    if (!(zhi >= J0_ASY_Z)) return r.small8 ? NV_SMALL8 : NV_SMALL;
    if (zlo < J0_ASY_Z)
        return r.mix6 ? (r.small8 ? (rot1 ? NV_MIX6_8R : NV_MIX6_8) : NV_MIX6) : (r.small8 ? NV_MIX12_8 : NV_MIX12);
    const int codes[6] = {NV_M2, NV_M3, NV_M4, NV_M6, NV_M8, NV_M12};
    const int rcodes[3] = {NV_M2R, NV_M3R, NV_M4R};
    for (int i = 0; i < 6; ++i)
        if (r.zM[i] <= zlo) return (rot1 && i < 3) ? rcodes[i] : codes[i];
    return NV_M12;
}

// relative cost per entry of each variant (VALU operations, measured from the
// compiled loops)
constexpr double NV_COST[NV_COUNT] = {0.9, 1.9, 1.7, 0.85, 0.9, 1.0, 1.1, 1.2, 1.35, 0.7, 1.7, 1.5,
                                      0.68, 0.73, 0.83, 1.4};

hank_status build_dev_plan(DevPlan& dp, hipStream_t s) {
    const Plan& p = dp.plan;
    const Grid& g = p.g;
    const int64_t N = g.N;
    dp.G = grid_args(g);
    dp.G.lean = (!p.direct && p.eps >= 1e-9) ? 1 : 0; // near budget eps/8 >= 1.25e-10
    hank_status st;
    if (g.col_pert || g.row_pert) {
        if ((st = dev_alloc(dp.b, size_t(N + 1), dp.bytes))) return st;
        if (g.row_pert && (st = dev_alloc(dp.v, size_t(N), dp.bytes))) return st;
        HIP_TRY(launch_roots(N + 1, dp.b, g.row_pert ? N : 0, dp.v, s));
    }
    if (g.row_pert) {
        if ((st = dev_alloc(dp.e, size_t(N), dp.bytes))) return st;
        HIP_TRY(launch_dht_e(N, dp.b, dp.e, s));
    }
    std::vector<double> nutab_host; // kept until the stream synchronisation below
    if (g.nu > 0) {
        // fewest Hankel pairs (valid for this order) whose remainder at the
        // switch z = 20 + nu/2 is within the near field's budget
        const double budget = p.direct ? 1e-17 : p.eps / 8.0, zsw = 20.0 + 0.5 * g.nu;
        for (int M = std::max(1, int(std::ceil(g.nu / 2.0 - 0.25))); M <= NU_HANKEL_PAIRS; ++M)
            if (rem_bound(g.nu, M, zsw) <= budget) {
                dp.mnu = M;
                break;
            }
        nutab_host.resize(NU_TAB_SIZE);
        build_nu_table(g.nu, nutab_host.data());
        if ((st = dev_alloc(dp.nutab, size_t(NU_TAB_SIZE), dp.bytes))) return st;
        HIP_TRY(hipMemcpyAsync(dp.nutab, nutab_host.data(), NU_TAB_SIZE * sizeof(double), hipMemcpyHostToDevice, s));
    }
    // near-field work items: partial slots in row order, so that a row
    // tile's slots are consecutive; the tiles themselves run longest first,
    // so that the short ones fill the tail of a launch
    std::vector<NearTile>& tiles = dp.tiles;
    std::vector<RowTile>& rts = dp.rts;
    const int64_t chunk = near_chunk(p.near);
    const NearRule rule = near_rule(p);
    for (auto& seg : p.near)
        for (int64_t k = seg.k0; k < seg.k1; k += 64) {
            RowTile r{};
            r.k0 = k;
            r.nk = int32_t(std::min<int64_t>(64, seg.k1 - k));
            r.slot0 = int64_t(tiles.size());
            for (int64_t n = 1; n < seg.ncut; n += chunk) {
                NearTile t{};
                t.k0 = k;
                t.nk = r.nk;
                t.n0 = n;
                t.n1 = std::min(seg.ncut, n + chunk);
                // k_near also evaluates the columns from n1 up to the next
                // multiple of 4 past n0 (with c = 0): the last block's variant
                // covers them too
                const int64_t n1p = t.n0 + ((t.n1 - t.n0 + 3) & ~int64_t(3));
                for (int64_t nb = t.n0, b = 0; nb < t.n1; nb += 64, ++b) {
                    const int v = near_block_variant(g, rule, t.k0, t.k0 + t.nk - 1, nb, std::min(nb + 63, n1p - 1));
                    t.bvar[b >> 3] |= uint32_t(v) << (4 * (b & 7));
                }
                t.slot = int64_t(tiles.size());
                tiles.push_back(t);
            }
            r.ntiles = int64_t(tiles.size()) - r.slot0;
            dp.rt_max_tiles = std::max(dp.rt_max_tiles, r.ntiles);
            if (r.ntiles == 1)
                tiles.back().sole = 1;
            else
                dp.rts_red.push_back(r);
            rts.push_back(r);
        }
    // relative cost of a tile: its 64-column blocks priced by their variant
    auto tile_cost = [&](const NearTile& T) {
        double c = 0;
        for (int64_t nb = T.n0, b = 0; nb < T.n1; nb += 64, ++b)
            c += double(std::min<int64_t>(64, T.n1 - nb)) * NV_COST[(T.bvar[b >> 3] >> (4 * (b & 7))) & 15];
        return c;
    };
    std::stable_sort(tiles.begin(), tiles.end(),
                     [&](const NearTile& a, const NearTile& b) { return tile_cost(a) > tile_cost(b); });
    if ((st = dev_alloc(dp.d_tiles, tiles.size(), dp.bytes))) return st;
    if ((st = dev_alloc(dp.d_rts, rts.size(), dp.bytes))) return st;
    if ((st = dev_alloc(dp.d_rts_red, dp.rts_red.size(), dp.bytes))) return st;
    if (!tiles.empty())
        HIP_TRY(hipMemcpyAsync(dp.d_tiles, tiles.data(), tiles.size() * sizeof(NearTile), hipMemcpyHostToDevice, s));
    if (!rts.empty())
        HIP_TRY(hipMemcpyAsync(dp.d_rts, rts.data(), rts.size() * sizeof(RowTile), hipMemcpyHostToDevice, s));
    if (!dp.rts_red.empty())
        HIP_TRY(hipMemcpyAsync(dp.d_rts_red, dp.rts_red.data(), dp.rts_red.size() * sizeof(RowTile),
                               hipMemcpyHostToDevice, s));

    // far-field blocks (the scratch only holds one chirp kernel at a time)
    size_t work_elems = 0;
    for (auto& hb : p.blocks) work_elems = std::max(work_elems, size_t(hb.L));
    if (!p.blocks.empty())
        if ((st = dev_alloc(reinterpret_cast<char*&>(dp.work), work_elems * 16, dp.bytes))) return st;
    std::vector<std::vector<GroupDev>> hg(p.blocks.size());
    std::vector<std::vector<TermDev>> ht(p.blocks.size());
    dp.blocks.resize(p.blocks.size());
    for (size_t i = 0; i < p.blocks.size(); ++i) {
        const Block& hb = p.blocks[i];
        DevBlock& d = dp.blocks[i];
        d.hb = hb;
        for (auto& G : hb.groups) hg[i].push_back(GroupDev{G.a, G.e, G.t0, G.t1, G.scale});
        for (auto& T : hb.terms) ht[i].push_back(TermDev{T.b, T.m, T.kre, T.kim});
        if ((st = dev_alloc(d.groups, hg[i].size(), dp.bytes))) return st;
        if ((st = dev_alloc(d.terms, ht[i].size(), dp.bytes))) return st;
        HIP_TRY(hipMemcpyAsync(d.groups, hg[i].data(), hg[i].size() * sizeof(GroupDev), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d.terms, ht[i].data(), ht[i].size() * sizeof(TermDev), hipMemcpyHostToDevice, s));
        const bool any64 = hb.g64 > 0, any32 = hb.g64 < int32_t(hb.groups.size());
        if (any64 && (st = dev_alloc(reinterpret_cast<char*&>(d.H), size_t(hb.L) * 16, dp.bytes))) return st;
        if (any32 && (st = dev_alloc(reinterpret_cast<char*&>(d.H32), size_t(hb.L) * 8, dp.bytes))) return st;
        FarArgs& A = d.args;
        A.ka = hb.ka;
        A.na = hb.na;
        A.nrows = hb.kb - hb.ka + 1;
        A.ncols = hb.nb - hb.na + 1;
        A.L = hb.L;
        A.L1 = hb.L1;
        A.L2 = hb.L2;
        int lg = 0;
        while ((int64_t(1) << lg) < hb.L) ++lg;
        A.twshift = 23 - lg;
        A.ngroups = int32_t(hb.groups.size());
        A.g0 = 0;
        A.g1 = A.ngroups;
        A.ar = g.ar;
        A.br = g.br;
        A.ac = g.ac;
        A.bc = g.bc;
        A.D = g.D;
        A.Dr = g.Dr;
        A.Qc = g.Qc;
        A.Kka = g.ar * hb.ka + g.br;
        A.Nna = g.ac * hb.na + g.bc;
        A.pi_Qc = dp.G.pi_Qc;
        A.r0 = hb.r0;
        A.w0 = hb.w0;
        A.eref = hb.eref;
        A.lref = hb.lref;
        A.bref = hb.bref;
        A.row_pert = g.row_pert;
        A.col_pert = g.col_pert;
        A.groups = d.groups;
        A.terms = d.terms;
        if (any64) HIP_TRY(launch_chirp_spectrum(A, false, dp.work, d.H, s));
        if (any32) HIP_TRY(launch_chirp_spectrum(A, true, dp.work, d.H32, s));
    }
    // the host vectors above must outlive the asynchronous copies
    HIP_TRY(hipStreamSynchronize(s));
    return HANK_OK;
}

// Right-hand sides a plan is balanced for: nrhs rounded up to a power of two
// (at most 64); plans are cached per bucket.
// Right-hand sides a plan is made for: 1 for order nu > 0 (its near field
// sums one right-hand side at a time) and for up to three right-hand sides,
// which run as that many single transforms (measured on Fourier-Bessel 2e4
// and Schlomilch 3e4 at 1e-8 and DHT 8192 at 1e-14: 2 right-hand sides 17-31%
// faster that way than on the several-right-hand-side MFMA kernel, 3 8-12%
// faster, 4 equal to 13% slower, 5 or more slower).
constexpr int64_t SINGLE_RHS_MAX = 3;
int64_t plan_nrhs(int64_t nrhs, int nu) { return (nu > 0 || nrhs <= SINGLE_RHS_MAX) ? 1 : nrhs; }

int64_t rhs_bucket(int64_t nrhs) {
    int64_t b = 1;
    while (b < nrhs && b < 64) b *= 2;
    return b;
}

Key plan_key(int task, int64_t N, double eps, const hank_options* o, int dev, int64_t nrhs) {
    int mode = o ? o->plan_mode : 0, prec = o ? o->precision : 0, direct = o ? o->direct : 0;
    int far = o ? o->prefer_far : 0;
    uint64_t eb;
    std::memcpy(&eb, &eps, 8);
    int M = o ? o->M : 0, nu = o ? o->nu : 0, shift = o ? o->shift : 0;
    nrhs = plan_nrhs(nrhs, nu);
    return Key{task, N, eb, mode + 4 * M + 128 * (nu + 16 * shift), prec,
               (direct * 2 + far) * 128 + int(rhs_bucket(nrhs)), dev};
}

hank_status get_plan(int task, int64_t N, double eps, const hank_options* o, hipStream_t s, DevPlan*& out,
                     int64_t nrhs = 1, const Plan* prebuilt = nullptr) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hank_status st = ensure_tables(dev);
    if (st) return st;
    int mode = o ? o->plan_mode : 0, prec = o ? o->precision : 0, direct = o ? o->direct : 0;
    Key key = plan_key(task, N, eps, o, dev, nrhs);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        out = it->second.get();
        out->last_use = ++g_use_clock;
        out->call = g_call;
        return HANK_OK;
    }
    std::unique_ptr<DevPlan> dp(new DevPlan);
    dp->device = dev;
    try {
        dp->plan = prebuilt ? *prebuilt
                            : make_plan(task, N, eps, mode, prec, direct != 0, cost_model_for(o),
                                        rhs_bucket(plan_nrhs(nrhs, o ? o->nu : 0)), o ? o->M : 0, o ? o->nu : 0,
                                        o ? o->shift : 0);
    } catch (const std::exception& ex) {
        return fail(HANK_EINVAL, std::string("planning failed: ") + ex.what());
    }
    st = build_dev_plan(*dp, s);
    if (st) return st; // dp's destructor frees what was allocated
    out = dp.get();
    out->last_use = ++g_use_clock;
    out->call = g_call;
    g_cache[key] = std::move(dp);
    // past the limit: down to three quarters of it, so that evictions (each a
    // device synchronisation) come in groups
    if (cache_total() > g_cache_limit) evict_to(g_cache_limit / 4 * 3);
    return HANK_OK;
}

// ---- optional per-kernel timing (hank_profile) ----
enum { K_NEAR = 0, K_NEAR_MULTI, K_NEAR_REDUCE, K_PASS_A, K_PASS_B, K_PASS_C, K_FAR_REDUCE, K_NEAR_NU, K_COUNT };
const char* const k_names[K_COUNT] = {"near",   "near_multi", "near_reduce", "pass_a",
                                      "pass_b", "pass_c",     "far_reduce",  "near_nu"};
struct Pending {
    int kind;
    hipEvent_t a, b;
    double bytes, work;
};
bool g_prof = false;
int g_graphs = 0; // live batch graphs (they hold pointers into cached plans)
std::vector<Pending> g_pending;
struct Acc {
    int64_t launches = 0;
    double ms = 0, bytes = 0, work = 0;
} g_acc[K_COUNT];

hank_status prof_begin(hipEvent_t& ev, hipStream_t s) {
    ev = nullptr;
    if (!g_prof) return HANK_OK;
    HIP_TRY(hipEventCreate(&ev));
    HIP_TRY(hipEventRecord(ev, s));
    return HANK_OK;
}

hank_status prof_end(int kind, hipEvent_t a, double bytes, double work, hipStream_t s) {
    if (!g_prof || !a) return HANK_OK;
    hipEvent_t b;
    HIP_TRY(hipEventCreate(&b));
    HIP_TRY(hipEventRecord(b, s));
    g_pending.push_back(Pending{kind, a, b, bytes, work});
    return HANK_OK;
}

hank_status prof_collect() {
    for (auto& p : g_pending) {
        HIP_TRY(hipEventSynchronize(p.b));
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, p.a, p.b));
        Acc& a = g_acc[p.kind];
        a.launches += 1;
        a.ms += ms;
        a.bytes += p.bytes;
        a.work += p.work;
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_pending.clear();
    return HANK_OK;
}

// ---- execution of a list of jobs ----
// A job is a plan applied to nrhs coefficient columns.  All jobs of one call
// share its launches: one near-field launch per kind over every job's tiles,
// one reduce, and the far field in waves by block index (blocks of one job
// overlap in rows, blocks of different jobs never share output), each wave
// split by FFT shape into one launch per pass.
struct Job {
    DevPlan* dp;
    const double* c;
    int64_t ldc;
    double* f;
    int64_t ldo;
    int64_t nrhs;
};

// Device buffers shared by all calls (grow-only), ordered across streams by
// an event recorded at the end of every call.
struct Scratch {
    void* p = nullptr;
    size_t bytes = 0;
};
// Host copies of uploaded descriptors stay alive until the stream has consumed
// them: a ring of slots, each reused only after its upload event completed.
struct UploadSlot {
    std::vector<NearProb> probs;
    std::vector<FarDesc> descs;
    hipEvent_t done = nullptr;
    bool pending = false;
};
struct Executor {
    Scratch probs, partial, descs, work, fpart;
    Scratch inv; // D_v f of the inverse DHT
    UploadSlot slots[4];
    int next_slot = 0;
    hipEvent_t done = nullptr;
    hipStream_t last = nullptr;
    bool used = false;
    // the last upload, so that a repeated identical call skips it
    std::vector<char> sig;
} g_ex;

hank_status ensure(Scratch& b, size_t bytes, hipStream_t s) {
    if (bytes <= b.bytes) return HANK_OK;
    if (b.p) {
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = std::max(bytes, size_t(4096));
    hipError_t e = hank_malloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? HANK_ENOMEM : HANK_EDEVICE,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    b.bytes = want;
    g_ex.sig.clear(); // contents are gone
    return HANK_OK;
}

// Workspace budget of one far-field wave (HANK_WAVE_MB, default 4096 MB).
size_t wave_budget() {
    static const size_t b = [] {
        const char* v = std::getenv("HANK_WAVE_MB");
        return size_t((v ? std::atof(v) : 4096.0) * 1048576.0);
    }();
    return b;
}

// Group chunks of a far-field block applied to nrhs right-hand sides: one
// (rhs, chunk) item is L/8 threads per pass, and enough items run side by side
// to give the chip about eight waves per compute unit (2048 waves).  A chunk
// keeps at least two groups so that the per-column set-up is shared.  The
// rule depends on the request alone, so a request sums in the same order
// inside any batch.
int32_t far_chunks(int64_t L, int32_t ngroups, int64_t nrhs) {
    const double target_threads = 2048.0 * 64.0;
    const double items = target_threads / (double(L) / 8.0);
    int64_t want = int64_t(std::ceil(items / double(nrhs)));
    want = std::min<int64_t>(want, (ngroups + 1) / 2);
    return int32_t(std::max<int64_t>(1, want));
}

// A launch set of the far field: descriptors [d0, d1) of one FFT shape and
// precision; a record with L1 = 0 separates waves.
struct FarLaunch {
    bool fp32;
    int32_t L1, L2;
    size_t d0, d1;       // descriptors [d0, d1)
    int64_t nac, nb, nr; // grid sizes of the column passes, pass B and the chunk reduction
    double bytesA, bytesB, bytesC, bytesR, work;
};

// Everything the launches of a list of jobs need, built on the host: near
// descriptors, far descriptors (buf and part as offsets into the work and
// chunk-sum buffers), launch sets and buffer sizes.
struct Prepared {
    std::vector<NearProb> probs; // single rhs order 0, then order nu > 0, then several rhs
    int32_t nsingle = 0, nnu = 0;
    int64_t pbase = 0, ntiles1 = 0, ntilesnu = 0, ntilesm = 0, nrts = 0;
    int64_t nrts1 = 0; // row tiles of the problems with one right-hand side (the first ones)
    int64_t nwv1 = 0;  // waves of their reduce
    double near_entries = 0, nu_entries = 0, multi_entries = 0;
    std::vector<FarDesc> descs;
    std::vector<FarLaunch> launches;
    size_t work_need = 0, part_need = 0;
};

void prepare_jobs(const std::vector<Job>& jobs_in, Prepared& PR, size_t budget = wave_budget()) {
    // the near-field kernels take at most 64 right-hand sides: split wider jobs
    // (order nu > 0: one right-hand side per job)
    std::vector<Job> jobs;
    for (const Job& J : jobs_in) {
        const int64_t w = plan_nrhs(J.nrhs, J.dp->plan.g.nu) == 1 ? 1 : 64;
        for (int64_t j0 = 0; j0 < J.nrhs; j0 += w) {
            Job P = J;
            P.c = J.c + j0 * J.ldc;
            P.f = J.f + j0 * J.ldo;
            P.nrhs = std::min<int64_t>(w, J.nrhs - j0);
            jobs.push_back(P);
        }
    }

    // ---------- near field descriptors: single right-hand side jobs first ----------
    auto near_class = [](const Job& J) { return J.dp->plan.g.nu > 0 ? 1 : (J.nrhs == 1 ? 0 : 2); };
    std::stable_sort(jobs.begin(), jobs.end(),
                     [&](const Job& x, const Job& y) { return near_class(x) < near_class(y); });
    auto& probs = PR.probs;
    int64_t &pbase = PR.pbase, &nrts = PR.nrts;
    for (size_t i = 0; i < jobs.size(); ++i) {
        const Job& J = jobs[i];
        NearProb P{};
        P.G = J.dp->G;
        P.c = J.c;
        P.b = J.dp->b;
        P.e = J.dp->e;
        P.f = J.f;
        P.tiles = J.dp->d_tiles;
        // k_near writes the rows of sole tiles itself: its problems reduce
        // only the other row tiles
        const bool own = near_class(J) == 0;
        P.rts = own ? J.dp->d_rts_red : J.dp->d_rts;
        const int64_t nrt = int64_t(own ? J.dp->rts_red.size() : J.dp->rts.size());
        P.ldc = J.ldc;
        P.ldo = J.ldo;
        P.nrhs = int32_t(J.nrhs);
        P.nu = J.dp->plan.g.nu;
        P.nutab = J.dp->nutab;
        P.mnu = J.dp->mnu;
        P.pbase = pbase;
        const int64_t nt = int64_t(J.dp->tiles.size());
        const int cls = near_class(J);
        int64_t& count = cls == 0 ? PR.ntiles1 : cls == 1 ? PR.ntilesnu : PR.ntilesm;
        P.tile_start = count;
        count += nt;
        P.rt_start = nrts;
        nrts += nrt;
        if (J.nrhs == 1) {
            PR.nrts1 = nrts;
            P.wpr = J.dp->rt_max_tiles > 4 ? 4 : 1;
            if (P.wpr == 4) PR.nwv1 = (PR.nwv1 + 3) & ~int64_t(3);
            P.wv_start = PR.nwv1;
            PR.nwv1 += nrt * P.wpr;
        } else {
            P.wpr = 1;
            P.wv_start = PR.nwv1; // after every wave of the reduce of single right-hand sides
        }
        pbase += nt * J.nrhs * 64;
        (cls == 0 ? PR.nsingle : PR.nnu) += cls < 2;
        (cls == 0 ? PR.near_entries : cls == 1 ? PR.nu_entries : PR.multi_entries) +=
            double(J.dp->plan.near_entries) * double(J.nrhs);
        probs.push_back(P);
    }

    // ---------- far field descriptors, by wave ----------
    size_t& part_need = PR.part_need;
    auto& descs = PR.descs;
    auto& launches = PR.launches;
    size_t maxblocks = 0;
    for (auto& J : jobs) maxblocks = std::max(maxblocks, J.dp->blocks.size());
    size_t& work_need = PR.work_need;
    for (size_t bi = 0; bi < maxblocks; ++bi) {
        // (job, group range) items of this wave
        struct Item {
            size_t job;
            int32_t g0, g1;
            bool f32;
        };
        std::vector<std::vector<Item>> sub(1);
        std::vector<size_t> subbytes(1, 0);
        for (size_t ji = 0; ji < jobs.size(); ++ji) {
            Job& J = jobs[ji];
            if (bi >= J.dp->blocks.size()) continue;
            const DevBlock& d = J.dp->blocks[bi];
            // the FP64 groups [0, g64) and the FP32 groups [g64, ngroups)
            const int32_t g64 = d.hb.g64, ng = d.args.ngroups;
            const int32_t lo[2] = {0, g64}, hi[2] = {g64, ng};
            for (int pr = 0; pr < 2; ++pr) {
                if (hi[pr] <= lo[pr]) continue;
                const size_t esz = pr ? 8 : 16;
                const int32_t cnt = hi[pr] - lo[pr];
                const size_t per_group = size_t(d.args.L) * esz * size_t(J.nrhs);
                size_t gb = std::max<size_t>(1, std::min<size_t>(size_t(cnt), budget / per_group));
                gb = std::min(gb, group_batch(size_t(d.args.L) * esz, size_t(cnt)));
                int si = 0;
                for (int32_t g0 = lo[pr]; g0 < hi[pr]; g0 += int32_t(gb), ++si) {
                    const int32_t g1 = std::min(hi[pr], g0 + int32_t(gb));
                    const size_t need = per_group * size_t(g1 - g0);
                    // group batches of one block and precision go to successive
                    // sub-waves (each pass C adds into f)
                    size_t k = size_t(si);
                    while (k < sub.size() && subbytes[k] + need > budget && subbytes[k] > 0) ++k;
                    if (k >= sub.size()) {
                        sub.emplace_back();
                        subbytes.push_back(0);
                        k = sub.size() - 1;
                    }
                    sub[k].push_back(Item{ji, g0, g1, pr == 1});
                    subbytes[k] += need;
                    si = int(k);
                }
            }
        }
        for (size_t k = 0; k < sub.size(); ++k) {
            if (sub[k].empty()) continue;
            // one launch set per FFT shape and precision
            std::map<std::tuple<bool, int32_t, int32_t>, std::vector<Item>> shapes;
            for (auto& it : sub[k]) {
                const Job& J = jobs[it.job];
                const DevBlock& d = J.dp->blocks[bi];
                shapes[{it.f32, d.args.L1, d.args.L2}].push_back(it);
            }
            size_t off = 0; // bytes within the work buffer for this sub-wave
            for (auto& kv : shapes) {
                FarLaunch Ln{};
                Ln.fp32 = std::get<0>(kv.first);
                Ln.L1 = std::get<1>(kv.first);
                Ln.L2 = std::get<2>(kv.first);
                const double esz = Ln.fp32 ? 8.0 : 16.0;
                Ln.d0 = descs.size();
                for (auto& it : kv.second) {
                    const Job& J = jobs[it.job];
                    const DevBlock& d = J.dp->blocks[bi];
                    FarDesc D{};
                    D.A = d.args;
                    D.A.g0 = it.g0;
                    D.A.g1 = it.g1;
                    D.c = J.c;
                    D.b = J.dp->b;
                    D.e = J.dp->e;
                    D.f = J.f;
                    D.H = it.f32 ? d.H32 : d.H;
                    D.ldc = J.ldc;
                    D.ldo = J.ldo;
                    D.nrhs = int32_t(J.nrhs);
                    const int32_t ng = it.g1 - it.g0;
                    D.nchunk = far_chunks(d.args.L, ng, J.nrhs);
                    D.gchunk = (ng + D.nchunk - 1) / D.nchunk;
                    D.nchunk = (ng + D.gchunk - 1) / D.gchunk;
                    D.buf = reinterpret_cast<void*>(off); // offsets, made absolute below
                    D.part = nullptr;
                    const double GL = double(ng) * double(J.nrhs) * double(d.args.L);
                    off += size_t(GL * esz);
                    const double cols = double(d.args.ncols), rws = double(d.args.nrows), nr = double(J.nrhs);
                    // a strip of at most L1 columns on the FP64 wave kernels hands pass B
                    // only its one nonzero input per column
                    const bool x0fused = !it.f32 && d.args.L1 == 4096 && (d.args.L2 == 256 || d.args.L2 == 512) &&
                                         d.args.ncols <= d.args.L1;
                    D.x0off = -1;
                    if (x0fused) {
                        D.x0off = int64_t(off);
                        off += size_t(double(ng) * nr * cols * esz);
                        off = (off + 255) & ~size_t(255);
                    }
                    // the work buffer columns j1 < ncols carry data (pass A -> pass B) and
                    // j1 < nrows results (pass B -> pass C); the others are not moved
                    const double L1 = double(d.args.L1);
                    const double fa = std::min(cols, L1) / L1, fc = std::min(rws, L1) / L1;
                    const double ain = x0fused ? double(ng) * nr * cols * esz : GL * esz * fa; // A -> B
                    Ln.bytesA += ain + cols * (8.0 * nr + (d.args.col_pert ? 8.0 : 0.0));
                    Ln.bytesB += ain + GL * esz * fc + double(d.args.L) * esz;
                    Ln.bytesC += GL * esz * fc + rws * (d.args.row_pert ? 8.0 : 0.0);
                    if (D.nchunk > 1) {
                        D.part = reinterpret_cast<double*>(part_need);
                        part_need += size_t(D.nchunk) * size_t(J.nrhs) * size_t(d.args.nrows) * sizeof(double);
                        Ln.bytesC += rws * nr * 8.0 * D.nchunk;
                        Ln.bytesR += rws * nr * 8.0 * (D.nchunk + 2.0);
                    } else {
                        Ln.bytesC += rws * nr * 16.0;
                    }
                    Ln.work += GL;
                    descs.push_back(D);
                }
                Ln.d1 = descs.size();
                const int32_t rows = far_rows_per_wg(Ln.L1);
                // pass B on the FP64 row kernel (L1 = 4096) holds two 512-thread
                // workgroups per compute unit; a launch with fewer (item, row)
                // pairs than that splits each pair's groups over bsplit
                // workgroups (pass B transforms the groups independently, so
                // the results do not change)
                // (HANK_PASSB_SPLIT=0, read per call, turns the split off)
                int32_t bsplit = 1;
                const char* split_env = std::getenv("HANK_PASSB_SPLIT");
                if (!Ln.fp32 && Ln.L1 == 4096 && !(split_env && std::atoi(split_env) == 0)) {
                    int64_t pairs = 0;
                    int32_t gmax = 1;
                    for (size_t di = Ln.d0; di < Ln.d1; ++di) {
                        const FarDesc& D = descs[di];
                        pairs += int64_t(D.nrhs) * D.nchunk * ((D.A.L2 + rows - 1) / rows);
                        gmax = std::max(gmax, D.gchunk);
                    }
                    const int64_t slots = 2 * 256;
                    if (pairs > 0 && pairs < slots)
                        bsplit = int32_t(std::min<int64_t>(gmax, (slots + pairs - 1) / pairs));
                }
                for (size_t di = Ln.d0; di < Ln.d1; ++di) {
                    FarDesc& D = descs[di];
                    const int64_t items = int64_t(D.nrhs) * D.nchunk;
                    D.wg_ac = Ln.nac;
                    Ln.nac += items * (D.A.L1 / col_width(D.A.L2, Ln.fp32));
                    D.bsplit = bsplit;
                    D.wg_b = Ln.nb;
                    Ln.nb += items * ((D.A.L2 + rows - 1) / rows) * bsplit;
                    D.wg_r = Ln.nr;
                    if (D.nchunk > 1) Ln.nr += int64_t(D.nrhs) * ((D.A.nrows + 255) / 256);
                }
                launches.push_back(Ln);
            }
            work_need = std::max(work_need, off);
            launches.push_back(FarLaunch{}); // sub-wave boundary
        }
    }
}

// The launches of prepared jobs on stream s, given the device copies of the
// descriptors and the partial-sum buffer.
hank_status enqueue_jobs(const Prepared& PR, const NearProb* dprobs, const FarDesc* ddesc, double* dpart,
                         hipStream_t s) {
    hank_status st;
    hipEvent_t ev;
    const int32_t nprob = int32_t(PR.probs.size());
    const int32_t nsingle = PR.nsingle, nnu = PR.nnu;
    const int64_t ntiles1 = PR.ntiles1, ntilesm = PR.ntilesm, nrts = PR.nrts, pbase = PR.pbase;
    if (ntiles1 > 0) {
        if ((st = prof_begin(ev, s))) return st;
        HIP_TRY(launch_near(dprobs, nsingle, ntiles1, dpart, s));
        if ((st = prof_end(K_NEAR, ev, 8.0 * 64.0 * double(ntiles1), PR.near_entries, s))) return st;
    }
    if (PR.ntilesnu > 0) {
        if ((st = prof_begin(ev, s))) return st;
        HIP_TRY(launch_near_nu(dprobs + nsingle, nnu, PR.ntilesnu, dpart, s));
        if ((st = prof_end(K_NEAR_NU, ev, 8.0 * 64.0 * double(PR.ntilesnu), PR.nu_entries, s))) return st;
    }
    if (ntilesm > 0) {
        if ((st = prof_begin(ev, s))) return st;
        HIP_TRY(launch_near_multi(dprobs + nsingle + nnu, nprob - nsingle - nnu, ntilesm, dpart, s));
        if ((st = prof_end(K_NEAR_MULTI, ev, 0.0, PR.multi_entries, s))) return st;
    }
    if ((st = prof_begin(ev, s))) return st;
    HIP_TRY(launch_near_reduce(dprobs, nprob, PR.nwv1, PR.nrts1, nrts, dpart, s));
    if ((st = prof_end(K_NEAR_REDUCE, ev, 8.0 * double(pbase), 0.0, s))) return st;

    for (auto& Ln : PR.launches) {
        if (Ln.L1 == 0) continue; // sub-wave boundary: the stream orders the waves
        const double bytes[3] = {Ln.bytesA, Ln.bytesB, Ln.bytesC};
        const int64_t grid[3] = {Ln.nac, Ln.nb, Ln.nac};
        const int32_t nd = int32_t(Ln.d1 - Ln.d0);
        for (int w = 0; w < 3; ++w) {
            if ((st = prof_begin(ev, s))) return st;
            HIP_TRY(launch_far_pass(w, Ln.fp32, Ln.L1, Ln.L2, ddesc + Ln.d0, nd, grid[w], s));
            if ((st = prof_end(K_PASS_A + w, ev, bytes[w], Ln.work, s))) return st;
        }
        if (Ln.nr > 0) {
            if ((st = prof_begin(ev, s))) return st;
            HIP_TRY(launch_far_reduce(ddesc + Ln.d0, nd, Ln.nr, s));
            if ((st = prof_end(K_FAR_REDUCE, ev, Ln.bytesR, 0.0, s))) return st;
        }
    }
    return HANK_OK;
}

// Copy the near and far descriptors of PR to dprobs and ddescs on stream s.
// The host copies live in a ring of four slots, each reused only after the
// copy that read it has completed.
hank_status upload_descriptors(const Prepared& PR, void* dprobs, void* ddescs, hipStream_t s) {
    UploadSlot& u = g_ex.slots[g_ex.next_slot];
    g_ex.next_slot = (g_ex.next_slot + 1) % 4;
    if (!u.done) HIP_TRY(hipEventCreateWithFlags(&u.done, hipEventDisableTiming));
    if (u.pending) HIP_TRY(hipEventSynchronize(u.done));
    u.probs = PR.probs;
    u.descs = PR.descs;
    if (!u.probs.empty())
        HIP_TRY(hipMemcpyAsync(dprobs, u.probs.data(), u.probs.size() * sizeof(NearProb), hipMemcpyHostToDevice, s));
    if (!u.descs.empty())
        HIP_TRY(hipMemcpyAsync(ddescs, u.descs.data(), u.descs.size() * sizeof(FarDesc), hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(u.done, s));
    u.pending = true;
    return HANK_OK;
}

hank_status run_jobs(std::vector<Job>& jobs_in, hipStream_t s) {
    hank_status st;
    Prepared PR;
    prepare_jobs(jobs_in, PR);
    if (!g_ex.done) HIP_TRY(hipEventCreateWithFlags(&g_ex.done, hipEventDisableTiming));
    if (g_ex.used && g_ex.last != s) HIP_TRY(hipStreamWaitEvent(s, g_ex.done, 0));

    // ---------- uploads (skipped when identical to the previous call) ----------
    if ((st = ensure(g_ex.work, PR.work_need, s))) return st;
    if ((st = ensure(g_ex.fpart, std::max<size_t>(PR.part_need, 8), s))) return st;
    for (auto& D : PR.descs) {
        D.x0 = D.x0off >= 0 ? static_cast<char*>(g_ex.work.p) + D.x0off : nullptr;
        D.buf = static_cast<char*>(g_ex.work.p) + reinterpret_cast<size_t>(D.buf);
        if (D.nchunk > 1)
            D.part = reinterpret_cast<double*>(static_cast<char*>(g_ex.fpart.p) + reinterpret_cast<size_t>(D.part));
    }
    if ((st = ensure(g_ex.partial, size_t(std::max<int64_t>(PR.pbase, 1)) * sizeof(double), s))) return st;
    std::vector<char> sig;
    auto add = [&](const void* p, size_t n) {
        const char* q = static_cast<const char*>(p);
        sig.insert(sig.end(), q, q + n);
    };
    add(PR.probs.data(), PR.probs.size() * sizeof(NearProb));
    add(PR.descs.data(), PR.descs.size() * sizeof(FarDesc));
    if (sig != g_ex.sig) {
        if ((st = ensure(g_ex.probs, PR.probs.size() * sizeof(NearProb), s))) return st;
        if ((st = ensure(g_ex.descs, PR.descs.size() * sizeof(FarDesc), s))) return st;
        if ((st = upload_descriptors(PR, g_ex.probs.p, g_ex.descs.p, s))) return st;
        g_ex.sig.swap(sig);
    }
    const NearProb* dprobs = static_cast<const NearProb*>(g_ex.probs.p);
    double* dpart = static_cast<double*>(g_ex.partial.p);

    const FarDesc* ddesc = static_cast<const FarDesc*>(g_ex.descs.p);
    if ((st = enqueue_jobs(PR, dprobs, ddesc, dpart, s))) return st;
    HIP_TRY(hipEventRecord(g_ex.done, s));
    g_ex.last = s;
    g_ex.used = true;
    return HANK_OK;
}

bool valid_task(int task) { return task >= 0 && task <= 4; }

hank_status check_args(int32_t task, const double* c, int64_t N, int64_t nrhs, int64_t ldc, double eps,
                       const double* out, int64_t ldo) {
    if (!valid_task(task)) return fail(HANK_EINVAL, "unknown task");
    if (!c || !out) return fail(HANK_EINVAL, "null pointer");
    int64_t nmin = (task == HANK_TASK_SCHLOMILCH || task == HANK_TASK_FOURIER_BESSEL) ? 2 : 1;
    if (N < nmin || N > (int64_t(1) << 24)) return fail(HANK_EINVAL, "N out of range");
    if (nrhs < 1 || ldc < N || ldo < N) return fail(HANK_EINVAL, "nrhs/ldc/ldo out of range");
    if (!std::isfinite(eps) || eps < 1e-15 || eps >= 1.0) return fail(HANK_EINVAL, "eps must lie in [1e-15, 1)");
    uintptr_t c0 = uintptr_t(c), c1 = uintptr_t(c + (nrhs - 1) * ldc + N);
    uintptr_t o0 = uintptr_t(out), o1 = uintptr_t(out + (nrhs - 1) * ldo + N);
    if (c0 < o1 && o0 < c1) return fail(HANK_EINVAL, "out overlaps c");
    return HANK_OK;
}

hank_status transform(int32_t task, const double* c, int64_t N, int64_t nrhs, int64_t ldc, double eps,
                      double* out, int64_t ldo, const hank_options* o, hank_stream_t stream) {
    hank_status st = check_args(task, c, N, nrhs, ldc, eps, out, ldo);
    if (st) return st;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    ++g_call;
    hipStream_t s = (hipStream_t)stream;
    DevPlan* dp = nullptr;
    if ((st = get_plan(task, N, eps, o, s, dp, nrhs))) return st;
    std::vector<Job> jobs{Job{dp, c, ldc, out, ldo, nrhs}};
    return run_jobs(jobs, s);
}

// Device bytes a request occupies while in flight: the far-field workspace
// of its largest block plus its near-field partials.
int64_t request_bytes(const DevPlan& dp, int64_t nrhs) {
    double far = 0;
    for (auto& b : dp.blocks) {
        const double per = 16.0 * double(b.hb.g64) + 8.0 * double(b.args.ngroups - b.hb.g64);
        far = std::max(far, double(b.args.L) * per * double(nrhs));
    }
    return int64_t(far + double(dp.tiles.size()) * 64.0 * 8.0 * double(nrhs));
}

} // namespace

// ---------------------------------------------------------------------------
// Continuous-batching server
// ---------------------------------------------------------------------------
// Requests arrive at their arrival time into a queue (or are rejected when
// max_pending wait already).  Planner threads build the plans of arrived
// requests (host planning and device tables on their own streams, outside the
// library lock), so planning overlaps the batches running on the GPU; a
// request whose plan is ready is pinned in the cache until its batch retires.
// The worker admits ready requests in arrival order into batches of at most
// max_batch requests and about one time slice of modelled GPU work, within
// the device-byte budget (workspace and plan of each request in flight), and
// keeps up to two batches in flight on its stream.
struct hank_server {
    using clock = std::chrono::steady_clock;
    struct Rec {
        hank_request req;
        double arrival = 0; // seconds after start
        double done = -1;
        int32_t state = 0;  // 0 waiting, 1 admitted, 2 done, 3 rejected
        int32_t pstate = 0; // plan: 0 not asked for, 1 queued or building, 2 ready (pinned), 3 failed
        DevPlan* dp = nullptr;
        int64_t bytes = 0; // device bytes while in flight: workspace and plan
        double est = 0;    // modelled GPU seconds (the planner's cost model)
    };
    struct Batch {
        std::vector<int64_t> tickets;
        hipEvent_t ev = nullptr;
        int64_t bytes = 0;
    };
    int64_t budget = 0, max_pending = 0;
    int32_t max_batch = 1;
    // modelled GPU time per batch (HANK_SERVE_SLICE_MS, default 4 ms)
    double slice_s = [] {
        const char* e = std::getenv("HANK_SERVE_SLICE_MS");
        return (e ? std::atof(e) : 4.0) * 1e-3;
    }();
    // planner threads (HANK_SERVE_PLANNERS, default min(8, cores / 2))
    int nplanners = [] {
        const char* e = std::getenv("HANK_SERVE_PLANNERS");
        const int hw = int(std::max(2u, std::thread::hardware_concurrency()));
        return std::max(1, e ? std::atoi(e) : std::min(8, hw / 2));
    }();
    hipStream_t stream = nullptr;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv, pcv;
    std::vector<Rec> recs;
    std::vector<int64_t> order; // tickets sorted by arrival (built at start)
    size_t next_arrival = 0;    // index into order of the next not-yet-arrived request
    std::deque<int64_t> waiting;
    std::deque<int64_t> plan_queue;              // arrived tickets whose plan is wanted
    std::map<Key, std::vector<int64_t>> building; // plans being built -> tickets waiting for them
    std::deque<Batch> inflight;
    int64_t inflight_bytes = 0;
    int admitting = 0; // batches taken from the queue but not yet in flight
    int64_t batches = 0, batched = 0, plans_built = 0;
    bool started = false, stop = false, stop_planners = false;
    clock::time_point t0;
    std::thread worker;
    std::vector<std::thread> planners;
    hank_status error = HANK_OK;
    std::string error_msg;

    double now() const { return std::chrono::duration<double>(clock::now() - t0).count(); }

    static hank_options options_of(const hank_request& r) {
        hank_options o{};
        o.precision = r.precision;
        o.nu = r.nu;
        o.shift = r.shift;
        return o;
    }

    // request tk has its plan dp (pinned for it); caller holds mu and g_mu
    void plan_ready(int64_t tk, DevPlan* dp) {
        Rec& r = recs[size_t(tk)];
        r.dp = dp;
        r.pstate = 2;
        r.bytes = request_bytes(*dp, r.req.nrhs) + int64_t(dp->bytes);
        r.est = dp->plan.cost * double(r.req.nrhs) / double(std::max<int64_t>(1, dp->plan.nrhs));
    }

    // release the pin of a request's plan; caller holds mu
    void unpin(Rec& r) {
        if (r.pstate != 2 || !r.dp) return;
        std::lock_guard<std::recursive_mutex> g(g_mu);
        --r.dp->pins;
        r.dp = nullptr;
        r.pstate = 0;
    }

    void plan_loop() {
        (void)hipSetDevice(device);
        hipStream_t ps = nullptr;
        if (hipStreamCreateWithFlags(&ps, hipStreamNonBlocking) != hipSuccess) ps = nullptr;
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            if (plan_queue.empty()) {
                if (stop_planners) break;
                pcv.wait(lk);
                continue;
            }
            const int64_t tk = plan_queue.front();
            plan_queue.pop_front();
            const hank_request req = recs[size_t(tk)].req;
            const hank_options o = options_of(req);
            const Key key = plan_key(req.task, req.N, req.eps, &o, device, req.nrhs);
            {
                std::lock_guard<std::recursive_mutex> g(g_mu);
                auto it = g_cache.find(key);
                if (it != g_cache.end()) {
                    DevPlan* dp = it->second.get();
                    ++dp->pins;
                    dp->last_use = ++g_use_clock;
                    plan_ready(tk, dp);
                    cv.notify_all();
                    continue;
                }
            }
            auto b = building.find(key);
            if (b != building.end()) {
                b->second.push_back(tk);
                continue;
            }
            building[key] = std::vector<int64_t>{tk};
            lk.unlock();
            // host planning and device tables, outside both locks
            std::unique_ptr<DevPlan> np(new DevPlan);
            np->device = device;
            hank_status st = HANK_OK;
            std::string msg;
            try {
                np->plan = make_plan(req.task, req.N, req.eps, 0, req.precision, false, cost_model_for(&o),
                                     rhs_bucket(plan_nrhs(req.nrhs, req.nu)), 0, req.nu, req.shift);
            } catch (const std::exception& ex) {
                st = HANK_EINVAL;
                msg = std::string("planning failed: ") + ex.what();
            }
            if (!st && !ps) st = HANK_EDEVICE, msg = "planner stream";
            if (!st && (st = build_dev_plan(*np, ps))) msg = hank_last_error();
            lk.lock();
            std::vector<int64_t> tickets;
            tickets.swap(building[key]);
            building.erase(key);
            {
                std::lock_guard<std::recursive_mutex> g(g_mu);
                DevPlan* dp = nullptr;
                auto it = g_cache.find(key);
                if (it != g_cache.end()) {
                    dp = it->second.get(); // built meanwhile by another caller
                } else if (!st) {
                    dp = np.get();
                    g_cache[key] = std::move(np);
                    ++plans_built;
                }
                if (dp) {
                    dp->last_use = ++g_use_clock;
                    dp->pins += int32_t(tickets.size());
                    for (int64_t t : tickets) plan_ready(t, dp);
                    if (cache_total() > g_cache_limit) evict_to(g_cache_limit / 4 * 3);
                } else {
                    for (int64_t t : tickets) recs[size_t(t)].pstate = 3;
                    error = st;
                    error_msg = msg;
                }
            }
            cv.notify_all();
        }
        lk.unlock();
        if (ps) (void)hipStreamDestroy(ps);
    }

    void run() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            if (!started) {
                if (stop) break;
                cv.wait(lk);
                continue;
            }
            const double t = now();
            // arrivals: into the queue (their plans wanted), or rejected when it is full
            bool asked = false;
            while (next_arrival < order.size() && recs[size_t(order[next_arrival])].arrival <= t) {
                const int64_t tk = order[next_arrival];
                Rec& r = recs[size_t(tk)];
                if (int64_t(waiting.size()) >= max_pending) {
                    r.state = 3;
                } else {
                    waiting.push_back(tk);
                    r.pstate = 1;
                    plan_queue.push_back(tk);
                    asked = true;
                }
                ++next_arrival;
            }
            if (asked) pcv.notify_all();
            // retire finished batches
            while (!inflight.empty() && hipEventQuery(inflight.front().ev) == hipSuccess) {
                const double td = now();
                for (int64_t tk : inflight.front().tickets) {
                    Rec& r = recs[size_t(tk)];
                    r.state = 2;
                    r.done = td;
                    unpin(r);
                }
                inflight_bytes -= inflight.front().bytes;
                (void)hipEventDestroy(inflight.front().ev);
                inflight.pop_front();
                cv.notify_all();
            }
            // admit a batch: ready requests in arrival order
            if (inflight.size() < 2 && !waiting.empty()) {
                Batch b;
                std::vector<hank_request> reqs;
                double est = 0;
                std::deque<int64_t> keep;
                bool full = false;
                for (int64_t tk : waiting) {
                    Rec& r = recs[size_t(tk)];
                    if (full || r.pstate == 1) {
                        keep.push_back(tk);
                        continue;
                    }
                    if (r.pstate == 3) { // its plan could not be built
                        r.state = 3;
                        continue;
                    }
                    if (r.bytes > budget) { // can never run within the budget
                        r.state = 3;
                        unpin(r);
                        continue;
                    }
                    const bool fits = b.tickets.empty() ? (inflight_bytes == 0 || inflight_bytes + r.bytes <= budget)
                                                        : (inflight_bytes + b.bytes + r.bytes <= budget &&
                                                           est + r.est <= slice_s); // about one time slice
                    if (!fits) {
                        keep.push_back(tk);
                        full = true;
                        continue;
                    }
                    b.tickets.push_back(tk);
                    b.bytes += r.bytes;
                    est += r.est;
                    r.state = 1;
                    reqs.push_back(r.req);
                    if (int32_t(b.tickets.size()) >= max_batch) full = true;
                }
                waiting.swap(keep);
                if (!b.tickets.empty()) {
                    ++admitting;
                    lk.unlock();
                    hank_status st = hank_batch(reqs.data(), int64_t(reqs.size()), stream);
                    if (st == HANK_OK && hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) == hipSuccess &&
                        hipEventRecord(b.ev, stream) == hipSuccess) {
                        lk.lock();
                        --admitting;
                        inflight_bytes += b.bytes;
                        inflight.push_back(b);
                        ++batches;
                        batched += int64_t(b.tickets.size());
                    } else {
                        lk.lock();
                        --admitting;
                        error = st ? st : HANK_EDEVICE;
                        error_msg = hank_last_error();
                        for (int64_t tk : b.tickets) {
                            recs[size_t(tk)].state = 3;
                            unpin(recs[size_t(tk)]);
                        }
                        cv.notify_all();
                    }
                    continue;
                }
            }
            const bool all_arrived = next_arrival >= order.size();
            if (stop && all_arrived && waiting.empty() && inflight.empty()) break;
            if (all_arrived && waiting.empty() && inflight.empty()) {
                cv.notify_all();
                cv.wait_for(lk, std::chrono::milliseconds(1));
                continue;
            }
            // short wait: the next arrival, a plan or a batch completing
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
        (void)hipSetDevice(cur);
    }
};

extern "C" {

hank_status hank_server_create(int64_t budget_bytes, int32_t max_batch, int64_t max_pending, hank_stream_t stream,
                               hank_server** out) {
    if (!out || budget_bytes <= 0 || max_batch < 1 || max_pending < 1) return fail(HANK_EINVAL, "bad server arguments");
    hank_server* s = new hank_server;
    s->budget = budget_bytes;
    s->max_batch = max_batch;
    s->max_pending = max_pending;
    s->stream = (hipStream_t)stream;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(HANK_EDEVICE, "hipGetDevice failed");
    }
    {
        std::lock_guard<std::recursive_mutex> lk(g_mu);
        hank_status st = ensure_tables(s->device);
        if (st) {
            delete s;
            return st;
        }
    }
    s->worker = std::thread([s] { s->run(); });
    for (int i = 0; i < s->nplanners; ++i) s->planners.emplace_back([s] { s->plan_loop(); });
    *out = s;
    return HANK_OK;
}

hank_status hank_server_warm(hank_server* srv, const hank_request* r) {
    if (!srv || !r) return fail(HANK_EINVAL, "null pointer");
    hank_status st = check_args(r->task, r->c, r->N, r->nrhs, r->ldc, r->eps, r->out, r->ldo);
    if (st) return st;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    ++g_call;
    hank_options o = hank_server::options_of(*r);
    DevPlan* dp = nullptr;
    return get_plan(r->task, r->N, r->eps, &o, srv->stream, dp, r->nrhs);
}

hank_status hank_server_submit(hank_server* srv, const hank_request* r, double arrival_s, int64_t* ticket) {
    if (!srv || !r || !ticket) return fail(HANK_EINVAL, "null pointer");
    hank_status st = check_args(r->task, r->c, r->N, r->nrhs, r->ldc, r->eps, r->out, r->ldo);
    if (st) return st;
    hank_options o = hank_server::options_of(*r);
    if (o.nu < 0 || o.nu > HANK_NU_MAX || o.shift < 0 || o.shift > HANK_SHIFT_MAX ||
        (o.nu > 0 && r->task == HANK_TASK_DHT0) || (o.shift > 0 && r->task != HANK_TASK_SCHLOMILCH &&
                                                     r->task != HANK_TASK_SCHLOMILCH_PAPER_GRID) ||
        r->precision < 0 || r->precision > 2)
        return fail(HANK_EINVAL, "request options out of range");
    std::lock_guard<std::mutex> lk(srv->mu);
    hank_server::Rec rec;
    rec.req = *r;
    rec.arrival = (arrival_s < 0 && srv->started) ? srv->now() : std::max(0.0, arrival_s);
    *ticket = int64_t(srv->recs.size());
    srv->recs.push_back(rec);
    if (srv->started) { // keep `order` sorted by arrival for the not-yet-arrived part
        auto pos = std::upper_bound(srv->order.begin() + long(srv->next_arrival), srv->order.end(), rec.arrival,
                                    [&](double a, int64_t t) { return a < srv->recs[size_t(t)].arrival; });
        srv->order.insert(pos, *ticket);
    }
    srv->cv.notify_all();
    return HANK_OK;
}

hank_status hank_server_start(hank_server* srv) {
    if (!srv) return fail(HANK_EINVAL, "null pointer");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->started) return HANK_OK;
    srv->order.resize(srv->recs.size());
    for (size_t i = 0; i < srv->order.size(); ++i) srv->order[i] = int64_t(i);
    std::stable_sort(srv->order.begin(), srv->order.end(),
                     [&](int64_t a, int64_t b) { return srv->recs[size_t(a)].arrival < srv->recs[size_t(b)].arrival; });
    srv->t0 = hank_server::clock::now();
    srv->started = true;
    srv->cv.notify_all();
    return HANK_OK;
}

hank_status hank_server_drain(hank_server* srv) {
    if (!srv) return fail(HANK_EINVAL, "null pointer");
    std::unique_lock<std::mutex> lk(srv->mu);
    if (!srv->started) return fail(HANK_EINVAL, "server not started");
    srv->cv.wait(lk, [&] {
        return srv->next_arrival >= srv->order.size() && srv->waiting.empty() && srv->inflight.empty() &&
               srv->admitting == 0;
    });
    if (srv->error) return fail(srv->error, srv->error_msg);
    return HANK_OK;
}

hank_status hank_server_status(hank_server* srv, int64_t ticket, int32_t* state, double* latency_ms) {
    if (!srv || !state) return fail(HANK_EINVAL, "null pointer");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (ticket < 0 || ticket >= int64_t(srv->recs.size())) return fail(HANK_EINVAL, "unknown ticket");
    const hank_server::Rec& r = srv->recs[size_t(ticket)];
    *state = r.state;
    if (latency_ms) *latency_ms = r.state == 2 ? 1e3 * (r.done - r.arrival) : -1.0;
    return HANK_OK;
}

hank_status hank_server_stats(hank_server* srv, hank_server_summary* out) {
    if (!srv || !out) return fail(HANK_EINVAL, "null pointer");
    std::lock_guard<std::mutex> lk(srv->mu);
    hank_server_summary st{};
    std::vector<double> lat;
    double first = 1e300, last = 0;
    for (auto& r : srv->recs) {
        ++st.submitted;
        first = std::min(first, r.arrival);
        if (r.state == 3) ++st.rejected;
        if (r.state == 2) {
            lat.push_back(1e3 * (r.done - r.arrival));
            last = std::max(last, r.done);
        }
    }
    st.completed = int64_t(lat.size());
    st.batches = srv->batches;
    st.mean_batch = srv->batches ? double(srv->batched) / double(srv->batches) : 0.0;
    st.plans_built = srv->plans_built;
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double q) { return lat[std::min(lat.size() - 1, size_t(q * double(lat.size() - 1) + 0.5))]; };
        st.p50_ms = pct(0.50);
        st.p90_ms = pct(0.90);
        st.p99_ms = pct(0.99);
        st.max_ms = lat.back();
        double sum = 0;
        for (double v : lat) sum += v;
        st.mean_ms = sum / double(lat.size());
        st.wall_s = last - first;
        st.throughput = st.wall_s > 0 ? double(st.completed) / st.wall_s : 0.0;
    }
    *out = st;
    return HANK_OK;
}

hank_status hank_server_destroy(hank_server* srv) {
    if (!srv) return fail(HANK_EINVAL, "null pointer");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        if (!srv->started) {
            srv->started = true; // let the worker drain nothing and exit
            srv->t0 = hank_server::clock::now();
        }
        srv->cv.notify_all();
    }
    srv->worker.join();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop_planners = true;
        srv->plan_queue.clear();
        srv->pcv.notify_all();
    }
    for (auto& t : srv->planners) t.join();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (auto& r : srv->recs) srv->unpin(r); // requests that never ran
    }
    delete srv;
    return HANK_OK;
}

} // extern "C"

extern "C" {

hank_status hank_schlomilch(const double* c, int64_t N, double eps, double* out, hank_stream_t stream) {
    return transform(HANK_TASK_SCHLOMILCH, c, N, 1, N, eps, out, N, nullptr, stream);
}

hank_status hank_fourier_bessel(const double* c, int64_t N, double eps, double* out, hank_stream_t stream) {
    return transform(HANK_TASK_FOURIER_BESSEL, c, N, 1, N, eps, out, N, nullptr, stream);
}

hank_status hank_dht0(const double* c, int64_t N, double eps, double* out, hank_stream_t stream) {
    return transform(HANK_TASK_DHT0, c, N, 1, N, eps, out, N, nullptr, stream);
}

hank_status hank_dht0_inverse(const double* f, int64_t N, double eps, double* c, hank_stream_t stream) {
    hank_status st = check_args(HANK_TASK_DHT0, f, N, 1, N, eps, c, N);
    if (st) return st;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    ++g_call;
    hipStream_t s = (hipStream_t)stream;
    DevPlan* dp = nullptr;
    if ((st = get_plan(HANK_TASK_DHT0, N, eps, nullptr, s, dp, 1))) return st;
    if (!g_ex.done) HIP_TRY(hipEventCreateWithFlags(&g_ex.done, hipEventDisableTiming));
    if (g_ex.used && g_ex.last != s) HIP_TRY(hipStreamWaitEvent(s, g_ex.done, 0));
    if ((st = ensure(g_ex.inv, size_t(N) * sizeof(double), s))) return st;
    double* w = static_cast<double*>(g_ex.inv.p);
    HIP_TRY(launch_dht_scale(N, dp->v, dp->b, f, w, false, s)); // D_v f
    std::vector<Job> jobs{Job{dp, w, N, c, N, 1}};
    if ((st = run_jobs(jobs, s))) return st;                   // J_0(...) D_v f
    HIP_TRY(launch_dht_scale(N, dp->v, dp->b, c, c, true, s)); // D_v ... / j_{0,N+1}^2
    HIP_TRY(hipEventRecord(g_ex.done, s));
    return HANK_OK;
}

hank_status hank_dht0_weights(int64_t N, double* v, hank_stream_t stream) {
    if (!v || N < 1) return fail(HANK_EINVAL, "bad arguments");
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hank_status st = ensure_tables(dev);
    if (st) return st;
    HIP_TRY(launch_roots(N, nullptr, N, v, (hipStream_t)stream));
    return HANK_OK;
}

hank_status hank_transform(int32_t task, const double* c, int64_t N, int64_t nrhs, int64_t ldc, double eps,
                           double* out, int64_t ldo, const hank_options* options, hank_stream_t stream) {
    return transform(task, c, N, nrhs, ldc, eps, out, ldo, options, stream);
}

// Checks a request list and turns it into jobs (plans built as needed, on s).
static hank_status batch_jobs(const hank_request* reqs, int64_t count, hipStream_t s, std::vector<Job>& jobs) {
    if (count < 0 || (count > 0 && !reqs)) return fail(HANK_EINVAL, "bad request list");
    for (int64_t i = 0; i < count; ++i) {
        const hank_request& r = reqs[i];
        hank_status st = check_args(r.task, r.c, r.N, r.nrhs, r.ldc, r.eps, r.out, r.ldo);
        if (st) return fail(st, "request " + std::to_string(i) + ": " + t_err);
        for (int64_t j = 0; j < i; ++j) { // outputs must not overlap each other
            const hank_request& q = reqs[j];
            uintptr_t a0 = uintptr_t(r.out), a1 = uintptr_t(r.out + (r.nrhs - 1) * r.ldo + r.N);
            uintptr_t b0 = uintptr_t(q.out), b1 = uintptr_t(q.out + (q.nrhs - 1) * q.ldo + q.N);
            if (a0 < b1 && b0 < a1) return fail(HANK_EINVAL, "request " + std::to_string(i) + ": output overlaps request " + std::to_string(j));
            uintptr_t c0 = uintptr_t(q.c), c1 = uintptr_t(q.c + (q.nrhs - 1) * q.ldc + q.N);
            uintptr_t d0 = uintptr_t(r.c), d1 = uintptr_t(r.c + (r.nrhs - 1) * r.ldc + r.N);
            if ((a0 < c1 && c0 < a1) || (b0 < d1 && d0 < b1))
                return fail(HANK_EINVAL, "requests " + std::to_string(j) + " and " + std::to_string(i) + ": an output overlaps an input");
        }
    }
    if (count == 0) return HANK_OK;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    // host planning of the keys not cached yet, in parallel threads
    std::map<Key, std::pair<int64_t, Plan>> fresh;
    for (int64_t i = 0; i < count; ++i) {
        hank_options o{};
        o.precision = reqs[i].precision;
        o.nu = reqs[i].nu;
        o.shift = reqs[i].shift;
        Key k = plan_key(reqs[i].task, reqs[i].N, reqs[i].eps, &o, dev, reqs[i].nrhs);
        if (!g_cache.count(k) && !fresh.count(k)) fresh[k] = {i, Plan()};
    }
    if (fresh.size() > 1) {
        std::vector<std::pair<const Key, std::pair<int64_t, Plan>>*> todo;
        for (auto& kv : fresh) todo.push_back(&kv);
        std::atomic<size_t> next{0};
        std::atomic<bool> bad{false};
        auto worker = [&]() {
            for (size_t t; (t = next++) < todo.size();) {
                const hank_request& r = reqs[todo[t]->second.first];
                hank_options o{};
                o.precision = r.precision;
                o.nu = r.nu;
                o.shift = r.shift;
                try {
                    todo[t]->second.second = make_plan(r.task, r.N, r.eps, 0, r.precision, false, cost_model_for(&o),
                                                       rhs_bucket(plan_nrhs(r.nrhs, r.nu)), 0, r.nu, r.shift);
                } catch (...) {
                    bad = true;
                }
            }
        };
        unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (unsigned i = 0; i < nt; ++i) th.emplace_back(worker);
        for (auto& t : th) t.join();
        if (bad) return fail(HANK_EINVAL, "planning failed for a request");
    }
    jobs.clear();
    for (int64_t i = 0; i < count; ++i) {
        const hank_request& r = reqs[i];
        hank_options o{};
        o.precision = r.precision;
        o.nu = r.nu;
        o.shift = r.shift;
        DevPlan* dp = nullptr;
        auto it = fresh.find(plan_key(r.task, r.N, r.eps, &o, dev, r.nrhs));
        const Plan* pre = (fresh.size() > 1 && it != fresh.end()) ? &it->second.second : nullptr;
        hank_status st = get_plan(r.task, r.N, r.eps, &o, s, dp, r.nrhs, pre);
        if (st) return st;
        jobs.push_back(Job{dp, r.c, r.ldc, r.out, r.ldo, r.nrhs});
    }
    return HANK_OK;
}

hank_status hank_batch(const hank_request* reqs, int64_t count, hank_stream_t stream) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    ++g_call;
    hipStream_t s = (hipStream_t)stream;
    std::vector<Job> jobs;
    hank_status st = batch_jobs(reqs, count, s, jobs);
    if (st || jobs.empty()) return st;
    return run_jobs(jobs, s);
}

// ---- a batch captured as a HIP graph ----
struct hank_graph {
    int device = 0;
    std::vector<DevPlan*> plans; // pinned while the graph exists
    void *work = nullptr, *fpart = nullptr, *partial = nullptr, *probs = nullptr, *descs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~hank_graph() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (void* p : {work, fpart, partial, probs, descs})
            if (p) (void)hipFree(p);
        (void)hipSetDevice(cur);
    }
};

hank_status hank_batch_graph_create(const hank_request* reqs, int64_t count, hank_stream_t stream,
                                    hank_graph** out) {
    if (!out) return fail(HANK_EINVAL, "null pointer");
    *out = nullptr;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    ++g_call;
    hipStream_t s = (hipStream_t)stream;
    std::vector<Job> jobs;
    hank_status st = batch_jobs(reqs, count, s, jobs);
    if (st) return st;
    if (jobs.empty()) return fail(HANK_EINVAL, "empty request list");
    Prepared PR;
    prepare_jobs(jobs, PR);
    std::unique_ptr<hank_graph> g(new hank_graph);
    HIP_TRY(hipGetDevice(&g->device));
    auto alloc = [&](void*& p, size_t bytes) -> hank_status {
        hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 256));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(e == hipErrorOutOfMemory ? HANK_ENOMEM : HANK_EDEVICE, "hipMalloc failed");
        }
        return HANK_OK;
    };
    if ((st = alloc(g->work, PR.work_need))) return st;
    if ((st = alloc(g->fpart, PR.part_need))) return st;
    if ((st = alloc(g->partial, size_t(PR.pbase) * sizeof(double)))) return st;
    if ((st = alloc(g->probs, PR.probs.size() * sizeof(NearProb)))) return st;
    if ((st = alloc(g->descs, PR.descs.size() * sizeof(FarDesc)))) return st;
    for (auto& D : PR.descs) {
        D.x0 = D.x0off >= 0 ? static_cast<char*>(g->work) + D.x0off : nullptr;
        D.buf = static_cast<char*>(g->work) + reinterpret_cast<size_t>(D.buf);
        if (D.nchunk > 1)
            D.part = reinterpret_cast<double*>(static_cast<char*>(g->fpart) + reinterpret_cast<size_t>(D.part));
    }
    // plans were built on s: finish before the descriptors are copied
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(g->probs, PR.probs.data(), PR.probs.size() * sizeof(NearProb), hipMemcpyHostToDevice));
    if (!PR.descs.empty())
        HIP_TRY(hipMemcpy(g->descs, PR.descs.data(), PR.descs.size() * sizeof(FarDesc), hipMemcpyHostToDevice));
    // capture the launches (kernels only) on a private stream
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const bool prof = g_prof;
    g_prof = false;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = enqueue_jobs(PR, static_cast<const NearProb*>(g->probs), static_cast<const FarDesc*>(g->descs),
                          static_cast<double*>(g->partial), cs);
        hipGraph_t gr = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &gr);
        g->graph = gr;
        if (!st && e2 != hipSuccess) st = fail(HANK_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    } else {
        st = fail(HANK_EDEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    g_prof = prof;
    (void)hipStreamDestroy(cs);
    if (st) return st;
    HIP_TRY(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    for (const Job& J : jobs)
        if (std::find(g->plans.begin(), g->plans.end(), J.dp) == g->plans.end()) g->plans.push_back(J.dp);
    for (DevPlan* dp : g->plans) ++dp->pins;
    ++g_graphs;
    *out = g.release();
    return HANK_OK;
}

hank_status hank_batch_graph_launch(hank_graph* g, hank_stream_t stream) {
    if (!g || !g->exec) return fail(HANK_EINVAL, "null graph");
    HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return HANK_OK;
}

hank_status hank_batch_graph_destroy(hank_graph* g) {
    if (!g) return HANK_OK;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    for (DevPlan* dp : g->plans) --dp->pins;
    delete g;
    --g_graphs;
    return HANK_OK;
}

const char* hank_last_error(void) { return t_err.c_str(); }

hank_status hank_profile(int32_t enable) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    hank_status st = prof_collect();
    if (st) return st;
    for (auto& a : g_acc) a = Acc();
    g_prof = enable != 0;
    return HANK_OK;
}

hank_status hank_profile_report(hank_kernel_stat* out, int32_t max, int32_t* count) {
    if (!count || (max > 0 && !out)) return fail(HANK_EINVAL, "null pointer");
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    hank_status st = prof_collect();
    if (st) return st;
    int32_t n = 0;
    for (int k = 0; k < K_COUNT; ++k) {
        if (g_acc[k].launches == 0) continue;
        if (n < max) {
            hank_kernel_stat& o = out[n];
            std::memset(&o, 0, sizeof o);
            std::strncpy(o.name, k_names[k], sizeof(o.name) - 1);
            o.launches = g_acc[k].launches;
            o.total_ms = g_acc[k].ms;
            o.bytes = g_acc[k].bytes;
            o.work = g_acc[k].work;
        }
        ++n;
    }
    *count = n;
    return HANK_OK;
}

// ---- autotuner of the FFT split ----
// Times passes A, B and C of a synthetic block (rows = columns = L/2, four
// transform groups, FP64, one right-hand side) for every split L1 x L2 the
// kernels support (L1 >= L2) within two steps of the default, L = 2^10 .. 2^23, and
// installs the fastest for plans built afterwards.
hank_status hank_autotune(hank_stream_t stream, int32_t* chosen) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hank_status st = ensure_tables(dev);
    if (st) return st;
    const int G = 4, lgmin = 10, lgmax = 23;
    const int64_t Lmax = int64_t(1) << lgmax;
    // device buffers for the largest case
    void *c = nullptr, *f = nullptr, *buf = nullptr, *H = nullptr, *part = nullptr, *dd = nullptr;
    GroupDev* dg = nullptr;
    TermDev* dt = nullptr;
    auto cleanup = [&]() {
        for (void* p : {c, f, buf, H, part, dd, (void*)dg, (void*)dt})
            if (p) (void)hipFree(p);
    };
    auto al = [&](void*& p, size_t bytes) -> bool { return hipMalloc(&p, bytes) == hipSuccess; };
    if (!al(c, size_t(Lmax) * 4) || !al(f, size_t(Lmax) * 4) || !al(buf, size_t(G) * size_t(Lmax) * 16) ||
        !al(H, size_t(Lmax) * 16) || !al(part, size_t(Lmax) * 4 * G) || !al(dd, sizeof(FarDesc)) ||
        !al(reinterpret_cast<void*&>(dg), sizeof(GroupDev) * G) || !al(reinterpret_cast<void*&>(dt), sizeof(TermDev) * G)) {
        (void)hipGetLastError();
        cleanup();
        return fail(HANK_ENOMEM, "autotune: out of device memory");
    }
    GroupDev hg[G];
    TermDev ht[G];
    for (int i = 0; i < G; ++i) {
        hg[i] = GroupDev{0, -i, i, i + 1, 1.0};
        ht[i] = TermDev{0, i, 0.5, 0.25};
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto run = [&]() -> hank_status {
        HIP_TRY(hipMemsetAsync(c, 0, size_t(Lmax) * 4, s));
        HIP_TRY(hipMemsetAsync(H, 0, size_t(Lmax) * 16, s));
        HIP_TRY(hipMemcpyAsync(dg, hg, sizeof(hg), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(dt, ht, sizeof(ht), hipMemcpyHostToDevice, s));
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        for (int lg = lgmin; lg <= lgmax; ++lg) {
            const int64_t L = int64_t(1) << lg;
            const int def = default_fft_l2(lg);
            int best = def;
            float best_ms = 1e30f;
            for (int l2 = std::max(3, def - 2); l2 <= std::min(10, def + 2); ++l2) {
                const int l1 = lg - l2;
                if (l1 < l2 || l1 > 13) continue; // the column passes assume L1 >= L2
                FarDesc D{};
                FarArgs& A = D.A;
                A.ka = A.na = 1;
                A.nrows = A.ncols = L / 2;
                A.L = L;
                A.L1 = int32_t(1) << l1;
                A.L2 = int32_t(1) << l2;
                A.twshift = 23 - lg;
                A.ngroups = G;
                A.g0 = 0;
                A.g1 = G;
                A.ar = A.ac = 1;
                A.D = Lmax;
                A.Dr = A.Qc = Lmax;
                A.Kka = A.Nna = 1;
                A.pi_Qc = 1e-6;
                A.r0 = A.w0 = A.eref = A.lref = A.bref = 1.0;
                A.groups = dg;
                A.terms = dt;
                D.c = static_cast<const double*>(c);
                D.f = static_cast<double*>(f);
                D.buf = buf;
                D.x0off = -1;
                D.x0 = nullptr;
                D.H = H;
                D.part = static_cast<double*>(part);
                D.ldc = D.ldo = L / 2;
                D.nrhs = 1;
                D.nchunk = far_chunks(L, G, 1);
                D.gchunk = (G + D.nchunk - 1) / D.nchunk;
                D.nchunk = (G + D.gchunk - 1) / D.gchunk;
                const int64_t nac = int64_t(D.nchunk) * (A.L1 / col_width(A.L2, false));
                const int32_t rows = far_rows_per_wg(A.L1);
                const int64_t nb = int64_t(D.nchunk) * ((A.L2 + rows - 1) / rows);
                HIP_TRY(hipMemcpyAsync(dd, &D, sizeof(D), hipMemcpyHostToDevice, s));
                const FarDesc* pd = static_cast<const FarDesc*>(dd);
                float ms = 1e30f;
                for (int rep = 0; rep < 4; ++rep) {
                    HIP_TRY(hipEventRecord(e0, s));
                    HIP_TRY(launch_far_pass(0, false, A.L1, A.L2, pd, 1, nac, s));
                    HIP_TRY(launch_far_pass(1, false, A.L1, A.L2, pd, 1, nb, s));
                    HIP_TRY(launch_far_pass(2, false, A.L1, A.L2, pd, 1, nac, s));
                    HIP_TRY(hipEventRecord(e1, s));
                    HIP_TRY(hipEventSynchronize(e1));
                    float t = 0;
                    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
                    if (rep > 0) ms = std::min(ms, t);
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best = l2;
                }
            }
            set_fft_split(lg, best);
            if (chosen) chosen[lg] = best;
        }
        return HANK_OK;
    };
    st = run();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    cleanup();
    return st;
}

hank_status hank_autotune_save(const char* path) {
    if (!path) return fail(HANK_EINVAL, "null path");
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    FILE* fp = std::fopen(path, "w");
    if (!fp) return fail(HANK_EINVAL, std::string("cannot write ") + path);
    std::fprintf(fp, "# FFT splits: log2(L) log2(L2), L = L1 x L2 (hank_autotune)\n");
    for (int lg = 0; lg < 32; ++lg)
        if (tuned_fft_split(lg) > 0) std::fprintf(fp, "%d %d\n", lg, tuned_fft_split(lg));
    const bool ok = std::fclose(fp) == 0;
    return ok ? HANK_OK : fail(HANK_EINVAL, std::string("cannot write ") + path);
}

hank_status hank_autotune_load(const char* path) {
    if (!path) return fail(HANK_EINVAL, "null path");
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    FILE* fp = std::fopen(path, "r");
    if (!fp) return fail(HANK_EINVAL, std::string("cannot read ") + path);
    std::vector<std::pair<int, int>> splits;
    char line[256];
    int lineno = 0;
    while (std::fgets(line, sizeof line, fp)) {
        ++lineno;
        char* q = line;
        while (*q == ' ' || *q == '\t') ++q;
        if (*q == '#' || *q == '\n' || *q == '\0') continue;
        int lg = 0, l2 = 0;
        char extra = 0;
        if (std::sscanf(q, "%d %d %c", &lg, &l2, &extra) != 2 || !valid_fft_split(lg, l2)) {
            std::fclose(fp);
            return fail(HANK_EINVAL, std::string(path) + ":" + std::to_string(lineno) + ": not a supported split");
        }
        splits.emplace_back(lg, l2);
    }
    std::fclose(fp);
    for (auto& p : splits) set_fft_split(p.first, p.second);
    return HANK_OK;
}

hank_status hank_autotune_reset(void) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    for (int lg = 0; lg < 32; ++lg) set_fft_split(lg, 0);
    return HANK_OK;
}

hank_status hank_cache_clear(void) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (g_graphs > 0) return fail(HANK_EINVAL, "batch graphs still refer to cached plans");
    (void)hipDeviceSynchronize();
    ++g_call; // no call of the past holds on to its plans
    for (auto it = g_cache.begin(); it != g_cache.end();) // plans of running servers stay
        it = it->second->pins > 0 ? std::next(it) : g_cache.erase(it);
    return HANK_OK;
}

int64_t hank_cache_bytes(void) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    return cache_total();
}

hank_status hank_cache_limit(int64_t bytes) {
    if (bytes < 0) return fail(HANK_EINVAL, "negative cache limit");
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    g_cache_limit = bytes;
    ++g_call;
    evict_to(bytes);
    return HANK_OK;
}

double hank_param_s(int32_t nu, int32_t M, double eps) { return param_s(nu, M, eps); }
double hank_param_t(int32_t nu, int32_t T, double eps) { return param_t(nu, T, eps); }
double hank_param_neumann(int32_t K, double eps) { return param_neumann(K, eps); }
double hank_param_pK(int32_t K, double eps) { return param_pK(K, eps); }
double hank_param_qT(int32_t T, double eps) { return param_qT(T, eps); }

static hank_status host_plan(int32_t task, int64_t N, double eps, const hank_options* o, Plan& p) {
    if (!valid_task(task)) return fail(HANK_EINVAL, "unknown task");
    try {
        p = make_plan(task, N, eps, o ? o->plan_mode : 0, o ? o->precision : 0, o && o->direct,
                      cost_model_for(o), rhs_bucket(plan_nrhs(o && o->nrhs > 1 ? o->nrhs : 1, o ? o->nu : 0)), o ? o->M : 0,
                      o ? o->nu : 0, o ? o->shift : 0);
    } catch (const std::exception& ex) {
        return fail(HANK_EINVAL, ex.what());
    }
    return HANK_OK;
}

hank_status hank_plan_info(int32_t task, int64_t N, double eps, const hank_options* options,
                           hank_plan_summary* out) {
    if (!out) return fail(HANK_EINVAL, "null pointer");
    Plan p;
    hank_status st = host_plan(task, N, eps, options, p);
    if (st) return st;
    hank_plan_summary s{};
    s.M = p.M;
    s.K = p.K;
    s.T = p.T;
    s.P = p.P;
    s.nblocks = int32_t(p.blocks.size());
    s.s = p.s;
    s.alpha = p.alpha;
    s.beta = p.beta;
    s.near_entries = p.near_entries;
    s.first_direct = p.first_direct;
    s.bulk_fp32 = p.fp32;
    s.model_s = p.cost;
    for (auto& b : p.blocks) {
        const int64_t g32 = int64_t(b.groups.size()) - b.g64;
        s.far_transforms += int64_t(b.groups.size());
        s.fp32_transforms += int32_t(g32);
        s.fft_points += int64_t(b.groups.size()) * b.L;
        // one write and one read of each FFT point per pass boundary, only for
        // the work-buffer columns that carry data (j1 < ncols) or results (j1 < nrows)
        const double L1 = double(b.L1), fa = std::min(double(b.nb - b.na + 1), L1) / L1,
                     fc = std::min(double(b.kb - b.ka + 1), L1) / L1;
        s.fft_bytes += (16.0 * double(b.g64) + 8.0 * double(g32)) * double(b.L) * 2.0 * (fa + fc);
    }
    *out = s;
    return HANK_OK;
}

hank_status hank_plan_block(int32_t task, int64_t N, double eps, const hank_options* options, int32_t k,
                            hank_block_info* out) {
    if (!out) return fail(HANK_EINVAL, "null pointer");
    Plan p;
    hank_status st = host_plan(task, N, eps, options, p);
    if (st) return st;
    if (k < 0 || k >= int32_t(p.blocks.size())) return fail(HANK_EINVAL, "block index out of range");
    const Block& b = p.blocks[size_t(k)];
    out->row0 = b.ka;
    out->row1 = b.kb;
    out->col0 = b.na;
    out->col1 = b.nb;
    out->fft_len = b.L;
    out->groups = int32_t(b.groups.size());
    out->terms = int32_t(b.terms.size());
    out->zmin = b.s0;
    out->fft_l1 = b.L1;
    out->fft_l2 = b.L2;
    return HANK_OK;
}

// ---- the allocation-free form of hank_transform ----
// Workspace from the library's static device array (noalloc_scratch): near and
// far descriptors, near-field partials, far-field chunk sums and the far work
// buffer, in that order; the far field goes in as many group waves as the
// array needs.  The plan must already be cached.
hank_status hank_transform_noalloc(int32_t task, const double* c, int64_t N, int64_t nrhs, int64_t ldc, double eps,
                                   double* out, int64_t ldo, const hank_options* options, hank_stream_t stream) {
    hank_status st = check_args(task, c, N, nrhs, ldc, eps, out, ldo);
    if (st) return st;
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    void* base = nullptr;
    HIP_TRY(noalloc_scratch(&base));
    auto it = g_cache.find(plan_key(task, N, eps, options, dev, nrhs));
    if (it != g_cache.end()) it->second->last_use = ++g_use_clock;
    if (it == g_cache.end()) {
        Plan p;
        if ((st = host_plan(task, N, eps, options, p))) return st; // invalid options
        return fail(HANK_EUNSUPPORTED,
                    "hank_transform_noalloc: no plan for these arguments is cached on this device (it builds "
                    "none); one hank_transform call with the same task, N, eps, options and nrhs builds it");
    }
    std::vector<Job> jobs{Job{it->second.get(), c, ldc, out, ldo, nrhs}};
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    Prepared PR;
    size_t budget = NOALLOC_SCRATCH_BYTES, need = 0;
    for (;;) { // smaller far-field waves until the workspace fits
        PR = Prepared();
        prepare_jobs(jobs, PR, budget);
        need = al(PR.probs.size() * sizeof(NearProb)) + al(PR.descs.size() * sizeof(FarDesc)) +
               al(size_t(PR.pbase) * sizeof(double)) + al(PR.part_need) + al(PR.work_need);
        if (need <= NOALLOC_SCRATCH_BYTES || budget < (size_t(1) << 20)) break;
        budget /= 2;
    }
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(HANK_EUNSUPPORTED, "hank_transform_noalloc: the transform needs " + std::to_string(need) +
                                           " bytes of workspace, more than the " +
                                           std::to_string(NOALLOC_SCRATCH_BYTES) + " of the static scratch");
    char* p = static_cast<char*>(base);
    void* dprobs = p;
    p += al(PR.probs.size() * sizeof(NearProb));
    void* ddescs = p;
    p += al(PR.descs.size() * sizeof(FarDesc));
    double* dpart = reinterpret_cast<double*>(p);
    p += al(size_t(PR.pbase) * sizeof(double));
    char* fpart = p;
    p += al(PR.part_need);
    char* work = p;
    for (auto& D : PR.descs) {
        D.x0 = D.x0off >= 0 ? work + D.x0off : nullptr;
        D.buf = work + reinterpret_cast<size_t>(D.buf);
        if (D.nchunk > 1) D.part = reinterpret_cast<double*>(fpart + reinterpret_cast<size_t>(D.part));
    }
    if ((st = upload_descriptors(PR, dprobs, ddescs, s))) return st;
    return enqueue_jobs(PR, static_cast<const NearProb*>(dprobs), static_cast<const FarDesc*>(ddescs), dpart, s);
}

hank_status hank_root_offsets(int64_t nmax, double* b, hank_stream_t stream) {
    if (!b || nmax < 1) return fail(HANK_EINVAL, "bad arguments");
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hank_status st = ensure_tables(dev);
    if (st) return st;
    HIP_TRY(launch_roots(nmax, b, 0, nullptr, (hipStream_t)stream));
    return HANK_OK;
}

hank_status hank_j0(const double* z, int64_t count, double* out, hank_stream_t stream) {
    if (!z || !out || count < 0) return fail(HANK_EINVAL, "bad arguments");
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hank_status st = ensure_tables(dev);
    if (st) return st;
    HIP_TRY(launch_j0(z, count, out, (hipStream_t)stream));
    return HANK_OK;
}

} // extern "C"
