// api.cpp -- the C ABI (include/hank.h): argument checks, plan cache, device
// resources of a plan, and the launch sequence of one transform.
#include "../../include/hank.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
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

constexpr int64_t NEAR_CHUNK = 2048; // columns per near-field work item

struct DevBlock {
    Block hb;
    FarArgs args{};
    void* H = nullptr;
    GroupDev* groups = nullptr;
    TermDev* terms = nullptr;
};

struct DevPlan {
    Plan plan;
    int device = 0;
    double* b = nullptr; // root offsets b_1..b_{N+1}
    double* e = nullptr; // DHT row perturbations e_1..e_N
    NearTile* tiles = nullptr;
    int64_t ntiles = 0;
    RowTile* rt = nullptr;
    int64_t nrt = 0;
    double* partial = nullptr;
    std::vector<DevBlock> blocks;
    void* work = nullptr;
    size_t bytes = 0;
    GridArgs G{};

    ~DevPlan() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        auto fr = [](void* p) {
            if (p) (void)hipFree(p);
        };
        fr(b);
        fr(e);
        fr(tiles);
        fr(rt);
        fr(partial);
        fr(work);
        for (auto& d : blocks) {
            fr(d.H);
            fr(d.groups);
            fr(d.terms);
        }
        (void)hipSetDevice(cur);
    }
};

using Key = std::tuple<int, int64_t, uint64_t, int, int, int, int>;
std::map<Key, std::unique_ptr<DevPlan>> g_cache;
std::set<int> g_tables_ready;

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

template <typename T>
hank_status dev_alloc(T*& p, size_t count, size_t& total) {
    if (count == 0) count = 1;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, count * sizeof(T));
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

// Branches and Hankel term count of a near-field tile from bounds on z over it:
// z >= z~ (the perturbations e_k, b_n are non-negative) and z <= z~ + 0.25.
int32_t near_flags(const Grid& g, const NearTile& t) {
    const double zlo = g.ztilde(t.k0, t.n0);
    const double zhi = g.ztilde(t.k0 + t.nk - 1, t.n1 - 1) + 0.25;
    int32_t f = 0;
    if (zlo < J0_ASY_Z) f |= 1;
    if (zhi >= J0_ASY_Z) f |= 2;
    const double za = std::max(zlo, J0_ASY_Z);
    const int M = za < 28.0 ? 12 : za < 44.0 ? 8 : za < 65.0 ? 6 : za < 123.0 ? 5 : za < 376.0 ? 4 : 3;
    return f | (M << 8);
}

hank_status build_dev_plan(DevPlan& dp, hipStream_t s) {
    const Plan& p = dp.plan;
    const Grid& g = p.g;
    const int64_t N = g.N;
    dp.G = grid_args(g);
    hank_status st;
    if (g.col_pert || g.row_pert) {
        if ((st = dev_alloc(dp.b, size_t(N + 1), dp.bytes))) return st;
        HIP_TRY(launch_roots(N + 1, dp.b, s));
    }
    if (g.row_pert) {
        if ((st = dev_alloc(dp.e, size_t(N), dp.bytes))) return st;
        HIP_TRY(launch_dht_e(N, dp.b, dp.e, s));
    }
    // near-field work items
    std::vector<NearTile> tiles;
    std::vector<RowTile> rts;
    for (auto& seg : p.near)
        for (int64_t k = seg.k0; k < seg.k1; k += 64) {
            RowTile r{};
            r.k0 = k;
            r.nk = int32_t(std::min<int64_t>(64, seg.k1 - k));
            r.tile0 = int64_t(tiles.size());
            for (int64_t n = 1; n < seg.ncut; n += NEAR_CHUNK) {
                NearTile t{};
                t.k0 = k;
                t.nk = r.nk;
                t.n0 = n;
                t.n1 = std::min(seg.ncut, n + NEAR_CHUNK);
                t.flags = near_flags(g, t);
                tiles.push_back(t);
            }
            r.ntiles = int64_t(tiles.size()) - r.tile0;
            rts.push_back(r);
        }
    dp.ntiles = int64_t(tiles.size());
    dp.nrt = int64_t(rts.size());
    if ((st = dev_alloc(dp.tiles, tiles.size(), dp.bytes))) return st;
    if ((st = dev_alloc(dp.rt, rts.size(), dp.bytes))) return st;
    if ((st = dev_alloc(dp.partial, size_t(dp.ntiles) * 64, dp.bytes))) return st;
    if (!tiles.empty())
        HIP_TRY(hipMemcpyAsync(dp.tiles, tiles.data(), tiles.size() * sizeof(NearTile), hipMemcpyHostToDevice, s));
    if (!rts.empty())
        HIP_TRY(hipMemcpyAsync(dp.rt, rts.data(), rts.size() * sizeof(RowTile), hipMemcpyHostToDevice, s));

    // far-field blocks
    const size_t esz = p.fp32 ? 8 : 16;
    size_t work_elems = 0;
    for (auto& hb : p.blocks) {
        const size_t gb = group_batch(size_t(hb.L) * esz, hb.groups.size());
        work_elems = std::max(work_elems, size_t(hb.L) * std::max<size_t>(1, gb));
    }
    if (!p.blocks.empty())
        if ((st = dev_alloc(reinterpret_cast<char*&>(dp.work), work_elems * esz, dp.bytes))) return st;
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
        if ((st = dev_alloc(reinterpret_cast<char*&>(d.H), size_t(hb.L) * esz, dp.bytes))) return st;
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
        HIP_TRY(launch_chirp_spectrum(A, p.fp32, dp.work, d.H, s));
    }
    // the host vectors above must outlive the asynchronous copies
    HIP_TRY(hipStreamSynchronize(s));
    return HANK_OK;
}

hank_status get_plan(int task, int64_t N, double eps, const hank_options* o, hipStream_t s, DevPlan*& out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hank_status st = ensure_tables(dev);
    if (st) return st;
    int mode = o ? o->plan_mode : 0, prec = o ? o->precision : 0, direct = o ? o->direct : 0;
    int far = o ? o->prefer_far : 0;
    uint64_t eb;
    std::memcpy(&eb, &eps, 8);
    Key key{task, N, eb, mode, prec, direct * 2 + far, dev};
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        out = it->second.get();
        return HANK_OK;
    }
    std::unique_ptr<DevPlan> dp(new DevPlan);
    dp->device = dev;
    try {
        dp->plan = make_plan(task, N, eps, mode, prec, direct != 0, cost_model_for(o));
    } catch (const std::exception& ex) {
        return fail(HANK_EINVAL, std::string("planning failed: ") + ex.what());
    }
    st = build_dev_plan(*dp, s);
    if (st) return st; // dp's destructor frees what was allocated
    out = dp.get();
    g_cache[key] = std::move(dp);
    return HANK_OK;
}

// ---- optional per-kernel timing (hank_profile) ----
enum { K_NEAR = 0, K_NEAR_REDUCE, K_PASS_A, K_PASS_B, K_PASS_C, K_COUNT };
const char* const k_names[K_COUNT] = {"near", "near_reduce", "pass_a", "pass_b", "pass_c"};
struct Pending {
    int kind;
    hipEvent_t a, b;
    double bytes, work;
};
bool g_prof = false;
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

hank_status run_plan(DevPlan& dp, const double* c, double* f, hipStream_t s) {
    hank_status st;
    hipEvent_t ev;
    const double esz = dp.plan.fp32 ? 8.0 : 16.0;
    if ((st = prof_begin(ev, s))) return st;
    HIP_TRY(launch_near(dp.G, c, dp.b, dp.e, dp.tiles, dp.ntiles, dp.partial, s));
    if ((st = prof_end(K_NEAR, ev, 64.0 * 8.0 * double(dp.ntiles), double(dp.plan.near_entries), s))) return st;
    if ((st = prof_begin(ev, s))) return st;
    HIP_TRY(launch_near_reduce(dp.rt, dp.nrt, dp.partial, f, s));
    if ((st = prof_end(K_NEAR_REDUCE, ev, 64.0 * 8.0 * double(dp.ntiles) + 8.0 * double(dp.plan.g.N), 0.0, s)))
        return st;
    for (auto& d : dp.blocks) {
        const size_t gb = group_batch(size_t(d.args.L) * size_t(esz), size_t(d.args.ngroups));
        FarArgs A = d.args;
        for (int32_t g0 = 0; g0 < d.args.ngroups; g0 += int32_t(gb)) {
            A.g0 = g0;
            A.g1 = std::min(d.args.ngroups, g0 + int32_t(gb));
            const double G = double(A.g1 - A.g0), L = double(A.L);
            const double pert = (A.col_pert ? 8.0 : 0.0);
            const double bytes[3] = {G * L * esz + double(A.ncols) * (8.0 + pert),
                                     2.0 * G * L * esz + L * esz,
                                     G * L * esz + double(A.nrows) * (16.0 + (A.row_pert ? 8.0 : 0.0))};
            for (int w = 0; w < 3; ++w) {
                if ((st = prof_begin(ev, s))) return st;
                HIP_TRY(launch_far_pass(w, A, dp.plan.fp32, c, dp.b, dp.e, dp.work, d.H, f, s));
                if ((st = prof_end(K_PASS_A + w, ev, bytes[w], G * L, s))) return st;
            }
        }
    }
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
    hipStream_t s = (hipStream_t)stream;
    DevPlan* dp = nullptr;
    if ((st = get_plan(task, N, eps, o, s, dp))) return st;
    for (int64_t j = 0; j < nrhs; ++j)
        if ((st = run_plan(*dp, c + j * ldc, out + j * ldo, s))) return st;
    return HANK_OK;
}

} // namespace

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

hank_status hank_transform(int32_t task, const double* c, int64_t N, int64_t nrhs, int64_t ldc, double eps,
                           double* out, int64_t ldo, const hank_options* options, hank_stream_t stream) {
    return transform(task, c, N, nrhs, ldc, eps, out, ldo, options, stream);
}

hank_status hank_batch(const hank_request* reqs, int64_t count, hank_stream_t stream) {
    if (count < 0 || (count > 0 && !reqs)) return fail(HANK_EINVAL, "bad request list");
    for (int64_t i = 0; i < count; ++i) {
        const hank_request& r = reqs[i];
        hank_status st = check_args(r.task, r.c, r.N, r.nrhs, r.ldc, r.eps, r.out, r.ldo);
        if (st) return fail(st, "request " + std::to_string(i) + ": " + t_err);
    }
    for (int64_t i = 0; i < count; ++i) {
        const hank_request& r = reqs[i];
        hank_options o{};
        o.precision = r.precision;
        hank_status st = transform(r.task, r.c, r.N, r.nrhs, r.ldc, r.eps, r.out, r.ldo, &o, stream);
        if (st) return st;
    }
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

hank_status hank_cache_clear(void) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    (void)hipDeviceSynchronize();
    g_cache.clear();
    return HANK_OK;
}

int64_t hank_cache_bytes(void) {
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    int64_t t = 0;
    for (auto& kv : g_cache) t += int64_t(kv.second->bytes);
    return t;
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
                      cost_model_for(o));
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
    const double esz = p.fp32 ? 8.0 : 16.0;
    for (auto& b : p.blocks) {
        s.far_transforms += int64_t(b.groups.size());
        s.fft_points += int64_t(b.groups.size()) * b.L;
        s.fft_bytes += double(b.groups.size()) * double(b.L) * esz * 4.0;
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
    return HANK_OK;
}

hank_status hank_root_offsets(int64_t nmax, double* b, hank_stream_t stream) {
    if (!b || nmax < 1) return fail(HANK_EINVAL, "bad arguments");
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hank_status st = ensure_tables(dev);
    if (st) return st;
    HIP_TRY(launch_roots(nmax, b, (hipStream_t)stream));
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
