// Host-only driver for the sanitizer build of the planner and the table
// generators (planner.cpp, tables.cpp): plans for every task over a range of
// N, eps, plan modes, precisions, orders and right-hand-side counts, the
// rejected argument combinations, and the J_0 / J_nu / twiddle tables.  Built
// with -fsanitize=address,undefined by tests/test_sanitize.py; any sanitizer
// report or a broken plan invariant fails the run.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <stdexcept>

#include "../../paper_1501_01652_amd/csrc/plan.h"
#include "../../paper_1501_01652_amd/csrc/tables.h"

using namespace hank;

static int failures = 0;

static void check(bool ok, const char* what, int task, long long N, double eps) {
    if (!ok) {
        std::fprintf(stderr, "invariant failed: %s (task %d N %lld eps %g)\n", what, task, N, eps);
        ++failures;
    }
}

static void check_plan(const Plan& p, int task, long long N, double eps) {
    for (const Block& b : p.blocks) {
        check(b.ka >= 1 && b.kb <= N && b.ka <= b.kb, "block rows", task, N, eps);
        check(b.na >= 1 && b.nb <= N && b.na <= b.nb, "block columns", task, N, eps);
        check(b.L >= (b.kb - b.ka + 1) + (b.nb - b.na + 1) - 1, "FFT length", task, N, eps);
        check(int64_t(b.L1) * b.L2 == b.L, "FFT split", task, N, eps);
        check(b.g64 >= 0 && b.g64 <= int(b.groups.size()), "precision split", task, N, eps);
        for (const Group& g : b.groups)
            check(g.t0 >= 0 && g.t0 <= g.t1 && g.t1 <= int(b.terms.size()), "group terms", task, N, eps);
    }
    int64_t entries = 0;
    for (const NearSeg& s : p.near) {
        check(s.k0 >= 1 && s.k1 <= N + 1 && s.k0 < s.k1 && s.ncut >= 1 && s.ncut <= N + 1, "near segment", task, N,
              eps);
        entries += (s.k1 - s.k0) * (s.ncut - 1);
    }
    check(entries == p.near_entries, "near entry count", task, N, eps);
}

int main() {
    std::unique_ptr<DeviceTables> t(new DeviceTables);
    build_tables(*t);
    check(std::fabs(t->ser[0] - 1.0) < 1e-15, "J_0 series", 0, 0, 0);
    std::unique_ptr<double[]> nu(new double[NU_TAB_SIZE]);
    for (int v = 1; v <= HANK_NU_MAX; ++v) build_nu_table(v, nu.get());

    const CostModel cm;
    const long long Ns[] = {1, 2, 3, 17, 64, 100, 158, 159, 1000, 4096, 5000, 65536, 1 << 20, 1 << 22};
    const double epss[] = {1e-15, 1e-14, 1e-8, 1e-4, 0.3};
    int built = 0;
    for (int task = 0; task <= 4; ++task)
        for (long long N : Ns)
            for (double eps : epss)
                for (int mode = 0; mode <= 2; ++mode)
                    for (int prec = 0; prec <= 2; ++prec)
                        for (int nrhs : {1, 16}) {
                            if (N >= (1 << 20) && (prec == 2 || nrhs > 1 || mode == 2)) continue; // keep it short
                            try {
                                Plan p = make_plan(task, N, eps, mode, prec, false, cm, nrhs, 0, 0, 0);
                                check_plan(p, task, N, eps);
                                ++built;
                            } catch (const std::invalid_argument&) {
                                check(N < 2 && (task == 0 || task == 1 || task == 3 || task == 4), "rejected", task,
                                      N, eps);
                            }
                        }
    // orders, shifts and the M sweep
    for (int task : {0, 1, 3, 4})
        for (int v = 0; v <= HANK_NU_MAX; v += 3)
            for (long long N : {100LL, 5000LL, 65536LL}) {
                Plan p = make_plan(task, N, 1e-8, 0, 0, false, cm, 1, 0, v, (task == 0 || task == 3) ? v : 0);
                check_plan(p, task, N, 1e-8);
                ++built;
            }
    for (int M = 1; M <= 20; ++M) {
        try {
            Plan p = make_plan(0, 5000, 1e-11, 1, 0, false, cm, 1, M);
            check_plan(p, 0, 5000, 1e-11);
            ++built;
        } catch (const std::invalid_argument&) {
        }
    }
    // argument errors must throw, not crash
    int rejected = 0;
    auto expect_throw = [&](int task, long long N, double eps, int mode, int M, int v, long long shift) {
        try {
            (void)make_plan(task, N, eps, mode, 0, false, cm, 1, M, v, shift);
            std::fprintf(stderr, "accepted bad arguments: task %d N %lld eps %g mode %d M %d nu %d shift %lld\n", task,
                         N, eps, mode, M, v, shift);
            ++failures;
        } catch (const std::invalid_argument&) {
            ++rejected;
        }
    };
    expect_throw(0, 1, 1e-8, 0, 0, 0, 0);
    expect_throw(2, 0, 1e-8, 0, 0, 0, 0);
    expect_throw(2, (1LL << 24) + 1, 1e-8, 0, 0, 0, 0);
    expect_throw(2, 100, 0.0, 0, 0, 0, 0);
    expect_throw(2, 100, 1.0, 0, 0, 0, 0);
    expect_throw(2, 100, NAN, 0, 0, 0, 0);
    expect_throw(2, 100, 1e-16, 0, 0, 0, 0);
    expect_throw(2, 100, 1e-8, 3, 0, 0, 0);
    expect_throw(2, 100, 1e-8, 0, 5, 0, 0);
    expect_throw(2, 100, 1e-8, 1, 21, 0, 0);
    expect_throw(2, 100, 1e-8, 0, 0, 1, 0);
    expect_throw(0, 100, 1e-8, 0, 0, HANK_NU_MAX + 1, 0);
    expect_throw(1, 100, 1e-8, 0, 0, 0, 1);
    expect_throw(0, 100, 1e-8, 0, 0, 0, HANK_SHIFT_MAX + 1);
    std::printf("plans %d rejected %d failures %d\n", built, rejected, failures);
    return failures ? 1 : 0;
}
