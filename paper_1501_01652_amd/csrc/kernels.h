// kernels.h -- argument blocks and launchers of the device kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.h"

namespace hank {

// z~_kn = pi K_k N_n / D with K_k = ar k + br, N_n = ac n + bc; r^_k = K_k/Dr,
// w^_n = pi N_n / Qc.  pi/D is carried as hi + lo.
struct GridArgs {
    int64_t ar, br, ac, bc, D, Dr, Qc;
    double pi_Qc, piD_hi, piD_lo, invD;
    int32_t row_pert, col_pert;
};

// near-field work item: rows [k0, k0+nk) x columns [n0, n1); flags: bit 0 some
// entry has z < 20, bit 1 some entry has z >= 20, bits 8.. Hankel pairs needed
// for the smallest z >= 20 of the tile (remainder below 1e-17)
struct NearTile {
    int64_t k0, n0, n1;
    int32_t nk, flags;
};

// rows [k0, k0+nk) own partials of tiles [tile0, tile0+ntiles)
struct RowTile {
    int64_t k0, tile0, ntiles;
    int32_t nk, pad;
};

struct GroupDev {
    int32_t a, e, t0, t1;
    double scale;
};

struct TermDev {
    int32_t b, m;
    double kre, kim;
};

// One far-field block: rows ka.., columns na.., FFT length L = L1*L2.
struct FarArgs {
    int64_t ka, na, nrows, ncols, L;
    int32_t L1, L2, twshift, ngroups;
    int32_t g0, g1; // groups [g0, g1) of this launch; group g lives at buf + (g - g0) * L
    int64_t ar, br, ac, bc, D, Dr, Qc, Kka, Nna;
    double pi_Qc, r0, w0, eref, lref, bref;
    int32_t row_pert, col_pert;
    const GroupDev* groups;
    const TermDev* terms;
};

hipError_t upload_tables(const DeviceTables& t);
hipError_t launch_roots(int64_t nmax, double* b, hipStream_t s);
hipError_t launch_dht_e(int64_t N, const double* b, double* e, hipStream_t s);
hipError_t launch_j0(const double* z, int64_t n, double* out, hipStream_t s);
hipError_t launch_near(const GridArgs& G, const double* c, const double* b, const double* e,
                       const NearTile* tiles, int64_t ntiles, double* partial, hipStream_t s);
hipError_t launch_near_reduce(const RowTile* rt, int64_t nrt, const double* partial, double* f, hipStream_t s);
hipError_t launch_chirp_spectrum(const FarArgs& A, bool fp32, void* work, void* H, hipStream_t s);
// which: 0 pass A (inputs + column FFTs), 1 pass B (row FFT x H^ x inverse), 2 pass C (epilogue)
hipError_t launch_far_pass(int which, const FarArgs& A, bool fp32, const double* c, const double* b,
                           const double* e, void* work, const void* H, double* f, hipStream_t s);

} // namespace hank
