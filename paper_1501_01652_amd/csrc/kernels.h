// kernels.h -- argument blocks and launchers of the device kernels.
//
// Work is described by small device-resident descriptors so that one launch
// can cover the same kind of work for many transforms (several right-hand
// sides, several requests of a batch): near-field tiles name their problem,
// far-field workgroups find their block through a workgroup map.
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

// One transform's near field: grid, coefficient columns c + j*ldc (j < nrhs),
// root offsets b and DHT row perturbations e.
struct NearProb {
    GridArgs G;
    const double* c;
    const double* b;
    const double* e;
    int64_t ldc;
    int32_t nrhs, pad;
};

// near-field work item: rows [k0, k0+nk) x columns [n0, n1) of problem prob;
// its nrhs x 64 partial sums start at partial + pbase.  flags: bit 0 some
// entry has z < 20, bit 1 some entry has z >= 20, bits 8.. Hankel pairs needed
// for the smallest z >= 20 of the tile (remainder below 1e-17)
struct NearTile {
    int64_t k0, n0, n1, pbase;
    int32_t nk, flags, prob, pad;
};

// rows [k0, k0+nk) own the partials of tiles [tile0, tile0+ntiles), which
// start at partial + pbase (nrhs x 64 per tile); column j goes to f + j*ldo
struct RowTile {
    int64_t k0, tile0, ntiles, pbase;
    double* f;
    int64_t ldo;
    int32_t nk, nrhs;
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
    int32_t g0, g1; // groups [g0, g1) of this launch
    int64_t ar, br, ac, bc, D, Dr, Qc, Kka, Nna;
    double pi_Qc, r0, w0, eref, lref, bref;
    int32_t row_pert, col_pert;
    const GroupDev* groups;
    const TermDev* terms;
};

// A block applied to nrhs right-hand sides: the work buffer holds
// (j * (g1-g0) + (g - g0)) * L elements for rhs j and group g.  The groups
// are cut into nchunk chunks of gchunk groups, one workgroup set per
// (rhs, chunk).  With nchunk > 1 pass C leaves chunk sums in
// part[(j * nchunk + chunk) * nrows + k'] and k_far_reduce adds them to f in
// chunk order; with nchunk == 1 pass C adds into f itself.
struct FarDesc {
    FarArgs A;
    const double* c;
    const double* b;
    const double* e;
    double* f;
    void* buf;
    const void* H;
    double* part;
    int64_t ldc, ldo;
    int32_t nrhs, nchunk, gchunk, pad;
};

// workgroup -> descriptor, workgroup index within its (rhs, chunk) set,
// right-hand side and group chunk (for k_far_reduce: row block and rhs)
struct WgMap {
    int32_t desc, wg, j, chunk;
};

hipError_t upload_tables(const DeviceTables& t);
hipError_t launch_roots(int64_t nmax, double* b, hipStream_t s);
hipError_t launch_dht_e(int64_t N, const double* b, double* e, hipStream_t s);
hipError_t launch_j0(const double* z, int64_t n, double* out, hipStream_t s);
// single right-hand-side tiles (k_near) and multi right-hand-side tiles
// (k_near_multi: J_0 evaluated once per entry, product on FP64 MFMA for nrhs >= 16)
hipError_t launch_near(const NearProb* probs, const NearTile* tiles, int64_t ntiles, double* partial,
                       hipStream_t s);
hipError_t launch_near_multi(const NearProb* probs, const NearTile* tiles, int64_t ntiles, bool mfma,
                             double* partial, hipStream_t s);
hipError_t launch_near_reduce(const RowTile* rt, int64_t nrt, const double* partial, hipStream_t s);
hipError_t launch_chirp_spectrum(const FarArgs& A, bool fp32, void* work, void* H, hipStream_t s);
// which: 0 pass A (inputs + column FFTs), 1 pass B (row FFT x H^ x inverse), 2 pass C (epilogue).
// All descriptors of one launch share fp32 and the FFT split (L1, L2).
// workgroups per block of the column passes (L1/8) and of pass B
int32_t far_rows_per_wg(int32_t L1);
hipError_t launch_far_pass(int which, bool fp32, int32_t L1, int32_t L2, const FarDesc* descs,
                           const WgMap* map, int64_t nwg, hipStream_t s);
// f += sum over chunks of part, 256 rows per workgroup
hipError_t launch_far_reduce(const FarDesc* descs, const WgMap* map, int64_t nwg, hipStream_t s);

} // namespace hank
