// kernels.h -- argument blocks and launchers of the device kernels.
//
// Work is described by small device-resident descriptors so that one launch
// can cover the same kind of work for many transforms (several right-hand
// sides, several requests of a batch).  A launch gets one descriptor per
// transform (or per far-field block of a transform) with the offset of its
// first workgroup in the grid; a workgroup finds its descriptor by binary
// search over those offsets, so the host work per call does not grow with
// the number of workgroups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.h"

namespace hank {

// z~_kn = pi K_k N_n / D with K_k = ar k + br, N_n = ac n + bc; r^_k = K_k/Dr,
// w^_n = pi N_n / Qc.  pi/D is carried as hi + lo.
struct GridArgs {
    int64_t ar, br, ac, bc, D, Dr, Qc;
    double pi_Qc, piD_hi, piD_lo, invD, invQc;
    int32_t row_pert, col_pert;
    int32_t lean, pad; // lean: the near field's per-entry budget is at least 1.25e-10 (eps >= 1e-9)
};

// columns of one near-field tile (its coefficients are staged in LDS)
constexpr int NEAR_TILE_COLS = 2048;

// Near-field kernel variant of a block of 64 columns of a tile, chosen on
// the host from bounds on z over the block and the near field's share of the
// error budget: NV_SMALL only z < 20 (tabulated Taylor pieces), NV_MIX* both
// branches (each lane takes its own; the Hankel side with 12 or 6 pairs),
// NV_M* only z >= 20 with 2..12 Hankel pairs.
// NV_*8: the same with the tabulated small-argument pieces truncated to 8 terms
// (error below 6.2e-10, for per-entry budgets from 1.25e-9 up; the
// multiple-right-hand-side kernel runs them in full).
// NV_*R: the same with the residual phase factor e^{i rho}, rho = (e_k + r^_k) b_n,
// taken to first order, 1 + i rho, for blocks where rho <= sqrt(eps/6.4): the
// dropped terms are below rho^2/2 times the amplitude (<= 0.2 at z >= 20), so
// below eps/64 per entry.
enum NearVariant {
    NV_SMALL = 0, NV_MIX12, NV_MIX6, NV_M2, NV_M3, NV_M4, NV_M6, NV_M8, NV_M12,
    NV_SMALL8, NV_MIX12_8, NV_MIX6_8, NV_M2R, NV_M3R, NV_M4R, NV_MIX6_8R, NV_COUNT
};
static_assert(NV_COUNT <= 16, "variant codes are 4 bits");

// near-field work item of a plan: rows [k0, k0+nk) x columns [n0, n1).  Its
// partial sums (nrhs x 64) sit in slot `slot` of the transform's partial
// area.  bvar: the variant of column block b (columns n0 + 64b ...) in bits
// 4(b%8).. of bvar[b/8].
struct NearTile {
    int64_t k0, n0, n1, slot;
    int32_t nk;
    int32_t sole; // the only tile of its rows: k_near writes f itself (the other kernels ignore it)
    uint32_t bvar[4];
};

// rows [k0, k0+nk) of a plan own the partial slots [slot0, slot0+ntiles)
struct RowTile {
    int64_t k0, slot0, ntiles;
    int32_t nk, pad;
};

// One transform's near field in a launch: grid, coefficient columns
// c + j*ldc and outputs f + j*ldo (j < nrhs), root offsets b, DHT row
// perturbations e, the plan's tiles and row tiles (device), the grid offsets
// of its first tile (tile_start, within the launch) and first row tile
// (rt_start), and the start of its partial area (pbase; slot s of it at
// pbase + s*nrhs*64).  With one right-hand side the reduce gives each row
// tile wpr waves (1, or 4 when a row tile has more than 4 tiles), the first
// of them at wave wv_start of its launch (a multiple of 4 when wpr = 4).
struct NearProb {
    GridArgs G;
    const double* c;
    const double* b;
    const double* e;
    double* f;
    const NearTile* tiles;
    const RowTile* rts;
    int64_t ldc, ldo, tile_start, rt_start, pbase, wv_start;
    int32_t nrhs, nu;      // nu > 0: Schlomilch of order nu (k_near_nu, one right-hand side)
    const double* nutab;   // the plan's J_nu table (build_nu_table), nu > 0 only
    int32_t mnu;           // Hankel pairs k_near_nu needs at z >= 20 + nu/2 (<= NU_HANKEL_PAIRS)
    int32_t wpr;
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
// (rhs, chunk) item.  With nchunk > 1 pass C leaves chunk sums in
// part[(j * nchunk + chunk) * nrows + k'] and k_far_reduce adds them to f in
// chunk order; with nchunk == 1 pass C adds into f itself.  wg_ac, wg_b,
// wg_r: grid offsets of the descriptor's first workgroup in the column
// passes (L1/8 per item), pass B (ceil(L2/rows) per item) and the chunk
// reduction (ceil(nrows/256) per rhs).
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
    int64_t wg_ac, wg_b, wg_r;
    int32_t nrhs, nchunk, gchunk;
    // workgroups of pass B (the FP64 row kernel) per (item, row): each takes
    // its share of the chunk's groups (0 or 1: all of them)
    int32_t bsplit;
    // Blocks of at most L1 = 4096 columns on the FP64 wave-column/row kernels:
    // pass A stores only each column's one nonzero input, x0[j][g][j1] (j1 <
    // ncols), and pass B forms its rows from it; x0off is its offset in the
    // work area (-1: not used), x0 the address.
    int64_t x0off;
    void* x0;
};

hipError_t upload_tables(const DeviceTables& t);

// Size of the static device workspace of the allocation-free entry point, and
// its address on the current device (hipGetSymbolAddress, once per device).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(256) << 20; // HANK_NOALLOC_SCRATCH_BYTES of hank.h
hipError_t noalloc_scratch(void** ptr);
// b[n-1] = j_{0,n} - (n-1/4) pi for n <= nmax (b may be null) and, if v is
// given, v[n-1] = 2/J_1(j_{0,n})^2 for n <= nv (nv <= nmax)
hipError_t launch_roots(int64_t nmax, double* b, int64_t nv, double* v, hipStream_t s);
// dst = src * v elementwise (N entries), also divided by j_{0,N+1}^2 when final
// (b holds N+1 root offsets); dst may equal src
hipError_t launch_dht_scale(int64_t N, const double* v, const double* b, const double* src, double* dst,
                            bool final, hipStream_t s);
hipError_t launch_dht_e(int64_t N, const double* b, double* e, hipStream_t s);
hipError_t launch_j0(const double* z, int64_t n, double* out, hipStream_t s);
// Near field of nprob transforms with ntiles tiles in all: single
// right-hand-side transforms (k_near) and transforms of 2..64 right-hand
// sides (k_near_multi: J_0 evaluated once per entry as the A operand of
// FP64 MFMA); then f = sum of the partials, nrt row tiles in all: those of
// the problems with one right-hand side (the first ones) in nwv1 waves, the
// others from row tile nrt1 on.  k_near writes the rows of a tile that is the
// only one of its row tile (NearTile::sole) itself, and the order-0
// single-right-hand-side problems list only their other row tiles.
hipError_t launch_near(const NearProb* probs, int32_t nprob, int64_t ntiles, double* partial, hipStream_t s);
// near field of order nu > 0 (one right-hand side per problem)
hipError_t launch_near_nu(const NearProb* probs, int32_t nprob, int64_t ntiles, double* partial, hipStream_t s);
hipError_t launch_near_multi(const NearProb* probs, int32_t nprob, int64_t ntiles, double* partial, hipStream_t s);
hipError_t launch_near_reduce(const NearProb* probs, int32_t nprob, int64_t nwv1, int64_t nrt1, int64_t nrt,
                              const double* partial, hipStream_t s);
hipError_t launch_chirp_spectrum(const FarArgs& A, bool fp32, void* work, void* H, hipStream_t s);
// Columns per workgroup of the column passes (A, C) for column FFTs of L2
// points: 128-byte row segments (8 FP64 or 16 FP32 columns) for
// 64 <= L2 < 512, 8 otherwise (the split keeps L1 >= L2, so L1 >= 8 columns
// always, >= 16 from L2 = 64); HANK_COLW_BIG = 4 halves the FP64 workgroup's
// LDS from L2 = 512 on.
#ifndef HANK_COLW_BIG
#define HANK_COLW_BIG 8
#endif
__host__ __device__ constexpr int col_width(int L2, bool fp32) {
    return L2 >= 512 ? (fp32 ? 8 : HANK_COLW_BIG) : (fp32 && L2 >= 64 ? 16 : 8);
}

// which: 0 pass A (inputs + column FFTs), 1 pass B (row FFT x H^ x inverse), 2 pass C (epilogue).
// All ndesc descriptors of one launch share fp32 and the FFT split (L1, L2);
// nwg is the grid size of that pass.
// workgroups per item of the column passes (L1/8) and of pass B
int32_t far_rows_per_wg(int32_t L1);
hipError_t launch_far_pass(int which, bool fp32, int32_t L1, int32_t L2, const FarDesc* descs, int32_t ndesc,
                           int64_t nwg, hipStream_t s);
// f += sum over chunks of part, 256 rows per workgroup
hipError_t launch_far_reduce(const FarDesc* descs, int32_t ndesc, int64_t nwg, hipStream_t s);

} // namespace hank
