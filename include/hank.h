/*
 * hank.h -- C ABI of the MI355X (gfx950) library for fast order-0 Bessel sums
 *
 *     f_k = sum_{n=1}^{N} c_n J_0(r_k w_n),   1 <= k <= N,
 *
 * after A. Townsend, "A fast analysis-based discrete Hankel transform using
 * asymptotic expansions" (Sec. 1, eq. (2)).  Three tasks:
 *
 *   Schlomilch expansion     w_n = n pi,        r_k = (k-1)/(N-1)      (Sec. 4)
 *   Fourier-Bessel expansion w_n = j_{0,n},     r_k = (k-1)/(N-1)      (Sec. 5)
 *   discrete Hankel transform of order 0
 *                            w_n = j_{0,n},     r_k = j_{0,k}/j_{0,N+1} (Sec. 6, eq. (DHT))
 *
 * with j_{0,n} the n-th positive root of J_0.  The Schlomilch and
 * Fourier-Bessel tasks also exist on the paper's own grid r_k = k/N, and both
 * may be of integer order nu <= 8 (J_nu in place of J_0; hank_options.nu).
 * The inverse DHT is hank_dht0_inverse.
 *
 * The result is accurate to O(eps * sum_n |c_n|) (Sec. 1): the library picks
 * every algorithmic parameter (number of asymptotic terms, block partition,
 * Neumann/Taylor truncation) from eps and N by the paper's error bounds.
 *
 * Conventions shared by every entry point:
 *   - c and out are DEVICE pointers to FP64 arrays owned by the caller;
 *     c has N entries (or ldc*nrhs), out has N entries (or ldo*nrhs).
 *     Column j of a multi-right-hand-side call starts at c + j*ldc and
 *     out + j*ldo.  out must not overlap c.
 *   - stream is a hipStream_t (NULL: the default stream).  Calls enqueue work
 *     on it and return without waiting; out is valid once the stream reaches
 *     that point.  The first call for a given (task, N, eps, options) builds a
 *     plan (host parameter selection, device root tables, chirp spectra) and
 *     synchronises the stream once while doing so; later calls reuse it.
 *   - On any error nothing is written to out and the call returns a non-zero
 *     status; hank_last_error() gives a message (per calling thread).
 *   - Calls from several host threads are serialised inside the library.
 *     Results are deterministic: the same inputs give bitwise the same out.
 */
#ifndef HANK_H
#define HANK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HANK_OK = 0,
    HANK_EINVAL = 1,       /* bad argument (null pointer, N, eps, overlap, ...) */
    HANK_ENOMEM = 2,       /* device allocation failed (nothing was written)     */
    HANK_EDEVICE = 3,      /* a HIP runtime call failed                           */
    HANK_EUNSUPPORTED = 4  /* valid request outside what this build supports      */
} hank_status;

/* Task codes for the generic entry points. */
enum {
    HANK_TASK_SCHLOMILCH = 0,            /* w_n = n pi,     r_k = (k-1)/(N-1)        */
    HANK_TASK_FOURIER_BESSEL = 1,        /* w_n = j_{0,n},  r_k = (k-1)/(N-1)        */
    HANK_TASK_DHT0 = 2,                  /* w_n = j_{0,n},  r_k = j_{0,k}/j_{0,N+1}  */
    HANK_TASK_SCHLOMILCH_PAPER_GRID = 3, /* w_n = n pi,     r_k = k/N   (Sec. 4)     */
    HANK_TASK_FOURIER_BESSEL_PAPER_GRID = 4 /* w_n = j_{0,n}, r_k = k/N (Sec. 5)     */
};

typedef void* hank_stream_t; /* a hipStream_t */

/* Options; pass NULL for the defaults (all zero). */
typedef struct {
    int32_t plan_mode;  /* 0: GPU-tuned partition and per-block truncation (default)
                           1: the paper's parameters (Table 4, K and T of Sec. 5.1/6)
                           2: as 1 with P = 0: one far block Q_1 and everything else
                              summed directly, the O(N^{3/2}) scheme of Sec. 3.3   */
    int32_t precision;  /* 0: auto -- FP32 transform bulk iff eps >= 1e-6, else FP64
                           1: FP64 bulk   2: FP32 bulk (any eps; accuracy then limited) */
    int32_t direct;     /* 1: skip the fast method and sum every entry on the GPU (the
                           O(N^2) direct-summation baseline of Sec. 2.1)             */
    int32_t prefer_far; /* 1: tuned mode prices direct entries 1000x higher, so the
                           fast method is used wherever it is valid (small N tests)  */
    int32_t nrhs;       /* hank_plan_info / hank_plan_block only: right-hand sides to
                           plan for (0 means 1).  The transform calls plan for their
                           own nrhs (rounded up to a power of two, at most 64): with
                           several right-hand sides J_0 is evaluated once per direct
                           entry, so the tuned partition moves toward the near field */
    int32_t M;          /* plan modes 1 and 2: number of asymptotic terms M of eq.
                           (HankelExpansion) in place of Table 4's max(floor(0.3 ln
                           (1/eps)), 3), 1 <= M <= 20; s_{nu,M}(eps), alpha and P
                           follow from it (the M sweep of Sec. 4.3).  0: Table 4.
                           HANK_EINVAL in mode 0, outside [0, 20], or below the
                           smallest M whose remainder bound covers the highest
                           Bessel order the plan uses (M >= mu_max/2 - 1/4)      */
    int32_t nu;         /* Schlomilch and Fourier-Bessel tasks: order of the sum,
                           f_k = sum_n c_n J_nu(r_k w_n), 0 <= nu <= 8 (Sec. 4, and
                           eq. (FourierBessel): still at the roots of J_0)          */
    int32_t shift;      /* Schlomilch tasks only: w_n = (n + shift) pi, 0 <= shift <=
                           1024 (Remark 4.1; the paper's (n + nu) pi is shift = nu).
                           nu on the DHT, shift on a task other than Schlomilch, or
                           either out of range: HANK_EINVAL.
                           With nu > 0 the near field sums one right-hand side at a
                           time (several are accepted and run column by column)    */
} hank_options;

/* ---- The three transforms (Sec. 4, 5, 6) ---------------------------------
 * c: device, N doubles.  out: device, N doubles.  eps in [1e-15, 1).
 * Schlomilch and Fourier-Bessel need N >= 2 (their grid (k-1)/(N-1)), the
 * DHT N >= 1.  N <= 2^24.
 * Errors: HANK_EINVAL for a null pointer, N out of range, eps not finite or
 * outside [1e-15, 1), or out overlapping c; HANK_ENOMEM, HANK_EDEVICE. */
hank_status hank_schlomilch(const double* c, int64_t N, double eps, double* out,
                            hank_stream_t stream);
hank_status hank_fourier_bessel(const double* c, int64_t N, double eps, double* out,
                                hank_stream_t stream);
hank_status hank_dht0(const double* c, int64_t N, double eps, double* out,
                      hank_stream_t stream);

/* Generic form: any task code above, nrhs >= 1 right-hand sides stored as
 * columns (c + j*ldc, out + j*ldo, ldc >= N, ldo >= N), options may be NULL. */
hank_status hank_transform(int32_t task, const double* c, int64_t N, int64_t nrhs,
                           int64_t ldc, double eps, double* out, int64_t ldo,
                           const hank_options* options, hank_stream_t stream);

/* ---- Allocation-free form of hank_transform ---------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * transform as hank_transform, with its workspace (descriptors, near-field
 * partial sums, far-field chunk sums and work buffer) taken from a static
 * device array of HANK_NOALLOC_SCRATCH_BYTES that the library holds on each
 * GPU it runs on until the process ends.  It calls no hipMalloc, hipFree or
 * other allocating routine, so it builds no plan: the plan for (task, N, eps,
 * options, nrhs rounded up to a power of two) must be cached already, e.g. by
 * one hank_transform call with the same arguments; otherwise it returns
 * HANK_EUNSUPPORTED.  A transform whose workspace does not fit the array, even
 * with the far field cut into single-group waves, also returns
 * HANK_EUNSUPPORTED (large nrhs at large N).  Far-field groups may be summed
 * in other waves than by hank_transform, so results agree with it to rounding,
 * not bitwise.  Every call on a GPU shares that GPU's array: calls that can
 * overlap on one GPU (different streams, several threads) race and must be
 * ordered by the caller; calls on one stream are ordered by it.  Other
 * arguments, errors and the effect on out as for hank_transform. */
#define HANK_NOALLOC_SCRATCH_BYTES (256ll << 20)
hank_status hank_transform_noalloc(int32_t task, const double* c, int64_t N, int64_t nrhs, int64_t ldc,
                                   double eps, double* out, int64_t ldo, const hank_options* options,
                                   hank_stream_t stream);

/* ---- Batched submission ---------------------------------------------------
 * Enqueue many independent transforms (different tasks, N, eps, nrhs) at once;
 * their work is merged into shared launches.  Each request follows the
 * conventions of hank_transform.  All requests are validated before any work
 * is enqueued; on error nothing is enqueued. */
typedef struct {
    int32_t task;
    int32_t precision; /* as hank_options.precision */
    int64_t N;
    int64_t nrhs;
    int64_t ldc, ldo;
    double eps;
    const double* c;
    double* out;
    int32_t nu;    /* as hank_options.nu (order; Schlomilch and Fourier-Bessel) */
    int32_t shift; /* as hank_options.shift (Schlomilch)                         */
} hank_request;

hank_status hank_batch(const hank_request* reqs, int64_t count, hank_stream_t stream);

/* A batch captured once as a HIP graph and replayed without host work: the
 * same requests (the same c and out pointers; their contents may change
 * between launches) on the stream of each launch.  The graph owns its
 * workspace, so launches of different graphs and ordinary calls do not share
 * buffers; launches of one graph must not overlap each other.  Plans are built
 * (on `stream`) at creation; the graph keeps pointers into the plan cache, so
 * hank_cache_clear fails while graphs exist.  Destroy a graph only after its
 * last launch has completed.  Errors as for hank_batch (nothing is captured). */
typedef struct hank_graph hank_graph;
hank_status hank_batch_graph_create(const hank_request* reqs, int64_t count, hank_stream_t stream,
                                    hank_graph** out);
hank_status hank_batch_graph_launch(hank_graph* graph, hank_stream_t stream);
hank_status hank_batch_graph_destroy(hank_graph* graph);

/* ---- Serving: continuous batching ---------------------------------------------
 * A server owns a worker thread and a stream.  Submitted requests become
 * eligible at their arrival time (seconds after hank_server_start; a negative
 * arrival means "now"), wait in a queue, and are admitted in arrival order into
 * batches while (a) the device bytes of the admitted, unfinished requests stay
 * within budget_bytes and (b) a batch holds at most max_batch requests.  Up to
 * two batches are in flight on the stream, so a new batch is enqueued while
 * the previous one runs.  A request that arrives while max_pending requests
 * are already waiting is rejected (state 3) and never run.  Latency is
 * completion minus arrival (host clock).  max_batch = 1 gives the plain
 * one-request-at-a-time form on the same path.  Requests follow the
 * conventions of hank_transform; their buffers must stay valid until done.
 * Plans: planner threads (HANK_SERVE_PLANNERS, default min(8, cores/2)) build
 * the plan of each arrived request whose plan is not cached -- host planning
 * and device tables on their own streams, while batches run -- and a request
 * is admitted once its plan is ready; its plan stays pinned in the cache until
 * its batch completes, and its device bytes (workspace and plan) count against
 * budget_bytes while in flight.  A request whose plan cannot be built, or
 * whose device bytes exceed budget_bytes, is rejected.  hank_server_warm builds a request's plan in advance. */
typedef struct hank_server hank_server;

typedef struct {
    int64_t submitted, completed, rejected, batches;
    double mean_batch;                 /* requests per batch                      */
    double p50_ms, p90_ms, p99_ms, max_ms, mean_ms; /* latency of completed requests */
    double wall_s;                     /* first arrival to last completion        */
    double throughput;                 /* completed requests per second of wall_s */
    int64_t plans_built;               /* plans the planner threads built          */
} hank_server_summary;

hank_status hank_server_create(int64_t budget_bytes, int32_t max_batch, int64_t max_pending,
                               hank_stream_t stream, hank_server** out);
hank_status hank_server_warm(hank_server* srv, const hank_request* req);
hank_status hank_server_submit(hank_server* srv, const hank_request* req, double arrival_s, int64_t* ticket);
hank_status hank_server_start(hank_server* srv);
hank_status hank_server_drain(hank_server* srv);
/* state: 0 waiting, 1 admitted, 2 done, 3 rejected */
hank_status hank_server_status(hank_server* srv, int64_t ticket, int32_t* state, double* latency_ms);
hank_status hank_server_stats(hank_server* srv, hank_server_summary* out);
hank_status hank_server_destroy(hank_server* srv);

/* ---- FFT autotuner ---------------------------------------------------------
 * Times the far-field passes on a synthetic block for each FFT length
 * L = 2^10 .. 2^23 and the splits L = L1 x L2 the kernels support near the
 * default, and installs the fastest split per length for plans built from
 * then on (cached plans keep theirs; hank_cache_clear rebuilds).  chosen, if
 * not NULL, receives log2(L2) per log2(L) for indices 10..23 (24 entries).
 * Runs on `stream` and synchronises it; about a second. */
hank_status hank_autotune(hank_stream_t stream, int32_t* chosen);
/* Back to the default split for plans built from then on. */
hank_status hank_autotune_reset(void);
/* The installed splits as a text file, one "log2(L) log2(L2)" line per tuned
 * length: hank_autotune_save writes them to path (host only); hank_autotune_load
 * installs those of path for plans built from then on, so that a process can
 * reuse an earlier process's tuning.  A file that cannot be read or written, or
 * a line that is not a split the kernels support (L1 >= L2, L1 <= 8192,
 * 2^6 <= L <= 2^23), returns HANK_EINVAL; on a bad line nothing is installed. */
hank_status hank_autotune_save(const char* path);
hank_status hank_autotune_load(const char* path);

/* ---- Library state --------------------------------------------------------- */
const char* hank_last_error(void);   /* message of the calling thread's last error */
hank_status hank_cache_clear(void);  /* drop every cached plan (device sync first)  */
int64_t hank_cache_bytes(void);      /* device bytes held by cached plans          */
/* Limit of the plan cache in device bytes (default 16 GiB; 0 keeps nothing
 * that is not in use).  Past it the least recently used plans are freed --
 * not those pinned by a live batch graph or by a server request that is
 * waiting or running, nor those of the call in progress -- down to three
 * quarters of the limit.  Freeing synchronises the device.  A freed plan is
 * built again on its next use, with bitwise the same results.
 * HANK_EINVAL for a negative limit. */
hank_status hank_cache_limit(int64_t bytes);

/* ---- Kernel timing -----------------------------------------------------------
 * hank_profile(1) brackets every kernel launch of later transforms with HIP
 * events on the caller's stream (and clears the counters); hank_profile(0)
 * stops.  hank_profile_report waits for the recorded events and returns one
 * entry per kernel kind: launches, summed duration, and the ALGORITHMIC bytes
 * (what the kernel must read and write at minimum) and work units (near field:
 * matrix entries; far-field passes: FFT points x groups) of those launches.
 * out may hold max entries; *count receives the number of kinds. */
typedef struct {
    char name[24];
    int64_t launches;
    double total_ms;
    double bytes;
    double work;
} hank_kernel_stat;

hank_status hank_profile(int32_t enable);
hank_status hank_profile_report(hank_kernel_stat* out, int32_t max, int32_t* count);

/* ---- Parameter selection, exposed for inspection (host only, no GPU) -----
 * s_{nu,M}(eps): four fixed-point steps on the remainder bound (Sec. 3.1). */
double hank_param_s(int32_t nu, int32_t M, double eps);
/* t_{nu,T}(eps) of Sec. 3.2. */
double hank_param_t(int32_t nu, int32_t T, double eps);
/* 2 (eps/5.2)^(1/K) / e, the Neumann perturbation limit of Lemma 3.1. */
double hank_param_neumann(int32_t K, double eps);
/* p_K(eps) (eq. (pKe)) and q_T(eps) (eq. (qTe)). */
double hank_param_pK(int32_t K, double eps);
double hank_param_qT(int32_t T, double eps);

/* Summary of the plan the library would use (host only, no GPU). */
typedef struct {
    int32_t M;             /* asymptotic terms (Table 4) of the paper rule          */
    int32_t K, T;          /* Neumann and Taylor truncation (Sec. 5.1 / 6); 0 if none */
    int32_t P;             /* partitions (Table 4; tuned mode: strips per side)     */
    int32_t nblocks;       /* far-field blocks                                      */
    double s;              /* s_{nu,M}(eps) used for the partition                  */
    double alpha, beta;    /* Table 4                                                */
    int64_t near_entries;  /* matrix entries summed directly                        */
    int64_t far_transforms;/* complex chirp-z transforms over all blocks            */
    int64_t fft_points;    /* sum over transforms of their FFT length               */
    double fft_bytes;      /* algorithmic bytes of the far-field passes             */
    int32_t first_direct;  /* columns (FB) or rows (DHT) summed directly, paper rule */
    int32_t bulk_fp32;     /* 1 if the transform bulk runs in FP32                  */
    int32_t fp32_transforms; /* transforms run in FP32 (all with bulk_fp32; with an
                              FP64 bulk, those whose contribution is small enough
                              that FP32 rounding stays within eps/8)            */
    double model_s;        /* GPU seconds of one transform by the planner's cost
                              model (for the nrhs the plan is balanced for)    */
} hank_plan_summary;

hank_status hank_plan_info(int32_t task, int64_t N, double eps, const hank_options* options,
                           hank_plan_summary* out);

/* Far-field block k of that plan (0 <= k < nblocks): rows [row0,row1] and
 * columns [col0,col1] (1-based, inclusive), FFT length and group count. */
typedef struct {
    int64_t row0, row1, col0, col1;
    int64_t fft_len;
    int32_t groups;
    int32_t terms;
    double zmin; /* smallest z = r_k w_n inside the block */
    int32_t fft_l1, fft_l2; /* split fft_len = l1 * l2: row FFTs of l1, column FFTs of l2 points */
} hank_block_info;

hank_status hank_plan_block(int32_t task, int64_t N, double eps, const hank_options* options,
                            int32_t k, hank_block_info* out);

/* ---- Inverse DHT (Sec. 6, eqs. (selfinverse) and (inverseTest)) ----------
 * The DHT is its own inverse up to diagonal scalings as N grows:
 *     (1/j_{0,N+1}^2) J D_v J D_v ~ I,   J = J_0(j_0 j_0^T / j_{0,N+1}),
 *     v_n = 2 / J_1(j_{0,n})^2.
 * hank_dht0_inverse applies c = (1/j_{0,N+1}^2) D_v J D_v f, the inverse of
 * hank_dht0 in that sense: f and c are device FP64 arrays of N entries that
 * must not overlap; the transform J runs by the fast method with accuracy eps,
 * so |c_k - exact_k| = O(eps * v_k/j_{0,N+1}^2 * sum_n v_n |f_n|).  The plan is
 * hank_dht0's (same cache entry); the call enqueues a scaling, the transform
 * and a scaling on stream.  Errors as for hank_dht0. */
hank_status hank_dht0_inverse(const double* f, int64_t N, double eps, double* c, hank_stream_t stream);
/* v[n-1] = 2 / J_1(j_{0,n})^2 for n = 1..N (the weights above), computed on
 * the GPU with the roots (J_1 at a root is -J_0' from the last Newton step).
 * v: device, N doubles.  HANK_EINVAL for a null pointer or N < 1. */
hank_status hank_dht0_weights(int64_t N, double* v, hank_stream_t stream);

/* ---- Device building blocks, exposed for testing ------------------------- */
/* b[n-1] = j_{0,n} - (n - 1/4) pi for n = 1..nmax (Lemma 3.2), computed on the
 * GPU by McMahon's expansion and Newton's method.  b: device, nmax doubles. */
hank_status hank_root_offsets(int64_t nmax, double* b, hank_stream_t stream);
/* out[i] = J_0(z[i]) by the library's device evaluator.  z, out: device. */
hank_status hank_j0(const double* z, int64_t count, double* out, hank_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* HANK_H */
