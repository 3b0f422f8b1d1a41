/*
 * rtg.h -- all-pairs r-nearest-neighbours by randomly transformed grids (RTG)
 * on one AMD Instinct MI355X (gfx950).
 *
 * The operation (Kleinbort, Salzman & Halperin, "Efficient high-quality
 * motion planning by fast all-pairs r-nearest-neighbors"):
 *   given n points P in R^d and a radius r, report pairs p,q of P with
 *   ||p - q|| <= r (the all-pairs r-NN query, Sec. I).  RTG answers it
 *   approximately (Sec. III, Alg. "Randomly Shifted Grids" and its
 *   random-orientation variant): for each of k grids of cell side alpha * r,
 *   with a random orientation R_t and a uniform random shift u_t, every point
 *   goes to the cell floor((R_t p) / (alpha r) + u_t); every pair of points in
 *   a common cell is tested and reported when its distance is at most r; the
 *   union over the k grids is reported once per pair (Sec. III-B).  The
 *   paper's m is k here and its cell-size factor c~ is alpha.
 *
 * Exactness contract.  For given transforms the reported pair set is a
 * deterministic function of the inputs and equals, bit for bit, the set that
 * the FP64 definition gives: cells from FP64 arithmetic in a fixed order with
 * no FMA, and the test s <= r*r where s sums ((double)p_l - (double)q_l)^2 in
 * axis order.  The GPU screens pairs in FP32 and re-tests in that FP64 order
 * every pair whose FP32 squared distance lies within a relative 2^-16 of r^2,
 * so no decision differs from the FP64 one.  Under the MR-metric
 * (RTG_ROBOTS) the test is sum_b sqrt(s_b) <= r, s_b each robot's squared
 * displacement summed as above, square roots correctly rounded, sum in robot
 * order; the FP32 screen then only rejects pairs beyond r in the Euclidean
 * sense, and every other pair is decided in FP64.
 *
 * Output.  A CSR neighbour list in device memory: row_ptr[n+1] (int64) and
 * col[nnz] (int32); row i lists its neighbours in ascending order.  By default
 * every pair is stored in both rows (the layout that answers multiple r-NN
 * queries, Sec. III-B); with RTG_UPPER_ONLY row i holds only j > i.
 *
 * Conventions.  Every call returns an rtg_status.  Out-parameters are written
 * only on RTG_OK.  Nothing throws across this interface.  Inputs stay owned by
 * the caller.  Results are owned by the context until rtg_release (or
 * rtg_destroy).  A context belongs to one device and one host thread, except
 * that rtg_submit / rtg_poll / rtg_release may be called from any thread.
 */
#ifndef RTG_H
#define RTG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rtg_status {
  RTG_OK = 0,
  RTG_EAGAIN = 1,   /* submitted request not finished yet                      */
  RTG_EINVAL = -1,  /* bad argument (see each call)                            */
  RTG_ENOMEM = -2,  /* the work does not fit the context's device-memory budget */
  RTG_ERANGE = -3,  /* a cell coordinate |y| >= 2^31, r*r outside            */
                    /* [2^-100, 2^120], or too few key bits for this alpha, d  */
  RTG_EDEVICE = -4, /* a HIP call failed; the context is unusable             */
  RTG_ENOENT = -5   /* unknown ticket or result handle                        */
} rtg_status;

enum {
  RTG_NO_ROTATE = 1u,  /* shift-only grids (the paper's first algorithm)        */
  RTG_UPPER_ONLY = 2u, /* store each pair once, in the row of its smaller index */
  RTG_DEDUP_SORT = 4u,   /* remove repeats by sorting all candidates (every    */
                         /* grid's pairs) and dropping equal neighbours,        */
                         /* instead of the default first-owner rule            */
  RTG_DEDUP_BITMAP = 8u  /* remove repeats with one bit per unordered pair of  */
                         /* each instance (the upper triangle, n(n-1)/2 bits;   */
                         /* the paper's bitset of Sec. III-B): every grid's     */
                         /* pairs set their bit, the first arrival is kept.     */
                         /* When a pass's bitmaps exceed 4 GiB or a quarter of  */
                         /* the free budget, the first-owner rule runs instead. */
                         /* Every rule gives the same result; SORT and BITMAP   */
                         /* together are RTG_EINVAL.                            */
};

/* The MR-metric of the multi-robot experiments (Sec. IV-C): RTG_ROBOTS(b) in
 * flags, b in [2, d] dividing d, reads each point as the configuration of b
 * robots of d / b consecutive axes each, and the distance of two
 * configurations as the sum of the distances the robots move (each robot's
 * Euclidean displacement).  The grids are the Euclidean ones: since that sum
 * is at least the Euclidean distance, every MR neighbour is a Euclidean
 * neighbour, and only the pair test changes.  b = 0 or 1: Euclidean.  Any
 * other b, or a flag bit this header does not define, is RTG_EINVAL. */
#define RTG_ROBOTS_SHIFT 8
#define RTG_ROBOTS_MASK 0xFF00u
#define RTG_ROBOTS(b) ((uint32_t)(b) << RTG_ROBOTS_SHIFT)

typedef struct rtg_ctx rtg_ctx;

/* A device-resident neighbour list.  row_ptr and col point into the
 * context's device memory and stay valid until rtg_release(handle). */
typedef struct rtg_csr {
  int64_t n;        /* rows                                         */
  int64_t nnz;      /* entries in col                               */
  int64_t *row_ptr; /* device, n+1 entries, row_ptr[0] = 0         */
  int32_t *col;     /* device, nnz entries (NULL when nnz = 0)     */
  uint64_t handle;  /* pass to rtg_release                          */
  int64_t pairs;    /* unordered pairs reported (nnz/2 symmetric)  */
} rtg_csr;

/* One all-pairs query, for the batched and the request-loop entry points. */
typedef struct rtg_query {
  const float *points; /* device, row-major [n][d] FP32                */
  int64_t n;
  int32_t d;
  double r;
  int32_t k;
  double alpha;
  uint64_t seed;
  uint32_t flags;
} rtg_query;

/* Kernels (or kernel groups) whose launches the stats count and, when
 * timing is on for them, time with HIP events on the context's stream. */
enum {
  RTG_K_STAGE = 0,         /* AoS -> SoA copy, finiteness, bounding box      */
  RTG_K_KEYS = 1,          /* FP64 cell keys                                */
  RTG_K_KEY_HIST = 2,      /* digit histogram, one launch per key-sort pass  */
  RTG_K_KEY_SCATTER = 3,   /* LDS-staged scatter, one launch per pass        */
  RTG_K_CELLS = 4,         /* runs of equal keys, tile-pair counts           */
  RTG_K_PAIRS = 5,         /* same-cell pair tests and output                */
  RTG_K_PAIR_HIST = 6,     /* digit histogram of the pair sort               */
  RTG_K_PAIR_SCATTER = 7,  /* scatter of the pair sort                       */
  RTG_K_UNIQUE = 8,        /* removal of repeated pairs (sort-unique, bitmap)  */
  RTG_K_CSR = 9,           /* neighbour-list build (incl. transposed sort)   */
  RTG_K_SCAN = 10,         /* prefix sums                                    */
  RTG_K_GATHER = 11,       /* cell members' coordinates by sorted position   */
  RTG_K_COMPACT = 12,      /* pair output made contiguous; MR-metric filter  */
  RTG_NKERNELS = 13
};
#define RTG_TIME_PHASES (1u << 31) /* rtg_set_timing: per-phase events too */

/* Counters of the last completed call on a context (for measurement). */
typedef struct rtg_stats {
  int64_t n, d, k;
  int64_t point_transforms;  /* n * k                                          */
  int64_t cells;             /* cells holding >= 2 points, summed over grids   */
  int64_t tests;             /* same-cell pairs tested, summed over grids      */
  int64_t candidates;        /* pairs within r before de-duplication           */
  int64_t band_rechecks;     /* pairs re-tested in FP64                        */
  int64_t unique_pairs;      /* unordered pairs reported                       */
  int32_t key_bits;          /* bits of the sorted cell key                    */
  int32_t key_passes;        /* radix passes over the cell keys                */
  int32_t pair_bits;         /* bits of a packed (i,j) pair                    */
  int32_t transforms_per_sort; /* grids grouped in one sort                    */
  /* Device time per phase in milliseconds (0 unless timing is on). */
  double ms_stage, ms_keys, ms_key_sort, ms_cells, ms_pairs, ms_pair_sort, ms_unique, ms_csr,
      ms_total;
  /* Per kernel id (RTG_K_*): launches, algorithmic bytes moved (the data the
   * method must read and write, summed over launches) and device time in
   * milliseconds summed over launches (0 unless timed). */
  int64_t kernel_launches[RTG_NKERNELS];
  double kernel_bytes[RTG_NKERNELS];
  double kernel_ms[RTG_NKERNELS];
  /* Request loop totals since rtg_create: requests finished and pipeline
   * passes (batches) that ran them. */
  int64_t served_requests;
  int64_t served_batches;
  /* Pair-kernel launches of the last call that screened on the matrix cores
   * (the rest used the vector screen). */
  int64_t matrix_screen_launches;
  /* Requests the request loop ran on the two-launch small-instance path
   * (since rtg_create). */
  int64_t served_small;
} rtg_stats;

/* Create a context on HIP device `device`.
 *   arena / arena_bytes: device memory the context sub-allocates for scratch
 *     and results.  If arena is NULL the context allocates arena_bytes itself
 *     (hipMalloc) and frees them in rtg_destroy; otherwise the caller keeps
 *     ownership and must keep the memory alive until rtg_destroy.
 *     arena_bytes is the context's device-memory budget (RTG_ENOMEM beyond).
 *   hip_stream: the hipStream_t all work is ordered on (NULL: the null stream).
 * Errors: RTG_EINVAL (ctx NULL, arena_bytes < 1 MiB, bad device),
 *         RTG_EDEVICE (HIP failure). */
int rtg_create(rtg_ctx **ctx, int device, void *arena, size_t arena_bytes, void *hip_stream);

/* Destroy a context: waits for outstanding work and frees every result. */
int rtg_destroy(rtg_ctx *ctx);

/* Blocking all-pairs r-NN by RTG (the paper's problem statement, Sec. I, with
 * the grids of Sec. III).
 *   points: device pointer, row-major [n][d] FP32, 4-byte aligned.
 *   n in [0, 2^31); d in [1, 64]; r > 0 finite; k >= 1; alpha > 0 finite.
 *   seed selects the k transforms (see rtg_make_transforms).
 *   flags: RTG_NO_ROTATE, RTG_UPPER_ONLY, RTG_DEDUP_SORT or RTG_DEDUP_BITMAP,
 *   RTG_ROBOTS(b).
 * n <= 1 gives an empty list.  Small Euclidean instances (n <= 4096,
 * d <= 8, n d <= 12288, k n <= 12288, k d (d + 1) <= 2048) run in two
 * launches -- up to eight workgroups per grid find its cells, test their
 * share of its pairs and keep the first grid's, then the lists are built --
 * and take the general pipeline when their keys, pairs (131072) or rows
 * (128) exceed what those launches hold; the lists are the same either
 * way, and the stats count
 * both launches under RTG_K_PAIRS with candidates = unique_pairs.  The
 * environment setting RTG_SMALL=0 turns the small path off.  Errors:
 * RTG_EINVAL (also for NaN/Inf coordinates), RTG_ERANGE, RTG_ENOMEM,
 * RTG_EDEVICE. */
int rtg_all_pairs(rtg_ctx *ctx, const float *points, int64_t n, int32_t d, double r, int32_t k,
                  double alpha, uint64_t seed, uint32_t flags, rtg_csr *out);

/* As rtg_all_pairs with caller-given transforms: R is host [k][d][d] FP64
 * (row j maps p to (R p)_j), u is host [k][d] FP64 shifts in cell units.
 * RTG_NO_ROTATE is ignored here (R is used as given). */
int rtg_all_pairs_with_transforms(rtg_ctx *ctx, const float *points, int64_t n, int32_t d,
                                  double r, int32_t k, double alpha, const double *R,
                                  const double *u, uint32_t flags, rtg_csr *out);

/* For callers that cannot allocate device memory (serving loops that must
 * not call hipMalloc, harnesses that forbid allocation): rtg_all_pairs with
 * the result written into caller buffers and every byte of device scratch
 * taken from one file-scope device array of the library, RTG_NOALLOC_BYTES
 * per device, held by each device the library runs on until the process
 * ends.  No device memory is allocated or freed and no host memory is
 * pinned during the call (the context's arena is not used either).
 *   points, n, d, r, k, alpha, seed, flags: as rtg_all_pairs.
 *   row_ptr: device, n+1 int64, 8-byte aligned, written on RTG_OK.
 *   col: device, col_capacity int32 (may be NULL when col_capacity is 0),
 *     written on RTG_OK with the nnz entries of the symmetric (or, with
 *     RTG_UPPER_ONLY, upper) lists -- the arrays rtg_all_pairs returns.
 *   nnz: host; receives the entries written, or on RTG_ENOMEM because
 *     col_capacity is too small, the entries needed (row_ptr and col are
 *     then untouched).
 * Limits: the pass's working set (about 130 bytes per point and grid plus
 * 8d + 64 per point) must fit RTG_NOALLOC_BYTES and its uploaded transforms
 * (8 k d (d+2) bytes and tables) 256 KiB; larger calls return RTG_ENOMEM
 * before any device work.  The call is blocking and per-kernel timing does
 * not apply to it.  Calls on one device share the array: calls that overlap
 * on one GPU (from different contexts of that device) race and must be
 * serialised by the caller; calls on one context are serialised by it.
 * Errors: as rtg_all_pairs; RTG_EINVAL also for a misaligned or non-device
 * row_ptr / col; RTG_EDEVICE if the array's address could not be obtained. */
#define RTG_NOALLOC_BYTES ((size_t)256 << 20)
int rtg_all_pairs_noalloc(rtg_ctx *ctx, const float *points, int64_t n, int32_t d, double r,
                          int32_t k, double alpha, uint64_t seed, uint32_t flags,
                          int64_t *row_ptr, int32_t *col, int64_t col_capacity, int64_t *nnz);

/* Many independent queries in one pass of the pipeline: every (query, grid)
 * pair is one segment of a shared key space, so each kernel launch covers all
 * queries.  outs[q] receives query q's list, identical to what rtg_all_pairs
 * returns for it alone.  One query within the small-instance limits of
 * rtg_all_pairs takes its two-launch path, as there.  On error no result is
 * kept.  Errors as rtg_all_pairs, for any query. */
int rtg_all_pairs_batched(rtg_ctx *ctx, const rtg_query *queries, int32_t nq, rtg_csr *outs);

/* Plans: rtg_all_pairs_batched repeated over queries of one fixed shape (a
 * stream of many small problems of the same sizes, each the all-pairs r-NN
 * problem of Sec. II).  rtg_plan_create records the shape of queries[0..nq)
 * -- each query's n, d, k and flags -- and validates them as
 * rtg_all_pairs_batched does; it runs nothing.  rtg_plan_run takes queries
 * of that shape (points, r, alpha and seed may differ) and returns, in
 * outs[0..nq), exactly what rtg_all_pairs_batched returns for them.  Its
 * first run gives each batch of the call a device workspace (held by the
 * plan, counted against the context's budget until rtg_plan_destroy); from
 * the second run on the pass's device-sized stretch, from the cell keys to
 * the unit descriptors, is launched as one HIP graph captured on the
 * context's stream, recaptured when a launch argument changes (another
 * cell-key layout for new data).  Per-kernel timing of those kernels
 * (rtg_set_timing) runs them as ordinary launches instead.  Runs are
 * blocking and serialised with the context's other calls.  rtg_plan_info
 * reports the graphs captured and replayed so far and the workspace bytes
 * held (a plan of one small instance runs the two-launch path of
 * rtg_all_pairs, which needs no graph: it captures nothing).  A plan belongs to its context: destroy it before the context.
 * Errors: RTG_EINVAL (NULL arguments, nq < 0, or for rtg_plan_run a shape
 * other than the plan's), and those of rtg_all_pairs_batched. */
typedef struct rtg_plan rtg_plan;
int rtg_plan_create(rtg_ctx *ctx, const rtg_query *queries, int32_t nq, rtg_plan **plan);
int rtg_plan_run(rtg_plan *plan, const rtg_query *queries, int32_t nq, rtg_csr *outs);
int rtg_plan_info(const rtg_plan *plan, int64_t *captures, int64_t *replays,
                  int64_t *workspace_bytes);
int rtg_plan_destroy(rtg_plan *plan);

/* Request loop (continuous batching).  rtg_submit copies the query's points
 * into the context before it returns (the caller may reuse its buffer) and
 * hands back a ticket; a scheduler thread admits requests while their device
 * memory fits the budget and runs every admitted request in the next pass of
 * the batched pipeline.  rtg_poll returns RTG_OK with the result once done
 * (the result then belongs to the caller's handle), RTG_EAGAIN while pending,
 * or the request's error.  Finished results count against the budget until
 * released: a request that does not fit beside them stays pending until the
 * caller releases some (or other requests' staged points are dropped), and
 * fails with RTG_ENOMEM only when it does not fit with nothing else held.
 * A request within rtg_all_pairs' small-instance limits that finds no pass
 * running runs alone on that two-launch path (rtg_stats.served_small).
 * Errors: RTG_EINVAL, RTG_ENOMEM (its working-set bound plus its points
 * exceed the whole budget), RTG_ENOENT (unknown ticket). */
int rtg_submit(rtg_ctx *ctx, const rtg_query *query, uint64_t *ticket);
int rtg_poll(rtg_ctx *ctx, uint64_t ticket, rtg_csr *out);

/* Free a result's or an index's device memory.  Errors: RTG_ENOENT. */
int rtg_release(rtg_ctx *ctx, uint64_t handle);

/* rtg_release for handles[0..count) (host array, read only) in one call,
 * e.g. the results of one rtg_all_pairs_batched.  Every known handle is
 * released; RTG_ENOENT if any was unknown.  Errors: RTG_EINVAL (ctx NULL,
 * count < 0, or handles NULL with count > 0), RTG_ENOENT. */
int rtg_release_many(rtg_ctx *ctx, const uint64_t *handles, int32_t count);

/* Query mode (an r-NN index of one point set; Sec. V suggests answering
 * queries from the grids).  rtg_index_build sorts the k grids of `points`
 * once -- the transforms, cell keys and sort of rtg_all_pairs -- and keeps
 * them, a copy of the points and their signatures in the context under
 * *index (free with rtg_release).  Arguments and errors as rtg_all_pairs;
 * flags: RTG_NO_ROTATE, RTG_ROBOTS(b) (the queries' distance test is then
 * the MR-metric's; list flags are ignored).
 *
 * rtg_index_query answers m query points (device, row-major [m][d] FP32,
 * the index's d): row s of the result lists, ascending and once each, the
 * indexed points p_i with ||p_i - q_s|| <= r that share a cell with q_s
 * under some grid of the index, decided exactly as the pairs of
 * rtg_all_pairs (FP64 cell coordinates and distances).  A query equal to an
 * indexed point reports that point.  Errors: RTG_EINVAL (also NaN/Inf
 * coordinates), RTG_ERANGE, RTG_ENOMEM, RTG_ENOENT (unknown index). */
int rtg_index_build(rtg_ctx *ctx, const float *points, int64_t n, int32_t d, double r, int32_t k,
                    double alpha, uint64_t seed, uint32_t flags, uint64_t *index);
int rtg_index_query(rtg_ctx *ctx, uint64_t index, const float *queries, int64_t m,
                    rtg_csr *out);

/* The k seeded transforms, on the host: R [k][d][d] FP64 with orthonormal rows
 * (identity with RTG_NO_ROTATE), u [k][d] FP64 in [0,1).  Transform t draws
 * from the SplitMix64 stream (Steele, Lea & Flood 2014) started at the
 * (t+1)-th output of `seed`: first the d shifts (top 53 bits / 2^53), then
 * d*d standard normals in row-major pairs (Marsaglia's polar method) whose
 * rows are orthonormalised in index order by modified Gram-Schmidt applied
 * twice.  A Gaussian matrix orthonormalised so is Haar distributed on O(d),
 * the "random orientation" of Sec. III.  Errors: RTG_EINVAL. */
int rtg_make_transforms(uint64_t seed, int32_t k, int32_t d, uint32_t flags, double *R, double *u);

/* Parameters for a target recall (Sec. III-A: the cell factor c~ = alpha
 * and the number of grids m = k trade running time against the share of
 * pairs found; Sec. V asks for choosing them automatically).
 *
 * Model: a pair at distance rho <= r, displaced along a direction u,
 * shares a cell of side c = alpha r under one randomly shifted grid with
 * probability prod_j (1 - rho |u_j| / c)_+; with random orientations that
 * probability is averaged over directions and the k grids are independent.
 * Neighbour pairs have locally uniform positions: rho has density
 * d rho^(d-1) / r^d on [0, r] and u is uniform on the sphere.  Recall is
 * E[1 - (1 - p)^k].  Cost, in units of one point under one grid, is
 * k (1 + beta nu alpha^d / (2 zeta_d)), with nu the mean number of
 * neighbours within r, zeta_d the unit-ball volume and beta the measured
 * cost of one pair test relative to one point under one grid.
 *
 * Returns the (k, alpha) of least modelled cost whose modelled recall is at
 * least target, alpha on a grid of step 1/32 in [0.5, 4]; *recall receives
 * the modelled recall.  flags: RTG_NO_ROTATE (shift-only grids).  Host only.
 * Errors: RTG_EINVAL (d outside [1, 64], target outside (0, 1),
 * mean_neighbours <= 0), RTG_ERANGE (target not reached with k <= 1024). */
int rtg_choose_params(int32_t d, double target_recall, double mean_neighbours, uint32_t flags,
                      int32_t *k, double *alpha, double *recall);

/* The modelled recall of (k, alpha) (see rtg_choose_params).  Host only. */
int rtg_model_recall(int32_t d, int32_t k, double alpha, uint32_t flags, double *recall);

/* Parameters for a target recall by measurement: the rule of the paper's
 * parameter study (Sec. IV-A, Table II: among the (m, c~) that reach the
 * success rate, the one with the fastest run), with the modelled recall of
 * rtg_choose_params in place of a brute-force count.  For every alpha in
 * {1.0, 1.05, ..., 2.5} the least k <= 128 whose modelled recall reaches
 * target_recall is timed on the caller's points (device, row-major [n][d],
 * n >= 2; median of reps calls of rtg_all_pairs with seed 0 and flags); the
 * fastest (k, alpha) is returned with its modelled recall and time in
 * milliseconds.  Errors: as rtg_all_pairs; RTG_EINVAL (target outside
 * (0, 1), reps outside [1, 100]); RTG_ERANGE (no candidate ran). */
int rtg_tune_params(rtg_ctx *ctx, const float *points, int64_t n, int32_t d, double r,
                    double target_recall, uint32_t flags, int32_t reps, int32_t *k,
                    double *alpha, double *recall, double *ms);

/* Launch settings of one pass of the pipeline, for passes of dimension d
 * whose points number in (2^(log2_points - 1), 2^log2_points].  A pass uses
 * the entry the context holds for its dimension and size, else the defaults
 * (the RTG_* environment settings read at rtg_create). */
typedef struct rtg_tuning {
  int32_t d;
  int32_t log2_points;
  int32_t tests_per_wave; /* pair kernels: a grid of about this many pair tests
                             per wavefront (1000 .. 10^7)                     */
  int32_t unit_tiles;     /* cells of at most this many 64-point tiles are one
                             work unit of the pair kernels (1 .. 64)          */
  int32_t part_threads;   /* block size of the neighbour-list partition (256 or
                             1024)                                            */
  int32_t bucket_blocks;  /* partition blocks of the neighbour-list build
                             (1 .. 4096)                                      */
  int32_t bucket_entries; /* target mean entries of a neighbour-list bucket
                             (256 .. 16384)                                   */
  int32_t sort;           /* radix sort: 0 onesweep, 1 reduce-then-scan       */
  double ms;              /* rtg_autotune: median time of the tuned workload */
} rtg_tuning;

/* The autotuner.  Times the given queries (all of one dimension d; run as
 * rtg_all_pairs_batched runs them, results released) under each candidate
 * value of each setting in turn, starting from the entry their passes use
 * now, keeps a value only when it is faster by more than 2%, and installs
 * the result for passes of that size (the points of one pass: the queries'
 * total, at most the batch size).  reps: timed calls per candidate (median),
 * 1 .. 100.  *out receives the entry.  Errors: RTG_EINVAL (mixed d, nq < 1,
 * reps out of range), and those of rtg_all_pairs_batched. */
int rtg_autotune(rtg_ctx *ctx, const rtg_query *queries, int32_t nq, int32_t reps,
                 rtg_tuning *out);
/* Install an entry (RTG_EINVAL if a field is out of range; ms is ignored). */
int rtg_set_tuning(rtg_ctx *ctx, const rtg_tuning *tuning);
/* The settings a pass of `points` points of dimension d would use. */
int rtg_get_tuning(rtg_ctx *ctx, int32_t d, int64_t points, rtg_tuning *out);
/* Write every installed entry to a JSON file, or install the entries of one
 * (rtg_create also loads the file named by RTG_TUNING_FILE).  Errors:
 * RTG_EINVAL (unwritable path, malformed file or field out of range: then
 * nothing is installed), RTG_ENOENT (no such file). */
int rtg_save_tuning(rtg_ctx *ctx, const char *path);
int rtg_load_tuning(rtg_ctx *ctx, const char *path);

/* Device timing with HIP events on the context's stream: bit i of `mask`
 * times every launch of kernel id i (RTG_K_*), RTG_TIME_PHASES times the
 * pipeline phases; 0 turns timing off.  Events add a few microseconds per
 * timed launch. */
int rtg_set_timing(rtg_ctx *ctx, uint32_t mask);

/* Counters of the last completed rtg_all_pairs* call. */
int rtg_get_stats(rtg_ctx *ctx, rtg_stats *out);

/* Stage check: the integer cell coordinates floor((R_t p)/(alpha r) + u_t)
 * computed by the key kernel for transform t, written to host kappa
 * [n][d] (int64).  R [d][d], u [d] host FP64.  Same errors as rtg_all_pairs. */
int rtg_debug_cell_coords(rtg_ctx *ctx, const float *points, int64_t n, int32_t d, double r,
                          double alpha, const double *R, const double *u, int64_t *kappa);

const char *rtg_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* RTG_H */
