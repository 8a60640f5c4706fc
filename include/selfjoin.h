/*
 * selfjoin.h -- C ABI of the MI355X (gfx950) Euclidean epsilon self-join.
 *
 * The operation (Gowanlock & Karsin, "GPU Accelerated Similarity Self-Join
 * for Multi-Dimensional Data", Section 3.1, problem statement): given a set D
 * of n points in d dimensions and a radius epsilon, return every ordered
 * tuple (a, b) of points of D with dist(a, b) <= epsilon, dist being the
 * Euclidean (L2) distance over all d dimensions.  The result may be much
 * larger than D and may exceed device memory; D itself must fit (Section
 * 3.1, last paragraph).
 *
 * Canonical predicate.  A pair (i, j) is in the result iff
 *     acc <= eps2,   eps2 = epsilon * epsilon   (binary64, one rounding),
 *     acc = sum over t = 0 .. d-1 in the caller's dimension order of
 *           diff*diff, diff = (double)p_i[t] - (double)p_j[t],
 * every operation a separately rounded binary64 operation.  Whatever
 * precision the device filters use, every include/exclude decision equals
 * this predicate's.
 *
 * Result convention.  Indices are the caller's row indices 0 .. n-1.  The
 * result holds (i, i) for every point and both (i, j) and (j, i) for every
 * pair, so |R| = n * (S_D + 1) with S_D the selectivity of Section 5.2.
 * Pairs are returned sorted ascending by (i, j).
 *
 * Method (Algorithm 1 and Sections 3.2, 4.1, 4.2, 4.4): dimensions are
 * reordered by variance estimated on a 1% sample, points are binned into a
 * grid of cells of side >= epsilon over the first k reordered dimensions
 * (only non-empty cells stored), each query cell searches the 3^k adjacent
 * cells by binary search, and candidate pairs are filtered by their distance
 * over all d dimensions with a short-circuit once the partial sum of squares
 * exceeds the threshold.  Results are produced in batches (Section 3.2.2).
 *
 * Conventions for every entry point:
 *  - Return value: SJ_OK (0) or a negative SJ_ERR_* code.  On error,
 *    out-parameters are left untouched and selfjoin_last_error() returns a
 *    message for the calling thread (valid until that thread's next call).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *    ordered on it; each call returns only after its work on `stream` is
 *    complete, so buffers may be reused immediately after the call.
 *  - Pointers marked "host or device" may point to host memory (pageable or
 *    pinned) or to device memory of the current HIP device.
 *  - A handle is used by one thread at a time; distinct handles may be used
 *    concurrently.  The handle lives on the HIP device that was current when
 *    it was built, and that device must be current for every later call.
 *  - Maximum sizes: n <= 2^32 - 1, 1 <= d <= SJ_MAX_DIM.
 */
#ifndef SELFJOIN_H
#define SELFJOIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SJ_OK                 0
#define SJ_ERR_INVALID_ARG   -1  /* NULL pointer, n or d out of range, epsilon <= 0 or not finite, NaN/Inf coordinates, bad option */
#define SJ_ERR_OUT_OF_MEMORY -2  /* a device or pinned-host allocation failed */
#define SJ_ERR_DEVICE        -3  /* a HIP runtime call failed */
#define SJ_ERR_KEY_OVERFLOW  -4  /* an explicit k makes the linearised cell id exceed 63 bits, or the
                                    adjacency lists of the cells exceed 2^32 - 1 entries */
#define SJ_ERR_STATE         -5  /* call out of order, e.g. fetch before run */
#define SJ_ERR_RANGE         -6  /* fetch offset beyond the result */

#define SJ_MAX_DIM 128

/* Distance filter used by selfjoin_run. */
enum sj_precision {
    SJ_PREC_FP32 = 0, /* difference form (a-b)^2 summed in FP32 on the vector ALUs, with short-circuit */
    SJ_PREC_FP16 = 1, /* |a|^2+|b|^2-2a.b on the matrix cores, FP16 operands, FP32 accumulation,
                         FP64 recheck of the error band; falls back to BF16 when the centred data
                         exceed the FP16 range */
    SJ_PREC_BF16 = 2  /* as SJ_PREC_FP16 with BF16 operands */
};

typedef struct sj_index sj_index; /* opaque; owns every device buffer it uses */

typedef struct sj_options {
    uint32_t struct_size;   /* sizeof(sj_options), for ABI versioning */
    int32_t  k;             /* indexed dimensions (Section 4.1); 0 = choose automatically in [k_min, k_max]; clamped to d */
    uint32_t k_min, k_max;  /* automatic k range; defaults 4 and 8 */
    uint32_t reorder;       /* 1 = order dimensions by descending sample variance (Section 4.2); 0 = index the first k input dimensions */
    uint32_t shortc;        /* 1 = stop a distance once its partial sum exceeds the threshold (Section 4.4) */
    uint32_t precision;     /* enum sj_precision */
    uint64_t batch_pairs;   /* b_s of Section 3.2.2: maximum result pairs held on the device per batch; 0 = automatic (as many as fit) */
    uint32_t min_batches;   /* minimum number of batches n_b (Section 3.2.2 uses >= 3); 0 or 1 = as few as possible */
    uint32_t autotune;      /* selfjoin_run_batched only: 1 = time candidate tile lengths and queue granularities on the batch and keep the fastest */
    uint64_t mem_budget;    /* device bytes the result buffers may use; 0 = a default share of free device memory */
    uint32_t fp32_form;     /* SJ_PREC_FP32 arithmetic: enum sj_fp32_form */
    uint32_t sortidu;       /* 1 = SORTIDU (Section 4.3): points of each cell sorted by one un-indexed
                               dimension u, and each block of queries searches every adjacent cell only
                               for points within epsilon of the block's u-range; 0 = off */
} sj_options;

/* How the FP32 filter evaluates squared distances.  Both are exact filters
 * (their FP32 error is bounded and pairs inside the bound are rechecked in
 * FP64); they differ in speed only.
 *   DIFFERENCE: sum of (a_t - b_t)^2, two vector operations per dimension.
 *   NORM:       |a|^2 + |b|^2 - 2 a.b from per-point prefix norms, one fused
 *               multiply-add per dimension; its error grows with the norms, so
 *               AUTO takes it only up to 16 dimensions and when the band
 *               stays narrow against eps^2. */
enum sj_fp32_form { SJ_FP32_AUTO = 0, SJ_FP32_DIFFERENCE = 1, SJ_FP32_NORM = 2 };

/* Work units of the single-join distance kernel (sj_info.units), chosen at
 * build from the cells' sizes; either gives the same result.
 *   CELL:        a unit holds the queries of one cell (FP32: 64 lanes with up
 *                to 4 queries each; matrix cores: a workgroup of 256 queries).
 *   SMALL_CELLS: taken when more than a quarter of the lane work of CELL units
 *                would fall on idle query slots (FP32: one query per lane;
 *                matrix cores: one wave of 32 queries). */
enum sj_units { SJ_UNITS_CELL = 1, SJ_UNITS_SMALL_CELLS = 2 };

/* Fills *opts with the defaults: k = 0 (auto, 4..8), reorder = 1,
 * shortc = 1, precision = SJ_PREC_FP32, batch_pairs = 0, min_batches = 0,
 * mem_budget = 0, fp32_form = SJ_FP32_AUTO, sortidu = 0.  Callers built against an
 * older header may pass a shorter struct (struct_size); missing fields take
 * their defaults. */
void selfjoin_default_options(sj_options *opts);

/*
 * Builds the grid index (Algorithm 1: reorderVariance, constructIndex).
 *   points   host or device, row-major float32 [n][d], caller-owned; read
 *            during the call only (the index keeps its own reordered copy).
 *   n, d     point count (0 allowed: an empty result) and dimension count.
 *   epsilon  search radius, finite and > 0.
 *   opts     NULL for the defaults.
 *   out      receives the new handle; release it with selfjoin_free.
 * Errors: SJ_ERR_INVALID_ARG for bad arguments or non-finite coordinates,
 * SJ_ERR_KEY_OVERFLOW when an explicit k cannot be linearised in 63 bits or
 * gives more than 2^32 - 1 adjacent-cell entries over all non-empty cells
 * (automatic k stays below both limits), SJ_ERR_OUT_OF_MEMORY, SJ_ERR_DEVICE.
 */
int selfjoin_build_index(const float *points, uint64_t n, uint32_t d,
                         double epsilon, const sj_options *opts, void *stream,
                         sj_index **out);

/*
 * Runs the join (Algorithm 1: computeNumBatches and the batch loop of
 * SelfJoinKernel; Section 3.2.2 batching).  On success *total_pairs = |R|.
 * The sorted result stays owned by the handle (in device memory when it fits
 * the budget, else in pinned host memory) until selfjoin_free.  Calling it
 * again returns the same total without recomputing.
 * Batches cover ranges of caller indices in order, so the batches together
 * hold the result in (i, j) order.  In an FP32 self-join of several
 * batches each unordered pair is evaluated once: a batch skips candidates
 * of earlier batches and hands the mirrored pairs of later batches on in
 * device memory (a spill of about a quarter of |R| at its peak; when the
 * spill would not fit, or the caller's row order makes it overflow, the
 * batches run one-directionally instead, with the same result).
 */
int selfjoin_run(sj_index *idx, void *stream, uint64_t *total_pairs);

/*
 * Copies result pairs [first, first + max_pairs) of the sorted result.
 *   out_i, out_j  host or device uint32 arrays of max_pairs entries, or NULL
 *                 to skip that column.
 *   out_dist      host or device float array, or NULL: the Euclidean
 *                 distance of each pair recomputed in FP32 (difference form,
 *                 caller's dimension order); relative error <= 1e-5.
 *   n_written     receives min(max_pairs, |R| - first).
 * Errors: SJ_ERR_STATE before a successful selfjoin_run, SJ_ERR_RANGE when
 * first > |R|.
 */
int selfjoin_fetch_pairs(sj_index *idx, uint64_t first, uint64_t max_pairs,
                         uint32_t *out_i, uint32_t *out_j, float *out_dist,
                         uint64_t *n_written, void *stream);

/* Counters and timings of the last build and run. */
typedef struct sj_info {
    uint32_t struct_size;     /* sizeof(sj_info) */
    uint32_t d;
    uint64_t n;
    double   epsilon;
    uint32_t k;               /* indexed dimensions used */
    uint32_t precision;
    uint64_t n_cells;         /* non-empty grid cells |G| */
    uint64_t candidates;      /* ordered candidate pairs C: sum over points of the sizes of their adjacent non-empty cells */
    uint64_t evaluated;       /* candidate pairs the distance kernel evaluated (each unordered pair once when tiles are symmetric; about half of the ordered pairs in FP32 multi-batch runs) */
    uint64_t rechecks;        /* pairs sent to the FP64 boundary recheck */
    uint64_t pairs;           /* |R| (valid after run) */
    uint32_t batches;         /* batches used by the last run */
    uint32_t result_on_host;  /* 1 when the result was streamed to pinned host memory */
    float    ms_build;        /* device time of the index build (events) */
    float    ms_join;         /* device time of the distance kernels of the last run */
    float    ms_sort;         /* device time of result sorting of the last run */
    float    ms_run;          /* device time of the whole last run */
    uint32_t join_launches;   /* launches of the distance kernel in the last run (reruns after an undersized buffer included) */
    uint32_t fp32_form;       /* form of the FP32 filter (enum sj_fp32_form; 0 on the matrix-core path) */
    uint32_t units;           /* work units of the distance kernel (enum sj_units; set by the build, 0 for an empty input) */
} sj_info;

/*
 * Row starts of the result as a CSR neighbour table (the neighbour table
 * of Algorithm 1, constructNeighborTable): offsets[i] = index of the first
 * pair (i, .) in the sorted result (the number of pairs of rows below i),
 * offsets[n] = |R|.  With the j column of selfjoin_fetch_pairs (out_i =
 * NULL) as the neighbour array, the neighbours of point i are
 * neighbours[offsets[i] .. offsets[i+1]).  In a self-join every point is its
 * own neighbour, so no row is empty; a query handle's rows may be.
 *   offsets  host or device, n + 1 entries, caller-owned.
 * Errors: SJ_ERR_STATE before a successful run, SJ_ERR_INVALID_ARG for NULL.
 */
int selfjoin_fetch_offsets(sj_index *idx, uint64_t *offsets, void *stream);

/*
 * The general similarity join Q join_eps E (Section 3.1: the self-join is the
 * case Q = E): every pair (q, e) of a query point q of Q and an indexed
 * point e of E with dist(q, e) <= epsilon, under the canonical predicate
 * above (caller's dimension order, FP64).  E is an index built by
 * selfjoin_build_index, whose epsilon, k, grid, dimension order, precision
 * and options the join uses; Q is binned into E's grid and searched against
 * E's cells (Algorithm 1's kernel with the query points taken from Q).
 *   entries  the index of E.  It is only read: it may still be run and
 *            fetched itself, and several query handles may share it.  If the
 *            caller frees it first, its memory is released with the last
 *            query handle built on it.
 *   queries  host or device, row-major float32 [m][d] (d = E's d),
 *            caller-owned; read during the call only.
 *   m        query count (0 allowed: an empty result), m <= 2^32 - 1.
 *   out      receives the query handle, an sj_index of its own: selfjoin_run
 *            joins Q with E; selfjoin_fetch_pairs returns (i, j) = (query row,
 *            row of E) sorted by (i, j), with no self pairs unless Q and E
 *            share points; selfjoin_fetch_offsets returns m + 1 row starts
 *            (rows may be empty); selfjoin_get_info reports n = m;
 *            selfjoin_get_perm returns E's order.  Release with selfjoin_free.
 * Errors: SJ_ERR_INVALID_ARG for NULL arguments, NaN/Inf query coordinates,
 * entries that is itself a query handle, a current device other than E's,
 * or (FP16 index only) an epsilon so large against E's range that query
 * coordinates could leave the FP16 range (build E with SJ_PREC_BF16 or
 * SJ_PREC_FP32 then); SJ_ERR_OUT_OF_MEMORY; SJ_ERR_DEVICE.
 */
int selfjoin_build_query(const sj_index *entries, const float *queries, uint64_t m,
                         void *stream, sj_index **out);

/*
 * As selfjoin_fetch_offsets, for callers that cannot allocate memory (tight
 * serving loops, code that must not call hipMalloc in its steady state): it
 * allocates nothing.  Its temporaries (the scan's partial sums, the per-row
 * counts for host output, the staging of a host-resident result) live in
 * one fixed 64 MiB device array that the library holds on each device it
 * runs on until the process ends.
 *   offsets  host or device, n + 1 entries, caller-owned.  Device offsets
 *            are counted and scanned in place (any n); host offsets need
 *            (n + 1) * 8 bytes of the array for the counts, so n can be at
 *            most about 6.2 * 10^6 for host output.
 * Every call on a device shares that device's array.  The library takes a
 * per-device lock for the call and completes the call's device work before
 * returning, so calls from threads of one process do not overlap; calls
 * from several processes on one device share nothing.
 * Errors: as selfjoin_fetch_offsets, plus SJ_ERR_INVALID_ARG when n is too
 * large for the fixed array (selfjoin_fetch_offsets has no such limit).
 */
int selfjoin_fetch_offsets_noalloc(sj_index *idx, uint64_t *offsets, void *stream);

/* info->struct_size must be set by the caller. */
int selfjoin_get_info(const sj_index *idx, sj_info *info);

/* perm[r] = caller dimension placed at position r by the variance reorder;
 * writes min(cap, d) entries. */
int selfjoin_get_perm(const sj_index *idx, uint32_t *perm, uint32_t cap);

/* Releases the handle and all its memory (an index that query handles
 * still use: when the last of them is freed).  NULL is ignored. */
void selfjoin_free(sj_index *idx);

/* ------------------------------------------------------------------------
 * Many independent self-joins at once.
 *
 * Each job is the problem of Section 3.1 on its own point set.  Every job
 * gets its own grid index (as selfjoin_build_index, automatic k per job);
 * the distance filtering of ALL jobs then runs as one persistent
 * matrix-core kernel over a shared work queue, captured together with the
 * result sort into a hipGraph and replayed.  Results are exact (canonical
 * predicate) and sorted by (i, j) per job.
 * ---------------------------------------------------------------------- */
typedef struct sj_job {
    const float *points;  /* host or device, row-major float32 [n][d], caller-owned, read during the call */
    uint64_t n;           /* 0 .. 2^20 - 1 points */
    uint32_t d;           /* 1 .. 77 dimensions (matrix-core K padding <= 80) */
    uint32_t reserved;
    double epsilon;       /* finite, > 0 */
} sj_job;

typedef struct sj_batch sj_batch; /* opaque; owns every job's index and the shared result */

typedef struct sj_batch_info {
    uint32_t struct_size;     /* sizeof(sj_batch_info) */
    uint32_t njobs;
    uint64_t pairs;           /* total |R| over all jobs */
    uint64_t candidates;      /* total ordered candidate pairs */
    uint64_t evaluated;       /* pair evaluations of the persistent kernel */
    uint64_t rechecks;        /* FP64 band rechecks */
    uint64_t capacity;        /* key slots of the shared result buffer */
    uint64_t n_wu;            /* work units in the shared queue */
    uint32_t tile_candidates; /* candidate stretch per work unit (tile shape) */
    uint32_t queue_grab;      /* work units a wave takes from the queue at once */
    uint32_t grid;            /* workgroups of the persistent launch */
    uint32_t tuned;           /* 0 defaults, 1 tuned now, 2 taken from the tuning cache */
    float    ms_build;        /* sum of the jobs' index builds (device events; builds overlap) */
    float    ms_estimate;     /* sum of the jobs' sampled counts (device events) */
    float    ms_graph;        /* last replay of the captured graph: join + ids + sort + bounds */
    float    ms_host_build;   /* wall time of all index builds and sampled counts */
    float    ms_host_prepare; /* wall time of the job table, queue and buffer set-up */
    float    ms_tune;         /* wall time of the autotuner (0 when cached or off) */
} sj_batch_info;

/* Builds every job's index, pre-sizes the shared result from sampled
 * counts, captures the persistent join + sort into a hipGraph and replays
 * it once.  opts (NULL = defaults) apply to every job; the precision is
 * SJ_PREC_FP16 unless SJ_PREC_BF16 is asked for (SJ_PREC_FP32 selects FP16
 * here).  Errors as selfjoin_build_index, plus SJ_ERR_INVALID_ARG for njobs
 * outside [1, 65536], n >= 2^20 or d > 77. */
int selfjoin_run_batched(const sj_job *jobs, uint32_t njobs, const sj_options *opts,
                         void *stream, sj_batch **out);

/* Replays the captured graph (same result); *ms receives its device time. */
int selfjoin_batch_replay(sj_batch *batch, float *ms);

/* Slot range of job `job` in the batch result: *count pairs. */
int selfjoin_batch_range(const sj_batch *batch, uint32_t job, uint64_t *first, uint64_t *count);

/* As selfjoin_fetch_pairs, for the pairs [first, first + max_pairs) of one
 * job (indices are the job's own row indices). */
int selfjoin_batch_fetch(sj_batch *batch, uint32_t job, uint64_t first, uint64_t max_pairs,
                         uint32_t *out_i, uint32_t *out_j, float *out_dist,
                         uint64_t *n_written, void *stream);

/* info->struct_size must be set by the caller. */
int selfjoin_batch_get_info(const sj_batch *batch, sj_batch_info *info);

/* Releases the batch and all its memory.  NULL is ignored. */
void selfjoin_batch_free(sj_batch *batch);

/* ------------------------------------------------------------------------
 * Device memory held between calls.
 *
 * Device blocks the library frees (result buffers, work lists, sort and
 * build temporaries) go to a per-device cache once the device has finished
 * the work queued before the free, and later calls on that device reuse
 * them instead of calling hipMalloc and hipFree again.  The cache holds at
 * most a quarter of the device's memory, or SJ_CACHE_BYTES bytes when that
 * environment variable is set when the device is first used (0: no
 * caching).  Cached blocks count as free memory for the automatic memory
 * budget, and an allocation that fails empties the device's cache and is
 * tried once more; memory that other code of the process wants (a tensor
 * library's own allocator) is not given back by itself.
 * ---------------------------------------------------------------------- */

/* Frees every block cached for the current device, the pinned host blocks
 * cached for results streamed to the host (SJ_HOST_CACHE_BYTES caps them;
 * default an eighth of host memory, at most 64 GiB) and the calling
 * thread's kept build temporaries.  *released (may be NULL) receives the
 * cached bytes freed.  Call it with no run of the library in flight on the
 * device from another thread.  Errors: SJ_ERR_DEVICE when the current
 * device cannot be read. */
int selfjoin_release_cache(uint64_t *released);

/* Message of the calling thread's last error ("" if none). */
const char *selfjoin_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SELFJOIN_H */
