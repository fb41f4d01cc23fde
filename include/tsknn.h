/*
 * tsknn — exact k-nearest-neighbour scan over multi-dimensional time series
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: Bachmann & Freytag, "An Analytical Approach to Improving Time
 * Warping on Multidimensional Time Series" (arXiv 1811.11076).
 *   - Distances (Sec. 2.1): DTW = the smallest sum of squared Euclidean point
 *     distances along a warping path (no final square root); DK (dog-keeper,
 *     discrete Frechet) = the smallest maximum Euclidean point distance along
 *     a warping path.
 *   - Sakoe-Chiba band (Sec. 2.2) optional for both.
 *   - k-NN query (Sec. 1): the k database series closest to each query.
 *   - Pruning: DTW uses LB_Box (Sec. 3, eq. (1)); DK uses the greedy upper
 *     bound of Alg. 1 to seed the threshold (Sec. 4.3) and the sparse-DK
 *     semantics of Alg. 3 (cells above the threshold are dead).
 *   Results are exact: identical to evaluating every pair with the full DP
 *   and sorting by (distance, id).
 *
 * Conventions for every call:
 *   - Return value: TSK_OK (0) or one of the TSK_ERR_* codes below.  On
 *     error no output is written and tsk_last_error() describes the cause.
 *     No C++ exception crosses this boundary.
 *   - All argument validation happens before any device work.
 *   - "_dev" pointers are device memory on the current HIP device; "_host"
 *     pointers are host memory.  The caller owns every buffer it passes.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous on that stream unless stated otherwise.
 *   - Series values are float32, array-of-structs [length][dim], several
 *     series concatenated; offsets (int64, n+1 entries, offsets[0] == 0,
 *     strictly increasing) delimit series i as rows offsets[i]..offsets[i+1]-1.
 *     Lengths must be in [1, TSK_MAX_LEN]; dim in [1, TSK_MAX_DIM].
 *   - Non-finite series values are undefined behaviour.
 */
#ifndef TSKNN_H
#define TSKNN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSK_VERSION_MAJOR 0
#define TSK_VERSION_MINOR 1

#define TSK_MAX_DIM 32      /* k-NN and range queries; above 8 dimensions the
                               series are stored and scanned padded with zero
                               coordinates to 12, 16, 24 or 32 (same costs and
                               bounds, bit for bit) by the general kernels */
#define TSK_SUB_MAX_DIM 8   /* subsequence search */
#define TSK_MLP_MAX_DIM 8   /* the learned order's encoder */
#define TSK_MAX_LEN 4096
#define TSK_MAX_K 64

enum {
    TSK_OK = 0,
    TSK_ERR_INVALID_ARG = 1,
    TSK_ERR_OOM = 2,
    TSK_ERR_DEVICE = 3,
    TSK_ERR_UNSUPPORTED = 4,
    TSK_ERR_IO = 5,
    TSK_ERR_CANCELLED = 6
};

/* Distance (Sec. 2.1). */
enum { TSK_DTW = 0, TSK_DK = 1 };

/* Sakoe-Chiba band (Sec. 2.2).  For a pair of lengths (m, n) with
 * L = max(m, n) the half-width is w = r (TSK_BAND_ABS) or
 * w = floor(frac * L) (TSK_BAND_FRAC), and cell (i, j) is inside iff
 *   |i (n-1) - j (m-1)| (L-1) <= w (m-1) (n-1),
 * which is |i - j| <= w for equal lengths; every cell is inside when m == 1
 * or n == 1.  TSK_BAND_NONE: no band. */
enum { TSK_BAND_NONE = 0, TSK_BAND_ABS = 1, TSK_BAND_FRAC = 2 };
typedef struct {
    int32_t mode;
    int32_t r;
    float frac;
} tsk_band;

/* Candidate order for a query.  The order never changes the result, only
 * how early the threshold falls (and so how much work is pruned). */
enum { TSK_ORDER_PLAIN = 0, TSK_ORDER_GIVEN = 1, TSK_ORDER_LEARNED = 2 };

enum { TSK_TUNE_OFF = 0, TSK_TUNE_CACHED = 1 };

typedef struct tsk_index tsk_index;

/* Encoder that predicts distances for TSK_ORDER_LEARNED (not part of the
 * paper's method: it only reorders candidates, so results never change). */
typedef struct tsk_model tsk_model;

/* Per-call counters (all int64) and device times.  Counts are over all
 * (query, candidate) pairs of the call. */
typedef struct {
    int64_t pairs;          /* n_queries * n_series */
    int64_t seed_pairs;     /* pairs evaluated by the threshold-seeding pass */
    int64_t bound_pruned;   /* pairs discarded by a bound before any DP */
    int64_t dp_started;     /* pairs whose DP began */
    int64_t dp_completed;   /* DPs that ended with a value <= threshold */
    int64_t dp_abandoned;   /* DPs stopped early (value > threshold) */
    int64_t dp_cells;       /* DP cells evaluated (lane-cells, dead ones too) */
    int64_t bound_steps;    /* LB_Box terms + greedy moves of the optional
                               pass over the survivors */
    int64_t fallback_pairs; /* pairs that left the fast DP for the general one */
    int64_t dp_valid_cells; /* DP cells inside the matrix and the band */
    int64_t calls;          /* calls accumulated (tsk_index_profile) */
    float ms_total;         /* device time of the whole call */
    float ms_seed;          /* envelope + threshold seed kernels */
    float ms_bound;         /* bound pass + survivor compaction */
    float ms_dp;            /* DP kernels */
    float ms_final;         /* output kernel */
    float ms_bound_kernel;  /* the bound kernel alone (LB_Box or corner) */
    float ms_dp_fast;       /* the lane-per-pair DP kernel alone */
    float ms_dp_general;    /* the general (fallback) DP kernel alone */
    int64_t dp_valid_cells_general; /* of dp_valid_cells: general DP's share */
    float ms_order;         /* TSK_ORDER_LEARNED: query embedding, scores and
                               per-query candidate order */
    int64_t seed_steps;     /* greedy moves of the threshold-seeding walks
                               (bound_steps counts the other bound work) */
    int64_t chunks;         /* query chunks: launches of each per-chunk kernel */
} tsk_stats;

typedef struct {
    int64_t size;                  /* sizeof(tsk_query_opts) */
    int32_t order;                 /* TSK_ORDER_PLAIN, _GIVEN or _LEARNED */
    int32_t seed_count;            /* candidates per query used to seed the
                                      threshold (0 = library default: 128
                                      with the corner-bound seed, else 512
                                      for DK and 1024 for DTW) */
    const int32_t *order_dev;      /* TSK_ORDER_GIVEN: [n_queries][n_series]
                                      candidate ids, each row a permutation;
                                      the first seed_count entries form the
                                      seed set, and with surv_order 2
                                      survivors are processed in this order */
    int32_t use_graph;             /* 1: the call (all its chunks of
                                      queries) runs as one captured HIP
                                      graph, cached on the index and
                                      replayed while the call repeats (same
                                      pointers, offsets, k, distance, band,
                                      options and encoder); excludes
                                      profile; uneven-length DTW needs its
                                      queries to fit one chunk (up to
                                      min(2^30 / n_series, 65535) of them);
                                      with stats_host only ms_total is
                                      timed */
    int32_t dp_kernel;             /* 0 auto, 1 force the general DP */
    int32_t profile;               /* 1: record per-stage HIP events on the
                                      stream and add this call's counters to
                                      the index's profile, without any
                                      synchronisation (tsk_index_profile) */
    int32_t walk_pass;             /* DK: greedy walks (Alg. 1) over the
                                      survivors of the corner bound before
                                      the DP: -1 auto, 0 off, 1 on */
    int32_t task_size;             /* survivors per wave task of the sparse-DK
                                      kernel (0 = library default: 64, 128
                                      or 256 from 2^16 / 2^19 series up) */
    int32_t tube_rows;             /* rows per lane window of the sparse-DK
                                      kernel: 8, 16 or 32 (0 = library
                                      default, 16);
                                      pairs whose live cells outgrow it finish
                                      in the general DP */
    int32_t lb_qgroup;             /* queries per wave of the length-bucket
                                      LB_Box kernel: 2, 4 or 8 (0 or 1 = 4,
                                      16 = 8);
                                      equal lengths: 1 = one pair per 8
                                      lanes, each sum abandoned once above
                                      the threshold (query envelopes up to
                                      64 KiB, else as 0); 16 = 16 queries
                                      sharing each candidate load; 0 = 16 for
                                      databases above 256 MiB, else 8; other
                                      values = 8 */
    int32_t dk_band_slots;         /* unbanded DK on equal lengths: 0 = the
                                      sparse-DK tube kernel; 32, 56, 64, 104
                                      or 128 = the lockstep banded kernel in
                                      a virtual band of (slots-1)/2, pairs
                                      whose live cells reach its edge finish
                                      in the general DP (exact either way) */
    int32_t surv_order;            /* survivors' DP order: 1 = ascending
                                      bound (likely neighbours first), 2 =
                                      the query's candidate order, 0 =
                                      library default (DTW 1, DK 2) */
    int32_t dp_rows;               /* tile shape of the general DP: rows per
                                      lane of its skewed strips (1, 2 or 4;
                                      0 = 4) */
    int32_t dp_waves_per_cu;       /* persistent waves per compute unit of
                                      the lane-per-pair DP kernels: 8, 16
                                      or 32 (0 = library default) */
    int32_t dk_seed;               /* DK threshold seed: 0 = greedy walks
                                      (Alg. 1), 1 = the diagonal path's
                                      largest cost (equal lengths only) */
    int32_t tune;                  /* TSK_TUNE_CACHED: take seed_count,
                                      tube_rows, task_size, walk_pass,
                                      lb_qgroup, dk_band_slots, surv_order,
                                      dp_rows, dp_waves_per_cu, dk_seed,
                                      bound_seed and dtw_cascade
                                      from the index's tuning cache
                                      for this (distance, band, k), if
                                      tsk_tune filled it; TSK_TUNE_OFF: as
                                      given */
    const tsk_model *model;        /* TSK_ORDER_LEARNED: the encoder; each
                                      query's candidates are taken in
                                      ascending embedding distance.  The
                                      index caches the candidates' embeddings
                                      for the model's current parameters */
    const volatile int32_t *cancel_flag_host; /* nullable host flag, read before
                                      each chunk of queries (and before any
                                      device work): non-zero stops the call
                                      with TSK_ERR_CANCELLED.  Work already
                                      enqueued still runs on the stream;
                                      rows of queries not reached are not
                                      written */
    int32_t lb_both;               /* DTW on an index of equal-length series:
                                      1 = after the query-envelope LB_Box,
                                      also the candidate-envelope one (eq. (1)
                                      in the paper's own orientation) for the
                                      survivors of queries of that length,
                                      keeping the larger bound.  Needs
                                      N x length x 2 x dim floats of
                                      workspace; 0 = off (default).  k-NN
                                      only (ignored by range queries) */
    int32_t raw_keys;              /* 1: out_dist_dev receives each rank's
                                      ranking key instead of its distance
                                      (DK: the squared DK, whose correctly
                                      rounded sqrt is the distance; DTW: the
                                      distance itself), so that per-shard
                                      rows can be merged by (key, id)
                                      exactly; 0 = distances (default) */
    int32_t bound_seed;            /* threshold seed set: 1 = each query's
                                      seed_count candidates of smallest
                                      corner bound (every path's first and
                                      last cells: max of their costs for DK,
                                      sum for DTW; computed for every pair
                                      first; in the plain order with
                                      seed_count <= 512 and at least 32
                                      candidates per seed, the smallest of
                                      each of 2 * seed_count equal segments
                                      of the candidates, and the seed_count
                                      smallest of those), 2 = the first seed_count
                                      candidates of the query's order;
                                      0 = library default (DK: 1 for the
                                      plain order, 2 for given and learned
                                      orders; DTW: as the cascade).  DK on
                                      LDS-sized queries and DTW on equal
                                      lengths (where the seed is the
                                      diagonal path's cost sum unless the
                                      cascade runs); k-NN only */
    int32_t dtw_cascade;           /* DTW on equal lengths: 1 = the corner
                                      bound prunes first, with the threshold
                                      seeded by greedy walks (Alg. 1, summing
                                      costs) over the candidates of smallest
                                      corner bound; LB_Box (eq. (1)) is
                                      computed only for its survivors, which
                                      then run in ascending LB_Box; 2 =
                                      LB_Box for every pair; 3 = the corner
                                      bound and seed of 1 without LB_Box
                                      (its survivors run in ascending corner
                                      bound); 0 = library default (1 for the
                                      plain order unless bound_seed is 2 or
                                      lb_qgroup names an LB_Box kernel,
                                      else 2) */
    int32_t dk_box;                /* DK on an equal-length index with the
                                      corner cascade (the plain order's
                                      default, or bound_seed = 1): 1 = the
                                      corner survivors are also bounded by
                                      the DK box bound (tsk_pair_dk_box) and
                                      the DP runs on those it keeps, in
                                      ascending bound; 0 or 2 = off */
    int32_t lb_prefix;             /* DTW cascade, LB_Box of the corner
                                      survivors: after this many points of
                                      the candidate (a multiple of 64), a
                                      pair whose partial LB_Box scaled to all
                                      its points stays below the threshold
                                      keeps the partial sum (itself a lower
                                      bound) and stops; -1 = every point;
                                      0 = library default (64 when the
                                      banded lane-per-pair DP follows, else
                                      every point) */
} tsk_query_opts;

typedef struct {
    int64_t size;                  /* sizeof(tsk_index_opts) */
    int64_t workspace_limit_bytes; /* bound on the workspace of a query call
                                      (0 = library default: chunks of up to
                                      2^30 (query, series) pairs and 65535
                                      queries); calls
                                      split their queries into chunks whose
                                      workspace fits (at least one query per
                                      chunk) */
} tsk_index_opts;

/* Library version. */
int tsk_version(int *major, int *minor);

/* Text of the last error on the calling thread; valid until the next tsk_*
 * call on that thread.  Never NULL. */
const char *tsk_last_error(void);

/* Builds a read-only index over n_series database series (Sec. 1: the
 * database the k-NN query scans).  values_dev: [offsets_host[n]][dim] float32
 * device AoS; offsets_host: n+1 int64 host offsets.  The library copies the
 * data into its own device layouts (an AoS copy and 64-series struct-of-arrays
 * tiles), so the caller may free its buffers once the stream has completed.
 * *out receives an index owned by the caller (free with tsk_index_free).
 * Errors: INVALID_ARG (null pointers, n < 1, bad offsets), UNSUPPORTED
 * (dim or a length outside the supported range), OOM, DEVICE. */
int tsk_index_build(const float *values_dev, const int64_t *offsets_host, int64_t n_series,
                    int32_t dim, const tsk_index_opts *opts, void *hip_stream, tsk_index **out);

/* Opt-in input check (series values must be finite; the scan does not test
 * them): *first_bad_host (nullable) receives the index of the first
 * non-finite float of values_dev[0 .. count), or -1.  Returns TSK_OK when
 * all are finite, TSK_ERR_INVALID_ARG otherwise (or for NULL values with
 * count > 0, count < 0).  Synchronous on hip_stream. */
int tsk_validate_values(const float *values_dev, int64_t count, int64_t *first_bad_host,
                        void *hip_stream);

/* Frees an index and its device memory after synchronising its stream.
 * NULL is accepted. */
int tsk_index_free(tsk_index *index);

/* Number of series and dimensionality of an index. */
int tsk_index_info(const tsk_index *index, int64_t *n_series, int32_t *dim);

/* Exact k-NN query (Sec. 1; pruning of Sec. 3 and Sec. 4).  For every query
 * q the k database series with the smallest (distance, id) are written to
 * out_ids_dev[q*k .. q*k+k-1] (int64 ids, ascending) and out_dist_dev (float32:
 * DTW sums, or DK as the correctly rounded sqrt of the squared DK).  Ranks
 * without a finite distance (k > n_series, or an infeasible band) get
 * (-1, +inf).  q_values_dev / q_offsets_host: the queries, as for an index.
 * opts may be NULL.  stats_host (nullable): if given, the call synchronises
 * the stream and fills the counters.  The index is only read; calls on one
 * index must not overlap in time (the per-index workspace is shared).
 * Errors: INVALID_ARG, UNSUPPORTED (k > TSK_MAX_K, dim mismatch), OOM, DEVICE. */
int tsk_knn_query(const tsk_index *index, const float *q_values_dev, const int64_t *q_offsets_host,
                  int64_t n_queries, int32_t k, int32_t dist, tsk_band band,
                  const tsk_query_opts *opts, int64_t *out_ids_dev, float *out_dist_dev,
                  tsk_stats *stats_host, void *hip_stream);

/* Size of the fixed device workspace of tsk_knn_query_noalloc (bytes). */
#define TSK_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * exact k-NN query as tsk_knn_query, with the same arguments, outputs and
 * errors, except that its workspace is a fixed device array of
 * TSK_NOALLOC_SCRATCH_BYTES inside the library (one per device, held from
 * the first such call on that device until the process ends) and the call
 * allocates nothing: no hipMalloc, hipFree or allocating library routine.
 * The caller still passes the queries and the outputs (device memory).
 * Queries are split into chunks whose workspace fits the array (the
 * workspace per query grows with the database: about 20-24 bytes per series,
 * plus the staged query); a call whose single query does not fit returns
 * TSK_ERR_INVALID_ARG before any device work.  No statistics.  Excluded
 * (TSK_ERR_UNSUPPORTED): use_graph, profile, TSK_ORDER_LEARNED, lb_both.
 * The array is shared by every call on a device and keeps the last call's
 * contents (each call clears what must start at zero): calls that overlap
 * in time on one device race, so the caller serialises them, on one stream
 * or by synchronising. */
int tsk_knn_query_noalloc(const tsk_index *index, const float *q_values_dev,
                          const int64_t *q_offsets_host, int64_t n_queries, int32_t k,
                          int32_t dist, tsk_band band, const tsk_query_opts *opts,
                          int64_t *out_ids_dev, float *out_dist_dev, void *hip_stream);

/* Range query (Sec. 1: all database series within a distance of the
 * query, the paper's second query type beside k-NN), through the same
 * bound and DP kernels with the threshold fixed at the radius (no seeding,
 * no tightening).  Hits of query q are written in ascending id order to
 * out_ids_dev / out_dist_dev[out_offsets_host[q] .. out_offsets_host[q+1])
 * (distances as for tsk_knn_query: DTW sums; DK the correctly rounded sqrt
 * of the squared DK; a hit is a series whose reported distance is
 * <= radius).  out_offsets_host: [n_queries + 1] host int64, always filled.
 * band: by pointer (NULL = no band).  radius: a hit's fp32 distance is
 * <= radius (taken as the largest fp32 value not above it).
 * capacity: entries of the output buffers; if the hits exceed it, nothing
 * but the offsets is written and INVALID_ARG is returned (call again with
 * capacity >= out_offsets_host[n_queries]).  Synchronous.  opts as for
 * tsk_knn_query (use_graph excluded; walk_pass and seed_count ignored).
 * Errors: INVALID_ARG (radius < 0 or NaN, NULL outputs, capacity), as
 * tsk_knn_query otherwise. */
int tsk_range_query(const tsk_index *index, const float *q_values_dev,
                    const int64_t *q_offsets_host, int64_t n_queries, double radius,
                    int32_t dist, const tsk_band *band, const tsk_query_opts *opts,
                    int64_t capacity,
                    int64_t *out_ids_dev, float *out_dist_dev, int64_t *out_offsets_host,
                    tsk_stats *stats_host, void *hip_stream);

/* ---------------------------------------------------------------- subsequence search */

/* Longest query of tsk_subseq_query (16 rows per lane of one wave). */
#define TSK_SUB_MAX_QLEN 1024

typedef struct {
    int64_t size;         /* sizeof(tsk_subseq_opts) */
    int32_t chunk_cols;   /* start columns per work item (0 = library default:
                             64 to 4096, about 2^18 items per group of queries) */
    int32_t seed;         /* 1: greedy bounds (Alg. 2) seed the threshold
                             (default); 0: no seeding (the threshold only falls
                             as matches are found; much slower, for checks) */
    int32_t waves_per_cu; /* waves per compute unit of the DP kernel
                             (0 = 16, at most 32) */
    int32_t reserved;
} tsk_subseq_opts;

/* Subsequence k-NN (Sec. 4.1-4.2; Alg. 2 and Alg. 3 with SUB): a match of a
 * query may start and end anywhere in a series.  The subsequence DK of
 * (query S, series T) is min over a <= b of DK(S, T[a..b]) (squared point
 * costs, as for tsk_knn_query, reported as the correctly rounded sqrt).  For
 * every query the k series with the smallest (subsequence DK, id) are written
 * to out_ids_dev / out_dist_dev[q*k .. q*k+k-1], with the match's end column
 * (the first column b reaching the minimum) in out_end_dev and its start (the
 * latest a with DK(S, T[a..b]) equal to it) in out_start_dev; empty ranks get
 * (-1, +inf, -1, -1).
 * series_dev: caller-owned device fp32 AoS [s_offsets_host[n_series]][dim]
 * (no index: the series are read in place, lengths 1 .. 2^31-1);
 * q_values_dev / q_offsets_host: the queries, lengths 1 .. TSK_SUB_MAX_QLEN.
 * All output buffers are device [n_queries * k]; out_start_dev may be NULL
 * (no start pass).  opts may be NULL.  stats_host (nullable): pairs, seed_pairs
 * (greedy walks that reached the last row), bound_pruned (work items skipped
 * by their row-0 minimum), dp_started / dp_completed / dp_abandoned (work
 * items swept / with a value <= threshold / without), dp_cells, dp_valid_cells,
 * bound_steps (greedy moves + row-0 costs scanned), ms_total / ms_seed /
 * ms_dp / ms_final.  The call allocates its working memory and is
 * synchronous.  Errors: INVALID_ARG, UNSUPPORTED (dim outside
 * [1, TSK_SUB_MAX_DIM], k > TSK_MAX_K, query longer than TSK_SUB_MAX_QLEN),
 * OOM, DEVICE. */
int tsk_subseq_query(const float *series_dev, const int64_t *s_offsets_host, int64_t n_series,
                     int32_t dim, const float *q_values_dev, const int64_t *q_offsets_host,
                     int64_t n_queries, int32_t k, const tsk_subseq_opts *opts,
                     int64_t *out_ids_dev, float *out_dist_dev, int64_t *out_end_dev,
                     int64_t *out_start_dev, tsk_stats *stats_host, void *hip_stream);

/* Reads (and with reset != 0 clears) the profile accumulated by calls made
 * with opts->profile = 1 on this index: counters summed over those calls and
 * per-stage device milliseconds measured by HIP events recorded on each
 * call's stream.  Synchronises with those events.  Errors: INVALID_ARG. */
int tsk_index_profile(tsk_index *index, tsk_stats *out, int32_t reset);

/* Full-DP distance of every (query, database series) pair with no pruning
 * (Sec. 2.1 definitions through the same DP kernels as the k-NN path):
 * out_keys_dev[q * n_series + c] = DTW, or the SQUARED DK (float32).  Used
 * to check the DP against an independent implementation. */
int tsk_pair_distances(const tsk_index *index, const float *q_values_dev,
                       const int64_t *q_offsets_host, int64_t n_queries, int32_t dist,
                       tsk_band band, float *out_keys_dev, void *hip_stream);

/* DK distances from squared DK keys (as tsk_pair_distances writes them):
 * out_dev[i] = the correctly rounded fp32 square root of keys_dev[i] (Sec.
 * 2.1: DK is the largest Euclidean point distance on the best path, the keys
 * hold its square), the same rounding as the k-NN outputs; +inf stays +inf.
 * Both device arrays of n floats on the current device; out_dev may equal
 * keys_dev (in place).  Asynchronous on the stream.  Errors: INVALID_ARG. */
int tsk_dk_distances(const float *keys_dev, float *out_dev, int64_t n, void *hip_stream);

/* DK box bound of every pair (Sec. 3's boxes with the maximum in place of
 * eq. (1)'s sum; Sec. 2.1: DK is the largest point distance on the best
 * warping path): out_dev[q * n_series + c] = the largest, over the points
 * t_j of series c, of the squared distance of t_j to the box (per-dimension
 * [min, max]) of the query rows that the band lets column j align with,
 * float32 terms in the point cost's order; it never exceeds the squared DK
 * of the pair (tsk_pair_distances), and +inf where a column's window is
 * empty.  The same kernel as the k-NN option dk_box, with no threshold.
 * Needs an index of equal-length series (queries of any length).
 * out_dev: device float [n_queries * n_series].  Synchronous.  Errors:
 * INVALID_ARG, UNSUPPORTED (series of unequal length), OOM, DEVICE. */
int tsk_pair_dk_box(const tsk_index *index, const float *q_values_dev,
                    const int64_t *q_offsets_host, int64_t n_queries, tsk_band band,
                    float *out_dev, void *hip_stream);

/* Per-pair bounds through the same kernels as the k-NN path, with no
 * threshold (no early return):
 *   out_lb_dev[q*N + c]  = LB_Box with the query's band envelope and the
 *                          candidate's points (eq. (1) with the roles of
 *                          the two series exchanged), summed over the
 *                          candidate's points in order in float32;
 *   out_ub_dev[q*N + c]  = the greedy path bound of Alg. 1: for TSK_DK the
 *                          maximum squared cost along the greedy path, for
 *                          TSK_DTW the float32 sum of costs along it;
 *   out_steps_dev[q*N+c] = number of greedy moves (int32).
 * Any output pointer may be NULL. */
int tsk_pair_bounds(const tsk_index *index, const float *q_values_dev,
                    const int64_t *q_offsets_host, int64_t n_queries, int32_t dist,
                    tsk_band band, float *out_lb_dev, float *out_ub_dev,
                    int32_t *out_steps_dev, void *hip_stream);

typedef struct {
    int64_t size;           /* sizeof(tsk_tune_opts) */
    int32_t sample_queries; /* queries per trial (0 = min(n_queries, 64)) */
    int32_t reps;           /* timed repetitions per trial, best kept (0 = 2) */
} tsk_tune_opts;

/* Autotuner (not in the paper: a scheduling aid whose choices never change
 * results).  Times k-NN calls on the first sample_queries queries for a set
 * of settings of the work-shaping options (seed size; DK sparse-DP window
 * rows, survivors per wave task and the greedy pass; queries per wave of the
 * length-bucket LB_Box kernel), one option at a time from the library
 * defaults (coordinate descent), keeping the fastest.  *best_out receives
 * base (nullable: defaults) with the tuned fields set, *best_ms_out
 * (nullable) its time; the choice is cached on the index for (dist, band,
 * k) and used by calls with opts->tune = TSK_TUNE_CACHED.  Synchronous.
 * Errors: as tsk_knn_query. */
int tsk_tune(tsk_index *index, const float *q_values_dev, const int64_t *q_offsets_host,
             int64_t n_queries, int32_t k, int32_t dist, tsk_band band,
             const tsk_query_opts *base, const tsk_tune_opts *tune_opts,
             tsk_query_opts *best_out, float *best_ms_out, void *hip_stream);

/* ------------------------------------------------------------------------
 * Learned candidate ordering.  An MLP encoder maps a series, resampled to
 * `points` points by linear interpolation at t_k = k (L-1) / (points-1),
 * to an embedding: (points * dim) -> hidden -> hidden -> embed, ReLU on the
 * hidden layers, bfloat16 weights and layer inputs (nearest-even rounding of
 * fp32 master values where the products read them), fp32 accumulation and
 * biases.  The distance of two series is predicted as the Euclidean distance
 * of their embeddings; training fits it to DK distances by mean squared
 * error with Adam.  Parameters are laid out flat in this order:
 * W1 [hidden][points*dim], b1 [hidden], W2 [hidden][hidden], b2 [hidden],
 * W3 [embed][hidden], b3 [embed] (row-major).
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t size;    /* sizeof(tsk_mlp_shape) */
    int32_t dim;     /* series dimensionality (1..TSK_MLP_MAX_DIM) */
    int32_t points;  /* resampled points (2..256; 32 by default if 0) */
    int32_t hidden;  /* hidden width (multiple of 32, <= 1024; 256 if 0) */
    int32_t embed;   /* embedding width (multiple of 32, <= 256; 64 if 0) */
} tsk_mlp_shape;

typedef struct {
    int64_t size;    /* sizeof(tsk_train_opts) */
    int32_t epochs;  /* passes over the pairs (>= 1) */
    int32_t batch;   /* pairs per step (1..65536) */
    float lr;        /* Adam step size (> 0) */
    float beta1, beta2, eps; /* 0 selects 0.9, 0.999, 1e-8 */
    uint64_t seed;   /* order of the pairs in each epoch (splitmix64 stream) */
} tsk_train_opts;

/* Creates an encoder on the current device: He-uniform weights
 * (U(-sqrt(6/fan_in), sqrt(6/fan_in)) from a splitmix64 stream seeded with
 * `seed`), zero biases, zero Adam state.  *out is owned by the caller.
 * Errors: INVALID_ARG, UNSUPPORTED (shape out of range), OOM, DEVICE. */
int tsk_model_create(const tsk_mlp_shape *shape, uint64_t seed, tsk_model **out);

/* Frees an encoder (NULL accepted) after synchronising the device. */
int tsk_model_free(tsk_model *model);

/* Shape and parameter count of an encoder (outputs nullable). */
int tsk_model_info(const tsk_model *model, tsk_mlp_shape *shape, int64_t *n_params);

/* Copies the fp32 master parameters to host memory [n_params] (flat layout
 * above), or replaces them from host memory (also clearing the Adam state
 * and step count).  n must equal the parameter count.  Synchronous. */
int tsk_model_get_params(const tsk_model *model, float *out_host, int64_t n);
int tsk_model_set_params(tsk_model *model, const float *in_host, int64_t n);

/* Embeddings of n series given as for tsk_index_build: out_dev receives
 * [n][embed] float32.  Asynchronous on the stream. */
int tsk_model_embed(tsk_model *model, const float *values_dev, const int64_t *offsets_host,
                    int64_t n_series, float *out_dev, void *hip_stream);

/* Loss and parameter gradient of one batch of pairs (a_host[i], b_host[i])
 * of the given series with target distances target_host[i] (the forward and
 * backward passes of one training step, without the update).  out_loss_host
 * and out_grad_host ([n_params], nullable) are host outputs; synchronous.
 * Errors: INVALID_ARG (ids outside [0, n_series), n_pairs < 1), OOM, DEVICE. */
int tsk_model_batch_grad(tsk_model *model, const float *values_dev, const int64_t *offsets_host,
                         int64_t n_series, const int32_t *a_host, const int32_t *b_host,
                         const float *target_host, int64_t n_pairs, float *out_loss_host,
                         float *out_grad_host, void *hip_stream);

/* Trains on n_pairs pairs of the given series: every epoch takes the pairs
 * in a fresh shuffled order, in batches of opts->batch, each batch one
 * forward, backward and Adam step on the device.  out_epoch_loss_host
 * (nullable, [epochs]) receives each epoch's mean batch loss.  Synchronous.
 * Errors: INVALID_ARG, OOM, DEVICE. */
int tsk_model_train(tsk_model *model, const float *values_dev, const int64_t *offsets_host,
                    int64_t n_series, const int32_t *a_host, const int32_t *b_host,
                    const float *target_host, int64_t n_pairs, const tsk_train_opts *opts,
                    float *out_epoch_loss_host, void *hip_stream);

/* Writes / reads an encoder (shape, fp32 master parameters) to / from a
 * binary file.  Errors: IO (cannot open, short read, bad header), plus those
 * of tsk_model_create for load. */
int tsk_model_save(const tsk_model *model, const char *path);
int tsk_model_load(const char *path, tsk_model **out);

#ifdef __cplusplus
}
#endif

#endif /* TSKNN_H */
