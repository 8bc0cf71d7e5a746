/*
 * panorama.h - C ABI of the MI355X pruned k-NN scan (progressive distance
 * refinement with Cauchy-Schwarz pruning over a PCA basis).
 *
 * The method: vectors are rotated by an orthogonal, energy-compacting
 * transform T (the PCA basis of Section 4.1) and stored level-major (Section
 * 6.1).  A candidate's squared distance to the query is built up one level of
 * dimensions at a time (Eq. 1-2); after each level a lower bound from the
 * tail energies of query and candidate (Eq. 3; Eq. 4 for eps < 1) is compared
 * with the running k-th best distance and the candidate is dropped as soon as
 * the bound exceeds it (Algorithm 1).  At eps = 1 the result equals exact
 * k-NN over the candidate set (Problem 1), the candidate set being the
 * vectors of the probed IVF lists (Problem 2 with IVF, Section 6.1).
 *
 * Conventions shared by every entry point:
 *  - Status: every call returns pano_status.  PANO_OK is 0; any other value
 *    leaves outputs unspecified and sets a thread-local message readable with
 *    pano_last_error().  Nothing aborts and no C++ exception crosses the ABI.
 *  - Ownership: opaque handles (pano_ctx, pano_transform, pano_index) are
 *    created and freed only by the library.  Array arguments are borrowed for
 *    the duration of the call; output arrays are allocated by the caller.
 *  - Memory spaces: arguments named *_host are host memory; arguments named
 *    *_dev are device memory on the context's GPU.  Row-major float32 rows of
 *    length d unless stated otherwise.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 *    stream).  Calls enqueue their GPU work on it and return when the results
 *    are in the output arrays (they synchronise the stream before returning),
 *    except a search with PANO_SEARCH_ASYNC, whose results are complete in
 *    stream order.
 *  - Distances are squared Euclidean distances.  The reported distance of a
 *    result is the canonical D(q, x): sum over j = 0..d-1, in that order, of
 *    ((double)q_j - (double)x_j)^2 with every product and sum rounded to
 *    FP64, then rounded to float32.  Results are ordered by ascending
 *    (D, id); missing results are id -1 and distance +inf.
 */
#ifndef PANORAMA_H
#define PANORAMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PANO_OK = 0,
    PANO_EINVAL = 1,       /* invalid argument (shape, range, non-finite input) */
    PANO_ENOMEM = 2,       /* device or host allocation failed */
    PANO_EDEVICE = 3,      /* a HIP runtime call failed */
    PANO_EUNSUPPORTED = 4, /* valid request the library does not implement */
    PANO_EBUSY = 5         /* resource temporarily exhausted */
} pano_status;

typedef enum { PANO_F32 = 0, PANO_BF16 = 1 } pano_dtype;

typedef struct pano_ctx pano_ctx;
typedef struct pano_transform pano_transform;
typedef struct pano_index pano_index;
typedef struct pano_pq_index pano_pq_index;

/* Thread-local description of the last failure on this thread ("" if none). */
const char *pano_last_error(void);

/* Library version string. */
const char *pano_version(void);

/* Create a context bound to HIP device `device`.  The context owns scratch
 * memory reused across searches.  A context may be used by one thread at a
 * time. */
pano_status pano_ctx_create(int device, pano_ctx **out);
/* Destroy a context; every index built on it must be freed first. */
void pano_ctx_destroy(pano_ctx *ctx);

/* Device memory (bytes) the context currently keeps for search scratch.  A
 * context grows its scratch to the largest search it has run (by 1.25x the
 * request when it grows) and keeps it; a serving loop charges this resident
 * amount against its memory budget. */
pano_status pano_ctx_scratch_bytes(const pano_ctx *ctx, int64_t *bytes);

/* Wait for all work on the context's device and report, in
 * *nonfinite_queries, the queries with a non-finite value that asynchronous
 * searches (PANO_SEARCH_ASYNC) on this context met since the last call;
 * EINVAL if there were any.  The count is reset. */
pano_status pano_ctx_status(pano_ctx *ctx, int64_t *nonfinite_queries);

/* Release the context's search scratch memory and its captured search graph
 * (the next search allocates again).  Call only while no search runs on the
 * context. */
pano_status pano_ctx_trim(pano_ctx *ctx);

/*
 * build_transform: the PCA basis of Section 4.1, fitted on the host in FP64.
 * x_host [n][d] float32 rows.  The mean mu and covariance are accumulated in
 * FP64 over a seeded sample of `fit_sample` rows (fit_sample <= 0 or >= n:
 * every row); T's rows are the eigenvectors of the covariance sorted by
 * descending eigenvalue, each signed so that its largest-magnitude entry is
 * positive.  Vectors are mapped to T (v - mu).  Also records lambda and the
 * energy-compaction constant alpha (Section 4.1, E(m) ~ exp(-alpha m / d)).
 * Errors: EINVAL if n < 2, d < 1 or x has a non-finite value.
 */
pano_status pano_build_transform(const float *x_host, int64_t n, int32_t d, int64_t fit_sample,
                                 uint64_t seed, pano_transform **out);

/* Identity transform (mu = 0, T = I): raw-vector pruning. */
pano_status pano_transform_identity(int32_t d, pano_transform **out);

/* A caller-supplied transform: mu_host [d], T_host [d][d] row-major FP64.
 * EINVAL if T is not orthonormal to 1e-9 (max |T T^t - I|). */
pano_status pano_transform_from(int32_t d, const double *mu_host, const double *T_host,
                                pano_transform **out);

/* Copy out the transform.  Any output pointer may be NULL.  mu_host [d],
 * T_host [d][d], lambda_host [d] (0 for caller-supplied transforms). */
pano_status pano_transform_get(const pano_transform *tf, int32_t *d, double *mu_host,
                               double *T_host, double *lambda_host, double *alpha);
void pano_transform_free(pano_transform *tf);

/*
 * ivf_assign: the coarse quantiser of IVF (Section 6.1): Lloyd's k-means in
 * raw space.  x_dev [n][d]; centroids_dev [nlist][d] and assign_dev [n]
 * (int32) are outputs.  Initial centroids come from greedy k-means++ (D^2
 * sampling of 2 + ln(nlist) candidates per step, keeping the one that lowers
 * the potential most) over a seeded sample of max(65536, min(262144,
 * 64 nlist)) rows (all rows if n is smaller), drawn with `seed`; each of
 * `iters` iterations assigns every row to its nearest centroid
 * on the GPU and recomputes the means (an empty cluster keeps its centroid).
 * The final assignment pass gives each row the list with the smallest key
 * (D, l), D the canonical distance (the FP64 sum of squared differences in
 * coordinate order, rounded to float32) and ties to the smaller list: an FP32
 * score with a certified margin keeps the lists that can hold that key, and
 * these are rescored canonically (the iterations before it assign by the FP32
 * score ||c||^2 - 2 <x, c> alone).  nlist = 1
 * gives the flat index (centroid = mean, every row in list 0).
 * Errors: EINVAL if nlist < 1 or nlist > n.
 */
pano_status pano_ivf_assign(pano_ctx *ctx, const float *x_dev, int64_t n, int32_t d,
                            int32_t nlist, int32_t iters, uint64_t seed, float *centroids_dev,
                            int32_t *assign_dev, void *stream);

/*
 * build_levels: pack the index (Section 6.1 level-major batches, Section 6.5
 * tail energies).  x_dev [n][d] raw rows; centroids_dev [nlist][d];
 * assign_dev [n] in [0, nlist).  m_host [L+1] level cuts with m[0] = 0 <
 * m[1] < ... < m[L] = d (Eq. 2), 1 <= L <= 64.  `block` is the batch size B:
 * 64, 128 or 256 (0 = 256; the scan encodes a slot in 8 bits).  The first
 * level may hold at most 64 dimensions, and the level widths, each padded to a
 * multiple of 4, may sum to at most 4096.  Each list is cut into blocks of B
 * vectors; within a block all B level-l slices are contiguous, then level l+1
 * (each slice padded to a multiple of 4 floats with zeros).  Per vector the tail norms
 * sqrt(R_x^(l,d)) for l = 0..L-1 are stored (4L bytes).  The index keeps a
 * device copy of the raw rows (used for the canonical rescoring) and of the
 * centroids; it lives in device memory and is owned by the handle.
 * store = PANO_BF16 additionally stores the level slices in bfloat16.
 * Errors: EINVAL on inconsistent shapes or cuts or a block size outside
 * {0, 64, 128, 256} (checked before anything else, so these are reported even
 * for null handles); ENOMEM.
 */
pano_status pano_build_levels(pano_ctx *ctx, const pano_transform *tf, const float *x_dev,
                              int64_t n, int32_t d, const float *centroids_dev,
                              const int32_t *assign_dev, int32_t nlist, const int32_t *m_host,
                              int32_t L, int32_t block, pano_dtype store, pano_index **out,
                              void *stream);

/* Tuning knobs of a search (0 = library default for every field). */
typedef struct {
    int32_t group;        /* max queries sharing one scan work item (1..16) */
    int32_t blocks_per_item; /* blocks of a list scanned by one work item */
    int32_t seed_pool;    /* candidates of the nearest list ranked to seed d_k */
    int32_t seed_count;   /* of those, how many get their exact distance */
    int32_t grid;         /* persistent scan workgroups (0 = 3 per CU pruned,
                             2 per CU brute force) */
    int32_t use_bf16;     /* 1: the pruned scan reads the bfloat16 level slices
                             (index built with PANO_BF16, else EINVAL); its
                             bounds and committed distances carry a certified
                             bfloat16 margin and the merge rescores the
                             boundary band from the FP32 rows, so the result
                             equals the FP32 search's */
    int32_t reserved[6];  /* [0]: refine a whole level on the matrix cores while at
                             least this many pairs of a block (workgroup scan) or
                             of a 64-slot step (per-wave scan) survive (0 = 64);
                             [1]: scan mode: 0 or 1 = the workgroup scan (one
                             persistent kernel, a local top-k per work item),
                             3 = no pruning (the brute-force scan of
                             pano_search_bruteforce; same answer), for
                             workloads whose bounds prune too little, 4 = the
                             per-wave scan (every wavefront pulls its own work
                             items; level 1 and dense levels on the matrix
                             cores, later levels level-synchronously over a
                             compacted pair list, survivors appended to the
                             result buffers); other values are EINVAL;
                             [2]: lanes per pair in the per-pair walk of the
                             workgroup scan: 1, 2 or 4 (0 = 4 when at most
                             64 pairs of a block survive, 2 up to 128, else
                             1); other values are EINVAL;
                             [3]: levels per step of the walk with four lanes
                             per pair: 1, or 2 (both requested together; 0 =
                             2 when no level is wider than 64 dimensions);
                             [4]: 1 = keep each list's queries in arrival
                             order; 0 = order them by their approximate
                             distance to the list's centroid, so that a query
                             group holds queries at similar distance (work
                             order only, the answer is the same) */
} pano_search_params;

/* Search flags. */
#define PANO_SEARCH_STATS 1u  /* collect counters, readable with pano_stats_get (runs eagerly) */
#define PANO_SEARCH_EAGER 2u  /* do not replay the captured graph of the search */
#define PANO_SEARCH_TIMING 4u /* run eagerly with events around the phases and
                                 write only the ms_* fields of the counters
                                 (the kernels are those of an ordinary search,
                                 without the counting of PANO_SEARCH_STATS) */
#define PANO_SEARCH_ASYNC 8u  /* return without waiting: the results are
                                 complete in stream order on `stream` (a
                                 query whose result buffer overflows is
                                 answered by an exact fallback on the device);
                                 a query with a non-finite value gets
                                 (-1, +inf) and is reported by the next
                                 pano_ctx_status call on the context.
                                 A later search on the same context, on any
                                 stream, is ordered after it (they share the
                                 context's scratch); the caller keeps the
                                 query and output buffers alive until the
                                 stream reaches the end.  Not with STATS or
                                 TIMING. */

/*
 * search: k nearest neighbours of each query among the vectors of its probed
 * lists (exact at probe for eps = 1; Algorithm 1 with Eq. 4 for eps < 1).
 * q_dev [nq][d] float32.  nprobe_dev [nq] int32 per-query probe counts, or
 * NULL to use nprobe_all for every query; probe counts are clamped to
 * [1, nlist].  With nprobe_dev, a positive nprobe_all is an upper bound on
 * the per-query counts (larger ones are clamped to it) and sizes the probe
 * tables as nq x nprobe_all; 0 sizes them for nlist probes per query.  The
 * probe set of a query is its nprobe nearest lists by (D(q, centroid),
 * list id).  k in [1, 128].  eps in [0, 1] (Eq. 4; 1 = exact).  Outputs
 * ids_dev [nq][k] int64 (row index of the vector in build_levels' x) and
 * dists_dev [nq][k] float32 (canonical D), ascending by (D, id).  `params`
 * may be NULL.  Errors: EINVAL if k < 1 or k > 128, nq < 0, eps outside
 * [0, 1] or a query is non-finite; ENOMEM if scratch cannot be allocated.  An ordinary
 * search launches a graph (captured once per launch configuration on the
 * context's own stream) on `stream`; eager, counting and timing searches run
 * on the context's streams after the work already queued on `stream`.
 */
pano_status pano_search(pano_index *idx, const float *q_dev, int64_t nq, int32_t k,
                        const int32_t *nprobe_dev, int32_t nprobe_all, float eps,
                        int64_t *ids_dev, float *dists_dev, const pano_search_params *params,
                        uint32_t flags, void *stream);

/*
 * search_ctx: pano_search run on context `ctx` (its streams, scratch memory
 * and graph cache) instead of the context the index was built on.  ctx must
 * be on the index's device.  Searches on different contexts may run
 * concurrently from different threads, also on the same index (a serving
 * loop keeps one context per worker); one context serves one thread at a
 * time.  PANO_SEARCH_STATS writes the index's counters, so at most one
 * search of an index should ask for them at a time.
 */
pano_status pano_search_ctx(pano_ctx *ctx, pano_index *idx, const float *q_dev, int64_t nq, int32_t k,
                            const int32_t *nprobe_dev, int32_t nprobe_all, float eps, int64_t *ids_dev,
                            float *dists_dev, const pano_search_params *params, uint32_t flags,
                            void *stream);

/*
 * refine: k nearest neighbours of each query among its own candidate ids
 * (a first pass's top-kprime, e.g. from a quantized index), with the
 * point-centric form of Algorithm 1 (batch B = 1 in the table of the two
 * modes; Section 6.4, Refine): candidates are taken in groups of 64 in the
 * given order, each refined level by level from the index's level-major
 * blocks and dropped at its first level whose bound (Eq. 3; Eq. 4 for
 * eps < 1) exceeds the query's running d_k; the first group seeds d_k.
 * q_dev [nq][d] float32; cand_dev [nq][kprime] int64 row ids of
 * build_levels' x, -1 for an empty slot; the ids of one row must be
 * distinct.  Outputs ids_dev [nq][k] int64 and dists_dev [nq][k] float32
 * (canonical D, ascending (D, id); -1 / +inf padding).  At eps = 1 the
 * result is the exact k-NN over the candidate set.  Runs on the index's
 * context, after the work queued on `stream`; returns when done.  Errors:
 * EINVAL if k < 1 or k > 128, kprime < 1, eps outside [0, 1], a query is
 * non-finite or a candidate id is outside [-1, n).  The first call on an index builds a
 * map from row id to block position (8 bytes per row, kept by the index).
 */
pano_status pano_refine(pano_index *idx, const float *q_dev, int64_t nq, int32_t k, const int64_t *cand_dev,
                        int32_t kprime, float eps, int64_t *ids_dev, float *dists_dev, void *stream);

/*
 * audit_bounds: the certified per-level bounds of sampled (query, row) pairs
 * as the GPU computes them from the index, for checking the pruning's
 * soundness (the bounds of Section 5: Eq. 3, Cauchy-Schwarz on the tails,
 * with the margins of the floating-point analysis) against an exact
 * distance.  Pair i is query pair_q_dev[i] (int32, a row of q_dev [nq][d]
 * float32) and row pair_row_dev[i] (int64, a row id of build_levels' x).
 * For level l = 0..L-1, bounds_dev[i][l][0..3] (float32) receives lower and
 * upper bounds on the stored-frame distance ||y_q - y_x||^2 after levels
 * 0..l, where y_q is the transformed query and y_x the stored FP32 row:
 * [0], [1] with the head distance summed from coordinate differences (the
 * form of the per-pair passes), [2], [3] in the dot-product form of the
 * matrix-core levels (level energies from the tails minus twice the product).
 * Bounds are those of eps = 1 and use the same bound functions and margins
 * as the scans.  bf16 != 0 (an index built with PANO_BF16): heads are read
 * from the bfloat16 tiles with the bfloat16 margins; the distance bounded is
 * still the one to the FP32 row.  rows_dev (may be NULL) [npairs][2][d_pad]
 * float32 receives y_q and y_x (padding columns zero).  Device pointers,
 * caller-owned; runs on the index's context after the work queued on
 * `stream` and returns when done.  Errors: EINVAL for a query or row index
 * out of range, or bf16 on an index without bfloat16 tiles.
 */
pano_status pano_audit_bounds(pano_index *idx, const float *q_dev, int64_t nq, const int32_t *pair_q_dev,
                              const int64_t *pair_row_dev, int64_t npairs, int32_t bf16, float *bounds_dev,
                              float *rows_dev, void *stream);

/*
 * search_noalloc: pano_search for callers that cannot allocate memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, semantics and results as pano_search without
 * flags, but no call allocates: every scratch buffer of the search comes from
 * a fixed device array of 64 MiB per GPU that the library reserves when it
 * is loaded (set up on the first context created on that GPU, or on the first
 * call) and keeps until the process ends; no graph is captured, every kernel
 * runs on `stream` in order, and the call returns when the results are in
 * ids_dev / dists_dev.  A search whose scratch (about nq x (nlist +
 * 2 nprobe + d) x 4 bytes plus the per-query result buffers) exceeds the array
 * fails with EINVAL and a message giving the bytes it needs; split the batch.
 * Every call on one GPU shares that GPU's array and each call clears what it
 * needs cleared: calls that overlap on one GPU (from several threads or
 * streams) race and must be serialised by the caller.
 */
pano_status pano_search_noalloc(pano_index *idx, const float *q_dev, int64_t nq, int32_t k,
                                const int32_t *nprobe_dev, int32_t nprobe_all, float eps, int64_t *ids_dev,
                                float *dists_dev, const pano_search_params *params, void *stream);

/*
 * search_scratch_bytes: device scratch memory (bytes) that a pano_search of
 * nq queries with this k, probe setting (per_query_nprobe != 0: a per-query
 * array bounded by nprobe_all, or by nlist if nprobe_all is 0; else
 * nprobe_all for all) and params needs on its context, beside the caller's
 * queries and outputs.  Includes the key buffer of the exact fallback for one
 * query (8 bytes per slot of its largest possible probe set).  Used for
 * memory-based admission.
 */
pano_status pano_search_scratch_bytes(const pano_index *idx, int64_t nq, int32_t k,
                                      int32_t per_query_nprobe, int32_t nprobe_all,
                                      const pano_search_params *params, int64_t *bytes);

/*
 * search_bruteforce: the same contract as pano_search with pruning disabled:
 * every probed candidate's full distance is computed from the same level-major
 * tiles with the same work decomposition (the same-GPU brute-force baseline).
 * eps is ignored.
 */
pano_status pano_search_bruteforce(pano_index *idx, const float *q_dev, int64_t nq, int32_t k,
                                   const int32_t *nprobe_dev, int32_t nprobe_all, int64_t *ids_dev,
                                   float *dists_dev, const pano_search_params *params,
                                   uint32_t flags, void *stream);

typedef struct {
    int64_t n;
    int32_t d;
    int32_t d_pad;          /* sum of the level widths padded to 4 */
    int32_t nlist;
    int32_t L;
    int32_t block;
    int32_t has_bf16;
    int64_t nblocks;
    int64_t max_list_len;
    int64_t bytes_levels;   /* FP32 level tiles */
    int64_t bytes_levels_bf16;
    int64_t bytes_tails;    /* 4 L bytes per stored slot */
    int64_t bytes_ids;
    int64_t bytes_raw;      /* raw rows kept for the canonical rescoring */
    double transform_err_max; /* certified bound on ||stored - exact rotated|| */
    double sigma_ratio;     /* sigma_max / sigma_min of the FP32 transform */
} pano_index_info_t;

pano_status pano_index_info(const pano_index *idx, pano_index_info_t *out);

/* Copy the level cuts (m[0..L]) and the per-list lengths (nlist) to host. */
pano_status pano_index_layout(const pano_index *idx, int32_t *m_host, int64_t *list_len_host);

/* Counters of the last search on this index with PANO_SEARCH_STATS. */
typedef struct {
    int64_t nq;
    int64_t candidates;      /* (query, candidate) pairs in the probe sets */
    int64_t dims_read;       /* coordinates read by the scan, sum over pairs */
    int64_t level_reads[64]; /* pairs that read level l (l < 64) */
    int64_t items;           /* scan work items */
    int64_t committed;       /* entries written to the per-query result buffers */
    int64_t band;            /* entries rescored with the canonical recipe */
    int64_t fallback_queries;/* queries answered by the exact fallback path */
    double ms_total;         /* device time of the whole search */
    double ms_scan;          /* device time of the scan kernel */
    double ms_merge;         /* device time of merge + rescoring */
    double ms_prep;          /* device time of transform, probe, work list, seed */
    int64_t scan_bytes;      /* bytes of level slices, tails and ids touched */
    int64_t scan_cycles[6];  /* scan phases summed over workgroups (shader clock
                                cycles of one lane): pull, level 1, later levels,
                                commit, publish, spare */
} pano_stats_t;

pano_status pano_stats_get(const pano_index *idx, pano_stats_t *out);

/* Free an index (and the context's cached search graph if it was captured
 * for this index).  Call before destroying the index's context.  NULL is a
 * no-op. */
void pano_index_free(pano_index *idx);

/* ===================================================================== IVFPQ
 * The method over product-quantized vectors (Section 4.2 spectrum shaping,
 * Section 6.2 the IVFPQ scan).
 */

/*
 * shape_plan: Procedure 1 of Section 4.2 (Robin Hood inter-level shaping) on
 * expected per-coordinate variances lambda_host [d] (the PCA eigenvalues,
 * descending).  Level energies are sums of the variances over the levels cut
 * by m_host [L+1] (m[0] = 0 < ... < m[L] = d); the cap is tau = kappa times
 * their mean (kappa >= 1).  Levels are visited front to back; a level above
 * the cap is rotated together with the fewest following coordinates s >= 1
 * that bring its expected energy after a Haar rotation of the block,
 * b / (b + s) times the block total, to tau or below (s stops at the last
 * coordinate); the block's coordinates then carry its mean variance.  All
 * sums run in coordinate order, and an energy within a relative 1e-9 of tau
 * counts as within the cap.  Writes the rotated blocks as (start,
 * length) pairs into blocks_host [2 * cap] in plan order and their count into
 * *nblocks.  Host only.  Errors: EINVAL on bad cuts, kappa < 1 or a plan
 * longer than cap (then *nblocks is the length needed).
 */
pano_status pano_shape_plan(const double *lambda_host, int32_t d, const int32_t *m_host, int32_t L,
                            double kappa, int32_t *blocks_host, int32_t cap, int32_t *nblocks);

/*
 * transform_shape: the shaped transform U R T_PCA of Section 4.2.  R applies
 * a Haar-random rotation to each block of pano_shape_plan (with the
 * transform's eigenvalues and the given cuts and kappa), in plan order; when
 * isotropize is nonzero, U applies an independent Haar rotation within each
 * level (Procedure 2).  The rotations come from a counter-based generator
 * seeded by `seed` (splitmix64, Box-Muller normals, Householder QR with the
 * sign fix that makes Q Haar-distributed).  The result keeps mu; its lambda
 * holds the expected per-coordinate variances after shaping.  A transform
 * without eigenvalues (pano_transform_from) gets no R.  Host only; the caller
 * owns *out.  Errors: EINVAL on bad cuts or kappa < 1.
 */
pano_status pano_transform_shape(const pano_transform *pca, const int32_t *m_host, int32_t L, double kappa,
                                 int32_t isotropize, uint64_t seed, pano_transform **out);

/*
 * pq_build: the IVFPQ index of Section 6.2 over the shaped frame of tf.
 * Each row x of x_dev [n][d] (device, FP32), assigned to list l, is coded by
 * its residual T (x - mu) - y_c(l) in the shaped frame, y_c(l) = T (c_l - mu)
 * (FP64, each coordinate summed in order; kept for the search), split into
 * M = d / dsub sub-vectors of dsub coordinates (dsub in {1, 2, 4, 8, 16};
 * M <= 128, since the scan keeps a query's table of M x 256 floats in LDS);
 * each sub-quantizer has 256 codewords, trained by Lloyd iterations (`iters`,
 * FP64 means, an empty cell keeps its codeword) on a seeded sample of
 * max(256, min(n, sample)) rows from 256 sample rows spread over the sample,
 * and every row is coded by its nearest codewords (FP32 distance, ties to the
 * smaller code).  The levels m_host [L+1] (1 <= L <= 64) must have equal
 * widths that fall on sub-vector boundaries, with at most 16 sub-quantizers
 * per level.  Lists follow assign_dev [n] in [0, nlist) with
 * centroids_dev [nlist][d] (raw space, for probing).  Layout in device
 * memory, per list, blocks of 256 slots: the codes of a block level by level,
 * each level slot by slot (a slot's codes of the level in 4 * ceil(M/L/4)
 * bytes, zero padded), then the norms of each slot's reconstruction beyond
 * levels 1..L-1 (FP32, level-major), then the slot ids.  The index owns its
 * memory.  Errors: EINVAL on shapes, cuts, dsub or M; ENOMEM.
 */
pano_status pano_pq_build(pano_ctx *ctx, const pano_transform *tf, const float *x_dev, int64_t n, int32_t d,
                          const float *centroids_dev, const int32_t *assign_dev, int32_t nlist,
                          const int32_t *m_host, int32_t L, int32_t dsub, int32_t iters, int64_t sample,
                          uint64_t seed, pano_pq_index **out, void *stream);

#define PANO_PQ_BRUTE 16u /* pq_search: read every sub-quantizer of every
                             candidate (no pruning): the brute-force scan of
                             the same codes */

/*
 * pq_search: k nearest candidates of each query by the PQ distance over its
 * probed lists (Section 6.2 with Algorithm 1's level loop).  The probe set is
 * that of pano_search (canonical (D, l) order in raw space).  The query's
 * shaped coordinates y_i = sum_j T_ij (q_j - mu_j) are summed in coordinate
 * order in FP64, and its residual for list l is z = y - y_c(l); the list's
 * table entry (m, c) is float32 of the FP64 sum of (z_j - C[m][c][j])^2 over
 * the sub-vector in order; a candidate's distance is float32 of the FP64 sum
 * of its M entries in sub-quantizer order.  A candidate is dropped after a
 * level once the bound P + (a - b)^2 + 2 (1 - eps) a b (Eq. 3/4: P the
 * entries read so far, a and b the norms of the residual z and of the
 * reconstruction beyond the level, with certified rounding margins) exceeds
 * the running k-th distance; at eps = 1 the answer
 * is the first k by (distance, id), exactly, padded with (-1, +inf).
 * q_dev [nq][d]; nprobe as in pano_search (at most 1024 lists per query);
 * 1 <= k <= 128; ids_dev [nq][k] int64, dists_dev [nq][k] float.  flags:
 * PANO_PQ_BRUTE, PANO_SEARCH_STATS (counts for pano_pq_stats).  Blocks until
 * the results are written.  Errors: EINVAL (sizes, a query with a non-finite
 * value), ENOMEM.
 */
pano_status pano_pq_search(pano_ctx *ctx, pano_pq_index *idx, const float *q_dev, int64_t nq, int32_t k,
                           const int32_t *nprobe_dev, int32_t nprobe_all, float eps, int64_t *ids_dev,
                           float *dists_dev, uint32_t flags, void *stream);

/* Counters of the last pq_search with PANO_SEARCH_STATS: out[0] table
 * look-ups done, out[1] look-ups of the unpruned scan (candidates x M),
 * out[2] queries answered by the exact fallback, out[3] candidates, out[4]
 * bytes of codes and tail norms the scan read (a block's level is read
 * whole once any of its slots is alive); *ms_scan the scan kernel's
 * duration. */
pano_status pano_pq_stats(const pano_pq_index *idx, int64_t *out5, double *ms_scan);

/* Copy out the trained quantizer: codebooks_host [M][256][dsub] FP32 and
 * codes_host [n][M] (row order); either may be NULL.  *M_out and *dsub_out
 * if non-NULL. */
pano_status pano_pq_export(const pano_pq_index *idx, float *codebooks_host, uint8_t *codes_host, int32_t *M_out,
                           int32_t *dsub_out);
void pano_pq_free(pano_pq_index *idx);

#ifdef __cplusplus
}
#endif

#endif /* PANORAMA_H */
