/*
 * detlsh.h - C ABI of the MI355X (gfx950) DET-LSH indexing-and-query library.
 *
 * DET-LSH (Wei, Peng, Lee, Palpanas; PVLDB 17(9), 2024) answers c^2-k-ANN
 * queries (Def. 2, Sec. 3.1) over a set D of n points in R^d under Euclidean
 * distance.  The library implements its hot path on one GPU:
 *
 *   encoding phase  (Sec. 4.1, Eq. 1, Alg. 1, Alg. 2)  L*K Gaussian projections,
 *                   equal-frequency breakpoints from a sample, uint8 region codes
 *   indexing phase  (Sec. 4.2, Alg. 3)                  one DE-Tree per projected
 *                   space, stored as leaf runs of a permutation of the points
 *   query phase     (Sec. 4.3, Alg. 4-7, Sec. 5.2)      range query with region
 *                   lower bounds over the L spaces, growing radius, exact
 *                   verification of the candidates and top-k
 *
 * General conventions
 *  - Every function returns detlsh_status; DETLSH_OK == 0.  On failure the
 *    thread-local message returned by detlsh_last_error() says why.  No C++
 *    exception crosses this interface.
 *  - "device" pointers are HIP device allocations of the current device (for
 *    example torch CUDA tensors on ROCm); "host" pointers are ordinary memory.
 *    A host pointer where a device pointer is required gives DETLSH_EINVAL.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Every call that
 *    takes a stream returns only after its results are complete (it
 *    synchronises `stream`), so inputs may be freed and outputs read as soon
 *    as it returns; detlsh_query_async is the exception (stream-ordered: it
 *    returns once its work is enqueued).
 *  - Matrices are row-major and densely packed unless stated otherwise.
 *  - An index is read-only after it is built: any number of threads may call
 *    detlsh_query on it concurrently, each with its own stream; every call
 *    has a workspace of its own (allocated, or reused from an earlier call:
 *    see detlsh_trim; a server, below, allocates once instead).
 *    detlsh_free must not race with queries, and every server on the index
 *    must be destroyed first.
 */
#ifndef DETLSH_H
#define DETLSH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct detlsh_index_s* detlsh_index;

typedef enum {
    DETLSH_OK = 0,
    DETLSH_EINVAL = 1,      /* an argument is out of range or of the wrong kind   */
    DETLSH_ENOMEM = 2,      /* device or host memory could not be allocated       */
    DETLSH_EBUSY = 3,       /* a wait timed out (serving)                         */
    DETLSH_EDEVICE = 4,     /* a HIP call failed; the message names it            */
    DETLSH_ECANCELED = 5,   /* the request was cancelled (serving)                */
    DETLSH_EINTERNAL = 6    /* an internal invariant failed                        */
} detlsh_status;

/* Verification precision of a query (Sec. 4.3 exact verification). */
enum {
    DETLSH_FP32 = 0,        /* candidate distances in FP32, direct differences   */
    DETLSH_BF16_RERANK = 1  /* BF16 distances (FP32 accumulate) keep the best
                               rerank_mult*k, which are re-ranked exactly in FP32 */
};

/* Initial radius policy of Alg. 7. */
enum {
    DETLSH_RMIN_MAGIC = 0,  /* the smallest radius that satisfies both conditions of
                               the "magic" r_min of Sec. 5.2: |S(r_min)| >= beta*n+k
                               and |S(r_min/c)| < beta*n+k                         */
    DETLSH_RMIN_FIXED = 1   /* Alg. 7 from the caller's r_min, radius r_min*c^t   */
};

/* Projection of the encoding phase. */
enum {
    DETLSH_PROJ_GAUSSIAN = 0,  /* the L*K hashes h_ij(o) = a_ij . o of Eq. 1, a ~ N(0,1)^d */
    DETLSH_PROJ_PAA = 1        /* DET-ONLY (Sec. 6.1): one space (L = 1) of K PAA segment
                                  means, segment j averaging coordinates
                                  [j*floor(d/K), (j+1)*floor(d/K)); needs d >= K and
                                  ignores A                                          */
};

/* ------------------------------------------------------------------------ */
/* index build                                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t seed;              /* seed of the library's own draws of A and of the
                                   sample when the two pointers below are NULL   */
    int32_t max_leaf;           /* DE-Tree leaf capacity (Alg. 3 max_size); 0 -> 256 */
    int32_t keep_bf16;          /* 1: keep a BF16 copy of X for DETLSH_BF16_RERANK */
    int32_t proj_bf16;          /* 1: projection GEMM with BF16 inputs, FP32 sums  */
    int32_t projection;         /* DETLSH_PROJ_GAUSSIAN (0) or DETLSH_PROJ_PAA (1)  */
    const float* A;             /* host, (L*K) x d, row i*K+j = hash h_ij of Eq. 1,
                                   entries N(0,1); NULL -> drawn from `seed`       */
    const int64_t* sample_ids;  /* host, floor(sample_frac*n) distinct ids in [0,n)
                                   used to choose breakpoints (Alg. 1); NULL ->
                                   drawn uniformly without replacement from seed */
    int32_t borrow_x;           /* 1: the index reads X in place instead of a copy
                                   of its own; X must then stay allocated and
                                   unchanged until detlsh_free, or until a
                                   detlsh_insert, which moves the points into an
                                   array the index owns.  0: X is copied      */
} detlsh_build_opts;

/*
 * Build an index over X (device, n x d FP32).  Encoding phase (Sec. 4.1):
 * projects every point with the L*K hashes h_ij(o) = a_ij . o (Eq. 1), selects
 * N_r+1 breakpoints per projected dimension from the projections of
 * floor(sample_frac*n) sampled points (evaluated in IEEE double) by sorting them (equal-frequency rule of
 * Sec. 4.1, B(z) = the max(1, floor((z-1) n_s / N_r))-th smallest sampled value,
 * B(1) = minimum, B(N_r+1) = maximum) and gives every coordinate the code
 * #{z in 2..N_r : B(z) <= h} (Alg. 2; a value equal to a breakpoint belongs to
 * the upper region).  Indexing phase (Alg. 3): for each of the L projected
 * spaces, the points are ordered into leaf runs of a DE-Tree whose root has
 * one child per vector of first code bits and whose overfull nodes are split
 * on the dimension whose next bit divides them most evenly (Sec. 4.2).
 *
 * Limits (else DETLSH_EINVAL): n >= 1, d >= 1, 1 <= K <= 32 and
 * L in {1, 2, 4, 8} with L*K' <= 64, where K' is the smallest of 4, 8, 16, 32
 * that is >= K, N_r a power of two in [2, 256], 0 < sample_frac <= 1 with
 * floor(sample_frac*n) >= N_r, n < 2^31.  The kernels run K' dimensions per
 * tree: the K' - K extra ones have zero projection rows, so every point and
 * query projects to 0 there (all their breakpoints 0, every code N_r - 1) and
 * no bound, tree split or answer changes; every array this interface returns
 * or takes (A, B, codes, leaf boxes, projections) has the caller's K.  The
 * (L, K') limits are the kernels' register budget: the range query is compiled
 * per (L, K'), keeping a point's 2*L*K' cell edges (or its L screen vectors) in
 * registers, 128 of a wave's VGPRs at L*K' = 64.
 * X is copied (the caller may free it when the call returns) unless
 * opts->borrow_x is set.  On success *out owns all of its other device memory
 * until detlsh_free.
 */
detlsh_status detlsh_build_index(const float* X, int64_t n, int32_t d, int32_t L,
                                 int32_t K, int32_t N_r, double sample_frac,
                                 const detlsh_build_opts* opts, void* stream,
                                 detlsh_index* out);

/*
 * Build an index from given encoding-phase results instead of computing them:
 * A (host, (L*K) x d), B (host, (L*K) x (N_r+1), B[e][z-1] = B_e(z)) and the
 * codes (host, n x (L*K) uint8, column e = i*K + j).  The DE-Trees are built
 * from the codes as in detlsh_build_index.  Used to feed the query phase with
 * an encoding computed elsewhere.  Same limits and ownership as above.
 */
detlsh_status detlsh_index_import(const float* X, int64_t n, int32_t d, int32_t L,
                                  int32_t K, int32_t N_r, const float* A,
                                  const float* B, const uint8_t* codes,
                                  const detlsh_build_opts* opts, void* stream,
                                  detlsh_index* out);

typedef struct {
    int64_t n;
    int32_t d, L, K, N_r;
    int64_t n_s;                 /* breakpoint sample size                         */
    int32_t max_leaf;
    int32_t has_bf16;
    int64_t n_leaves[8];         /* leaf runs per tree (first L entries valid)     */
    size_t device_bytes;         /* device memory owned by the index               */
} detlsh_info;

detlsh_status detlsh_index_info(detlsh_index idx, detlsh_info* out);

/*
 * Copy encoding results to host buffers (any pointer may be NULL to skip it):
 * A ((L*K) x d), B ((L*K) x (N_r+1)), codes (n x (L*K), column e = i*K+j) and
 * the sample ids (n_s).
 */
detlsh_status detlsh_export(detlsh_index idx, float* A, float* B, uint8_t* codes,
                            int64_t* sample_ids);

/*
 * Copy DE-Tree `tree` (0-based) to host buffers: perm (n ids in leaf order),
 * leaf_start (n_leaves + 1 offsets into perm), leaf_lo / leaf_hi (n_leaves x K
 * lowest / highest region code of each leaf's node, i.e. its bit prefixes).
 * `cap` is the capacity of the leaf arrays in leaves; DETLSH_EINVAL if short.
 */
detlsh_status detlsh_export_tree(detlsh_index idx, int32_t tree, int32_t* perm,
                                 int32_t* leaf_start, uint8_t* leaf_lo,
                                 uint8_t* leaf_hi, int64_t cap);

/*
 * Projected coordinates of nq rows (device, nq x d) with the index's hashes:
 * out (device, nq x (L*K) FP32), h_ij(q) = a_ij . q (Eq. 1).
 */
detlsh_status detlsh_project(detlsh_index idx, const float* Q, int64_t nq, float* out,
                             void* stream);

/* ------------------------------------------------------------------------ */
/* query                                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t precision;          /* DETLSH_FP32 (default) or DETLSH_BF16_RERANK       */
    int32_t rerank_mult;        /* BF16 form keeps rerank_mult*k for the FP32 rerank;
                                   0 -> 4                                             */
    int32_t rmin_policy;        /* DETLSH_RMIN_MAGIC (default) or DETLSH_RMIN_FIXED  */
    int32_t max_rounds;         /* FIXED: radius rounds (1..64) before S = D; 0 -> 64 */
    double r_min;               /* FIXED: initial radius, > 0                        */
    size_t workspace_bytes;     /* per-call workspace budget; 0 -> 8 GiB             */
    int32_t verify;             /* candidate verification: 0 automatic, 1 gathered
                                   rows of S, 2 masked dense MFMA over all rows,
                                   3 as 2 with BF16 products screening for the FP32
                                   form (index built with keep_bf16; same results) */
    int32_t granularity;        /* DETLSH_POINT (0): a point enters by its cell's
                                   bound; DETLSH_LEAF (1): by its DE-Tree leaf's box
                                   (the query-phase optimisation; MAGIC only)       */
    int32_t filter;             /* range filter of the magic radius, point
                                   granularity (same candidates either way):
                                   0 automatic (the screen when N_S <= 0.12 n),
                                   1 every bound of every pair evaluated,
                                   2 an MFMA screen by the ball around each cell
                                   (clamped to the interior breakpoint range),
                                   then the exact bounds of the pairs it keeps
                                   (L <= 4; other shapes use 1)                   */
} detlsh_query_opts;

/* Candidate granularity of the range query. */
enum {
    DETLSH_POINT = 0,
    DETLSH_LEAF = 1             /* a leaf whose bound is within the radius gives all
                                   its points; the stop tree's leaves are taken in
                                   order of (bound, smallest point id) until |S|
                                   reaches N_S, so the query may stop inside a tree */
};

/*
 * c^2-k-ANN query (Alg. 7) for nq rows of Q (device, nq x d FP32).
 *
 * The candidate predicate of tree i at radius r is LB_i(q,o)^2 <= (eps r)^2,
 * where LB_i is the distance from the projected query to the cell of o in the
 * i-th projected space (the box between the breakpoints around o's regions,
 * Sec. 4.3; the lowest region is open below, the highest open above) and
 * eps = sqrt(chi^2_{alpha1}(K)), alpha1 = e^{-1/L} (Lemma 3, Eq. 2).  Trees are
 * added to S in order 1..L; the query stops as soon as
 * |S| >= N_S = k + ceil(beta*n) (checked after every tree) or, after all L
 * trees, when k points of S lie within c*r; otherwise r <- c*r.  Under
 * DETLSH_RMIN_MAGIC the start radius is the smallest one satisfying both
 * conditions of the magic r_min (Sec. 5.2), so the query ends in its first
 * round.  If N_S >= n, S = D (MAGIC).  Under DETLSH_RMIN_FIXED the radii are
 * r_t = r_min c^t (t < max_rounds); a query that meets neither condition within
 * max_rounds rounds is answered over S = D; verification is the gathered FP32
 * form.
 *
 * out_ids (device, nq x k int64) and out_dists (device, nq x k FP32) receive
 * the k members of S nearest to each query, ascending by (distance, id);
 * N_S is computed in IEEE double from the double `beta` as k + ceil(beta*n);
 * distances are Euclidean (not squared).  Limits: 1 <= k <= min(n, 1024)
 * (the top-k keeps its k results and the candidates of its last radix digit
 * in LDS; BF16 form: rerank_mult*k <= 1024, needs an index built with keep_bf16),
 * c > 1, 0 <= beta <= 1, nq >= 0 (0 is a no-op), FIXED needs r_min > 0.
 *
 * Verification (both forms give the top-k of S by FP32 distance computed by
 * direct differences, ties by id): the gathered form reads the rows of S; the
 * masked dense form computes q.o for every row with MFMA, keeps members of S
 * whose ||q||^2 + ||o||^2 - 2 q.o lies within an upper bound of the k-th
 * distance plus the FP32 rounding bound of that expression, and re-ranks those
 * few exactly.  DETLSH_BF16_RERANK runs the dense products in BF16 (FP32
 * accumulation), keeps members within the (rerank_mult*k)-th exact distance of
 * a subset of S, and re-ranks them exactly in FP32.
 */
detlsh_status detlsh_query(detlsh_index idx, const float* Q, int64_t nq, int32_t k,
                           double c, double beta, const detlsh_query_opts* opts,
                           int64_t* out_ids, float* out_dists, void* stream);

/*
 * detlsh_query in stream order: every step is enqueued on `stream` after the
 * work already there, and the call returns without waiting for the device
 * (no host synchronisation anywhere on its path).  Q must stay valid, and the
 * outputs unread, until the stream has run past the call (for example: an
 * event recorded after it has completed, or a later synchronisation); its
 * workspace is reused by later calls only after that point.  Arguments,
 * limits and results are those of detlsh_query, plus out_status (device, nq
 * int32), written on the stream: 0 for a query answered as detlsh_query
 * answers it, 1 (MAGIC) when its candidate count left the planned range
 * [N_S, cap] of the sampled magic radius, 3 (FIXED) when the radius ladder
 * ended without a stop.  For a nonzero status the query's outputs are
 * unspecified: detlsh_query answers it (it runs those fallbacks itself; the
 * first is a probability below 1e-6 per query by the planned margins).
 * Calls on different streams run concurrently on the device.
 */
detlsh_status detlsh_query_async(detlsh_index idx, const float* Q, int64_t nq, int32_t k,
                                 double c, double beta, const detlsh_query_opts* opts,
                                 int64_t* out_ids, float* out_dists, int32_t* out_status,
                                 void* stream);

/*
 * (r, c)-ANN query (Alg. 6) for nq rows of Q (device, nq x d FP32) with one
 * search radius r >= 0: the L spaces are visited in order, space i adding the
 * points whose cell lies within eps*r of the projected query (the predicate of
 * detlsh_query); as soon as |S| >= ceil(beta*n) + 1 (the paper's beta*n + 1)
 * the point of S nearest to the query is returned; after all L spaces it is
 * returned if some point of S lies within c*r; otherwise nothing.
 * out_ids (device, nq int64) receives the point or -1 for nothing, out_dists
 * (device, nq FP32) its Euclidean distance or +inf.  Ties by the smaller id.
 * opts may be NULL; its precision must be DETLSH_FP32 (verification is the
 * gathered FP32 form); its radius fields are ignored.  Limits: r >= 0,
 * c > 1, 0 <= beta <= 1.
 */
detlsh_status detlsh_query_rc(detlsh_index idx, const float* Q, int64_t nq, double r, double c,
                              double beta, const detlsh_query_opts* opts, int64_t* out_ids,
                              float* out_dists, void* stream);

/* ------------------------------------------------------------------------ */
/* query without device allocation                                          */
/* ------------------------------------------------------------------------ */

/* Size of the fixed device array that detlsh_query_noalloc works in. */
#define DETLSH_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the query of
 * detlsh_query (magic radius; same arguments, same kernels, bit-identical
 * results) run entirely inside one fixed array of DETLSH_NOALLOC_SCRATCH_BYTES
 * bytes that the library's code object places on every device it runs on and
 * that stays there until the process ends.  No device memory is allocated or
 * freed.  Q, out_ids and out_dists are the caller's device buffers, as for
 * detlsh_query.  The array keeps the last call's contents; the query path
 * writes or clears everything it reads.  Overlapping calls on one device would
 * race on the array, so the library serialises them (a per-process lock) and
 * each call returns only after its work on `stream` is complete.
 * Limits: those of detlsh_query, DETLSH_RMIN_MAGIC only (FIXED: DETLSH_EINVAL),
 * and the array must hold one query with its fallback over all n points (about
 * 40 bytes per point) plus nq*L*K*4 bytes of query projections, else
 * DETLSH_ENOMEM with the sizes in the message.  Queries are run in as many
 * passes as the array requires.
 */
detlsh_status detlsh_query_noalloc(detlsh_index idx, const float* Q, int64_t nq, int32_t k,
                                   double c, double beta, const detlsh_query_opts* opts,
                                   int64_t* out_ids, float* out_dists, void* stream);

/* DETLSH_NOALLOC_SCRATCH_BYTES as compiled into the library. */
size_t detlsh_noalloc_scratch_bytes(void);

/* ------------------------------------------------------------------------ */
/* incremental insertion                                                    */
/* ------------------------------------------------------------------------ */

/*
 * Append m points (X_new: device, m x d FP32) to the index; they get ids
 * n .. n+m-1.  The encoding is frozen: the new points are projected with the
 * index's A and encoded against its breakpoints (Alg. 2), the DE-Trees are
 * rebuilt over all codes (bulk build, so the index equals one imported with
 * the concatenated codes), and derived arrays follow.  X_new is copied.  Must
 * not run concurrently with queries or servers on the index.  Limits: m >= 0
 * (0 is a no-op), n + m < 2^31; DETLSH_ENOMEM leaves the index unchanged.
 */
detlsh_status detlsh_insert(detlsh_index idx, const float* X_new, int64_t m, void* stream);

/* ------------------------------------------------------------------------ */
/* persistence                                                              */
/* ------------------------------------------------------------------------ */

/*
 * Write the index to a file (checkpoint): a header (n, d, L, K, N_r, n_s,
 * max_leaf, BF16 options), then A, B, the sample ids, the codes and X, and a
 * 64-bit checksum of the payload.  Derived arrays (trees, norms, BF16 copies,
 * the guess subset) are not stored; detlsh_index_load rebuilds them from the
 * codes, so a loaded index answers every query bit-identically.  path is a
 * host string; an existing file is replaced.  DETLSH_EINVAL if the file cannot
 * be written.
 */
detlsh_status detlsh_index_save(detlsh_index idx, const char* path);

/*
 * Read an index written by detlsh_index_save onto the current device.
 * DETLSH_EINVAL for a file that is missing, truncated, of another format or
 * whose checksum does not match; DETLSH_ENOMEM if it does not fit.
 */
detlsh_status detlsh_index_load(const char* path, void* stream, detlsh_index* out);

/*
 * detlsh_query with every intermediate exposed, for step-by-step checks.
 * Qp (device, nq x (L*K) FP32) replaces the query projections when not NULL.
 * For each query t it writes: cand_counts[t] = |S|; cand_ids[t*cand_cap + s]
 * (device int32, s < min(|S|, cand_cap)) the members of S in no particular
 * order;
 * first_tree[t*cand_cap + s] the 1-based first tree whose range query
 * admitted that member; thr[t] = the squared projected radius (eps r)^2 at
 * which the query stopped; stop_tree[t] = tree after which it stopped
 * (1-based); rounds[t] = radius rounds used.  Any of these pointers may be
 * NULL.  Results are identical to detlsh_query's.
 */
detlsh_status detlsh_query_debug(detlsh_index idx, const float* Qp, const float* Q,
                                 int64_t nq, int32_t k, double c, double beta,
                                 const detlsh_query_opts* opts, int32_t* cand_ids,
                                 int64_t cand_cap, int64_t* cand_counts,
                                 int32_t* first_tree, float* thr, int32_t* stop_tree,
                                 int32_t* rounds, int64_t* out_ids, float* out_dists,
                                 void* stream);

/* ------------------------------------------------------------------------ */
/* serving: continuous batching over a fixed device workspace               */
/* ------------------------------------------------------------------------ */

/*
 * A server answers many independent query requests (each an Alg. 7 query of
 * nq rows, as detlsh_query) on one index without allocating device memory per
 * request.  It owns `slots` worker threads, each with its own HIP stream of
 * default priority and an equal share of one workspace of workspace_bytes
 * allocated at creation.  Requests are taken in arrival order; when a slot
 * becomes free it forms a batch from the oldest waiting request and appends
 * the waiting queries of later requests with the same (k, beta, options, and
 * c under DETLSH_RMIN_FIXED; under MAGIC, c does not enter the computation),
 * up to max_batch queries or as many as its workspace holds (continuous
 * batching).  A request larger than that is served in pieces, possibly on
 * several slots at once.  Every query's result is independent of the batch it
 * ran in: a request returns bit-identical ids and distances alone or in a mix.
 *
 * detlsh_server_create: slots in [1, 16] (0 -> 2), max_batch in [1, 65535]
 *   (0 -> 1024), workspace_bytes >= 1 MiB.  ENOMEM if the workspace cannot be
 *   allocated.  The index must outlive the server.
 */
typedef struct detlsh_server_s* detlsh_server;

detlsh_status detlsh_server_create(detlsh_index idx, size_t workspace_bytes, int32_t slots,
                                   int32_t max_batch, detlsh_server* out);

/*
 * Queue a request.  Q (device, nq x d FP32), out_ids (device, nq x k int64)
 * and out_dists (device, nq x k FP32) must stay valid until detlsh_server_wait
 * has returned something other than DETLSH_EBUSY for the ticket.  The server
 * reads Q on its own streams: the work that writes Q must be complete when
 * submit is called, and the outputs are complete when wait returns DETLSH_OK.  opts is
 * copied (NULL -> FP32, MAGIC; its workspace_bytes is ignored).  Arguments are
 * checked here as detlsh_query checks them: an invalid request gets
 * DETLSH_EINVAL and no ticket, a request of which not one query fits a slot's
 * workspace gets DETLSH_ENOMEM; neither affects other requests.  nq == 0 is
 * accepted and completes at once.  *ticket identifies the request.
 */
detlsh_status detlsh_server_submit(detlsh_server srv, const float* Q, int64_t nq, int32_t k,
                                   double c, double beta, const detlsh_query_opts* opts,
                                   int64_t* out_ids, float* out_dists, uint64_t* ticket);

typedef struct {
    double t_submit;            /* CLOCK_MONOTONIC seconds: accepted by submit     */
    double t_start;             /* its first queries began on a slot               */
    double t_end;               /* its last results were complete in HBM           */
    int32_t batches;            /* batches that served its queries                 */
    int32_t max_batch_requests; /* most requests sharing one of those batches      */
    int64_t max_batch_queries;  /* most queries in one of those batches            */
} detlsh_request_info;

/*
 * Wait up to timeout_us microseconds (< 0: no limit, 0: poll) for a request.
 * Returns DETLSH_EBUSY if it is still running (the ticket stays valid);
 * otherwise the request's own status (DETLSH_OK, DETLSH_ECANCELED, or the
 * error of the batch that failed it, with its message in detlsh_last_error),
 * fills *info when info is not NULL, and releases the ticket.  DETLSH_EINVAL
 * for an unknown ticket.
 */
detlsh_status detlsh_server_wait(detlsh_server srv, uint64_t ticket, int64_t timeout_us,
                                 detlsh_request_info* info);

/*
 * Cancel a request: queries not yet started are dropped, queries already on a
 * slot finish, and the request then reports DETLSH_ECANCELED (its outputs
 * partly written).  DETLSH_OK if the cancellation took effect, DETLSH_EBUSY if
 * the request had already finished (wait reports its own status),
 * DETLSH_EINVAL for an unknown ticket.
 */
detlsh_status detlsh_server_cancel(detlsh_server srv, uint64_t ticket);

/*
 * Stop the server: requests not yet started are cancelled, running batches
 * finish, the threads are joined and the workspace freed.  Tickets not waited
 * for are discarded.  Must not race with other calls on the same server.
 */
void detlsh_server_destroy(detlsh_server srv);

/* ------------------------------------------------------------------------ */
/* kernel timing                                                            */
/* ------------------------------------------------------------------------ */

/*
 * While enabled, every kernel launch of the library is bracketed by HIP events
 * on the launch stream and its duration added to a per-kernel total.
 * detlsh_profile_read copies up to `max` entries (name, launches, total ms)
 * and returns their number in *count.  Process-wide; reset with `reset`.
 */
detlsh_status detlsh_profile_enable(int32_t on, int32_t reset);
detlsh_status detlsh_profile_read(const char** names, int64_t* launches, double* total_ms,
                                  int32_t max, int32_t* count);

/*
 * Work counters of the profiled queries, summed over every device while
 * profiling is enabled: "exact_survivors", the (query, point) pairs that the
 * range filter's MFMA screen kept and its exact pass evaluated, and
 * "exact_candidates", those whose exact key passed the threshold (the
 * candidates of Sec. 5.2's range query).  Copies up to `max` (name, value)
 * entries and returns their number in *count; waits for the device work the
 * library has enqueued.  detlsh_profile_enable(..., reset = 1) zeroes them.
 */
detlsh_status detlsh_profile_counters(const char** names, int64_t* values, int32_t max, int32_t* count);

/*
 * Measured issue rate of the range filter's bound arithmetic on the current
 * device: `lanes` synthetic cells (a multiple of 256), each against `nq`
 * projected queries with the filter's own per-(tree, dimension) sequence
 * (median-of-three clamp, subtraction, fused multiply-add: 3 operations) and
 * one minimum per tree, at L = 4, K = 16 (196 lane operations per cell and
 * query; the lower bounds of Sec. 4.3, readings R5 and R6).  Three launches
 * on the null stream; the fastest of the last two is reported as lane
 * operations per second in *lane_ops_per_s and its duration in *ms (may be
 * NULL).  Synchronous; allocates from the device cache.  EINVAL on bad
 * arguments, EDEVICE on a HIP error.
 */
detlsh_status detlsh_probe_valu(int32_t nq, int64_t lanes, double* lane_ops_per_s, double* ms);

void detlsh_free(detlsh_index idx);

/*
 * Device memory is cached per device instead of freed: a detlsh_query call
 * (also _rc and _debug) keeps its workspace when it returns normally (a call
 * that fails frees its own), and detlsh_free drains the device and keeps the
 * index's arrays.  Later calls take the smallest idle buffer that is large
 * enough (a build: at most twice the size it needs); at most 32 stay idle per
 * device.  detlsh_trim frees every idle buffer of the process on every
 * device, giving that memory back; buffers in use are not touched.  Any
 * thread, any time.  An allocation that fails trims the cache and retries.
 */
void detlsh_trim(void);
const char* detlsh_last_error(void);   /* thread-local; valid until the next call */

#ifdef __cplusplus
}
#endif
#endif /* DETLSH_H */
