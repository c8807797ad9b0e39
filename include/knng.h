/*
 * knng.h -- C ABI of the MI355X (gfx950) online approximate k-nn graph
 * builder of "Fast Online k-nn Graph Building" (Debatty, Michiardi & Mees,
 * arXiv 1602.06819).
 *
 * One GPU holds one graph: the points, one adjacency list of the k most
 * similar nodes per node (Section 1), and the bookkeeping for insertion.
 * Dissimilarity is the squared Euclidean distance (the paper's synthetic
 * data uses Euclidean distance, Section 8.1.1; squaring keeps the order).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Memory.  The library never allocates device memory.  The caller owns
 *    and allocates the graph storage and the workspace (sizes from
 *    knng_storage_bytes / knng_workspace_bytes, 256-byte aligned device
 *    pointers) and every input/output buffer.  Pointers named *_dev are
 *    device pointers; *_host are host pointers.  The handle keeps the
 *    storage and workspace pointers (they must outlive it) but no input or
 *    output pointer.
 *  - Streams.  Every call only enqueues work on `stream` (stream-ordered);
 *    inputs must stay valid, and outputs are only complete, once the stream
 *    has passed the call.  Calls on one handle must be issued on one stream
 *    (or ordered by the caller); calls on one handle are not thread safe.
 *  - Lists.  A list row holds min(k, n-1) entries sorted by the key
 *    (distance, id) ascending -- ties in distance go to the smaller id --
 *    followed by padding entries (id -1, distance INT32_MAX for uint8 data,
 *    +inf for float data).
 *  - Errors.  Every check (arguments, capacity, state) happens before any
 *    launch; on error nothing is enqueued and the graph is unchanged, so an
 *    insert is all-or-nothing.  knng_last_error() gives a thread-local text.
 *    A failed launch or an asynchronous device fault reported by HIP is
 *    returned as KNNG_EDEVICE.  No C++ exception crosses this ABI.
 */
#ifndef KNNG_H
#define KNNG_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct knng_graph knng_graph;   /* opaque handle */

typedef enum {
  KNNG_OK = 0,
  KNNG_EINVAL = -1,     /* invalid argument or unsupported combination   */
  KNNG_ECAPACITY = -2,  /* n + b would exceed params.capacity, or a call
                           exceeds params.max_batch                         */
  KNNG_ENOMEM = -3,     /* storage or workspace smaller than required      */
  KNNG_EDEVICE = -4,    /* a HIP call failed                               */
  KNNG_ESTATE = -5,     /* call not valid in the handle's state            */
  KNNG_EUNSUPPORTED = -6 /* not available in this build of the library    */
} knng_status;

typedef enum { KNNG_U8 = 0, KNNG_F32 = 1 } knng_dtype;

/* Stages timed by knng_timing_* (one HIP event pair per launch). */
typedef enum {
  KNNG_STAGE_INGEST = 0,  /* points -> stored rows                          */
  KNNG_STAGE_EXACT = 1,   /* brute-force tiles (knng_build_exact)           */
  KNNG_STAGE_SEARCH = 2,  /* iGNNS of the points of an insert batch         */
  KNNG_STAGE_PEERS = 3,   /* lists of the new nodes (search result + batch) */
  KNNG_STAGE_UPDATE = 4,  /* update proposals (Algorithm 2)                 */
  KNNG_STAGE_MERGE = 5,   /* proposals merged into the lists               */
  KNNG_STAGE_QUERY = 6,   /* iGNNS of knng_search / knng_query              */
  KNNG_NUM_STAGES = 7
} knng_stage;
typedef enum {
  KNNG_SCORE_EXACT = 0,
  KNNG_SCORE_BF16 = 1,
  KNNG_SCORE_FP8 = 2,
  KNNG_SCORE_BF16_MFMA = 3
} knng_score;

/* Dissimilarity.  KNNG_METRIC_L2: squared Euclidean distance.
 * KNNG_METRIC_COSINE (float data only): points are normalized to unit length
 * when stored and when searched, and the dissimilarity is the squared
 * distance of the normalized points, 2 (1 - cos), in [0, 4]; a zero vector
 * stays zero.  The method applies to any dissimilarity (Section 3).
 * KNNG_METRIC_INNER_PRODUCT (float data with KNNG_SCORE_EXACT only): the
 * dissimilarity is the negated inner product -(x . y), float32, possibly
 * negative; a similarity that is not a metric.  The expansion test takes the
 * similarity exp(x . y), so a candidate is dropped when its dissimilarity
 * exceeds the best one's by more than ln(expansion_num / expansion_den).
 * Every distance handed out or taken in (search results, knng_get_lists,
 * knng_load) is that float value; lists are ordered by it ascending (the
 * largest inner product first) and padded with +infinity.  Partitioning,
 * partitioned search and the GNNS baseline take the squared L2 distance
 * only and reject such a graph with KNNG_EINVAL. */
typedef enum {
  KNNG_METRIC_L2 = 0,
  KNNG_METRIC_COSINE = 1,
  KNNG_METRIC_INNER_PRODUCT = 2
} knng_metric;

/*
 * Parameters (Section 3 and Algorithm 2 of the paper).
 *  dim        coordinates per point: 1 .. 256 for uint8 data; for float
 *             data 1 .. 256 (KNNG_SCORE_EXACT), .. 512 (KNNG_SCORE_BF16),
 *             .. 1024 (KNNG_SCORE_FP8).
 *  k          list length, 1 .. 64.
 *  dtype      KNNG_U8: uint8 points, exact integer distances (int32);
 *             KNNG_F32: float32 points, float distances.
 *  score      how the search scores candidates (float data): KNNG_SCORE_EXACT
 *             float32 rows; KNNG_SCORE_BF16 bfloat16 copies (VALU dot
 *             products); KNNG_SCORE_BF16_MFMA the same rows scored on the
 *             bfloat16 matrix cores as |q|^2 - 2 q.x + |x|^2 (dim <= 128;
 *             each row carries its squared norm); KNNG_SCORE_FP8 E4M3 codes
 *             with a per-row scale (rows above 256 coordinates on the FP8
 *             matrix cores).  Reduced-precision scores keep 2k
 *             (bfloat16) or 4k (FP8) candidates, at most 128 (at most 64
 *             for k <= 16), and re-rank them by the float32 distance;
 *             every stored distance is float32.  KNNG_U8 requires
 *             KNNG_SCORE_EXACT.
 *  capacity   largest number of nodes the graph may ever hold (< 2^31).
 *  max_batch  largest batch (insert) or query count per call.
 *  speedup    iGNNS budget: B(n) = min(n, max(k, ceil(n / speedup)))
 *             similarity computations per search (Section 3), >= 1.
 *  expansion_num / expansion_den
 *             expansion coefficient e = num / den > 1 (Section 3): a random
 *             restart node r is discarded iff
 *             den * (1 + d_r) > num * (1 + d_best), i.e. similarity
 *             1 / (1 + d) below s_max / e.
 *  depth      DEPTH of the Update procedure (Algorithm 2), 1 .. 8, with
 *             k + k^2 + ... + k^depth <= 2^24 (the workspace holds that many
 *             proposal slots per batch point; k = 10 allows depth 7).
 *  seed       seed of the restart permutations (see knng_search).
 *  metric     knng_metric (0 = squared L2).
 */
typedef struct {
  int32_t  dim;
  int32_t  k;
  int32_t  dtype;          /* knng_dtype */
  int32_t  score;          /* knng_score */
  int64_t  capacity;
  int64_t  max_batch;
  int32_t  speedup;
  int32_t  expansion_num;
  int32_t  expansion_den;
  int32_t  depth;
  uint64_t seed;
  int32_t  metric;         /* knng_metric */
} knng_params;

/* Bytes of graph storage for params->capacity nodes (0 if params are
 * invalid; see knng_last_error). */
size_t knng_storage_bytes(const knng_params* params);

/* Bytes of workspace needed for calls of up to params->max_batch points
 * (0 if params are invalid). */
size_t knng_workspace_bytes(const knng_params* params);

/*
 * Build the exact k-nn graph of n points by brute force and return a new
 * handle in *out (Section 2.1, naive method: every pairwise distance, keep
 * the k best per node; Section 8.5.2 builds its initial and ground-truth
 * graphs this way).
 *  x_dev   [n][dim] uint8 or float32, row-major, device memory.
 *  n       2 .. capacity (lists hold min(k, n-1) entries).
 * The points are copied into the storage; node ids are 0 .. n-1.
 */
knng_status knng_build_exact(const knng_params* params, const void* x_dev, int64_t n,
                             void* storage_dev, size_t storage_bytes,
                             void* workspace_dev, size_t workspace_bytes,
                             hipStream_t stream, knng_graph** out);

/*
 * Create a handle from points and lists supplied by the caller (for
 * example a saved graph).  ids_dev [n][k] int32 and d_dev [n][k] (int32 for
 * uint8 data, float for float data) must already satisfy the list
 * convention above; they are copied into the storage.
 */
knng_status knng_load(const knng_params* params, const void* x_dev, int64_t n,
                      const int32_t* ids_dev, const void* d_dev,
                      void* storage_dev, size_t storage_bytes,
                      void* workspace_dev, size_t workspace_bytes,
                      hipStream_t stream, knng_graph** out);

/*
 * iGNNS search (Section 3) of m points against the current graph, with
 * explicit restart keys.  Per query: random restarts drawn without
 * replacement along a keyed permutation of [0, n) (full-period LCG modulo
 * 2^ceil(log2 n), parameters from SplitMix64 of (seed, key)), each
 * discarded by the expansion test; eager first-improvement climbing along
 * the stored lists; stop right after B(n) distance evaluations.  Evaluated
 * nodes are never evaluated again.  The result is the k best evaluated
 * nodes by (distance, id).
 *  q_dev      [m][dim] points (uint8 or float32), device.
 *  keys_dev   [m] uint64 restart keys, device (an insert uses its new id).
 *  ids_dev    [m][k] int32 out;  d_dev [m][k] int32 / float out.
 *  evals_dev  [m] int32 out (distance evaluations), or NULL.
 *  list_reads_dev [m] int32 out (adjacency lists read by the climb), or NULL.
 *  trace_dev  [m][trace_stride] int32 out: evaluated ids in evaluation
 *             order, -1 after the last; or NULL.  trace_stride >= B(n).
 * Read-only with respect to the graph.  Any m >= 0 (below 2^31); with the
 * cosine metric the call's queries are normalized into the workspace, which
 * holds 2 * max_batch of them (KNNG_ECAPACITY beyond).
 */
knng_status knng_search(knng_graph* g, const void* q_dev, int64_t m,
                        const uint64_t* keys_dev, int32_t* ids_dev, void* d_dev,
                        int32_t* evals_dev, int32_t* list_reads_dev, int32_t* trace_dev,
                        int64_t trace_stride, hipStream_t stream);

/*
 * GNNS, the search iGNNS improves on (the baseline of the paper's
 * comparison): every restart (drawn along the same keyed permutation) is
 * climbed from; at each node every unvisited neighbour is evaluated and the
 * search moves to the closest of them, by (distance, id), if it is strictly
 * closer than the node; it stops after `restarts` restarts and their
 * climbs, or after B(n) evaluations (set speedup = 1 for no budget).
 * Evaluated nodes are never evaluated again.  Arguments as knng_search;
 * uint8 graphs, or float graphs with KNNG_SCORE_EXACT (float32 scoring;
 * KNNG_EINVAL otherwise).  Read-only.
 */
knng_status knng_search_gnns(knng_graph* g, const void* q_dev, int64_t m,
                             const uint64_t* keys_dev, int32_t restarts, int32_t* ids_dev,
                             void* d_dev, int32_t* evals_dev, int32_t* trace_dev,
                             int64_t trace_stride, hipStream_t stream);

/*
 * Insert a batch of b points (Algorithms 1 and 2, batch form).  With n the
 * size before the call, the points get ids n .. n+b-1 and:
 *  (i)   each is searched with iGNNS on the pre-batch graph, key = its id;
 *  (ii)  its list is the k best of its search result and the other batch
 *        points;
 *  (iii) Update: from its search result, nodes up to DEPTH-1 hops away along
 *        the pre-batch lists are each visited once; each receives a proposal
 *        (node, distance, new id);
 *  (iv)  every pre-batch list becomes the k best of itself and its
 *        proposals by (distance, id).
 * b = 1 is the paper's sequential insertion.
 *  x_dev          [b][dim] points, device.
 *  first_id_host  out: n (ids are first_id .. first_id + b - 1), or NULL.
 *  sims_dev       [b] int32 out: similarities spent per point (search
 *                 evaluations + (b - 1) peers + update evaluations), or NULL.
 *  stats_dev      [b][3] int32 out: per point (search evaluations,
 *                 adjacency lists read by the search, update evaluations),
 *                 or NULL.
 * Needs n + b <= capacity (KNNG_ECAPACITY otherwise) and b <= max_batch.
 */
knng_status knng_insert_batch(knng_graph* g, const void* x_dev, int64_t b,
                              int64_t* first_id_host, int32_t* sims_dev,
                              int32_t* stats_dev, hipStream_t stream);

/*
 * The naive method of Section 2.1 in online form, the baseline the paper's
 * search is measured against: insert b points (ids n .. n+b-1) by
 * comparing each with every node.  Each new node's list is its k best among
 * all n + b nodes, and each pre-batch node's list becomes the k best of
 * itself and the b new nodes, by (distance, id).  From an exact graph (e.g.
 * knng_build_exact) the graph stays exact; costs b (n + b) + n b distance
 * evaluations (brute-force tiles on the matrix cores, as knng_build_exact).
 *  x_dev          [b][dim] points, device.
 *  first_id_host  out: n, or NULL.
 * Needs n + b <= capacity (KNNG_ECAPACITY otherwise) and b <= max_batch.
 */
knng_status knng_insert_exact(knng_graph* g, const void* x_dev, int64_t b,
                              int64_t* first_id_host, hipStream_t stream);

/*
 * Read-only k-nn query of m points on the current graph (the k-nn search
 * problem of Section 2.2, answered with the iGNNS search of Section 3):
 * iGNNS with the keys 2^62 + s, where s counts every query this handle has
 * answered before (the first query of a handle has s = 0).  Any m >= 0
 * (below 2^31; cosine metric: at most 2 * max_batch per call).
 *  ids_dev [m][k] int32, d_dev [m][k] int32/float, evals_dev and
 *  list_reads_dev [m] int32 (as for knng_search) or NULL.
 */
knng_status knng_query(knng_graph* g, const void* q_dev, int64_t m,
                       int32_t* ids_dev, void* d_dev, int32_t* evals_dev,
                       int32_t* list_reads_dev, hipStream_t stream);

/*
 * One serving epoch: a batch of b insert points and m read-only queries
 * admitted together, all against the snapshot S of the n nodes present
 * before the call.  Equivalent to knng_query(q) on S followed by
 * knng_insert_batch(x) on S, with bit-identical results (the query keys are
 * the next m query-sequence keys; the insert keys are the new ids), but the
 * searches of both run in one launch.  Either part may be empty (b = 0 or
 * m = 0); b <= max_batch, n + b <= capacity (cosine metric: b + m <=
 * 2 * max_batch).
 *  x_dev          [b][dim] insert points, device (may be NULL if b = 0).
 *  q_dev          [m][dim] query points; q_ids_dev [m][k] int32 out,
 *                 q_d_dev [m][k] int32 / float out, q_evals_dev and
 *                 q_list_reads_dev [m] int32 out (as for knng_search) or NULL.
 *  first_id_host  out: n, or NULL.   sims_dev [b] int32 out, or NULL.
 *  stats_dev      [b][3] int32 out (as for knng_insert_batch), or NULL.
 */
knng_status knng_epoch(knng_graph* g, const void* x_dev, int64_t b, const void* q_dev,
                       int64_t m, int32_t* q_ids_dev, void* q_d_dev, int32_t* q_evals_dev,
                       int32_t* q_list_reads_dev, int64_t* first_id_host, int32_t* sims_dev,
                       int32_t* stats_dev, hipStream_t stream);

/*
 * Balanced k-medoids partitioning of the current graph's nodes into p
 * parts (Algorithm 4 on one compute node; Section 6).  capacity =
 * n * imb_num / (p * imb_den).  Initial medoids: the first p distinct ids of
 * the restart permutation keyed 2^61 (seed `seed`).  Each of `iters`
 * iterations assigns the nodes in id order, each to the medoid maximizing
 * similarity * (1 - size / capacity) with similarity 1 / (1 + d) (exact
 * comparisons; ties to the smaller medoid index), then computes each part's
 * new medoid from shortest paths in the graph (Section 6): over the k-nn
 * graph taken as undirected (u and v joined if either list holds the
 * other; edge length = the stored distance of the pair), through the
 * part's nodes only, the member that reaches the most members, then has
 * the smallest sum of path lengths to them (summed in increasing id order;
 * exact integers for uint8 graphs), then the smaller id.
 *  p              1 .. 64, at most n.   imb_num / imb_den in [1, 64].
 *  scratch_dev    device scratch of knng_partition_scratch_bytes(g, p)
 *                 bytes (about 20 n min(n, 256) bytes for the shortest-path
 *                 slots, plus O(n (p + k))), 256-byte aligned (owned by the
 *                 caller).
 *  part_dev       [n] int32 out: the part of every node (last assignment).
 *  medoids_dev    [p] int32 out: the medoids after the last update.
 */
size_t knng_partition_scratch_bytes(const knng_graph* g, int32_t p);
knng_status knng_partition(knng_graph* g, int32_t p, int32_t iters, int32_t imb_num,
                           int32_t imb_den, uint64_t seed, void* scratch_dev,
                           size_t scratch_bytes, int32_t* part_dev, int32_t* medoids_dev,
                           hipStream_t stream);

/*
 * Partitioned search (Algorithm 3 on one device): each query is searched
 * with iGNNS in every part separately -- within a part, nodes of other parts
 * are never drawn, evaluated or counted, and the budget is B(n_t) of the
 * part's size -- and the k best of the p partial results are returned.  All
 * m * p searches run in one launch.  uint8 graphs, or float graphs with
 * KNNG_SCORE_EXACT (not with the cosine metric).
 *  part_dev      [n] int32 part of each node (0 .. p-1), e.g. from
 *                knng_partition.
 *  scratch_dev   knng_search_partitioned_scratch_bytes(g, m, p) bytes.
 *  ids_dev, d_dev [m][k] out; evals_dev [m] out (sum over the parts) or NULL.
 */
size_t knng_search_partitioned_scratch_bytes(const knng_graph* g, int64_t m, int32_t p);
knng_status knng_search_partitioned(knng_graph* g, const void* q_dev, int64_t m,
                                    const uint64_t* keys_dev, const int32_t* part_dev, int32_t p,
                                    void* scratch_dev, size_t scratch_bytes, int32_t* ids_dev,
                                    void* d_dev, int32_t* evals_dev, hipStream_t stream);

/*
 * knng_search_partitioned without the caller's scratch, for callers that
 * cannot allocate device memory per call (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  The per-call
 * scratch (knng_search_partitioned_scratch_bytes(g, m, p) bytes) comes from
 * a static device array of 32 MiB that the library holds on every GPU it
 * runs on until the process ends; calls needing more return KNNG_ECAPACITY
 * (with k <= 16 and p = 8 that is about 31,000 queries per call).  Nothing
 * is allocated: no hipMalloc, hipFree or allocating library routine.  The
 * calling thread's current device must be the graph's device.  Every call
 * on one GPU shares that GPU's array, so calls that overlap on one GPU
 * (other streams, other threads, other handles) race; calls on one stream
 * are ordered.  Every byte of the scratch a call reads it has written
 * first, so the previous call's contents never reach a result.  Arguments
 * and results as knng_search_partitioned.
 */
knng_status knng_search_partitioned_noalloc(knng_graph* g, const void* q_dev, int64_t m,
                                            const uint64_t* keys_dev, const int32_t* part_dev,
                                            int32_t p, int32_t* ids_dev, void* d_dev,
                                            int32_t* evals_dev, hipStream_t stream);

/* Copy lists of nodes [first, first + count) out: ids_dev [count][k] int32,
 * d_dev [count][k] int32/float (either may be NULL). */
knng_status knng_get_lists(const knng_graph* g, int64_t first, int64_t count,
                           int32_t* ids_dev, void* d_dev, hipStream_t stream);

/* Copy points [first, first + count) out as [count][dim] in the input dtype
 * (for the cosine metric: the stored, unit-length points). */
knng_status knng_get_points(const knng_graph* g, int64_t first, int64_t count,
                            void* x_dev, hipStream_t stream);

/* Bytes of one scoring row of the search (the layout of knng_get_rows):
 * uint8 data: dim rounded up to 16 bytes of int8 (coordinate - 128);
 * float data: 2 * dim rounded up to 16 (KNNG_SCORE_BF16, bfloat16; with
 * KNNG_SCORE_BF16_MFMA followed by a 16-byte chunk whose first 4 bytes hold
 * the float32 squared norm of the stored bfloat16 row and the rest zeros),
 * dim rounded up to 16 (KNNG_SCORE_FP8, E4M3 codes),
 * or 4 * dim rounded up to 16 (KNNG_SCORE_EXACT, the float32 rows).  -1 for
 * a NULL handle. */
int32_t knng_row_bytes(const knng_graph* g);

/* Copy the scoring rows of nodes [first, first + count) out, as stored:
 * rows_dev [count][knng_row_bytes(g)] bytes (zero padded), and for
 * KNNG_SCORE_FP8 the row scales scale_dev [count] float (a node's
 * coordinates are approximated by scale * code).  Either pointer may be
 * NULL; scale_dev is ignored for other formats.  For checking the
 * quantizers: bfloat16 by round-to-nearest-even, E4M3 codes
 * RNE(x / scale) with scale = max |x| / 448 per row. */
knng_status knng_get_rows(const knng_graph* g, int64_t first, int64_t count, void* rows_dev,
                          float* scale_dev, hipStream_t stream);

/* Stage timing.  knng_timing_enable(g, 1) clears the accumulated times and
 * from then on records a HIP event pair on the call's stream around every
 * launch of each stage; knng_timing_enable(g, 0) stops recording.
 * knng_timing_read waits for the recorded events and returns, per stage,
 * the summed GPU milliseconds (ms_host[KNNG_NUM_STAGES]) and the number of
 * launches (launches_host[KNNG_NUM_STAGES]); either pointer may be NULL. */
knng_status knng_timing_enable(knng_graph* g, int enable);
knng_status knng_timing_read(knng_graph* g, double* ms_host, int64_t* launches_host);

/* Step counters of the iGNNS search kernel (Section 3), for profiling.
 * Only the profiling build of the library (compiled with
 * KNNG_STEP_COUNTERS: libknng_counters.so) counts; there every search
 * launch adds its searches' totals, and knng_step_counters waits for the
 * device, copies the KNNG_NUM_STEP_COUNTERS totals to counters_host (host
 * memory, uint64_t) and clears them if reset is nonzero.  The regular
 * build returns KNNG_EUNSUPPORTED.  A step is one gather-and-decide round
 * of a search: a restart window (up to 64 permutation positions) or a list
 * scan (the current node's list). */
typedef enum {
  KNNG_SC_SEARCHES = 0,         /* searches run                               */
  KNNG_SC_EVALUATIONS = 1,      /* similarity evaluations committed           */
  KNNG_SC_WINDOW_STEPS = 2,     /* restart-window steps                       */
  KNNG_SC_SCAN_STEPS = 3,       /* list-scan steps                            */
  KNNG_SC_WINDOW_CANDS = 4,     /* candidates of restart windows              */
  KNNG_SC_SCAN_CANDS = 5,       /* candidates of list scans                   */
  KNNG_SC_WINDOW_VISITED = 6,   /* window candidates found visited            */
  KNNG_SC_SCAN_VISITED = 7,     /* list candidates found visited              */
  KNNG_SC_WINDOW_COMMITTED = 8, /* evaluations committed by windows           */
  KNNG_SC_SCAN_COMMITTED = 9,   /* evaluations committed by list scans        */
  KNNG_SC_RESTARTS_TAKEN = 10,  /* restarts that started a climb              */
  KNNG_SC_MOVES = 11,           /* climb moves                                */
  KNNG_SC_WINDOW_KEPT = 12,     /* window candidates whose score was kept from
                                   the window before (not gathered again)     */
  KNNG_NUM_STEP_COUNTERS = 13
} knng_step_counter;
knng_status knng_step_counters(knng_graph* g, uint64_t* counters_host, int reset);

/* Number of nodes (counting every insert already enqueued). */
int64_t knng_size(const knng_graph* g);

/* The search budget B(n) = min(n, max(k, ceil(n / speedup))) for a graph
 * of n nodes (Section 3: n / speedup similarities per search); n < 0 means
 * the graph's current size.  -1 for a NULL handle. */
int64_t knng_budget(const knng_graph* g, int64_t n);

/* Number of queries answered by knng_query so far (the next query's s). */
int64_t knng_query_count(const knng_graph* g);

/* Thread-local text of the last error ("" if none). */
const char* knng_last_error(void);

/* Free the handle (no device memory is freed: the caller owns it). */
void knng_destroy(knng_graph* g);

#ifdef __cplusplus
}
#endif

#endif /* KNNG_H */
