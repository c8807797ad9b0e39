// Host-side layout of the graph storage and workspace, kernel argument
// blocks and launcher declarations.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "knng.h"

namespace knng {

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Scoring-row formats of the search.
enum RowFormat { ROW_I8 = 0, ROW_BF16 = 1, ROW_FP8 = 2, ROW_F32 = 3 };

// Storage (one graph at capacity N):
//   vec    [N][row_bytes]  scoring rows: int8 (uint8 coordinate - 128),
//                          bfloat16 or FP8 E4M3 codes; zero padded.  For
//                          float32 scoring this is the master array itself.
//   scale  [N]             float32 row scale (FP8 only)
//   master [N][mstride]    float32 rows (float graphs; mstride = dim rounded
//                          up to 4)
//   norms  [N]             squared norm: int32 (uint8 graphs) or float32
//   ids    [N][k_pad]      int32      list ids, sorted by (distance, id)
//   dist   [N][k_pad]      32-bit distance patterns (int32, or float32 bits);
//                          padding: id -1 and the largest pattern
//   head   [N]             int32      first pending proposal per node (-1)
struct StorageLayout {
  int dim = 0, k = 0, k_pad = 0, row_bytes = 0, format = ROW_I8, mstride = 0;
  int coord_bytes = 0;   // bytes of a scoring row's coordinates (<= row_bytes)
  int norm_off = -1;     // byte offset of a float32 row term inside the row, or -1
  bool is_float = false;
  bool cosine = false; // rows normalized to unit length (cosine metric)
  bool ip = false;     // inner-product metric: distances are sortable keys of -(x . y)
  int32_t pad = 0;     // distance padding pattern
  int64_t cap = 0;
  size_t off_vec = 0, off_scale = 0, off_qnorm = 0, off_master = 0, off_norms = 0, off_ids = 0,
         off_dist = 0, off_head = 0, total = 0;
};

// Workspace (calls of up to M points):
//   res_ids/res_d search results [M][k_pad]
//   evals/upd     per point counters
//   props         proposals [M * props_per_point] {target, dist, src, next}
//   touched       targets with at least one proposal
//   counters      [0] proposals, [1] touched
//   partial       brute-force split partial lists (keys)
//   keys          restart keys of a call
//   sets          visited / processed bitsets in global memory, one per
//                 block, for graphs whose bitset does not fit in LDS
//   cand          float exact graph: candidate keys of a chunk of nodes
//   fronts        update level arrays that do not fit in LDS, per block
//   qbuf          cosine metric: the normalized rows of a search's queries
struct WorkspaceLayout {
  int64_t M = 0;
  int64_t props_per_point = 0;
  int64_t partial_lists = 0;   // capacity in lists of k_pad keys
  int64_t set_slots = 0, set_words_pad = 0;
  int64_t cand_rows = 0;
  size_t off_res_ids = 0, off_res_d = 0, off_evals = 0,
         off_upd = 0, off_lreads = 0, off_props = 0, off_touched = 0, off_counters = 0, off_partial = 0,
         off_keys = 0, off_sets = 0, off_cand = 0, off_fronts = 0, off_qbuf = 0, total = 0;
};

struct Proposal {
  int32_t target;
  int32_t dist;
  int32_t src;
  int32_t next;
};

// ---- kernel argument blocks -------------------------------------------------
struct IngestArgs {
  const uint8_t* x;    // [m][dim]
  int8_t* dst;         // [m][row_bytes]
  int32_t* norms;      // [m]
  int64_t m;
  int dim, row_bytes;
};

struct IngestF32Args {
  const float* x;      // [m][dim]
  float* master;       // [m][stride]
  float* norms;        // [m]
  char* score;         // [m][row_bytes] (BF16 / FP8 formats)
  float* scale;        // [m] (FP8)
  float* qnorm;        // [m] (FP8): squared norm of the quantized row, scale^2 sum v^2
  int64_t m;
  int dim, stride, row_bytes, format;
  int coord_bytes;     // bytes of the row's coordinates
  int norm_off;        // >= 0: the squared norm of the stored row (float32) at this byte
                       // offset of the row, zeros after it to the end of the row
  int cosine;          // normalize rows to unit length first
  float* qout;         // if set: write only the normalized rows [m][dim] here
};

struct ExactArgs {
  const void* qvec; const uint32_t* qnorm; int32_t nq; int32_t q_id_base;
  const void* dvec; const uint32_t* dnorm; int32_t nd; int32_t d_id_base;
  int row_bytes, k;
  int32_t split_len;     // database rows per split (multiple of the tile)
  int32_t nsplit;
  int exclude_self;      // skip database id == query id
  int ip;                // float32: candidates by the inner product (keys of -(q . x))
  int32_t* out_ids; int32_t* out_d; int out_stride;   // when nsplit == 1 and no cand
  uint64_t* partial;     // [nsplit][nq][k] keys when nsplit > 1
  uint64_t* cand;        // float32: [nq][km] candidate keys
};

struct RerankArgs {
  const float* rows; int stride; int dim;   // float32 rows of the graph
  int32_t q_id_base; int32_t nq;            // nodes q_id_base .. + nq - 1
  const uint64_t* cand; int km;             // [nq][km] candidate keys
  int k;
  int ip;                                   // inner-product dissimilarity keys
  int32_t* out_ids; int32_t* out_d; int out_stride;
};

// One group of search rows: its queries, restart keys and outputs.
struct SearchRows {
  const int8_t* qvec;    // uint8 graphs: ingested query rows [count][row_bytes], or null:
  const void* qraw;      // raw queries [count][dim] (uint8 or float32)
  const uint64_t* keys; uint64_t key_base;   // key = keys ? keys[i] : key_base + i
  int32_t* out_ids; int32_t* out_d; int out_stride;
  int32_t* out_evals;
  int32_t* out_list_reads;   // neighbour lists read per query (may be null)
  int32_t* trace; int64_t trace_stride;
  int32_t count;
  int decode;            // write float32 dissimilarities, not sortable keys (inner product)
};

struct SearchArgs {
  int format;                              // RowFormat of vec
  const void* vec; int row_bytes;          // scoring rows
  int coord_bytes;                         // bytes of a row's coordinates (<= row_bytes)
  int side2_off;                           // >= 0: side2 is the float32 at this byte offset
                                           // of the row rather than in the side2 array
  const uint32_t* side;                    // per-row value: int8 norms, FP8 scales
  const uint32_t* side2;                   // second per-row value: the squared norm of the
                                           // stored row (FP8 with its scale, or bfloat16)
  const float* master; int master_stride; int master_chunks;   // float graphs (re-rank)
  const int32_t* nbr_ids; int k, k_pad;
  int keep;              // result entries kept by the search (k, more before a re-rank)
  int32_t n;             // snapshot size
  int32_t B;             // budget
  uint32_t m_mod;        // permutation modulus m = 2^ceil(log2 n)
  int32_t e_num, e_den;
  uint64_t seed;
  int dim;
  // rows [0, rows[0].count) come from group 0, the next rows[1].count from
  // group 1 (one launch searches both on the same snapshot)
  SearchRows rows[2];
  int32_t m;             // rows[0].count + rows[1].count (set by the launcher)
  uint32_t pad_bits;     // distance padding of absent entries
  int ip;                // inner-product metric: keys of -(q . x), additive expansion test
  float ip_margin;       // ln(e_num / e_den): the inner-product expansion margin
  uint32_t* gvis; int64_t gvis_slots;  // global visited sets (null: LDS)
  int32_t vis_words, vis_words_pad;    // set by the launcher from n
  int32_t restarts;      // GNNS mode: number of restarts (launch_search_gnns)
  unsigned long long* step_counters;   // profiling build: KNNG_NUM_STEP_COUNTERS totals
  // partitioned search (launch_search_part): node -> partition, partitions,
  // and the budget of each partition
  const int32_t* node_part; int32_t nparts; const int32_t* part_budget;
};

// Balanced k-medoids (partition.hip).  Rows of the distance evaluations as
// in UpdateArgs (int8 rows or float32 rows).
struct PartitionArgs {
  int format;
  const void* vec; int row_bytes; int dim;
  int32_t n, p;
  int64_t N, P;                 // capacity weight: w(m) = N - |C(m)| P
  int32_t* medoids;             // [p]
  uint32_t* D;                  // [n][p] distance bits node -> medoid
  int32_t* part;                // [n]
  int32_t* members;             // [n] node ids grouped by partition, ascending
  int32_t* offsets;             // [p + 1]
  double* sums;                 // [n] sum of path lengths to the reached members
  int32_t* unreached;           // [n] members of the own partition not reached
  int is_float;
  // the graph, taken as undirected: stored lists (out-edges) and in-edges
  const int32_t* nbr_ids; const int32_t* nbr_d; int k, k_pad;
  const int32_t* in_off;        // [n + 1] in-edge offsets
  const int32_t* in_src;        // [n k] source of each in-edge
  const int32_t* in_w;          // [n k] its stored distance bits
  int32_t* pos;                 // [n] index of a node within its partition's members
  // per-slot shortest-path scratch (one wavefront per slot, slot_len entries)
  uint64_t* sp_dist; int32_t* sp_cur; int32_t* sp_next; int32_t* sp_inq;
  int32_t slots; int64_t slot_len;
};

struct PeerArgs {
  int format;                                     // ROW_I8 or ROW_F32 (float rows)
  const void* bvec; int row_bytes; int dim;       // batch rows, ids id_base + i
  int32_t b; int32_t id_base;
  int k, k_pad;
  const int32_t* res_ids; const int32_t* res_d;   // search results [b][k_pad]
  int32_t* list_ids; int32_t* list_d;             // lists of the new nodes [b][k_pad]
  int32_t pad;
  int ip;                                         // inner-product dissimilarity keys
};

struct UpdateArgs {
  int format;                                     // ROW_I8 or ROW_F32 (float rows)
  const void* vec; int row_bytes; int dim;        // rows of the distance evaluations
  int32_t* nbr_ids; int32_t* nbr_d; int k, k_pad;
  int32_t* head;
  const void* bvec; int32_t b; int32_t id_base;
  const int32_t* res_ids; const int32_t* res_d;
  int depth;
  Proposal* props; int32_t* touched; int32_t* counters;
  const int32_t* evals; const int32_t* list_reads;
  int32_t* sims;                                  // may be null
  int32_t* stats;                                 // [b][3] or null
  int32_t n;             // snapshot size (processed-set bitset covers [0, n))
  uint32_t* gset; int64_t gset_slots;             // global processed sets (null: LDS)
  int32_t set_words, set_words_pad;   // set by the launcher from n
  int front_cap;         // slots of one level array (largest expanded level)
  int32_t* gfront;       // level arrays in global memory [b][2][front_cap] (null: LDS)
  int ip;                      // inner-product dissimilarity keys
};

struct MergeArgs {
  int32_t* nbr_ids; int32_t* nbr_d; int k, k_pad;
  int32_t* head;
  const Proposal* props; const int32_t* touched; const int32_t* counters;
  int32_t max_touched;
  int32_t pad;
};

// ---- LDS needs of the online kernels (bytes per wavefront) -------------------
size_t search_lds_bytes(int64_t n, int k_pad, bool global_visited);
size_t update_lds_bytes(int64_t n, int64_t front_cap, bool global_set, bool global_front);
constexpr size_t LDS_LIMIT = 65536;
// Bitsets up to this size stay in LDS; larger graphs use global bitsets.
constexpr size_t LDS_SET_LIMIT = 40960;
// bfloat16 rows of up to this many coordinates are scored on the matrix
// cores and carry their squared norm inside the row.
constexpr int BF16_MFMA_DIM = 128;

// ---- launchers (each returns the hipError_t of its launch) ------------------
hipError_t launch_ingest_u8(const IngestArgs& a, hipStream_t s);
hipError_t launch_ingest_f32(const IngestF32Args& a, hipStream_t s);
hipError_t launch_exact_u8(const ExactArgs& a, hipStream_t s);
hipError_t launch_merge_lists(int32_t* ids, int32_t* d, const int32_t* tids, const int32_t* td,
                              int k_pad, int k, int64_t count, int32_t pad, hipStream_t s);
hipError_t launch_exact_f32(const ExactArgs& a, int km, hipStream_t s);
hipError_t launch_rerank_f32(const RerankArgs& a, hipStream_t s);
hipError_t launch_split_merge(const uint64_t* partial, int32_t nq, int32_t nsplit, int k,
                              int32_t* out_ids, int32_t* out_d, int out_stride, hipStream_t s);
hipError_t launch_search(const SearchArgs& a, hipStream_t s);
hipError_t launch_search_gnns(const SearchArgs& a, hipStream_t s);
hipError_t launch_search_part(const SearchArgs& a, hipStream_t s);
hipError_t launch_partition_iteration(const PartitionArgs& a, hipStream_t s);
hipError_t launch_in_edges(const PartitionArgs& a, int32_t* counts, hipStream_t s);
hipError_t launch_set_medoids(int32_t* medoids, const int32_t* host_ids, int p, hipStream_t s);
hipError_t launch_part_budgets(const int32_t* part, int32_t n, int32_t p, int k, int speedup,
                               int32_t* counts, int32_t* budgets, hipStream_t s);
hipError_t launch_merge_partitions(const int32_t* ids, const int32_t* d, const int32_t* evals,
                                   int stride, int32_t m, int32_t p, int k, int32_t* out_ids,
                                   int32_t* out_d, int out_stride, int32_t* out_evals,
                                   int32_t pad, hipStream_t s);
hipError_t launch_search_bf16(const SearchArgs& a, hipStream_t s, unsigned grid, size_t lds);
hipError_t launch_search_fp8(const SearchArgs& a, hipStream_t s, unsigned grid, size_t lds);
hipError_t launch_search_f32(const SearchArgs& a, hipStream_t s, unsigned grid, size_t lds);
hipError_t launch_search_f32_gnns(const SearchArgs& a, hipStream_t s, unsigned grid,
                                  size_t lds);
hipError_t launch_search_f32_part(const SearchArgs& a, hipStream_t s, unsigned grid,
                                  size_t lds);
hipError_t launch_peers(const PeerArgs& a, hipStream_t s);
hipError_t launch_update(const UpdateArgs& a, hipStream_t s);
hipError_t launch_merge(const MergeArgs& a, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s);
hipError_t launch_copy_lists(const int32_t* src_ids, const int32_t* src_d, int src_stride,
                             int32_t* dst_ids, int32_t* dst_d, int dst_stride, int64_t rows,
                             int k, int64_t id_limit, int32_t pad, hipStream_t s, int mode = 0);
hipError_t launch_export_u8(const int8_t* vec, int row_bytes, int dim, int64_t rows,
                            uint8_t* out, hipStream_t s);
hipError_t launch_export_f32(const float* rows, int stride, int dim, int64_t count, float* out,
                             hipStream_t s);

}  // namespace knng
