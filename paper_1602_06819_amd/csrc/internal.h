// Host-side layout of the graph storage and workspace, kernel argument
// blocks and launcher declarations.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "knng.h"

namespace knng {

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Storage (one graph at capacity N):
//   vec    [N][row_bytes]  int8 rows  (uint8 coordinate - 128, zero padded)
//   norms  [N]             int32      (sum of squares of the int8 row)
//   ids    [N][k_pad]      int32      list ids, sorted by (distance, id)
//   dist   [N][k_pad]      int32      list distances (padding INT32_MAX / -1)
//   head   [N]             int32      first pending proposal per node (-1)
struct StorageLayout {
  int dim = 0, k = 0, k_pad = 0, row_bytes = 0;
  int64_t cap = 0;
  size_t off_vec = 0, off_norms = 0, off_ids = 0, off_dist = 0, off_head = 0, total = 0;
};

// Workspace (calls of up to M points):
//   res_ids/res_d search results [M][k_pad]
//   evals/upd     per point counters
//   props         proposals [M * props_per_point] {target, dist, src, next}
//   touched       targets with at least one proposal
//   counters      [0] proposals, [1] touched
//   partial       brute-force split partial lists (keys)
struct WorkspaceLayout {
  int64_t M = 0;
  int64_t props_per_point = 0;
  int64_t partial_lists = 0;   // capacity in lists of k_pad keys
  size_t off_res_ids = 0, off_res_d = 0, off_evals = 0,
         off_upd = 0, off_lreads = 0, off_props = 0, off_touched = 0, off_counters = 0, off_partial = 0,
         off_keys = 0, total = 0;
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

struct ExactArgs {
  const int8_t* qvec; const int32_t* qnorm; int32_t nq; int32_t q_id_base;
  const int8_t* dvec; const int32_t* dnorm; int32_t nd; int32_t d_id_base;
  int row_bytes, k;
  int32_t split_len;     // database rows per split (multiple of the tile)
  int32_t nsplit;
  int exclude_self;      // skip database id == query id
  int32_t* out_ids; int32_t* out_d; int out_stride;   // when nsplit == 1
  uint64_t* partial;     // [nsplit][nq][k] keys when nsplit > 1
};

struct SearchArgs {
  const int8_t* vec; int row_bytes;
  const int32_t* nbr_ids; int k, k_pad;
  int32_t n;             // snapshot size
  int32_t B;             // budget
  uint32_t m_mod;        // permutation modulus m = 2^ceil(log2 n)
  int32_t e_num, e_den;
  uint64_t seed;
  const int8_t* qvec;    // ingested query rows [m][row_bytes], or null:
  const uint8_t* qraw;   // raw uint8 queries [m][dim]
  int dim;
  int32_t m;
  const uint64_t* keys; uint64_t key_base;   // key = keys ? keys[i] : key_base + i
  int32_t* out_ids; int32_t* out_d; int out_stride;
  int32_t* out_evals;
  int32_t* out_list_reads;   // neighbour lists read per query (may be null)
  int32_t* trace; int64_t trace_stride;
  int32_t vis_words, vis_words_pad;   // set by the launcher from n
};

struct PeerArgs {
  const int8_t* bvec; const int32_t* bnorm; int32_t b; int32_t id_base;   // batch rows, ids id_base + i
  int row_bytes, k, k_pad;
  const int32_t* res_ids; const int32_t* res_d;   // search results [b][k_pad]
  int32_t* list_ids; int32_t* list_d;             // lists of the new nodes [b][k_pad]
};

struct UpdateArgs {
  const int8_t* vec; int row_bytes;
  int32_t* nbr_ids; int32_t* nbr_d; int k, k_pad;
  int32_t* head;
  const int8_t* bvec; const int32_t* bnorm; int32_t b; int32_t id_base;
  const int32_t* res_ids; const int32_t* res_d;
  int depth;
  Proposal* props; int32_t* touched; int32_t* counters;
  const int32_t* evals; const int32_t* list_reads;
  int32_t* sims;                                  // may be null
  int32_t* stats;                                 // [b][3] or null
  int32_t n;             // snapshot size (processed-set bitset covers [0, n))
  int32_t set_words, set_words_pad;   // set by the launcher from n
  int front_cap;         // slots of one level array (largest expanded level)
};

struct MergeArgs {
  int32_t* nbr_ids; int32_t* nbr_d; int k, k_pad;
  int32_t* head;
  const Proposal* props; const int32_t* touched; const int32_t* counters;
  int32_t max_touched;
};

// ---- LDS needs of the online kernels (bytes per wavefront) -------------------
size_t search_lds_bytes(int64_t n, int k_pad);
size_t update_lds_bytes(int64_t n, int64_t front_cap);
constexpr size_t LDS_LIMIT = 65536;

// ---- launchers (each returns the hipError_t of its launch) ------------------
hipError_t launch_ingest_u8(const IngestArgs& a, hipStream_t s);
hipError_t launch_exact_u8(const ExactArgs& a, hipStream_t s);
hipError_t launch_split_merge(const uint64_t* partial, int32_t nq, int32_t nsplit, int k,
                              int32_t* out_ids, int32_t* out_d, int out_stride, hipStream_t s);
hipError_t launch_search_u8(const SearchArgs& a, hipStream_t s);
hipError_t launch_peers_u8(const PeerArgs& a, hipStream_t s);
hipError_t launch_update_u8(const UpdateArgs& a, hipStream_t s);
hipError_t launch_merge(const MergeArgs& a, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s);
hipError_t launch_copy_lists(const int32_t* src_ids, const int32_t* src_d, int src_stride,
                             int32_t* dst_ids, int32_t* dst_d, int dst_stride, int64_t rows,
                             int k, int64_t id_limit, hipStream_t s);
hipError_t launch_export_u8(const int8_t* vec, int row_bytes, int dim, int64_t rows,
                            uint8_t* out, hipStream_t s);

}  // namespace knng
