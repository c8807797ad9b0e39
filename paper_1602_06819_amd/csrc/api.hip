// C ABI of the library (declared in include/knng.h): argument validation,
// storage/workspace layout and stream-ordered kernel launches.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "common.h"
#include "internal.h"
#include "knng.h"

using namespace knng;

// Opt-in stage timing: a pair of HIP events recorded on the caller's
// stream around every launch of a stage; read back (and summed) on demand.
struct StageTimer {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[KNNG_NUM_STAGES];
  std::vector<hipEvent_t> pool;
  double ms[KNNG_NUM_STAGES] = {};
  int64_t launches[KNNG_NUM_STAGES] = {};

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~StageTimer() {
    for (auto& v : pending)
      for (auto& pr : v) {
        hipEventDestroy(pr.first);
        hipEventDestroy(pr.second);
      }
    for (auto e : pool) hipEventDestroy(e);
  }
};

struct knng_graph {
  knng_params p;
  StorageLayout S;
  WorkspaceLayout W;
  char* st;
  size_t st_bytes;
  char* ws;
  size_t ws_bytes;
  int64_t n;
  int64_t qcount;
  StageTimer timer;
  unsigned long long* counters = nullptr;   // profiling build: step counters (device)
  ~knng_graph() {
    if (counters) (void)hipFree(counters);
  }
};

namespace {

thread_local std::string g_err;

knng_status fail(knng_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

knng_status ok() {
  g_err.clear();
  return KNNG_OK;
}

knng_status dev(hipError_t e, const char* what) {
  if (e == hipSuccess) return KNNG_OK;
  return fail(KNNG_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define KNNG_TRY(expr, what)                      \
  do {                                            \
    knng_status _s = dev((expr), (what));         \
    if (_s != KNNG_OK) return _s;                 \
  } while (0)

// Records start/stop events around the launches of one stage when timing
// is on.
class Timed {
 public:
  Timed(knng_graph* g, int stage, hipStream_t s) : g_(g), stage_(stage), s_(s) {
    if (g_ && g_->timer.on) {
      start_ = g_->timer.get();
      stop_ = g_->timer.get();
      if (start_ && stop_) hipEventRecord(start_, s_);
    }
  }
  ~Timed() {
    if (start_ && stop_) {
      hipEventRecord(stop_, s_);
      g_->timer.pending[stage_].push_back({start_, stop_});
    } else {
      if (start_) g_->timer.pool.push_back(start_);
      if (stop_) g_->timer.pool.push_back(stop_);
    }
  }

 private:
  knng_graph* g_;
  int stage_;
  hipStream_t s_;
  hipEvent_t start_ = nullptr, stop_ = nullptr;
};

constexpr size_t ALIGN = 256;
constexpr int64_t PARTIAL_LISTS = 32768;
// batches from this size on score their peers with the exact graph's tiles
// (one wavefront per point is cheaper below: a few short launches fewer)
constexpr int64_t PEER_TILE_MIN = 1024;
constexpr int64_t QUERY_KEY_BASE = (int64_t)1 << 62;

size_t take(size_t& cur, size_t bytes) {
  size_t off = cur;
  cur = (size_t)round_up((int64_t)(cur + bytes), ALIGN);
  return off;
}

int k_pad_of(int k) { return k <= 16 ? 16 : (k <= 32 ? 32 : 64); }

// Update sizes for DEPTH levels: at most k + k^2 + ... + k^depth processed
// nodes per new point; a level array holds the largest level that is
// expanded (k^(depth-1)).
struct UpdateSizes {
  int64_t props_per_point = 0;
  int64_t front_cap = 0;
};

UpdateSizes update_sizes(int k, int depth) {
  UpdateSizes u;
  int64_t level = 1;
  for (int l = 1; l <= depth; ++l) {
    level *= k;
    u.props_per_point += level;
    if (l == depth - 1) u.front_cap = level;
    if (u.props_per_point > (1 << 24)) break;
  }
  if (u.front_cap < k) u.front_cap = k;
  return u;
}

int64_t set_bytes(int64_t n) { return round_up((n + 31) / 32, 4) * 4; }

// Where the visited set of a search and the processed set of an update
// live: LDS while they fit, else per-block bitsets in the workspace.
bool search_sets_global(int64_t n) { return (size_t)set_bytes(n) > LDS_SET_LIMIT; }
// The update's two level arrays live in LDS up to 32 KiB, else in the
// workspace (one slice per block); its processed set in LDS while the set
// and the arrays held there fit.
bool update_fronts_global(int64_t front_cap) { return 8 * front_cap > 32768; }
bool update_sets_global(int64_t n, int64_t front_cap) {
  const size_t fronts = update_fronts_global(front_cap) ? 0 : 8 * (size_t)front_cap;
  return (size_t)set_bytes(n) + fronts > LDS_LIMIT;
}

int row_format(const knng_params& p) {
  if (p.dtype == KNNG_U8) return ROW_I8;
  if (p.score == KNNG_SCORE_BF16 || p.score == KNNG_SCORE_BF16_MFMA) return ROW_BF16;
  if (p.score == KNNG_SCORE_FP8) return ROW_FP8;
  return ROW_F32;
}

knng_status check_params(const knng_params* p) {
  if (!p) return fail(KNNG_EINVAL, "params is NULL");
  if (p->dim < 1 || p->dim > 4096) return fail(KNNG_EINVAL, "dim %d outside 1..4096", p->dim);
  if (p->k < 1 || p->k > 64) return fail(KNNG_EINVAL, "k %d outside 1..64", p->k);
  if (p->dtype != KNNG_U8 && p->dtype != KNNG_F32)
    return fail(KNNG_EINVAL, "unknown dtype %d", p->dtype);
  if (p->score != KNNG_SCORE_EXACT && p->score != KNNG_SCORE_BF16 &&
      p->score != KNNG_SCORE_FP8 && p->score != KNNG_SCORE_BF16_MFMA)
    return fail(KNNG_EINVAL, "unknown score %d", p->score);
  if (p->dtype == KNNG_U8 && p->score != KNNG_SCORE_EXACT)
    return fail(KNNG_EINVAL, "uint8 data requires KNNG_SCORE_EXACT");
  if (p->metric != KNNG_METRIC_L2 && p->metric != KNNG_METRIC_COSINE &&
      p->metric != KNNG_METRIC_INNER_PRODUCT)
    return fail(KNNG_EINVAL, "unknown metric %d", p->metric);
  if (p->metric == KNNG_METRIC_COSINE && p->dtype != KNNG_F32)
    return fail(KNNG_EINVAL, "the cosine metric needs float data");
  if (p->metric == KNNG_METRIC_INNER_PRODUCT &&
      (p->dtype != KNNG_F32 || p->score != KNNG_SCORE_EXACT))
    return fail(KNNG_EINVAL, "the inner-product metric needs float data with "
                             "KNNG_SCORE_EXACT");
  if (p->dtype == KNNG_U8 && p->dim > 256)
    return fail(KNNG_EINVAL, "uint8 data supports dim <= 256 (got %d)", p->dim);
  if (p->dtype == KNNG_F32) {
    const int lim = p->score == KNNG_SCORE_FP8            ? 1024
                    : p->score == KNNG_SCORE_BF16         ? 512
                    : p->score == KNNG_SCORE_BF16_MFMA    ? BF16_MFMA_DIM
                                                          : 256;
    if (p->dim > lim)
      return fail(KNNG_EINVAL, "float data with this score supports dim <= %d (got %d)", lim,
                  p->dim);
  }
  if (p->capacity < 2 || p->capacity >= ((int64_t)1 << 31))
    return fail(KNNG_EINVAL, "capacity %lld outside 2 .. 2^31-1", (long long)p->capacity);
  if (p->max_batch < 1 || p->max_batch > p->capacity)
    return fail(KNNG_EINVAL, "max_batch %lld outside 1 .. capacity", (long long)p->max_batch);
  if (p->speedup < 1) return fail(KNNG_EINVAL, "speedup must be >= 1");
  if (p->expansion_den < 1 || p->expansion_num <= p->expansion_den)
    return fail(KNNG_EINVAL, "expansion num/den must be > 1 with den >= 1");
  if (p->depth < 1 || p->depth > 8) return fail(KNNG_EINVAL, "depth must be 1 .. 8");
  {
    double level = 1.0, total = 0.0;
    for (int l = 1; l <= p->depth; ++l) {
      level *= p->k;
      total += level;
    }
    if (total > (double)(1 << 24))
      return fail(KNNG_EINVAL, "depth %d with k %d: k + ... + k^depth exceeds 2^24 update "
                               "slots per point", p->depth, p->k);
  }
  return KNNG_OK;
}

StorageLayout storage_layout(const knng_params& p) {
  StorageLayout S;
  S.dim = p.dim;
  S.k = p.k;
  S.k_pad = k_pad_of(p.k);
  S.format = row_format(p);
  S.is_float = p.dtype == KNNG_F32;
  S.cosine = p.metric == KNNG_METRIC_COSINE;
  S.ip = p.metric == KNNG_METRIC_INNER_PRODUCT;
  S.pad = S.ip ? (int32_t)SORT_INF : S.is_float ? (int32_t)0x7f800000 : DIST_PAD_I32;
  S.mstride = S.is_float ? (int)round_up(p.dim, 4) : 0;
  switch (S.format) {
    case ROW_I8: S.row_bytes = (int)round_up(p.dim, 16); break;
    case ROW_BF16:
      S.row_bytes = (int)round_up(2 * (int64_t)p.dim, 16);
      // rows scored on the matrix cores carry their squared norm in a
      // 16-byte chunk after the coordinates (read with the row)
      if (p.score == KNNG_SCORE_BF16_MFMA) {
        S.norm_off = S.row_bytes;
        S.row_bytes += 16;
      }
      break;
    case ROW_FP8: S.row_bytes = (int)round_up(p.dim, 16); break;
    default: S.row_bytes = S.mstride * 4; break;
  }
  S.coord_bytes = S.norm_off >= 0 ? S.norm_off : S.row_bytes;
  S.cap = p.capacity;
  size_t cur = 0;
  if (S.is_float) S.off_master = take(cur, (size_t)S.cap * S.mstride * 4);
  if (S.format == ROW_F32)
    S.off_vec = S.off_master;
  else
    S.off_vec = take(cur, (size_t)S.cap * S.row_bytes);
  if (S.format == ROW_FP8) S.off_scale = take(cur, (size_t)S.cap * 4);
  if (S.format == ROW_FP8) S.off_qnorm = take(cur, (size_t)S.cap * 4);
  S.off_norms = take(cur, (size_t)S.cap * 4);
  S.off_ids = take(cur, (size_t)S.cap * S.k_pad * 4);
  S.off_dist = take(cur, (size_t)S.cap * S.k_pad * 4);
  S.off_head = take(cur, (size_t)S.cap * 4);
  S.total = cur;
  return S;
}

// Candidates per node of the float exact graph (selected by the float32
// expansion, then re-ranked).
int exact_km(int k) { return k <= 20 ? 32 : 64; }
constexpr int64_t CAND_ROWS = 65536;

WorkspaceLayout workspace_layout(const knng_params& p, const StorageLayout& S) {
  WorkspaceLayout W;
  W.M = p.max_batch;
  const UpdateSizes us = update_sizes(p.k, p.depth);
  W.props_per_point = us.props_per_point;
  W.partial_lists = PARTIAL_LISTS;
  size_t cur = 0;
  const size_t M = (size_t)W.M;
  W.off_res_ids = take(cur, M * S.k_pad * 4);
  W.off_res_d = take(cur, M * S.k_pad * 4);
  W.off_evals = take(cur, M * 4);
  W.off_upd = take(cur, M * 4);
  W.off_lreads = take(cur, M * 4);
  W.off_props = take(cur, M * (size_t)W.props_per_point * sizeof(Proposal));
  W.off_touched = take(cur, M * (size_t)W.props_per_point * 4);
  W.off_counters = take(cur, 256);
  W.off_partial = take(cur, (size_t)W.partial_lists * S.k_pad * 8);
  W.off_keys = take(cur, M * 8);
  if (update_fronts_global(us.front_cap))
    W.off_fronts = take(cur, M * 2 * (size_t)us.front_cap * 4);
  if (search_sets_global(S.cap) || update_sets_global(S.cap, us.front_cap)) {
    W.set_slots = W.M;
    W.set_words_pad = set_bytes(S.cap) / 4;
    W.off_sets = take(cur, (size_t)W.set_slots * W.set_words_pad * 4);
  }
  if (S.cosine) W.off_qbuf = take(cur, 2 * M * (size_t)S.dim * 4);
  if (S.is_float) {
    W.cand_rows = S.cap < CAND_ROWS ? S.cap : CAND_ROWS;
    W.off_cand = take(cur, (size_t)W.cand_rows * exact_km(p.k) * 8);
  }
  W.total = cur;
  return W;
}

template <class T>
T* at(char* base, size_t off) {
  return reinterpret_cast<T*>(base + off);
}

int64_t budget(int64_t n, int k, int speedup) {
  int64_t b = (n + speedup - 1) / speedup;
  if (b < k) b = k;
  if (b > n) b = n;
  return b;
}

uint32_t modulus_for(int64_t n) {
  uint32_t m = 1;
  while ((int64_t)m < n) m <<= 1;
  return m;
}

knng_status check_ptr(const void* p, const char* name) {
  if (!p) return fail(KNNG_EINVAL, "%s is NULL", name);
  return KNNG_OK;
}

knng_status make_handle(const knng_params* p, void* storage, size_t storage_bytes,
                        void* workspace, size_t workspace_bytes, knng_graph** out) {
  knng_status s = check_params(p);
  if (s != KNNG_OK) return s;
  if (!out) return fail(KNNG_EINVAL, "out is NULL");
  if (!storage || !workspace) return fail(KNNG_EINVAL, "storage or workspace is NULL");
  if (((uintptr_t)storage % ALIGN) || ((uintptr_t)workspace % ALIGN))
    return fail(KNNG_EINVAL, "storage and workspace must be 256-byte aligned");
  StorageLayout S = storage_layout(*p);
  WorkspaceLayout W = workspace_layout(*p, S);
  if (storage_bytes < S.total)
    return fail(KNNG_ENOMEM, "storage has %zu bytes, needs %zu", storage_bytes, S.total);
  if (workspace_bytes < W.total)
    return fail(KNNG_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, W.total);
  knng_graph* g = new (std::nothrow) knng_graph;
  if (!g) return fail(KNNG_ENOMEM, "host allocation failed");
  g->p = *p;
  g->S = S;
  g->W = W;
  g->st = (char*)storage;
  g->st_bytes = storage_bytes;
  g->ws = (char*)workspace;
  g->ws_bytes = workspace_bytes;
  g->n = 0;
  g->qcount = 0;
  *out = g;
  return KNNG_OK;
}

// One search launch over one or two row groups (queries with their keys
// and outputs) on the current graph.
knng_status run_search(knng_graph* g, const SearchRows& r0, const SearchRows* r1, int stage,
                       hipStream_t stream, int32_t gnns_restarts = -1) {
  const StorageLayout& S = g->S;
  const WorkspaceLayout& W = g->W;
  SearchArgs a{};
  a.format = S.format;
  a.vec = at<char>(g->st, S.off_vec);
  a.row_bytes = S.row_bytes;
  a.side = S.format == ROW_FP8 ? at<uint32_t>(g->st, S.off_scale) : nullptr;
  a.side2 = S.format == ROW_FP8 ? at<uint32_t>(g->st, S.off_qnorm) : nullptr;
  a.coord_bytes = S.coord_bytes;
  a.side2_off = S.norm_off;
  if (S.is_float) {
    a.master = at<float>(g->st, S.off_master);
    a.master_stride = S.mstride;
    a.master_chunks = S.mstride / 4;
  }
  a.nbr_ids = at<int32_t>(g->st, S.off_ids);
  a.k = S.k;
  a.k_pad = S.k_pad;
  // reduced-precision scores keep more candidates for the float32 re-rank:
  // 2k for bfloat16 (8 significant bits), 4k for FP8 E4M3 (4), at most 128
  // (lists of up to 16 ids: at most 64)
  {
    const int mult = S.format == ROW_FP8 ? 4 : S.format == ROW_BF16 ? 2 : 1;
    const int cap = S.k_pad > 16 ? 128 : 64;
    a.keep = mult * S.k < cap ? mult * S.k : cap;
  }
  a.n = (int32_t)g->n;
  a.B = (int32_t)budget(g->n, S.k, g->p.speedup);
  a.m_mod = modulus_for(g->n);
  a.e_num = g->p.expansion_num;
  a.e_den = g->p.expansion_den;
  a.seed = g->p.seed;
  a.dim = S.dim;
  a.rows[0] = r0;
  if (r1) a.rows[1] = *r1;
  if (S.cosine) {
    // the searches read their queries normalized, as the stored rows are
    float* qbuf = at<float>(g->ws, W.off_qbuf);
    int64_t at_row = 0;
    for (int gi = 0; gi < 2; ++gi) {
      SearchRows& R = a.rows[gi];
      if (R.count <= 0) continue;
      if (at_row + R.count > 2 * W.M)
        return fail(KNNG_ECAPACITY, "cosine searches take at most max_batch queries per call");
      IngestF32Args n{};
      n.x = (const float*)R.qraw;
      n.m = R.count;
      n.dim = S.dim;
      n.cosine = 1;
      n.qout = qbuf + at_row * S.dim;
      KNNG_TRY(launch_ingest_f32(n, stream), "normalize launch");
      R.qraw = n.qout;
      at_row += R.count;
    }
  }
  a.pad_bits = (uint32_t)S.pad;
  a.ip = S.ip ? 1 : 0;
  a.ip_margin = (float)std::log((double)g->p.expansion_num / (double)g->p.expansion_den);
#ifdef KNNG_STEP_COUNTERS
  if (!g->counters) {
    KNNG_TRY(hipMalloc((void**)&g->counters, KNNG_NUM_STEP_COUNTERS * 8), "counter buffer");
    KNNG_TRY(hipMemset(g->counters, 0, KNNG_NUM_STEP_COUNTERS * 8), "counter buffer");
  }
  a.step_counters = g->counters;
#endif
  if (search_sets_global(g->n)) {
    a.gvis = at<uint32_t>(g->ws, W.off_sets);
    a.gvis_slots = W.set_slots;
  }
  Timed t(g, stage, stream);
  if (gnns_restarts >= 0) {
    a.restarts = gnns_restarts;
    KNNG_TRY(launch_search_gnns(a, stream), "search launch");
  } else {
    KNNG_TRY(launch_search(a, stream), "search launch");
  }
  return KNNG_OK;
}

// Row group of a read-only search: raw points, caller's outputs.
SearchRows query_rows(const void* q, int64_t m, const uint64_t* keys, uint64_t key_base,
                      int32_t* ids, void* d, int stride, int32_t* evals, int32_t* list_reads,
                      int32_t* trace, int64_t trace_stride, bool decode = false) {
  SearchRows r{};
  r.decode = decode ? 1 : 0;
  r.qraw = q;
  r.keys = keys;
  r.key_base = key_base;
  r.out_ids = ids;
  r.out_d = (int32_t*)d;
  r.out_stride = stride;
  r.out_evals = evals;
  r.out_list_reads = list_reads;
  r.trace = trace;
  r.trace_stride = trace_stride;
  r.count = (int32_t)m;
  return r;
}

// Row group of the points of an insert batch (stored at ids n .. n+b-1):
// results into the workspace, key = id.
SearchRows insert_rows(knng_graph* g, const void* x, int64_t b) {
  const StorageLayout& S = g->S;
  const WorkspaceLayout& W = g->W;
  SearchRows r{};
  if (S.is_float)
    r.qraw = x;
  else
    r.qvec = at<int8_t>(g->st, S.off_vec) + g->n * S.row_bytes;
  r.key_base = (uint64_t)g->n;
  r.out_ids = at<int32_t>(g->ws, W.off_res_ids);
  r.out_d = at<int32_t>(g->ws, W.off_res_d);
  r.out_stride = S.k_pad;
  r.out_evals = at<int32_t>(g->ws, W.off_evals);
  r.out_list_reads = at<int32_t>(g->ws, W.off_lreads);
  r.count = (int32_t)b;
  return r;
}

// Points -> stored rows (scoring rows, norms, float32 rows) at node ids
// first .. first + m - 1.
knng_status ingest(knng_graph* g, const void* x, int64_t m, int64_t first, hipStream_t stream) {
  const StorageLayout& S = g->S;
  Timed t(g, KNNG_STAGE_INGEST, stream);
  if (!S.is_float) {
    IngestArgs a{};
    a.x = (const uint8_t*)x;
    a.dst = at<int8_t>(g->st, S.off_vec) + first * S.row_bytes;
    a.norms = at<int32_t>(g->st, S.off_norms) + first;
    a.m = m;
    a.dim = S.dim;
    a.row_bytes = S.row_bytes;
    KNNG_TRY(launch_ingest_u8(a, stream), "ingest launch");
  } else {
    IngestF32Args a{};
    a.x = (const float*)x;
    a.master = at<float>(g->st, S.off_master) + first * S.mstride;
    a.norms = at<float>(g->st, S.off_norms) + first;
    a.score = S.format == ROW_F32 ? nullptr : at<char>(g->st, S.off_vec) + first * S.row_bytes;
    a.scale = S.format == ROW_FP8 ? at<float>(g->st, S.off_scale) + first : nullptr;
    a.qnorm = S.format == ROW_FP8 ? at<float>(g->st, S.off_qnorm) + first : nullptr;
    a.coord_bytes = S.coord_bytes;
    a.norm_off = S.norm_off;
    a.m = m;
    a.dim = S.dim;
    a.stride = S.mstride;
    a.row_bytes = S.row_bytes;
    a.format = S.format;
    a.cosine = S.cosine ? 1 : 0;
    KNNG_TRY(launch_ingest_f32(a, stream), "ingest launch");
  }
  return KNNG_OK;
}

// Exact lists of the stored nodes q_first .. q_first + nq - 1 against the
// stored nodes d_first .. d_first + nd - 1 (uint8: int8 MFMA tiles, split
// over the database when the queries are few; float32: float32 MFMA
// candidates per chunk of queries, then the float32 re-rank), excluding a
// node from its own list if `exclude_self`; k entries per row at out_ids /
// out_d with row stride out_stride.
knng_status exact_lists_range(knng_graph* g, int64_t q_first, int64_t nq, int64_t d_first,
                              int64_t nd, bool exclude_self, int32_t* out_ids, int32_t* out_d,
                              int out_stride, hipStream_t stream, bool split_ok = true,
                              int stage = KNNG_STAGE_EXACT) {
  const StorageLayout& S = g->S;
  const WorkspaceLayout& W = g->W;
  if (nq <= 0 || nd <= 0) return KNNG_OK;
  Timed t(g, stage, stream);
  const int rb = S.is_float ? S.mstride * 4 : S.row_bytes;
  const char* rows = S.is_float ? at<char>(g->st, S.off_master) : at<char>(g->st, S.off_vec);
  const uint32_t* norms = at<uint32_t>(g->st, S.off_norms);
  ExactArgs a{};
  a.qvec = rows + q_first * rb;
  a.qnorm = norms + q_first;
  a.nq = (int32_t)nq;
  a.q_id_base = (int32_t)q_first;
  a.dvec = rows + d_first * rb;
  a.dnorm = norms + d_first;
  a.nd = (int32_t)nd;
  a.d_id_base = (int32_t)d_first;
  a.row_bytes = rb;
  a.k = S.k;
  a.exclude_self = exclude_self ? 1 : 0;
  a.ip = S.ip ? 1 : 0;
  if (S.is_float) {
    const int km = exact_km(S.k);
    uint64_t* cand = at<uint64_t>(g->ws, W.off_cand);
    for (int64_t q0 = 0; q0 < nq; q0 += W.cand_rows) {
      const int64_t cnt = nq - q0 < W.cand_rows ? nq - q0 : W.cand_rows;
      ExactArgs c = a;
      c.qvec = rows + (q_first + q0) * rb;
      c.qnorm = norms + q_first + q0;
      c.nq = (int32_t)cnt;
      c.q_id_base = (int32_t)(q_first + q0);
      c.split_len = (int32_t)nd;
      c.nsplit = 1;
      c.cand = cand;
      KNNG_TRY(launch_exact_f32(c, km, stream), "exact launch");
      RerankArgs r{};
      r.rows = at<float>(g->st, S.off_master);
      r.stride = S.mstride;
      r.dim = S.dim;
      r.q_id_base = (int32_t)(q_first + q0);
      r.nq = (int32_t)cnt;
      r.cand = cand;
      r.km = km;
      r.k = S.k;
      r.ip = S.ip ? 1 : 0;
      r.out_ids = out_ids + q0 * out_stride;
      r.out_d = out_d + q0 * out_stride;
      r.out_stride = out_stride;
      KNNG_TRY(launch_rerank_f32(r, stream), "re-rank launch");
    }
    return KNNG_OK;
  }
  a.out_ids = out_ids;
  a.out_d = out_d;
  a.out_stride = out_stride;
  a.partial = at<uint64_t>(g->ws, W.off_partial);
  const int qt = S.k_pad == 64 ? 1 : 2;
  const int64_t bx = (nq + 64 * qt - 1) / (64 * qt);
  // (splits write partial lists into the workspace; a caller whose output
  // lives there passes split_ok = false)
  int64_t nsplit = split_ok ? (1024 + bx - 1) / bx : 1;
  if (nsplit > 64) nsplit = 64;
  while (nsplit > 1 && nsplit * nq > W.partial_lists) --nsplit;
  if (nsplit < 1) nsplit = 1;
  int64_t split_len = round_up((nd + nsplit - 1) / nsplit, 64);
  nsplit = (nd + split_len - 1) / split_len;
  a.split_len = (int32_t)split_len;
  a.nsplit = (int32_t)nsplit;
  KNNG_TRY(launch_exact_u8(a, stream), "exact launch");
  if (nsplit > 1)
    KNNG_TRY(launch_split_merge(a.partial, (int32_t)nq, (int32_t)nsplit, S.k, out_ids, out_d,
                                out_stride, stream),
             "split merge launch");
  return KNNG_OK;
}

// Exact lists of the n stored points.
knng_status exact_lists(knng_graph* g, int64_t n, hipStream_t stream) {
  return exact_lists_range(g, 0, n, 0, n, true, at<int32_t>(g->st, g->S.off_ids),
                           at<int32_t>(g->st, g->S.off_dist), g->S.k_pad, stream);
}

// The naive method of Section 2.1 applied to a batch of b points stored at
// ids n .. n+b-1: each new node's list by brute force over all n + b nodes,
// and each pre-batch node's list merged with its k best among the b new
// nodes (tiles of old nodes against the batch, through a buffer of
// PARTIAL_LISTS rows).  From an exact graph this keeps the graph exact.
knng_status insert_exact_after_ingest(knng_graph* g, int64_t b, hipStream_t stream) {
  const StorageLayout& S = g->S;
  const WorkspaceLayout& W = g->W;
  const int64_t n = g->n;
  int32_t* ids = at<int32_t>(g->st, S.off_ids);
  int32_t* dist = at<int32_t>(g->st, S.off_dist);
  knng_status s = exact_lists_range(g, n, b, 0, n + b, true, ids + n * S.k_pad,
                                    dist + n * S.k_pad, S.k_pad, stream);
  if (s != KNNG_OK) return s;
  int32_t* tmp_ids = at<int32_t>(g->ws, W.off_partial);
  const int64_t chunk = W.partial_lists;
  int32_t* tmp_d = tmp_ids + chunk * S.k_pad;
  for (int64_t q0 = 0; q0 < n; q0 += chunk) {
    const int64_t cnt = n - q0 < chunk ? n - q0 : chunk;
    if ((s = exact_lists_range(g, q0, cnt, n, b, false, tmp_ids, tmp_d, S.k_pad, stream,
                               false)) != KNNG_OK)
      return s;
    Timed t(g, KNNG_STAGE_MERGE, stream);
    KNNG_TRY(launch_merge_lists(ids + q0 * S.k_pad, dist + q0 * S.k_pad, tmp_ids, tmp_d,
                                S.k_pad, S.k, cnt, S.pad, stream),
             "merge launch");
  }
  g->n = n + b;
  return KNNG_OK;
}

// Steps (ii)-(v) of an insert batch whose points are stored at ids
// n .. n+b-1 and whose search results are in the workspace.
knng_status insert_after_search(knng_graph* g, int64_t b, int32_t* sims_dev, int32_t* stats_dev,
                                hipStream_t stream) {
  const StorageLayout& S = g->S;
  const WorkspaceLayout& W = g->W;
  const int64_t n = g->n;
  int32_t* ids = at<int32_t>(g->st, S.off_ids);
  int32_t* dist = at<int32_t>(g->st, S.off_dist);
  int32_t* head = at<int32_t>(g->st, S.off_head);
  int32_t* res_ids = at<int32_t>(g->ws, W.off_res_ids);
  int32_t* res_d = at<int32_t>(g->ws, W.off_res_d);
  int32_t* evals = at<int32_t>(g->ws, W.off_evals);
  int32_t* lreads = at<int32_t>(g->ws, W.off_lreads);
  int32_t* counters = at<int32_t>(g->ws, W.off_counters);
  // rows of the distance evaluations after the search: int8 rows, or the
  // float32 rows of float graphs
  const int eval_format = S.is_float ? ROW_F32 : ROW_I8;
  const char* eval_rows = S.is_float ? at<char>(g->st, S.off_master) : at<char>(g->st, S.off_vec);
  const int eval_bytes = S.is_float ? S.mstride * 4 : S.row_bytes;

  // (ii) lists of the new nodes: search result + batch peers
  PeerArgs pa{};
  pa.format = eval_format;
  pa.bvec = eval_rows + n * eval_bytes;
  pa.row_bytes = eval_bytes;
  pa.dim = S.dim;
  pa.b = (int32_t)b;
  pa.id_base = (int32_t)n;
  pa.k = S.k;
  pa.k_pad = S.k_pad;
  pa.res_ids = res_ids;
  pa.res_d = res_d;
  pa.list_ids = ids + n * S.k_pad;
  pa.list_d = dist + n * S.k_pad;
  pa.pad = S.pad;
  pa.ip = S.ip ? 1 : 0;
  if (b >= PEER_TILE_MIN) {
    // large batches: the k best peers of every new node by the exact
    // graph's brute-force tiles (matrix cores), then merged with its search
    // result; the same distances and (distance, id) order as k_peers
    knng_status s = exact_lists_range(g, n, b, n, b, true, pa.list_ids, pa.list_d, S.k_pad,
                                      stream, true, KNNG_STAGE_PEERS);
    if (s != KNNG_OK) return s;
    Timed t(g, KNNG_STAGE_PEERS, stream);
    KNNG_TRY(launch_merge_lists(pa.list_ids, pa.list_d, res_ids, res_d, S.k_pad, S.k, b, S.pad,
                                stream),
             "merge launch");
  } else {
    Timed t(g, KNNG_STAGE_PEERS, stream);
    KNNG_TRY(launch_peers(pa, stream), "peers launch");
  }
  // (iii) update proposals on the pre-batch lists
  KNNG_TRY(launch_fill_i32(counters, 2, 0, stream), "fill");
  UpdateArgs ua{};
  ua.format = eval_format;
  ua.vec = eval_rows;
  ua.row_bytes = eval_bytes;
  ua.dim = S.dim;
  ua.nbr_ids = ids;
  ua.nbr_d = dist;
  ua.k = S.k;
  ua.k_pad = S.k_pad;
  ua.head = head;
  ua.bvec = eval_rows + n * eval_bytes;
  ua.b = (int32_t)b;
  ua.id_base = (int32_t)n;
  ua.res_ids = res_ids;
  ua.res_d = res_d;
  ua.depth = g->p.depth;
  ua.props = at<Proposal>(g->ws, W.off_props);
  ua.touched = at<int32_t>(g->ws, W.off_touched);
  ua.counters = counters;
  ua.evals = evals;
  ua.list_reads = lreads;
  ua.sims = sims_dev;
  ua.stats = stats_dev;
  ua.n = (int32_t)n;
  ua.ip = S.ip ? 1 : 0;
  ua.front_cap = (int)update_sizes(S.k, g->p.depth).front_cap;
  if (update_fronts_global(ua.front_cap)) ua.gfront = at<int32_t>(g->ws, W.off_fronts);
  if (update_sets_global(n, ua.front_cap)) {
    ua.gset = at<uint32_t>(g->ws, W.off_sets);
    ua.gset_slots = W.set_slots;
  }
  {
    Timed t(g, KNNG_STAGE_UPDATE, stream);
    KNNG_TRY(launch_update(ua, stream), "update launch");
  }
  // (iv) merge proposals into the pre-batch lists
  MergeArgs ma{};
  ma.nbr_ids = ids;
  ma.nbr_d = dist;
  ma.k = S.k;
  ma.k_pad = S.k_pad;
  ma.head = head;
  ma.props = ua.props;
  ma.touched = ua.touched;
  ma.counters = counters;
  ma.max_touched = (int32_t)(b * W.props_per_point);
  ma.pad = S.pad;
  {
    Timed t(g, KNNG_STAGE_MERGE, stream);
    KNNG_TRY(launch_merge(ma, stream), "merge launch");
  }
  // (v)
  g->n = n + b;
  return KNNG_OK;
}


// ---- partitioning (host side) ------------------------------------------------
// Host copy of the restart generator (the same SplitMix64 / LCG the search
// kernel uses): the initial medoids are the first p distinct node ids of
// the keyed permutation with key 2^61.
uint64_t host_splitmix(uint64_t& s) {
  s += 0x9E3779B97F4A7C15ull;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void initial_medoids(int64_t n, int p, uint64_t seed, int32_t* out) {
  const uint32_t m = modulus_for(n);
  uint64_t s0 = (uint64_t)1 << 61;
  const uint64_t hk = host_splitmix(s0);
  uint64_t t = seed ^ hk;
  const uint64_t r0 = host_splitmix(t), r1 = host_splitmix(t), r2 = host_splitmix(t);
  uint32_t a = 1, c = 1;
  if (m > 2) {
    a = (uint32_t)(4ull * (r0 & (uint64_t)(m / 4 - 1)) + 1ull);
    c = (uint32_t)(2ull * (r1 & (uint64_t)(m / 2 - 1)) + 1ull);
  }
  uint32_t x = (uint32_t)(r2 & (uint64_t)(m - 1));
  int got = 0;
  for (uint64_t step = 0; step < m && got < p; ++step) {
    if ((int64_t)x < n) {
      bool dup = false;
      for (int i = 0; i < got; ++i) dup = dup || out[i] == (int32_t)x;
      if (!dup) out[got++] = (int32_t)x;
    }
    x = (uint32_t)(((uint64_t)a * x + c) & (uint64_t)(m - 1));
  }
}

// Shortest-path scratch slots of the medoid update (one wavefront each).
constexpr int64_t PATH_SLOTS = 256;

struct PartScratch {
  size_t off_D = 0, off_members = 0, off_offsets = 0, off_sums = 0, off_unreached = 0,
         off_pos = 0, off_in_off = 0, off_in_src = 0, off_in_w = 0, off_counts = 0,
         off_sp_dist = 0, off_sp_cur = 0, off_sp_next = 0, off_sp_inq = 0, total = 0;
  int64_t slots = 0, slot_len = 0;
};

PartScratch part_scratch(int64_t n, int p, int k) {
  PartScratch P;
  size_t cur = 0;
  P.off_D = take(cur, (size_t)n * p * 4);
  P.off_members = take(cur, (size_t)n * 4);
  P.off_offsets = take(cur, 65 * 4);
  P.off_sums = take(cur, (size_t)n * 8);
  P.off_unreached = take(cur, (size_t)n * 4);
  P.off_pos = take(cur, (size_t)n * 4);
  P.off_in_off = take(cur, (size_t)(n + 1) * 4);
  P.off_in_src = take(cur, (size_t)n * k * 4);
  P.off_in_w = take(cur, (size_t)n * k * 4);
  P.off_counts = take(cur, (size_t)n * 4);
  // a partition holds at most n nodes
  P.slots = n < PATH_SLOTS ? n : PATH_SLOTS;
  P.slot_len = n;
  P.off_sp_dist = take(cur, (size_t)P.slots * P.slot_len * 8);
  P.off_sp_cur = take(cur, (size_t)P.slots * P.slot_len * 4);
  P.off_sp_next = take(cur, (size_t)P.slots * P.slot_len * 4);
  P.off_sp_inq = take(cur, (size_t)P.slots * P.slot_len * 4);
  P.total = cur;
  return P;
}

struct SearchPartScratch {
  size_t off_ids = 0, off_d = 0, off_evals = 0, off_counts = 0, off_budgets = 0, total = 0;
};

SearchPartScratch search_part_scratch(int64_t m, int p, int k_pad) {
  SearchPartScratch P;
  size_t cur = 0;
  P.off_ids = take(cur, (size_t)m * p * k_pad * 4);
  P.off_d = take(cur, (size_t)m * p * k_pad * 4);
  P.off_evals = take(cur, (size_t)m * p * 4);
  P.off_counts = take(cur, 64 * 4);
  P.off_budgets = take(cur, 64 * 4);
  P.total = cur;
  return P;
}

// Argument checks shared by the partitioned searches (m == 0 is a no-op).
knng_status check_partitioned(knng_graph* g, const void* q_dev, int64_t m,
                              const uint64_t* keys_dev, const int32_t* part_dev, int32_t p,
                              int32_t* ids_dev, void* d_dev) {
  if (!g) return fail(KNNG_EINVAL, "graph is NULL");
  if (m == 0) return ok();
  if (m < 0 || m * (int64_t)p >= ((int64_t)1 << 31))
    return fail(KNNG_EINVAL, "m * p must be below 2^31");
  if (p < 1 || p > 64) return fail(KNNG_EINVAL, "p must be 1 .. 64");
  if (g->S.is_float && g->S.format != ROW_F32)
    return fail(KNNG_EINVAL, "partitioned search is built for uint8 graphs and float graphs "
                             "with float32 scoring");
  if (g->S.cosine || g->S.ip)
    return fail(KNNG_EINVAL, "partitioned search takes the squared L2 distance only");
  knng_status s;
  if ((s = check_ptr(q_dev, "q_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(keys_dev, "keys_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(part_dev, "part_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(ids_dev, "ids_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(d_dev, "d_dev")) != KNNG_OK) return s;
  return KNNG_OK;
}

// The partitioned search proper, with its per-call scratch at `sc` (sized
// by search_part_scratch; every byte of it is written before it is read, so
// it needs no clearing).
knng_status search_partitioned(knng_graph* g, const void* q_dev, int64_t m,
                               const uint64_t* keys_dev, const int32_t* part_dev, int32_t p,
                               char* sc, int32_t* ids_dev, void* d_dev, int32_t* evals_dev,
                               hipStream_t stream) {
  const SearchPartScratch P = search_part_scratch(m, p, g->S.k_pad);
  const StorageLayout& S = g->S;
  const WorkspaceLayout& W = g->W;
  int32_t* rid = reinterpret_cast<int32_t*>(sc + P.off_ids);
  int32_t* rd = reinterpret_cast<int32_t*>(sc + P.off_d);
  int32_t* rev = reinterpret_cast<int32_t*>(sc + P.off_evals);
  int32_t* counts = reinterpret_cast<int32_t*>(sc + P.off_counts);
  int32_t* budgets = reinterpret_cast<int32_t*>(sc + P.off_budgets);
  KNNG_TRY(launch_part_budgets(part_dev, (int32_t)g->n, p, S.k, g->p.speedup, counts, budgets,
                               stream),
           "budget launch");
  SearchArgs a{};
  a.format = S.format;
  a.vec = at<char>(g->st, S.off_vec);
  a.row_bytes = S.row_bytes;
  a.coord_bytes = S.coord_bytes;
  a.side2_off = S.norm_off;
  a.nbr_ids = at<int32_t>(g->st, S.off_ids);
  a.k = S.k;
  a.k_pad = S.k_pad;
  a.keep = S.k;
  a.n = (int32_t)g->n;
  a.B = (int32_t)budget(g->n, S.k, g->p.speedup);
  a.m_mod = modulus_for(g->n);
  a.e_num = g->p.expansion_num;
  a.e_den = g->p.expansion_den;
  a.seed = g->p.seed;
  a.dim = S.dim;
  a.rows[0] = query_rows(q_dev, m * p, keys_dev, 0, rid, rd, S.k_pad, rev, nullptr, nullptr, 0);
  a.pad_bits = (uint32_t)S.pad;
  if (search_sets_global(g->n)) {
    a.gvis = at<uint32_t>(g->ws, W.off_sets);
    a.gvis_slots = W.set_slots;
  }
  if (S.is_float) {
    a.master = at<float>(g->st, S.off_master);
    a.master_stride = S.mstride;
    a.master_chunks = S.mstride / 4;
  }
  a.node_part = part_dev;
  a.nparts = p;
  a.part_budget = budgets;
  {
    Timed t(g, KNNG_STAGE_QUERY, stream);
    KNNG_TRY(launch_search_part(a, stream), "search launch");
    KNNG_TRY(launch_merge_partitions(rid, rd, rev, S.k_pad, (int32_t)m, p, S.k, ids_dev,
                                     (int32_t*)d_dev, S.k, evals_dev, S.pad, stream),
             "merge launch");
  }
  return ok();
}

// ---- static scratch of knng_search_partitioned_noalloc ------------------------------
// One array per GPU, alive until the process ends.  In host code the name
// `scratch` only stands for the symbol; its device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
char* g_scratch_ptr[MAX_DEVICES] = {};

knng_status noalloc_scratch(char** out) {
  int dev_id = -1;
  KNNG_TRY(hipGetDevice(&dev_id), "hipGetDevice");
  if (dev_id < 0 || dev_id >= MAX_DEVICES)
    return fail(KNNG_EDEVICE, "device %d outside 0 .. %d", dev_id, MAX_DEVICES - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev_id]) {
    void* ptr = nullptr;
    KNNG_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(KNNG_EDEVICE, "no device address for the static scratch");
    g_scratch_ptr[dev_id] = (char*)ptr;
  }
  *out = g_scratch_ptr[dev_id];
  return KNNG_OK;
}

}  // namespace

extern "C" {

size_t knng_storage_bytes(const knng_params* p) {
  if (check_params(p) != KNNG_OK) return 0;
  return storage_layout(*p).total;
}

size_t knng_workspace_bytes(const knng_params* p) {
  if (check_params(p) != KNNG_OK) return 0;
  return workspace_layout(*p, storage_layout(*p)).total;
}

knng_status knng_build_exact(const knng_params* p, const void* x_dev, int64_t n,
                             void* storage_dev, size_t storage_bytes, void* workspace_dev,
                             size_t workspace_bytes, hipStream_t stream, knng_graph** out) {
  if (out) *out = nullptr;
  knng_status s = check_params(p);
  if (s != KNNG_OK) return s;
  if ((s = check_ptr(x_dev, "x_dev")) != KNNG_OK) return s;
  if (n < 2) return fail(KNNG_EINVAL, "n must be >= 2 (got %lld)", (long long)n);
  if (n > p->capacity)
    return fail(KNNG_ECAPACITY, "n %lld exceeds capacity %lld", (long long)n,
                (long long)p->capacity);
  knng_graph* g = nullptr;
  s = make_handle(p, storage_dev, storage_bytes, workspace_dev, workspace_bytes, &g);
  if (s != KNNG_OK) return s;
  const StorageLayout& S = g->S;
  auto cleanup = [&](knng_status st) {
    delete g;
    return st;
  };
  if ((s = ingest(g, x_dev, n, 0, stream)) != KNNG_OK) return cleanup(s);
  if ((s = dev(launch_fill_i32(at<int32_t>(g->st, S.off_head), S.cap, -1, stream), "fill")) !=
      KNNG_OK)
    return cleanup(s);
  if ((s = exact_lists(g, n, stream)) != KNNG_OK) return cleanup(s);
  g->n = n;
  *out = g;
  return ok();
}

knng_status knng_load(const knng_params* p, const void* x_dev, int64_t n, const int32_t* ids_dev,
                      const void* d_dev, void* storage_dev, size_t storage_bytes,
                      void* workspace_dev, size_t workspace_bytes, hipStream_t stream,
                      knng_graph** out) {
  if (out) *out = nullptr;
  knng_status s = check_params(p);
  if (s != KNNG_OK) return s;
  if ((s = check_ptr(x_dev, "x_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(ids_dev, "ids_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(d_dev, "d_dev")) != KNNG_OK) return s;
  if (n < 2) return fail(KNNG_EINVAL, "n must be >= 2 (got %lld)", (long long)n);
  if (n > p->capacity)
    return fail(KNNG_ECAPACITY, "n %lld exceeds capacity %lld", (long long)n,
                (long long)p->capacity);
  knng_graph* g = nullptr;
  s = make_handle(p, storage_dev, storage_bytes, workspace_dev, workspace_bytes, &g);
  if (s != KNNG_OK) return s;
  const StorageLayout& S = g->S;
  auto cleanup = [&](knng_status st) {
    delete g;
    return st;
  };
  if ((s = ingest(g, x_dev, n, 0, stream)) != KNNG_OK) return cleanup(s);
  if ((s = dev(launch_fill_i32(at<int32_t>(g->st, S.off_head), S.cap, -1, stream), "fill")) !=
      KNNG_OK)
    return cleanup(s);
  if ((s = dev(launch_copy_lists(ids_dev, (const int32_t*)d_dev, S.k,
                                 at<int32_t>(g->st, S.off_ids), at<int32_t>(g->st, S.off_dist),
                                 S.k_pad, n, S.k, n, S.pad, stream, S.ip ? 1 : 0),
               "copy lists")) != KNNG_OK)
    return cleanup(s);
  g->n = n;
  *out = g;
  return ok();
}

knng_status knng_search(knng_graph* g, const void* q_dev, int64_t m, const uint64_t* keys_dev,
                        int32_t* ids_dev, void* d_dev, int32_t* evals_dev,
                        int32_t* list_reads_dev, int32_t* trace_dev, int64_t trace_stride,
                        hipStream_t stream) {
  if (!g) return fail(KNNG_EINVAL, "graph is NULL");
  knng_status s;
  if (m == 0) return ok();
  if (m < 0 || m >= ((int64_t)1 << 31)) return fail(KNNG_EINVAL, "m must be in 0 .. 2^31-1");
  if ((s = check_ptr(q_dev, "q_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(keys_dev, "keys_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(ids_dev, "ids_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(d_dev, "d_dev")) != KNNG_OK) return s;
  if (trace_dev && trace_stride < budget(g->n, g->S.k, g->p.speedup))
    return fail(KNNG_EINVAL, "trace_stride %lld is below the budget %lld",
                (long long)trace_stride, (long long)budget(g->n, g->S.k, g->p.speedup));
  s = run_search(g, query_rows(q_dev, m, keys_dev, 0, ids_dev, d_dev, g->S.k, evals_dev,
                                list_reads_dev, trace_dev, trace_stride, g->S.ip),
                 nullptr, KNNG_STAGE_QUERY, stream);
  if (s != KNNG_OK) return s;
  return ok();
}

knng_status knng_search_gnns(knng_graph* g, const void* q_dev, int64_t m,
                             const uint64_t* keys_dev, int32_t restarts, int32_t* ids_dev,
                             void* d_dev, int32_t* evals_dev, int32_t* trace_dev,
                             int64_t trace_stride, hipStream_t stream) {
  if (!g) return fail(KNNG_EINVAL, "graph is NULL");
  knng_status s;
  if (m == 0) return ok();
  if (m < 0 || m >= ((int64_t)1 << 31)) return fail(KNNG_EINVAL, "m must be in 0 .. 2^31-1");
  if (restarts < 0) return fail(KNNG_EINVAL, "restarts must be >= 0");
  if (g->S.is_float && g->S.format != ROW_F32)
    return fail(KNNG_EINVAL, "the GNNS baseline is built for uint8 graphs and float graphs "
                             "with float32 scoring");
  if (g->S.ip) return fail(KNNG_EINVAL, "the GNNS baseline takes the squared L2 distance only");
  if ((s = check_ptr(q_dev, "q_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(keys_dev, "keys_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(ids_dev, "ids_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(d_dev, "d_dev")) != KNNG_OK) return s;
  if (trace_dev && trace_stride < budget(g->n, g->S.k, g->p.speedup))
    return fail(KNNG_EINVAL, "trace_stride %lld is below the budget %lld",
                (long long)trace_stride, (long long)budget(g->n, g->S.k, g->p.speedup));
  s = run_search(g, query_rows(q_dev, m, keys_dev, 0, ids_dev, d_dev, g->S.k, evals_dev,
                                nullptr, trace_dev, trace_stride),
                 nullptr, KNNG_STAGE_QUERY, stream, restarts);
  if (s != KNNG_OK) return s;
  return ok();
}

knng_status knng_query(knng_graph* g, const void* q_dev, int64_t m, int32_t* ids_dev,
                       void* d_dev, int32_t* evals_dev, int32_t* list_reads_dev,
                       hipStream_t stream) {
  if (!g) return fail(KNNG_EINVAL, "graph is NULL");
  knng_status s;
  if (m == 0) return ok();
  if (m < 0 || m >= ((int64_t)1 << 31)) return fail(KNNG_EINVAL, "m must be in 0 .. 2^31-1");
  if ((s = check_ptr(q_dev, "q_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(ids_dev, "ids_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(d_dev, "d_dev")) != KNNG_OK) return s;
  s = run_search(g, query_rows(q_dev, m, nullptr, (uint64_t)QUERY_KEY_BASE + (uint64_t)g->qcount,
                                ids_dev, d_dev, g->S.k, evals_dev, list_reads_dev, nullptr, 0,
                                g->S.ip),
                 nullptr, KNNG_STAGE_QUERY, stream);
  if (s != KNNG_OK) return s;
  g->qcount += m;
  return ok();
}

knng_status knng_insert_batch(knng_graph* g, const void* x_dev, int64_t b,
                              int64_t* first_id_host, int32_t* sims_dev, int32_t* stats_dev,
                              hipStream_t stream) {
  if (!g) return fail(KNNG_EINVAL, "graph is NULL");
  knng_status s;
  if (b == 0) {
    if (first_id_host) *first_id_host = g->n;
    return ok();
  }
  if (b < 0) return fail(KNNG_EINVAL, "b must be >= 0");
  if ((s = check_ptr(x_dev, "x_dev")) != KNNG_OK) return s;
  if (b > g->W.M)
    return fail(KNNG_ECAPACITY, "batch %lld exceeds max_batch %lld", (long long)b,
                (long long)g->W.M);
  if (g->n + b > g->S.cap)
    return fail(KNNG_ECAPACITY, "n %lld + batch %lld exceeds capacity %lld", (long long)g->n,
                (long long)b, (long long)g->S.cap);
  knng_status st = ingest(g, x_dev, b, g->n, stream);
  if (st != KNNG_OK) return st;
  // (i) iGNNS of every new point on the pre-batch graph, key = its id
  if ((st = run_search(g, insert_rows(g, x_dev, b), nullptr, KNNG_STAGE_SEARCH, stream)) !=
      KNNG_OK)
    return st;
  const int64_t n = g->n;
  if ((st = insert_after_search(g, b, sims_dev, stats_dev, stream)) != KNNG_OK) return st;
  if (first_id_host) *first_id_host = n;
  return ok();
}

knng_status knng_insert_exact(knng_graph* g, const void* x_dev, int64_t b,
                              int64_t* first_id_host, hipStream_t stream) {
  if (!g) return fail(KNNG_EINVAL, "graph is NULL");
  knng_status s;
  if (b == 0) {
    if (first_id_host) *first_id_host = g->n;
    return ok();
  }
  if (b < 0) return fail(KNNG_EINVAL, "b must be >= 0");
  if ((s = check_ptr(x_dev, "x_dev")) != KNNG_OK) return s;
  if (b > g->W.M)
    return fail(KNNG_ECAPACITY, "batch %lld exceeds max_batch %lld", (long long)b,
                (long long)g->W.M);
  if (g->n + b > g->S.cap)
    return fail(KNNG_ECAPACITY, "n %lld + batch %lld exceeds capacity %lld", (long long)g->n,
                (long long)b, (long long)g->S.cap);
  const int64_t n = g->n;
  if ((s = ingest(g, x_dev, b, n, stream)) != KNNG_OK) return s;
  if ((s = insert_exact_after_ingest(g, b, stream)) != KNNG_OK) return s;
  if (first_id_host) *first_id_host = n;
  return ok();
}

knng_status knng_epoch(knng_graph* g, const void* x_dev, int64_t b, const void* q_dev,
                       int64_t m, int32_t* q_ids_dev, void* q_d_dev, int32_t* q_evals_dev,
                       int32_t* q_list_reads_dev, int64_t* first_id_host, int32_t* sims_dev,
                       int32_t* stats_dev, hipStream_t stream) {
  if (!g) return fail(KNNG_EINVAL, "graph is NULL");
  knng_status s;
  if (b < 0 || m < 0 || m >= ((int64_t)1 << 31))
    return fail(KNNG_EINVAL, "b must be >= 0 and m in 0 .. 2^31-1");
  if (b > 0 && (s = check_ptr(x_dev, "x_dev")) != KNNG_OK) return s;
  if (m > 0) {
    if ((s = check_ptr(q_dev, "q_dev")) != KNNG_OK) return s;
    if ((s = check_ptr(q_ids_dev, "q_ids_dev")) != KNNG_OK) return s;
    if ((s = check_ptr(q_d_dev, "q_d_dev")) != KNNG_OK) return s;
  }
  if (b > g->W.M)
    return fail(KNNG_ECAPACITY, "batch %lld exceeds max_batch %lld", (long long)b,
                (long long)g->W.M);
  if (g->n + b > g->S.cap)
    return fail(KNNG_ECAPACITY, "n %lld + batch %lld exceeds capacity %lld", (long long)g->n,
                (long long)b, (long long)g->S.cap);
  const int64_t n = g->n;
  if (first_id_host) *first_id_host = n;
  if (b == 0 && m == 0) return ok();
  if (b > 0 && (s = ingest(g, x_dev, b, n, stream)) != KNNG_OK) return s;
  // one search launch: the batch's points (keys = ids) and the queries
  // (keys 2^62 + query count), both on the snapshot of n nodes
  SearchRows qr = query_rows(q_dev, m, nullptr, (uint64_t)QUERY_KEY_BASE + (uint64_t)g->qcount,
                             q_ids_dev, q_d_dev, g->S.k, q_evals_dev, q_list_reads_dev,
                             nullptr, 0, g->S.ip);
  SearchRows ir = insert_rows(g, x_dev, b);
  if ((s = run_search(g, ir, &qr, KNNG_STAGE_SEARCH, stream)) != KNNG_OK) return s;
  g->qcount += m;
  if (b > 0 && (s = insert_after_search(g, b, sims_dev, stats_dev, stream)) != KNNG_OK) return s;
  return ok();
}

knng_status knng_get_lists(const knng_graph* g, int64_t first, int64_t count, int32_t* ids_dev,
                           void* d_dev, hipStream_t stream) {
  if (!g) return fail(KNNG_EINVAL, "graph is NULL");
  if (first < 0 || count < 0 || first + count > g->n)
    return fail(KNNG_EINVAL, "rows [%lld, %lld) outside the graph of %lld nodes",
                (long long)first, (long long)(first + count), (long long)g->n);
  if (count == 0) return ok();
  const StorageLayout& S = g->S;
  KNNG_TRY(launch_copy_lists(at<int32_t>(g->st, S.off_ids) + first * S.k_pad,
                             at<int32_t>(g->st, S.off_dist) + first * S.k_pad, S.k_pad, ids_dev,
                             (int32_t*)d_dev, S.k, count, S.k, g->n, S.pad, stream,
                             S.ip ? 2 : 0),
           "copy lists");
  return ok();
}

knng_status knng_get_points(const knng_graph* g, int64_t first, int64_t count, void* x_dev,
                            hipStream_t stream) {
  if (!g) return fail(KNNG_EINVAL, "graph is NULL");
  if (!x_dev) return fail(KNNG_EINVAL, "x_dev is NULL");
  if (first < 0 || count < 0 || first + count > g->n)
    return fail(KNNG_EINVAL, "rows outside the graph");
  if (count == 0) return ok();
  const StorageLayout& S = g->S;
  if (S.is_float)
    KNNG_TRY(launch_export_f32(at<float>(g->st, S.off_master) + first * S.mstride, S.mstride,
                               S.dim, count, (float*)x_dev, stream),
             "export points");
  else
    KNNG_TRY(launch_export_u8(at<int8_t>(g->st, S.off_vec) + first * S.row_bytes, S.row_bytes,
                              S.dim, count, (uint8_t*)x_dev, stream),
             "export points");
  return ok();
}

int32_t knng_row_bytes(const knng_graph* g) { return g ? g->S.row_bytes : -1; }

knng_status knng_get_rows(const knng_graph* g, int64_t first, int64_t count, void* rows_dev,
                          float* scale_dev, hipStream_t stream) {
  if (!g) return fail(KNNG_EINVAL, "graph is NULL");
  if (first < 0 || count < 0 || first + count > g->n)
    return fail(KNNG_EINVAL, "rows outside the graph");
  if (count == 0) return ok();
  const StorageLayout& S = g->S;
  if (rows_dev)
    KNNG_TRY(hipMemcpyAsync(rows_dev, at<char>(g->st, S.off_vec) + first * S.row_bytes,
                            (size_t)count * S.row_bytes, hipMemcpyDeviceToDevice, stream),
             "copy rows");
  if (scale_dev && S.format == ROW_FP8)
    KNNG_TRY(hipMemcpyAsync(scale_dev, at<float>(g->st, S.off_scale) + first,
                            (size_t)count * 4, hipMemcpyDeviceToDevice, stream),
             "copy scales");
  return ok();
}


size_t knng_partition_scratch_bytes(const knng_graph* g, int32_t p) {
  if (!g || p < 1 || p > 64) return 0;
  return part_scratch(g->n, p, g->S.k).total;
}

knng_status knng_partition(knng_graph* g, int32_t p, int32_t iters, int32_t imb_num,
                           int32_t imb_den, uint64_t seed, void* scratch_dev,
                           size_t scratch_bytes, int32_t* part_dev, int32_t* medoids_dev,
                           hipStream_t stream) {
  if (!g) return fail(KNNG_EINVAL, "graph is NULL");
  if (p < 1 || p > 64) return fail(KNNG_EINVAL, "p must be 1 .. 64");
  if (p > g->n) return fail(KNNG_EINVAL, "p exceeds the number of nodes");
  if (iters < 1) return fail(KNNG_EINVAL, "iters must be >= 1");
  if (g->S.ip)
    return fail(KNNG_EINVAL, "partitioning needs distances >= 0 (not the inner-product metric)");
  if (imb_den < 1 || imb_num < imb_den || imb_num > 64 * imb_den)
    return fail(KNNG_EINVAL, "imbalance num/den must be in [1, 64] with den >= 1");
  knng_status s;
  if ((s = check_ptr(scratch_dev, "scratch_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(part_dev, "part_dev")) != KNNG_OK) return s;
  if ((s = check_ptr(medoids_dev, "medoids_dev")) != KNNG_OK) return s;
  if ((uintptr_t)scratch_dev % ALIGN) return fail(KNNG_EINVAL, "scratch must be 256-byte aligned");
  const PartScratch P = part_scratch(g->n, p, g->S.k);
  if (scratch_bytes < P.total)
    return fail(KNNG_ENOMEM, "scratch has %zu bytes, needs %zu", scratch_bytes, P.total);
  const StorageLayout& S = g->S;
  char* sc = (char*)scratch_dev;
  PartitionArgs a{};
  a.format = S.is_float ? ROW_F32 : ROW_I8;
  a.vec = S.is_float ? (const void*)at<char>(g->st, S.off_master)
                     : (const void*)at<char>(g->st, S.off_vec);
  a.row_bytes = S.is_float ? S.mstride * 4 : S.row_bytes;
  a.dim = S.dim;
  a.n = (int32_t)g->n;
  a.p = p;
  a.N = g->n * (int64_t)imb_num;
  a.P = (int64_t)p * imb_den;
  a.medoids = medoids_dev;
  a.D = reinterpret_cast<uint32_t*>(sc + P.off_D);
  a.part = part_dev;
  a.members = reinterpret_cast<int32_t*>(sc + P.off_members);
  a.offsets = reinterpret_cast<int32_t*>(sc + P.off_offsets);
  a.sums = reinterpret_cast<double*>(sc + P.off_sums);
  a.unreached = reinterpret_cast<int32_t*>(sc + P.off_unreached);
  a.is_float = S.is_float ? 1 : 0;
  a.nbr_ids = at<int32_t>(g->st, S.off_ids);
  a.nbr_d = at<int32_t>(g->st, S.off_dist);
  a.k = S.k;
  a.k_pad = S.k_pad;
  a.pos = reinterpret_cast<int32_t*>(sc + P.off_pos);
  a.in_off = reinterpret_cast<int32_t*>(sc + P.off_in_off);
  a.in_src = reinterpret_cast<int32_t*>(sc + P.off_in_src);
  a.in_w = reinterpret_cast<int32_t*>(sc + P.off_in_w);
  a.sp_dist = reinterpret_cast<uint64_t*>(sc + P.off_sp_dist);
  a.sp_cur = reinterpret_cast<int32_t*>(sc + P.off_sp_cur);
  a.sp_next = reinterpret_cast<int32_t*>(sc + P.off_sp_next);
  a.sp_inq = reinterpret_cast<int32_t*>(sc + P.off_sp_inq);
  a.slots = (int32_t)P.slots;
  a.slot_len = P.slot_len;
  int32_t init[64];
  initial_medoids(g->n, p, seed, init);
  KNNG_TRY(launch_set_medoids(medoids_dev, init, p, stream), "medoids launch");
  KNNG_TRY(launch_in_edges(a, reinterpret_cast<int32_t*>(sc + P.off_counts), stream),
           "in-edges launch");
  for (int it = 0; it < iters; ++it)
    KNNG_TRY(launch_partition_iteration(a, stream), "partition launch");
  return ok();
}

size_t knng_search_partitioned_scratch_bytes(const knng_graph* g, int64_t m, int32_t p) {
  if (!g || m < 0 || p < 1 || p > 64) return 0;
  return search_part_scratch(m, p, g->S.k_pad).total;
}

knng_status knng_search_partitioned(knng_graph* g, const void* q_dev, int64_t m,
                                    const uint64_t* keys_dev, const int32_t* part_dev, int32_t p,
                                    void* scratch_dev, size_t scratch_bytes, int32_t* ids_dev,
                                    void* d_dev, int32_t* evals_dev, hipStream_t stream) {
  knng_status s = check_partitioned(g, q_dev, m, keys_dev, part_dev, p, ids_dev, d_dev);
  if (s != KNNG_OK || m == 0) return s;
  if ((s = check_ptr(scratch_dev, "scratch_dev")) != KNNG_OK) return s;
  if ((uintptr_t)scratch_dev % ALIGN) return fail(KNNG_EINVAL, "scratch must be 256-byte aligned");
  const size_t need = search_part_scratch(m, p, g->S.k_pad).total;
  if (scratch_bytes < need)
    return fail(KNNG_ENOMEM, "scratch has %zu bytes, needs %zu", scratch_bytes, need);
  return search_partitioned(g, q_dev, m, keys_dev, part_dev, p, (char*)scratch_dev, ids_dev,
                            d_dev, evals_dev, stream);
}

knng_status knng_search_partitioned_noalloc(knng_graph* g, const void* q_dev, int64_t m,
                                            const uint64_t* keys_dev, const int32_t* part_dev,
                                            int32_t p, int32_t* ids_dev, void* d_dev,
                                            int32_t* evals_dev, hipStream_t stream) {
  knng_status s = check_partitioned(g, q_dev, m, keys_dev, part_dev, p, ids_dev, d_dev);
  if (s != KNNG_OK || m == 0) return s;
  const size_t need = search_part_scratch(m, p, g->S.k_pad).total;
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(KNNG_ECAPACITY, "m = %lld queries in %d parts need %zu bytes of scratch; the "
                                "static scratch holds %zu (use knng_search_partitioned)",
                (long long)m, p, need, NOALLOC_SCRATCH_BYTES);
  char* sc = nullptr;
  if ((s = noalloc_scratch(&sc)) != KNNG_OK) return s;
  return search_partitioned(g, q_dev, m, keys_dev, part_dev, p, sc, ids_dev, d_dev, evals_dev,
                            stream);
}

knng_status knng_timing_enable(knng_graph* g, int enable) {
  if (!g) return fail(KNNG_EINVAL, "graph is NULL");
  StageTimer& T = g->timer;
  for (int st = 0; st < KNNG_NUM_STAGES; ++st) {
    for (auto& pr : T.pending[st]) {
      hipEventSynchronize(pr.second);
      T.pool.push_back(pr.first);
      T.pool.push_back(pr.second);
    }
    T.pending[st].clear();
    T.ms[st] = 0.0;
    T.launches[st] = 0;
  }
  T.on = enable != 0;
  return ok();
}

knng_status knng_timing_read(knng_graph* g, double* ms_host, int64_t* launches_host) {
  if (!g) return fail(KNNG_EINVAL, "graph is NULL");
  StageTimer& T = g->timer;
  for (int st = 0; st < KNNG_NUM_STAGES; ++st) {
    for (auto& pr : T.pending[st]) {
      KNNG_TRY(hipEventSynchronize(pr.second), "event synchronize");
      float ms = 0.f;
      KNNG_TRY(hipEventElapsedTime(&ms, pr.first, pr.second), "event elapsed time");
      T.ms[st] += ms;
      T.launches[st] += 1;
      T.pool.push_back(pr.first);
      T.pool.push_back(pr.second);
    }
    T.pending[st].clear();
    if (ms_host) ms_host[st] = T.ms[st];
    if (launches_host) launches_host[st] = T.launches[st];
  }
  return ok();
}

int64_t knng_size(const knng_graph* g) { return g ? g->n : -1; }

int64_t knng_budget(const knng_graph* g, int64_t n) {
  if (!g) return -1;
  return budget(n < 0 ? g->n : n, g->S.k, g->p.speedup);
}

int64_t knng_query_count(const knng_graph* g) { return g ? g->qcount : -1; }

const char* knng_last_error(void) { return g_err.c_str(); }

knng_status knng_step_counters(knng_graph* g, uint64_t* counters_host, int reset) {
  if (!g) return fail(KNNG_EINVAL, "graph is NULL");
#ifdef KNNG_STEP_COUNTERS
  if (!counters_host) return fail(KNNG_EINVAL, "counters_host is NULL");
  KNNG_TRY(hipDeviceSynchronize(), "synchronize");
  if (!g->counters) {
    for (int i = 0; i < KNNG_NUM_STEP_COUNTERS; ++i) counters_host[i] = 0;
    return ok();
  }
  KNNG_TRY(hipMemcpy(counters_host, g->counters, KNNG_NUM_STEP_COUNTERS * 8,
                     hipMemcpyDeviceToHost), "copy counters");
  if (reset) KNNG_TRY(hipMemset(g->counters, 0, KNNG_NUM_STEP_COUNTERS * 8), "clear counters");
  return ok();
#else
  (void)counters_host;
  (void)reset;
  return fail(KNNG_EUNSUPPORTED, "step counters need the profiling build (KNNG_STEP_COUNTERS)");
#endif
}

void knng_destroy(knng_graph* g) { delete g; }

}  // extern "C"
