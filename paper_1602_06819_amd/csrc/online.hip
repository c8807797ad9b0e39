// Online insertion kernels after the search (iGNNS is in search.h):
//
//   k_peers    list of each new node = k best of its search result and the
//              other points of the batch
//   k_update   Update (Algorithm 2) on the pre-batch lists: proposals
//              (node, distance, new id), bucketed per target node
//   k_merge    each target's list = k best of its list and proposals
//
// Distances come from an evaluation policy: EvalI8 (int8 rows, exact int32
// squared distance) or EvalF32 (the float32 distance of stored float
// distances, over the float32 rows).  Both return 32-bit patterns that
// order like the distances, so the list code is shared.
#include "common.h"
#include "device.h"
#include "internal.h"

namespace knng {

// ---- query rows ------------------------------------------------------------
// Lane `sub` of a group of G lanes holds the 16-byte chunks sub, sub + G, ...
// of the query as int8 (coordinate - 128), and every lane ends with |q|^2.
template <int G, int CPL>
__device__ __forceinline__ int32_t load_query_rows(const int8_t* q, int row_bytes,
                                                   v4i (&qc)[CPL]) {
  const int sub = lane_id() % G;
  int nrm = 0;
#pragma unroll
  for (int pp = 0; pp < CPL; ++pp) {
    int off = 16 * (sub + G * pp);
    qc[pp] = off < row_bytes ? *reinterpret_cast<const v4i*>(q + off) : v4i{0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 4; ++e) nrm = __builtin_amdgcn_sdot4(qc[pp][e], qc[pp][e], nrm, false);
  }
  return group_sum<G>(nrm);
}

// ---- distances of up to 64 candidates --------------------------------------
// Lane j holds candidate row index `idx` and a flag `load` (the row exists);
// groups of G lanes each take one candidate per pass.  Returns in lane j
// (j < cnt, load set) the exact squared distance |q|^2 + |x|^2 - 2 q.x
// (v_dot4 on int8 lanes).  All loads are issued before any arithmetic.
template <int G, int CPL>
__device__ __forceinline__ int32_t eval_rows(const int8_t* base, int row_bytes, int32_t idx,
                                             bool load, int cnt, const v4i (&qc)[CPL],
                                             int32_t qn) {
  constexpr int SLOTS = WAVE / G;
  const int lane = lane_id();
  const int slot = lane / G;
  const int sub = lane % G;
  const int passes = (cnt + SLOTS - 1) / SLOTS;
  const int32_t tagged = load ? idx : -1;        // row index, -1 when absent
  // the candidate of this lane's group in every pass (all lanes take part
  // in every cross-lane read; the reads are independent)
  int32_t cid[G];
#pragma unroll
  for (int p = 0; p < G; ++p) {
    const int c = p * SLOTS + slot;
    const int32_t v = G == 1 ? tagged : shfl_i32(tagged, c & 63);
    cid[p] = (p < passes && c < cnt) ? v : -1;
  }
  v4i xv[G][CPL];
#pragma unroll
  for (int p = 0; p < G; ++p) {
    const bool ok = cid[p] >= 0;
#pragma unroll
    for (int pp = 0; pp < CPL; ++pp) {
      const int off = 16 * (sub + G * pp);
      if (ok && off < row_bytes)
        xv[p][pp] = *reinterpret_cast<const v4i*>(base + (int64_t)cid[p] * row_bytes + off);
      else
        xv[p][pp] = v4i{0, 0, 0, 0};
    }
  }
  int32_t dg[G];
#pragma unroll
  for (int p = 0; p < G; ++p) {
    int xx = 0, qx = 0;
#pragma unroll
    for (int pp = 0; pp < CPL; ++pp) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        xx = __builtin_amdgcn_sdot4(xv[p][pp][e], xv[p][pp][e], xx, false);
        qx = __builtin_amdgcn_sdot4(qc[pp][e], xv[p][pp][e], qx, false);
      }
    }
    xx = group_sum<G>(xx);
    qx = group_sum<G>(qx);
    dg[p] = cid[p] >= 0 ? qn + xx - 2 * qx : DIST_PAD_I32;
  }
  if (G == 1) return dg[0];
  // candidate c's distance to lane c
  int32_t result = DIST_PAD_I32;
#pragma unroll
  for (int p = 0; p < G; ++p) {
    const int j = lane - p * SLOTS;
    const bool mine = j >= 0 && j < SLOTS;
    const int32_t got = shfl_i32(dg[p], mine ? j * G : 0);
    if (mine) result = got;
  }
  return result;
}

// ---- evaluation policies -------------------------------------------------------
template <int G, int CPL>
struct EvalI8 {
  v4i qc[CPL];
  int32_t qn;
  // query = row `i` of `rows`
  __device__ void load(const void* rows, int row_bytes, int dim, int64_t i) {
    qn = load_query_rows<G, CPL>((const int8_t*)rows + i * row_bytes, row_bytes, qc);
  }
  __device__ uint32_t dist(const void* rows, int row_bytes, int32_t idx, bool load, int cnt) {
    return (uint32_t)eval_rows<G, CPL>((const int8_t*)rows, row_bytes, idx, load, cnt, qc, qn);
  }
};

template <int CCPL, int CPB>
struct EvalF32 {
  float qc[CCPL][4];
  __device__ void load(const void* rows, int row_bytes, int dim, int64_t i) {
    canon_load_query<CCPL>((const float*)((const char*)rows + i * row_bytes), dim, qc);
  }
  __device__ uint32_t dist(const void* rows, int row_bytes, int32_t idx, bool load, int) {
    return canon_dist_lanes<CCPL, CPB>(qc, (const float*)rows, row_bytes / 4, row_bytes / 16,
                                       load ? idx : -1);
  }
};

// ---- batch peers -------------------------------------------------------------
template <class Eval>
__global__ __launch_bounds__(64) void k_peers(PeerArgs a) {
  __shared__ uint64_t tk_c[WAVE], tk_r[WAVE], tk_o[WAVE];
  const int lane = threadIdx.x;
  const int32_t i = blockIdx.x;
  if (i >= a.b) return;
  Eval ev;
  ev.load(a.bvec, a.row_bytes, a.dim, i);
  uint64_t rk = KEY_INF;
  if (lane < a.k) {
    int32_t id = a.res_ids[(int64_t)i * a.k_pad + lane];
    if (id >= 0) rk = make_key((uint32_t)a.res_d[(int64_t)i * a.k_pad + lane], id);
  }
  for (int32_t j0 = 0; j0 < a.b; j0 += WAVE) {
    int32_t j = j0 + lane;
    bool valid = j < a.b && j != i;
    int cnt = a.b - j0 < WAVE ? a.b - j0 : WAVE;
    uint32_t d = ev.dist(a.bvec, a.row_bytes, j, valid, cnt);
    lanes_topk_offer_ranked(rk, valid, make_key(d, a.id_base + j), a.k, tk_c, tk_r, tk_o);
  }
  if (lane < a.k_pad) {
    bool have = lane < a.k && rk != KEY_INF;
    a.list_ids[(int64_t)i * a.k_pad + lane] = have ? key_id(rk) : -1;
    a.list_d[(int64_t)i * a.k_pad + lane] = have ? (int32_t)key_dist(rk) : a.pad;
  }
}

// ---- update proposals ------------------------------------------------------
__device__ __forceinline__ void emit_proposal(const UpdateArgs& a, int32_t u, int32_t d,
                                              int32_t src) {
  int32_t slot = atomicAdd(&a.counters[0], 1);
  int32_t prev = atomicExch(&a.head[u], slot);
  Proposal p;
  p.target = u;
  p.dist = d;
  p.src = src;
  p.next = prev;
  a.props[slot] = p;
  if (prev == -1) {
    int32_t t = atomicAdd(&a.counters[1], 1);
    a.touched[t] = u;
  }
}

// One wavefront per new point.  Level 1 is the point's search result (its
// distances are reused); level l + 1 is the union of the pre-batch lists of
// the level-l nodes.  The processed set is a bitset over the snapshot (in
// LDS, or a per-block slice of the workspace for large graphs), so every
// node counts once whatever the order in which lanes reach it; the level
// arrays live in LDS.  Each processed node gets the proposal (node,
// distance, new id) if it beats the node's current k-th entry -- the only
// case in which the merge can keep it.  Distances are compared as 32-bit
// patterns (non-negative int32 or float32; the padding is the largest).
template <class Eval, bool GSET>
__global__ __launch_bounds__(64) void k_update(UpdateArgs a) {
  extern __shared__ uint32_t lds[];
  uint32_t* done_bits = GSET ? a.gset + (int64_t)blockIdx.x * a.set_words_pad : lds;
  int32_t* front = a.gfront ? a.gfront + (int64_t)blockIdx.x * 2 * a.front_cap
                           : reinterpret_cast<int32_t*>(lds + (GSET ? 0 : a.set_words_pad));
  int32_t* nxt = front + a.front_cap;
  __shared__ int32_t next_count;
  const int lane = threadIdx.x;
  const int32_t i = blockIdx.x;
  if (i >= a.b) return;
  const int32_t src = a.id_base + i;
  if (GSET) {
    for (int w = lane * 4; w < a.set_words_pad; w += WAVE * 4)
      *reinterpret_cast<v4i*>(done_bits + w) = v4i{0, 0, 0, 0};
    __threadfence();
  } else {
    for (int w = lane; w < a.set_words; w += WAVE) done_bits[w] = 0u;
  }
  __syncthreads();

  // level 1: the search result, distances reused
  int32_t u = -1, du = 0;
  if (lane < a.k) {
    u = a.res_ids[(int64_t)i * a.k_pad + lane];
    du = a.res_d[(int64_t)i * a.k_pad + lane];
  }
  bool fresh1 = u >= 0 && bit_set(done_bits, u);
  if (fresh1) {
    int32_t thr = a.nbr_d[(int64_t)u * a.k_pad + a.k - 1];
    if (du < thr) emit_proposal(a, u, du, src);
  }
  uint64_t m1 = ballot(fresh1);
  if (fresh1) front[rank_below(m1)] = u;
  int fcount = __popcll(m1);
  __syncthreads();

  int upd = 0;
  if (a.depth >= 2) {
    Eval ev;
    ev.load(a.bvec, a.row_bytes, a.dim, i);
    for (int level = 2; level <= a.depth; ++level) {
      const bool keep = level < a.depth;     // this level is expanded further
      if (lane == 0) next_count = 0;
      __syncthreads();
      const int total = fcount * a.k;
      for (int c0 = 0; c0 < total; c0 += WAVE) {
        int c = c0 + lane;
        int t = c / a.k;
        int sidx = c - t * a.k;
        int32_t w = -1;
        if (c < total) {
          int32_t ut = front[t];
          w = a.nbr_ids[(int64_t)ut * a.k_pad + sidx];
        }
        bool fresh = w >= 0 && bit_set(done_bits, w);
        __syncthreads();
        int cnt = total - c0 < WAVE ? total - c0 : WAVE;
        int32_t d = (int32_t)ev.dist(a.vec, a.row_bytes, w, fresh, cnt);
        if (fresh) {
          int32_t thr = a.nbr_d[(int64_t)w * a.k_pad + a.k - 1];
          if (d < thr) emit_proposal(a, w, d, src);
        }
        uint64_t mf = ballot(fresh);
        upd += __popcll(mf);
        if (keep) {
          int base = next_count;
          if (fresh && base + rank_below(mf) < a.front_cap) nxt[base + rank_below(mf)] = w;
          __syncthreads();
          if (lane == 0) next_count = base + __popcll(mf);
          __syncthreads();
        }
      }
      if (keep) {
        __syncthreads();
        fcount = next_count < a.front_cap ? next_count : a.front_cap;
        for (int s2 = lane; s2 < fcount; s2 += WAVE) front[s2] = nxt[s2];
        __syncthreads();
      }
    }
  }
  if (lane == 0) {
    if (a.sims) a.sims[i] = a.evals[i] + (a.b - 1) + upd;
    if (a.stats) {
      a.stats[3 * (int64_t)i + 0] = a.evals[i];
      a.stats[3 * (int64_t)i + 1] = a.list_reads[i];
      a.stats[3 * (int64_t)i + 2] = upd;
    }
  }
}

// ---- merge ----------------------------------------------------------------
// One wavefront per target node.  The proposals of a target are collected
// from its bucket and inserted into the lane-held list by (distance, id);
// the order in which the bucket was filled does not affect the result.
__global__ __launch_bounds__(64) void k_merge(MergeArgs a) {
  const int lane = threadIdx.x;
  const int32_t ntouched = a.counters[1];
  for (int32_t t = blockIdx.x; t < ntouched; t += gridDim.x) {
    const int32_t u = a.touched[t];
    uint64_t rk = KEY_INF;
    if (lane < a.k) {
      int32_t id = a.nbr_ids[(int64_t)u * a.k_pad + lane];
      if (id >= 0) rk = make_key((uint32_t)a.nbr_d[(int64_t)u * a.k_pad + lane], id);
    }
    int32_t p = a.head[u];
    while (p != -1) {
      Proposal pr = a.props[p];
      lanes_topk_insert(rk, make_key((uint32_t)pr.dist, pr.src), a.k);
      p = pr.next;
    }
    if (lane < a.k) {
      bool have = rk != KEY_INF;
      a.nbr_ids[(int64_t)u * a.k_pad + lane] = have ? key_id(rk) : -1;
      a.nbr_d[(int64_t)u * a.k_pad + lane] = have ? (int32_t)key_dist(rk) : a.pad;
    }
    if (lane == 0) a.head[u] = -1;
  }
}

// ---- launchers ---------------------------------------------------------------
// int8 rows: one 16-byte chunk per lane for rows of up to 64 bytes (a group
// of lanes reads a whole row with one load instruction); longer rows (up to
// 256 bytes): groups of 4 lanes, up to 64 bytes per lane.  float32 rows:
// the 16-lane layout of the stored float distance, ceil(dim / 64) chunks
// per lane.
template <template <class> class Fn, class Args>
static hipError_t dispatch_eval(int format, int row_bytes, const Args& a, hipStream_t s,
                                dim3 grid, size_t lds) {
  const int chunks = row_bytes / 16;
  if (format == ROW_I8) {
    if (chunks <= 1) return Fn<EvalI8<1, 1>>::go(a, s, grid, lds);
    if (chunks <= 2) return Fn<EvalI8<2, 1>>::go(a, s, grid, lds);
    if (chunks <= 4) return Fn<EvalI8<4, 1>>::go(a, s, grid, lds);
    if (chunks <= 8) return Fn<EvalI8<4, 2>>::go(a, s, grid, lds);
    if (chunks <= 16) return Fn<EvalI8<4, 4>>::go(a, s, grid, lds);
    return hipErrorInvalidValue;
  }
  if (chunks <= 16) return Fn<EvalF32<1, 8>>::go(a, s, grid, lds);
  if (chunks <= 32) return Fn<EvalF32<2, 4>>::go(a, s, grid, lds);
  if (chunks <= 64) return Fn<EvalF32<4, 2>>::go(a, s, grid, lds);
  if (chunks <= 128) return Fn<EvalF32<8, 1>>::go(a, s, grid, lds);
  if (chunks <= 256) return Fn<EvalF32<16, 1>>::go(a, s, grid, lds);
  return hipErrorInvalidValue;
}

template <class Eval>
struct PeerFn {
  static hipError_t go(const PeerArgs& a, hipStream_t s, dim3 grid, size_t lds) {
    hipLaunchKernelGGL((k_peers<Eval>), grid, dim3(64), lds, s, a);
    return hipGetLastError();
  }
};
template <class Eval>
struct UpdateFn {
  static hipError_t go(const UpdateArgs& a, hipStream_t s, dim3 grid, size_t lds) {
    if (a.gset)
      hipLaunchKernelGGL((k_update<Eval, true>), grid, dim3(64), lds, s, a);
    else
      hipLaunchKernelGGL((k_update<Eval, false>), grid, dim3(64), lds, s, a);
    return hipGetLastError();
  }
};

size_t update_lds_bytes(int64_t n, int64_t front_cap, bool global_set, bool global_front) {
  size_t bytes = global_set ? 0 : (size_t)round_up((n + 31) / 32, 4) * 4;
  return bytes + (global_front ? 0 : 2 * (size_t)front_cap * 4);
}

hipError_t launch_peers(const PeerArgs& a, hipStream_t s) {
  if (a.b <= 0) return hipSuccess;
  return dispatch_eval<PeerFn>(a.format, a.row_bytes, a, s, dim3((unsigned)a.b), 0);
}

hipError_t launch_update(const UpdateArgs& a, hipStream_t s) {
  if (a.b <= 0) return hipSuccess;
  UpdateArgs b = a;
  b.set_words = (int32_t)((a.n + 31) / 32);
  b.set_words_pad = (int32_t)round_up(b.set_words, 4);
  if (b.gset && a.b > a.gset_slots) return hipErrorInvalidValue;
  size_t lds = update_lds_bytes(a.n, a.front_cap, b.gset != nullptr, b.gfront != nullptr);
  return dispatch_eval<UpdateFn>(a.format, a.row_bytes, b, s, dim3((unsigned)a.b), lds);
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t s) {
  if (a.max_touched <= 0) return hipSuccess;
  int32_t blocks = a.max_touched < 8192 ? a.max_touched : 8192;
  hipLaunchKernelGGL(k_merge, dim3((unsigned)blocks), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace knng
