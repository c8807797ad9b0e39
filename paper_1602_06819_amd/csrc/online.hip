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
#include "eval.h"
#include "internal.h"

namespace knng {

// ---- batch peers -------------------------------------------------------------
template <class Eval>
__global__ __launch_bounds__(64) void k_peers(PeerArgs a) {
  __shared__ uint64_t tk_c[WAVE], tk_r[WAVE], tk_o[WAVE];
  const int lane = threadIdx.x;
  const int32_t i = blockIdx.x;
  if (i >= a.b) return;
  Eval ev;
  ev.load(a.bvec, a.row_bytes, a.dim, i);
  ev.ip = a.ip != 0;
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
  // Proposals are staged here and bucketed in bulk: one reservation of
  // proposal slots per flush instead of a dependent atomic per proposal.
  // The merge orders each bucket by (distance, id), so the order in which
  // proposals are bucketed never reaches the result.
  constexpr int PCAP = 512;
  __shared__ int32_t st_u[PCAP], st_d[PCAP];
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

  int staged = 0;                          // (uniform) proposals in the buffer
  auto flush = [&]() __attribute__((always_inline)) {
    if (staged == 0) return;
    int32_t base = 0;
    if (lane == 0) base = atomicAdd(&a.counters[0], staged);
    base = __shfl(base, 0, WAVE);
    for (int j0 = 0; j0 < staged; j0 += WAVE) {
      const int j = j0 + lane;
      const bool have = j < staged;
      int32_t u = 0, prev = 0;
      if (have) {
        u = st_u[j];
        const int32_t slot = base + j;
        prev = atomicExch(&a.head[u], slot);
        Proposal pr;
        pr.target = u;
        pr.dist = st_d[j];
        pr.src = src;
        pr.next = prev;
        a.props[slot] = pr;
      }
      // targets whose bucket this proposal opened
      const uint64_t first = ballot(have && prev == -1);
      if (first) {
        int32_t tb = 0;
        if (lane == 0) tb = atomicAdd(&a.counters[1], __popcll(first));
        tb = __shfl(tb, 0, WAVE);
        if (have && prev == -1) a.touched[tb + rank_below(first)] = u;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    staged = 0;
  };
  auto stage = [&](bool emit, int32_t u, int32_t d) __attribute__((always_inline)) {
    const uint64_t m = ballot(emit);
    const int cnt = __popcll(m);
    if (cnt == 0) return;
    if (staged + cnt > PCAP) flush();
    if (emit) {
      const int r = staged + rank_below(m);
      st_u[r] = u;
      st_d[r] = d;
    }
    staged += cnt;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  };

  // level 1: the search result, distances reused
  int32_t u = -1, du = 0;
  if (lane < a.k) {
    u = a.res_ids[(int64_t)i * a.k_pad + lane];
    du = a.res_d[(int64_t)i * a.k_pad + lane];
  }
  bool fresh1 = u >= 0 && bit_set(done_bits, u);
  int32_t thr1 = fresh1 ? a.nbr_d[(int64_t)u * a.k_pad + a.k - 1] : 0;
  stage(fresh1 && (uint32_t)du < (uint32_t)thr1, u, du);
  uint64_t m1 = ballot(fresh1);
  if (fresh1) front[rank_below(m1)] = u;
  int fcount = __popcll(m1);
  __syncthreads();

  int upd = 0;
  if (a.depth >= 2) {
    Eval ev;
    ev.load(a.bvec, a.row_bytes, a.dim, i);
    ev.ip = a.ip != 0;
    for (int level = 2; level <= a.depth; ++level) {
      const bool keep = level < a.depth;     // this level is expanded further
      if (lane == 0) next_count = 0;
      __syncthreads();
      const int total = fcount * a.k;
      // list entries of chunk c0 (candidate c = list slot c mod k of front
      // node c / k), fetched one chunk ahead of their evaluation
      auto fetch = [&](int c0) __attribute__((always_inline)) {
        const int c = c0 + lane;
        int32_t w = -1;
        if (c < total) {
          const int t = c / a.k;
          w = a.nbr_ids[(int64_t)front[t] * a.k_pad + (c - t * a.k)];
        }
        return w;
      };
      int32_t w_next = total > 0 ? fetch(0) : -1;
      for (int c0 = 0; c0 < total; c0 += WAVE) {
        const int32_t w = w_next;
        if (c0 + WAVE < total) w_next = fetch(c0 + WAVE);
        bool fresh = w >= 0 && bit_set(done_bits, w);
        // the target's current k-th distance travels with its row
        const int32_t thr = fresh ? a.nbr_d[(int64_t)w * a.k_pad + a.k - 1] : 0;
        __syncthreads();
        int cnt = total - c0 < WAVE ? total - c0 : WAVE;
        int32_t d = (int32_t)ev.dist(a.vec, a.row_bytes, w, fresh, cnt);
        stage(fresh && (uint32_t)d < (uint32_t)thr, w, d);
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
  flush();
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
