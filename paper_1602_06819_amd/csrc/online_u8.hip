// Online insertion kernels for uint8 points (rows stored as int8, exact
// int32 squared distances):
//
//   k_search_u8   iGNNS (Section 3), one wavefront per query
//   k_peers_u8    list of each new node = k best of its search result and
//                 the other points of the batch
//   k_update_u8   Update (Algorithm 2) on the pre-batch lists: proposals
//                 (node, distance, new id), bucketed per target node
//   k_merge       each target's list = k best of its list and proposals
//
// Sequential semantics on a 64-lane wavefront.  iGNNS is a sequential
// procedure: restart nodes are drawn one at a time and tested, and the
// eager climb moves to the *first* improving neighbour.  The kernel
// evaluates speculatively -- a whole window of 64 restart candidates, or a
// whole neighbour list, in parallel -- and then commits only the prefix the
// sequential rule would have evaluated (up to and including the first
// accepted restart or the first improving neighbour, and never past the
// budget).  Only committed evaluations are counted, marked visited and
// offered to the result list, so results, evaluation counts and the order
// of evaluations equal those of the sequential procedure.
#include "common.h"
#include "internal.h"

namespace knng {

typedef int v4i __attribute__((ext_vector_type(4)));

// ---- distances: G lanes per candidate, CPL 16-byte chunks per lane -------
// Lane `j` holds a candidate row index `idx` (valid or not).  Returns, in
// lane j (j < cnt), the exact squared distance of the query to row idx:
//   |q|^2 + |x|^2 - 2 q.x  with q.x and |x|^2 from v_dot4 on int8 lanes.
// All loads of a call are issued before any arithmetic.
template <int G, int CPL>
__device__ __forceinline__ int32_t eval_rows(const int8_t* base, int row_bytes, int32_t idx,
                                             bool valid, int cnt, const v4i (&qc)[CPL],
                                             int32_t qn) {
  constexpr int SLOTS = WAVE / G;
  const int lane = lane_id();
  const int slot = lane / G;
  const int sub = lane % G;
  const int passes = (cnt + SLOTS - 1) / SLOTS;
  const int vflag = valid ? 1 : 0;
  v4i xv[G][CPL];
  bool cv[G];
#pragma unroll
  for (int p = 0; p < G; ++p) {
    int c = p * SLOTS + slot;
    // every lane takes part in both cross-lane reads (a lane must never
    // read a register of a lane that is inactive at that point)
    int32_t cid = shfl_i32(idx, c & 63);
    int cval = shfl_i32(vflag, c & 63);
    bool ok = p < passes && c < cnt && cval != 0;
    cv[p] = ok;
#pragma unroll
    for (int pp = 0; pp < CPL; ++pp) {
      int off = 16 * (sub + G * pp);
      if (ok && off < row_bytes)
        xv[p][pp] = *reinterpret_cast<const v4i*>(base + (int64_t)cid * row_bytes + off);
      else
        xv[p][pp] = v4i{0, 0, 0, 0};
    }
  }
  int32_t result = DIST_PAD_I32;
#pragma unroll
  for (int p = 0; p < G; ++p) {
    if (p >= passes) continue;   // uniform: every lane skips the same passes
    int xx = 0, qx = 0;
#pragma unroll
    for (int pp = 0; pp < CPL; ++pp) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        xx = __builtin_amdgcn_sdot4(xv[p][pp][e], xv[p][pp][e], xx, false);
        qx = __builtin_amdgcn_sdot4(qc[pp][e], xv[p][pp][e], qx, false);
      }
    }
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) {
      xx += __shfl_xor(xx, off, WAVE);
      qx += __shfl_xor(qx, off, WAVE);
    }
    int32_t dg = cv[p] ? qn + xx - 2 * qx : DIST_PAD_I32;
    int j = lane - p * SLOTS;
    bool mine = j >= 0 && j < SLOTS;
    int32_t got = shfl_i32(dg, mine ? j * G : 0);
    if (mine) result = got;
  }
  return result;
}

template <int G, int CPL>
__device__ __forceinline__ void load_query(const int8_t* q, int row_bytes, v4i (&qc)[CPL]) {
  const int sub = lane_id() % G;
#pragma unroll
  for (int pp = 0; pp < CPL; ++pp) {
    int off = 16 * (sub + G * pp);
    qc[pp] = off < row_bytes ? *reinterpret_cast<const v4i*>(q + off) : v4i{0, 0, 0, 0};
  }
}

// ---- restart order: full-period LCG modulo m, parameters from SplitMix64 --
__device__ __forceinline__ uint64_t splitmix_next(uint64_t& s) {
  s += 0x9E3779B97F4A7C15ull;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct Lcg {
  uint32_t a, c, x0;
};

__device__ __forceinline__ Lcg restart_lcg(uint64_t seed, uint64_t key, uint32_t m) {
  uint64_t s = key;
  uint64_t hk = splitmix_next(s);
  uint64_t t = seed ^ hk;
  uint64_t r0 = splitmix_next(t);
  uint64_t r1 = splitmix_next(t);
  uint64_t r2 = splitmix_next(t);
  Lcg l;
  if (m <= 2) {
    l.a = 1;
    l.c = 1;
  } else {
    l.a = (uint32_t)(4ull * (r0 & (uint64_t)(m / 4 - 1)) + 1ull);
    l.c = (uint32_t)(2ull * (r1 & (uint64_t)(m / 2 - 1)) + 1ull);
  }
  l.x0 = (uint32_t)(r2 & (uint64_t)(m - 1));
  return l;
}

__device__ __forceinline__ bool vis_test(const uint32_t* vis, int32_t id) {
  return (vis[id >> 5] >> (id & 31)) & 1u;
}

// ---- iGNNS ------------------------------------------------------------------
template <int G, int CPL>
__global__ __launch_bounds__(64) void k_search_u8(SearchArgs a) {
  extern __shared__ uint32_t vis[];
  const int lane = threadIdx.x;
  const uint32_t mmask = a.m_mod - 1u;

  for (int32_t qi = blockIdx.x; qi < a.m; qi += gridDim.x) {
    for (int w = lane; w < a.vis_words; w += WAVE) vis[w] = 0u;
    __syncthreads();

    v4i qc[CPL];
    load_query<G, CPL>(a.qvec + (int64_t)qi * a.row_bytes, a.row_bytes, qc);
    const int32_t qn = a.qnorm[qi];
    const uint64_t key = a.keys ? a.keys[qi] : a.key_base + (uint64_t)qi;
    const Lcg lcg = restart_lcg(a.seed, key, a.m_mod);

    // lane j holds the map x -> A x + C of j LCG steps (lane 0: identity)
    uint32_t Ai = lcg.a, Ci = lcg.c;   // inclusive: lane + 1 steps
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
      uint32_t A2 = shfl_u32(Ai, lane >= off ? lane - off : lane);
      uint32_t C2 = shfl_u32(Ci, lane >= off ? lane - off : lane);
      if (lane >= off) {
        Ci = Ai * C2 + Ci;
        Ai = Ai * A2;
      }
    }
    uint32_t Aj = shfl_u32(Ai, lane > 0 ? lane - 1 : 0);
    uint32_t Cj = shfl_u32(Ci, lane > 0 ? lane - 1 : 0);
    if (lane == 0) {
      Aj = 1u;
      Cj = 0u;
    }

    uint64_t rk = KEY_INF;          // result list: lane j < k holds the j-th best
    int evals = 0;
    int list_reads = 0;             // neighbour lists read by the climb
    uint32_t P = 0;                 // permutation positions consumed
    uint32_t xP = lcg.x0;           // value at position P
    int32_t cur = -1, dcur = 0;
    bool climbing = false;
    bool done = a.B <= 0;
    int64_t trace_base = (int64_t)qi * a.trace_stride;

    while (!done) {
      int32_t cid;
      bool valid;
      int cnt;
      if (!climbing) {
        uint32_t pos = P + (uint32_t)lane;
        uint32_t x = (Aj * xP + Cj) & mmask;
        cid = (int32_t)x;
        bool in_range = pos < a.m_mod && x < (uint32_t)a.n;
        valid = in_range && !vis_test(vis, in_range ? cid : 0);
        cnt = WAVE;
      } else {
        cid = lane < a.k ? a.nbr_ids[(int64_t)cur * a.k_pad + lane] : -1;
        valid = cid >= 0 && !vis_test(vis, cid >= 0 ? cid : 0);
        cnt = a.k;
        ++list_reads;
      }
      int32_t d = eval_rows<G, CPL>(a.vec, a.row_bytes, cid, valid, cnt, qc, qn);

      uint64_t V = ballot(valid);
      uint64_t S;                   // the lane the sequential rule stops at
      if (!climbing) {
        // expansion test of each restart candidate against the best distance
        // including every candidate drawn before it (prefix minimum)
        int32_t pm = valid ? d : DIST_PAD_I32;
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
          int32_t t = __shfl_up(pm, off, WAVE);
          if (lane >= off) pm = min(pm, t);
        }
        int32_t best_prev = evals > 0 ? (int32_t)key_dist(shfl_u64(rk, 0)) : DIST_PAD_I32;
        pm = min(pm, best_prev);
        bool keep = valid && !((int64_t)a.e_den * (1 + (int64_t)d) >
                               (int64_t)a.e_num * (1 + (int64_t)pm));
        S = ballot(keep);
      } else {
        S = ballot(valid && d < dcur);
      }
      int f = S ? __ffsll((long long)S) - 1 : WAVE;
      uint64_t C = f < WAVE ? (V & ((2ull << f) - 1ull)) : V;
      int rem = a.B - evals;
      bool stop = false;
      if (__popcll(C) >= rem) {
        bool in = ((C >> lane) & 1ull) && rank_below(C) < rem;
        C = ballot(in);
        stop = true;
      }
      // commit: visited, trace, result list, count
      bool mine = (C >> lane) & 1ull;
      if (mine) atomicOr(&vis[cid >> 5], 1u << (cid & 31));
      if (a.trace && mine) {
        int r = rank_below(C);
        if (evals + r < a.trace_stride) a.trace[trace_base + evals + r] = cid;
      }
      lanes_topk_offer(rk, mine, make_key((uint32_t)d, cid), a.k);
      evals += __popcll(C);
      __syncthreads();
      if (stop) break;

      if (!climbing) {
        if (S) {
          cur = shfl_i32(cid, f);
          dcur = shfl_i32(d, f);
          P += (uint32_t)f + 1u;
          xP = (lcg.a * (uint32_t)cur + lcg.c) & mmask;
          climbing = true;
        } else {
          uint32_t x63 = shfl_u32((uint32_t)cid, WAVE - 1);
          P += WAVE;
          xP = (lcg.a * x63 + lcg.c) & mmask;
          if (P >= a.m_mod) done = true;
        }
      } else {
        if (S) {
          cur = shfl_i32(cid, f);
          dcur = shfl_i32(d, f);
        } else {
          climbing = false;
        }
      }
    }

    if (lane < a.out_stride) {
      bool have = lane < a.k && rk != KEY_INF;
      a.out_ids[(int64_t)qi * a.out_stride + lane] = have ? key_id(rk) : -1;
      a.out_d[(int64_t)qi * a.out_stride + lane] = have ? (int32_t)key_dist(rk) : DIST_PAD_I32;
    }
    if (lane == 0) {
      if (a.out_evals) a.out_evals[qi] = evals;
      if (a.out_list_reads) a.out_list_reads[qi] = list_reads;
      if (a.trace && evals < a.trace_stride) a.trace[trace_base + evals] = -1;
    }
    __syncthreads();
  }
}

// ---- batch peers -------------------------------------------------------------
template <int G, int CPL>
__global__ __launch_bounds__(64) void k_peers_u8(PeerArgs a) {
  const int lane = threadIdx.x;
  const int32_t i = blockIdx.x;
  if (i >= a.b) return;
  v4i qc[CPL];
  load_query<G, CPL>(a.bvec + (int64_t)i * a.row_bytes, a.row_bytes, qc);
  const int32_t qn = a.bnorm[i];
  uint64_t rk = KEY_INF;
  if (lane < a.k) {
    int32_t id = a.res_ids[(int64_t)i * a.k_pad + lane];
    if (id >= 0) rk = make_key((uint32_t)a.res_d[(int64_t)i * a.k_pad + lane], id);
  }
  for (int32_t j0 = 0; j0 < a.b; j0 += WAVE) {
    int32_t j = j0 + lane;
    bool valid = j < a.b && j != i;
    int cnt = a.b - j0 < WAVE ? a.b - j0 : WAVE;
    int32_t d = eval_rows<G, CPL>(a.bvec, a.row_bytes, j, valid, cnt, qc, qn);
    lanes_topk_offer(rk, valid, make_key((uint32_t)d, a.id_base + j), a.k);
  }
  if (lane < a.k_pad) {
    bool have = lane < a.k && rk != KEY_INF;
    a.list_ids[(int64_t)i * a.k_pad + lane] = have ? key_id(rk) : -1;
    a.list_d[(int64_t)i * a.k_pad + lane] = have ? (int32_t)key_dist(rk) : DIST_PAD_I32;
  }
}

// ---- update proposals ------------------------------------------------------
__device__ __forceinline__ uint32_t hash_u32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Insert id into the LDS set; true iff it was not there before.
__device__ __forceinline__ bool set_insert(int32_t* tab, int cap, int32_t id) {
  uint32_t h = hash_u32((uint32_t)id) & (uint32_t)(cap - 1);
  while (true) {
    int32_t old = atomicCAS(&tab[h], -1, id);
    if (old == -1) return true;
    if (old == id) return false;
    h = (h + 1u) & (uint32_t)(cap - 1);
  }
}

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
// the level-l nodes.  A per-point processed set (open addressing in LDS)
// makes every node count once, whatever the order in which lanes reach it;
// the level arrays live in LDS as well.  Each processed node gets the
// proposal (node, distance, new id) if it beats the node's current k-th
// entry -- the only case in which the merge can keep it.
template <int G, int CPL>
__global__ __launch_bounds__(64) void k_update_u8(UpdateArgs a) {
  extern __shared__ int32_t lds[];
  int32_t* setv = lds;                       // processed set, hash_cap slots
  int32_t* front = lds + a.hash_cap;         // current level, front_cap slots
  int32_t* nxt = front + a.front_cap;        // next level, front_cap slots
  __shared__ int32_t next_count;
  const int lane = threadIdx.x;
  const int32_t i = blockIdx.x;
  if (i >= a.b) return;
  const int32_t src = a.id_base + i;
  for (int s = lane; s < a.hash_cap; s += WAVE) setv[s] = -1;
  __syncthreads();

  // level 1: the search result, distances reused
  int32_t u = -1, du = 0;
  if (lane < a.k) {
    u = a.res_ids[(int64_t)i * a.k_pad + lane];
    du = a.res_d[(int64_t)i * a.k_pad + lane];
  }
  bool fresh1 = u >= 0 && set_insert(setv, a.hash_cap, u);
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
    v4i qc[CPL];
    load_query<G, CPL>(a.bvec + (int64_t)i * a.row_bytes, a.row_bytes, qc);
    const int32_t qn = a.bnorm[i];
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
        bool fresh = w >= 0 && set_insert(setv, a.hash_cap, w);
        __syncthreads();
        int cnt = total - c0 < WAVE ? total - c0 : WAVE;
        int32_t d = eval_rows<G, CPL>(a.vec, a.row_bytes, w, fresh, cnt, qc, qn);
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
      a.nbr_d[(int64_t)u * a.k_pad + lane] = have ? (int32_t)key_dist(rk) : DIST_PAD_I32;
    }
    if (lane == 0) a.head[u] = -1;
  }
}

// ---- launchers ---------------------------------------------------------------
template <template <int, int> class Fn, class Args>
static hipError_t dispatch_rows(int row_bytes, const Args& a, hipStream_t s, dim3 grid,
                                size_t lds) {
  const int chunks = row_bytes / 16;
  if (chunks <= 1) return Fn<1, 1>::go(a, s, grid, lds);
  if (chunks <= 2) return Fn<2, 1>::go(a, s, grid, lds);
  if (chunks <= 4) return Fn<4, 1>::go(a, s, grid, lds);
  if (chunks <= 8) return Fn<8, 1>::go(a, s, grid, lds);
  if (chunks <= 16) return Fn<16, 1>::go(a, s, grid, lds);
  return hipErrorInvalidValue;
}

template <int G, int CPL>
struct SearchFn {
  static hipError_t go(const SearchArgs& a, hipStream_t s, dim3 grid, size_t lds) {
    hipLaunchKernelGGL((k_search_u8<G, CPL>), grid, dim3(64), lds, s, a);
    return hipGetLastError();
  }
};
template <int G, int CPL>
struct PeerFn {
  static hipError_t go(const PeerArgs& a, hipStream_t s, dim3 grid, size_t lds) {
    hipLaunchKernelGGL((k_peers_u8<G, CPL>), grid, dim3(64), lds, s, a);
    return hipGetLastError();
  }
};
template <int G, int CPL>
struct UpdateFn {
  static hipError_t go(const UpdateArgs& a, hipStream_t s, dim3 grid, size_t lds) {
    hipLaunchKernelGGL((k_update_u8<G, CPL>), grid, dim3(64), lds, s, a);
    return hipGetLastError();
  }
};

hipError_t launch_search_u8(const SearchArgs& a, hipStream_t s) {
  if (a.m <= 0) return hipSuccess;
  size_t lds = (size_t)a.vis_words * 4;
  return dispatch_rows<SearchFn>(a.row_bytes, a, s, dim3((unsigned)a.m), lds);
}

hipError_t launch_peers_u8(const PeerArgs& a, hipStream_t s) {
  if (a.b <= 0) return hipSuccess;
  return dispatch_rows<PeerFn>(a.row_bytes, a, s, dim3((unsigned)a.b), 0);
}

hipError_t launch_update_u8(const UpdateArgs& a, hipStream_t s) {
  if (a.b <= 0) return hipSuccess;
  size_t lds = ((size_t)a.hash_cap + 2 * (size_t)a.front_cap) * 4;
  return dispatch_rows<UpdateFn>(a.row_bytes, a, s, dim3((unsigned)a.b), lds);
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t s) {
  if (a.max_touched <= 0) return hipSuccess;
  int32_t blocks = a.max_touched < 8192 ? a.max_touched : 8192;
  hipLaunchKernelGGL(k_merge, dim3((unsigned)blocks), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace knng
