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
//
// Latency.  A batch of 256 points gives one wavefront per query on a
// 1,024-SIMD chip, so the time of a batch is the length of the slowest
// query's chain of dependent steps.  Every evaluated candidate's adjacency
// row is therefore fetched together with its point row and staged in LDS:
// when the climb moves to a candidate (or a restart is accepted) its list
// is already on chip, and a climb step costs one round trip to memory.
#include "common.h"
#include "internal.h"

namespace knng {

typedef int v4i __attribute__((ext_vector_type(4)));

// DPP exchange inside groups of 2 / 4 lanes (no LDS traffic)
__device__ __forceinline__ int dpp_xor1(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
}
__device__ __forceinline__ int dpp_xor2(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
}
template <int G>
__device__ __forceinline__ int group_sum(int v) {
  if (G >= 2) v += dpp_xor1(v);
  if (G >= 4) v += dpp_xor2(v);
  return v;
}

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

// The same from a raw uint8 point of `dim` coordinates.
template <int G, int CPL>
__device__ __forceinline__ int32_t load_query_raw(const uint8_t* q, int dim, v4i (&qc)[CPL]) {
  const int sub = lane_id() % G;
  int nrm = 0;
#pragma unroll
  for (int pp = 0; pp < CPL; ++pp) {
    int off = 16 * (sub + G * pp);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int packed = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        int j = off + 4 * e + t;
        int v = j < dim ? (int)q[j] - 128 : 0;
        packed |= (v & 0xff) << (8 * t);
      }
      qc[pp][e] = packed;
      nrm = __builtin_amdgcn_sdot4(packed, packed, nrm, false);
    }
  }
  return group_sum<G>(nrm);
}

// ---- distances of up to 64 candidates --------------------------------------
// Lane j holds candidate row index `idx` and a flag `load` (the row exists);
// groups of G lanes each take one candidate per pass.  Returns in lane j
// (j < cnt, load set) the exact
// squared distance |q|^2 + |x|^2 - 2 q.x (v_dot4 on int8 lanes).  With
// LISTS, the group also fetches the candidate's adjacency row (16 ids) into
// lists[16 j ...].  All loads are issued before any arithmetic.
template <int G, int CPL, bool LISTS>
__device__ __forceinline__ int32_t eval_rows(const int8_t* base, int row_bytes, int32_t idx,
                                             bool load, int cnt, const v4i (&qc)[CPL],
                                             int32_t qn, const int32_t* nbr_ids,
                                             int32_t* lists) {
  constexpr int SLOTS = WAVE / G;
  constexpr int LROW = 16;                       // ids in a staged adjacency row
  constexpr int LCPL = (LROW / 4 + G - 1) / G;   // 16-byte list chunks per lane
  const int lane = lane_id();
  const int slot = lane / G;
  const int sub = lane % G;
  const int passes = (cnt + SLOTS - 1) / SLOTS;
  const int32_t tagged = load ? idx : -1;        // row index, -1 when absent
  // phase 1: the candidate of this lane's group in every pass (all lanes
  // take part in every cross-lane read; the reads are independent)
  int32_t cid[G];
#pragma unroll
  for (int p = 0; p < G; ++p) {
    const int c = p * SLOTS + slot;
    const int32_t v = G == 1 ? tagged : shfl_i32(tagged, c & 63);
    cid[p] = (p < passes && c < cnt) ? v : -1;
  }
  // phase 2: every gather of the call
  v4i xv[G][CPL];
  v4i lv[G][LISTS ? LCPL : 1];
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
    if (LISTS) {
#pragma unroll
      for (int lc = 0; lc < LCPL; ++lc) {
        const int chunk = sub + G * lc;
        if (ok && chunk < LROW / 4)
          lv[p][lc] = *reinterpret_cast<const v4i*>(nbr_ids + (int64_t)cid[p] * LROW + 4 * chunk);
      }
    }
  }
  // phase 3: distances (and staging of the adjacency rows)
  int32_t dg[G];
#pragma unroll
  for (int p = 0; p < G; ++p) {
    const int c = p * SLOTS + slot;
    if (LISTS) {
#pragma unroll
      for (int lc = 0; lc < LCPL; ++lc) {
        const int chunk = sub + G * lc;
        if (cid[p] >= 0 && chunk < LROW / 4)
          *reinterpret_cast<v4i*>(lists + c * LROW + 4 * chunk) = lv[p][lc];
      }
    }
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
  // phase 4: candidate c's distance to lane c
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

__device__ __forceinline__ bool bit_test(const uint32_t* bits, int32_t id) {
  return (bits[id >> 5] >> (id & 31)) & 1u;
}

// Set the bit of `id`; true iff it was clear before (LDS atomic).
__device__ __forceinline__ bool bit_set(uint32_t* bits, int32_t id) {
  uint32_t m = 1u << (id & 31);
  return (atomicOr(&bits[id >> 5], m) & m) == 0u;
}

// ---- iGNNS ------------------------------------------------------------------
// Candidates of a step are seen in two layouts: the "lane view" (candidate c
// in lane c: used for the sequential-order decisions with ballots) and the
// "group view" (candidate p * SLOTS + g handled by lane group g in pass p:
// used for the gathers and dot products).
//
// Software pipeline.  As soon as a step's distances are known, the step's
// outcome (the first improving neighbour or accepted restart, or the next
// restart window) determines the next step's candidates; their gathers are
// issued before this step's bookkeeping (visited marks, result list,
// counters), which then overlaps the next round trip to memory.  The
// bookkeeping is wavefront-local (no workgroup barrier, which would wait
// for the gathers in flight).
template <int G, int CPL, bool LISTS>
__global__ __launch_bounds__(64) void k_search_u8(SearchArgs a) {
  extern __shared__ uint32_t lds[];
  uint32_t* vis = lds;                                                  // visited bitset
  int32_t* lists = reinterpret_cast<int32_t*>(lds + a.vis_words_pad);   // staged rows
  __shared__ uint64_t tk_c[WAVE], tk_r[WAVE], tk_o[WAVE];
  constexpr int SLOTS = WAVE / G;
  constexpr int LROW = 16;                       // ids in a staged adjacency row
  constexpr int LCPL = (LROW / 4 + G - 1) / G;   // 16-byte list chunks per lane
  const int lane = threadIdx.x;
  const int slot = lane / G;
  const int sub = lane % G;
  const uint32_t mmask = a.m_mod - 1u;
  const uint32_t n = (uint32_t)a.n;

  for (int32_t qi = blockIdx.x; qi < a.m; qi += gridDim.x) {
    for (int w = lane; w < a.vis_words; w += WAVE) vis[w] = 0u;
    __syncthreads();

    v4i qc[CPL];
    const int32_t qn =
        a.qvec ? load_query_rows<G, CPL>(a.qvec + (int64_t)qi * a.row_bytes, a.row_bytes, qc)
               : load_query_raw<G, CPL>(a.qraw + (int64_t)qi * a.dim, a.dim, qc);
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
    uint32_t Ag[G], Cg[G];           // the same for this lane's group candidates
#pragma unroll
    for (int p = 0; p < G; ++p) {
      Ag[p] = G == 1 ? Aj : shfl_u32(Aj, p * SLOTS + slot);
      Cg[p] = G == 1 ? Cj : shfl_u32(Cj, p * SLOTS + slot);
    }

    uint64_t rk = KEY_INF;          // result list: lane j < k holds the j-th best
    uint64_t kth = KEY_INF;         // (uniform) the list's k-th key
    int32_t best = DIST_PAD_I32;    // (uniform) best distance evaluated so far
    int evals = 0;
    int list_reads = 0;             // neighbour lists scanned by the climb
    uint32_t P = 0;                 // permutation positions consumed
    uint32_t xP = lcg.x0;           // value at position P
    int32_t dcur = 0;
    bool climbing = false;
    const int64_t trace_base = (int64_t)qi * a.trace_stride;

    // current step's candidates: lane view (cidL, xL) and group view (cidG)
    int32_t cidL = -1;
    uint32_t xL = 0;
    int32_t cidG[G];
    v4i xv[G][CPL];
    v4i lv[G][LISTS ? LCPL : 1];

    auto window = [&]() {
      xL = (Aj * xP + Cj) & mmask;
      cidL = (P + (uint32_t)lane < a.m_mod && xL < n) ? (int32_t)xL : -1;
#pragma unroll
      for (int p = 0; p < G; ++p) {
        const uint32_t c = (uint32_t)(p * SLOTS + slot);
        const uint32_t xg = (Ag[p] * xP + Cg[p]) & mmask;
        cidG[p] = (P + c < a.m_mod && xg < n) ? (int32_t)xg : -1;
      }
    };
    auto climb_from = [&](int f) {
      cidL = lane < a.k ? lists[f * LROW + lane] : -1;
#pragma unroll
      for (int p = 0; p < G; ++p) {
        const int c = p * SLOTS + slot;
        cidG[p] = c < a.k ? lists[f * LROW + c] : -1;
      }
    };
    auto issue = [&]() {
#pragma unroll
      for (int p = 0; p < G; ++p) {
        const bool ok = cidG[p] >= 0;
#pragma unroll
        for (int pp = 0; pp < CPL; ++pp) {
          const int off = 16 * (sub + G * pp);
          if (ok && off < a.row_bytes)
            xv[p][pp] =
                *reinterpret_cast<const v4i*>(a.vec + (int64_t)cidG[p] * a.row_bytes + off);
          else
            xv[p][pp] = v4i{0, 0, 0, 0};
        }
        if (LISTS) {
#pragma unroll
          for (int lc = 0; lc < LCPL; ++lc) {
            const int chunk = sub + G * lc;
            if (ok && chunk < LROW / 4)
              lv[p][lc] = *reinterpret_cast<const v4i*>(a.nbr_ids + (int64_t)cidG[p] * LROW +
                                                        4 * chunk);
          }
        }
      }
    };

    bool done = a.B <= 0;
    if (!done) {
      window();
      issue();
    }
    while (!done) {
      // visited probe of the lane-view candidate (LDS) while gathers fly
      const bool seen = bit_test(vis, cidL >= 0 ? cidL : 0);
      // distances of the group-view candidates; stage their adjacency rows
      int32_t dg[G];
#pragma unroll
      for (int p = 0; p < G; ++p) {
        const int c = p * SLOTS + slot;
        if (LISTS) {
#pragma unroll
          for (int lc = 0; lc < LCPL; ++lc) {
            const int chunk = sub + G * lc;
            if (cidG[p] >= 0 && chunk < LROW / 4)
              *reinterpret_cast<v4i*>(lists + c * LROW + 4 * chunk) = lv[p][lc];
          }
        }
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
        dg[p] = cidG[p] >= 0 ? qn + xx - 2 * qx : DIST_PAD_I32;
      }
      int32_t d = dg[0];
      if (G > 1) {
        d = DIST_PAD_I32;
#pragma unroll
        for (int p = 0; p < G; ++p) {
          const int j = lane - p * SLOTS;
          const bool mine = j >= 0 && j < SLOTS;
          const int32_t got = shfl_i32(dg[p], mine ? j * G : 0);
          if (mine) d = got;
        }
      }
      const bool valid = cidL >= 0 && !seen;

      // the sequential rule on this step's candidates
      const uint64_t V = ballot(valid);
      uint64_t S;                   // the lane the sequential rule stops at
      if (!climbing) {
        // Expansion test (similarity 1/(1+d) below s_max / e).  A restart
        // that is rejected is never closer than the best so far, so the
        // best distance a candidate is tested against is the one before
        // the window, or the candidate's own distance if that is smaller.
        const int32_t bt = d < best ? d : best;
        const bool keep = valid && !((int64_t)a.e_den * (1 + (int64_t)d) >
                                     (int64_t)a.e_num * (1 + (int64_t)bt));
        S = ballot(keep);
      } else {
        S = ballot(valid && d < dcur);
      }
      const int f = S ? __ffsll((long long)S) - 1 : WAVE;
      uint64_t C = f < WAVE ? (V & ((2ull << f) - 1ull)) : V;
      const int rem = a.B - evals;
      bool stop = false;
      if (__popcll(C) >= rem) {
        const bool in = ((C >> lane) & 1ull) && rank_below(C) < rem;
        C = ballot(in);
        stop = true;
      }
      const bool mine = (C >> lane) & 1ull;
      const int32_t cid_now = cidL;
      const int32_t d_now = d;

      // the next step: decide its candidates and issue their gathers first
      if (!stop) {
        if (S) {
          const int32_t cur = readlane_i32(cid_now, f);
          dcur = readlane_i32(d_now, f);
          if (!climbing) {
            P += (uint32_t)f + 1u;
            xP = (lcg.a * (uint32_t)cur + lcg.c) & mmask;
            climbing = true;
          }
          if (LISTS) {
            climb_from(f);
          } else {
            cidL = lane < a.k ? a.nbr_ids[(int64_t)cur * a.k_pad + lane] : -1;
#pragma unroll
            for (int p = 0; p < G; ++p) {
              const int c = p * SLOTS + slot;
              cidG[p] = G == 1 ? cidL : shfl_i32(cidL, c & 63);
              if (c >= a.k) cidG[p] = -1;
            }
          }
          ++list_reads;
          issue();
        } else if (!climbing) {
          const uint32_t x63 = (uint32_t)readlane_i32((int32_t)xL, WAVE - 1);
          P += WAVE;
          xP = (lcg.a * x63 + lcg.c) & mmask;
          if (P >= a.m_mod) {
            done = true;
          } else {
            window();
            issue();
          }
        } else {
          climbing = false;        // local maximum: restart
          window();
          issue();
        }
      }

      // bookkeeping of this step: visited, trace, result list, count
      if (mine) atomicOr(&vis[cid_now >> 5], 1u << (cid_now & 31));
      if (a.trace && mine) {
        const int r = rank_below(C);
        if (evals + r < a.trace_stride) a.trace[trace_base + evals + r] = cid_now;
      }
      const uint64_t key = make_key((uint32_t)d_now, cid_now);
      if (ballot(mine && key < kth)) {
        wave_topk_offer_ranked(rk, mine, key, a.k, tk_c, tk_r, tk_o);
        kth = readlane_u64(rk, a.k - 1);
        best = (int32_t)key_dist(readlane_u64(rk, 0));
      }
      evals += __popcll(C);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (stop) break;
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
  __shared__ uint64_t tk_c[WAVE], tk_r[WAVE], tk_o[WAVE];
  const int lane = threadIdx.x;
  const int32_t i = blockIdx.x;
  if (i >= a.b) return;
  v4i qc[CPL];
  const int32_t qn = load_query_rows<G, CPL>(a.bvec + (int64_t)i * a.row_bytes, a.row_bytes, qc);
  uint64_t rk = KEY_INF;
  if (lane < a.k) {
    int32_t id = a.res_ids[(int64_t)i * a.k_pad + lane];
    if (id >= 0) rk = make_key((uint32_t)a.res_d[(int64_t)i * a.k_pad + lane], id);
  }
  for (int32_t j0 = 0; j0 < a.b; j0 += WAVE) {
    int32_t j = j0 + lane;
    bool valid = j < a.b && j != i;
    int cnt = a.b - j0 < WAVE ? a.b - j0 : WAVE;
    int32_t d = eval_rows<G, CPL, false>(a.bvec, a.row_bytes, j, valid, cnt, qc, qn, nullptr,
                                         nullptr);
    lanes_topk_offer_ranked(rk, valid, make_key((uint32_t)d, a.id_base + j), a.k, tk_c, tk_r,
                            tk_o);
  }
  if (lane < a.k_pad) {
    bool have = lane < a.k && rk != KEY_INF;
    a.list_ids[(int64_t)i * a.k_pad + lane] = have ? key_id(rk) : -1;
    a.list_d[(int64_t)i * a.k_pad + lane] = have ? (int32_t)key_dist(rk) : DIST_PAD_I32;
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
// the level-l nodes.  The processed set is a bitset over the snapshot in
// LDS, so every node counts once whatever the order in which lanes reach
// it; the level arrays live in LDS too.  Each processed node gets the
// proposal (node, distance, new id) if it beats the node's current k-th
// entry -- the only case in which the merge can keep it.
template <int G, int CPL>
__global__ __launch_bounds__(64) void k_update_u8(UpdateArgs a) {
  extern __shared__ uint32_t lds[];
  uint32_t* done_bits = lds;                                    // processed set
  int32_t* front = reinterpret_cast<int32_t*>(lds + a.set_words_pad);
  int32_t* nxt = front + a.front_cap;
  __shared__ int32_t next_count;
  const int lane = threadIdx.x;
  const int32_t i = blockIdx.x;
  if (i >= a.b) return;
  const int32_t src = a.id_base + i;
  for (int w = lane; w < a.set_words; w += WAVE) done_bits[w] = 0u;
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
    v4i qc[CPL];
    const int32_t qn =
        load_query_rows<G, CPL>(a.bvec + (int64_t)i * a.row_bytes, a.row_bytes, qc);
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
        int32_t d = eval_rows<G, CPL, false>(a.vec, a.row_bytes, w, fresh, cnt, qc, qn, nullptr,
                                             nullptr);
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
// One 16-byte chunk of a row per lane for rows of up to 64 bytes (a group
// of lanes reads a whole row with one load instruction, so one instruction
// fetches 64 / G rows); longer rows (up to 256 bytes): groups of 4 lanes,
// up to 64 bytes per lane.
template <template <int, int> class Fn, class Args>
static hipError_t dispatch_rows(int row_bytes, const Args& a, hipStream_t s, dim3 grid,
                                size_t lds) {
  const int chunks = row_bytes / 16;
  if (chunks <= 1) return Fn<1, 1>::go(a, s, grid, lds);
  if (chunks <= 2) return Fn<2, 1>::go(a, s, grid, lds);
  if (chunks <= 4) return Fn<4, 1>::go(a, s, grid, lds);
  if (chunks <= 8) return Fn<4, 2>::go(a, s, grid, lds);
  if (chunks <= 16) return Fn<4, 4>::go(a, s, grid, lds);
  return hipErrorInvalidValue;
}

template <int G, int CPL>
struct SearchFn {
  static hipError_t go(const SearchArgs& a, hipStream_t s, dim3 grid, size_t lds) {
    if (a.k_pad == 16)
      hipLaunchKernelGGL((k_search_u8<G, CPL, true>), grid, dim3(64), lds, s, a);
    else
      hipLaunchKernelGGL((k_search_u8<G, CPL, false>), grid, dim3(64), lds, s, a);
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

size_t search_lds_bytes(int64_t n, int k_pad) {
  int64_t words = round_up((n + 31) / 32, 4);
  size_t bytes = (size_t)words * 4;
  if (k_pad == 16) bytes += (size_t)WAVE * 16 * 4;   // staged adjacency rows
  return bytes;
}

size_t update_lds_bytes(int64_t n, int64_t front_cap) {
  return (size_t)round_up((n + 31) / 32, 4) * 4 + 2 * (size_t)front_cap * 4;
}

hipError_t launch_search_u8(const SearchArgs& a, hipStream_t s) {
  if (a.m <= 0) return hipSuccess;
  SearchArgs b = a;
  b.vis_words = (int32_t)((a.n + 31) / 32);
  b.vis_words_pad = (int32_t)round_up(b.vis_words, 4);
  size_t lds = search_lds_bytes(a.n, a.k_pad);
  unsigned grid = (unsigned)(a.m < 1048576 ? a.m : 1048576);
  return dispatch_rows<SearchFn>(a.row_bytes, b, s, dim3(grid), lds);
}

hipError_t launch_peers_u8(const PeerArgs& a, hipStream_t s) {
  if (a.b <= 0) return hipSuccess;
  return dispatch_rows<PeerFn>(a.row_bytes, a, s, dim3((unsigned)a.b), 0);
}

hipError_t launch_update_u8(const UpdateArgs& a, hipStream_t s) {
  if (a.b <= 0) return hipSuccess;
  UpdateArgs b = a;
  b.set_words = (int32_t)((a.n + 31) / 32);
  b.set_words_pad = (int32_t)round_up(b.set_words, 4);
  size_t lds = update_lds_bytes(a.n, a.front_cap);
  return dispatch_rows<UpdateFn>(a.row_bytes, b, s, dim3((unsigned)a.b), lds);
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t s) {
  if (a.max_touched <= 0) return hipSuccess;
  int32_t blocks = a.max_touched < 8192 ? a.max_touched : 8192;
  hipLaunchKernelGGL(k_merge, dim3((unsigned)blocks), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace knng
