// Device helpers shared by the gfx950 kernels of the k-nn graph builder.
//
// Keys.  Every ranking in the method uses the order (distance, id) with ties
// going to the smaller id.  Distances here are non-negative (int32 squared
// distances of uint8 points, or non-negative float32), so their 32-bit
// patterns order like the values, and a candidate is packed into one 64-bit
// key  (distance bits << 32) | id  whose unsigned order is exactly that
// lexicographic order.  KEY_INF (all ones) marks an empty slot.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace knng {

// Order-preserving 32-bit keys of float values of either sign (the
// dissimilarity of the inner-product metric, -(x . y), may be negative):
// non-negative floats get the sign bit set, negative ones are inverted, so
// the keys compare as unsigned integers like the values.  +inf maps to
// SORT_INF.  Non-negative distances (squared L2) keep their plain bits.
constexpr uint32_t SORT_INF = 0xff800000u;
__host__ __device__ __forceinline__ uint32_t sortable_from_float(float f) {
  const uint32_t b = __builtin_bit_cast(uint32_t, f);
  if ((b & 0x7fffffffu) == 0u) return 0x80000000u;        // -0 and +0: one key
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ __forceinline__ float float_from_sortable(uint32_t k) {
  const uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __builtin_bit_cast(float, b);
}


constexpr int WAVE = 64;
constexpr uint64_t KEY_INF = ~0ull;
constexpr int32_t DIST_PAD_I32 = 0x7fffffff;

__device__ __forceinline__ uint64_t make_key(uint32_t dbits, int32_t id) {
  return ((uint64_t)dbits << 32) | (uint32_t)id;
}
__device__ __forceinline__ uint32_t key_dist(uint64_t key) { return (uint32_t)(key >> 32); }
__device__ __forceinline__ int32_t key_id(uint64_t key) { return (int32_t)(uint32_t)key; }

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// ---- cross-lane moves (ds_bpermute based) ----------------------------------
__device__ __forceinline__ int shfl_i32(int v, int src) { return __shfl(v, src, WAVE); }
__device__ __forceinline__ uint32_t shfl_u32(uint32_t v, int src) {
  return (uint32_t)__shfl((int)v, src, WAVE);
}
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, WAVE);
  uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, WAVE);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
  uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, mask, WAVE);
  uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), mask, WAVE);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int delta) {
  uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, delta, WAVE);
  uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), delta, WAVE);
  return ((uint64_t)hi << 32) | lo;
}

// value of a lane chosen by a wave-uniform index (v_readlane: scalar result)
__device__ __forceinline__ int readlane_i32(int v, int lane) {
  return __builtin_amdgcn_readlane(v, lane);
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

// ballot over the whole wave (64-bit mask)
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// number of set bits of `mask` below this lane
__device__ __forceinline__ int rank_below(uint64_t mask) {
  return __popcll(mask & ((1ull << lane_id()) - 1ull));
}

__device__ __forceinline__ uint64_t min_u64(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint64_t max_u64(uint64_t a, uint64_t b) { return a < b ? b : a; }

// ---- a top-k list spread over lanes: lane j < k holds the j-th smallest --
// Inserts `cand` (uniform across the wave) if it beats the current k-th.
__device__ __forceinline__ void lanes_topk_insert(uint64_t& mine, uint64_t cand, int k) {
  const int lane = lane_id();
  uint64_t kth = readlane_u64(mine, k - 1);
  if (cand >= kth) return;
  int pos = __popcll(ballot(lane < k && mine < cand));
  uint64_t up = shfl_up_u64(mine, 1);
  if (lane < k) {
    if (lane > pos) mine = up;
    else if (lane == pos) mine = cand;
  }
}

// Offer every flagged lane's key to the lane-held top-k list.
__device__ __forceinline__ void lanes_topk_offer(uint64_t& mine, bool flag, uint64_t key, int k) {
  uint64_t kth = readlane_u64(mine, k - 1);
  uint64_t pass = ballot(flag && key < kth);
  while (pass) {
    int j = __ffsll((long long)pass) - 1;
    pass &= pass - 1;
    uint64_t cand = readlane_u64(key, j);
    lanes_topk_insert(mine, cand, k);
  }
}

// Offer many flagged keys at once (same result as lanes_topk_offer).  When
// more than two candidates qualify, every qualifying candidate and every
// list entry computes its rank in the union by counting smaller keys
// (LDS broadcast reads), and the k smallest are scattered into place.
// `cbuf`, `rbuf`, `obuf` are 64-entry LDS arrays owned by this wavefront.
__device__ __forceinline__ void lanes_topk_offer_ranked(uint64_t& mine, bool flag, uint64_t key,
                                                        int k, uint64_t* cbuf, uint64_t* rbuf,
                                                        uint64_t* obuf) {
  const int lane = lane_id();
  uint64_t kth = readlane_u64(mine, k - 1);
  bool pass = flag && key < kth;
  uint64_t P = ballot(pass);
  int np = __popcll(P);
  if (np == 0) return;
  if (np <= 2) {
    while (P) {
      int j = __ffsll((long long)P) - 1;
      P &= P - 1;
      lanes_topk_insert(mine, readlane_u64(key, j), k);
    }
    return;
  }
  if (pass) cbuf[rank_below(P)] = key;
  rbuf[lane] = mine;
  __syncthreads();
  // rank of this lane's candidate / list entry in the union
  int pos = WAVE;
  if (pass) {
    int r = 0;
    for (int t = 0; t < k; ++t) r += rbuf[t] < key;
    for (int t = 0; t < np; ++t) r += cbuf[t] < key;
    pos = r;
  }
  int rpos = WAVE;
  if (lane < k && mine != KEY_INF) {
    int r = lane;
    for (int t = 0; t < np; ++t) r += cbuf[t] < mine;
    rpos = r;
  }
  obuf[lane] = KEY_INF;
  __syncthreads();
  if (pos < k) obuf[pos] = key;
  if (rpos < k) obuf[rpos] = mine;
  __syncthreads();
  mine = lane < k ? obuf[lane] : KEY_INF;
  __syncthreads();
}

// A list of up to 2 * WAVE entries in two registers per lane: lane j holds
// the entries of ranks j (`lo`) and WAVE + j (`hi`).  Offer the flagged keys
// of the lanes: every qualifying candidate and every list entry computes
// its rank in the union by counting smaller keys (LDS broadcast reads), and
// the k smallest are scattered into place.  `cbuf` is a WAVE-entry and
// `rbuf`, `obuf` are 2 * WAVE-entry LDS arrays of this wavefront (a
// workgroup of one wavefront).
__device__ __forceinline__ void wave_topk_offer_ranked2(uint64_t& lo, uint64_t& hi, bool flag,
                                                        uint64_t key, int k, uint64_t* cbuf,
                                                        uint64_t* rbuf, uint64_t* obuf) {
  const int lane = lane_id();
  const uint64_t kth = k <= WAVE ? readlane_u64(lo, k - 1) : readlane_u64(hi, k - 1 - WAVE);
  const bool pass = flag && key < kth;
  const uint64_t P = ballot(pass);
  const int np = __popcll(P);
  if (np == 0) return;
  if (pass) cbuf[rank_below(P)] = key;
  rbuf[lane] = lo;
  rbuf[WAVE + lane] = hi;
  obuf[lane] = KEY_INF;
  obuf[WAVE + lane] = KEY_INF;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  int pos = 2 * WAVE;
  if (pass) {
    int r = 0;
    for (int t = 0; t < k; ++t) r += rbuf[t] < key;
    for (int t = 0; t < np; ++t) r += cbuf[t] < key;
    pos = r;
  }
  int rlo = 2 * WAVE, rhi = 2 * WAVE;
  if (lane < k && lo != KEY_INF) {
    int r = lane;
    for (int t = 0; t < np; ++t) r += cbuf[t] < lo;
    rlo = r;
  }
  if (WAVE + lane < k && hi != KEY_INF) {
    int r = WAVE + lane;
    for (int t = 0; t < np; ++t) r += cbuf[t] < hi;
    rhi = r;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (pos < k) obuf[pos] = key;
  if (rlo < k) obuf[rlo] = lo;
  if (rhi < k) obuf[rhi] = hi;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  lo = lane < k ? obuf[lane] : KEY_INF;
  hi = WAVE + lane < k ? obuf[WAVE + lane] : KEY_INF;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// The same for a workgroup of exactly one wavefront: LDS accesses of one
// wavefront complete in order, so wavefront-scope ordering suffices and no
// workgroup barrier (which would also wait for outstanding global loads)
// is issued.
__device__ __forceinline__ void wave_topk_offer_ranked(uint64_t& mine, bool flag, uint64_t key,
                                                       int k, uint64_t* cbuf, uint64_t* rbuf,
                                                       uint64_t* obuf) {
  const int lane = lane_id();
  uint64_t kth = readlane_u64(mine, k - 1);
  bool pass = flag && key < kth;
  uint64_t P = ballot(pass);
  int np = __popcll(P);
  if (np == 0) return;
  if (np <= 2) {
    while (P) {
      int j = __ffsll((long long)P) - 1;
      P &= P - 1;
      lanes_topk_insert(mine, readlane_u64(key, j), k);
    }
    return;
  }
  if (pass) cbuf[rank_below(P)] = key;
  rbuf[lane] = mine;
  obuf[lane] = KEY_INF;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  int pos = WAVE;
  if (pass) {
    int r = 0;
#pragma unroll 4
    for (int t = 0; t < k; ++t) r += rbuf[t] < key;
#pragma unroll 8
    for (int t = 0; t < np; ++t) r += cbuf[t] < key;
    pos = r;
  }
  int rpos = WAVE;
  if (lane < k && mine != KEY_INF) {
    int r = lane;
#pragma unroll 8
    for (int t = 0; t < np; ++t) r += cbuf[t] < mine;
    rpos = r;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (pos < k) obuf[pos] = key;
  if (rpos < k) obuf[rpos] = mine;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  mine = lane < k ? obuf[lane] : KEY_INF;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ---- register lists: KM keys sorted ascending, compile-time indexed -------
template <int KM>
__device__ __forceinline__ void reg_list_insert(uint64_t (&L)[KM], uint64_t cand) {
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    uint64_t lo = min_u64(L[j], cand);
    cand = max_u64(L[j], cand);
    L[j] = lo;
  }
}

// Merge two ascending lists, keeping the KM smallest in L (ascending).
// min(a[j], b[KM-1-j]) is bitonic and holds the KM smallest; a bitonic
// merge network then sorts it.
template <int KM>
__device__ __forceinline__ void reg_list_merge(uint64_t (&L)[KM], const uint64_t (&B)[KM]) {
#pragma unroll
  for (int j = 0; j < KM; ++j) L[j] = min_u64(L[j], B[KM - 1 - j]);
#pragma unroll
  for (int s = KM / 2; s >= 1; s >>= 1) {
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      if ((j & s) == 0) {
        uint64_t a = L[j], b = L[j + s];
        L[j] = min_u64(a, b);
        L[j + s] = max_u64(a, b);
      }
    }
  }
}

// Merge this lane's list with the list of lane (lane ^ mask).
template <int KM>
__device__ __forceinline__ void reg_list_merge_xor(uint64_t (&L)[KM], int mask) {
  uint64_t other[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) other[j] = shfl_xor_u64(L[j], mask);
  reg_list_merge<KM>(L, other);
}

}  // namespace knng
