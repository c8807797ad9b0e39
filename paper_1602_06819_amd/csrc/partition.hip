// Balanced k-medoids partitioning (Algorithm 4 of the paper, one compute
// node) and the merge of a partitioned search (Algorithm 3).
//
// One iteration = assign then update:
//   k_medoid_dist    distance of every node to every medoid, [n][p]
//   k_assign         nodes in id order, each to the medoid maximizing
//                    w(m) / (1 + d) with w(m) = N - |C(m)| P (the capacity
//                    weight 1 - |C(m)| / capacity scaled by N = n num,
//                    P = p den); exact cross-multiplied comparisons, ties
//                    to the smaller medoid index.  Inherently sequential
//                    (each choice changes the weights): one wavefront,
//                    lane m holds medoid m, the distance rows are staged
//                    through LDS 64 nodes at a time with the next block's
//                    loads in flight.
//   k_members        each partition's nodes in ascending id order, and
//                    each node's index among them
//   k_member_paths   per node, shortest paths (Section 6) to the members of
//                    its partition through the partition's nodes, over the
//                    k-nn graph taken as undirected (a node's list and the
//                    nodes whose lists hold it; edge length = the stored
//                    distance): the members it does not reach and the sum of
//                    its path lengths to the others
//   k_medoid_argmin  per partition, the member with the fewest unreached
//                    members, then the smallest sum (ties: smaller id),
//                    becomes the medoid
//
// The in-edges are gathered once per partitioning (k_in_degree,
// k_scan_offsets, k_in_fill); their order does not matter (shortest path
// lengths do not depend on the order of relaxations).
#include "common.h"
#include "device.h"
#include "eval.h"
#include "internal.h"

namespace knng {

struct MedoidList {
  int32_t m[64];
};

__global__ void k_set_medoids(int32_t* medoids, MedoidList l, int p) {
  if ((int)threadIdx.x < p) medoids[threadIdx.x] = l.m[threadIdx.x];
}

template <class Eval>
__global__ __launch_bounds__(64) void k_medoid_dist(PartitionArgs a) {
  const int32_t m = blockIdx.y;
  const int32_t u0 = blockIdx.x * WAVE;
  const int32_t u = u0 + (int32_t)threadIdx.x;
  Eval ev;
  ev.load(a.vec, a.row_bytes, a.dim, a.medoids[m]);
  const int cnt = a.n - u0 < WAVE ? a.n - u0 : WAVE;
  const uint32_t d = ev.dist(a.vec, a.row_bytes, u, u < a.n, cnt);
  if (u < a.n) a.D[(int64_t)u * a.p + m] = d;
}

// o beats b: w_o / (1 + d_o) > w_b / (1 + d_b), ties to the smaller index
__device__ __forceinline__ bool beats(int64_t wo, uint32_t dbits_o, int io, int64_t wb,
                                      uint32_t dbits_b, int ib, bool is_float) {
  if (io >= WAVE) return false;
  if (ib >= WAVE) return true;
  if (is_float) {
    const double l = (double)wo * (1.0 + (double)__uint_as_float(dbits_b));
    const double r = (double)wb * (1.0 + (double)__uint_as_float(dbits_o));
    return l > r || (l == r && io < ib);
  }
  const int64_t l = wo * (1 + (int64_t)dbits_b);
  const int64_t r = wb * (1 + (int64_t)dbits_o);
  return l > r || (l == r && io < ib);
}

__global__ __launch_bounds__(64) void k_assign(PartitionArgs a) {
  __shared__ uint32_t buf[2][WAVE * WAVE];
  const int lane = threadIdx.x;
  const bool act = lane < a.p;
  int64_t w = a.N;                         // lane m: N - |C(m)| P
  const int per = a.p;                     // distances per node
  const int nblk = (a.n + WAVE - 1) / WAVE;
  uint32_t reg[WAVE];                      // next block, lane-strided
  auto fetch = [&](int blk) {
    const int64_t base = (int64_t)blk * WAVE * per;
    const int64_t lim = (int64_t)a.n * per;
#pragma unroll
    for (int i = 0; i < WAVE; ++i) {
      const int64_t idx = base + (int64_t)i * WAVE + lane;
      if (i < per) reg[i] = idx < lim ? a.D[idx] : 0u;
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int i = 0; i < WAVE; ++i)
      if (i < per) buf[b][i * WAVE + lane] = reg[i];
  };
  fetch(0);
  stash(0);
  __syncthreads();
  for (int blk = 0; blk < nblk; ++blk) {
    const int cur = blk & 1;
    if (blk + 1 < nblk) fetch(blk + 1);
    const int32_t u0 = blk * WAVE;
    const int cnt = a.n - u0 < WAVE ? a.n - u0 : WAVE;
    for (int j = 0; j < cnt; ++j) {
      const uint32_t d = act ? buf[cur][j * per + lane] : 0u;
      int64_t bw = w;
      uint32_t bd = d;
      int bi = act ? lane : WAVE;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const int64_t ow = (int64_t)shfl_xor_u64((uint64_t)bw, off);
        const uint32_t od = (uint32_t)__shfl_xor((int)bd, off, WAVE);
        const int oi = __shfl_xor(bi, off, WAVE);
        if (beats(ow, od, oi, bw, bd, bi, a.is_float)) {
          bw = ow;
          bd = od;
          bi = oi;
        }
      }
      if (lane == bi) w -= a.P;
      if (lane == 0) a.part[u0 + j] = bi;
    }
    __syncthreads();
    if (blk + 1 < nblk) stash(cur ^ 1);
    __syncthreads();
  }
  // partition sizes -> offsets of the member lists
  const int32_t size = act ? (int32_t)((a.N - w) / a.P) : 0;
  int32_t incl = size;
#pragma unroll
  for (int off = 1; off < WAVE; off <<= 1) {
    const int32_t o = __shfl_up(incl, off, WAVE);
    if (lane >= off) incl += o;
  }
  if (act) a.offsets[lane] = incl - size;
  if (lane == 0) a.offsets[a.p] = a.n;
}

__global__ __launch_bounds__(64) void k_members(PartitionArgs a) {
  const int32_t m = blockIdx.x;
  const int32_t first = a.offsets[m];
  int32_t at = first;
  for (int32_t u0 = 0; u0 < a.n; u0 += WAVE) {
    const int32_t u = u0 + (int32_t)threadIdx.x;
    const bool mine = u < a.n && a.part[u] == m;
    const uint64_t b = ballot(mine);
    if (mine) {
      const int32_t j = at + rank_below(b);
      a.members[j] = u;
      a.pos[u] = j - first;
    }
    at += __popcll(b);
  }
}

// ---- in-edges of the k-nn graph -------------------------------------------------
__global__ void k_in_degree(PartitionArgs a, int32_t* counts) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)a.n * a.k) return;
  const int64_t u = e / a.k;
  const int32_t v = a.nbr_ids[u * a.k_pad + (e - u * a.k)];
  if (v >= 0 && v < a.n) atomicAdd(&counts[v], 1);
}

// exclusive prefix sums of counts[0 .. n) into off[0 .. n], one workgroup
__global__ __launch_bounds__(1024) void k_scan_offsets(const int32_t* counts, int32_t n,
                                                       int32_t* off) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t carry;
  const int t = threadIdx.x, lane = t % WAVE, w = t / WAVE;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int32_t base = 0; base < n; base += 1024) {
    const int32_t i = base + t;
    const int32_t c = i < n ? counts[i] : 0;
    int32_t incl = c;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const int32_t x = __shfl_up(incl, o, WAVE);
      if (lane >= o) incl += x;
    }
    if (lane == WAVE - 1) wsum[w] = incl;
    __syncthreads();
    int32_t before = carry;
    for (int j = 0; j < w; ++j) before += wsum[j];
    if (i < n) off[i] = before + incl - c;
    __syncthreads();
    if (t == 1023) carry = before + incl;
    __syncthreads();
  }
  if (t == 0) off[n] = carry;
}

__global__ void k_in_fill(PartitionArgs a, int32_t* cursor, int32_t* src, int32_t* w) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)a.n * a.k) return;
  const int64_t u = e / a.k;
  const int64_t at = u * a.k_pad + (e - u * a.k);
  const int32_t v = a.nbr_ids[at];
  if (v < 0 || v >= a.n) return;
  const int32_t slot = a.in_off[v] + atomicAdd(&cursor[v], 1);
  src[slot] = (int32_t)u;
  w[slot] = a.nbr_d[at];
}

// ---- shortest paths within a partition (Section 6) ------------------------------
// One wavefront per source node, in a scratch slot of its own: a worklist
// Bellman-Ford over the partition's nodes (lengths are non-negative, so the
// lengths settle within as many rounds as the partition has members; the
// loop is bounded by that).  Lengths are exact int64 sums of the stored
// distances (uint8 graphs) or float64 sums of the float32 ones, kept as
// 64-bit patterns that order like the values; UNREACHED marks a member not
// (yet) reached.  Lane 0 then sums the lengths in member order.
constexpr uint64_t UNREACHED = ~0ull;

__global__ __launch_bounds__(64) void k_member_paths(PartitionArgs a) {
  const int lane = threadIdx.x;
  uint64_t* dist = a.sp_dist + (int64_t)blockIdx.x * a.slot_len;
  int32_t* cur = a.sp_cur + (int64_t)blockIdx.x * a.slot_len;
  int32_t* nxt = a.sp_next + (int64_t)blockIdx.x * a.slot_len;
  int32_t* inq = a.sp_inq + (int64_t)blockIdx.x * a.slot_len;
  __shared__ int32_t s_next;
  for (int32_t u = blockIdx.x; u < a.n; u += gridDim.x) {
    const int32_t t = a.part[u];
    const int32_t lo = a.offsets[t];
    const int32_t nt = a.offsets[t + 1] - lo;
    for (int32_t l = lane; l < nt; l += WAVE) {
      dist[l] = UNREACHED;
      inq[l] = 0;
    }
    __threadfence();
    __syncthreads();
    if (lane == 0) {
      dist[a.pos[u]] = 0ull;
      cur[0] = a.pos[u];
    }
    __threadfence();
    __syncthreads();
    int32_t ncur = 1;
    for (int32_t round = 0; ncur > 0 && round <= nt; ++round) {
      if (lane == 0) s_next = 0;
      for (int32_t i = lane; i < ncur; i += WAVE) inq[cur[i]] = 0;
      __threadfence();
      __syncthreads();
      for (int32_t i = lane; i < ncur; i += WAVE) {
        const int32_t lx = cur[i];
        const int32_t x = a.members[lo + lx];
        const uint64_t dx = dist[lx];
        auto relax = [&](int32_t y, int32_t wbits) {
          if (y < 0 || a.part[y] != t) return;
          const int32_t ly = a.pos[y];
          uint64_t nd;
          if (a.is_float)
            nd = (uint64_t)__double_as_longlong(__longlong_as_double((long long)dx) +
                                                (double)__int_as_float(wbits));
          else
            nd = dx + (uint64_t)(uint32_t)wbits;
          const uint64_t old = atomicMin((unsigned long long*)&dist[ly], (unsigned long long)nd);
          if (nd < old && atomicExch(&inq[ly], 1) == 0) nxt[atomicAdd(&s_next, 1)] = ly;
        };
        for (int j = 0; j < a.k; ++j)
          relax(a.nbr_ids[(int64_t)x * a.k_pad + j], a.nbr_d[(int64_t)x * a.k_pad + j]);
        for (int32_t e = a.in_off[x]; e < a.in_off[x + 1]; ++e) relax(a.in_src[e], a.in_w[e]);
      }
      __threadfence();
      __syncthreads();
      ncur = s_next;
      int32_t* tmp = cur;
      cur = nxt;
      nxt = tmp;
      __syncthreads();
    }
    if (lane == 0) {
      int32_t missed = 0;
      double fs = 0.0;
      uint64_t is = 0;
      for (int32_t l = 0; l < nt; ++l) {
        const uint64_t v = dist[l];
        if (v == UNREACHED)
          ++missed;
        else if (a.is_float)
          fs += __longlong_as_double((long long)v);
        else
          is += v;
      }
      a.sums[u] = a.is_float ? fs : (double)is;
      a.unreached[u] = missed;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(64) void k_medoid_argmin(PartitionArgs a) {
  const int32_t m = blockIdx.x;
  const int32_t lo = a.offsets[m], hi = a.offsets[m + 1];
  if (hi <= lo) return;                    // empty partition keeps its medoid
  int32_t bm = 0x7fffffff;                 // (unreached, sum, id), smallest first
  double bs = 1e308;
  int32_t bu = 0x7fffffff;
  auto less = [](int32_t m1, double s1, int32_t u1, int32_t m2, double s2, int32_t u2) {
    return m1 < m2 || (m1 == m2 && (s1 < s2 || (s1 == s2 && u1 < u2)));
  };
  for (int32_t j = lo + (int32_t)threadIdx.x; j < hi; j += WAVE) {
    const int32_t u = a.members[j];
    if (less(a.unreached[u], a.sums[u], u, bm, bs, bu)) {
      bm = a.unreached[u];
      bs = a.sums[u];
      bu = u;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int32_t om = __shfl_xor(bm, off, WAVE);
    const double os = __shfl_xor(bs, off, WAVE);
    const int32_t ou = __shfl_xor(bu, off, WAVE);
    if (less(om, os, ou, bm, bs, bu)) {
      bm = om;
      bs = os;
      bu = ou;
    }
  }
  if (threadIdx.x == 0) a.medoids[m] = bu;
}

template <class Eval>
struct DistFn {
  static hipError_t go(const PartitionArgs& a, hipStream_t s, dim3 grid, size_t) {
    hipLaunchKernelGGL((k_medoid_dist<Eval>), grid, dim3(64), 0, s, a);
    return hipGetLastError();
  }
};

hipError_t launch_set_medoids(int32_t* medoids, const int32_t* host_ids, int p, hipStream_t s) {
  if (p < 1 || p > 64) return hipErrorInvalidValue;
  MedoidList l{};
  for (int i = 0; i < p; ++i) l.m[i] = host_ids[i];
  hipLaunchKernelGGL(k_set_medoids, dim3(1), dim3(64), 0, s, medoids, l, p);
  return hipGetLastError();
}

hipError_t launch_partition_iteration(const PartitionArgs& a, hipStream_t s) {
  if (a.n <= 0 || a.p < 1 || a.p > 64) return hipErrorInvalidValue;
  hipError_t e;
  const dim3 dgrid((unsigned)((a.n + WAVE - 1) / WAVE), (unsigned)a.p);
  if ((e = dispatch_eval<DistFn>(a.format, a.row_bytes, a, s, dgrid, 0)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_assign, dim3(1), dim3(64), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_members, dim3((unsigned)a.p), dim3(64), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (a.slots < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_member_paths, dim3((unsigned)a.slots), dim3(64), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_medoid_argmin, dim3((unsigned)a.p), dim3(64), 0, s, a);
  return hipGetLastError();
}

// In-edge lists (in_off, in_src, in_w) of the graph's n nodes; `counts` is
// [n] scratch, also used as the fill cursor.
hipError_t launch_in_edges(const PartitionArgs& a, int32_t* counts, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipError_t e;
  if ((e = launch_fill_i32(counts, a.n, 0, s)) != hipSuccess) return e;
  const int64_t edges = (int64_t)a.n * a.k;
  const unsigned blocks = (unsigned)((edges + 255) / 256);
  hipLaunchKernelGGL(k_in_degree, dim3(blocks), dim3(256), 0, s, a, counts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(1024), 0, s, counts, a.n,
                     const_cast<int32_t*>(a.in_off));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_fill_i32(counts, a.n, 0, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_in_fill, dim3(blocks), dim3(256), 0, s, a, counts,
                     const_cast<int32_t*>(a.in_src), const_cast<int32_t*>(a.in_w));
  return hipGetLastError();
}

// Partition sizes and budgets B_t = min(n_t, max(k, ceil(n_t / speedup))).
__global__ __launch_bounds__(256) void k_part_budgets(const int32_t* part, int32_t n, int32_t p,
                                                      int k, int speedup, int32_t* counts,
                                                      int32_t* budgets) {
  __shared__ int32_t c[64];
  if (threadIdx.x < 64) c[threadIdx.x] = 0;
  __syncthreads();
  for (int32_t u = threadIdx.x; u < n; u += blockDim.x) {
    const int32_t t = part[u];
    if (t >= 0 && t < p) atomicAdd(&c[t], 1);
  }
  __syncthreads();
  if ((int)threadIdx.x < p) {
    const int32_t nt = c[threadIdx.x];
    int32_t b = (nt + speedup - 1) / speedup;
    if (b < k) b = k;
    if (b > nt) b = nt;
    counts[threadIdx.x] = nt;
    budgets[threadIdx.x] = b;
  }
}

hipError_t launch_part_budgets(const int32_t* part, int32_t n, int32_t p, int k, int speedup,
                               int32_t* counts, int32_t* budgets, hipStream_t s) {
  if (p < 1 || p > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_part_budgets, dim3(1), dim3(256), 0, s, part, n, p, k, speedup, counts,
                     budgets);
  return hipGetLastError();
}

// The k best of the p partial results of each query (rows q p .. q p + p - 1).
__global__ __launch_bounds__(64) void k_merge_partitions(const int32_t* ids, const int32_t* d,
                                                         const int32_t* evals, int stride,
                                                         int32_t m, int32_t p, int k,
                                                         int32_t* out_ids, int32_t* out_d,
                                                         int out_stride, int32_t* out_evals,
                                                         int32_t pad) {
  __shared__ uint64_t tk_c[WAVE], tk_r[WAVE], tk_o[WAVE];
  const int lane = threadIdx.x;
  const int32_t q = blockIdx.x;
  if (q >= m) return;
  uint64_t rk = KEY_INF;
  const int total = p * k;
  for (int c0 = 0; c0 < total; c0 += WAVE) {
    const int c = c0 + lane;
    const int t = c / k, j = c - (c / k) * k;
    bool have = false;
    uint64_t key = KEY_INF;
    if (c < total) {
      const int64_t row = (int64_t)q * p + t;
      const int32_t id = ids[row * stride + j];
      if (id >= 0) {
        have = true;
        key = make_key((uint32_t)d[row * stride + j], id);
      }
    }
    lanes_topk_offer_ranked(rk, have, key, k, tk_c, tk_r, tk_o);
  }
  if (lane < out_stride) {
    const bool have = lane < k && rk != KEY_INF;
    out_ids[(int64_t)q * out_stride + lane] = have ? key_id(rk) : -1;
    out_d[(int64_t)q * out_stride + lane] = have ? (int32_t)key_dist(rk) : pad;
  }
  if (out_evals) {
    int32_t e = 0;
    for (int t = lane; t < p; t += WAVE) e += evals[(int64_t)q * p + t];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) e += __shfl_xor(e, off, WAVE);
    if (lane == 0) out_evals[q] = e;
  }
}

hipError_t launch_merge_partitions(const int32_t* ids, const int32_t* d, const int32_t* evals,
                                   int stride, int32_t m, int32_t p, int k, int32_t* out_ids,
                                   int32_t* out_d, int out_stride, int32_t* out_evals,
                                   int32_t pad, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge_partitions, dim3((unsigned)m), dim3(64), 0, s, ids, d, evals,
                     stride, m, p, k, out_ids, out_d, out_stride, out_evals, pad);
  return hipGetLastError();
}

}  // namespace knng
