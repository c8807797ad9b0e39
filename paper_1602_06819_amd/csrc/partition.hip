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
//   k_members        each partition's nodes in ascending id order
//   k_member_sums    per node, the sum of its distances to its partition
//   k_medoid_argmin  per partition, the member with the smallest sum (ties:
//                    smaller id) becomes the medoid
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
  int32_t at = a.offsets[m];
  for (int32_t u0 = 0; u0 < a.n; u0 += WAVE) {
    const int32_t u = u0 + (int32_t)threadIdx.x;
    const bool mine = u < a.n && a.part[u] == m;
    const uint64_t b = ballot(mine);
    if (mine) a.members[at + rank_below(b)] = u;
    at += __popcll(b);
  }
}

template <class Eval>
__global__ __launch_bounds__(64) void k_member_sums(PartitionArgs a) {
  const int32_t u = blockIdx.x;
  const int32_t m = a.part[u];
  const int32_t lo = a.offsets[m], hi = a.offsets[m + 1];
  Eval ev;
  ev.load(a.vec, a.row_bytes, a.dim, u);
  double fs = 0.0;
  int64_t is = 0;
  for (int32_t j0 = lo; j0 < hi; j0 += WAVE) {
    const int32_t j = j0 + (int32_t)threadIdx.x;
    const bool ok = j < hi;
    const int32_t v = ok ? a.members[j] : 0;
    const int cnt = hi - j0 < WAVE ? hi - j0 : WAVE;
    const uint32_t d = ev.dist(a.vec, a.row_bytes, v, ok, cnt);
    if (ok) {
      if (a.is_float)
        fs += (double)__uint_as_float(d);
      else
        is += (int64_t)d;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    fs += __shfl_xor(fs, off, WAVE);
    is += (int64_t)shfl_xor_u64((uint64_t)is, off);
  }
  if (threadIdx.x == 0) a.sums[u] = a.is_float ? fs : (double)is;
}

__global__ __launch_bounds__(64) void k_medoid_argmin(PartitionArgs a) {
  const int32_t m = blockIdx.x;
  const int32_t lo = a.offsets[m], hi = a.offsets[m + 1];
  if (hi <= lo) return;                    // empty partition keeps its medoid
  double bs = 1e308;
  int32_t bu = 0x7fffffff;
  for (int32_t j = lo + (int32_t)threadIdx.x; j < hi; j += WAVE) {
    const int32_t u = a.members[j];
    const double s = a.sums[u];
    if (s < bs || (s == bs && u < bu)) {
      bs = s;
      bu = u;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double os = __shfl_xor(bs, off, WAVE);
    const int32_t ou = __shfl_xor(bu, off, WAVE);
    if (os < bs || (os == bs && ou < bu)) {
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
template <class Eval>
struct SumFn {
  static hipError_t go(const PartitionArgs& a, hipStream_t s, dim3 grid, size_t) {
    hipLaunchKernelGGL((k_member_sums<Eval>), grid, dim3(64), 0, s, a);
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
  if ((e = dispatch_eval<SumFn>(a.format, a.row_bytes, a, s, dim3((unsigned)a.n), 0)) !=
      hipSuccess)
    return e;
  hipLaunchKernelGGL(k_medoid_argmin, dim3((unsigned)a.p), dim3(64), 0, s, a);
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
