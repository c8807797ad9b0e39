// Distance evaluation of up to 64 candidates per wavefront call, shared by
// the kernels after the search (peers, update, partitioning):
//   EvalI8    int8 rows, exact int32 squared distance
//   EvalF32   float32 rows, the float32 distance of stored float distances
// Both return 32-bit patterns that order like the distances.
#pragma once

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
  bool ip = false;       // (float rows only)
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
  bool ip = false;       // inner-product metric: keys of -(q . x)
  __device__ void load(const void* rows, int row_bytes, int dim, int64_t i) {
    canon_load_query<CCPL>((const float*)((const char*)rows + i * row_bytes), dim, qc);
  }
  __device__ uint32_t dist(const void* rows, int row_bytes, int32_t idx, bool load, int) {
    return canon_dist_lanes<CCPL, CPB>(qc, (const float*)rows, row_bytes / 4, row_bytes / 16,
                                       load ? idx : -1, ip);
  }
};

// ---- dispatch by row format ------------------------------------------------------
// int8 rows: one 16-byte chunk per lane for rows of up to 64 bytes (a group
// of lanes reads a whole row with one load instruction); longer rows (up to
// 256 bytes): groups of 4 lanes, up to 64 bytes per lane.  float32 rows:
// the 16-lane layout of the stored float distance, ceil(dim / 64) chunks
// per lane.
template <template <class> class Fn, class Args>
inline hipError_t dispatch_eval(int format, int row_bytes, const Args& a, hipStream_t s,
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

}  // namespace knng
