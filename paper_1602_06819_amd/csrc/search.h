// iGNNS (Section 3 of the paper), one wavefront per query, for every row
// format of the library:
//
//   ScoreI8    int8 rows (uint8 coordinate - 128): exact int32 squared L2
//   ScoreBF16  bfloat16 rows: sum of (q - x)^2 in float32, q in float32
//   ScoreFP8   FP8 E4M3 rows with one float32 scale s per row:
//              sum of (q - s x)^2 in float32
//   ScoreF32   float32 rows: sum of (q - x)^2 in float32
//   ScoreFP8M  FP8 rows of 257-1024 coordinates on the matrix cores:
//              |q|^2 - 2 s q.v + s^2 sum v^2 from FP8 MFMA dot products
//   ScoreBF16M bfloat16 rows of up to 128 coordinates on the matrix cores:
//              |q|^2 - 2 q.x + |x|^2 from bfloat16 MFMA dot products
//
// Sequential semantics on a 64-lane wavefront.  Restart nodes are drawn one
// at a time and tested, and the eager climb moves to the *first* improving
// neighbour.  The kernel evaluates speculatively -- a window of 64 restart
// candidates, or a whole neighbour list -- and commits only the prefix the
// sequential rule evaluates (up to and including the first accepted restart
// or improving neighbour, never past the budget).  Only committed
// evaluations are counted, marked visited and offered to the result list,
// so results, counts and evaluation order are those of the sequential
// procedure on the same distances.
//
// Distances are handled as 32-bit patterns: int32 distances and non-negative
// float32 distances both order like their bit patterns, so ballots, the
// result list and keys (distance bits << 32 | id) are format independent.
//
// Candidates of a step are seen in two layouts: the "lane view" (candidate
// c in lane c: sequential-order decisions with ballots) and the "group
// view" (candidate p * SLOTS + g handled by lane group g in pass p: the
// gathers and dot products; a group of G lanes reads one row, 16 bytes per
// lane per load, CPL loads per lane).  Groups are lanes g*G .. g*G+G-1, or
// for the MFMA score lanes g, g+16, g+32, g+48 (the operand layout).
//
// Latency.  A batch gives one wavefront per query, so its time is the
// length of the slowest query's chain of dependent steps.  Every candidate's
// adjacency row (LROW ids) is fetched with its point row and staged in LDS,
// so a climb step costs one round trip to memory; and as soon as a step's
// outcome is known the next step's gathers are issued, before this step's
// bookkeeping (wavefront-local, no workgroup barrier), which then overlaps
// the next round trip.
#pragma once

#include "common.h"
#include "device.h"
#include "internal.h"

namespace knng {

// ---- scoring formats -----------------------------------------------------------
// |x|^2 is recomputed from the row (a stored norm would be one more gather
// on every candidate's critical path).
template <int G, int CPL>
struct ScoreI8 {
  static constexpr bool kSide = false;
  static constexpr bool kSide2 = false, kMfma = false, kBatch = false, kWide = false;
  v4i q[CPL];
  int32_t qq;
  __device__ __forceinline__ void load(const SearchArgs& a, const SearchRows& r, int32_t qi) {
    const int sub = lane_id() % G;
    int nrm = 0;
    if (r.qvec) {
      const int8_t* qr = r.qvec + (int64_t)qi * a.row_bytes;
#pragma unroll
      for (int pp = 0; pp < CPL; ++pp) {
        int off = 16 * (sub + G * pp);
        q[pp] = off < a.row_bytes ? *reinterpret_cast<const v4i*>(qr + off) : v4i{0, 0, 0, 0};
      }
    } else {
      const uint8_t* qr = (const uint8_t*)r.qraw + (int64_t)qi * a.dim;
#pragma unroll
      for (int pp = 0; pp < CPL; ++pp) {
        int off = 16 * (sub + G * pp);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          int packed = 0;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            int j = off + 4 * e + t;
            int v = j < a.dim ? (int)qr[j] - 128 : 0;
            packed |= (v & 0xff) << (8 * t);
          }
          q[pp][e] = packed;
        }
      }
    }
#pragma unroll
    for (int pp = 0; pp < CPL; ++pp)
#pragma unroll
      for (int e = 0; e < 4; ++e) nrm = __builtin_amdgcn_sdot4(q[pp][e], q[pp][e], nrm, false);
    qq = group_sum<G>(nrm);
  }
  __device__ __forceinline__ uint32_t dist(const v4i (&x)[CPL], uint32_t) const {
    int xx = 0, qx = 0;
#pragma unroll
    for (int pp = 0; pp < CPL; ++pp)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        xx = __builtin_amdgcn_sdot4(x[pp][e], x[pp][e], xx, false);
        qx = __builtin_amdgcn_sdot4(q[pp][e], x[pp][e], qx, false);
      }
    xx = group_sum<G>(xx);
    qx = group_sum<G>(qx);
    return (uint32_t)(qq + xx - 2 * qx);
  }
  // expansion test: keep r iff e_den (1 + d_r) <= e_num (1 + best)
  __device__ __forceinline__ static bool keep(uint32_t d, uint32_t best, int num, int den) {
    return !((int64_t)den * (1 + (int64_t)d) > (int64_t)num * (1 + (int64_t)best));
  }
};

// float32 query coordinates for the chunks of a row format with EPC
// coordinates per 16-byte chunk
template <int G, int CPL, int EPC>
__device__ __forceinline__ void load_query_f32(const SearchArgs& a, const SearchRows& r,
                                               int32_t qi, float (&q)[CPL][EPC]) {
  const int sub = lane_id() % G;
  const float* qr = (const float*)r.qraw + (int64_t)qi * a.dim;
#pragma unroll
  for (int pp = 0; pp < CPL; ++pp) {
    int c0 = EPC * (sub + G * pp);
#pragma unroll
    for (int e = 0; e < EPC; ++e) q[pp][e] = c0 + e < a.dim ? qr[c0 + e] : 0.f;
  }
}

__device__ __forceinline__ bool keep_f32(uint32_t d, uint32_t best, int num, int den) {
  return !((float)den * (1.f + __uint_as_float(d)) > (float)num * (1.f + __uint_as_float(best)));
}

template <int G, int CPL>
struct ScoreBF16 {
  static constexpr bool kSide = false;
  static constexpr bool kSide2 = false, kMfma = false, kBatch = false, kWide = true;
  float q[CPL][8];
  __device__ __forceinline__ void load(const SearchArgs& a, const SearchRows& r, int32_t qi) {
    load_query_f32<G, CPL, 8>(a, r, qi, q);
  }
  __device__ __forceinline__ uint32_t dist(const v4i (&x)[CPL], uint32_t) const {
    float s = 0.f;
#pragma unroll
    for (int pp = 0; pp < CPL; ++pp)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        uint32_t w = (uint32_t)x[pp][e];
        float d0 = q[pp][2 * e] - bf16_lo(w);
        float d1 = q[pp][2 * e + 1] - bf16_hi(w);
        s = fmaf(d0, d0, s);
        s = fmaf(d1, d1, s);
      }
    return __float_as_uint(group_sum<G>(s));
  }
  __device__ __forceinline__ static bool keep(uint32_t d, uint32_t best, int num, int den) {
    return keep_f32(d, best, num, den);
  }
};

// FP8 rows hold codes v with x ~ s v; the score is sum of (q - s v)^2.
template <int G, int CPL>
struct ScoreFP8 {
  static constexpr bool kSide = true;    // the row scale
  static constexpr bool kSide2 = false, kMfma = false, kBatch = false, kWide = true;
  float q[CPL][16];
  __device__ __forceinline__ void load(const SearchArgs& a, const SearchRows& r, int32_t qi) {
    load_query_f32<G, CPL, 16>(a, r, qi, q);
  }
  __device__ __forceinline__ uint32_t dist(const v4i (&x)[CPL], uint32_t side) const {
    const float scale = __uint_as_float(side);
    float s = 0.f;
#pragma unroll
    for (int pp = 0; pp < CPL; ++pp)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float v[4];
        e4m3x4_to_f32((uint32_t)x[pp][e], v);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const float d = __builtin_fmaf(-scale, v[t], q[pp][4 * e + t]);
          s = __builtin_fmaf(d, d, s);
        }
      }
    return __float_as_uint(group_sum<G>(s));
  }
  __device__ __forceinline__ static bool keep(uint32_t d, uint32_t best, int num, int den) {
    return keep_f32(d, best, num, den);
  }
};

// float32 rows.  With the inner-product metric the score is the sortable
// key of -(q . x), and the expansion test, on exp(q . x), discards a restart
// whose inner product is more than ln e below the best one's.
template <int G, int CPL>
struct ScoreF32 {
  static constexpr bool kSide = false;
  static constexpr bool kSide2 = false, kMfma = false, kBatch = false, kWide = false;
  float q[CPL][4];
  bool ip;
  float margin;
  __device__ __forceinline__ void load(const SearchArgs& a, const SearchRows& r, int32_t qi) {
    load_query_f32<G, CPL, 4>(a, r, qi, q);
    ip = a.ip != 0;
    margin = a.ip_margin;
  }
  __device__ __forceinline__ uint32_t dist(const v4i (&x)[CPL], uint32_t) const {
    float s = 0.f;
    if (ip) {
#pragma unroll
      for (int pp = 0; pp < CPL; ++pp)
#pragma unroll
        for (int e = 0; e < 4; ++e) s = fmaf(q[pp][e], __int_as_float(x[pp][e]), s);
      return sortable_from_float(-group_sum<G>(s));
    }
#pragma unroll
    for (int pp = 0; pp < CPL; ++pp)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float d0 = q[pp][e] - __int_as_float(x[pp][e]);
        s = fmaf(d0, d0, s);
      }
    return __float_as_uint(group_sum<G>(s));
  }
  __device__ __forceinline__ bool keep(uint32_t d, uint32_t best, int num, int den) const {
    if (ip) return !(float_from_sortable(d) - float_from_sortable(best) > margin);
    return keep_f32(d, best, num, den);
  }
};

// FP8 rows scored on the matrix cores.  One 16x16x128 FP8 MFMA multiplies a
// 16-row A operand by 16 candidate rows over 128 coordinates; A holds the
// query in row 0 and zeros elsewhere, so one instruction gives the query's
// dot products with 16 candidates.  Lane l serves candidate l % 16 (the
// slot) and coordinate group l / 16 (the sub): the two operands pair their
// bytes lane group by lane group, so the query and the rows use the same
// chunk of coordinates per lane.  The query is encoded in two FP8 terms,
// q ~ sq (h + l / 16), which keeps about 8 significant bits; the row term
// s^2 sum v^2 is stored at ingest.  The score is |q|^2 - 2 s q.v + s^2 sum
// v^2, i.e. |q - s v|^2 up to rounding (the MFMA's internal sum is not an
// exact float32 sum), clamped at 0; it is valid in the candidates' sub-0
// lanes 0-15.
template <int CPL>
struct ScoreFP8M {
  static_assert(CPL % 2 == 0, "an MFMA step takes two 16-byte chunks per lane");
  static constexpr bool kSide = true, kSide2 = true, kMfma = true, kBatch = false, kWide = true;
  static constexpr int G = 4;
  v4i qh[CPL], ql[CPL];
  float qq;                       // |q|^2
  float qs;                       // the query's code scale sq
  __device__ __forceinline__ void load(const SearchArgs& a, const SearchRows& r, int32_t qi) {
    const int lane = lane_id();
    const int slot = lane % 16, sub = lane / 16;
    const float* qr = (const float*)r.qraw + (int64_t)qi * a.dim;
    float nrm = 0.f, mx = 0.f;
    for (int j = lane; j < a.dim; j += WAVE) {
      const float v = qr[j];
      nrm = __builtin_fmaf(v, v, nrm);
      mx = fmaxf(mx, fabsf(v));
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      nrm += __shfl_xor(nrm, off, WAVE);
      mx = fmaxf(mx, __shfl_xor(mx, off, WAVE));
    }
    qq = nrm;
    qs = mx / 448.f;
    // encode the coordinates into LDS, then take this lane's chunks from there
    __shared__ __align__(16) uint8_t qhb[64 * CPL], qlb[64 * CPL];
    for (int j = lane; j < 64 * CPL; j += WAVE) {
      const float v = (j < a.dim && qs > 0.f) ? qr[j] / qs : 0.f;
      const uint32_t h = f32_to_e4m3(v);
      float hv[4];
      e4m3x4_to_f32(h, hv);
      qhb[j] = (uint8_t)h;
      qlb[j] = (uint8_t)f32_to_e4m3((v - hv[0]) * 16.f);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int pp = 0; pp < CPL; ++pp) {
      const int c0 = 16 * (sub + G * pp);
      qh[pp] = slot == 0 ? *reinterpret_cast<const v4i*>(qhb + c0) : v4i{0, 0, 0, 0};
      ql[pp] = slot == 0 ? *reinterpret_cast<const v4i*>(qlb + c0) : v4i{0, 0, 0, 0};
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __device__ __forceinline__ uint32_t dist(const v4i (&x)[CPL], uint32_t side,
                                           uint32_t side2) const {
    v4f ah = {0.f, 0.f, 0.f, 0.f}, al = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < CPL / 2; ++i) {
      const v8i b = __builtin_shufflevector(x[2 * i], x[2 * i + 1], 0, 1, 2, 3, 4, 5, 6, 7);
      const v8i h = __builtin_shufflevector(qh[2 * i], qh[2 * i + 1], 0, 1, 2, 3, 4, 5, 6, 7);
      const v8i l = __builtin_shufflevector(ql[2 * i], ql[2 * i + 1], 0, 1, 2, 3, 4, 5, 6, 7);
      // format 0 (FP8 E4M3) for both operands, unit block scales (E8M0 127)
      ah = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(h, b, ah, 0, 0, 0, 127, 0, 127);
      al = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(l, b, al, 0, 0, 0, 127, 0, 127);
    }
    const float dot = qs * __builtin_fmaf(al[0], 0.0625f, ah[0]);   // q . v
    const float d = __builtin_fmaf(-2.f * __uint_as_float(side), dot, qq + __uint_as_float(side2));
    return __float_as_uint(d > 0.f ? d : 0.f);
  }
  __device__ __forceinline__ static bool keep(uint32_t d, uint32_t best, int num, int den) {
    return keep_f32(d, best, num, den);
  }
};

// bfloat16 rows scored on the matrix cores.  One 16x16x32 bfloat16 MFMA
// multiplies a 16-row A operand by 16 candidate rows over 32 coordinates:
// A holds the query in two bfloat16 terms, q ~ h + l with h = bf16(q) and
// l = bf16(q - h) (about 16 significant bits), in rows 0 and 1, and zeros
// elsewhere, so one instruction gives both terms' dot products with 16
// candidates.  Lane l serves candidate l % 16 (the slot) and the 8
// coordinates 8 (l / 16) .. of each 32-coordinate block (the sub); the
// operands pair their elements lane by lane, so the query and the rows use
// the same chunk of coordinates per lane.  The row term |x|^2 of the stored
// bfloat16 row is kept at ingest.  The score is |q|^2 - 2 q.x + |x|^2, i.e.
// |q - x|^2 up to rounding (the expanded form cancels: its error is a few
// float32 units of |q|^2 + |x|^2 rather than of the distance), clamped at
// 0; it is valid in the candidates' sub-0 lanes 0-15.
template <int CPL>
struct ScoreBF16M {
  static constexpr bool kSide = false, kSide2 = true, kMfma = true, kBatch = true, kWide = true;
  static constexpr int G = 4;
  v4i qa[CPL];                    // A operand: row 0 h, row 1 l, other rows 0
  float qq;                       // |q|^2
  __device__ __forceinline__ void load(const SearchArgs& a, const SearchRows& r, int32_t qi) {
    const int lane = lane_id();
    const int slot = lane % 16, sub = lane / 16;
    const float* qr = (const float*)r.qraw + (int64_t)qi * a.dim;
    float nrm = 0.f;
    for (int j = lane; j < a.dim; j += WAVE) nrm = __builtin_fmaf(qr[j], qr[j], nrm);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) nrm += __shfl_xor(nrm, off, WAVE);
    qq = nrm;
#pragma unroll
    for (int pp = 0; pp < CPL; ++pp) {
      const int c0 = 8 * (sub + G * pp);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        uint32_t w = 0u;
        if (slot < 2) {
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            const int j = c0 + 2 * e + t;
            const float v = j < a.dim ? qr[j] : 0.f;
            const uint32_t h = f32_to_bf16(v);
            const uint32_t part = slot == 0 ? h : f32_to_bf16(v - bf16_lo(h));
            w |= part << (16 * t);
          }
        }
        qa[pp][e] = (int)w;
      }
    }
  }
  __device__ __forceinline__ uint32_t finish(const v4f& acc, uint32_t side2) const {
    const float dot = acc[0] + acc[1];                                  // q . x
    const float d = __builtin_fmaf(-2.f, dot, qq + __uint_as_float(side2));
    return __float_as_uint(d > 0.f ? d : 0.f);
  }
  // one pass: the blocks' products are independent and summed afterwards
  __device__ __forceinline__ uint32_t dist(const v4i (&x)[CPL], uint32_t,
                                           uint32_t side2) const {
    const v4f z = {0.f, 0.f, 0.f, 0.f};
    v4f part[CPL];
#pragma unroll
    for (int pp = 0; pp < CPL; ++pp)
      part[pp] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, qa[pp]),
                                                         __builtin_bit_cast(v8bf, x[pp]), z, 0,
                                                         0, 0);
#pragma unroll
    for (int pp = 1; pp < CPL; ++pp) part[0] += part[pp];
    return finish(part[0], side2);
  }
  // NP passes at once, block by block across the passes
  template <int NP>
  __device__ __forceinline__ void dist_all(const v4i (&x)[NP][CPL], const uint32_t (&side2)[NP],
                                           uint32_t (&out)[NP]) const {
    v4f acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int pp = 0; pp < CPL; ++pp)
#pragma unroll
      for (int p = 0; p < NP; ++p)
        acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, qa[pp]),
                                                         __builtin_bit_cast(v8bf, x[p][pp]),
                                                         acc[p], 0, 0, 0);
#pragma unroll
    for (int p = 0; p < NP; ++p) out[p] = finish(acc[p], side2[p]);
  }
  __device__ __forceinline__ static bool keep(uint32_t d, uint32_t best, int num, int den) {
    return keep_f32(d, best, num, den);
  }
};

// ---- the search ----------------------------------------------------------------
// CCPL > 0 (float graphs): the kept candidates are re-ranked by the float32
// distance of stored float distances (CCPL chunks per lane of a 16-lane
// group, CPB passes in flight) and the k best by that distance are the
// result.
//
// PB < G (long rows): a step's G passes are split into groups of PB passes
// whose rows do not all fit in registers.  Group 0 is gathered with the
// step's issue; while group j is scored, group j + 1 is gathered into the
// other of two register buffers.
//
// GNNS (the baseline of the comparison in the paper's evaluation): every
// restart is climbed from, a list scan evaluates every unvisited neighbour
// and moves to the closest of them if it is strictly closer than the
// current node, and the search ends after a.restarts restarts and their
// climbs (or at the budget).
//
// PART (partitioned search on one device): row r of a group searches query
// r / nparts within partition r % nparts only -- nodes of other partitions
// are never evaluated or counted, as if absent -- with that partition's
// budget; the rows' results are merged afterwards (k_merge_partitions).
template <class Score, int G, int CPL, int LROW, bool GVIS, int CCPL, int CPB, int PB,
          bool GNNS = false, bool PART = false, bool K2 = false, int WPE = 1, bool KEEP = false>
__global__ __launch_bounds__(64, WPE) void k_search(SearchArgs a) {
  extern __shared__ uint32_t lds[];
  __shared__ uint64_t tk_c[WAVE], tk_r[K2 ? 2 * WAVE : WAVE], tk_o[K2 ? 2 * WAVE : WAVE];
  // With the visited set in global memory, a filter in LDS of the nodes the
  // climb has evaluated.  A restart candidate is drawn from a permutation,
  // so it never repeats an earlier restart: it can only have been visited
  // by a climb step, and when its filter bit is clear it was not; the
  // global set is probed only for the others (and for every list-scan
  // candidate).
  constexpr bool FILT = GVIS && KEEP;
  constexpr int FILT_WORDS = FILT ? 2048 : 1;     // 64 Kbit
  __shared__ uint32_t filt[FILT_WORDS];
  auto filt_bit = [](int32_t id) __attribute__((always_inline)) {
    return ((uint32_t)id * 0x9E3779B1u) >> (32 - 16);
  };
  static_assert(G % PB == 0, "pass groups must divide the passes");
  constexpr int NG = G / PB;                      // pass groups per step
  constexpr int NB = NG > 1 ? 2 : 1;              // register buffers
  constexpr int SLOTS = WAVE / G;
  constexpr bool LISTS = LROW > 0;
  constexpr int LCH = LISTS ? LROW / 4 : 1;       // 16-byte chunks of a staged row
  constexpr int LCPL = (LCH + G - 1) / G;         // list chunks per lane
  const int lane = threadIdx.x;
  // lane -> (candidate slot, lane in the row group): row-major groups of G
  // lanes, or column-major for the MFMA score (candidate = lane % SLOTS)
  constexpr bool CM = Score::kMfma;
  const int slot = CM ? lane % SLOTS : lane / G;
  const int sub = CM ? lane / SLOTS : lane % G;
  const uint32_t mmask = a.m_mod - 1u;
  const uint32_t n = (uint32_t)a.n;
  int32_t* lists = reinterpret_cast<int32_t*>(lds + (GVIS ? 0 : a.vis_words_pad));
  const char* rows = (const char*)a.vec;

  for (int32_t qg = blockIdx.x; qg < a.m; qg += gridDim.x) {
    // the row's group and index in it (uniform across the wavefront)
    const bool g0 = qg < a.rows[0].count;
    const SearchRows& R = g0 ? a.rows[0] : a.rows[1];
    const int32_t qi = g0 ? qg : qg - a.rows[0].count;      // output row
    const int32_t part = PART ? qi % a.nparts : 0;          // partition searched
    const int32_t qq = PART ? qi / a.nparts : qi;           // query of the row
    const int32_t Bq = PART ? a.part_budget[part] : a.B;    // the row's budget
    uint32_t* vis = GVIS ? a.gvis + (int64_t)blockIdx.x * a.vis_words_pad : lds;
    if (GVIS) {
      for (int w = lane * 4; w < a.vis_words_pad; w += WAVE * 4)
        *reinterpret_cast<v4i*>(vis + w) = v4i{0, 0, 0, 0};
      if (FILT)
        for (int w = lane * 4; w < FILT_WORDS; w += WAVE * 4)
          *reinterpret_cast<v4i*>(filt + w) = v4i{0, 0, 0, 0};
      __threadfence();
    } else {
      for (int w = lane; w < a.vis_words; w += WAVE) vis[w] = 0u;
    }
    __syncthreads();

    Score sc;
    sc.load(a, R, qq);
    const uint64_t key = R.keys ? R.keys[qq] : R.key_base + (uint64_t)qq;
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
    // The same for this lane's group candidates.  Wide groups (16 lanes
    // per row, 16 passes) take the group-view positions from the lane view
    // with one shuffle per pass instead, which keeps 32 registers free.
    constexpr bool KEEP_AC = G < 16;
    uint32_t Ag[KEEP_AC ? G : 1], Cg[KEEP_AC ? G : 1];
    if constexpr (KEEP_AC) {
#pragma unroll
      for (int p = 0; p < G; ++p) {
        Ag[p] = G == 1 ? Aj : shfl_u32(Aj, p * SLOTS + slot);
        Cg[p] = G == 1 ? Cj : shfl_u32(Cj, p * SLOTS + slot);
      }
    }

    uint64_t rk = KEY_INF;          // result list: lane j < kk holds the j-th best
    uint64_t rk2 = KEY_INF;         // K2: lane j holds the (WAVE + j)-th best
    uint64_t kth = KEY_INF;         // (uniform) the list's kk-th key
    uint32_t best = 0xffffffffu;    // (uniform) best distance bits so far
    const int kk = a.keep;          // entries kept (k, or more before a re-rank)
    int evals = 0;
    int list_reads = 0;             // neighbour lists scanned by the climb
    uint32_t P = 0;                 // permutation positions consumed
    uint32_t xP = lcg.x0;           // value at position P
    uint32_t dcur = 0;
    bool climbing = false;
    const int64_t trace_base = (int64_t)qi * R.trace_stride;

    // KEEP: restart windows resumed after a climb.  A window that accepts
    // the restart of lane f has scored its positions after f too; the climb
    // leaves the permutation where it was, so the next window starts at
    // exactly those positions.  Their scores are kept (lane j of the next
    // window = lane f + 1 + j of this one) and only the positions beyond are
    // gathered; the visited probe and every decision are taken again.  It
    // pays where many wavefronts share the memory system (thousands of
    // searches per launch) and costs a lone wavefront its extra
    // instructions.
    constexpr bool REUSE = KEEP && !PART;
    // One gather-issue site after the step's branches when a step gathers
    // its rows in one pass group (fewer registers: 244 instead of 252-366
    // VGPRs for bfloat16 rows of 128 coordinates); steps of several
    // double-buffered pass groups allocate better with the issue inlined in
    // the move and window branches (with one site, 40-150 VGPRs spilled for
    // bfloat16 rows of 512 and FP8 rows of 960 coordinates; none without).
    constexpr bool ONE_ISSUE = NG == 1;
    static_assert(ONE_ISSUE || !REUSE, "kept window scores need the single issue site");
    uint32_t sd = 0xffffffffu;      // kept scores, lane view of the next window
    int nsave = 0;                  // (uniform) positions kept at the last acceptance
    int skip = 0;                   // (uniform) leading positions of this window kept

    int32_t cidL = -1;              // lane view
    uint32_t xL = 0;
    int32_t cidG[G];                // group view
    int32_t pg[G];                  // PART: partitions of the group-view candidates
    int32_t partL = -1;             // PART: partition of the lane-view candidate
    v4i xv[NB][PB][CPL];            // gathered rows, by buffer and pass in group
    v4i lv[NB][PB][LCPL];           // gathered adjacency rows
    uint32_t sv[NB][PB];            // per-row side value (FP8 scale)
    uint32_t sv2[NB][PB];           // second side value (FP8 quantized norm)

    auto window = [&]() __attribute__((always_inline)) {
      xL = (Aj * xP + Cj) & mmask;
      cidL = (P + (uint32_t)lane < a.m_mod && xL < n) ? (int32_t)xL : -1;
#pragma unroll
      for (int p = 0; p < G; ++p) {
        const uint32_t c = (uint32_t)(p * SLOTS + slot);
        uint32_t xg;
        if constexpr (KEEP_AC)
          xg = (Ag[p] * xP + Cg[p]) & mmask;
        else
          xg = shfl_u32(xL, (int)c);
        cidG[p] = (P + c < a.m_mod && xg < n) ? (int32_t)xg : -1;
      }
    };
    auto issue_group = [&](int gi, int buf) __attribute__((always_inline)) {
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        const int p = gi * PB + q;
        const bool ok = cidG[p] >= 0;
        // rows of kept positions are not gathered again (their lists are)
        const bool okr = ok && (!REUSE || p * SLOTS + slot >= skip);
        const char* row = rows + (int64_t)(okr ? cidG[p] : 0) * a.row_bytes;
#pragma unroll
        for (int pp = 0; pp < CPL; ++pp) {
          const int off = 16 * (sub + G * pp);
          if (okr && off < a.coord_bytes)
            xv[buf][q][pp] = *reinterpret_cast<const v4i*>(row + off);
          else
            xv[buf][q][pp] = v4i{0, 0, 0, 0};
        }
        if (Score::kSide) sv[buf][q] = okr ? a.side[cidG[p]] : 0u;
        if (Score::kSide2) {
          if (a.side2_off >= 0)
            sv2[buf][q] = okr ? *reinterpret_cast<const uint32_t*>(row + a.side2_off) : 0u;
          else
            sv2[buf][q] = okr ? a.side2[cidG[p]] : 0u;
        }
        if (PART) pg[p] = ok ? a.node_part[cidG[p]] : -1;
        if (LISTS) {
#pragma unroll
          for (int lc = 0; lc < LCPL; ++lc) {
            const int chunk = sub + G * lc;
            if (ok && chunk < LCH)
              lv[buf][q][lc] = *reinterpret_cast<const v4i*>(
                  a.nbr_ids + (int64_t)cidG[p] * a.k_pad + 4 * chunk);
          }
        }
      }
    };
    auto issue = [&]() __attribute__((always_inline)) {
      if (PART) partL = cidL >= 0 ? a.node_part[cidL] : -1;
      issue_group(0, 0);
    };

    // A list scan whose k candidates fit one pass is decided in the group
    // view itself ("spaced": candidate c is owned by its group's first lane,
    // c * G, or c in the MFMA layout), without moving distances to the lane
    // view.
    const bool climb_spaced = G > 1 && (a.k + SLOTS - 1) / SLOTS == 1;

    int restarts_used = 0;          // GNNS: restarts taken
    bool done = Bq <= 0 || (GNNS && a.restarts <= 0);
#ifdef KNNG_STEP_COUNTERS
    unsigned long long stc[KNNG_NUM_STEP_COUNTERS] = {};   // this search's step counters
#endif
    if (!done) {
      window();
      issue();
    }
    while (!done) {
      const bool spaced = climbing && climb_spaced;
      const int32_t cand = spaced ? cidG[0] : cidL;   // this lane's candidate
      const bool owner = !spaced || sub == 0;
      // visited probe of this lane's candidate while the gathers fly
      bool seen;
      if constexpr (FILT) {
        const int32_t cc = cand >= 0 ? cand : 0;
        const uint32_t fb = filt_bit(cc);
        const bool maybe = climbing || ((filt[fb >> 5] >> (fb & 31)) & 1u);
        seen = maybe && gbit_test(vis, cc);
      } else {
        seen = GVIS ? gbit_test(vis, cand >= 0 ? cand : 0) : bit_test(vis, cand >= 0 ? cand : 0);
      }
      const bool climb_step = climbing;
      // distances of the group-view candidates; stage their adjacency rows.
      // A list scan has at most k candidates: when they fit in fewer passes
      // than G, only those passes are computed.
      uint32_t dg[G];
      uint32_t d = 0xffffffffu;
      auto stage = [&](int p, int buf, int q) __attribute__((always_inline)) {
        const int c = p * SLOTS + slot;
        if (LISTS) {
#pragma unroll
          for (int lc = 0; lc < LCPL; ++lc) {
            const int chunk = sub + G * lc;
            if (cidG[p] >= 0 && chunk < LCH)
              *reinterpret_cast<v4i*>(lists + c * LROW + 4 * chunk) = lv[buf][q][lc];
          }
        }
      };
      auto pass = [&](int p, int buf, int q) __attribute__((always_inline)) {
        stage(p, buf, q);
        if (REUSE && (p + 1) * SLOTS <= skip) {   // every score of the pass is kept
          dg[p] = 0xffffffffu;
          return;
        }
        uint32_t dd;
        if constexpr (Score::kSide2)
          dd = sc.dist(xv[buf][q], sv[buf][q], sv2[buf][q]);
        else
          dd = sc.dist(xv[buf][q], Score::kSide ? sv[buf][q] : 0u);
        dg[p] = cidG[p] >= 0 ? dd : 0xffffffffu;
      };
      auto to_lane = [&](int p) __attribute__((always_inline)) {
        const int j = lane - p * SLOTS;
        const bool mine = j >= 0 && j < SLOTS;
        const uint32_t got = (uint32_t)shfl_i32((int)dg[p], mine ? (CM ? j : j * G) : 0);
        if (mine) d = got;
      };
      const int act = climbing ? (a.k + SLOTS - 1) / SLOTS : G;
      if (G == 1) {
        pass(0, 0, 0);
        d = dg[0];
      } else if (act == 1) {
        pass(0, 0, 0);
        if (spaced)
          d = dg[0];
        else
          to_lane(0);
      } else if (NG == 1) {
        if constexpr (Score::kBatch) {
          // every pass's scores at once: the passes' dependent chains are
          // independent of each other and interleave
#pragma unroll
          for (int p = 0; p < G; ++p) stage(p, 0, p);
          uint32_t dd[G];
          sc.dist_all(xv[0], sv2[0], dd);
#pragma unroll
          for (int p = 0; p < G; ++p) dg[p] = cidG[p] >= 0 ? dd[p] : 0xffffffffu;
        } else {
#pragma unroll
          for (int p = 0; p < G; ++p) pass(p, 0, p);
        }
#pragma unroll
        for (int p = 0; p < G; ++p) to_lane(p);
      } else {
        const int ag = (act + PB - 1) / PB;       // pass groups holding candidates
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
          if (gi < ag) {
            if (gi + 1 < ag) issue_group(gi + 1, (gi + 1) % NB);
#pragma unroll
            for (int q = 0; q < PB; ++q) pass(gi * PB + q, gi % NB, q);
          } else {
#pragma unroll
            for (int q = 0; q < PB; ++q) dg[gi * PB + q] = 0xffffffffu;
          }
        }
#pragma unroll
        for (int p = 0; p < G; ++p) to_lane(p);
      }
      if (REUSE && skip > 0 && lane < skip) d = sd;   // kept scores of a resumed window
      const bool inpart = !PART || (spaced ? pg[0] : partL) == part;
      const bool valid = owner && cand >= 0 && !seen && inpart;

      // the sequential rule on this step's candidates
      const uint64_t V = ballot(valid);
      uint64_t S;                   // the lane the sequential rule stops at
      if (!climbing) {
        // Expansion test (similarity 1/(1+d) below s_max / e).  A restart
        // that is rejected is never closer than the best so far, so a
        // candidate is tested against the best before the window, or its
        // own distance if that is smaller.
        const uint32_t bt = d < best ? d : best;
        S = GNNS ? V : ballot(valid && sc.keep(d, bt, a.e_num, a.e_den));
        if (GNNS && S) ++restarts_used;
      } else if (GNNS) {
        // steepest: the closest unvisited neighbour, if closer than current
        uint64_t m = valid ? make_key(d, cand) : KEY_INF;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) m = min_u64(m, shfl_xor_u64(m, off));
        const bool better = m != KEY_INF && key_dist(m) < dcur;
        S = better ? ballot(valid && make_key(d, cand) == m) : 0ull;
      } else {
        S = ballot(valid && d < dcur);
      }
      const int f = S ? __ffsll((long long)S) - 1 : WAVE;
      uint64_t C = (GNNS && climbing) ? V : (f < WAVE ? (V & ((2ull << f) - 1ull)) : V);
      const int rem = Bq - evals;
      bool stop = false;
      if (__popcll(C) >= rem) {
        const bool in = ((C >> lane) & 1ull) && rank_below(C) < rem;
        C = ballot(in);
        stop = true;
      }
      const bool mine = (C >> lane) & 1ull;
      const int32_t cid_now = cand;
      const uint32_t d_now = d;
#ifdef KNNG_STEP_COUNTERS
      {
        const int w = climbing ? 1 : 0;                 // this step's kind
        stc[KNNG_SC_WINDOW_STEPS + w] += 1;
        stc[KNNG_SC_WINDOW_CANDS + w] += __popcll(ballot(owner && cand >= 0));
        stc[KNNG_SC_WINDOW_VISITED + w] += __popcll(ballot(owner && cand >= 0 && seen));
        stc[KNNG_SC_WINDOW_COMMITTED + w] += __popcll(C);
        if (S && !stop) stc[climbing ? KNNG_SC_MOVES : KNNG_SC_RESTARTS_TAKEN] += 1;
        if (REUSE && !climbing)
          stc[KNNG_SC_WINDOW_KEPT] += __popcll(ballot(cand >= 0 && lane < skip));
      }
#endif

      // the next step: decide its candidates and issue their gathers first
      // (one window draw and one issue site, whichever way the step went)
      if (!stop) {
        bool draw = false;
        if (S) {
          const int32_t cur = readlane_i32(cid_now, f);
          dcur = (uint32_t)readlane_i32((int32_t)d_now, f);
          if (!climbing) {
            P += (uint32_t)f + 1u;
            xP = (lcg.a * (uint32_t)cur + lcg.c) & mmask;
            climbing = true;
            if (REUSE) {
              nsave = WAVE - 1 - f;
              sd = (uint32_t)shfl_i32((int32_t)d_now, lane + f + 1 < WAVE ? lane + f + 1 : lane);
            }
          }
          if (LISTS) {
            const int fc = spaced ? (CM ? f : f / G) : f;   // candidate index of lane f
            if (!climb_spaced) cidL = lane < a.k ? lists[fc * LROW + lane] : -1;
#pragma unroll
            for (int p = 0; p < G; ++p) {
              const int c = p * SLOTS + slot;
              cidG[p] = c < a.k ? lists[fc * LROW + c] : -1;
            }
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
          if constexpr (!ONE_ISSUE) issue();
        } else if (!climbing) {
          const uint32_t x63 = (uint32_t)readlane_i32((int32_t)xL, WAVE - 1);
          P += WAVE;
          xP = (lcg.a * x63 + lcg.c) & mmask;
          nsave = 0;
          if (P >= a.m_mod) {
            done = true;
          } else if constexpr (ONE_ISSUE) {
            draw = true;
          } else {
            window();
            issue();
          }
        } else if (GNNS && restarts_used >= a.restarts) {
          done = true;             // local maximum after the last restart
        } else {
          climbing = false;        // local maximum: restart
          if constexpr (ONE_ISSUE) {
            draw = true;
          } else {
            window();
            issue();
          }
        }
        if constexpr (ONE_ISSUE) {
          // a window drawn after a climb resumes the kept positions
          skip = draw ? nsave : 0;
          if (draw) {
            nsave = 0;
            window();
          }
          if (!done) issue();
        }
      }

      // bookkeeping of this step: visited, trace, result list, count
      if (mine) atomicOr(&vis[cid_now >> 5], 1u << (cid_now & 31));
      if (FILT && mine && climb_step) {
        const uint32_t fb = filt_bit(cid_now);
        atomicOr(&filt[fb >> 5], 1u << (fb & 31));
      }
      if (R.trace && mine) {
        const int r = rank_below(C);
        if (evals + r < R.trace_stride) R.trace[trace_base + evals + r] = cid_now;
      }
      const uint64_t key = make_key(d_now, cid_now);
      if (ballot(mine && key < kth)) {
        if (K2 && kk > WAVE) {
          wave_topk_offer_ranked2(rk, rk2, mine, key, kk, tk_c, tk_r, tk_o);
          kth = readlane_u64(rk2, kk - 1 - WAVE);
        } else {
          wave_topk_offer_ranked(rk, mine, key, kk, tk_c, tk_r, tk_o);
          kth = readlane_u64(rk, kk - 1);
        }
        best = key_dist(readlane_u64(rk, 0));
      }
      evals += __popcll(C);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (stop) break;
    }

    if constexpr (CCPL > 0) {
      float qc[CCPL][4];
      canon_load_query<CCPL>((const float*)R.qraw + (int64_t)qq * a.dim, a.dim, qc);
      const bool have = lane < kk && rk != KEY_INF;
      const int32_t cid = have ? key_id(rk) : -1;
      const uint32_t d32 = canon_dist_lanes<CCPL, CPB>(qc, a.master, a.master_stride,
                                                       a.master_chunks, cid, a.ip != 0);
      const uint64_t nk = have ? make_key(d32, cid) : KEY_INF;
      uint64_t nk2 = KEY_INF;
      bool have2 = false;
      if (K2 && kk > WAVE) {
        have2 = WAVE + lane < kk && rk2 != KEY_INF;
        const int32_t cid2 = have2 ? key_id(rk2) : -1;
        const uint32_t e32 = canon_dist_lanes<CCPL, CPB>(qc, a.master, a.master_stride,
                                                         a.master_chunks, cid2, a.ip != 0);
        nk2 = have2 ? make_key(e32, cid2) : KEY_INF;
      }
      rk = KEY_INF;
      wave_topk_offer_ranked(rk, have, nk, a.k, tk_c, tk_r, tk_o);
      if (K2 && kk > WAVE) wave_topk_offer_ranked(rk, have2, nk2, a.k, tk_c, tk_r, tk_o);
    }
    if (lane < R.out_stride) {
      const bool have = lane < a.k && rk != KEY_INF;
      R.out_ids[(int64_t)qi * R.out_stride + lane] = have ? key_id(rk) : -1;
      uint32_t dbits = have ? key_dist(rk) : a.pad_bits;
      if (R.decode) dbits = __float_as_uint(float_from_sortable(dbits));
      R.out_d[(int64_t)qi * R.out_stride + lane] = dbits;
    }
#ifdef KNNG_STEP_COUNTERS
    if (a.step_counters && lane == 0) {
      stc[KNNG_SC_SEARCHES] = 1;
      stc[KNNG_SC_EVALUATIONS] = (unsigned long long)evals;
      for (int i = 0; i < KNNG_NUM_STEP_COUNTERS; ++i) atomicAdd(&a.step_counters[i], stc[i]);
    }
#endif
    if (lane == 0) {
      if (R.out_evals) R.out_evals[qi] = evals;
      if (R.out_list_reads) R.out_list_reads[qi] = list_reads;
      if (R.trace && evals < R.trace_stride) R.trace[trace_base + evals] = -1;
    }
    __syncthreads();
  }
}

// Launch of one instantiation; LROW from the list stride (adjacency rows
// of 16, 32 or 64 ids are staged in LDS), GVIS from the caller's choice.
// `vis_lds` is the LDS of the visited set (0 when it is global).
template <class Score, int G, int CPL, int CCPL, int CPB, int PB = G, bool GNNS = false,
          bool PART = false, int KPADS = 7, bool STAGE16 = true, int WPE = 1, bool KEEP = false>
hipError_t launch_search_t(const SearchArgs& a, hipStream_t s, unsigned grid, size_t vis_lds) {
  // KPADS: the list strides this instantiation serves (1: 16, 2: 32, 4: 64).
  // STAGE16: lists of 16 ids are gathered with every candidate's row and
  // staged in LDS (a climb move then reads its list without a round trip);
  // otherwise a move loads the one list it needs.  WPE: wavefronts per SIMD
  // the register allocation is bounded for.  KEEP: kept restart-window
  // scores (k_search).
  const bool gvis = a.gvis != nullptr;
  // lists of more than 16 ids with a re-ranked reduced-precision score keep
  // up to 2 * WAVE candidates (two per lane)
  constexpr bool W2 = Score::kWide && CCPL > 0;
  constexpr int L16 = STAGE16 ? 16 : 0;
#define KNNG_SEARCH_GO(LR, GV, K2)                                                        \
  hipLaunchKernelGGL((k_search<Score, G, CPL, LR, GV, CCPL, CPB, PB, GNNS, PART, K2, WPE, KEEP>), \
                     dim3(grid), dim3(64), vis_lds + (size_t)WAVE * (LR) * 4, s, a)
  if (a.keep > 2 * WAVE || (a.keep > WAVE && !(W2 && a.k_pad > 16)))
    return hipErrorInvalidValue;
  if (a.k_pad == 16) {
    if constexpr ((KPADS & 1) != 0) {
      if (gvis) KNNG_SEARCH_GO(L16, true, false); else KNNG_SEARCH_GO(L16, false, false);
    } else {
      return hipErrorInvalidValue;
    }
  } else if (a.k_pad == 32) {
    if constexpr ((KPADS & 2) != 0) {
      if (gvis) KNNG_SEARCH_GO(32, true, W2); else KNNG_SEARCH_GO(32, false, W2);
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    if constexpr ((KPADS & 4) == 0) {
      return hipErrorInvalidValue;
    } else if constexpr (PB < G) {
      if (gvis) KNNG_SEARCH_GO(64, true, W2); else KNNG_SEARCH_GO(64, false, W2);
    } else {
      if (gvis) KNNG_SEARCH_GO(0, true, W2); else KNNG_SEARCH_GO(0, false, W2);
    }
  }
#undef KNNG_SEARCH_GO
  return hipGetLastError();
}

}  // namespace knng
