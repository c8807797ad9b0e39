// Device helpers of the online kernels: lane-group reductions, the restart
// permutation, bit sets, and the number formats of the scoring rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace knng {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// ---- sums inside groups of G consecutive lanes --------------------------------
// DPP for groups of 2 / 4 lanes (no LDS traffic), xor shuffles above.  The
// summation order is fixed: pairs at distance 1, then 2, 4, ...
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
  if (G >= 8) v += __shfl_xor(v, 4, WAVE);
  if (G >= 16) v += __shfl_xor(v, 8, WAVE);
  if (G >= 32) v += __shfl_xor(v, 16, WAVE);
  if (G >= 64) v += __shfl_xor(v, 32, WAVE);
  return v;
}
template <int G>
__device__ __forceinline__ float group_sum(float v) {
  if (G >= 2) v += __int_as_float(dpp_xor1(__float_as_int(v)));
  if (G >= 4) v += __int_as_float(dpp_xor2(__float_as_int(v)));
  if (G >= 8) v += __shfl_xor(v, 4, WAVE);
  if (G >= 16) v += __shfl_xor(v, 8, WAVE);
  if (G >= 32) v += __shfl_xor(v, 16, WAVE);
  if (G >= 64) v += __shfl_xor(v, 32, WAVE);
  return v;
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

// ---- bit sets -------------------------------------------------------------
__device__ __forceinline__ bool bit_test(const uint32_t* bits, int32_t id) {
  return (bits[id >> 5] >> (id & 31)) & 1u;
}
// Set the bit of `id`; true iff it was clear before.
__device__ __forceinline__ bool bit_set(uint32_t* bits, int32_t id) {
  uint32_t m = 1u << (id & 31);
  return (atomicOr(&bits[id >> 5], m) & m) == 0u;
}
// The same on a bit set in global memory, read at device scope (the word
// may have been set by this wavefront's own atomics, which bypass L1).
__device__ __forceinline__ bool gbit_test(const uint32_t* bits, int32_t id) {
  uint32_t w = __hip_atomic_load(bits + (id >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return (w >> (id & 31)) & 1u;
}

// ---- number formats ------------------------------------------------------------
// bfloat16 -> float: the 16 bits are the top half of the float.
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// float -> bfloat16, round to nearest even (finite inputs).
__device__ __forceinline__ uint32_t f32_to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  uint32_t lsb = (u >> 16) & 1u;
  return (u + 0x7fffu + lsb) >> 16;
}

// OCP FP8 E4M3 (1 sign, 4 exponent bits with bias 7, 3 mantissa bits; no
// infinities, 0x7f / 0xff are NaN; largest finite 448): the four codes of a
// 32-bit word (byte t = element t) -> float, by gfx950's packed conversion,
// which reads OCP E4M3 and is exact (every E4M3 value is a float; checked
// against the definition for all 254 finite codes).  The library never
// stores a NaN code (its quantizer saturates at 448).
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void e4m3x4_to_f32(uint32_t w, float (&v)[4]) {
  const v2f lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
  const v2f hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
  v[0] = lo.x;
  v[1] = lo.y;
  v[2] = hi.x;
  v[3] = hi.y;
}

// float -> OCP FP8 E4M3, round to nearest even, saturating to +-448.
__device__ __forceinline__ uint32_t f32_to_e4m3(float x) {
  uint32_t u = __float_as_uint(x);
  uint32_t s = (u >> 24) & 0x80u;
  float a = fabsf(x);
  if (!(a < 464.0f)) return s | 0x7eu;               // >= 464 rounds past 448: saturate
  if (a < 0.015625f) {                                // below 2^-6: subnormal grid 2^-9
    float q = a * 512.0f;                             // exact
    uint32_t r = (uint32_t)__builtin_rintf(q);        // nearest even
    return s | r;                                     // r <= 8 (8 = smallest normal)
  }
  uint32_t au = __float_as_uint(a);
  uint32_t e = (au >> 23) - 120u;                     // biased e4m3 exponent, 1..15
  uint32_t mant = au & 0x7fffffu;
  uint32_t keep = mant >> 20, rest = mant & 0xfffffu;
  uint32_t half = 0x80000u;
  uint32_t r = keep + ((rest > half || (rest == half && (keep & 1u))) ? 1u : 0u);
  if (r == 8u) {
    r = 0u;
    ++e;
  }
  return s | (e << 3) | r;                            // e = 15, r = 7 excluded above
}

// ---- the float32 distance of stored float distances -----------------------------
// Every float32 distance a float graph stores (lists, search results,
// proposals) is computed by this one function of (q, x), so that equal
// pairs give equal bits wherever they are evaluated.  Order of operations:
// a group of 16 lanes per pair; 16-byte chunk c (coordinates 4c .. 4c+3)
// belongs to lane c mod 16, which accumulates its chunks in ascending
// order, coordinates in ascending order, each term as one fused
// multiply-add of the squared difference; the 16 lane sums are then added
// in a butterfly over lane distances 1, 2, 4 and 8.  Coordinates past the
// dimension are zero on both sides and add exact zeros.  With m terms per
// lane (m = 4 ceil(chunks / 16)) the relative error is below (m + 4 + 1) u,
// u = 2^-24: about 7e-7 at 128 coordinates, 1.2e-6 at 960.
constexpr int CANON_G = 16;

// Canonical-layout query: lane (lane % 16) holds chunks lane % 16 + 16 t.
template <int CPL>
__device__ __forceinline__ void canon_load_query(const float* q, int dim, float (&qc)[CPL][4]) {
  const int sub = lane_id() % CANON_G;
#pragma unroll
  for (int t = 0; t < CPL; ++t) {
    const int c0 = 4 * (sub + CANON_G * t);
#pragma unroll
    for (int e = 0; e < 4; ++e) qc[t][e] = c0 + e < dim ? q[c0 + e] : 0.f;
  }
}

// Canonical distances from the query to up to 64 candidates given in lane
// view (lane c holds candidate id `cid`, -1 for none) among the rows of
// `base` (`stride` floats per row, 16-byte aligned, zero padded).  Returns
// in lane c the distance bits of its candidate (+inf bits when none).  PB
// passes of 4 candidates have their loads in flight together.  Must be
// called by the whole wavefront in uniform control flow.  With `ip` the
// same order of operations sums the products q x (one fused multiply-add
// per coordinate) and the result is the sortable key of -(q . x) (SORT_INF
// when none).
template <int CPL, int PB>
__device__ __forceinline__ uint32_t canon_dist_lanes(const float (&qc)[CPL][4], const float* base,
                                                     int64_t stride, int chunks, int32_t cid,
                                                     bool ip = false) {
  const int lane = lane_id();
  const int slot = lane / CANON_G;
  const int sub = lane % CANON_G;
  uint32_t out = ip ? SORT_INF : 0x7f800000u;
  const uint64_t any = ballot(cid >= 0);
  const int hi = any ? 64 - __clzll((long long)any) : 0;   // highest candidate lane + 1
  const int passes = (hi + 3) / 4;
  for (int p0 = 0; p0 < passes; p0 += PB) {
    int32_t cg[PB];
    v4f xv[PB][CPL];
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const int c = 4 * (p0 + pb) + slot;
      const int32_t v = shfl_i32(cid, c & 63);
      cg[pb] = (p0 + pb < passes) ? v : -1;
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        const int ch = sub + CANON_G * t;
        if (cg[pb] >= 0 && ch < chunks)
          xv[pb][t] = *reinterpret_cast<const v4f*>(base + (int64_t)cg[pb] * stride + 4 * ch);
        else
          xv[pb][t] = v4f{0.f, 0.f, 0.f, 0.f};
      }
    }
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      float s = 0.f;
      if (ip) {
#pragma unroll
        for (int t = 0; t < CPL; ++t)
#pragma unroll
          for (int e = 0; e < 4; ++e) s = __builtin_fmaf(qc[t][e], xv[pb][t][e], s);
      } else {
#pragma unroll
        for (int t = 0; t < CPL; ++t)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float d = qc[t][e] - xv[pb][t][e];
            s = __builtin_fmaf(d, d, s);
          }
      }
      s = group_sum<CANON_G>(s);
      const float got = __int_as_float(shfl_i32(__float_as_int(s), (lane % 4) * CANON_G));
      if (lane / 4 == p0 + pb && cid >= 0)
        out = ip ? sortable_from_float(-got) : __float_as_uint(got);
    }
  }
  return out;
}

}  // namespace knng
