// Exact k-nn by brute force on MFMA (the naive method of Section 2.1:
// compute every pairwise distance, keep the k best per node).
//
// uint8 points, rows stored as int8 (x - 128):
//   d(q, x) = |q|^2 + |x|^2 - 2 q.x
// with q.x from v_mfma_i32_16x16x64_i8 (exact int32 accumulation:
// |q.x| <= dim * 128^2) and the norms precomputed at ingest.  Every value
// is an exact integer, so the result is bit-identical to the exact
// integer distance.
//
// float32 points: the same expansion with q.x from v_mfma_f32_16x16x4_f32
// (for the inner-product metric, -(q.x) itself as a sortable key)
// selects KM >= k candidates per node (clamped at zero); k_rerank_f32 then
// computes the stored float32 distance of each candidate and keeps the k
// best by it.  The expansion's rounding error (a few units in the last
// place of |q|^2 + |x|^2) is far below the gaps that KM - k spare
// candidates cover on the data this library targets; the parity tests
// compare against the float64 exact graph.
//
// Tiling.  A block is 4 waves; a wave owns QT tiles of 16 queries.  For a
// database tile of 16 rows, the MFMAs of one 64-byte slice of the rows
// give a 16 x 16 block of dot products (A = 16 database rows, B = 16
// queries); lane l then holds query (l % 16) against database rows
// 4 (l / 16) + r, r = 0..3.  A float32 slice is 16 coordinates: lane l
// loads coordinates 4 (l / 16) .. +3 of it and feeds component t to the
// t-th of four MFMAs, the same permutation on both operands, so the four
// MFMAs sum the slice's products.  Each lane keeps a sorted register list
// of its query's KM best keys (distance bits, id) over the rows it sees (a
// quarter of the database); at the end the four lanes of a query merge
// their lists with two bitonic merges over lane shuffles.  KM >= k entries
// are a superset of the top k.
//
// Selection (uint8).  A candidate whose distance is above the lane's list
// end cannot enter; the few that can are queued in LDS while a query
// tile's 16-row blocks are scored, then inserted: every lane takes its
// queued keys in order, so the wavefront runs as many insertions as the
// longest queue rather than one for every position where some lane had a
// candidate.  The kept set is the KM smallest keys either way.
//
// Splits (uint8).  When there are few queries, blockIdx.y splits the
// database into ranges; each writes a partial list and k_split_merge
// merges them.
#include <type_traits>

#include "common.h"
#include "device.h"
#include "internal.h"

namespace knng {

// Insert `cand` (< L[KM - 1]) into the ascending list L: every slot is
// compared with the old list at once (the comparisons are monotone in the
// slot), then each slot takes its own key, its left neighbour's or cand.
template <int KM>
__device__ __forceinline__ void reg_list_place(uint64_t (&L)[KM], uint64_t cand) {
  bool c[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) c[j] = cand < L[j];
#pragma unroll
  for (int j = KM - 1; j >= 1; --j) L[j] = c[j - 1] ? L[j - 1] : (c[j] ? cand : L[j]);
  L[0] = c[0] ? cand : L[0];
}

template <bool F32, int QT, int DT, int KM, int NCH>
__global__ __launch_bounds__(256, (!F32 && KM == 16 && NCH == 1) ? 3 : 1) void k_exact(ExactArgs a) {
  typedef typename std::conditional<F32, v4f, v4i>::type vec4;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15;
  const int grp = lane >> 4;
  const int32_t q0 = (int32_t)(blockIdx.x * 4 + wave) * (16 * QT);
  const int split = blockIdx.y;
  const int32_t d_begin = split * a.split_len;
  int32_t d_end = d_begin + a.split_len;
  if (d_end > a.nd) d_end = a.nd;
  const char* qrows = (const char*)a.qvec;
  const char* drows = (const char*)a.dvec;
  // uint8: queued keys of one query tile, slot-major (slot * 256 + thread)
  constexpr int NQ = F32 ? 1 : 4 * DT;
  __shared__ uint64_t queue[NQ * 256];

  // query operands (B), kept in registers
  vec4 bq[QT][NCH];
  uint32_t qn[QT];
  int32_t qid[QT];
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    int32_t q = q0 + 16 * t + col;
    qid[t] = q;
    int32_t qc = q < a.nq ? q : a.nq - 1;
    qn[t] = a.qnorm[qc];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      int off = 64 * c + 16 * grp;
      if (off < a.row_bytes)
        bq[t][c] = *reinterpret_cast<const vec4*>(qrows + (int64_t)qc * a.row_bytes + off);
      else
        bq[t][c] = vec4{0, 0, 0, 0};
    }
  }

  uint64_t L[QT][KM];
  // uint8 screen: a row can enter only if its distance |q|^2 + (|x|^2 - 2 q.x)
  // is at most the list end's, so the per-row part |x|^2 - 2 q.x is compared
  // with thq = min(list end, SCREEN_CAP) - |q|^2 before anything else is
  // computed.  Every uint8 distance is below 256 * 255^2 < SCREEN_CAP; rows
  // outside the tile range take the norm FAR_NORM, whose per-row part
  // (|2 q.x| <= 2 * 256 * 128^2) stays above any thq.
  constexpr int32_t SCREEN_CAP = 1 << 29, FAR_NORM = 1 << 30;
  int32_t thq[QT];
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    thq[t] = SCREEN_CAP - (int32_t)qn[t];
#pragma unroll
    for (int j = 0; j < KM; ++j) L[t][j] = KEY_INF;
  }

  for (int32_t d0 = d_begin; d0 < d_end; d0 += 16 * DT) {
    vec4 av[DT][NCH];
    uint32_t dn[DT][4];
#pragma unroll
    for (int dt = 0; dt < DT; ++dt) {
      int32_t r = d0 + 16 * dt + col;
      int32_t rc = r < a.nd ? r : a.nd - 1;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        int off = 64 * c + 16 * grp;
        if (off < a.row_bytes)
          av[dt][c] = *reinterpret_cast<const vec4*>(drows + (int64_t)rc * a.row_bytes + off);
        else
          av[dt][c] = vec4{0, 0, 0, 0};
      }
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        int32_t orow = d0 + 16 * dt + 4 * grp + rr;
        dn[dt][rr] = a.dnorm[orow < a.nd ? orow : a.nd - 1];
      }
    }
    if constexpr (!F32) {
      if (d0 + 16 * DT > d_end) {   // the range's last tile (wave-uniform)
#pragma unroll
        for (int dt = 0; dt < DT; ++dt)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr)
            if (d0 + 16 * dt + 4 * grp + rr >= d_end) dn[dt][rr] = (uint32_t)FAR_NORM;
      }
    }
#pragma unroll
    for (int t = 0; t < QT; ++t) {
      int nq = 0;                   // uint8: keys queued for this query tile
      if constexpr (F32) {
#pragma unroll
        for (int dt = 0; dt < DT; ++dt) {
          uint32_t dist[4];
          v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e)
              acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[dt][c][e], bq[t][c][e], acc, 0, 0, 0);
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            if (a.ip) {
              dist[rr] = sortable_from_float(-acc[rr]);
            } else {
              float v = __uint_as_float(qn[t]) + __uint_as_float(dn[dt][rr]) - 2.f * acc[rr];
              dist[rr] = __float_as_uint(v > 0.f ? v : 0.f);
            }
          }
          // (no screen: on the float32 tiles the branch costs more than it
          // saves, measured)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int32_t orow = d0 + 16 * dt + 4 * grp + rr;
            bool ok = orow < d_end &&
                      !(a.exclude_self && a.d_id_base + orow == a.q_id_base + qid[t]);
            uint64_t key = ok ? make_key(dist[rr], a.d_id_base + orow) : KEY_INF;
            if (key < L[t][KM - 1]) reg_list_insert<KM>(L[t], key);
          }
        }
      } else {
        // every block's MFMAs first, so no result is read right after issue
        v4i acc[DT];
#pragma unroll
        for (int dt = 0; dt < DT; ++dt) {
          acc[dt] = v4i{0, 0, 0, 0};
#pragma unroll
          for (int c = 0; c < NCH; ++c)
            acc[dt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av[dt][c], bq[t][c], acc[dt], 0, 0, 0);
        }
#pragma unroll
        for (int dt = 0; dt < DT; ++dt) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int32_t part = (int32_t)dn[dt][rr] - 2 * acc[dt][rr];
            if (part <= thq[t]) {
              const int32_t orow = d0 + 16 * dt + 4 * grp + rr;
              if (!(a.exclude_self && a.d_id_base + orow == a.q_id_base + qid[t])) {
                queue[nq * 256 + threadIdx.x] =
                    make_key((uint32_t)((int32_t)qn[t] + part), a.d_id_base + orow);
                ++nq;
              }
            }
          }
        }
      }
      if constexpr (!F32) {
        // the queue in arrival order (nq <= 4 DT slots)
        for (int r = 0; r < nq; ++r) {
          const uint64_t key = queue[r * 256 + threadIdx.x];
          if (key < L[t][KM - 1]) {
            reg_list_place<KM>(L[t], key);
            const uint32_t e = key_dist(L[t][KM - 1]);
            thq[t] = (e < (uint32_t)SCREEN_CAP ? (int32_t)e : SCREEN_CAP) - (int32_t)qn[t];
          }
        }
      }
    }
  }

#pragma unroll
  for (int t = 0; t < QT; ++t) {
    reg_list_merge_xor<KM>(L[t], 16);
    reg_list_merge_xor<KM>(L[t], 32);
  }
  if (grp != 0) return;
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    int32_t q = qid[t];
    if (q >= a.nq) continue;
    if (a.cand) {
      uint64_t* dst = a.cand + (int64_t)q * KM;
#pragma unroll
      for (int j = 0; j < KM; ++j) dst[j] = L[t][j];
    } else if (a.nsplit == 1) {
#pragma unroll
      for (int j = 0; j < KM; ++j) {
        if (j < a.out_stride) {
          bool have = j < a.k && L[t][j] != KEY_INF;
          a.out_ids[(int64_t)q * a.out_stride + j] = have ? key_id(L[t][j]) : -1;
          a.out_d[(int64_t)q * a.out_stride + j] =
              have ? (int32_t)key_dist(L[t][j]) : DIST_PAD_I32;
        }
      }
    } else {
      uint64_t* dst = a.partial + ((int64_t)split * a.nq + q) * KM;
#pragma unroll
      for (int j = 0; j < KM; ++j) dst[j] = L[t][j];
    }
  }
}

// float32 rows longer than 16 slices (dimension above 256): the same tiles
// with the coordinates in blocks of NCH 64-byte slices; the query operands
// of each block are re-read per database tile (L1/L2 hits) and the products
// accumulate across blocks.
template <int DT, int KM, int NCH>
__global__ __launch_bounds__(256) void k_exact_f32_long(ExactArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15;
  const int grp = lane >> 4;
  const int32_t q = (int32_t)(blockIdx.x * 4 + wave) * 16 + col;
  const int32_t qc = q < a.nq ? q : a.nq - 1;
  const float* qrow = (const float*)a.qvec + (int64_t)qc * (a.row_bytes / 4);
  const float qn = __uint_as_float(a.qnorm[qc]);
  const int nkb = (a.row_bytes + 64 * NCH - 1) / (64 * NCH);
  uint64_t L[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) L[j] = KEY_INF;

  for (int32_t d0 = 0; d0 < a.nd; d0 += 16 * DT) {
    v4f acc[DT];
#pragma unroll
    for (int dt = 0; dt < DT; ++dt) acc[dt] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int kb = 0; kb < nkb; ++kb) {
      v4f bq[NCH];
      v4f av[DT][NCH];
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int off = 64 * (kb * NCH + c) + 16 * grp;
        bq[c] = off < a.row_bytes ? *reinterpret_cast<const v4f*>((const char*)qrow + off)
                                  : v4f{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int dt = 0; dt < DT; ++dt) {
        const int32_t r = d0 + 16 * dt + col;
        const int32_t rc = r < a.nd ? r : a.nd - 1;
        const char* drow = (const char*)a.dvec + (int64_t)rc * a.row_bytes;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const int off = 64 * (kb * NCH + c) + 16 * grp;
          av[dt][c] = off < a.row_bytes ? *reinterpret_cast<const v4f*>(drow + off)
                                        : v4f{0.f, 0.f, 0.f, 0.f};
        }
      }
#pragma unroll
      for (int dt = 0; dt < DT; ++dt)
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            acc[dt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[dt][c][e], bq[c][e], acc[dt], 0, 0, 0);
    }
#pragma unroll
    for (int dt = 0; dt < DT; ++dt) {
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int32_t orow = d0 + 16 * dt + 4 * grp + rr;
        const int32_t on = orow < a.nd ? orow : a.nd - 1;
        const float v = qn + __uint_as_float(a.dnorm[on]) - 2.f * acc[dt][rr];
        const uint32_t dist = a.ip ? sortable_from_float(-acc[dt][rr])
                                   : __float_as_uint(v > 0.f ? v : 0.f);
        const bool ok = orow < a.nd &&
                        !(a.exclude_self && a.d_id_base + orow == a.q_id_base + q);
        const uint64_t key = ok ? make_key(dist, a.d_id_base + orow) : KEY_INF;
        if (key < L[KM - 1]) reg_list_insert<KM>(L, key);
      }
    }
  }
  reg_list_merge_xor<KM>(L, 16);
  reg_list_merge_xor<KM>(L, 32);
  if (grp != 0 || q >= a.nq) return;
  uint64_t* dst = a.cand + (int64_t)q * KM;
#pragma unroll
  for (int j = 0; j < KM; ++j) dst[j] = L[j];
}

// float32 re-rank of the candidate lists: one wavefront per query; lane
// j < km takes candidate j, computes the stored float32 distance, and the
// k best by (distance, id) are written.
template <int CCPL, int CPB>
__global__ __launch_bounds__(64) void k_rerank_f32(RerankArgs a) {
  __shared__ uint64_t tk_c[WAVE], tk_r[WAVE], tk_o[WAVE];
  const int lane = threadIdx.x;
  const int32_t q = blockIdx.x;
  if (q >= a.nq) return;
  float qc[CCPL][4];
  canon_load_query<CCPL>(a.rows + (int64_t)(a.q_id_base + q) * a.stride, a.dim, qc);
  const uint64_t ck = lane < a.km ? a.cand[(int64_t)q * a.km + lane] : KEY_INF;
  const bool have = ck != KEY_INF;
  const int32_t cid = have ? key_id(ck) : -1;
  const uint32_t d32 =
      canon_dist_lanes<CCPL, CPB>(qc, a.rows, a.stride, a.stride / 4, cid, a.ip != 0);
  uint64_t rk = KEY_INF;
  wave_topk_offer_ranked(rk, have, have ? make_key(d32, cid) : KEY_INF, a.k, tk_c, tk_r, tk_o);
  if (lane < a.out_stride) {
    const bool ok = lane < a.k && rk != KEY_INF;
    const int32_t pad = a.ip ? (int32_t)SORT_INF : (int32_t)0x7f800000;
    a.out_ids[(int64_t)q * a.out_stride + lane] = ok ? key_id(rk) : -1;
    a.out_d[(int64_t)q * a.out_stride + lane] = ok ? (int32_t)key_dist(rk) : pad;
  }
}

// Merge nsplit sorted partial lists of km keys per query: one wave per
// query, lane s follows list s; k rounds of a wave-wide minimum.
__global__ __launch_bounds__(64) void k_split_merge(const uint64_t* partial, int32_t nq,
                                                     int32_t nsplit, int km, int k,
                                                     int32_t* out_ids, int32_t* out_d,
                                                     int out_stride) {
  const int lane = threadIdx.x;
  const int32_t q = blockIdx.x;
  if (q >= nq) return;
  int h = 0;
  const uint64_t* mine = partial + ((int64_t)lane * nq + q) * km;
  for (int j = 0; j < out_stride; ++j) {
    uint64_t head = (lane < nsplit && h < km) ? mine[h] : KEY_INF;
    uint64_t m = head;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = min_u64(m, shfl_xor_u64(m, off));
    if (j < k && m != KEY_INF) {
      if (head == m) ++h;
      if (lane == 0) {
        out_ids[(int64_t)q * out_stride + j] = key_id(m);
        out_d[(int64_t)q * out_stride + j] = (int32_t)key_dist(m);
      }
    } else if (lane == 0) {
      out_ids[(int64_t)q * out_stride + j] = -1;
      out_d[(int64_t)q * out_stride + j] = DIST_PAD_I32;
    }
  }
}

hipError_t launch_split_merge(const uint64_t* partial, int32_t nq, int32_t nsplit, int k,
                              int32_t* out_ids, int32_t* out_d, int out_stride, hipStream_t s) {
  if (nsplit > 64) return hipErrorInvalidValue;
  int km = out_stride;  // partial lists are written with KM == list stride
  hipLaunchKernelGGL(k_split_merge, dim3((unsigned)nq), dim3(64), 0, s, partial, nq, nsplit, km,
                     k, out_ids, out_d, out_stride);
  return hipGetLastError();
}

template <bool F32, int QT, int DT, int KM, int NCH>
static hipError_t launch_exact_t(const ExactArgs& a, hipStream_t s) {
  dim3 grid((unsigned)((a.nq + 64 * QT - 1) / (64 * QT)), (unsigned)a.nsplit);
  hipLaunchKernelGGL((k_exact<F32, QT, DT, KM, NCH>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int QT, int KM>
static hipError_t launch_exact_nch(const ExactArgs& a, hipStream_t s) {
  const int nch = (a.row_bytes + 63) / 64;
  switch (nch) {
    case 1: return launch_exact_t<false, QT, 4, KM, 1>(a, s);
    case 2: return launch_exact_t<false, QT, 4, KM, 2>(a, s);
    case 3:
    case 4: return launch_exact_t<false, QT, 2, KM, 4>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_exact_u8(const ExactArgs& a, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  switch (a.out_stride) {
    case 16: return launch_exact_nch<2, 16>(a, s);
    case 32: return launch_exact_nch<2, 32>(a, s);
    case 64: return launch_exact_nch<1, 64>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// float32 rows of row_bytes (a multiple of 16): 64-byte slices in
// registers; km candidates per query (32 or 64) into a.cand.
template <int KM>
static hipError_t launch_exact_f32_km(const ExactArgs& a, hipStream_t s) {
  const int nch = (a.row_bytes + 63) / 64;
  constexpr int QT = KM == 32 ? 2 : 1;
  if (nch <= 1) return launch_exact_t<true, QT, 4, KM, 1>(a, s);
  if (nch <= 2) return launch_exact_t<true, QT, 4, KM, 2>(a, s);
  if (nch <= 4) return launch_exact_t<true, QT, 2, KM, 4>(a, s);
  // 96 coordinates: 6 slices, not 8 with two of zeros
  if (nch <= 6) return launch_exact_t<true, 1, 2, KM, 6>(a, s);
  if (nch <= 8) return launch_exact_t<true, 1, 2, KM, 8>(a, s);
  if (nch <= 16) return launch_exact_t<true, 1, 1, KM, 16>(a, s);
  dim3 grid((unsigned)((a.nq + 63) / 64));
  hipLaunchKernelGGL((k_exact_f32_long<2, KM, 8>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_exact_f32(const ExactArgs& a, int km, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  if (!a.cand || a.nsplit != 1) return hipErrorInvalidValue;
  if (km == 32) return launch_exact_f32_km<32>(a, s);
  if (km == 64) return launch_exact_f32_km<64>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_rerank_f32(const RerankArgs& a, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  const int chunks = a.stride / 4;
  dim3 grid((unsigned)a.nq);
#define KNNG_RERANK_GO(C, P) hipLaunchKernelGGL((k_rerank_f32<C, P>), grid, dim3(64), 0, s, a)
  if (chunks <= 16) KNNG_RERANK_GO(1, 8);
  else if (chunks <= 32) KNNG_RERANK_GO(2, 4);
  else if (chunks <= 64) KNNG_RERANK_GO(4, 2);
  else if (chunks <= 128) KNNG_RERANK_GO(8, 1);
  else if (chunks <= 256) KNNG_RERANK_GO(16, 1);
  else return hipErrorInvalidValue;
#undef KNNG_RERANK_GO
  return hipGetLastError();
}

// Each row of (ids, d) becomes the first k of itself and the sorted row of
// (tids, td), by (distance, id): one wavefront per row, every entry placed
// at its rank in the union (its index plus the entries of the other row
// before it; ids are distinct, so keys never tie).
__global__ __launch_bounds__(64) void k_merge_lists(int32_t* ids, int32_t* d, const int32_t* tids,
                                                    const int32_t* td, int k_pad, int k,
                                                    int64_t count, int32_t pad) {
  const int lane = threadIdx.x;
  for (int64_t r = blockIdx.x; r < count; r += gridDim.x) {
    const int64_t base = r * k_pad;
    const int32_t ia = lane < k ? ids[base + lane] : -1;
    const int32_t ib = lane < k ? tids[base + lane] : -1;
    const uint64_t ka = ia >= 0 ? make_key((uint32_t)d[base + lane], ia) : KEY_INF;
    const uint64_t kb = ib >= 0 ? make_key((uint32_t)td[base + lane], ib) : KEY_INF;
    int ra = lane, rb = lane;
    for (int t = 0; t < k; ++t) {
      const uint64_t oa = shfl_u64(ka, t);
      const uint64_t ob = shfl_u64(kb, t);
      rb += oa < kb ? 1 : 0;
      ra += ob < ka ? 1 : 0;
    }
    __builtin_amdgcn_wave_barrier();
    if (ka != KEY_INF && ra < k) {
      ids[base + ra] = key_id(ka);
      d[base + ra] = (int32_t)key_dist(ka);
    }
    if (kb != KEY_INF && rb < k) {
      ids[base + rb] = key_id(kb);
      d[base + rb] = (int32_t)key_dist(kb);
    }
    // entries past the union's length become padding
    const int total = __popcll(__ballot(ka != KEY_INF)) + __popcll(__ballot(kb != KEY_INF));
    if (lane < k && lane >= total) {
      ids[base + lane] = -1;
      d[base + lane] = pad;
    }
  }
}

hipError_t launch_merge_lists(int32_t* ids, int32_t* d, const int32_t* tids, const int32_t* td,
                              int k_pad, int k, int64_t count, int32_t pad, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t grid = count < 65536 ? count : 65536;
  hipLaunchKernelGGL(k_merge_lists, dim3((unsigned)grid), dim3(64), 0, s, ids, d, tids, td, k_pad,
                     k, count, pad);
  return hipGetLastError();
}

}  // namespace knng
