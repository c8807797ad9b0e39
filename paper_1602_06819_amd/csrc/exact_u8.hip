// Exact k-nn by brute force on int8 MFMA (the naive method of Section 2.1:
// compute every pairwise distance, keep the k best per node).
//
// Distances of uint8 points: with rows stored as int8 (x - 128),
//   d(q, x) = |q|^2 + |x|^2 - 2 q.x
// where q.x comes from v_mfma_i32_16x16x64_i8 (exact int32 accumulation:
// |q.x| <= dim * 128^2) and the norms are precomputed at ingest.  Every
// value is an exact integer, so the result is bit-identical to the exact
// integer distance.
//
// Tiling.  A block is 4 waves; a wave owns QT tiles of 16 queries.  For a
// database tile of 16 rows, one MFMA per 64-byte slice of the rows gives a
// 16 x 16 block of dot products (A = 16 database rows, B = 16 queries);
// lane l then holds query (l % 16) against database rows 4 (l / 16) + r,
// r = 0..3.  Each lane keeps a sorted register list of its query's KM best
// keys (distance, id) over the rows it sees (a quarter of the database);
// at the end the four lanes of a query merge their lists with two bitonic
// merges over lane shuffles.  Keeping KM >= k entries is a superset of the
// top k, so the first k of the merged list are exact.
//
// Splits.  When there are few queries, blockIdx.y splits the database into
// ranges; each writes a partial list and k_split_merge merges them.
#include "common.h"
#include "internal.h"

namespace knng {

typedef int v4i __attribute__((ext_vector_type(4)));

template <int QT, int DT, int KM, int NCH>
__global__ __launch_bounds__(256) void k_exact_u8(ExactArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15;
  const int grp = lane >> 4;
  const int32_t q0 = (int32_t)(blockIdx.x * 4 + wave) * (16 * QT);
  const int split = blockIdx.y;
  const int32_t d_begin = split * a.split_len;
  int32_t d_end = d_begin + a.split_len;
  if (d_end > a.nd) d_end = a.nd;

  // query operands (B), kept in registers
  v4i bq[QT][NCH];
  int32_t qn[QT];
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
        bq[t][c] = *reinterpret_cast<const v4i*>(a.qvec + (int64_t)qc * a.row_bytes + off);
      else
        bq[t][c] = v4i{0, 0, 0, 0};
    }
  }

  uint64_t L[QT][KM];
#pragma unroll
  for (int t = 0; t < QT; ++t)
#pragma unroll
    for (int j = 0; j < KM; ++j) L[t][j] = KEY_INF;

  for (int32_t d0 = d_begin; d0 < d_end; d0 += 16 * DT) {
    v4i av[DT][NCH];
    int32_t dn[DT][4];
#pragma unroll
    for (int dt = 0; dt < DT; ++dt) {
      int32_t r = d0 + 16 * dt + col;
      int32_t rc = r < a.nd ? r : a.nd - 1;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        int off = 64 * c + 16 * grp;
        if (off < a.row_bytes)
          av[dt][c] = *reinterpret_cast<const v4i*>(a.dvec + (int64_t)rc * a.row_bytes + off);
        else
          av[dt][c] = v4i{0, 0, 0, 0};
      }
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        int32_t orow = d0 + 16 * dt + 4 * grp + rr;
        dn[dt][rr] = a.dnorm[orow < a.nd ? orow : a.nd - 1];
      }
    }
#pragma unroll
    for (int t = 0; t < QT; ++t) {
#pragma unroll
      for (int dt = 0; dt < DT; ++dt) {
        v4i acc = v4i{0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < NCH; ++c)
          acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av[dt][c], bq[t][c], acc, 0, 0, 0);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          int32_t orow = d0 + 16 * dt + 4 * grp + rr;
          int32_t dist = qn[t] + dn[dt][rr] - 2 * acc[rr];
          bool ok = orow < d_end &&
                    !(a.exclude_self && a.d_id_base + orow == a.q_id_base + qid[t]);
          uint64_t key = ok ? make_key((uint32_t)dist, a.d_id_base + orow) : KEY_INF;
          if (key < L[t][KM - 1]) reg_list_insert<KM>(L[t], key);
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
    if (a.nsplit == 1) {
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

template <int QT, int DT, int KM, int NCH>
static hipError_t launch_exact_t(const ExactArgs& a, hipStream_t s) {
  dim3 grid((unsigned)((a.nq + 64 * QT - 1) / (64 * QT)), (unsigned)a.nsplit);
  hipLaunchKernelGGL((k_exact_u8<QT, DT, KM, NCH>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int QT, int KM>
static hipError_t launch_exact_nch(const ExactArgs& a, hipStream_t s) {
  const int nch = (a.row_bytes + 63) / 64;
  switch (nch) {
    case 1: return launch_exact_t<QT, 4, KM, 1>(a, s);
    case 2: return launch_exact_t<QT, 4, KM, 2>(a, s);
    case 3:
    case 4: return launch_exact_t<QT, 2, KM, 4>(a, s);
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

}  // namespace knng
