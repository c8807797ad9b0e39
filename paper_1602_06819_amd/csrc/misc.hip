// Ingest and small data-movement kernels.
//
// Ingest of uint8 points: a coordinate x in [0, 255] is stored as the int8
// value x - 128.  Squared Euclidean distance is invariant under a common
// shift, so distances computed on the shifted rows are the exact integer
// distances of the original points, and the rows feed int8 dot-product and
// int8 MFMA instructions directly.  Rows are zero padded to row_bytes (a
// multiple of 16); padding contributes nothing to any distance.  The row's
// squared norm (an int32: at most 4096 * 128^2) is stored beside it.
//
// Ingest of float32 points (normalized to unit length first for the cosine
// metric): the float32 row itself (zero padded to a multiple of 4
// coordinates: the rows of the stored float distances), its
// squared norm (for the exact graph's expansion), and the scoring row of
// the search: bfloat16 by round-to-nearest-even, or FP8 E4M3 codes
// RNE(x / s) with one scale s = max |x| / 448 per row (s = 0 for a zero
// row, whose codes are then all zero).
#include "common.h"
#include "device.h"
#include "internal.h"

namespace knng {

// One wave per row; each lane converts 4 coordinates at a time.
__global__ __launch_bounds__(256) void k_ingest_u8(IngestArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= a.m) return;
  const uint8_t* src = a.x + row * a.dim;
  int8_t* dst = a.dst + row * a.row_bytes;
  int acc = 0;
  for (int c = lane * 4; c < a.row_bytes; c += 256) {
    int packed = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      int j = c + t;
      int v = (j < a.dim) ? ((int)src[j] - 128) : 0;
      packed |= (v & 0xff) << (8 * t);
    }
    *reinterpret_cast<int*>(dst + c) = packed;
    acc = __builtin_amdgcn_sdot4(packed, packed, acc, false);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) a.norms[row] = acc;
}

hipError_t launch_ingest_u8(const IngestArgs& a, hipStream_t s) {
  if (a.m <= 0) return hipSuccess;
  dim3 grid((unsigned)((a.m + 3) / 4));
  hipLaunchKernelGGL(k_ingest_u8, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// One wave per row; lane j takes coordinates j, j + 64, ...  Sums are taken
// per lane in ascending coordinate order and then over lanes in an xor tree,
// so a row's values depend on the row only.  With `cosine` the row is first
// divided by its Euclidean norm (a zero row stays zero), and every stored
// value derives from the normalized row; with `qout` only the normalized
// row is written, [m][dim], for the queries of a search.
__device__ __forceinline__ float wave_sum_sq(const float* src, int dim, int lane) {
  float s = 0.f;
  for (int j = lane; j < dim; j += WAVE) s = __builtin_fmaf(src[j], src[j], s);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, WAVE);
  return s;
}

__global__ __launch_bounds__(256) void k_ingest_f32(IngestF32Args a) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= a.m) return;                          // uniform per wavefront
  const float* src = a.x + row * a.dim;
  float div = 1.f;
  if (a.cosine) {
    const float len = __builtin_sqrtf(wave_sum_sq(src, a.dim, lane));
    div = len > 0.f ? len : 1.f;
  }
  auto value = [&](int j) { return a.cosine ? src[j] / div : src[j]; };
  if (a.qout) {
    float* qrow = a.qout + row * a.dim;
    for (int j = lane; j < a.dim; j += WAVE) qrow[j] = value(j);
    return;
  }
  float* mrow = a.master + row * a.stride;
  float nrm = 0.f, mx = 0.f;
  for (int j = lane; j < a.stride; j += WAVE) {
    const float v = j < a.dim ? value(j) : 0.f;
    mrow[j] = v;
    nrm = __builtin_fmaf(v, v, nrm);
    mx = fmaxf(mx, fabsf(v));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    nrm += __shfl_xor(nrm, off, WAVE);
    mx = fmaxf(mx, __shfl_xor(mx, off, WAVE));
  }
  if (lane == 0) a.norms[row] = nrm;
  if (a.format == ROW_BF16) {
    uint16_t* brow = reinterpret_cast<uint16_t*>(a.score + row * a.row_bytes);
    float qn = 0.f;                                // sum of the stored values squared
    for (int j = lane; j < a.coord_bytes / 2; j += WAVE) {
      const uint32_t h = j < a.dim ? f32_to_bf16(value(j)) : 0u;
      brow[j] = (uint16_t)h;
      const float v = bf16_lo(h);
      qn = __builtin_fmaf(v, v, qn);
    }
    if (a.norm_off >= 0) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) qn += __shfl_xor(qn, off, WAVE);
      uint32_t* tail = reinterpret_cast<uint32_t*>(a.score + row * a.row_bytes + a.norm_off);
      const int words = (a.row_bytes - a.norm_off) / 4;
      if (lane < words) tail[lane] = lane == 0 ? __float_as_uint(qn) : 0u;
    }
  } else if (a.format == ROW_FP8) {
    const float scale = mx / 448.f;
    uint8_t* frow = reinterpret_cast<uint8_t*>(a.score + row * a.row_bytes);
    float qn = 0.f;                                // sum of the decoded codes squared
    for (int j = lane; j < a.row_bytes; j += WAVE) {
      const uint32_t c = (j < a.dim && scale > 0.f) ? f32_to_e4m3(value(j) / scale) : 0u;
      frow[j] = (uint8_t)c;
      float v[4];
      e4m3x4_to_f32(c, v);
      qn = __builtin_fmaf(v[0], v[0], qn);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) qn += __shfl_xor(qn, off, WAVE);
    if (lane == 0) {
      a.scale[row] = scale;
      a.qnorm[row] = scale * scale * qn;
    }
  }
}

hipError_t launch_ingest_f32(const IngestF32Args& a, hipStream_t s) {
  if (a.m <= 0) return hipSuccess;
  dim3 grid((unsigned)((a.m + 3) / 4));
  hipLaunchKernelGGL(k_ingest_f32, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

// Copy k entries per row between list arrays of different strides; entries
// k .. dst_stride-1 of the destination are set to padding.  An id outside
// [0, id_limit) becomes a padding entry, so lists supplied by a caller can
// never make a kernel read outside the graph.
// `mode` 1 turns float32 distances into sortable keys (lists supplied to the
// library for the inner-product metric), 2 turns keys back into float32
// distances (lists read out); 0 copies the bits.  `pad` is the stored
// padding value (decoded like the entries in mode 2).
__global__ void k_copy_lists(const int32_t* src_ids, const int32_t* src_d, int src_stride,
                             int32_t* dst_ids, int32_t* dst_d, int dst_stride, int64_t rows,
                             int k, int64_t id_limit, int32_t pad, int mode) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = rows * dst_stride;
  if (i >= total) return;
  int64_t r = i / dst_stride;
  int j = (int)(i - r * dst_stride);
  if (j < k) {
    int32_t id = src_ids ? src_ids[r * src_stride + j] : -1;
    bool ok = id >= 0 && (int64_t)id < id_limit;
    if (dst_ids) dst_ids[i] = ok ? id : -1;
    if (dst_d) {
      int32_t v = pad;
      if (ok && src_d) {
        v = src_d[r * src_stride + j];
        if (mode == 1) v = (int32_t)sortable_from_float(__int_as_float(v));
      }
      // mode 2 decodes stored keys, the padding included
      if (mode == 2) v = __float_as_int(float_from_sortable((uint32_t)v));
      dst_d[i] = v;
    }
  } else {
    if (dst_ids) dst_ids[i] = -1;
    if (dst_d) dst_d[i] = mode == 2 ? __float_as_int(float_from_sortable((uint32_t)pad)) : pad;
  }
}

hipError_t launch_copy_lists(const int32_t* src_ids, const int32_t* src_d, int src_stride,
                             int32_t* dst_ids, int32_t* dst_d, int dst_stride, int64_t rows,
                             int k, int64_t id_limit, int32_t pad, hipStream_t s, int mode) {
  int64_t total = rows * dst_stride;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_lists, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     src_ids, src_d, src_stride, dst_ids, dst_d, dst_stride, rows, k, id_limit,
                     pad, mode);
  return hipGetLastError();
}

// int8 rows back to uint8 points (x + 128), dropping the padding.
__global__ void k_export_u8(const int8_t* vec, int row_bytes, int dim, int64_t rows,
                            uint8_t* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * dim) return;
  int64_t r = i / dim;
  int j = (int)(i - r * dim);
  out[i] = (uint8_t)((int)vec[r * row_bytes + j] + 128);
}

hipError_t launch_export_u8(const int8_t* vec, int row_bytes, int dim, int64_t rows,
                            uint8_t* out, hipStream_t s) {
  int64_t total = rows * dim;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_export_u8, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, vec,
                     row_bytes, dim, rows, out);
  return hipGetLastError();
}

// float32 rows (stride floats) back to points of dim coordinates.
__global__ void k_export_f32(const float* rows, int stride, int dim, int64_t count, float* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count * dim) return;
  int64_t r = i / dim;
  int j = (int)(i - r * dim);
  out[i] = rows[r * stride + j];
}

hipError_t launch_export_f32(const float* rows, int stride, int dim, int64_t count, float* out,
                             hipStream_t s) {
  int64_t total = count * dim;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_export_f32, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, rows,
                     stride, dim, count, out);
  return hipGetLastError();
}

}  // namespace knng
