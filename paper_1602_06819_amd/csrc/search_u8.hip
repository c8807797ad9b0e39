// iGNNS launches for int8 rows (uint8 graphs), and the format dispatch.
#include "search.h"

namespace knng {

// LDS of the visited bitset (the staged adjacency rows are added per
// instantiation by launch_search_t).
size_t search_lds_bytes(int64_t n, int k_pad, bool global_visited) {
  (void)k_pad;
  return global_visited ? 0 : (size_t)round_up((n + 31) / 32, 4) * 4;
}

// One 16-byte chunk of a row per lane for rows of up to 32 bytes (a group
// of lanes reads a whole row with one load instruction, so one instruction
// fetches 64 / G rows); rows of 33-64 bytes: 2 lanes of 2 chunks (32 rows per
// pass: a restart window takes 2 passes and fewer group reductions and
// transposes than with 4 lanes of one chunk, measured 5% faster inserts at
// d = 64); longer rows (up to 256 bytes): 2 lanes of up to 8 chunks (also
// measured faster than 4 lanes at d = 128 and 256).
static hipError_t launch_search_i8(const SearchArgs& a, hipStream_t s, unsigned grid,
                                   size_t lds) {
  const int chunks = a.row_bytes / 16;
  if (chunks <= 1) return launch_search_t<ScoreI8<1, 1>, 1, 1, 0, 1>(a, s, grid, lds);
  if (chunks <= 2) return launch_search_t<ScoreI8<2, 1>, 2, 1, 0, 1>(a, s, grid, lds);
  if (chunks <= 4) return launch_search_t<ScoreI8<2, 2>, 2, 2, 0, 1>(a, s, grid, lds);
  if (chunks <= 8) return launch_search_t<ScoreI8<2, 4>, 2, 4, 0, 1>(a, s, grid, lds);
  if (chunks <= 16) return launch_search_t<ScoreI8<2, 8>, 2, 8, 0, 1>(a, s, grid, lds);
  return hipErrorInvalidValue;
}

// The GNNS baseline on int8 rows (same shapes).
static hipError_t launch_search_i8_gnns(const SearchArgs& a, hipStream_t s, unsigned grid,
                                        size_t lds) {
  const int chunks = a.row_bytes / 16;
  if (chunks <= 1) return launch_search_t<ScoreI8<1, 1>, 1, 1, 0, 1, 1, true>(a, s, grid, lds);
  if (chunks <= 2) return launch_search_t<ScoreI8<2, 1>, 2, 1, 0, 1, 2, true>(a, s, grid, lds);
  if (chunks <= 4) return launch_search_t<ScoreI8<2, 2>, 2, 2, 0, 1, 2, true>(a, s, grid, lds);
  if (chunks <= 8) return launch_search_t<ScoreI8<2, 4>, 2, 4, 0, 1, 2, true>(a, s, grid, lds);
  if (chunks <= 16) return launch_search_t<ScoreI8<2, 8>, 2, 8, 0, 1, 2, true>(a, s, grid, lds);
  return hipErrorInvalidValue;
}

hipError_t launch_search_gnns(const SearchArgs& a0, hipStream_t s) {
  SearchArgs a = a0;
  a.m = a.rows[0].count + a.rows[1].count;
  if (a.m <= 0) return hipSuccess;
  if (a.format != ROW_I8 && a.format != ROW_F32) return hipErrorInvalidValue;
  a.vis_words = (int32_t)((a.n + 31) / 32);
  a.vis_words_pad = (int32_t)round_up(a.vis_words, 4);
  const bool gvis = a.gvis != nullptr;
  const size_t lds = search_lds_bytes(a.n, a.k_pad, gvis);
  int64_t grid = a.m < 1048576 ? a.m : 1048576;
  if (gvis && grid > a.gvis_slots) grid = a.gvis_slots;
  if (grid < 1) return hipErrorInvalidValue;
  if (a.format == ROW_F32) return launch_search_f32_gnns(a, s, (unsigned)grid, lds);
  return launch_search_i8_gnns(a, s, (unsigned)grid, lds);
}

// Partitioned search on int8 rows: rows are (query, partition) pairs.
hipError_t launch_search_part(const SearchArgs& a0, hipStream_t s) {
  SearchArgs a = a0;
  a.m = a.rows[0].count + a.rows[1].count;
  if (a.m <= 0) return hipSuccess;
  if ((a.format != ROW_I8 && a.format != ROW_F32) || a.nparts < 1 || !a.node_part ||
      !a.part_budget)
    return hipErrorInvalidValue;
  a.vis_words = (int32_t)((a.n + 31) / 32);
  a.vis_words_pad = (int32_t)round_up(a.vis_words, 4);
  const bool gvis = a.gvis != nullptr;
  const size_t lds = search_lds_bytes(a.n, a.k_pad, gvis);
  int64_t grid = a.m < 1048576 ? a.m : 1048576;
  if (gvis && grid > a.gvis_slots) grid = a.gvis_slots;
  if (grid < 1) return hipErrorInvalidValue;
  const unsigned gr = (unsigned)grid;
  if (a.format == ROW_F32) return launch_search_f32_part(a, s, gr, lds);
  const int chunks = a.row_bytes / 16;
  if (chunks <= 1) return launch_search_t<ScoreI8<1, 1>, 1, 1, 0, 1, 1, false, true>(a, s, gr, lds);
  if (chunks <= 2) return launch_search_t<ScoreI8<2, 1>, 2, 1, 0, 1, 2, false, true>(a, s, gr, lds);
  if (chunks <= 4) return launch_search_t<ScoreI8<2, 2>, 2, 2, 0, 1, 2, false, true>(a, s, gr, lds);
  if (chunks <= 8) return launch_search_t<ScoreI8<2, 4>, 2, 4, 0, 1, 2, false, true>(a, s, gr, lds);
  if (chunks <= 16) return launch_search_t<ScoreI8<2, 8>, 2, 8, 0, 1, 2, false, true>(a, s, gr, lds);
  return hipErrorInvalidValue;
}

hipError_t launch_search(const SearchArgs& a0, hipStream_t s) {
  SearchArgs a = a0;
  a.m = a.rows[0].count + a.rows[1].count;
  if (a.m <= 0) return hipSuccess;
  a.vis_words = (int32_t)((a.n + 31) / 32);
  a.vis_words_pad = (int32_t)round_up(a.vis_words, 4);
  const bool gvis = a.gvis != nullptr;
  const size_t lds = search_lds_bytes(a.n, a.k_pad, gvis);
  int64_t grid = a.m < 1048576 ? a.m : 1048576;
  if (gvis && grid > a.gvis_slots) grid = a.gvis_slots;
  if (grid < 1) return hipErrorInvalidValue;
  switch (a.format) {
    case ROW_I8: return launch_search_i8(a, s, (unsigned)grid, lds);
    case ROW_BF16: return launch_search_bf16(a, s, (unsigned)grid, lds);
    case ROW_FP8: return launch_search_fp8(a, s, (unsigned)grid, lds);
    case ROW_F32: return launch_search_f32(a, s, (unsigned)grid, lds);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace knng
