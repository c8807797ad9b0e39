// iGNNS launches for float graphs with bfloat16 scoring rows, then the
// float32 re-rank of the kept candidates.  Row shapes by dimension (16-byte
// chunks of a scoring row; groups of G lanes read one row; CPL chunks per
// lane):
//   dim <= 64     8 chunks  G 4, CPL 2 (k <= 16) or G 2, CPL 4
//   dim <= 96    12 chunks  G 4, CPL 3 (k <= 16)
//   dim <= 128   16 chunks  G 4, CPL 4 (k <= 16) or G 2, CPL 8
//   dim <= 256   32 chunks  G 4, CPL 8
//   dim <= 512   64 chunks  G 8, CPL 8, passes in groups of 2
// (fewer lanes per row with more chunks each: fewer passes, group
// reductions and transposes per restart window, measured 10-25% faster
// with 20-id lists; with lists of up to 16 ids the 4-lane layout scans a
// list in one pass of 16 with half the work per lane, measured faster)
// The re-rank uses the layout of the stored float32 distance:
// ceil(dim / 64) chunks per lane of a 16-lane group.
#include "search.h"

namespace knng {

hipError_t launch_search_bf16(const SearchArgs& a, hipStream_t s, unsigned grid, size_t lds) {
  // KNNG_SCORE_BF16_MFMA (rows of up to 128 coordinates carrying their
  // norm) on the matrix cores (ScoreBF16M): 16 candidates per pass, 4 lanes
  // per row, one 16-byte chunk per lane per 32-coordinate MFMA block.  With
  // one wavefront per query the MFMA latency lies on every step's chain:
  // measured slower than the VALU form, which is the default.
  if (a.side2_off >= 0) {
    if (a.dim <= 32) return launch_search_t<ScoreBF16M<1>, 4, 1, 1, 8>(a, s, grid, lds);
    if (a.dim <= 64) return launch_search_t<ScoreBF16M<2>, 4, 2, 1, 8>(a, s, grid, lds);
    if (a.dim <= 96) return launch_search_t<ScoreBF16M<3>, 4, 3, 2, 4>(a, s, grid, lds);
    if (a.dim <= 128) return launch_search_t<ScoreBF16M<4>, 4, 4, 2, 4>(a, s, grid, lds);
  }
  // VALU dot products.
  // lists of up to 16 ids: 4 lanes per row (a list scan is one pass of 16);
  // longer lists: 2 lanes per row (32 candidates per pass).  Lists of 16
  // ids are loaded by the climb move that needs them rather than staged with
  // every candidate's row: on a 1M-node graph that took a third of the
  // search's HBM traffic and its removal made 16,384 searches 14% faster.
  // Rows of up to 96 coordinates (3 chunks per lane) fit the register
  // bound for 3 wavefronts per SIMD (5% faster again).
  if (a.dim <= 64)
    return a.k_pad == 16 ? launch_search_t<ScoreBF16<4, 2>, 4, 2, 1, 8, 4, false, false, 1, false>(a, s, grid, lds)
                         : launch_search_t<ScoreBF16<2, 4>, 2, 4, 1, 8, 2, false, false, 6>(a, s, grid, lds);
  // Launches of thousands of searches keep the scored positions of a
  // restart window across the climb it starts (16,384 searches on 1M nodes
  // 130.2 -> 118.2 ms; the same change made lone-wavefront launches of the
  // integer search 7% slower).
  if (a.dim <= 96 && a.k_pad == 16)
    return a.m >= 2048
               ? launch_search_t<ScoreBF16<4, 3>, 4, 3, 2, 4, 4, false, false, 1, false, 3, true>(a, s, grid, lds)
               : launch_search_t<ScoreBF16<4, 3>, 4, 3, 2, 4, 4, false, false, 1, false, 3>(a, s, grid, lds);
  if (a.dim <= 128)
    return a.k_pad == 16 ? launch_search_t<ScoreBF16<4, 4>, 4, 4, 2, 4, 4, false, false, 1, false>(a, s, grid, lds)
                         : launch_search_t<ScoreBF16<2, 8>, 2, 8, 2, 4, 2, false, false, 6>(a, s, grid, lds);
  if (a.dim <= 256) return launch_search_t<ScoreBF16<4, 8>, 4, 8, 4, 2>(a, s, grid, lds);
  // long rows (up to 512 coordinates): 8 lanes per row, 8 chunks per
  // lane, passes in groups of 2 with double-buffered gathers
  if (a.dim <= 512) return launch_search_t<ScoreBF16<8, 8>, 8, 8, 8, 1, 2>(a, s, grid, lds);
  return hipErrorInvalidValue;
}

}  // namespace knng
