// iGNNS launches for float graphs with FP8 E4M3 scoring rows, then the
// float32 re-rank of the kept candidates.  Row shapes by dimension (16-byte
// chunks of a scoring row; groups of G lanes read one row; CPL chunks per
// lane):
//   dim <= 64     4 chunks  G 4, CPL 1 (k <= 16) or G 2, CPL 2
//   dim <= 128    8 chunks  G 4, CPL 2 (k <= 16) or G 2, CPL 4
//   dim <= 256   16 chunks  G 4, CPL 4 (k <= 16) or G 2, CPL 8
//   dim <= 1024  64 chunks  FP8 MFMA: 16 candidates per pass, 4 lanes per row
// (fewer lanes per row with more chunks each: fewer passes, group
// reductions and transposes per restart window, measured 10-25% faster
// with 20-id lists; with lists of up to 16 ids the 4-lane layout scans a
// list in one pass of 16 with half the work per lane, measured faster)
// The re-rank uses the layout of the stored float32 distance:
// ceil(dim / 64) chunks per lane of a 16-lane group.
#include "search.h"

namespace knng {

hipError_t launch_search_fp8(const SearchArgs& a, hipStream_t s, unsigned grid, size_t lds) {
  // lists of up to 16 ids: 4 lanes per row (a list scan is one pass of 16);
  // longer lists: 2 lanes per row (32 candidates per pass)
  if (a.dim <= 64)
    return a.k_pad == 16 ? launch_search_t<ScoreFP8<4, 1>, 4, 1, 1, 8, 4, false, false, 1>(a, s, grid, lds)
                         : launch_search_t<ScoreFP8<2, 2>, 2, 2, 1, 8, 2, false, false, 6>(a, s, grid, lds);
  if (a.dim <= 128)
    return a.k_pad == 16 ? launch_search_t<ScoreFP8<4, 2>, 4, 2, 2, 4, 4, false, false, 1>(a, s, grid, lds)
                         : launch_search_t<ScoreFP8<2, 4>, 2, 4, 2, 4, 2, false, false, 6>(a, s, grid, lds);
  if (a.dim <= 256)
    return a.k_pad == 16 ? launch_search_t<ScoreFP8<4, 4>, 4, 4, 4, 2, 4, false, false, 1>(a, s, grid, lds)
                         : launch_search_t<ScoreFP8<2, 8>, 2, 8, 4, 2, 2, false, false, 6>(a, s, grid, lds);
  // long rows (up to 1024 coordinates) on the matrix cores: 16 candidates
  // per pass, 4 lanes per row, one pass (or two) per double-buffered group
  if (a.dim <= 512) return launch_search_t<ScoreFP8M<8>, 4, 8, 8, 1, 2>(a, s, grid, lds);
  if (a.dim <= 1024) return launch_search_t<ScoreFP8M<16>, 4, 16, 16, 1, 1>(a, s, grid, lds);
  return hipErrorInvalidValue;
}

}  // namespace knng
