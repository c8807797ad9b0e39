// iGNNS launches for float graphs with float32 scoring rows, then the
// float32 re-rank of the kept candidates.  Row shapes by dimension (16-byte
// chunks of a scoring row; groups of G lanes read one row; CPL chunks per
// lane):
//   dim <= 64    16 chunks  G 4, CPL 4 (k <= 16) or G 2, CPL 8
//   dim <= 128   32 chunks  G 4, CPL 8
//   dim <= 256   64 chunks  G 8, CPL 8
// (fewer lanes per row with more chunks each: fewer passes, group
// reductions and transposes per restart window, measured 10-25% faster
// with 20-id lists; with lists of up to 16 ids the 4-lane layout scans a
// list in one pass of 16 with half the work per lane, measured faster)
// The re-rank uses the layout of the stored float32 distance:
// ceil(dim / 64) chunks per lane of a 16-lane group.
#include "search.h"

namespace knng {

hipError_t launch_search_f32(const SearchArgs& a, hipStream_t s, unsigned grid, size_t lds) {
  // lists of up to 16 ids: 4 lanes per row (a list scan is one pass of 16);
  // longer lists: 2 lanes per row (32 candidates per pass)
  if (a.dim <= 64)
    return a.k_pad == 16 ? launch_search_t<ScoreF32<4, 4>, 4, 4, 1, 8, 4, false, false, 1>(a, s, grid, lds)
                         : launch_search_t<ScoreF32<2, 8>, 2, 8, 1, 8, 2, false, false, 6>(a, s, grid, lds);
  if (a.dim <= 128) return launch_search_t<ScoreF32<4, 8>, 4, 8, 2, 4>(a, s, grid, lds);
  if (a.dim <= 256) return launch_search_t<ScoreF32<8, 8>, 8, 8, 4, 2>(a, s, grid, lds);
  return hipErrorInvalidValue;
}

// The GNNS baseline on float32 rows.
hipError_t launch_search_f32_gnns(const SearchArgs& a, hipStream_t s, unsigned grid,
                                  size_t lds) {
  if (a.dim <= 64)
    return launch_search_t<ScoreF32<2, 8>, 2, 8, 1, 8, 2, true>(a, s, grid, lds);
  if (a.dim <= 128)
    return launch_search_t<ScoreF32<4, 8>, 4, 8, 2, 4, 4, true>(a, s, grid, lds);
  if (a.dim <= 256)
    return launch_search_t<ScoreF32<8, 8>, 8, 8, 4, 2, 8, true>(a, s, grid, lds);
  return hipErrorInvalidValue;
}

// Partitioned search on float32 rows.
hipError_t launch_search_f32_part(const SearchArgs& a, hipStream_t s, unsigned grid,
                                  size_t lds) {
  if (a.dim <= 64)
    return launch_search_t<ScoreF32<2, 8>, 2, 8, 1, 8, 2, false, true>(a, s, grid, lds);
  if (a.dim <= 128)
    return launch_search_t<ScoreF32<4, 8>, 4, 8, 2, 4, 4, false, true>(a, s, grid, lds);
  if (a.dim <= 256)
    return launch_search_t<ScoreF32<8, 8>, 8, 8, 4, 2, 8, false, true>(a, s, grid, lds);
  return hipErrorInvalidValue;
}

}  // namespace knng
