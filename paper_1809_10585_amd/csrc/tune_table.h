// Launch-shape table of the schedule builder, written by
// paper_1809_10585_amd/tune.py from timings of hodlr_qr on MI355X (exp-kernel
// HODLR matrices, leaf 256, eps 1e-10).  The first row with n <= n_max and
// rank_cap <= cap_max applies; shapes beyond the last row take its values.
#pragma once
#include <cstdint>

namespace hqh {
struct TuneRow {
  int64_t n_max;
  int cap_max;
  int mm_rt64_rows;
  int tr_small_chunks;
};
constexpr TuneRow kTuneTable[] = {
    {1 << 30, 1 << 30, 32768, 4},
};
}  // namespace hqh
