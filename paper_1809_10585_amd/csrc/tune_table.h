// Launch-shape table of the schedule builder, written by
// paper_1809_10585_amd/tune.py from timings of hodlr_qr on MI355X (exp-kernel
// HODLR matrices at rank capacity 16, Gaussian HODLR matrices at capacity 64;
// leaf 256, eps 1e-10).  The first row with n <= n_max and rank_cap <= cap_max
// applies; shapes beyond the last row take its values.
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
    {4096, 32, 32768, 4},  // expkernel(n=4096,leaf=256): 10.40 ms (32768/4: 10.40 ms)
    {16384, 32, 4096, 4},  // expkernel(n=16384,leaf=256): 38.68 ms (32768/4: 38.88 ms)
    {1073741824, 32, 32768, 4},  // expkernel(n=65536,leaf=256): 157.84 ms (32768/4: 157.84 ms)
    {4096, 1073741824, 32768, 2},  // gaussian(n=4096,leaf=256): 143.58 ms (32768/4: 143.66 ms)
    {1073741824, 1073741824, 4096, 1},  // gaussian(n=16384,leaf=256): 631.55 ms (32768/4: 632.41 ms)
};
}  // namespace hqh
