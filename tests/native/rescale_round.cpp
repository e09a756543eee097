// Host harness for the fixed-point rounding of the exact rescale
// (hers_common.h: round_F).  Each input line holds
// "W K gamma", then y_0 .. y_{K-1}, then the fraction words fr_phi[r][w]
// (r-major, w from the lowest word), then fr_psi[0 .. W-1].  Output per line:
// the two-word sum's round(F) and its near-half flag, and the W-word round(F).
#include <cstdio>
#include <cinttypes>
#include <cstring>
#include "../../paper_2003_12197_amd/csrc/hers_common.h"

int main() {
  static HersConsts C;
  unsigned W, K;
  uint64_t gamma;
  while (std::scanf("%u %u %" SCNu64, &W, &K, &gamma) == 3) {
    if (W < 1 || W > HC_MAXW || K < 1 || K > HC_MAXP) return 2;
    std::memset(&C, 0, sizeof C);
    uint32_t y[HC_MAXP];
    for (unsigned r = 0; r < K; ++r)
      if (std::scanf("%u", &y[r]) != 1) return 2;
    for (unsigned r = 0; r < K; ++r)
      for (unsigned w = 0; w < W; ++w)
        if (std::scanf("%" SCNu64, &C.fr_phi[r][w]) != 1) return 2;
    for (unsigned w = 0; w < W; ++w)
      if (std::scanf("%" SCNu64, &C.fr_psi[w]) != 1) return 2;
    bool nh_short = false, nh_full = false;
    const int64_t rs = round_F(C, y, K, gamma, W, W > 2 ? W - 2 : 0, &nh_short);
    const int64_t rw = round_F(C, y, K, gamma, W, 0, &nh_full);
    std::printf("%" PRId64 " %d %" PRId64 "\n", rs, (int)nh_short, rw);
  }
  return 0;
}
