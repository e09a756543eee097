// Host harness for the double-precision modular arithmetic of ntt.h (ModQF,
// ModQB, u64 <-> double conversions).  Reads lines "op q a w" from stdin and
// writes one result per line; the test compares them with exact integer
// arithmetic.  Ops: F (ModQF::mul, a >= 0), B (ModQB::mul, a signed), R
// (ModQB::red of a), C (u64_to_f then f_to_u64 of a).
#include <cstdio>
#include <cinttypes>
#include "../../paper_2003_12197_amd/csrc/ntt.h"

int main() {
  char op;
  long long q_in, a_in, w_in;
  while (std::scanf(" %c %lld %lld %lld", &op, &q_in, &a_in, &w_in) == 4) {
    const double q = (double)q_in, qinv = 1.0 / q;
    const double a = (double)a_in, w = (double)w_in;
    switch (op) {
      case 'F': std::printf("%.0f\n", ModQF{q, qinv}.mul(a, w, 0.0)); break;
      case 'B': std::printf("%.0f\n", ModQB{q, qinv}.mul(a, w)); break;
      case 'R': std::printf("%.0f\n", ModQB{q, qinv}.red(a)); break;
      case 'C': std::printf("%" PRIu64 "\n", f_to_u64(u64_to_f((uint64_t)a_in))); break;
      default: return 2;
    }
  }
  return 0;
}
