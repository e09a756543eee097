// Host harness for the decryption scale (hers_common.h: decrypt_coeff_frac
// and decrypt_coeff_exact) on the constants of a resolved context
// (params.cpp: precompute).  First line: "n t_bits k qbits_0 .. qbits_{k-1}";
// then one coefficient per line as its k residues x_i.  Output per
// coefficient: the fraction form's flag and value (0 when not taken), and the
// exact form's value.
#include <cinttypes>
#include <cstdio>
#include <cstring>

#include "../../paper_2003_12197_amd/csrc/params.h"

int main() {
  unsigned n, tb, k;
  if (std::scanf("%u %u %u", &n, &tb, &k) != 3 || k < 1 || k > HC_MAXQ) return 2;
  hers_params prm;
  std::memset(&prm, 0, sizeof prm);
  prm.n = n;
  prm.t_bits = tb;
  prm.k = k;
  for (unsigned i = 0; i < k; ++i)
    if (std::scanf("%u", &prm.qbits[i]) != 1) return 2;
  prm.d_max = 1;
  prm.feature_bound = 1;
  static hers::HostTables T;
  const std::string err = hers::precompute(prm, &T);
  if (!err.empty()) {
    std::fprintf(stderr, "%s\n", err.c_str());
    return 3;
  }
  std::printf("t %u", T.C.t);
  for (unsigned i = 0; i < k; ++i) std::printf(" %" PRIu64, T.C.q[i]);
  std::printf("\n");
  std::fflush(stdout);
  uint64_t x[HC_MAXQ];
  for (;;) {
    for (unsigned i = 0; i < k; ++i)
      if (std::scanf("%" SCNu64, &x[i]) != 1) return 0;
    uint32_t v = 0;
    const bool fast = decrypt_coeff_frac(T.C, x, &v);
    std::printf("%d %u %u\n", (int)fast, fast ? v : 0u, decrypt_coeff_exact(T.C, x));
  }
}
