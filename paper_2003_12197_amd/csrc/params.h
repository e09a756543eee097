// params.h -- host-side parameter resolution and precompute for libhers.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/hers.h"
#include "hers_common.h"

namespace hers {

struct HostTables {
  HersConsts C;
  // negacyclic NTT twiddles in bit-reversed order: tw[j] = psi^brv(j), itw[j] = psi^-brv(j)
  std::vector<uint64_t> qtw, qtw_sh, qitw, qitw_sh;   // [k][n]
  std::vector<uint32_t> ptw, ptw_sh, pitw, pitw_sh;   // [K][n]
  std::vector<uint32_t> ttw, ttw_sh, titw, titw_sh;   // [n]
  hers_info info;
};

// Resolves the prime rule and fills `info`; returns an error message or "".
std::string resolve(const hers_params& prm, hers_info* info);

// Full precompute (constants + twiddle tables).
std::string precompute(const hers_params& prm, HostTables* out);

// Host modular helpers (exposed for the host self-checks).
uint64_t powmod(uint64_t a, uint64_t e, uint64_t m);
bool is_prime_u64(uint64_t n);

}  // namespace hers
