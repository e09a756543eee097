// ntt.h -- negacyclic number-theoretic transforms over Z_p[x]/(x^n + 1).
//
// The paper replaces the O(n^2) ring product by NTTs (Sec. 3.2, footnote on
// O(n log n)).  Forward: Cooley-Tukey with the powers of a primitive 2n-th
// root psi merged into the butterflies, natural-order input, bit-reversed
// output, so that out[i] = a(psi^(2 brv(i) + 1)).  Inverse: Gentleman-Sande,
// bit-reversed input, natural output, scaled by n^-1.  Twiddles:
// tw[j] = psi^brv(j), itw[j] = psi^-brv(j) with Shoup companions.
//
// The transforms are written once for a workgroup that owns the polynomial in
// LDS (tid, nthr) and compile unchanged for a single host thread (tid = 0,
// nthr = 1), which is how the host-side checks run them.
#pragma once
#include "hers_common.h"

#if defined(__HIP_DEVICE_COMPILE__)
#define HERS_SYNC() __syncthreads()
#else
#define HERS_SYNC() ((void)0)
#endif

struct ModP {
  uint32_t p;
  HD uint32_t add(uint32_t a, uint32_t b) const { return add_p(a, b, p); }
  HD uint32_t sub(uint32_t a, uint32_t b) const { return sub_p(a, b, p); }
  HD uint32_t mul(uint32_t a, uint32_t w, uint32_t wsh) const { return shoup_p(a, w, wsh, p); }
};

struct ModQ {
  uint64_t q;
  HD uint64_t add(uint64_t a, uint64_t b) const { return add_q(a, b, q); }
  HD uint64_t sub(uint64_t a, uint64_t b) const { return sub_q(a, b, q); }
  HD uint64_t mul(uint64_t a, uint64_t w, uint64_t wsh) const { return shoup_q(a, w, wsh, q); }
};

template <class M, class T>
HD void ntt_forward(T* a, const T* tw, const T* twsh, M mod, uint32_t n, uint32_t logn,
                    uint32_t tid, uint32_t nthr) {
  uint32_t lt = logn - 1;
  for (uint32_t m = 1; m < n; m <<= 1, --lt) {
    const uint32_t half = 1u << lt;
    for (uint32_t bf = tid; bf < (n >> 1); bf += nthr) {
      const uint32_t i = bf >> lt, j = bf & (half - 1);
      const uint32_t idx = (i << (lt + 1)) + j;
      const T w = tw[m + i], ws = twsh[m + i];
      const T u = a[idx];
      const T v = mod.mul(a[idx + half], w, ws);
      a[idx] = mod.add(u, v);
      a[idx + half] = mod.sub(u, v);
    }
    HERS_SYNC();
  }
}

template <class M, class T>
HD void ntt_inverse(T* a, const T* itw, const T* itwsh, T ninv, T ninv_sh, M mod, uint32_t n,
                    uint32_t logn, uint32_t tid, uint32_t nthr) {
  uint32_t lt = 0;
  for (uint32_t m = n >> 1; m >= 1; m >>= 1, ++lt) {
    const uint32_t half = 1u << lt;
    for (uint32_t bf = tid; bf < (n >> 1); bf += nthr) {
      const uint32_t i = bf >> lt, j = bf & (half - 1);
      const uint32_t idx = (i << (lt + 1)) + j;
      const T w = itw[m + i], ws = itwsh[m + i];
      const T u = a[idx], v = a[idx + half];
      a[idx] = mod.add(u, v);
      a[idx + half] = mod.mul(mod.sub(u, v), w, ws);
    }
    HERS_SYNC();
  }
  for (uint32_t j = tid; j < n; j += nthr) a[j] = mod.mul(a[j], ninv, ninv_sh);
  HERS_SYNC();
  (void)logn;
}

HD uint32_t bit_reverse(uint32_t x, uint32_t bits) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __brev(x) >> (32 - bits);
#else
  uint32_t r = 0;
  for (uint32_t i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
#endif
}
