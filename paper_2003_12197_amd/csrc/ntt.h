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
// nthr = 1).
#pragma once
#include "hers_common.h"

#if defined(__HIP_DEVICE_COMPILE__)
#define HERS_SYNC() __syncthreads()
#else
#define HERS_SYNC() ((void)0)
#endif

// Lazy forms (Harvey, "Faster arithmetic for number-theoretic transforms",
// 2014): mul_lazy leaves a w - floor(a wsh / 2^W) q in [0, 2m) without the
// final correction; red2 subtracts 2m once.  Butterfly values stay in [0, 4m),
// which needs 4m below the word size (p < 2^30, q < 2^62).
struct ModP {
  uint32_t p;
  HD uint32_t add(uint32_t a, uint32_t b) const { return add_p(a, b, p); }
  HD uint32_t sub(uint32_t a, uint32_t b) const { return sub_p(a, b, p); }
  HD uint32_t mul(uint32_t a, uint32_t w, uint32_t wsh) const { return shoup_p(a, w, wsh, p); }
  HD uint32_t mul_lazy(uint32_t a, uint32_t w, uint32_t wsh) const { return a * w - mulhi32(a, wsh) * p; }
  HD uint32_t red2(uint32_t a) const { return a >= 2 * p ? a - 2 * p : a; }
  HD uint32_t two() const { return 2 * p; }
  HD uint32_t full(uint32_t a) const { a = a >= 2 * p ? a - 2 * p : a; return a >= p ? a - p : a; }
};

struct ModQ {
  uint64_t q;
  HD uint64_t add(uint64_t a, uint64_t b) const { return add_q(a, b, q); }
  HD uint64_t sub(uint64_t a, uint64_t b) const { return sub_q(a, b, q); }
  HD uint64_t mul(uint64_t a, uint64_t w, uint64_t wsh) const { return shoup_q(a, w, wsh, q); }
  HD uint64_t mul_lazy(uint64_t a, uint64_t w, uint64_t wsh) const { return a * w - mulhi64(a, wsh) * q; }
  HD uint64_t red2(uint64_t a) const { return a >= 2 * q ? a - 2 * q : a; }
  HD uint64_t two() const { return 2 * q; }
  HD uint64_t full(uint64_t a) const { a = a >= 2 * q ? a - 2 * q : a; return a >= q ? a - q : a; }
};

// Arithmetic mod q < 2^48 on exact integers held in doubles (all values below
// 2^50, so every operand and every partial result used below is an integer
// that a double holds exactly).  a w mod q: hi = fl(a w) and lo = a w - hi
// (exact, by one fused multiply-add) split the product; qt = rint(hi / q)
// (within 3/4 of hi / q, the reciprocal's and the product's rounding errors
// being below 2^-52 relative); hi - qt q then lies in [-3q/4, 3q/4] and comes
// exactly out of one fused multiply-add, and |lo| <= a w 2^-53 < q / 8, so
// r = (hi - qt q) + lo is exact and in (-q, q); one conditional add of q
// gives [0, q).  These are full-rate double operations where the 64-bit
// integer Shoup product takes half-rate 32-bit multiply-adds.
struct ModQF {
  double q, qinv;   // qinv = fl(1 / q)
  HD double mul_lazy(double a, double w, double) const {
#pragma clang fp contract(off)
    const double hi = a * w;
    const double lo = __builtin_fma(a, w, -hi);
    const double qt = __builtin_rint(hi * qinv);
    const double r = __builtin_fma(-qt, q, hi) + lo;
    return r < 0.0 ? r + q : r;
  }
  HD double mul(double a, double w, double ws) const { return mul_lazy(a, w, ws); }
  // x mod q for an integer 0 <= x < 2^50: x - rint(x / q) q is exact and in (-q, q)
  HD double reduce(double x) const {
#pragma clang fp contract(off)
    const double r = __builtin_fma(-__builtin_rint(x * qinv), q, x);
    return r < 0.0 ? r + q : r;
  }
  HD double red2(double a) const { return a >= 2.0 * q ? a - 2.0 * q : a; }
  HD double two() const { return 2.0 * q; }
  HD double full(double a) const { a = a >= 2.0 * q ? a - 2.0 * q : a; return a >= q ? a - q : a; }
};

// Exact conversions between integers below 2^52 and doubles: a double with
// exponent field 0x433 holds 2^52 + (its 52 mantissa bits).
HD double u64_to_f(uint64_t v) {
  return __builtin_bit_cast(double, v | 0x4330000000000000ull) - 4503599627370496.0;
}
HD uint64_t f_to_u64(double x) {
  return __builtin_bit_cast(uint64_t, x + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}

// ---- LDS layout
// A polynomial in LDS has one padding element after every 16 (element j at
// PADX(j)), so lanes reading 16 consecutive elements, or elements 16 apart,
// fall in different banks.
#define PADX(j) ((j) + ((j) >> 4))
HD uint32_t padded_len(uint32_t n) { return n + (n >> 4); }

// Copies n words src[j] into LDS at dst[PADX(j)], converted by conv, four per
// lane at a time so their global loads are in flight together (a loop of one
// load per iteration waits on each in turn); n not a multiple of 4 nthr goes
// one word at a time.
template <class D, class S, class F>
HD void load_padded(D* dst, const S* __restrict__ src, uint32_t n, uint32_t tid, uint32_t nthr, F conv) {
  if (n % (4 * nthr) == 0) {
    for (uint32_t j = tid; j < n; j += 4 * nthr) {
      const S v0 = src[j], v1 = src[j + nthr], v2 = src[j + 2 * nthr], v3 = src[j + 3 * nthr];
      dst[PADX(j)] = conv(v0);
      dst[PADX(j + nthr)] = conv(v1);
      dst[PADX(j + 2 * nthr)] = conv(v2);
      dst[PADX(j + 3 * nthr)] = conv(v3);
    }
  } else {
    for (uint32_t j = tid; j < n; j += nthr) dst[PADX(j)] = conv(src[j]);
  }
}

// Calls f(j, src[j]) (f2: f(j, a[j], b[j])) for j = tid, tid + nthr, ... < n,
// loading four words per lane before using them, as load_padded does.
template <class S, class F>
HD void for_each_loaded(const S* __restrict__ src, uint32_t n, uint32_t tid, uint32_t nthr, F f) {
  if (n % (4 * nthr) == 0) {
    for (uint32_t j = tid; j < n; j += 4 * nthr) {
      const S v0 = src[j], v1 = src[j + nthr], v2 = src[j + 2 * nthr], v3 = src[j + 3 * nthr];
      f(j, v0);
      f(j + nthr, v1);
      f(j + 2 * nthr, v2);
      f(j + 3 * nthr, v3);
    }
  } else {
    for (uint32_t j = tid; j < n; j += nthr) f(j, src[j]);
  }
}
template <class S, class F>
HD void for_each_loaded2(const S* __restrict__ a, const S* __restrict__ b, uint32_t n, uint32_t tid, uint32_t nthr,
                         F f) {
  if (n % (4 * nthr) == 0) {
    for (uint32_t j = tid; j < n; j += 4 * nthr) {
      const S a0 = a[j], a1 = a[j + nthr], a2 = a[j + 2 * nthr], a3 = a[j + 3 * nthr];
      const S b0 = b[j], b1 = b[j + nthr], b2 = b[j + 2 * nthr], b3 = b[j + 3 * nthr];
      f(j, a0, b0);
      f(j + nthr, a1, b1);
      f(j + 2 * nthr, a2, b2);
      f(j + 3 * nthr, a3, b3);
    }
  } else {
    for (uint32_t j = tid; j < n; j += nthr) f(j, a[j], b[j]);
  }
}

// ---- radix-16 passes
// The stages are taken in passes of R <= 4.  In a pass over stages
// s0 .. s0+R-1 (forward, half = n >> (s+1)) the 2^R elements
// idx = c (n >> s0) + j h + o, j < 2^R, with h = n >> (s0+R), c < 2^s0 and o < h,
// are closed under the pass's butterflies: a virtual thread (c, o) loads them
// into registers with their 2^R - 1 twiddles, runs the R stages, and stores
// them back.  Virtual threads of a pass touch disjoint elements, so one
// barrier per pass suffices (and a single host thread can run them in turn).

// One forward pass from src to dst, each in LDS (padded index) or, with
// SRC_G / DST_G, in global memory (plain index).  FIN (the last pass of a
// transform): each value is reduced to [0, m) before it is stored, which saves
// the transform a further pass over LDS and a barrier.
template <int R, bool SRC_G, bool DST_G, bool FIN, class M, class T>
HD void ntt_fwd_pass_io(const T* src, T* dst, const T* tw, const T* twsh, M mod, uint32_t n, uint32_t s0,
                        uint32_t tid, uint32_t nthr) {
  constexpr uint32_t E = 1u << R;
  const uint32_t lh = 31 - __builtin_clz(n >> (s0 + R));   // log2 h
  const uint32_t h = 1u << lh;
  const uint32_t vts = n >> R;
  for (uint32_t vt = tid; vt < vts; vt += nthr) {
    const uint32_t c = vt >> lh, o = vt & (h - 1);
    const uint32_t base = (c << (lh + R)) + o;
    T x[E];
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) x[j] = SRC_G ? src[base + j * h] : src[PADX(base + j * h)];
#pragma unroll
    for (uint32_t t = 0; t < R; ++t) {                // stage s0 + t: pairs (j, j + E/2^(t+1))
      const uint32_t span = E >> (t + 1);
      const uint32_t m = 1u << (s0 + t);
#pragma unroll
      for (uint32_t j = 0; j < E; ++j) {
        if (j & span) continue;
        const uint32_t i = (c << t) + (j / (2 * span));
        const T w = tw[m + i], ws = twsh[m + i];
        const T u = mod.red2(x[j]);                     // [0, 2m)
        const T v = mod.mul_lazy(x[j + span], w, ws);   // [0, 2m)
        x[j] = u + v;                                   // [0, 4m)
        x[j + span] = u - v + mod.two();                // (0, 4m)
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) {
      const T v = FIN ? mod.full(x[j]) : x[j];
      if constexpr (DST_G) dst[base + j * h] = v;
      else dst[PADX(base + j * h)] = v;
    }
  }
  HERS_SYNC();
}

template <int R, bool FIN = false, class M, class T>
HD void ntt_fwd_pass(T* a, const T* tw, const T* twsh, M mod, uint32_t n, uint32_t s0, uint32_t tid, uint32_t nthr) {
  ntt_fwd_pass_io<R, false, false, FIN>(a, a, tw, twsh, mod, n, s0, tid, nthr);
}

// One inverse pass from src to dst, each in LDS (padded index) or, with
// SRC_G / DST_G, in global memory (plain index).  FIN (the last pass): each
// value is scaled by ninv (a full product, [0, m)) before it is stored.
template <int R, bool SRC_G, bool DST_G, bool FIN, class M, class T>
HD void ntt_inv_pass_io(const T* src, T* dst, const T* itw, const T* itwsh, M mod, uint32_t n, uint32_t lh0,
                        uint32_t tid, uint32_t nthr, T ninv, T ninv_sh) {
  // stages with half = 2^lh0 .. 2^(lh0+R-1); elements idx = c 2^(lh0+R) + j 2^lh0 + o
  constexpr uint32_t E = 1u << R;
  const uint32_t h = 1u << lh0;
  const uint32_t vts = n >> R;
  for (uint32_t vt = tid; vt < vts; vt += nthr) {
    const uint32_t c = vt >> lh0, o = vt & (h - 1);
    const uint32_t base = (c << (lh0 + R)) + o;
    T x[E];
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) x[j] = SRC_G ? src[base + j * h] : src[PADX(base + j * h)];
#pragma unroll
    for (uint32_t t = 0; t < R; ++t) {                // half = 2^(lh0+t): pairs (j, j + 2^t)
      const uint32_t span = 1u << t;
      const uint32_t m = n >> (lh0 + t + 1);
#pragma unroll
      for (uint32_t j = 0; j < E; ++j) {
        if (j & span) continue;
        const uint32_t i = (c << (R - 1 - t)) + (j >> (t + 1));
        const T w = itw[m + i], ws = itwsh[m + i];
        const T u = x[j], v = x[j + span];
        x[j] = mod.red2(u + v);                                // [0, 2m)
        x[j + span] = mod.mul_lazy(u - v + mod.two(), w, ws);  // [0, 2m)
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) {
      const T v = FIN ? mod.mul(x[j], ninv, ninv_sh) : x[j];
      if constexpr (DST_G) dst[base + j * h] = v;
      else dst[PADX(base + j * h)] = v;
    }
  }
  HERS_SYNC();
}

template <int R, bool FIN = false, class M, class T>
HD void ntt_inv_pass(T* a, const T* itw, const T* itwsh, M mod, uint32_t n, uint32_t lh0, uint32_t tid,
                     uint32_t nthr, T ninv = T(0), T ninv_sh = T(0)) {
  ntt_inv_pass_io<R, false, false, FIN>(a, a, itw, itwsh, mod, n, lh0, tid, nthr, ninv, ninv_sh);
}

// Forward transform in passes of rmax (<= 4) stages; input in [0, 4m), output in [0, m).
// RMAX caps rmax at compile time (fewer registers for the passes).
template <int RMAX = 4, class M, class T>
HD void ntt_forward16(T* a, const T* tw, const T* twsh, M mod, uint32_t n, uint32_t logn, uint32_t tid,
                      uint32_t nthr, uint32_t rmax = 4) {
  if (rmax > (uint32_t)RMAX) rmax = RMAX;
  uint32_t s0 = 0;
  while (s0 < logn) {
    const uint32_t r = logn - s0 < rmax ? logn - s0 : rmax;
    if (s0 + r < logn) {
      switch (r) {
        case 4: if constexpr (RMAX >= 4) ntt_fwd_pass<4>(a, tw, twsh, mod, n, s0, tid, nthr); break;
        case 3: ntt_fwd_pass<3>(a, tw, twsh, mod, n, s0, tid, nthr); break;
        case 2: ntt_fwd_pass<2>(a, tw, twsh, mod, n, s0, tid, nthr); break;
        default: ntt_fwd_pass<1>(a, tw, twsh, mod, n, s0, tid, nthr); break;
      }
    } else {                                          // the last pass stores reduced values
      switch (r) {
        case 4: if constexpr (RMAX >= 4) ntt_fwd_pass<4, true>(a, tw, twsh, mod, n, s0, tid, nthr); break;
        case 3: ntt_fwd_pass<3, true>(a, tw, twsh, mod, n, s0, tid, nthr); break;
        case 2: ntt_fwd_pass<2, true>(a, tw, twsh, mod, n, s0, tid, nthr); break;
        default: ntt_fwd_pass<1, true>(a, tw, twsh, mod, n, s0, tid, nthr); break;
      }
    }
    s0 += r;
  }
  if (logn == 0) {
    for (uint32_t j = tid; j < n; j += nthr) a[PADX(j)] = mod.full(a[PADX(j)]);
    HERS_SYNC();
  }
}

// Inverse transform in passes of rmax (<= 4) stages, scaled by n^-1; input in [0, 2m),
// output in [0, m).  RMAX as for ntt_forward16.
template <int RMAX = 4, class M, class T>
HD void ntt_inverse16(T* a, const T* itw, const T* itwsh, T ninv, T ninv_sh, M mod, uint32_t n, uint32_t logn,
                      uint32_t tid, uint32_t nthr, uint32_t rmax = 4) {
  if (rmax > (uint32_t)RMAX) rmax = RMAX;
  uint32_t lh0 = 0;
  while (lh0 < logn) {
    const uint32_t r = logn - lh0 < rmax ? logn - lh0 : rmax;
    if (lh0 + r < logn) {
      switch (r) {
        case 4: if constexpr (RMAX >= 4) ntt_inv_pass<4>(a, itw, itwsh, mod, n, lh0, tid, nthr); break;
        case 3: ntt_inv_pass<3>(a, itw, itwsh, mod, n, lh0, tid, nthr); break;
        case 2: ntt_inv_pass<2>(a, itw, itwsh, mod, n, lh0, tid, nthr); break;
        default: ntt_inv_pass<1>(a, itw, itwsh, mod, n, lh0, tid, nthr); break;
      }
    } else {                                          // the last pass stores scaled values
      switch (r) {
        case 4: if constexpr (RMAX >= 4) ntt_inv_pass<4, true>(a, itw, itwsh, mod, n, lh0, tid, nthr, ninv, ninv_sh); break;
        case 3: ntt_inv_pass<3, true>(a, itw, itwsh, mod, n, lh0, tid, nthr, ninv, ninv_sh); break;
        case 2: ntt_inv_pass<2, true>(a, itw, itwsh, mod, n, lh0, tid, nthr, ninv, ninv_sh); break;
        default: ntt_inv_pass<1, true>(a, itw, itwsh, mod, n, lh0, tid, nthr, ninv, ninv_sh); break;
      }
    }
    lh0 += r;
  }
  if (logn == 0) {
    for (uint32_t j = tid; j < n; j += nthr) a[PADX(j)] = mod.mul(a[PADX(j)], ninv, ninv_sh);
    HERS_SYNC();
  }
}

// The forward transform (as ntt_forward16, input in [0, 4m), output in
// [0, m)) of the n words at g in global memory, in place, with the LDS buffer
// a: the first pass reads g (consecutive words across the lanes), and the
// result goes back to g from LDS (the last pass's own elements are
// consecutive words per lane, which would make every store instruction
// strided): one trip through LDS fewer than a load into LDS, ntt_forward16
// and a store.  With more stages than one pass holds, the last pass takes as
// many stages as it can and the middle passes the rest.
template <int RMAX = 4, class M, class T>
HD void ntt_forward16_g(T* g, T* a, const T* tw, const T* twsh, M mod, uint32_t n, uint32_t logn, uint32_t tid,
                        uint32_t nthr, uint32_t rmax = 4) {
  if (rmax > (uint32_t)RMAX) rmax = RMAX;
  if (rmax < 1) rmax = 1;
  if (logn <= rmax) {                                   // one pass, global to global
    switch (logn) {
      case 4: if constexpr (RMAX >= 4) ntt_fwd_pass_io<4, true, true, true>(g, g, tw, twsh, mod, n, 0, tid, nthr); break;
      case 3: if constexpr (RMAX >= 3) ntt_fwd_pass_io<3, true, true, true>(g, g, tw, twsh, mod, n, 0, tid, nthr); break;
      case 2: if constexpr (RMAX >= 2) ntt_fwd_pass_io<2, true, true, true>(g, g, tw, twsh, mod, n, 0, tid, nthr); break;
      case 1: ntt_fwd_pass_io<1, true, true, true>(g, g, tw, twsh, mod, n, 0, tid, nthr); break;
      default:
        for (uint32_t j = tid; j < n; j += nthr) g[j] = mod.full(g[j]);
        HERS_SYNC();
        break;
    }
    return;
  }
  const uint32_t r0 = rmax;
  const uint32_t rl = logn - r0 < rmax ? logn - r0 : rmax;
  switch (r0) {                                         // first pass: global to LDS
    case 4: if constexpr (RMAX >= 4) ntt_fwd_pass_io<4, true, false, false>(g, a, tw, twsh, mod, n, 0, tid, nthr); break;
    case 3: if constexpr (RMAX >= 3) ntt_fwd_pass_io<3, true, false, false>(g, a, tw, twsh, mod, n, 0, tid, nthr); break;
    case 2: if constexpr (RMAX >= 2) ntt_fwd_pass_io<2, true, false, false>(g, a, tw, twsh, mod, n, 0, tid, nthr); break;
    default: ntt_fwd_pass_io<1, true, false, false>(g, a, tw, twsh, mod, n, 0, tid, nthr); break;
  }
  const uint32_t s_last = logn - rl;
  uint32_t s0 = r0;
  while (s0 < s_last) {                                 // middle passes in LDS
    const uint32_t r = s_last - s0 < rmax ? s_last - s0 : rmax;
    switch (r) {
      case 4: if constexpr (RMAX >= 4) ntt_fwd_pass<4>(a, tw, twsh, mod, n, s0, tid, nthr); break;
      case 3: if constexpr (RMAX >= 3) ntt_fwd_pass<3>(a, tw, twsh, mod, n, s0, tid, nthr); break;
      case 2: if constexpr (RMAX >= 2) ntt_fwd_pass<2>(a, tw, twsh, mod, n, s0, tid, nthr); break;
      default: ntt_fwd_pass<1>(a, tw, twsh, mod, n, s0, tid, nthr); break;
    }
    s0 += r;
  }
  switch (rl) {                                         // last pass in LDS, reduced
    case 4: if constexpr (RMAX >= 4) ntt_fwd_pass<4, true>(a, tw, twsh, mod, n, s_last, tid, nthr); break;
    case 3: if constexpr (RMAX >= 3) ntt_fwd_pass<3, true>(a, tw, twsh, mod, n, s_last, tid, nthr); break;
    case 2: if constexpr (RMAX >= 2) ntt_fwd_pass<2, true>(a, tw, twsh, mod, n, s_last, tid, nthr); break;
    default: ntt_fwd_pass<1, true>(a, tw, twsh, mod, n, s_last, tid, nthr); break;
  }
  for (uint32_t j = tid; j < n; j += nthr) g[j] = a[PADX(j)];
}

// The inverse transform (as ntt_inverse16, input in [0, 2m), output in
// [0, m)) of the n words at g in global memory, in place, with the LDS buffer
// a: the first pass reads g and the last pass writes g (scaled by ninv), so
// the polynomial makes two fewer trips through LDS than a load into LDS,
// ntt_inverse16 and a store would.  With more stages than one pass holds, the
// last pass takes as many stages as it can and the middle passes the rest.
template <int RMAX = 4, class M, class T>
HD void ntt_inverse16_g(T* g, T* a, const T* itw, const T* itwsh, T ninv, T ninv_sh, M mod, uint32_t n,
                        uint32_t logn, uint32_t tid, uint32_t nthr, uint32_t rmax = 4) {
  if (rmax > (uint32_t)RMAX) rmax = RMAX;
  if (rmax < 1) rmax = 1;
  if (logn <= rmax) {                                   // one pass, global to global
    switch (logn) {
      case 4: if constexpr (RMAX >= 4) ntt_inv_pass_io<4, true, true, true>(g, g, itw, itwsh, mod, n, 0, tid, nthr, ninv, ninv_sh); break;
      case 3: if constexpr (RMAX >= 3) ntt_inv_pass_io<3, true, true, true>(g, g, itw, itwsh, mod, n, 0, tid, nthr, ninv, ninv_sh); break;
      case 2: if constexpr (RMAX >= 2) ntt_inv_pass_io<2, true, true, true>(g, g, itw, itwsh, mod, n, 0, tid, nthr, ninv, ninv_sh); break;
      case 1: ntt_inv_pass_io<1, true, true, true>(g, g, itw, itwsh, mod, n, 0, tid, nthr, ninv, ninv_sh); break;
      default:
        for (uint32_t j = tid; j < n; j += nthr) g[j] = mod.mul(g[j], ninv, ninv_sh);
        HERS_SYNC();
        break;
    }
    return;
  }
  const uint32_t r0 = rmax;
  const uint32_t rl = logn - r0 < rmax ? logn - r0 : rmax;
  switch (r0) {                                         // first pass: global to LDS
    case 4: if constexpr (RMAX >= 4) ntt_inv_pass_io<4, true, false, false>(g, a, itw, itwsh, mod, n, 0, tid, nthr, ninv, ninv_sh); break;
    case 3: if constexpr (RMAX >= 3) ntt_inv_pass_io<3, true, false, false>(g, a, itw, itwsh, mod, n, 0, tid, nthr, ninv, ninv_sh); break;
    case 2: if constexpr (RMAX >= 2) ntt_inv_pass_io<2, true, false, false>(g, a, itw, itwsh, mod, n, 0, tid, nthr, ninv, ninv_sh); break;
    default: ntt_inv_pass_io<1, true, false, false>(g, a, itw, itwsh, mod, n, 0, tid, nthr, ninv, ninv_sh); break;
  }
  const uint32_t lh_last = logn - rl;
  uint32_t lh0 = r0;
  while (lh0 < lh_last) {                               // middle passes in LDS
    const uint32_t r = lh_last - lh0 < rmax ? lh_last - lh0 : rmax;
    switch (r) {
      case 4: if constexpr (RMAX >= 4) ntt_inv_pass<4>(a, itw, itwsh, mod, n, lh0, tid, nthr); break;
      case 3: if constexpr (RMAX >= 3) ntt_inv_pass<3>(a, itw, itwsh, mod, n, lh0, tid, nthr); break;
      case 2: if constexpr (RMAX >= 2) ntt_inv_pass<2>(a, itw, itwsh, mod, n, lh0, tid, nthr); break;
      default: ntt_inv_pass<1>(a, itw, itwsh, mod, n, lh0, tid, nthr); break;
    }
    lh0 += r;
  }
  switch (rl) {                                         // last pass: LDS to global, scaled
    case 4: if constexpr (RMAX >= 4) ntt_inv_pass_io<4, false, true, true>(a, g, itw, itwsh, mod, n, lh_last, tid, nthr, ninv, ninv_sh); break;
    case 3: if constexpr (RMAX >= 3) ntt_inv_pass_io<3, false, true, true>(a, g, itw, itwsh, mod, n, lh_last, tid, nthr, ninv, ninv_sh); break;
    case 2: if constexpr (RMAX >= 2) ntt_inv_pass_io<2, false, true, true>(a, g, itw, itwsh, mod, n, lh_last, tid, nthr, ninv, ninv_sh); break;
    default: ntt_inv_pass_io<1, false, true, true>(a, g, itw, itwsh, mod, n, lh_last, tid, nthr, ninv, ninv_sh); break;
  }
}

// The inverse transform with passes of at most RMAX stages fixed at compile
// time (the radix-16 pass keeps 16 elements and their twiddles in registers;
// a kernel with a tight register budget takes radix 8).
template <int RMAX, class M, class T>
HD void ntt_inverse_upto(T* a, const T* itw, const T* itwsh, T ninv, T ninv_sh, M mod, uint32_t n, uint32_t logn,
                         uint32_t tid, uint32_t nthr) {
  static_assert(RMAX >= 1 && RMAX <= 4, "1 to 4 stages per pass");
  uint32_t lh0 = 0;
  while (lh0 < logn) {
    const uint32_t r = logn - lh0 < (uint32_t)RMAX ? logn - lh0 : (uint32_t)RMAX;
    if (lh0 + r < logn) {
      switch (r) {
        case 4: if constexpr (RMAX >= 4) ntt_inv_pass<4>(a, itw, itwsh, mod, n, lh0, tid, nthr); break;
        case 3: if constexpr (RMAX >= 3) ntt_inv_pass<3>(a, itw, itwsh, mod, n, lh0, tid, nthr); break;
        case 2: if constexpr (RMAX >= 2) ntt_inv_pass<2>(a, itw, itwsh, mod, n, lh0, tid, nthr); break;
        default: ntt_inv_pass<1>(a, itw, itwsh, mod, n, lh0, tid, nthr); break;
      }
    } else {                                          // the last pass stores scaled values
      switch (r) {
        case 4: if constexpr (RMAX >= 4) ntt_inv_pass<4, true>(a, itw, itwsh, mod, n, lh0, tid, nthr, ninv, ninv_sh); break;
        case 3: if constexpr (RMAX >= 3) ntt_inv_pass<3, true>(a, itw, itwsh, mod, n, lh0, tid, nthr, ninv, ninv_sh); break;
        case 2: if constexpr (RMAX >= 2) ntt_inv_pass<2, true>(a, itw, itwsh, mod, n, lh0, tid, nthr, ninv, ninv_sh); break;
        default: ntt_inv_pass<1, true>(a, itw, itwsh, mod, n, lh0, tid, nthr, ninv, ninv_sh); break;
      }
    }
    lh0 += r;
  }
  if (logn == 0) {
    for (uint32_t j = tid; j < n; j += nthr) a[PADX(j)] = mod.mul(a[PADX(j)], ninv, ninv_sh);
    HERS_SYNC();
  }
}

// ---- balanced double-precision transforms (every q < 2^45)
// Values are exact integers held in doubles, kept in a signed (balanced)
// range instead of [0, 4q), so a butterfly needs no conditional corrections.
//   mul(a, w) = a w mod q as some r with |r| < 0.7 q, for |a| <= 16 q and
//     0 <= w < q: hi = fl(a w), lo = a w - hi (exact, one fused multiply-add),
//     qt = rint(hi / q), within 0.63 of hi / q since |hi / q| < 2^49 and the
//     rounding errors are below 2^-52 relative; r = (hi - qt q) + lo, both
//     steps exact, with |lo| <= a w 2^-53 < q / 16.
//   red(x) = x - rint(x / q) q, |red(x)| <= q/2 + 1, for |x| < 2^50.
// A forward (Cooley-Tukey) stage maps (u, v) to (u + v w, u - v w), growing
// magnitudes by < 0.7 q; an inverse (Gentleman-Sande) stage maps (u, v) to
// (u + v, (u - v) w), doubling the sum.  Each pass (at most 4 stages) starts
// from values of magnitude <= q and reduces what it stores, so no value
// exceeds 16 q (< 2^49).
struct ModQB {
  double q, qinv;   // qinv = fl(1 / q)
  HD double mul(double a, double w) const {
#pragma clang fp contract(off)
    const double hi = a * w;
    const double lo = __builtin_fma(a, w, -hi);
    return __builtin_fma(-__builtin_rint(hi * qinv), q, hi) + lo;
  }
  HD double red(double x) const {
#pragma clang fp contract(off)
    return __builtin_fma(-__builtin_rint(x * qinv), q, x);
  }
  HD double canon(double x) const {   // [0, q) from |x| < 2^50
    const double r = red(x);
    return r < 0.0 ? r + q : r;
  }
};

// FIN (the last pass): stored values are brought to [0, q).
template <int R, bool FIN = false>
HD void ntt_fwd_pass_b(double* a, const double* tw, ModQB mod, uint32_t n, uint32_t s0, uint32_t tid,
                       uint32_t nthr) {
  constexpr uint32_t E = 1u << R;
  const uint32_t lh = 31 - __builtin_clz(n >> (s0 + R));   // log2 h
  const uint32_t h = 1u << lh;
  const uint32_t vts = n >> R;
  for (uint32_t vt = tid; vt < vts; vt += nthr) {
    const uint32_t c = vt >> lh, o = vt & (h - 1);
    const uint32_t base = (c << (lh + R)) + o;
    double x[E];
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) x[j] = a[PADX(base + j * h)];
#pragma unroll
    for (uint32_t t = 0; t < R; ++t) {
      const uint32_t span = E >> (t + 1);
      const uint32_t m = 1u << (s0 + t);
#pragma unroll
      for (uint32_t j = 0; j < E; ++j) {
        if (j & span) continue;
        const double v = mod.mul(x[j + span], tw[m + (c << t) + (j / (2 * span))]);
        const double u = x[j];
        x[j] = u + v;
        x[j + span] = u - v;
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) a[PADX(base + j * h)] = FIN ? mod.canon(mod.red(x[j])) : mod.red(x[j]);
  }
  HERS_SYNC();
}

// FIN (the last pass): stored values are scaled by ninv and brought to [0, q).
template <int R, bool FIN = false>
HD void ntt_inv_pass_b(double* a, const double* itw, ModQB mod, uint32_t n, uint32_t lh0, uint32_t tid,
                       uint32_t nthr, double ninv = 0.0) {
  constexpr uint32_t E = 1u << R;
  const uint32_t h = 1u << lh0;
  const uint32_t vts = n >> R;
  for (uint32_t vt = tid; vt < vts; vt += nthr) {
    const uint32_t c = vt >> lh0, o = vt & (h - 1);
    const uint32_t base = (c << (lh0 + R)) + o;
    double x[E];
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) x[j] = a[PADX(base + j * h)];
#pragma unroll
    for (uint32_t t = 0; t < R; ++t) {
      const uint32_t span = 1u << t;
      const uint32_t m = n >> (lh0 + t + 1);
#pragma unroll
      for (uint32_t j = 0; j < E; ++j) {
        if (j & span) continue;
        const double u = x[j], v = x[j + span];
        x[j] = u + v;
        x[j + span] = mod.mul(u - v, itw[m + (c << (R - 1 - t)) + (j >> (t + 1))]);
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < E; ++j)
      a[PADX(base + j * h)] = FIN ? mod.canon(mod.mul(mod.red(x[j]), ninv)) : mod.red(x[j]);
  }
  HERS_SYNC();
}

// Stages s_begin .. logn - 1 of the forward transform below, on the values its
// earlier passes stored; output in [0, q).
template <int RMAX = 4>
HD void ntt_forward_b_from(double* a, const double* tw, ModQB mod, uint32_t n, uint32_t logn, uint32_t s_begin,
                           uint32_t tid, uint32_t nthr, uint32_t rmax = 4) {
  if (rmax > (uint32_t)RMAX) rmax = RMAX;
  uint32_t s0 = s_begin;
  while (s0 < logn) {
    const uint32_t r = logn - s0 < rmax ? logn - s0 : rmax;
    if (s0 + r < logn) {
      switch (r) {
        case 4: if constexpr (RMAX >= 4) ntt_fwd_pass_b<4>(a, tw, mod, n, s0, tid, nthr); break;
        case 3: ntt_fwd_pass_b<3>(a, tw, mod, n, s0, tid, nthr); break;
        case 2: ntt_fwd_pass_b<2>(a, tw, mod, n, s0, tid, nthr); break;
        default: ntt_fwd_pass_b<1>(a, tw, mod, n, s0, tid, nthr); break;
      }
    } else {                                          // the last pass stores values in [0, q)
      switch (r) {
        case 4: if constexpr (RMAX >= 4) ntt_fwd_pass_b<4, true>(a, tw, mod, n, s0, tid, nthr); break;
        case 3: ntt_fwd_pass_b<3, true>(a, tw, mod, n, s0, tid, nthr); break;
        case 2: ntt_fwd_pass_b<2, true>(a, tw, mod, n, s0, tid, nthr); break;
        default: ntt_fwd_pass_b<1, true>(a, tw, mod, n, s0, tid, nthr); break;
      }
    }
    s0 += r;
  }
  if (s_begin >= logn) {
    for (uint32_t j = tid; j < n; j += nthr) a[PADX(j)] = mod.canon(a[PADX(j)]);
    HERS_SYNC();
  }
}

// Forward transform of values in [0, q) (or of magnitude <= q); output in [0, q).
template <int RMAX = 4>
HD void ntt_forward_b(double* a, const double* tw, ModQB mod, uint32_t n, uint32_t logn, uint32_t tid,
                      uint32_t nthr, uint32_t rmax = 4) {
  ntt_forward_b_from<RMAX>(a, tw, mod, n, logn, 0, tid, nthr, rmax);
}

// Inverse transform scaled by n^-1 (ninv in [0, q)) of values of magnitude
// <= q; output in [0, q).
template <int RMAX = 4>
HD void ntt_inverse_b(double* a, const double* itw, double ninv, ModQB mod, uint32_t n, uint32_t logn,
                      uint32_t tid, uint32_t nthr, uint32_t rmax = 4) {
  if (rmax > (uint32_t)RMAX) rmax = RMAX;
  uint32_t lh0 = 0;
  while (lh0 < logn) {
    const uint32_t r = logn - lh0 < rmax ? logn - lh0 : rmax;
    if (lh0 + r < logn) {
      switch (r) {
        case 4: if constexpr (RMAX >= 4) ntt_inv_pass_b<4>(a, itw, mod, n, lh0, tid, nthr); break;
        case 3: ntt_inv_pass_b<3>(a, itw, mod, n, lh0, tid, nthr); break;
        case 2: ntt_inv_pass_b<2>(a, itw, mod, n, lh0, tid, nthr); break;
        default: ntt_inv_pass_b<1>(a, itw, mod, n, lh0, tid, nthr); break;
      }
    } else {                                          // the last pass stores scaled values in [0, q)
      switch (r) {
        case 4: if constexpr (RMAX >= 4) ntt_inv_pass_b<4, true>(a, itw, mod, n, lh0, tid, nthr, ninv); break;
        case 3: ntt_inv_pass_b<3, true>(a, itw, mod, n, lh0, tid, nthr, ninv); break;
        case 2: ntt_inv_pass_b<2, true>(a, itw, mod, n, lh0, tid, nthr, ninv); break;
        default: ntt_inv_pass_b<1, true>(a, itw, mod, n, lh0, tid, nthr, ninv); break;
      }
    }
    lh0 += r;
  }
  if (logn == 0) {
    for (uint32_t j = tid; j < n; j += nthr) a[PADX(j)] = mod.canon(mod.mul(a[PADX(j)], ninv));
    HERS_SYNC();
  }
}

// The inverse transform's stages of half 2^0 .. 2^(lh_end - 1), without the
// scaling: the passes before a last pass that the caller runs itself.
template <int RMAX = 4>
HD void ntt_inverse_b_upto(double* a, const double* itw, ModQB mod, uint32_t n, uint32_t lh_end, uint32_t tid,
                           uint32_t nthr, uint32_t rmax = 4) {
  if (rmax > (uint32_t)RMAX) rmax = RMAX;
  uint32_t lh0 = 0;
  while (lh0 < lh_end) {
    const uint32_t r = lh_end - lh0 < rmax ? lh_end - lh0 : rmax;
    switch (r) {
      case 4: if constexpr (RMAX >= 4) ntt_inv_pass_b<4>(a, itw, mod, n, lh0, tid, nthr); break;
      case 3: ntt_inv_pass_b<3>(a, itw, mod, n, lh0, tid, nthr); break;
      case 2: ntt_inv_pass_b<2>(a, itw, mod, n, lh0, tid, nthr); break;
      default: ntt_inv_pass_b<1>(a, itw, mod, n, lh0, tid, nthr); break;
    }
    lh0 += r;
  }
}

// ---- balanced passes in registers, at the edges of a transform
// With n / 2^R lanes, the elements tid + j n / 2^R (j < 2^R) of lane tid are
// exactly those of one virtual thread of the first forward pass (stages
// 0 .. R-1) and of the last inverse pass (halves n / 2^R .. n / 2).  A kernel
// holding them in registers runs those passes there, which saves a round trip
// through LDS and a barrier; the butterflies and reductions are those of
// ntt_fwd_pass_b / ntt_inv_pass_b, so the values are the same.
template <int R>
HD void ntt_fwd_first_regs_b(double (&x)[1 << R], const double* tw, ModQB mod) {
  constexpr uint32_t E = 1u << R;
#pragma unroll
  for (uint32_t t = 0; t < R; ++t) {
    const uint32_t span = E >> (t + 1);
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) {
      if (j & span) continue;
      const double v = mod.mul(x[j + span], tw[(1u << t) + j / (2 * span)]);
      const double u = x[j];
      x[j] = u + v;
      x[j + span] = u - v;
    }
  }
#pragma unroll
  for (uint32_t j = 0; j < E; ++j) x[j] = mod.red(x[j]);
}

// The last inverse pass on values stored by the earlier passes, scaled by
// ninv: output in [0, q).
template <int R>
HD void ntt_inv_last_regs_b(double (&x)[1 << R], const double* itw, double ninv, ModQB mod) {
  constexpr uint32_t E = 1u << R;
#pragma unroll
  for (uint32_t t = 0; t < R; ++t) {
    const uint32_t span = 1u << t;
#pragma unroll
    for (uint32_t j = 0; j < E; ++j) {
      if (j & span) continue;
      const double u = x[j], v = x[j + span];
      x[j] = u + v;
      x[j + span] = mod.mul(u - v, itw[(E >> (t + 1)) + (j >> (t + 1))]);
    }
  }
#pragma unroll
  for (uint32_t j = 0; j < E; ++j) x[j] = mod.canon(mod.mul(mod.red(x[j]), ninv));
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
