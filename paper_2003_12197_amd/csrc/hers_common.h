// hers_common.h -- constants layout and modular arithmetic shared by the host
// precompute and the gfx950 kernels of libhers.
//
// Moduli
//   q_i  ciphertext primes (App. A: R_q = Z_q[x]/(x^n+1)), 30..61 bits, 64-bit words
//   p_r  primes < 2^30 of the exact-product base P (internal): the tensor of
//        centred representatives is exact over Z once P > 4 max|X|
//   t    plaintext prime, < 2^22
// All primes are 1 mod 2n so x^n + 1 splits and the negacyclic NTT exists.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define HD __host__ __device__ __forceinline__
#else
#define HD inline
#endif

#define HC_MAXQ 8      // ciphertext primes
#define HC_MAXP 32     // exact-product base primes
#define HC_MAXL 64     // gadget digits (evaluation keys)
#define HC_MAXW 10     // 64-bit words of the rescale's fixed-point fractions

typedef unsigned __int128 u128;

// Per-context constants, resident in device memory and read with uniform
// indices (scalar loads).  "sh" = Shoup companion floor(w 2^W / m), W = 32 or 64.
struct HersConsts {
  uint32_t n, logn, k, K, L, w_bits, t;
  uint32_t dig_one_sub;                // 1: every gadget digit is below 2 q_i for every i (one subtraction reduces it)

  // ---- ciphertext primes q_i
  uint64_t q[HC_MAXQ];
  uint64_t q_mu64[HC_MAXQ];            // floor(2^64 / q_i)
  uint64_t q_m128h[HC_MAXQ];           // floor(2^128 / q_i), high word
  uint64_t q_m128l[HC_MAXQ];           //                      low word
  uint64_t q_bar[HC_MAXQ];             // floor(2^(2 beta) / q_i), beta = bit length
  uint32_t q_beta[HC_MAXQ];
  uint64_t q_r64[HC_MAXQ], q_r64_sh[HC_MAXQ];        // 2^64 mod q_i
  uint64_t q_ninv[HC_MAXQ], q_ninv_sh[HC_MAXQ];      // n^-1 mod q_i
  uint64_t q_delta[HC_MAXQ], q_delta_sh[HC_MAXQ];    // Delta = floor(q/t) mod q_i
  uint64_t q_hatinv[HC_MAXQ], q_hatinv_sh[HC_MAXQ];  // (q/q_i)^-1 mod q_i
  uint64_t q_t[HC_MAXQ], q_t_sh[HC_MAXQ];            // t mod q_i
  uint64_t garner[HC_MAXQ][HC_MAXQ];                 // [i][j]: q_j^-1 mod q_i, j < i
  uint64_t garner_sh[HC_MAXQ][HC_MAXQ];
  uint64_t half_digit[HC_MAXQ];                      // mixed-radix digits of (q-1)/2
  // rescale constants: t (P/p_r) / q = I_r + phi_r and t P / q = J + psi,
  // integer parts modulo q_i, fractions in fr_words 64-bit words (little-endian)
  uint64_t fr_I[HC_MAXP][HC_MAXQ];                   // I_r mod q_i
  uint64_t fr_J[HC_MAXQ], fr_J_sh[HC_MAXQ];          // J mod q_i
  uint64_t fr_phi[HC_MAXP][HC_MAXW];
  uint64_t fr_psi[HC_MAXW];
  uint32_t fr_words, pad2;

  // ---- exact-product base primes p_r
  uint32_t p[HC_MAXP];
  uint64_t p_mu64[HC_MAXP];                          // floor(2^64 / p_r)
  uint32_t p_ninv[HC_MAXP], p_ninv_sh[HC_MAXP];
  uint32_t p_hatinv[HC_MAXP], p_hatinv_sh[HC_MAXP];  // (P/p_r)^-1 mod p_r
  double   p_inv[HC_MAXP];                           // 1 / p_r
  uint32_t Qw_p[HC_MAXQ][HC_MAXP];                   // (q_0 ... q_{i-1}) mod p_r
  uint32_t Qw_p_sh[HC_MAXQ][HC_MAXP];
  uint32_t qmod_p[HC_MAXP];                          // q mod p_r
  uint32_t p_r64[HC_MAXP], p_r64_sh[HC_MAXP];        // 2^64 mod p_r
  uint64_t phat_q[HC_MAXP][HC_MAXQ];                 // (P / p_r) mod q_i
  uint64_t P_q[HC_MAXQ];                             // P mod q_i

  // ---- plaintext prime t
  uint64_t t_mu64;                                   // floor(2^64 / t)
  uint32_t t_ninv, t_ninv_sh;
  uint32_t Qw_t[HC_MAXQ], Qw_t_sh[HC_MAXQ];          // (q_0 ... q_{i-1}) mod t
  uint32_t qmod_t, qinv_t, qinv_t_sh, pad1;
  // decryption by fractions: dec_c[i] = floor(t 2^64 / q_i); the rounded
  // fixed-point sum is taken while its low word is below dec_lo_max =
  // 2^64 - sum_i q_i (0: never)
  uint64_t dec_c[HC_MAXQ];
  uint64_t dec_lo_max;

  // ---- gadget (relinearization digits), key order
  uint32_t g_rho[HC_MAXL], g_shift[HC_MAXL];
  uint64_t g_val[HC_MAXL][HC_MAXQ];                  // g mod q_i
  uint64_t g_val_sh[HC_MAXL][HC_MAXQ];
};

// ============================================================== 32-bit moduli

HD uint32_t mulhi32(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }
HD uint64_t mulhi64(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a * b) >> 64); }

HD uint32_t add_p(uint32_t a, uint32_t b, uint32_t p) { uint32_t s = a + b; return s >= p ? s - p : s; }
HD uint32_t sub_p(uint32_t a, uint32_t b, uint32_t p) { return a >= b ? a - b : a + p - b; }

// a * w mod p for a < 2^32, w < p < 2^31, wsh = floor(w 2^32 / p) (Shoup).
HD uint32_t shoup_p(uint32_t a, uint32_t w, uint32_t wsh, uint32_t p) {
  uint32_t qh = mulhi32(a, wsh);
  uint32_t r = a * w - qh * p;
  return r >= p ? r - p : r;
}

// x mod p for any 64-bit x, mu = floor(2^64 / p), p < 2^31.
HD uint32_t red_p(uint64_t x, uint32_t p, uint64_t mu) {
  uint64_t qh = mulhi64(x, mu);
  uint64_t r = x - qh * (uint64_t)p;
  return (uint32_t)(r >= p ? r - p : r);
}

// ============================================================== 64-bit moduli

HD uint64_t add_q(uint64_t a, uint64_t b, uint64_t q) { uint64_t s = a + b; return s >= q ? s - q : s; }
HD uint64_t sub_q(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }

// a * w mod q for a < 2^64, w < q < 2^63, wsh = floor(w 2^64 / q) (Shoup).
HD uint64_t shoup_q(uint64_t a, uint64_t w, uint64_t wsh, uint64_t q) {
  uint64_t qh = mulhi64(a, wsh);
  uint64_t r = a * w - qh * q;
  return r >= q ? r - q : r;
}

// x mod q for any 64-bit x, mu = floor(2^64 / q).
HD uint64_t red_q(uint64_t x, uint64_t q, uint64_t mu) {
  uint64_t qh = mulhi64(x, mu);
  uint64_t r = x - qh * q;
  return r >= q ? r - q : r;
}

// Barrett reduction of x < 2^(2 beta), q of bit length beta <= 62,
// mu = floor(2^(2 beta) / q) (Handbook of Applied Cryptography, Alg. 14.42).
HD uint64_t barrett_q(u128 x, uint64_t q, uint64_t mu, uint32_t beta) {
  uint64_t q1 = (uint64_t)(x >> (beta - 1));
  uint64_t q3 = (uint64_t)(((u128)q1 * mu) >> (beta + 1));
  uint64_t r = (uint64_t)x - q3 * q;
  if (r >= q) r -= q;
  if (r >= q) r -= q;
  return r;
}

HD uint64_t mul_q(uint64_t a, uint64_t b, uint64_t q, uint64_t mu, uint32_t beta) {
  return barrett_q((u128)a * b, q, mu, beta);
}

// Shoup companion floor(w 2^64 / q) for w < q < 2^63, from M = floor(2^128 / q).
HD uint64_t shoup_companion_q(uint64_t w, uint64_t q, uint64_t mh, uint64_t ml) {
  u128 lo = (u128)w * ml;
  u128 e = (u128)w * mh + (uint64_t)(lo >> 64);   // floor(w M / 2^64): Q - 1 or Q
  uint64_t est = (uint64_t)e;
  u128 r = ((u128)w << 64) - (u128)est * q;
  if (r >= (u128)q) est += 1;
  return est;
}

// ============================================================== Philox4x64-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): two 64x64->128 multiplies per round, ten rounds, key bumped by the
// Weyl constants between rounds.

#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

struct Philox4 { uint64_t v[4]; };

HD Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1) {
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
    uint64_t lo0 = PHILOX_M0 * c0, hi0 = mulhi64(PHILOX_M0, c0);
    uint64_t lo1 = PHILOX_M1 * c2, hi1 = mulhi64(PHILOX_M1, c2);
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  Philox4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// Domains separating the uses of one seed.
#define HERS_DOMAIN_KEYGEN 1
#define HERS_DOMAIN_GALLERY 2
#define HERS_DOMAIN_PROBE 3
#define HERS_DOMAIN_ENROLL 4
#define HERS_DOMAIN_RERANK_ITEMS 5
#define HERS_DOMAIN_RERANK_PROBE 6
#define HERS_DOMAIN_PROBE_SK 7

// Word w of object (o0, o1, o2) under key (seed, domain).
HD uint64_t philox_word(uint64_t seed, uint64_t domain, uint64_t o0, uint64_t o1, uint64_t o2, uint64_t w) {
  Philox4 b = philox4x64_10(w >> 2, o0, o1, o2, seed, domain);
  return b.v[w & 3];
}

HD int cbd20(uint64_t w) {
  const uint64_t m = (1ULL << 20) - 1;
  return __builtin_popcountll(w & m) - __builtin_popcountll((w >> 20) & m);
}

// ============================================================== exact CRT helpers

// Mixed-radix digits a_i of x in [0, q) given residues v_i = x mod q_i
// (Garner): x = a_0 + a_1 q_0 + a_2 q_0 q_1 + ..., 0 <= a_i < q_i.
// Returns whether x > (q - 1)/2, i.e. whether the centred representative of x is x - q.
template <int KQ = 0>
HD bool garner_digits(const HersConsts& C, const uint64_t* v, uint64_t* a) {
  const uint32_t k = KQ ? KQ : C.k;
  for (uint32_t i = 0; i < k; ++i) {
    const uint64_t qi = C.q[i];
    uint64_t acc = v[i];
    for (uint32_t j = 0; j < i; ++j) {
      uint64_t aj = a[j] >= qi ? red_q(a[j], qi, C.q_mu64[i]) : a[j];
      acc = sub_q(acc, aj, qi);
      acc = shoup_q(acc, C.garner[i][j], C.garner_sh[i][j], qi);
    }
    a[i] = acc;
  }
  for (int i = (int)k - 1; i >= 0; --i)
    if (a[i] != C.half_digit[i]) return a[i] > C.half_digit[i];
  return false;
}

// x mod p_r for x < 2^96 (high word below 2^32).
HD uint32_t red128_p(const HersConsts& C, u128 x, uint32_t r) {
  const uint32_t p = C.p[r];
  const uint32_t lo = red_p((uint64_t)x, p, C.p_mu64[r]);
  const uint32_t hi = shoup_p((uint32_t)(uint64_t)(x >> 64), C.p_r64[r], C.p_r64_sh[r], p);
  return add_p(lo, hi, p);
}

// x mod q_i for any 128-bit x.
HD uint64_t red128_q(const HersConsts& C, u128 x, uint32_t i) {
  const uint64_t q = C.q[i];
  const uint64_t lo = red_q((uint64_t)x, q, C.q_mu64[i]);
  const uint64_t hi = shoup_q((uint64_t)(x >> 64), C.q_r64[i], C.q_r64_sh[i], q);
  return add_q(lo, hi, q);
}

// Centred representative of the mixed-radix number (a, neg) modulo p_r.
// sum_i a_i Qw_i < k 2^92: accumulated exactly, reduced once.
template <int KQ = 0>
HD uint32_t mixed_to_p(const HersConsts& C, const uint64_t* a, bool neg, uint32_t r) {
  const uint32_t p = C.p[r];
  const uint32_t k = KQ ? KQ : C.k;
  u128 acc = 0;
  for (uint32_t i = 0; i < k; ++i) acc += (u128)a[i] * C.Qw_p[i][r];
  const uint32_t v = red128_p(C, acc, r);
  return neg ? sub_p(v, C.qmod_p[r], p) : v;
}

// Centred representative of (a, neg) modulo t.
template <int KQ = 0>
HD uint32_t mixed_to_t(const HersConsts& C, const uint64_t* a, bool neg) {
  const uint32_t t = C.t;
  uint32_t acc = 0;
  for (uint32_t i = 0; i < (KQ ? KQ : C.k); ++i) {
    uint32_t ai = red_p(a[i], t, C.t_mu64);
    acc = add_p(acc, shoup_p(ai, C.Qw_t[i], C.Qw_t_sh[i], t), t);
  }
  return neg ? sub_p(acc, C.qmod_t, t) : acc;
}

// Scale and round of one coefficient (Alg. "Ciphertext Multiplication"):
// given x_r = X mod p_r of an integer X with |X| < P/4, returns
// c_i = [round(t X / q)]_q mod q_i.
// With y_r = [x_r (P/p_r)^-1]_{p_r}, X = sum_r y_r (P/p_r) - gamma P, where
// gamma is the nearest integer to sum_r y_r / p_r (the quarter of headroom
// covers the double-precision error).  Hence
//   t X / q = sum_r y_r (I_r + phi_r) - gamma (J + psi),
// I_r, J integers and phi_r, psi in [0, 1), and
//   round(t X / q) = sum_r y_r I_r - gamma J + round(F),  F = sum_r y_r phi_r - gamma psi.
// F is formed in fixed point with 64 fr_words fraction bits, truncated
// fractions: the error is below max(sum_r y_r, gamma) 2^-(64 fr_words), less
// than 1/(2q), while t X / q (denominator q, odd) is at least 1/(2q) away from
// every half-integer, so the rounding is exact.
// KQ, KP, FW fix k, K and fr_words at compile time (0 = read from C), so
// the fixed-point words stay in statically indexed registers.
//
// Short form: the same sum over the top two fraction words only (words
// w0 .. W-1 with w0 = W - 2) differs from the W-word F by less than
// max(sum_r y_r, gamma) 2^-128 < 2^-93.  When its fraction is more than 2^-64
// away from 1/2, it rounds as the W-word F does; only a fraction within 2^-64
// of 1/2 (probability about 2^-63 per coefficient) takes the W-word sum.
template <int FW = 0>
HD int64_t round_F(const HersConsts& C, const uint32_t* y, uint32_t K, uint64_t gamma, uint32_t W, uint32_t w0,
                   bool* near_half) {
  // F in fixed point: f[0 .. W-1] fraction words, f[W] the integer part (two's complement)
  uint64_t f[(FW ? FW : HC_MAXW) + 1];
#pragma unroll
  for (uint32_t w = 0; w <= W; ++w) f[w] = 0;
#pragma unroll
  for (uint32_t r = 0; r < K; ++r) {
    uint64_t carry = 0;
#pragma unroll
    for (uint32_t w = w0; w < W; ++w) {
      const u128 v = (u128)y[r] * C.fr_phi[r][w] + f[w] + carry;
      f[w] = (uint64_t)v;
      carry = (uint64_t)(v >> 64);
    }
    f[W] += carry;
  }
  {
    uint64_t carry = 0, borrow = 0;
#pragma unroll
    for (uint32_t w = w0; w < W; ++w) {
      const u128 g = (u128)gamma * C.fr_psi[w] + carry;
      carry = (uint64_t)(g >> 64);
      const uint64_t gl = (uint64_t)g;
      const uint64_t d = f[w] - gl - borrow;
      borrow = (f[w] < gl || (f[w] == gl && borrow)) ? 1 : 0;
      f[w] = d;
    }
    f[W] -= carry + borrow;
  }
  // fraction in [1/2 - 2^-64, 1/2 + 2^-64): top word 2^63 - 1 or 2^63
  *near_half = f[W - 1] - ((1ull << 63) - 1) < 2;
  return (int64_t)f[W] + (int64_t)(f[W - 1] >> 63);   // round(F)
}

// ALL = false takes the two-word form and returns true when its fraction is
// within 2^-64 of 1/2: the caller then calls again with ALL = true (W words).
template <int KQ = 0, int KP = 0, int FW = 0, bool ALL = false>
HD bool scale_round_coeff(const HersConsts& C, const uint32_t* x, uint64_t* out) {
  const uint32_t k = KQ ? KQ : C.k, K = KP ? KP : C.K, W = FW ? FW : C.fr_words;
  uint32_t y[KP ? KP : HC_MAXP];
  double s = 0.0;
#pragma unroll
  for (uint32_t r = 0; r < K; ++r) {
    y[r] = shoup_p(x[r], C.p_hatinv[r], C.p_hatinv_sh[r], C.p[r]);
    s += (double)y[r] * C.p_inv[r];
  }
  const uint64_t gamma = (uint64_t)__builtin_rint(s);
  const uint32_t w0 = ALL || W <= 2 ? 0 : W - 2;
  bool near_half = false;
  const int64_t rf = round_F<FW>(C, y, K, gamma, W, w0, &near_half);
#pragma unroll
  for (uint32_t i = 0; i < k; ++i) {
    const uint64_t q = C.q[i];
    // sum_r y_r (I_r mod q_i) - gamma (J mod q_i) + round(F), offset by 2^8 q_i and reduced once:
    // gamma <= K <= 32 and |round(F)| < K 2^30 <= 2^35 < 224 q_i (q_i > 2^29), so the sum is
    // positive, and below 2^8 2^61 + K 2^91 + 2^35 < 2^97
    u128 acc = ((u128)q << 8) - (u128)gamma * C.fr_J[i] + (u128)(__int128)rf;
#pragma unroll
    for (uint32_t r = 0; r < K; ++r) acc += (u128)y[r] * C.fr_I[r][i];
    out[i] = red128_q(C, acc, i);
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_sched_barrier(0);
#endif
  }
  return w0 != 0 && near_half;
}

// Decryption scale (Alg. "Decryption"): given x mod q_i of x = [c0 + c1 s]_q,
// returns [round(t x / q)]_t in [0, t): with t x = q Y + T as above, Y = -T q^-1 mod t.
// Exact CRT form (Garner digits of t x, its centred representative).
template <int KQ = 0>
HD uint32_t decrypt_coeff_exact(const HersConsts& C, const uint64_t* x) {
  uint64_t tx[KQ ? KQ : HC_MAXQ], a[KQ ? KQ : HC_MAXQ];
  for (uint32_t i = 0; i < (KQ ? KQ : C.k); ++i) tx[i] = shoup_q(x[i], C.q_t[i], C.q_t_sh[i], C.q[i]);
  const bool neg = garner_digits<KQ>(C, tx, a);
  uint32_t T = mixed_to_t<KQ>(C, a, neg);
  uint32_t y = shoup_p(T, C.qinv_t, C.qinv_t_sh, C.t);
  return y ? C.t - y : 0;
}

// The same value from fractions.  With y_i = [x_i (q/q_i)^-1]_{q_i},
// x = sum_i y_i q/q_i - a q for an integer 0 <= a < k, so
// t x / q = sum_i y_i t / q_i - a t and round(t x / q) = round(S) mod t,
// S = sum_i y_i t / q_i (each term below t).  With c_i = floor(t 2^64 / q_i),
// A = sum_i y_i c_i (exact in 128 bits) lies below 2^64 S by less than
// sum_i y_i < sum_i q_i, so for B = A + 2^63 the value floor(B / 2^64) is
// round(S) whenever B mod 2^64 < 2^64 - sum_i q_i (no carry can be missing).
// Returns false, leaving *v unset, when that low word is too close to the
// carry (never for the small noise of a valid ciphertext: t x / q is then
// close to an integer, so B mod 2^64 is close to 1/2).
template <int KQ = 0>
HD bool decrypt_coeff_frac(const HersConsts& C, const uint64_t* x, uint32_t* v) {
  u128 B = (u128)1 << 63;
#pragma unroll
  for (uint32_t i = 0; i < (KQ ? KQ : C.k); ++i)
    B += (u128)shoup_q(x[i], C.q_hatinv[i], C.q_hatinv_sh[i], C.q[i]) * C.dec_c[i];
  if ((uint64_t)B >= C.dec_lo_max) return false;
  *v = red_p((uint64_t)(B >> 64), C.t, C.t_mu64);
  return true;
}

template <int KQ = 0>
HD uint32_t decrypt_coeff(const HersConsts& C, const uint64_t* x) {
  uint32_t v;
  if (decrypt_coeff_frac<KQ>(C, x, &v)) return v;
  return decrypt_coeff_exact<KQ>(C, x);
}
