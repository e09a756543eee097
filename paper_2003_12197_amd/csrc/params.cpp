// params.cpp -- prime selection, roots of unity, NTT tables and the constants
// of the exact base conversions (host only).
//
// Prime rule (the paper fixes n = 4096, t = 1,032,193 and three 36-bit primes
// in q, Sec. 4.1, but not how they are chosen): for each requested width b,
// the largest prime below 2^b that is 1 mod 2n and not yet taken; t the
// largest such prime below 2^t_bits.  The exact-product base P takes the
// largest primes below 2^30 that are 1 mod 2n, as many as needed for
// P > 4 max|X|, X a coefficient of sum_i of d_max products of centred
// representatives: |X| <= 2 d_max n ((q-1)/2)^2.
#include "params.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace hers {

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod(r, a, m);
    a = mulmod(a, a, m);
    e >>= 1;
  }
  return r;
}

static uint64_t invmod(uint64_t a, uint64_t p) { return powmod(a % p, p - 2, p); }  // p prime

bool is_prime_u64(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : small) {
    if (n % p == 0) return n == p;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  // deterministic Miller-Rabin for n < 3.3e24 with the first 12 prime bases
  for (uint64_t a : small) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = mulmod(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

static bool taken(const std::vector<uint64_t>& v, uint64_t p) {
  for (uint64_t x : v) if (x == p) return true;
  return false;
}

// Largest prime below 2^bits, 1 mod two_n, not in `used`; 0 if none.
static uint64_t ntt_prime(uint32_t bits, uint64_t two_n, const std::vector<uint64_t>& used) {
  uint64_t top = (bits >= 64) ? ~0ULL : ((1ULL << bits) - 1);
  uint64_t p = top / two_n * two_n + 1;
  if (p > top) p -= two_n;
  while (p > two_n) {
    if (!taken(used, p) && is_prime_u64(p)) return p;
    p -= two_n;
  }
  return 0;
}

static uint64_t smallest_generator(uint64_t p) {
  std::vector<uint64_t> f;
  uint64_t m = p - 1;
  for (uint64_t d = 2; d * d <= m; ++d) {
    if (m % d == 0) {
      f.push_back(d);
      while (m % d == 0) m /= d;
    }
  }
  if (m > 1) f.push_back(m);
  for (uint64_t g = 2; g < p; ++g) {
    bool ok = true;
    for (uint64_t x : f)
      if (powmod(g, (p - 1) / x, p) == 1) { ok = false; break; }
    if (ok) return g;
  }
  return 0;
}

// A primitive 2n-th root of unity: psi^n = -1.
static uint64_t root_2n(uint64_t p, uint64_t two_n) {
  for (uint64_t g = 2; g < p; ++g) {
    uint64_t c = powmod(g, (p - 1) / two_n, p);
    if (powmod(c, two_n / 2, p) == p - 1) return c;
  }
  return 0;
}

static uint32_t bitrev(uint32_t x, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

static uint64_t sh64(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }
static uint32_t sh32(uint32_t w, uint32_t p) { return (uint32_t)(((uint64_t)w << 32) / p); }

// ---- unsigned multi-word integers for the rescale constants (little-endian
// 32-bit limbs, no leading zero limbs)
struct Big {
  std::vector<uint32_t> w;
};

static void big_trim(Big& a) {
  while (!a.w.empty() && !a.w.back()) a.w.pop_back();
}

static Big big_from(uint64_t v) {
  Big a;
  a.w = {(uint32_t)v, (uint32_t)(v >> 32)};
  big_trim(a);
  return a;
}

static Big big_mul(const Big& a, const Big& b) {
  Big c;
  c.w.assign(a.w.size() + b.w.size() + 1, 0);
  for (size_t i = 0; i < a.w.size(); ++i) {
    uint64_t carry = 0;
    for (size_t j = 0; j < b.w.size(); ++j) {
      const uint64_t v = (uint64_t)a.w[i] * b.w[j] + c.w[i + j] + carry;
      c.w[i + j] = (uint32_t)v;
      carry = v >> 32;
    }
    for (size_t j = i + b.w.size(); carry; ++j) {
      const uint64_t v = (uint64_t)c.w[j] + carry;
      c.w[j] = (uint32_t)v;
      carry = v >> 32;
    }
  }
  big_trim(c);
  return c;
}

static size_t big_bits(const Big& a) {
  return a.w.empty() ? 0 : 32 * (a.w.size() - 1) + (32 - __builtin_clz(a.w.back()));
}

static bool big_bit(const Big& a, size_t i) { return i / 32 < a.w.size() && ((a.w[i / 32] >> (i % 32)) & 1); }

static Big big_shl(const Big& a, size_t bits) {
  Big c;
  c.w.assign(a.w.size() + bits / 32 + 1, 0);
  for (size_t i = 0; i < a.w.size(); ++i) {
    const uint64_t v = (uint64_t)a.w[i] << (bits % 32);
    c.w[i + bits / 32] |= (uint32_t)v;
    c.w[i + bits / 32 + 1] |= (uint32_t)(v >> 32);
  }
  big_trim(c);
  return c;
}

static int big_cmp(const Big& a, const Big& b) {
  if (a.w.size() != b.w.size()) return a.w.size() < b.w.size() ? -1 : 1;
  for (size_t i = a.w.size(); i-- > 0;)
    if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
  return 0;
}

static void big_sub_in(Big& a, const Big& b) {   // a -= b, a >= b
  int64_t borrow = 0;
  for (size_t i = 0; i < a.w.size(); ++i) {
    int64_t v = (int64_t)a.w[i] - (i < b.w.size() ? (int64_t)b.w[i] : 0) - borrow;
    borrow = v < 0;
    a.w[i] = (uint32_t)(v + (borrow << 32));
  }
  big_trim(a);
}

// quotient and remainder of a / b (b > 0), one bit at a time
static void big_divmod(const Big& a, const Big& b, Big* q, Big* r) {
  Big quo, rem;
  quo.w.assign(a.w.size() + 1, 0);
  for (size_t i = big_bits(a); i-- > 0;) {
    rem = big_shl(rem, 1);
    if (big_bit(a, i)) {
      if (rem.w.empty()) rem.w.push_back(0);
      rem.w[0] |= 1;
    }
    if (big_cmp(rem, b) >= 0) {
      big_sub_in(rem, b);
      quo.w[i / 32] |= 1u << (i % 32);
    }
  }
  big_trim(quo);
  *q = quo;
  *r = rem;
}

static uint64_t big_mod_small(const Big& a, uint64_t m) {
  u128 v = 0;
  for (size_t i = a.w.size(); i-- > 0;) v = ((v << 32) | a.w[i]) % m;
  return (uint64_t)v;
}

static uint64_t big_word64(const Big& a, size_t w) {
  const uint64_t lo = 2 * w < a.w.size() ? a.w[2 * w] : 0, hi = 2 * w + 1 < a.w.size() ? a.w[2 * w + 1] : 0;
  return lo | (hi << 32);
}

std::string resolve(const hers_params& prm, hers_info* info) {
  std::memset(info, 0, sizeof(*info));
  const uint32_t n = prm.n;
  if (n < 256 || n > 8192 || (n & (n - 1))) return "n must be a power of two in [256, 8192]";
  if (prm.k < 1 || prm.k > HERS_MAX_QPRIMES) return "k must be in [1, 8]";
  if (prm.t_bits < 12 || prm.t_bits > 22) return "t_bits must be in [12, 22]";
  if (prm.d_max < 1 || prm.d_max > 1024) return "d_max must be in [1, 1024]";
  const uint64_t two_n = 2ULL * n;
  uint64_t t = ntt_prime(prm.t_bits, two_n, {});
  if (!t) return "no plaintext prime";
  std::vector<uint64_t> used{t};
  double log2q = 0;
  for (uint32_t i = 0; i < prm.k; ++i) {
    if (prm.qbits[i] < 30 || prm.qbits[i] > 61) return "qbits must be in [30, 61]";
    uint64_t p = ntt_prime(prm.qbits[i], two_n, used);
    if (!p) return "no ciphertext prime of the requested width";
    used.push_back(p);
    info->q[i] = p;
    log2q += std::log2((double)p);
  }
  info->n = n;
  info->k = prm.k;
  info->t = t;
  info->log2_q = log2q;
  // feature range guard: every score must be recovered exactly modulo t
  if ((double)prm.d_max * prm.feature_bound * prm.feature_bound >= (double)t / 2)
    return "d_max * feature_bound^2 must be below t/2";
  // gadget digits
  uint32_t L = 0;
  for (uint32_t i = 0; i < prm.k; ++i) {
    uint32_t bits = 64 - __builtin_clzll(info->q[i]);
    L += prm.w_bits ? (bits + prm.w_bits - 1) / prm.w_bits : 1;
  }
  if (L > HC_MAXL) return "too many relinearization digits";
  info->num_digits = L;
  // exact-product base: log2 P > log2(4 * 2 d_max n ((q-1)/2)^2) with one bit of slack
  const double need = 3.0 + std::log2((double)prm.d_max) + std::log2((double)n) + 2.0 * (log2q - 1.0) + 1.0;
  double have = 0;
  uint32_t K = 0;
  while (have < need) {
    if (K >= HC_MAXP) return "exact-product base would need more than 32 primes";
    uint64_t p = ntt_prime(30, two_n, used);
    if (!p) return "ran out of 30-bit NTT primes";
    used.push_back(p);
    info->aux[K++] = p;
    have += std::log2((double)p);
  }
  info->num_aux = K;
  info->log2_aux = have;
  info->d_max = prm.d_max;
  info->feature_bound = prm.feature_bound;
  return "";
}

std::string precompute(const hers_params& prm, HostTables* T) {
  hers_info info;
  std::string err = resolve(prm, &info);
  if (!err.empty()) return err;
  T->info = info;
  HersConsts& C = T->C;
  std::memset(&C, 0, sizeof(C));
  const uint32_t n = info.n, k = info.k, K = info.num_aux;
  uint32_t logn = 0;
  while ((1u << logn) < n) ++logn;
  C.n = n; C.logn = logn; C.k = k; C.K = K; C.L = info.num_digits; C.w_bits = prm.w_bits;
  {
    // a digit is below 2^w_bits, or (one digit per prime) below its prime: one conditional
    // subtraction reduces it mod q_i when that bound is below 2 q_i for every i
    uint64_t qmin = info.q[0], qmax = info.q[0];
    for (uint32_t i = 1; i < k; ++i) { qmin = std::min<uint64_t>(qmin, info.q[i]); qmax = std::max<uint64_t>(qmax, info.q[i]); }
    const uint64_t dmax = prm.w_bits ? (prm.w_bits >= 63 ? ~0ull : (1ull << prm.w_bits)) : qmax;
    C.dig_one_sub = dmax <= 2 * qmin ? 1u : 0u;
  }
  const uint64_t t = info.t;
  C.t = (uint32_t)t;
  const uint64_t two_n = 2ULL * n;

  // ---- ciphertext primes
  uint64_t q_mod_t = 1;
  for (uint32_t i = 0; i < k; ++i) q_mod_t = mulmod(q_mod_t, info.q[i] % t, t);
  for (uint32_t i = 0; i < k; ++i) {
    const uint64_t q = info.q[i];
    C.q[i] = q;
    C.q_mu64[i] = (uint64_t)(((u128)1 << 64) / q);
    u128 m128 = (~(u128)0) / q;
    C.q_m128h[i] = (uint64_t)(m128 >> 64);
    C.q_m128l[i] = (uint64_t)m128;
    uint32_t beta = 64 - __builtin_clzll(q);
    C.q_beta[i] = beta;
    C.q_bar[i] = (uint64_t)(((u128)1 << (2 * beta)) / q);
    C.q_r64[i] = (uint64_t)(((u128)1 << 64) % q);
    C.q_r64_sh[i] = sh64(C.q_r64[i], q);
    C.q_ninv[i] = invmod(n, q);
    C.q_ninv_sh[i] = sh64(C.q_ninv[i], q);
    // Delta = floor(q/t): Delta t = q - (q mod t) = -(q mod t) (mod q_i)
    C.q_delta[i] = mulmod((q - q_mod_t % q) % q, invmod(t, q), q);
    C.q_delta_sh[i] = sh64(C.q_delta[i], q);
    uint64_t qhat = 1;
    for (uint32_t j = 0; j < k; ++j) if (j != i) qhat = mulmod(qhat, info.q[j] % q, q);
    C.q_hatinv[i] = invmod(qhat, q);
    C.q_hatinv_sh[i] = sh64(C.q_hatinv[i], q);
    C.q_t[i] = t % q;
    C.q_t_sh[i] = sh64(C.q_t[i], q);
    for (uint32_t j = 0; j < i; ++j) {
      C.garner[i][j] = invmod(info.q[j] % q, q);
      C.garner_sh[i][j] = sh64(C.garner[i][j], q);
    }
  }
  // mixed-radix digits of (q - 1)/2, whose residue mod q_i is (q_i - 1)/2
  {
    uint64_t v[HC_MAXQ], a[HC_MAXQ];
    for (uint32_t i = 0; i < k; ++i) v[i] = (info.q[i] - 1) / 2;
    for (uint32_t i = 0; i < k; ++i) {
      uint64_t acc = v[i];
      for (uint32_t j = 0; j < i; ++j) {
        uint64_t aj = a[j] % info.q[i];
        acc = (acc + info.q[i] - aj) % info.q[i];
        acc = mulmod(acc, C.garner[i][j], info.q[i]);
      }
      a[i] = acc;
    }
    for (uint32_t i = 0; i < k; ++i) C.half_digit[i] = a[i];
  }

  // ---- exact-product base primes
  for (uint32_t r = 0; r < K; ++r) {
    const uint32_t p = (uint32_t)info.aux[r];
    C.p[r] = p;
    C.p_mu64[r] = (uint64_t)(((u128)1 << 64) / p);
    C.p_ninv[r] = (uint32_t)invmod(n, p);
    C.p_ninv_sh[r] = sh32(C.p_ninv[r], p);
    uint64_t phat = 1;
    for (uint32_t s = 0; s < K; ++s) if (s != r) phat = mulmod(phat, info.aux[s] % p, p);
    C.p_hatinv[r] = (uint32_t)invmod(phat, p);
    C.p_hatinv_sh[r] = sh32(C.p_hatinv[r], p);
    C.p_inv[r] = 1.0 / (double)p;
    uint64_t qm = 1;
    for (uint32_t i = 0; i < k; ++i) {
      C.Qw_p[i][r] = (uint32_t)qm;
      C.Qw_p_sh[i][r] = sh32((uint32_t)qm, p);
      qm = mulmod(qm, info.q[i] % p, p);
    }
    C.qmod_p[r] = (uint32_t)qm;
    C.p_r64[r] = (uint32_t)(((u128)1 << 64) % p);
    C.p_r64_sh[r] = sh32(C.p_r64[r], p);
    for (uint32_t i = 0; i < k; ++i) {
      uint64_t v = 1;
      for (uint32_t s = 0; s < K; ++s) if (s != r) v = mulmod(v, info.aux[s] % info.q[i], info.q[i]);
      C.phat_q[r][i] = v;
    }
  }
  for (uint32_t i = 0; i < k; ++i) {
    uint64_t v = 1;
    for (uint32_t s = 0; s < K; ++s) v = mulmod(v, info.aux[s] % info.q[i], info.q[i]);
    C.P_q[i] = v;
  }
  // rescale constants: t (P/p_r) / q = I_r + phi_r, t P / q = J + psi, fractions
  // in W words with 64 W > log2(K 2^30) + 1 + log2 q + 2 (exactness margin)
  {
    const double need = std::log2((double)K) + 30.0 + 1.0 + info.log2_q + 2.0;
    const uint32_t W = (uint32_t)std::ceil(need / 64.0);
    if (W > HC_MAXW) return "rescale fractions would need too many words";
    C.fr_words = W;
    Big Q = big_from(1), P = big_from(1);
    for (uint32_t i = 0; i < k; ++i) Q = big_mul(Q, big_from(info.q[i]));
    for (uint32_t r = 0; r < K; ++r) P = big_mul(P, big_from(info.aux[r]));
    auto split = [&](const Big& A, uint64_t* Imod, uint64_t* frac) {
      Big I, R, F, R2;
      big_divmod(A, Q, &I, &R);
      for (uint32_t i = 0; i < k; ++i) Imod[i] = big_mod_small(I, info.q[i]);
      big_divmod(big_shl(R, 64 * W), Q, &F, &R2);
      for (uint32_t w = 0; w < W; ++w) frac[w] = big_word64(F, w);
    };
    for (uint32_t r = 0; r < K; ++r) {
      Big Pr = big_from(t);
      for (uint32_t s = 0; s < K; ++s) if (s != r) Pr = big_mul(Pr, big_from(info.aux[s]));
      split(Pr, C.fr_I[r], C.fr_phi[r]);
    }
    split(big_mul(P, big_from(t)), C.fr_J, C.fr_psi);
    for (uint32_t i = 0; i < k; ++i) C.fr_J_sh[i] = sh64(C.fr_J[i], info.q[i]);
  }

  // ---- plaintext prime
  C.t_mu64 = (uint64_t)(((u128)1 << 64) / t);
  C.t_ninv = (uint32_t)invmod(n, t);
  C.t_ninv_sh = sh32(C.t_ninv, (uint32_t)t);
  {
    uint64_t qm = 1;
    for (uint32_t i = 0; i < k; ++i) {
      C.Qw_t[i] = (uint32_t)qm;
      C.Qw_t_sh[i] = sh32((uint32_t)qm, (uint32_t)t);
      qm = mulmod(qm, info.q[i] % t, t);
    }
    C.qmod_t = (uint32_t)qm;
    C.qinv_t = (uint32_t)invmod(qm, t);
    C.qinv_t_sh = sh32(C.qinv_t, (uint32_t)t);
  }
  {
    // decryption by fractions (hers_common.h: decrypt_coeff_frac)
    u128 qs = 0;
    bool ok = true;
    for (uint32_t i = 0; i < k; ++i) {
      ok &= t < info.q[i];
      C.dec_c[i] = ok ? (uint64_t)(((u128)t << 64) / info.q[i]) : 0;
      qs += info.q[i];
    }
    C.dec_lo_max = ok && qs < ((u128)1 << 64) ? (uint64_t)(((u128)1 << 64) - qs) : 0;
  }

  // ---- gadget: digit (rho, l) has value (q/q_rho) 2^(l w) mod q, which is 0 mod q_i for i != rho
  {
    uint32_t g = 0;
    for (uint32_t rho = 0; rho < k; ++rho) {
      uint32_t bits = 64 - __builtin_clzll(info.q[rho]);
      uint32_t L = prm.w_bits ? (bits + prm.w_bits - 1) / prm.w_bits : 1;
      for (uint32_t l = 0; l < L; ++l, ++g) {
        C.g_rho[g] = rho;
        C.g_shift[g] = l * prm.w_bits;
        for (uint32_t i = 0; i < k; ++i) {
          uint64_t v = 0;
          if (i == rho) {
            uint64_t qhat = 1;
            for (uint32_t j = 0; j < k; ++j) if (j != rho) qhat = mulmod(qhat, info.q[j] % info.q[i], info.q[i]);
            v = mulmod(qhat, powmod(2, l * prm.w_bits, info.q[i]), info.q[i]);
          }
          C.g_val[g][i] = v;
          C.g_val_sh[g][i] = sh64(v, info.q[i]);
        }
      }
    }
  }

  // ---- twiddle tables
  T->qtw.resize((size_t)k * n); T->qtw_sh.resize((size_t)k * n);
  T->qitw.resize((size_t)k * n); T->qitw_sh.resize((size_t)k * n);
  for (uint32_t i = 0; i < k; ++i) {
    const uint64_t q = info.q[i];
    uint64_t psi = root_2n(q, two_n);
    if (!psi) return "no 2n-th root of unity mod q_i";
    uint64_t ipsi = invmod(psi, q);
    for (uint32_t j = 0; j < n; ++j) {
      uint32_t e = bitrev(j, logn);
      uint64_t w = powmod(psi, e, q), iw = powmod(ipsi, e, q);
      T->qtw[(size_t)i * n + j] = w;
      T->qtw_sh[(size_t)i * n + j] = sh64(w, q);
      T->qitw[(size_t)i * n + j] = iw;
      T->qitw_sh[(size_t)i * n + j] = sh64(iw, q);
    }
  }
  T->ptw.resize((size_t)K * n); T->ptw_sh.resize((size_t)K * n);
  T->pitw.resize((size_t)K * n); T->pitw_sh.resize((size_t)K * n);
  for (uint32_t r = 0; r < K; ++r) {
    const uint32_t p = C.p[r];
    uint64_t psi = root_2n(p, two_n);
    if (!psi) return "no 2n-th root of unity mod p_r";
    uint64_t ipsi = invmod(psi, p);
    for (uint32_t j = 0; j < n; ++j) {
      uint32_t e = bitrev(j, logn);
      uint32_t w = (uint32_t)powmod(psi, e, p), iw = (uint32_t)powmod(ipsi, e, p);
      T->ptw[(size_t)r * n + j] = w;
      T->ptw_sh[(size_t)r * n + j] = sh32(w, p);
      T->pitw[(size_t)r * n + j] = iw;
      T->pitw_sh[(size_t)r * n + j] = sh32(iw, p);
    }
  }
  // slots are the values at psi_t^(2j+1), psi_t = g^((t-1)/2n) with g the smallest generator of Z_t^*
  {
    uint64_t g = smallest_generator(t);
    uint64_t psi = powmod(g, (t - 1) / two_n, t);
    if (powmod(psi, n, t) != t - 1) return "plaintext root of unity check failed";
    uint64_t ipsi = invmod(psi, t);
    T->ttw.resize(n); T->ttw_sh.resize(n); T->titw.resize(n); T->titw_sh.resize(n);
    for (uint32_t j = 0; j < n; ++j) {
      uint32_t e = bitrev(j, logn);
      uint32_t w = (uint32_t)powmod(psi, e, t), iw = (uint32_t)powmod(ipsi, e, t);
      T->ttw[j] = w; T->ttw_sh[j] = sh32(w, (uint32_t)t);
      T->titw[j] = iw; T->titw_sh[j] = sh32(iw, (uint32_t)t);
    }
  }
  return "";
}

}  // namespace hers
