// kernels.hip -- gfx950 kernels of the HERS encrypted-search path.
//
// Layouts (device memory, little-endian words)
//   canonical ciphertext   u64 [2][k][n]     residues mod q_i in [0, q_i)
//   search form, gallery   u32 [M][K][d][2][n] centred representative mod p_r, NTT domain
//   search form, probe     u32 [K][d][2][n]
//   accumulators           u32 [M][3][K][n]   sum_i of the tensor, NTT then coefficient domain
//   relin digits           u64 [M][L][k][n]   digit g of c2, reduced mod q_sigma
// Workgroups are 256 lanes (four wave64s).
#include <cstring>
#include <type_traits>

#include "kernels.h"

#include "ntt.h"

#define WG 256
// wider workgroups for kernels launched with few workgroups (one per probe
// ciphertext or block): more waves per CU hide the latency of their
// element-wise phases (k_encrypt needs ~133 VGPRs, so at most 512 lanes)
#define WG_ENC 512
#define WG_DEC 1024

extern "C" __global__ void __launch_bounds__(WG)
k_keygen(DevTabs T, uint64_t seed, uint8_t* __restrict__ sk, uint64_t* __restrict__ pk,
         uint64_t* __restrict__ rlk) {
  // Alg. "Key Generation": one workgroup per (job, residue rho); job 0 is the
  // public key, job 1 + g the evaluation key of gadget digit g.  Every
  // workgroup regenerates s from its counter, so no cross-workgroup traffic.
  extern __shared__ uint64_t lds64[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = C.k, tid = threadIdx.x;
  const uint32_t job = blockIdx.x, rho = blockIdx.y;
  const uint64_t q = C.q[rho];
  const ModQ mq{q};
  uint64_t* S = lds64;
  uint64_t* A = lds64 + padded_len(n);
  const uint64_t* tw = T.qtw + (size_t)rho * n;
  const uint64_t* twsh = T.qtw_sh + (size_t)rho * n;
  const uint64_t* itw = T.qitw + (size_t)rho * n;
  const uint64_t* itwsh = T.qitw_sh + (size_t)rho * n;

  for (uint32_t j = tid; j < n; j += WG) {
    uint64_t w = philox_word(seed, HERS_DOMAIN_KEYGEN, 0, 0, 0, j >> 6);
    uint64_t s = (w >> (j & 63)) & 1;
    S[PADX(j)] = s;
    if (job == 0 && rho == 0) sk[j] = (uint8_t)s;
  }
  // uniform a (job 0) or a_g (job 1 + g), residues rho, two per Philox block
  const uint64_t oa0 = job == 0 ? 1 : 3, oa1 = job == 0 ? 0 : job - 1;
  const uint64_t oe0 = job == 0 ? 2 : 4;
  for (uint32_t h = tid; h < n / 2; h += WG) {
    Philox4 b = philox4x64_10(((uint64_t)rho * n) / 2 + h, oa0, oa1, 0, seed, HERS_DOMAIN_KEYGEN);
    for (int s = 0; s < 2; ++s) {
      uint64_t lo = b.v[2 * s], hi = b.v[2 * s + 1];
      uint64_t v = add_q(shoup_q(red_q(hi, q, C.q_mu64[rho]), C.q_r64[rho], C.q_r64_sh[rho], q),
                         red_q(lo, q, C.q_mu64[rho]), q);
      A[PADX(2 * h + s)] = v;
    }
  }
  uint64_t* out = job == 0 ? pk : rlk + (size_t)(job - 1) * 2 * k * n;        // this key's [2][k][n]
  uint64_t* out_ntt = job == 0 ? T.pk_ntt : T.rlk_ntt + (size_t)(job - 1) * 2 * k * n;
  uint64_t* out_sh = job == 0 ? T.pk_ntt_sh : T.rlk_ntt_sh + (size_t)(job - 1) * 2 * k * n;
  __syncthreads();
  for (uint32_t j = tid; j < n; j += WG) out[((size_t)1 * k + rho) * n + j] = A[PADX(j)];
  ntt_forward16(S, tw, twsh, mq, n, C.logn, tid, WG, T.ntt_r);
  ntt_forward16(A, tw, twsh, mq, n, C.logn, tid, WG, T.ntt_r);
  const uint64_t gv = job == 0 ? 0 : C.g_val[job - 1][rho];
  const uint64_t gvsh = job == 0 ? 0 : C.g_val_sh[job - 1][rho];
  for (uint32_t j = tid; j < n; j += WG) {
    const uint64_t a = A[PADX(j)], s = S[PADX(j)];
    out_ntt[((size_t)1 * k + rho) * n + j] = a;
    out_sh[((size_t)1 * k + rho) * n + j] = shoup_companion_q(a, q, C.q_m128h[rho], C.q_m128l[rho]);
    uint64_t v = sub_q(0, mul_q(a, s, q, C.q_bar[rho], C.q_beta[rho]), q);        // -a s
    if (job) v = add_q(v, shoup_q(mul_q(s, s, q, C.q_bar[rho], C.q_beta[rho]), gv, gvsh, q), q);  // + g s^2
    A[PADX(j)] = v;
  }
  __syncthreads();
  ntt_inverse16(A, itw, itwsh, C.q_ninv[rho], C.q_ninv_sh[rho], mq, n, C.logn, tid, WG, T.ntt_r);
  for (uint32_t g4 = tid; g4 < n / 4; g4 += WG) {
    Philox4 b = philox4x64_10(g4, oe0, oa1, 0, seed, HERS_DOMAIN_KEYGEN);
    for (int s = 0; s < 4; ++s) {
      const uint32_t j = 4 * g4 + s;
      const int e = cbd20(b.v[s]);
      const uint64_t em = e >= 0 ? (uint64_t)e : q - (uint64_t)(-e);
      const uint64_t v = sub_q(A[PADX(j)], em, q);
      A[PADX(j)] = v;
      out[((size_t)0 * k + rho) * n + j] = v;
    }
  }
  __syncthreads();
  ntt_forward16(A, tw, twsh, mq, n, C.logn, tid, WG, T.ntt_r);
  for (uint32_t j = tid; j < n; j += WG) {
    out_ntt[((size_t)0 * k + rho) * n + j] = A[PADX(j)];
    out_sh[((size_t)0 * k + rho) * n + j] = shoup_companion_q(A[PADX(j)], q, C.q_m128h[rho], C.q_m128l[rho]);
  }
}

extern "C" __global__ void __launch_bounds__(WG)
k_load_keys(DevTabs T, const uint64_t* __restrict__ pk, const uint64_t* __restrict__ rlk) {
  // NTT form and Shoup companions of externally supplied keys: one workgroup
  // per key polynomial (key in [0, 1 + L), component, residue).
  extern __shared__ uint64_t lds64[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = C.k, tid = threadIdx.x;
  const uint32_t key = blockIdx.x, comp = blockIdx.y / k, rho = blockIdx.y % k;
  const uint64_t q = C.q[rho];
  const uint64_t* src = key == 0 ? pk : rlk + (size_t)(key - 1) * 2 * k * n;
  uint64_t* dst = key == 0 ? T.pk_ntt : T.rlk_ntt + (size_t)(key - 1) * 2 * k * n;
  uint64_t* dsh = key == 0 ? T.pk_ntt_sh : T.rlk_ntt_sh + (size_t)(key - 1) * 2 * k * n;
  const size_t off = ((size_t)comp * k + rho) * n;
  for (uint32_t j = tid; j < n; j += WG) lds64[PADX(j)] = src[off + j];
  __syncthreads();
  ntt_forward16(lds64, T.qtw + (size_t)rho * n, T.qtw_sh + (size_t)rho * n, ModQ{q}, n, C.logn, tid, WG, T.ntt_r);
  for (uint32_t j = tid; j < n; j += WG) {
    dst[off + j] = lds64[PADX(j)];
    dsh[off + j] = shoup_companion_q(lds64[PADX(j)], q, C.q_m128h[rho], C.q_m128l[rho]);
  }
}

extern "C" __global__ void __launch_bounds__(WG)
k_encode(DevTabs T, const int32_t* __restrict__ feats, int64_t ld, int64_t item_lo, int64_t item_hi,
         int64_t fbase, int32_t d, int64_t block0, uint32_t* __restrict__ pt) {
  // Eq. 3 with slot packing: slot j of (block b, dimension i) holds item
  // b n + j when item_lo <= b n + j < item_hi (feature column item - fbase),
  // else 0; the plaintext is the inverse negacyclic NTT mod t of the slots
  // placed at bit-reversed positions (out[i] = m(psi^(2 brv(i)+1))).
  extern __shared__ uint32_t lds32[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, tid = threadIdx.x, t = C.t;
  const uint32_t c = blockIdx.x;
  const uint32_t bl = c / d, i = c % d;
  const int64_t b = block0 + bl;
  for (uint32_t j = tid; j < n; j += WG) {
    const int64_t item = b * n + j;
    int64_t v = item >= item_lo && item < item_hi ? feats[(int64_t)i * ld + (item - fbase)] : 0;
    int64_t z = v % (int64_t)t;
    if (z < 0) z += t;
    lds32[PADX(bit_reverse(j, C.logn))] = (uint32_t)z;
  }
  __syncthreads();
  ntt_inverse16(lds32, T.titw, T.titw_sh, C.t_ninv, C.t_ninv_sh, ModP{t}, n, C.logn, tid, WG, T.ntt_r);
  for (uint32_t j = tid; j < n; j += WG) pt[(size_t)c * n + j] = lds32[PADX(j)];
}

extern "C" __global__ void __launch_bounds__(WG)
k_ct_add(DevTabs T, uint64_t* __restrict__ dst, const uint64_t* __restrict__ fresh, uint32_t nct, int32_t d,
         int64_t block0, int64_t first_empty_block) {
  // Server half of the online enrollment (App. B, Alg. "HERS Enrollment"):
  // CipherAdd of the fresh ciphertexts of blocks block0 .. into the running
  // ones, [a + b]_q per residue; a block at or past first_empty_block held no
  // item, so its running ciphertext is the trivial zero and becomes the
  // fresh one.  Layout [nct][2][k][n], ciphertext c of block block0 + c / d.
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = C.k;
  const uint64_t w = (uint64_t)blockIdx.x * WG + threadIdx.x;
  if (w >= (uint64_t)nct * 2 * k * n) return;
  const uint32_t rho = (uint32_t)((w >> C.logn) % k);
  const int64_t b = block0 + (int64_t)(w / ((uint64_t)2 * k * n) / d);
  dst[w] = b >= first_empty_block ? fresh[w] : add_q(dst[w], fresh[w], C.q[rho]);
}

template <bool QF>
__global__ void __launch_bounds__(WG_ENC)
k_encrypt(DevTabs T, const uint32_t* __restrict__ pt, QueryVals qv, int32_t qdim0,
          int32_t d, int64_t block0, uint64_t seed, uint32_t domain, uint64_t* __restrict__ canon) {
  // Alg. "Encryption" for ciphertext c (gallery: c = b_local d + i, or probe
  // dimension c) and residue rho: ct = ([Delta m + pk0 u + e1]_q, [pk1 u + e2]_q).
  extern __shared__ uint64_t lds64[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = C.k, tid = threadIdx.x;
  const uint32_t c = blockIdx.x, rho = blockIdx.y;
  const uint64_t q = C.q[rho];
  const ModQ mq{q};
  const bool query = pt == nullptr;                     // probe dimension qdim0 + c
  const uint64_t o0 = query ? 0 : (uint64_t)(block0 + c / d);
  const uint64_t o1 = query ? (uint64_t)(qdim0 + c) : c % d;
  uint64_t* U = lds64;
  uint64_t* V = lds64 + padded_len(n);
  uint64_t* W = V;                      // n/64 words of u, consumed before V is written
  for (uint32_t bk = tid; bk < n / 256; bk += WG_ENC) {
    Philox4 b = philox4x64_10(bk, o0, o1, 0, seed, domain);
    for (int s = 0; s < 4; ++s) W[4 * bk + s] = b.v[s];
  }
  __syncthreads();
  const uint64_t* pk0 = T.pk_ntt + (size_t)rho * n;
  const uint64_t* pk0s = T.pk_ntt_sh + (size_t)rho * n;
  const uint64_t* pk1 = T.pk_ntt + ((size_t)k + rho) * n;
  const uint64_t* pk1s = T.pk_ntt_sh + ((size_t)k + rho) * n;
  if constexpr (QF) {
    // u pk0 and u pk1 in double precision: products by ModQF, transforms balanced (ModQB)
    double* Uf = reinterpret_cast<double*>(U);
    double* Vf = reinterpret_cast<double*>(V);
    const ModQF mf{T.qf[rho], T.qf[HC_MAXQ + rho]};
    for (uint32_t j = tid; j < n; j += WG_ENC) Uf[PADX(j)] = (double)((W[j >> 6] >> (j & 63)) & 1);
    __syncthreads();
    const double* twf = T.qtw_f + (size_t)rho * n;
    const ModQB mb{mf.q, mf.qinv};
    ntt_forward_b(Uf, twf, mb, n, C.logn, tid, WG_ENC, T.ntt_r);
    for_each_loaded2(pk0, pk1, n, tid, WG_ENC, [&](uint32_t j, uint64_t k0, uint64_t k1) {
      const double u = Uf[PADX(j)];
      Vf[PADX(j)] = mf.mul(u, u64_to_f(k1), 0.0);
      Uf[PADX(j)] = mf.mul(u, u64_to_f(k0), 0.0);
    });
    __syncthreads();
    const double* itwf = T.qitw_f + (size_t)rho * n;
    const double ninv = T.qf[2 * HC_MAXQ + rho];
    ntt_inverse_b(Uf, itwf, ninv, mb, n, C.logn, tid, WG_ENC, T.ntt_r);
    ntt_inverse_b(Vf, itwf, ninv, mb, n, C.logn, tid, WG_ENC, T.ntt_r);
    for (uint32_t j = tid; j < n; j += WG_ENC) {
      U[PADX(j)] = f_to_u64(Uf[PADX(j)]);
      V[PADX(j)] = f_to_u64(Vf[PADX(j)]);
    }
    __syncthreads();
  } else {
    for (uint32_t j = tid; j < n; j += WG_ENC) U[PADX(j)] = (W[j >> 6] >> (j & 63)) & 1;
    __syncthreads();
    const uint64_t* tw = T.qtw + (size_t)rho * n;
    const uint64_t* twsh = T.qtw_sh + (size_t)rho * n;
    ntt_forward16(U, tw, twsh, mq, n, C.logn, tid, WG_ENC, T.ntt_r);
    for (uint32_t j = tid; j < n; j += WG_ENC) {
      const uint64_t u = U[PADX(j)];
      V[PADX(j)] = shoup_q(u, pk1[j], pk1s[j], q);
      U[PADX(j)] = shoup_q(u, pk0[j], pk0s[j], q);
    }
    __syncthreads();
    const uint64_t* itw = T.qitw + (size_t)rho * n;
    const uint64_t* itwsh = T.qitw_sh + (size_t)rho * n;
    ntt_inverse16(U, itw, itwsh, C.q_ninv[rho], C.q_ninv_sh[rho], mq, n, C.logn, tid, WG_ENC, T.ntt_r);
    ntt_inverse16(V, itw, itwsh, C.q_ninv[rho], C.q_ninv_sh[rho], mq, n, C.logn, tid, WG_ENC, T.ntt_r);
  }
  uint32_t qconst = 0;
  if (query) {
    int64_t z = (int64_t)qv.v[c] % (int64_t)C.t;
    if (z < 0) z += C.t;
    qconst = (uint32_t)z;
  }
  uint64_t* o_ct0 = canon + (((size_t)c * 2 + 0) * k + rho) * n;
  uint64_t* o_ct1 = canon + (((size_t)c * 2 + 1) * k + rho) * n;
  for (uint32_t g4 = tid; g4 < n / 4; g4 += WG_ENC) {
    Philox4 b1 = philox4x64_10(g4, o0, o1, 1, seed, domain);
    Philox4 b2 = philox4x64_10(g4, o0, o1, 2, seed, domain);
    for (int s = 0; s < 4; ++s) {
      const uint32_t j = 4 * g4 + s;
      const int e1 = cbd20(b1.v[s]), e2 = cbd20(b2.v[s]);
      const uint64_t m = query ? (j == 0 ? qconst : 0) : pt[(size_t)c * n + j];
      uint64_t v0 = add_q(U[PADX(j)], shoup_q(m, C.q_delta[rho], C.q_delta_sh[rho], q), q);
      v0 = e1 >= 0 ? add_q(v0, (uint64_t)e1, q) : sub_q(v0, (uint64_t)(-e1), q);
      uint64_t v1 = e2 >= 0 ? add_q(V[PADX(j)], (uint64_t)e2, q) : sub_q(V[PADX(j)], (uint64_t)(-e2), q);
      o_ct0[j] = v0;
      o_ct1[j] = v1;
    }
  }
}

extern "C" __global__ void __launch_bounds__(WG_ENC)
k_encrypt_sk(DevTabs T, QueryVals qv, int32_t qdim0, uint64_t seed, const uint64_t* __restrict__ S,
             const uint64_t* __restrict__ Ssh, uint64_t* __restrict__ canon) {
  // Probe dimension qdim0 + c, c = blockIdx.x, encrypted under the secret key (Sec. 3.2,
  // "Search Protocol": the client encrypts its query with its private key),
  // residue rho = blockIdx.y: ct = ([Delta m - a s + e]_q, a) with m the
  // constant [query_c]_t, a uniform (Philox object (0, c, 0): residue rho of
  // coefficient j from words 2(rho n + j), 2(rho n + j) + 1 as a 128-bit
  // integer), e centred binomial (object (0, c, 1), word j).  S, Ssh: the
  // secret key's NTT form mod each q_sigma with Shoup companions, [k][n].
  extern __shared__ uint64_t lds64[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = C.k, tid = threadIdx.x;
  const uint32_t c = blockIdx.x, rho = blockIdx.y, ci = (uint32_t)qdim0 + c;
  const uint64_t q = C.q[rho];
  const ModQ mq{q};
  uint64_t* A = lds64;
  uint64_t* o_ct0 = canon + (((size_t)c * 2 + 0) * k + rho) * n;
  uint64_t* o_ct1 = canon + (((size_t)c * 2 + 1) * k + rho) * n;
  for (uint32_t h = tid; h < n / 2; h += WG_ENC) {        // two coefficients per Philox block
    Philox4 b = philox4x64_10(((uint64_t)rho * n) / 2 + h, 0, ci, 0, seed, HERS_DOMAIN_PROBE_SK);
    for (int s = 0; s < 2; ++s) {
      const uint64_t lo = b.v[2 * s], hi = b.v[2 * s + 1];
      const uint64_t v = add_q(shoup_q(red_q(hi, q, C.q_mu64[rho]), C.q_r64[rho], C.q_r64_sh[rho], q),
                               red_q(lo, q, C.q_mu64[rho]), q);
      A[PADX(2 * h + s)] = v;
      o_ct1[2 * h + s] = v;
    }
  }
  __syncthreads();
  ntt_forward16(A, T.qtw + (size_t)rho * n, T.qtw_sh + (size_t)rho * n, mq, n, C.logn, tid, WG_ENC, T.ntt_r);
  for (uint32_t j = tid; j < n; j += WG_ENC)
    A[PADX(j)] = shoup_q(A[PADX(j)], S[(size_t)rho * n + j], Ssh[(size_t)rho * n + j], q);   // a s
  __syncthreads();
  ntt_inverse16(A, T.qitw + (size_t)rho * n, T.qitw_sh + (size_t)rho * n, C.q_ninv[rho], C.q_ninv_sh[rho], mq, n,
                C.logn, tid, WG_ENC, T.ntt_r);
  int64_t z = (int64_t)qv.v[c] % (int64_t)C.t;
  if (z < 0) z += C.t;
  const uint64_t dm = shoup_q((uint64_t)z, C.q_delta[rho], C.q_delta_sh[rho], q);   // Delta m_0
  for (uint32_t g4 = tid; g4 < n / 4; g4 += WG_ENC) {
    Philox4 be = philox4x64_10(g4, 0, ci, 1, seed, HERS_DOMAIN_PROBE_SK);
    for (int s = 0; s < 4; ++s) {
      const uint32_t j = 4 * g4 + s;
      const int e = cbd20(be.v[s]);
      uint64_t v = sub_q(j == 0 ? dm : 0, A[PADX(j)], q);
      v = e >= 0 ? add_q(v, (uint64_t)e, q) : sub_q(v, (uint64_t)(-e), q);
      o_ct0[j] = v;
    }
  }
}

template <int KQ>
__global__ void __launch_bounds__(WG)
k_lift(DevTabs T, const uint64_t* __restrict__ canon, uint32_t nct, int32_t d, int64_t block0,
       uint32_t* __restrict__ out) {
  // Exact centred lift of canonical residues mod q to residues mod p_r
  // (the representative in (-q/2, q/2) that the tensor product needs):
  // Garner mixed-radix digits decide the sign exactly, then the digits are
  // evaluated mod p_r.  Writes the search form (coefficient domain).
  // KQ: the number of q primes at compile time (0: read from C), so the
  // Garner digits stay in statically indexed registers
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = KQ ? KQ : C.k, K = C.K;
  const uint64_t idx = (uint64_t)blockIdx.x * WG + threadIdx.x;
  if (idx >= (uint64_t)nct * n) return;
  const uint32_t c = (uint32_t)(idx >> C.logn), j = (uint32_t)(idx & (n - 1));
  const int64_t b = block0 + c / d;
  const uint32_t i = c % d;
  for (uint32_t poly = 0; poly < 2; ++poly) {
    uint64_t v[KQ ? KQ : HC_MAXQ], a[KQ ? KQ : HC_MAXQ];
    for (uint32_t r = 0; r < k; ++r) v[r] = canon[(((size_t)c * 2 + poly) * k + r) * n + j];
    const bool neg = garner_digits<KQ>(C, v, a);
    for (uint32_t r = 0; r < K; ++r) {
      const size_t o = ((((size_t)b * K + r) * d + i) * 2 + poly) * n + j;
      out[o] = mixed_to_p<KQ>(C, a, neg, r);
    }
  }
}

template <int KQ>
__global__ void __launch_bounds__(WG)
k_unlift(DevTabs T, const uint32_t* __restrict__ coef, uint32_t nct, int32_t d, uint64_t* __restrict__ canon) {
  // The inverse of the lift, for exporting a search form: coef holds the
  // centred representative x of every coefficient modulo each p_r in the
  // coefficient domain, block-local layout [nct / d][K][d][2][n].  By CRT
  // over P, x = sum_r y_r (P/p_r) - gamma P with y_r = [x_r (P/p_r)^-1]_{p_r}
  // and gamma = round(sum_r y_r / p_r): |x| < q/2 is a negligible fraction of
  // P, so the double-precision sum (error below K 2^-52) rounds to the integer
  // gamma exactly.  Writes x mod q_i, the canonical residues [nct][2][k][n].
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = KQ ? KQ : C.k, K = C.K;
  const uint64_t idx = (uint64_t)blockIdx.x * WG + threadIdx.x;
  if (idx >= (uint64_t)nct * n) return;
  const uint32_t c = (uint32_t)(idx >> C.logn), j = (uint32_t)(idx & (n - 1));
  const uint32_t bl = c / d, i = c % d;
  for (uint32_t poly = 0; poly < 2; ++poly) {
    uint32_t y[HC_MAXP];
    double s = 0.0;
    for (uint32_t r = 0; r < K; ++r) {
      const uint32_t x = coef[((((size_t)bl * K + r) * d + i) * 2 + poly) * n + j];
      y[r] = shoup_p(x, C.p_hatinv[r], C.p_hatinv_sh[r], C.p[r]);
      s += (double)y[r] * C.p_inv[r];
    }
    const uint64_t gamma = (uint64_t)rint(s);
    for (uint32_t ii = 0; ii < k; ++ii) {
      const uint64_t q = C.q[ii];
      uint64_t acc = 0;
      for (uint32_t r = 0; r < K; ++r)
        acc = add_q(acc, mul_q(red_q(y[r], q, C.q_mu64[ii]), C.phat_q[r][ii], q, C.q_bar[ii], C.q_beta[ii]), q);
      acc = sub_q(acc, mul_q(gamma, C.P_q[ii], q, C.q_bar[ii], C.q_beta[ii]), q);
      canon[(((size_t)c * 2 + poly) * k + ii) * n + j] = acc;
    }
  }
}

extern "C" __global__ void __launch_bounds__(WG)
k_check_features(const int32_t* __restrict__ v, int64_t ld, int64_t cols, int32_t bound,
                 uint32_t* __restrict__ flag) {
  // Sets *flag when a value of row blockIdx.y (columns 0 .. cols - 1 of a
  // row-major array with row stride ld) lies outside [-bound, bound].
  const int32_t* row = v + (int64_t)blockIdx.y * ld;
  bool bad = false;
  for (int64_t c = (int64_t)blockIdx.x * WG + threadIdx.x; c < cols; c += (int64_t)gridDim.x * WG) {
    const int32_t x = row[c];
    bad |= x > bound || x < -bound;
  }
  if (bad) atomicOr(flag, 1u);
}

extern "C" __global__ void __launch_bounds__(WG)
k_check_canon(DevTabs T, const uint64_t* __restrict__ canon, uint64_t words, uint32_t* __restrict__ flag) {
  // Sets *flag when a residue of canonical ciphertexts [..][2][k][n] is not
  // below its prime q_i.
  const HersConsts& C = *T.C;
  bool bad = false;
  for (uint64_t w = (uint64_t)blockIdx.x * WG + threadIdx.x; w < words; w += (uint64_t)gridDim.x * WG)
    bad |= canon[w] >= C.q[(uint32_t)(w >> C.logn) % C.k];
  if (bad) atomicOr(flag, 1u);
}

// (at least 5 waves per SIMD: the register budget the inverse direction fits)
extern "C" __global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(5)))
k_ntt_p(DevTabs T, uint32_t* __restrict__ polys, uint32_t inner, int inverse, uint64_t req_stride) {
  // In-place negacyclic NTT mod p_r of polynomial blockIdx.x of set
  // blockIdx.y (at polys + blockIdx.y * req_stride words), where
  // r = (blockIdx.x / inner) mod K.
  extern __shared__ uint32_t lds32[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, tid = threadIdx.x;
  const uint32_t r = (blockIdx.x / inner) % C.K;
  uint32_t* a = polys + (size_t)blockIdx.y * req_stride + (size_t)blockIdx.x * n;
  const ModP mp{C.p[r]};
  // the first pass reads the polynomial from memory and the last one writes
  // it back, so it crosses LDS two times fewer than a load, transform and store
  if (inverse)
    ntt_inverse16_g(a, lds32, T.pitw + (size_t)r * n, T.pitw_sh + (size_t)r * n, C.p_ninv[r], C.p_ninv_sh[r], mp,
                    n, C.logn, tid, WG, T.ntt_r);
  else
    ntt_forward16_g(a, lds32, T.ptw + (size_t)r * n, T.ptw_sh + (size_t)r * n, mp, n, C.logn, tid, WG, T.ntt_r);
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ u32x4 load_stream(const u32x4* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// The hot loop (Alg. "HERS Search" with the tensor of Alg. "Ciphertext
// Multiplication", summed over the d dimensions before any rescale):
//   A0 = sum_i P_i0 G_bi0,  A1 = sum_i (P_i0 G_bi1 + P_i1 G_bi0),  A2 = sum_i P_i1 G_bi1
// slot-wise in the NTT domain mod p_r.  A lane owns 4 consecutive NTT slots of
// one prime (16-byte loads, 1 KiB per wave instruction) and NB blocks at a
// time, so one probe load serves NB gallery loads.  Dimensions go in batches
// of U; the loads of batch j + 1 are issued before the products of batch j
// (double buffering), so a wave's arithmetic overlaps its own memory traffic.
// Gallery rows are read once, so NT streams them past the cache.  Products of
// residues below 2^30 are < 2^60: A0 and A2 take one product per dimension and
// A1 two; the 64-bit sums are partially folded (three instructions) every 4
// dimensions and fully reduced at the end.  acc is indexed from blk_lo.
// a -> (a >> 34) (2^34 mod p) + (a mod 2^34), congruent mod p and below 2^60 + 2^34
__device__ __forceinline__ uint64_t fold34(uint64_t a, uint32_t c34) {
  return (uint64_t)(uint32_t)(a >> 34) * c34 + (a & ((1ull << 34) - 1));
}

template <int NB, int U, bool NT>
struct MacBatch {
  u32x4 P0[U], P1[U], G0[U][NB], G1[U][NB];
  __device__ __forceinline__ void load(const u32x4* pr, const u32x4* const (&gb)[NB], int32_t i, size_t row) {
#pragma unroll
    for (int v = 0; v < U; ++v) {
      const size_t o0 = (size_t)(2 * (i + v)) * row, o1 = o0 + row;
      P0[v] = pr[o0];
      P1[v] = pr[o1];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        G0[v][u] = load_stream<NT>(gb[u] + o0);
        G1[v][u] = load_stream<NT>(gb[u] + o1);
      }
    }
  }
};

template <int NB, int U, bool NT>
__global__ void __launch_bounds__(WG)
k_mac(DevTabs T, const uint32_t* __restrict__ gallery, const uint32_t* __restrict__ probe, int32_t d,
      int32_t dim0, int32_t dcount, int64_t blk_lo, int64_t blk_hi, uint32_t* __restrict__ acc) {
  static_assert(4 % U == 0, "U divides the fold period");
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, K = C.K;
  const uint32_t slot = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
  const uint32_t r = blockIdx.y;
  const uint32_t p = C.p[r];
  const uint64_t mu = C.p_mu64[r];
  const uint32_t c34 = (uint32_t)((1ull << 34) - (uint64_t)p * (mu >> 30));   // 2^34 mod p (mu = floor(2^64/p))
  const size_t row = n / 4;                               // u32x4 between dimension rows
  // dimensions dim0 .. dim0 + dcount - 1 of the d in the layouts
  const u32x4* pr = (const u32x4*)(probe + ((size_t)r * d + dim0) * 2 * n + slot);
  const int32_t dfull = dcount / U * U;
  // block group z takes the steps of NB blocks z, z + G, z + 2G, ... (G groups),
  // so the groups resident at one time read neighbouring blocks: one window of
  // the gallery sweeps forward, rather than G windows a group's length apart
  const int64_t stride = (int64_t)gridDim.z * NB;
  for (int64_t b = blk_lo + (int64_t)blockIdx.z * NB; b < blk_hi; b += stride) {
    const int64_t b1 = b + NB < blk_hi ? b + NB : blk_hi;
    const u32x4* gb[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int64_t bb = b + u < b1 ? b + u : b;          // a short tail recomputes block b, not stored
      gb[u] = (const u32x4*)(gallery + (((size_t)bb * K + r) * d + dim0) * 2 * n + slot);
    }
    uint64_t a0[NB][4], a1[NB][4], a2[NB][4];
#pragma unroll
    for (int u = 0; u < NB; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) { a0[u][s] = 0; a1[u][s] = 0; a2[u][s] = 0; }

    auto mac = [&](const u32x4& P0, const u32x4& P1, const u32x4 (&G0)[NB], const u32x4 (&G1)[NB]) {
#pragma unroll
      for (int u = 0; u < NB; ++u)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          a0[u][s] += (uint64_t)P0[s] * G0[u][s];
          a1[u][s] += (uint64_t)P0[s] * G1[u][s];
          a1[u][s] += (uint64_t)P1[s] * G0[u][s];
          a2[u][s] += (uint64_t)P1[s] * G1[u][s];
        }
    };
    // partial fold a -> (a >> 34) (2^34 mod p) + (a mod 2^34) < 2^60 + 2^34
    // (three instructions), which leaves room for 8 more products: all three
    // sums fold every 4 dimensions (a1 takes two products per dimension), and
    // at most 3 dimensions follow the last fold
    auto fold = [&]() {
#pragma unroll
      for (int u = 0; u < NB; ++u)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          a0[u][s] = fold34(a0[u][s], c34);
          a1[u][s] = fold34(a1[u][s], c34);
          a2[u][s] = fold34(a2[u][s], c34);
        }
    };

    MacBatch<NB, U, NT> cur, nxt;
    if (dfull) cur.load(pr, gb, 0, row);
    for (int32_t i = 0; i < dfull; i += U) {
      if (i + U < dfull) nxt.load(pr, gb, i + U, row);
#pragma unroll
      for (int v = 0; v < U; ++v) mac(cur.P0[v], cur.P1[v], cur.G0[v], cur.G1[v]);
      const int32_t done = i + U;
      if ((done & 3) == 0) fold();
      cur = nxt;
    }
    for (int32_t i = dfull; i < dcount; ++i) {              // remainder, one dimension at a time
      MacBatch<NB, 1, NT> one;
      one.load(pr, gb, i, row);
      mac(one.P0[0], one.P1[0], one.G0[0], one.G1[0]);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        a0[u][s] = red_p(a0[u][s], p, mu);
        a1[u][s] = red_p(a1[u][s], p, mu);
        a2[u][s] = red_p(a2[u][s], p, mu);
      }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if (b + u >= b1) break;
      u32x4* o = (u32x4*)(acc + ((size_t)(b + u - blk_lo) * 3 * K + r) * n + slot);
      const size_t comp = (size_t)K * n / 4;
      o[0] = u32x4{(uint32_t)a0[u][0], (uint32_t)a0[u][1], (uint32_t)a0[u][2], (uint32_t)a0[u][3]};
      o[comp] = u32x4{(uint32_t)a1[u][0], (uint32_t)a1[u][1], (uint32_t)a1[u][2], (uint32_t)a1[u][3]};
      o[2 * comp] = u32x4{(uint32_t)a2[u][0], (uint32_t)a2[u][1], (uint32_t)a2[u][2], (uint32_t)a2[u][3]};
    }
  }
}

// ---------------------------------------------------------------- multiply-accumulate + inverse NTT
// The same sums A0, A1, A2 for one probe, with the inverse transform of the
// accumulators fused in (n <= 4096).  A work item is (block b, prime r): the
// whole ring of that block and prime, NS groups of 4 slots per lane (n / (4 NS)
// lanes, group s of lane l holding slots 4 (l + s lanes) .. + 3, so every
// row load is coalesced).  With one group per lane the kernel fits 64
// registers: two 1024-lane workgroups per CU at n = 4096 (52 KB of LDS each).  Dimensions are loaded one ahead of the products
// (double buffering); the sums fold every 4 dimensions as in k_mac.  After
// the d loop the three sums, reduced mod p_r, go to LDS, are transformed back
// to the coefficient domain (inverse negacyclic NTT mod p_r, exactly as
// k_ntt_p) and are written out: the accumulators the rescale reads, without
// a separate transform launch and its round trip through memory.
// Items are visited item = w + j G (G workgroups) with r = item mod K; with G
// a multiple of lcm(K, 8) a workgroup keeps one prime, and since workgroups
// are dealt to the 8 XCDs round-robin, an XCD's workgroups share the primes
// r = w mod K, so the probe rows of those primes (d 2 n 4 bytes each) stay in
// that XCD's L2.
template <int NS, int MAXT>
__global__ void __launch_bounds__(MAXT, 8)
k_mac_intt(DevTabs T, const uint32_t* __restrict__ gallery, const uint32_t* __restrict__ probe, int32_t d,
           int32_t dim0, int32_t dcount, int64_t blk_lo, int64_t blk_hi, uint32_t* __restrict__ acc) {
  extern __shared__ uint32_t lds32[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, K = C.K, tid = threadIdx.x, nthr = blockDim.x;
  const uint32_t plen = padded_len(n);
  const uint64_t items = (uint64_t)(blk_hi - blk_lo) * K;
  for (uint64_t item = blockIdx.x; item < items; item += gridDim.x) {
    const uint32_t r = (uint32_t)(item % K);
    const int64_t bl = (int64_t)(item / K);
    const uint32_t p = C.p[r];
    const uint64_t mu = C.p_mu64[r];
    const uint32_t c34 = (uint32_t)((1ull << 34) - (uint64_t)p * (mu >> 30));   // 2^34 mod p
    // wave-uniform bases and 32-bit lane offsets (the loads take the
    // scalar-base form, so no 64-bit address is kept per lane)
    const char* pr = (const char*)(probe + ((size_t)r * d + dim0) * 2 * n);
    const char* gb = (const char*)(gallery + (((size_t)(blk_lo + bl) * K + r) * d + dim0) * 2 * n);
    const uint32_t rowb = n * 4, lane_off = tid * 16;
    uint64_t a0[NS][4], a1[NS][4], a2[NS][4];
#pragma unroll
    for (int g = 0; g < NS; ++g)
#pragma unroll
      for (int e = 0; e < 4; ++e) { a0[g][e] = 0; a1[g][e] = 0; a2[g][e] = 0; }
    // the gallery rows (HBM) of dimension i + 1 are in flight while
    // dimension i is multiplied; the probe rows (L2) are loaded when needed
    struct Gal { u32x4 G0[NS], G1[NS]; };
    auto load = [&](int32_t i, Gal& x) {
      const uint32_t o0 = 2 * (uint32_t)i * rowb + lane_off, o1 = o0 + rowb;
#pragma unroll
      for (int g = 0; g < NS; ++g) {
        x.G0[g] = __builtin_nontemporal_load((const u32x4*)(gb + (o0 + g * nthr * 16)));
        x.G1[g] = __builtin_nontemporal_load((const u32x4*)(gb + (o1 + g * nthr * 16)));
      }
    };
    Gal cur, nxt;
    load(0, cur);
    for (int32_t i = 0; i < dcount; ++i) {
      if (i + 1 < dcount) load(i + 1, nxt);
      const uint32_t o0 = 2 * (uint32_t)i * rowb + lane_off, o1 = o0 + rowb;
#pragma unroll
      for (int g = 0; g < NS; ++g) {
        const u32x4 P0 = *(const u32x4*)(pr + (o0 + g * nthr * 16));
        const u32x4 P1 = *(const u32x4*)(pr + (o1 + g * nthr * 16));
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          a0[g][e] += (uint64_t)P0[e] * cur.G0[g][e];
          a1[g][e] += (uint64_t)P0[e] * cur.G1[g][e];
          a1[g][e] += (uint64_t)P1[e] * cur.G0[g][e];
          a2[g][e] += (uint64_t)P1[e] * cur.G1[g][e];
        }
      }
      if (((i + 1) & 3) == 0) {      // fold: < 2^60 + 2^34, room for the next 4 dimensions' 8 products
#pragma unroll
        for (int g = 0; g < NS; ++g)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            a0[g][e] = fold34(a0[g][e], c34);
            a1[g][e] = fold34(a1[g][e], c34);
            a2[g][e] = fold34(a2[g][e], c34);
          }
      }
      cur = nxt;
    }
#pragma unroll
    for (int g = 0; g < NS; ++g)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t slot = 4 * (tid + g * nthr) + e;
        lds32[PADX(slot)] = red_p(a0[g][e], p, mu);
        lds32[plen + PADX(slot)] = red_p(a1[g][e], p, mu);
        lds32[2 * plen + PADX(slot)] = red_p(a2[g][e], p, mu);
      }
    __syncthreads();
    const ModP mp{p};
#pragma unroll 1
    for (int j = 0; j < 3; ++j)
      ntt_inverse_upto<3>(lds32 + j * plen, T.pitw + (size_t)r * n, T.pitw_sh + (size_t)r * n, C.p_ninv[r],
                          C.p_ninv_sh[r], mp, n, C.logn, tid, nthr);
#pragma unroll 1
    for (int j = 0; j < 3; ++j) {
      uint32_t* o = acc + (((size_t)bl * 3 + j) * K + r) * n;
      for (uint32_t c = tid; c < n; c += nthr) o[c] = lds32[j * plen + PADX(c)];
    }
    __syncthreads();                                       // LDS free for the next item
  }
}

// ---------------------------------------------------------------- batched multiply-accumulate
// Many probes against galleries of uneven size and d, one persistent launch.
// A work item is (group, block range of up to MB_BLOCKS blocks, prime r,
// 64-slot tile); a group is up to MB_PROBES probes of one gallery.  The
// workgroup's 16 waves are the group's probes: each lane keeps its probe's
// values for a chunk of MB_DC dimensions in registers.  The gallery words of
// a chunk for all the item's blocks (MB_BLOCKS x MB_DC x 64 slots, both
// polynomials) are staged once in LDS and read by every wave, so one HBM read
// of the gallery serves the whole group; the next chunk's words are loaded
// into registers while the current chunk is multiplied.
// The tensor's cross term is taken by Karatsuba: A1 = sum_i (P_i0 + P_i1)
// (G_i0 + G_i1) - A0 - A2 mod p, with both sums reduced mod p first (the
// gallery's once per staged word, shared by all probe waves), so a dimension
// costs three products instead of four and every accumulator takes one
// product (< 2^60) per dimension.  After every chunk each sum is folded
// cheaply, a -> (a >> 34) (2^34 mod p) + (a mod 2^34) < 2^60 + 2^34, which
// leaves room for the next chunk's 8 products (< 9 2^60 < 2^64); one full
// reduction at the end.  The residues written are the same.
// The wave index is read as wave-uniform, so probe and staging addresses are
// scalar bases plus the lane's offset.
// Workgroups take the items in a fixed order (static assignment, no atomics).
// PPW probes per wave: a workgroup of 64 MB_PROBES / PPW lanes.  With two,
// every staged gallery word read from LDS feeds both probes' products (half
// the LDS traffic per product) and the workgroup is half as wide, so two of
// them share a CU and one's barriers overlap the other's products; the
// probe rows are then loaded when a chunk starts instead of one chunk ahead.
// DC dimensions and BLK blocks per staged chunk (8 and 4 with one probe per
// wave; fewer with more probes per wave, whose registers then hold about as
// many sums and probe values).
template <int PPW, int DC, int BLK>
__global__ void __launch_bounds__(64 * MB_PROBES / PPW, 4)   // 4 waves per SIMD: two 512-lane (four 256-lane) workgroups per CU
k_mac_multi(DevTabs T, MacBatchArgs A) {
  constexpr uint32_t WGL = 64 * MB_PROBES / PPW;         // lanes
  constexpr uint32_t MB_PAIRS = BLK * DC * 64;            // (block, dimension, slot) words per staged chunk
  constexpr uint32_t PER_THREAD = MB_PAIRS / WGL;         // staged pairs per lane
  __shared__ uint2 tileG[MB_PAIRS];                    // [u][v][64]: (G0, G1) of a slot
  __shared__ uint32_t tileS[MB_PAIRS];                 // [u][v][64]: G0 + G1 mod p
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, K = C.K;
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t tiles = n / 64;
  // Item order: a pair (prime r, slot tile) holds the group's probe rows for
  // that pair (nprobe d 2 64 words, 1 MB for 16 probes at d = 128), which
  // every block of the gallery reuses.  Pairs are dealt to the XCDs by their
  // index mod 8 (workgroups go to the XCDs round-robin), and an XCD's
  // workgroups take the pair's block groups together, so the probe rows of
  // the pair are read from memory about once per XCD and then hit its L2
  // (taking items block group first would re-read them for every item).
  const uint32_t npairs = K * tiles;
  const uint32_t nx = gridDim.x % 8 == 0 ? 8 : 1;
  const uint32_t xcd = blockIdx.x % nx, lw = blockIdx.x / nx, nw = gridDim.x / nx;
  const uint64_t my_pairs = npairs > xcd ? (npairs - xcd + nx - 1) / nx : 0;   // pairs xcd, xcd + nx, ...
  for (int g = 0; g < A.ngroups; ++g)
  for (uint64_t t = lw; t < my_pairs * (uint64_t)((A.g[g].blk_hi - A.g[g].blk_lo + BLK - 1) / BLK);
       t += nw) {
    const MacGroup& G = A.g[g];
    const uint64_t nbg = (uint64_t)((G.blk_hi - G.blk_lo + BLK - 1) / BLK);
    const uint32_t pair = xcd + (uint32_t)(t / nbg) * nx;
    const uint32_t tile = pair % tiles;
    const uint32_t r = pair / tiles;
    const int64_t b0 = G.blk_lo + (int64_t)(t % nbg) * BLK;
    const int nblk = (int)(G.blk_hi - b0 < BLK ? G.blk_hi - b0 : BLK);
    const int32_t d = G.d;
    const uint32_t p = C.p[r];
    const uint64_t mu = C.p_mu64[r];
    const uint32_t c34 = (uint32_t)((1ull << 34) - (uint64_t)p * (mu >> 30));   // 2^34 mod p (mu = floor(2^64/p))
    const uint32_t slot = tile * 64 + lane;
    bool active[PPW];
    const uint32_t* pbase[PPW];
#pragma unroll
    for (int q = 0; q < PPW; ++q) {
      const uint32_t j = wave * PPW + q;                  // the group's probe j
      active[q] = j < (uint32_t)G.nprobe;
      pbase[q] = active[q] ? G.probe[j] + (size_t)r * d * 2 * n + tile * 64 : nullptr;
    }
    const uint32_t* gbase = G.gallery + tile * 64;
    // staged pair w = tid + e WGL of chunk dc: block b0 + u, dimension dc + v
    // with u, v from the wave-uniform row w / 64, slot w mod 64 = lane
    auto fetch = [&](int32_t dc, int32_t dn, uint2 (&reg)[PER_THREAD]) {
#pragma unroll
      for (int e = 0; e < (int)PER_THREAD; ++e) {
        const uint32_t uv = wave + e * (WGL / 64);
        const uint32_t u = uv / (uint32_t)dn, v = uv - u * (uint32_t)dn;
        if ((int)u < nblk) {
          const uint32_t* src = gbase + (((size_t)(b0 + u) * K + r) * d * 2 + 2 * (dc + v)) * n;
          reg[e] = uint2{__builtin_nontemporal_load(src + lane), __builtin_nontemporal_load(src + n + lane)};
        } else {
          reg[e] = uint2{0u, 0u};
        }
      }
    };
    uint64_t a0[PPW][BLK], a2[PPW][BLK], as[PPW][BLK];
#pragma unroll
    for (int q = 0; q < PPW; ++q)
#pragma unroll
      for (int u = 0; u < BLK; ++u) { a0[q][u] = 0; a2[q][u] = 0; as[q][u] = 0; }
    uint2 stage[PER_THREAD];
    uint32_t P0[PPW][DC], P1[PPW][DC];            // this lane's probe values (PPW 1: of the next chunk)
    auto fetch_probe = [&](int32_t dc, int32_t dn) {
#pragma unroll
      for (int q = 0; q < PPW; ++q)
#pragma unroll
        for (int v = 0; v < DC; ++v) {
          P0[q][v] = active[q] && v < dn ? pbase[q][(size_t)(2 * (dc + v)) * n + lane] : 0;
          P1[q][v] = active[q] && v < dn ? pbase[q][(size_t)(2 * (dc + v) + 1) * n + lane] : 0;
        }
    };
    fetch(0, d < DC ? d : DC, stage);
    if (PPW == 1) fetch_probe(0, d < DC ? d : DC);
    for (int32_t dc = 0; dc < d; dc += DC) {
      const int32_t dn = d - dc < DC ? d - dc : DC;
      __syncthreads();                                 // previous chunk fully consumed
#pragma unroll
      for (int e = 0; e < (int)PER_THREAD; ++e) {
        const uint32_t w = tid + e * WGL;
        tileG[w] = stage[e];
        tileS[w] = add_p(stage[e].x, stage[e].y, p);
      }
      __syncthreads();
      // PPW 1: this chunk's probe values were loaded one chunk ahead (copied
      // out before the next chunk's load); PPW > 1: loaded now, from L2
      uint32_t Q0[PPW][DC], Q1[PPW][DC];
      if (PPW > 1) fetch_probe(dc, dn);
#pragma unroll
      for (int q = 0; q < PPW; ++q)
#pragma unroll
        for (int v = 0; v < DC; ++v) { Q0[q][v] = P0[q][v]; Q1[q][v] = P1[q][v]; }
      if (dc + DC < d) {                            // next chunk in flight during the products
        const int32_t nd = d - dc - DC < DC ? d - dc - DC : DC;
        fetch(dc + DC, nd, stage);
        if (PPW == 1) fetch_probe(dc + DC, nd);
      }
      if (active[0]) {
        static_assert(DC <= 15, "a folded sum plus one chunk's products must stay below 2^64");
        if (dn == DC && nblk == BLK) {        // full chunk: no bounds in the product loop
#pragma unroll
          for (int v = 0; v < DC; ++v) {
            uint32_t qs[PPW];
#pragma unroll
            for (int q = 0; q < PPW; ++q) qs[q] = add_p(Q0[q][v], Q1[q][v], p);
#pragma unroll
            for (int u = 0; u < BLK; ++u) {
              const uint32_t w = (uint32_t)(u * DC + v) * 64 + lane;
              const uint2 gv = tileG[w];
              const uint32_t gs = tileS[w];
#pragma unroll
              for (int q = 0; q < PPW; ++q) {
                a0[q][u] += (uint64_t)Q0[q][v] * gv.x;
                a2[q][u] += (uint64_t)Q1[q][v] * gv.y;
                as[q][u] += (uint64_t)qs[q] * gs;
              }
            }
          }
        } else {
#pragma unroll
          for (int v = 0; v < DC; ++v) {
            if (v >= dn) break;
            uint32_t qs[PPW];
#pragma unroll
            for (int q = 0; q < PPW; ++q) qs[q] = add_p(Q0[q][v], Q1[q][v], p);
#pragma unroll
            for (int u = 0; u < BLK; ++u) {
              if (u >= nblk) break;
              const uint32_t w = ((uint32_t)u * dn + v) * 64 + lane;
              const uint2 gv = tileG[w];
              const uint32_t gs = tileS[w];
#pragma unroll
              for (int q = 0; q < PPW; ++q) {
                a0[q][u] += (uint64_t)Q0[q][v] * gv.x;
                a2[q][u] += (uint64_t)Q1[q][v] * gv.y;
                as[q][u] += (uint64_t)qs[q] * gs;
              }
            }
          }
        }
#pragma unroll
        for (int q = 0; q < PPW; ++q)
#pragma unroll
          for (int u = 0; u < BLK; ++u) {
            if (u >= nblk) break;
            a0[q][u] = fold34(a0[q][u], c34);
            a2[q][u] = fold34(a2[q][u], c34);
            as[q][u] = fold34(as[q][u], c34);
          }
      }
    }
#pragma unroll
    for (int q = 0; q < PPW; ++q) {
      if (!active[q]) break;
      uint32_t* ob = G.acc + (size_t)(wave * PPW + q) * G.acc_stride;
#pragma unroll
      for (int u = 0; u < BLK; ++u) {
        if (u >= nblk) break;
        const uint64_t x0 = red_p(a0[q][u], p, mu), x2 = red_p(a2[q][u], p, mu), xs = red_p(as[q][u], p, mu);
        // A1 = S - A0 - A2 mod p, all three below p
        uint64_t a1 = xs + 2 * (uint64_t)p - x0 - x2;
        a1 = a1 >= p ? a1 - p : a1;
        a1 = a1 >= p ? a1 - p : a1;
        uint32_t* o = ob + ((size_t)(b0 + u - G.blk_lo) * 3 * K + r) * n + slot;
        o[0] = (uint32_t)x0;
        o[(size_t)K * n] = (uint32_t)a1;
        o[(size_t)2 * K * n] = (uint32_t)x2;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- batched multiply-accumulate on the matrix cores
// For one base prime p and one slot, a group's sums form three matrix
// products over the d dimensions: A_{cc'}[probe][block] = sum_i P_c[probe][i]
// G_c'[block][i] (c, c' the two ciphertext polynomials; A0 = A_00,
// A1 = A_01 + A_10, A2 = A_11).  Every residue v < 2^30 is written in four
// balanced base-256 digits, v = sum_j s_j 256^j with s_0..s_2 in [-128, 127]
// and s_3 in [0, 64] -- the bytes of (v + 0x808080) XOR 0x808080 read as
// signed -- so a product of residues is sum_{i,j} s_i s_j 256^(i+j) and the
// sums over the dimensions are int8 x int8 matrix products, exact in int32
// (|sum| <= d 2^14), on the MFMA units (v_mfma_i32_16x16x64_i8).
// Per slot: 16-row tiles of (probe pair, polynomial, digit i) rows against 16
// columns of (block, polynomial) for 8 blocks, one tile per digit j of the
// gallery; a lane's four results of a tile are its (probe, c, block, c')
// entry for i = 0..3, so with the four j tiles it holds all 16 digit
// products of one entry and recombines them in registers:
// X = sum_k T_k 256^k mod p, T_k = sum_{i+j=k} C_ij, paired exactly in int32
// before the 64-bit sum, one reduction mod p.  The partner entry
// (c, c') = (1, 0) of (0, 1) is 17 lanes away (A1 = X_01 + X_10).
// A workgroup is MF_SLOTS waves, one slot each, over a tile of MF_SLOTS
// neighbouring slots of one prime for one group of up to 16 probes; it keeps
// the probes' digits of its slot in registers (d <= MF_DMAX) and sweeps the
// group's blocks 8 at a time.  The gallery words of 8 blocks x d dimensions x
// the slot tile are staged in LDS, transposed to [slot][block][c'][dim], in two
// buffers: while one group is multiplied, the next is written to the other
// buffer and the one after loads into registers, so a block group costs one
// barrier.  The results go through LDS (two buffers as well) so that every
// row of the tile is written at once.  Work items
// (group, prime, slot tile) are dealt so that the items reading the same
// 128-byte gallery lines (4 tiles x the groups) run on one XCD together.
// Exact like k_mac_multi: the same residues.
#define MF_SLOTS 8
#define MF_BLK 8
#define MF_DMAX 128
#define MF_KC (MF_DMAX / 64)
#define MF_DS (MF_DMAX + 4)                          // staged row of dimensions, padded (LDS banks)
#define MF_PS 68                                     // staged probe row of one 64-dimension step, padded
typedef int mf_v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t bal_digits(uint32_t v) { return (v + 0x00808080u) ^ 0x00808080u; }

// First of the four dimensions a lane's bytes 4 q .. 4 q + 3 of an MFMA operand
// hold within a 64-deep K step (lane group kq = lane / 16): 16 kq + 4 q.
__device__ __forceinline__ uint32_t mf_kbase(uint32_t kq, int q) { return 16 * kq + 4 * q; }

// 4 x 4 byte transpose: out[j] holds byte j of w0, w1, w2, w3 (in that order)
__device__ __forceinline__ void byte_transpose4(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint32_t* out) {
  const uint32_t t0 = __builtin_amdgcn_perm(w1, w0, 0x05010400u);   // w0.b0 w1.b0 w0.b1 w1.b1
  const uint32_t t1 = __builtin_amdgcn_perm(w1, w0, 0x07030602u);   // w0.b2 w1.b2 w0.b3 w1.b3
  const uint32_t t2 = __builtin_amdgcn_perm(w3, w2, 0x05010400u);
  const uint32_t t3 = __builtin_amdgcn_perm(w3, w2, 0x07030602u);
  out[0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
  out[1] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
  out[2] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
  out[3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
}

__global__ void __launch_bounds__(64 * MF_SLOTS, 1)
k_mac_mfma(DevTabs T, MacBatchArgs A) {
  constexpr uint32_t WGL = 64 * MF_SLOTS;
  static_assert(WGL == 2 * 2 * MF_DMAX && MF_SLOTS == 8, "a lane stages one (dimension, polynomial, half-tile) row");
  // LDS: two gallery buffers [slot][block][c'][MF_DS] (one K step of probe words [slot][probe][c][MF_PS]
  // reuses the first), two result buffers [probe][block][comp][slot]
  constexpr uint32_t GAL_WORDS = MF_SLOTS * MF_BLK * 2 * MF_DS, PRB_WORDS = MF_SLOTS * MB_PROBES * 2 * MF_PS;
  constexpr uint32_t OUT_WORDS = MB_PROBES * MF_BLK * 3 * MF_SLOTS;
  static_assert(PRB_WORDS <= 2 * GAL_WORDS, "probe staging fits the gallery buffers");
  __shared__ __attribute__((aligned(16))) uint32_t stg[2 * GAL_WORDS];
  __shared__ __attribute__((aligned(16))) uint32_t outb[2 * OUT_WORDS];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, K = C.K;
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t w = __builtin_amdgcn_readfirstlane(tid >> 6);     // the wave's slot in the tile
  const uint32_t tiles = n / MF_SLOTS;
  const uint32_t ng = (uint32_t)A.ngroups;
  // items: line group lg = (prime, 4 neighbouring tiles) x ng groups; line groups dealt to XCDs by lg mod 8
  const uint32_t nlg = K * tiles / 4;
  const uint32_t nx = gridDim.x % 8 == 0 ? 8 : 1;
  const uint32_t xcd = blockIdx.x % nx, lw = blockIdx.x / nx, nw = gridDim.x / nx;
  const uint32_t per_lg = 4 * ng;
  const uint64_t my_items = nlg > xcd ? (uint64_t)((nlg - xcd + nx - 1) / nx) * per_lg : 0;
  // MFMA lane roles: A rows (l & 15) = (probe pair half, polynomial, digit), B/C columns (l & 15) =
  // (block, polynomial), K range 16 (l >> 4) .. + 15 of a 64-dimension step; C rows 4 (l >> 4) + e
  const uint32_t arow = lane & 15, adig = arow & 3, apc = arow >> 2;
  const uint32_t col = lane & 15, cb = col >> 1, cc = col & 1;
  const uint32_t kq = lane >> 4;
  const uint32_t cpc = lane >> 4;                                     // C: (probe pair half, polynomial) of the lane
  // staging roles: the lane's half tile (4 slots), polynomial and dimension (gallery: one row per
  // block e; probes: probe (tid >> 8) + 2 e, polynomial, dimension of the K step)
  const uint32_t sh = tid & 1, sc = (tid >> 1) & 1, sdim = tid >> 2;
  const uint32_t pc_ = (tid >> 7) & 1, pdim = (tid >> 1) & 63, pj0 = tid >> 8;
  for (uint64_t u = lw; u < my_items; u += nw) {
    const uint32_t lg = xcd + (uint32_t)(u / per_lg) * nx;
    const uint32_t within = (uint32_t)(u % per_lg);
    const uint32_t g = within % ng;
    const uint32_t pair = lg * 4 + within / ng;
    const uint32_t tile = pair % tiles, r = pair / tiles;
    const MacGroup& G = A.g[g];
    const int32_t d = G.d;
    const int kcn = (d + 63) / 64;
    const uint32_t p = C.p[r];
    const uint32_t slot0 = tile * MF_SLOTS;
    // the recombination's constants: 2^(32 + 16 k) mod p for k = 0..3, balanced (|c_k| <= p/2), and
    // -p^-1 mod 2^32 for one Montgomery reduction by 2^32 (p^-1 by Newton's iteration: p p = 1 mod 8
    // for odd p, and each step doubles the correct low bits)
    int32_t cbal[4];
    {
      uint64_t v = (1ull << 32) % p;
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4) {
        cbal[k4] = v > p / 2 ? (int32_t)v - (int32_t)p : (int32_t)v;
        v = (v << 16) % p;
      }
    }
    uint32_t pinv = p;
#pragma unroll
    for (int it = 0; it < 4; ++it) pinv *= 2u - p * pinv;
    const uint32_t npinv = 0u - pinv;
    // ---- the probes' digits of this slot: per K step, rows (probe, c, dim) staged as [slot][probe][c][dim]
    mf_v4i Ad[MF_KC][8];
#pragma unroll
    for (int kc = 0; kc < MF_KC; ++kc) {
      if (kc >= kcn) {
#pragma unroll
        for (int R = 0; R < 8; ++R) Ad[kc][R] = mf_v4i{0, 0, 0, 0};
        continue;
      }
      // two passes, each issuing its loads before the first is written, so their latencies overlap
      constexpr uint32_t PRB_PER_LANE = MB_PROBES * 2 * 64 * (MF_SLOTS / 4) / WGL, PASS = PRB_PER_LANE / 2;
      const int32_t dim = kc * 64 + (int32_t)pdim;
      __syncthreads();                                                // staging buffer free
#pragma unroll
      for (uint32_t e0 = 0; e0 < PRB_PER_LANE; e0 += PASS) {
        u32x4 av[PASS];
#pragma unroll
        for (uint32_t e = 0; e < PASS; ++e) {
          const uint32_t j = pj0 + 2 * (e0 + e);
          av[e] = u32x4{0u, 0u, 0u, 0u};
          if ((int32_t)j < G.nprobe && dim < d)
            av[e] = *(const u32x4*)(G.probe[j] + (((size_t)r * d + dim) * 2 + pc_) * n + slot0 + 4 * sh);
        }
#pragma unroll
        for (uint32_t e = 0; e < PASS; ++e) {
          const uint32_t j = pj0 + 2 * (e0 + e);
#pragma unroll
          for (int s = 0; s < 4; ++s) stg[(((4 * sh + s) * MB_PROBES + j) * 2 + pc_) * MF_PS + pdim] = av[e][s];
        }
      }
      __syncthreads();
#pragma unroll
      for (int R = 0; R < 8; ++R) {
        const uint32_t j = 2 * R + (apc >> 1), c = apc & 1;
        const uint32_t* src = stg + ((w * MB_PROBES + j) * 2 + c) * MF_PS;
        uint32_t dg[4];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const u32x4 v = *(const u32x4*)(src + mf_kbase(kq, q4));
          uint32_t tr[4];
          byte_transpose4(bal_digits(v[0]), bal_digits(v[1]), bal_digits(v[2]), bal_digits(v[3]), tr);
          dg[q4] = adig == 0 ? tr[0] : adig == 1 ? tr[1] : adig == 2 ? tr[2] : tr[3];
        }
        Ad[kc][R] = mf_v4i{(int)dg[0], (int)dg[1], (int)dg[2], (int)dg[3]};
      }
    }
    // ---- gallery block groups of MF_BLK blocks, double-buffered in LDS; the group after next loads
    // into registers while the next is staged and the current one multiplied
    const int64_t nbg = (G.blk_hi - G.blk_lo + MF_BLK - 1) / MF_BLK;
    const size_t bstride = (size_t)K * d * 2 * n;                     // words between blocks
    const bool dim_ok = (int32_t)sdim < d;
    const size_t lane_off = ((size_t)sdim * 2 + sc) * n + 4 * sh;
    u32x4 pre[MF_BLK];
    auto fetch = [&](int64_t bg) {
      const int64_t b0 = G.blk_lo + bg * MF_BLK;
      const uint32_t* base = G.gallery + ((size_t)b0 * K + r) * d * 2 * n + slot0 + lane_off;
#pragma unroll
      for (uint32_t e = 0; e < MF_BLK; ++e) {
        pre[e] = u32x4{0u, 0u, 0u, 0u};
        if (dim_ok && b0 + e < G.blk_hi) pre[e] = *(const u32x4*)(base + e * bstride);
      }
    };
    auto stage = [&](uint32_t* buf) {
#pragma unroll
      for (uint32_t e = 0; e < MF_BLK; ++e)
#pragma unroll
        for (int s = 0; s < 4; ++s) buf[(((4 * sh + s) * MF_BLK + e) * 2 + sc) * MF_DS + sdim] = pre[e][s];
    };
    fetch(0);
    __syncthreads();                                                  // the probe staging's reads are done
    stage(stg);
    if (nbg > 1) fetch(1);
    __syncthreads();
    for (int64_t bg = 0; bg < nbg; ++bg) {
      const int64_t b0 = G.blk_lo + bg * MF_BLK;
      const uint32_t cur = (uint32_t)(bg & 1);
      const uint32_t* gcur = stg + cur * GAL_WORDS;
      uint32_t* ocur = outb + cur * OUT_WORDS;
      // B operands of this lane: digits j of (block cb, polynomial cc) over its 16 dimensions per K step
      mf_v4i Bd[MF_KC][4];
#pragma unroll
      for (int kc = 0; kc < MF_KC; ++kc) {
        if (kc >= kcn) {                                               // zero digits beyond d (A is zero there too)
#pragma unroll
          for (int j = 0; j < 4; ++j) Bd[kc][j] = mf_v4i{0, 0, 0, 0};
          continue;
        }
        const uint32_t* src = gcur + ((w * MF_BLK + cb) * 2 + cc) * MF_DS + kc * 64;
        uint32_t tr[4][4];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const u32x4 v = *(const u32x4*)(src + mf_kbase(kq, q4));
          byte_transpose4(bal_digits(v[0]), bal_digits(v[1]), bal_digits(v[2]), bal_digits(v[3]), tr[q4]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) Bd[kc][j] = mf_v4i{(int)tr[0][j], (int)tr[1][j], (int)tr[2][j], (int)tr[3][j]};
      }
      // row tile R's products go to the matrix cores before tile R - 1 is recombined on the VALU, so the
      // two overlap (two accumulator sets)
      auto products = [&](int R, mf_v4i (&acc)[4]) {
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = mf_v4i{0, 0, 0, 0};
        // every K step, also past d (zero operands there): no branch between the MFMAs, so the
        // scheduler can interleave them with the VALU work
#pragma unroll
        for (int kc = 0; kc < MF_KC; ++kc)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(Ad[kc][R], Bd[kc][j], acc[j], 0, 0, 0);
      };
      auto recombine = [&](int R, const mf_v4i (&acc)[4]) {
        // acc[j][i] = C_ij of (probe 2R + (cpc >> 1), c = cpc & 1, block cb, c' = cc).  The digit-column
        // sums T_k = sum_{i+j=k} C_ij pair up exactly in int32 (d <= 128: |C_ij| <= 2^21, 2^20 with a
        // digit 3 in [0, 64], 2^19 for C_33): U0 = T0 + 2^8 T1, U1 = T2 + 2^8 T3, U2 = T4 + 2^8 T5,
        // U3 = T6, each below 2^31 in magnitude, and X = U0 + 2^16 U1 + 2^32 U2 + 2^48 U3 mod p.
        // S = sum_k U_k c_k (c_k = 2^(32 + 16 k) mod p, balanced) is X 2^32 mod p with |S| < 2^32 p;
        // with m = -S p^-1 mod 2^32, S + m p is divisible by 2^32, and (S + m p) / 2^32, congruent
        // to X, lies in (-p, 2p): one conditional add and one conditional subtract of p remain
        const int32_t U0 = acc[0][0] + 256 * (acc[0][1] + acc[1][0]);
        const int32_t U1 = (acc[0][2] + acc[1][1] + acc[2][0]) + 256 * (acc[0][3] + acc[1][2] + acc[2][1] + acc[3][0]);
        const int32_t U2 = (acc[1][3] + acc[2][2] + acc[3][1]) + 256 * (acc[2][3] + acc[3][2]);
        const int32_t U3 = acc[3][3];
        const int64_t S = (int64_t)U0 * cbal[0] + (int64_t)U1 * cbal[1] + (int64_t)U2 * cbal[2] +
                          (int64_t)U3 * cbal[3];
        const uint32_t mq = (uint32_t)S * npinv;
        int32_t xt = (int32_t)(uint32_t)(((uint64_t)S + (uint64_t)mq * p) >> 32);
        xt += xt < 0 ? (int32_t)p : 0;
        const uint32_t X = (uint32_t)xt >= p ? (uint32_t)xt - p : (uint32_t)xt;
        const uint32_t Xp = (uint32_t)__shfl_xor((int)X, 17);          // (c, c') swapped
        const uint32_t c = cpc & 1;
        if (c == 0 || cc == 1) {                                       // (0,0) A0, (0,1) A1, (1,1) A2
          const uint32_t comp = c + cc;
          const uint32_t v = (c == 0 && cc == 1) ? add_p(X, Xp, p) : X;
          ocur[(((2 * R + (cpc >> 1)) * MF_BLK + cb) * 3 + comp) * MF_SLOTS + w] = v;
        }
      };
      mf_v4i accA[4], accB[4];
      products(0, accA);
      // the scheduler interleaves each tile's 8 MFMAs with the previous tile's recombination (one MFMA,
      // then up to 6 VALU instructions), so the matrix core and the VALU work side by side
      auto interleave = [&]() {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);
        }
      };
#pragma unroll
      for (int R = 0; R < 8; R += 2) {
        if (R + 1 < 8) products(R + 1, accB);
        recombine(R, accA);
        if (R + 1 < 8) interleave();
        if (R + 2 < 8) products(R + 2, accA);
        recombine(R + 1, accB);
        if (R + 2 < 8) interleave();
      }
      if (bg + 1 < nbg) stage(stg + (cur ^ 1) * GAL_WORDS);           // the next group, loaded meanwhile
      __syncthreads();
      if (bg + 2 < nbg) fetch(bg + 2);
      // rows (probe, block, comp) of MF_SLOTS words
#pragma unroll
      for (uint32_t it = 0; it < (OUT_WORDS / 4 + WGL - 1) / WGL; ++it) {
        const uint32_t e = tid + it * WGL;
        const uint32_t half = e % (MF_SLOTS / 4), row = e / (MF_SLOTS / 4);
        const uint32_t j = row / (MF_BLK * 3), b = (row / 3) % MF_BLK, comp = row % 3;
        if (e >= OUT_WORDS / 4 || (int32_t)j >= G.nprobe || b0 + b >= G.blk_hi) continue;
        const u32x4 v = *(const u32x4*)(ocur + row * MF_SLOTS + 4 * half);
        *(u32x4*)(G.acc + (size_t)j * G.acc_stride + (((size_t)(b0 + b - G.blk_lo) * 3 + comp) * K + r) * n + slot0 +
                  4 * half) = v;
      }
    }
  }
}

template <int KQ, int KP, int FW>
__global__ void __launch_bounds__(WG)
k_rescale(DevTabs T, const uint32_t* __restrict__ Xb, int64_t nblk, int64_t blk_lo, ScorePtrs SP,
          uint64_t* __restrict__ digits_b, uint64_t acc_stride, uint64_t dig_stride) {
  // Per coefficient of X_j (j = 0, 1, 2; residues mod p_r, |X| < P/4):
  // c_j = [round(t X_j / q)]_q.  c0, c1 go to the score ciphertext (before
  // relinearization); c2 is split into the gadget digits y_g.  Request
  // blockIdx.y of the round: accumulators at Xb + y acc_stride, digits at
  // digits_b + y dig_stride, score ciphertexts SP.p[y].
  const uint32_t* __restrict__ X = Xb + (size_t)blockIdx.y * acc_stride;
  uint64_t* __restrict__ digits = digits_b + (size_t)blockIdx.y * dig_stride;
  uint64_t* __restrict__ scores = SP.p[blockIdx.y];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = C.k, K = C.K, L = C.L;
  const uint64_t idx = (uint64_t)blockIdx.x * WG + threadIdx.x;
  if (idx >= (uint64_t)nblk * 3 * n) return;
  const uint64_t bj = idx >> C.logn;                  // n is a power of two
  const uint32_t c = (uint32_t)(idx & (n - 1));
  const int64_t bl = (int64_t)(bj / 3);
  const uint32_t j = (uint32_t)(bj % 3);
  uint32_t x[KP ? KP : HC_MAXP];
  for (uint32_t r = 0; r < (KP ? KP : K); ++r) x[r] = X[(bj * K + r) * n + c];
  uint64_t out[KQ ? KQ : HC_MAXQ];
  if (scale_round_coeff<KQ, KP, FW, false>(C, x, out)) {
    // two-word fraction within 2^-64 of 1/2 (rare): all W words.  The
    // residues and constants are read again, so that nothing of the two-word
    // pass stays live across it.
    const volatile uint32_t* Xv = X;
    for (uint32_t r = 0; r < (KP ? KP : K); ++r) x[r] = Xv[(bj * K + r) * n + c];
    scale_round_coeff<KQ, KP, FW, true>(*T.C_rare, x, out);
  }
  const int64_t b = blk_lo + bl;
  if (j < 2) {
    for (uint32_t i = 0; i < k; ++i) scores[(((size_t)b * 2 + j) * k + i) * n + c] = out[i];
    return;
  }
  // gadget digits come prime-major (all digits of q_rho, then of q_rho+1), so
  // out[rho] is indexed by the unrolled loop counter.  Each digit is written
  // once, as the integer it is (below q_rho, or 2^w_bits), in the slot of
  // residue 0 of its [L][k][n] block: the relinearization reduces it mod
  // every q_sigma as it reads it.
  uint32_t g = 0;
#pragma unroll
  for (uint32_t rho = 0; rho < (KQ ? KQ : k); ++rho) {
    const uint64_t y = shoup_q(out[rho], C.q_hatinv[rho], C.q_hatinv_sh[rho], C.q[rho]);
    if (!C.w_bits) {                                    // one digit per prime: digit rho is y itself
      digits[((size_t)bl * L + rho) * k * n + c] = y;
      continue;
    }
    for (; g < L && C.g_rho[g] == rho; ++g)
      digits[((size_t)bl * L + g) * k * n + c] = (y >> C.g_shift[g]) & ((1ULL << C.w_bits) - 1);
  }
}

template <bool QF>
__global__ void __launch_bounds__(WG)
k_ntt_q(DevTabs T, uint64_t* __restrict__ digits, uint64_t set_stride) {
  // Relinearization digits, first half: digit polynomial blockIdx.x (a
  // block's digit g) of set blockIdx.y is an integer polynomial stored once,
  // in the slot of residue 0 of its [k][n] row ([..][L][k][n]).  For every
  // q_sigma, last sigma first, read it (from cache after the first time),
  // reduce it, transform it forward (negacyclic NTT) and write residue sigma;
  // residue 0 overwrites the integer polynomial only after its last read.
  // QF: in double precision with balanced butterflies (ModQB), same residues.
  extern __shared__ uint64_t lds64[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = C.k, tid = threadIdx.x;
  uint64_t* a = digits + (size_t)blockIdx.y * set_stride + (size_t)blockIdx.x * k * n;
  const bool one_sub = C.dig_one_sub != 0;
  for (int32_t sg = (int32_t)k - 1; sg >= 0; --sg) {
    const uint64_t q = C.q[sg], mu = C.q_mu64[sg];
    __syncthreads();                                    // the previous residue's transform written back
    if constexpr (QF) {
      double* f = reinterpret_cast<double*>(lds64);
      load_padded(f, a, n, tid, WG, [&](uint64_t v) { return u64_to_f(one_sub ? (v >= q ? v - q : v) : red_q(v, q, mu)); });
      __syncthreads();
      ntt_forward_b(f, T.qtw_f + (size_t)sg * n, ModQB{T.qf[sg], T.qf[HC_MAXQ + sg]}, n, C.logn, tid, WG, T.ntt_r);
      for (uint32_t j = tid; j < n; j += WG) a[(size_t)sg * n + j] = f_to_u64(f[PADX(j)]);
    } else {
      load_padded(lds64, a, n, tid, WG, [&](uint64_t v) { return one_sub ? (v >= q ? v - q : v) : red_q(v, q, mu); });
      __syncthreads();
      ntt_forward16(lds64, T.qtw + (size_t)sg * n, T.qtw_sh + (size_t)sg * n, ModQ{q}, n, C.logn, tid, WG, T.ntt_r);
      for (uint32_t j = tid; j < n; j += WG) a[(size_t)sg * n + j] = lds64[PADX(j)];
    }
  }
}

template <bool QF, int NT>
__global__ void __launch_bounds__(NT)
k_relin_acc(DevTabs T, const uint64_t* __restrict__ digits_b, int64_t blk_lo, ScorePtrs SP, uint64_t dig_stride,
            const uint64_t* __restrict__ key, const uint64_t* __restrict__ key_sh) {
  // Relinearization (or key switching), second half, for residue sigma =
  // blockIdx.y of request z: c_comp += INTT(sum_g NTT(y_g) * key_g[comp])
  // mod q_sigma, key [L][2][k][n] in NTT form (the evaluation keys, or a
  // rotation key).  QF: one workgroup per block does both components -- one
  // pass over the digits (each read once) accumulates both key products, in
  // double precision, into two LDS buffers, then the two inverse transforms.
  // Otherwise one workgroup per (block blockIdx.x / 2, component
  // blockIdx.x mod 2), neighbours, so the second reads the digits from cache.
  extern __shared__ uint64_t lds64[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = C.k, L = C.L, tid = threadIdx.x;
  const uint32_t sg = blockIdx.y;
  const uint64_t q = C.q[sg];
  if constexpr (QF) {
    const int64_t bl = blockIdx.x, b = blk_lo + bl;
    const uint64_t* digits = digits_b + (size_t)blockIdx.z * dig_stride + (size_t)bl * L * k * n;
    uint64_t* dst0 = SP.p[blockIdx.z] + (((size_t)b * 2 + 0) * k + sg) * n;
    uint64_t* dst1 = SP.p[blockIdx.z] + (((size_t)b * 2 + 1) * k + sg) * n;
    // RA coefficients per lane at a time, so each digit's loads for all of
    // them are in flight together (the digit loop has a runtime bound); rings
    // smaller than RA NT coefficients take one coefficient at a time
    constexpr uint32_t RA = 4;
    const ModQF mq{T.qf[sg], T.qf[HC_MAXQ + sg]};
    double* f0 = reinterpret_cast<double*>(lds64);
    double* f1 = f0 + padded_len(n);
    const bool batched = n % (RA * NT) == 0;
    const uint32_t ra = batched ? RA : 1;
    for (uint32_t j0 = tid; j0 < n; j0 += ra * NT) {
      double a0[RA], a1[RA];
#pragma unroll
      for (uint32_t u = 0; u < RA; ++u) { a0[u] = 0.0; a1[u] = 0.0; }
      for (uint32_t g = 0; g < L; ++g) {
        const uint64_t* dg = digits + ((size_t)g * k + sg) * n + j0;
        const uint64_t* k0 = key + (((size_t)g * 2 + 0) * k + sg) * n + j0;
        const uint64_t* k1 = key + (((size_t)g * 2 + 1) * k + sg) * n + j0;
        uint64_t dv[RA], kv0[RA], kv1[RA];
#pragma unroll
        for (uint32_t u = 0; u < RA; ++u) {
          if (u >= ra) break;
          dv[u] = dg[u * NT];
          kv0[u] = k0[u * NT];
          kv1[u] = k1[u * NT];
        }
#pragma unroll
        for (uint32_t u = 0; u < RA; ++u) {
          if (u >= ra) break;
          const double dd = u64_to_f(dv[u]);
          const double s0 = a0[u] + mq.mul(dd, u64_to_f(kv0[u]), 0.0);
          const double s1 = a1[u] + mq.mul(dd, u64_to_f(kv1[u]), 0.0);
          a0[u] = s0 >= mq.q ? s0 - mq.q : s0;
          a1[u] = s1 >= mq.q ? s1 - mq.q : s1;
        }
      }
      for (uint32_t u = 0; u < ra; ++u) {
        f0[PADX(j0 + u * NT)] = a0[u];
        f1[PADX(j0 + u * NT)] = a1[u];
      }
    }
    __syncthreads();
    const double* itw = T.qitw_f + (size_t)sg * n;
    const double ninv = T.qf[2 * HC_MAXQ + sg];
    for (int comp = 0; comp < 2; ++comp) {
      double* f = comp ? f1 : f0;
      uint64_t* dst = comp ? dst1 : dst0;
      ntt_inverse_b(f, itw, ninv, ModQB{mq.q, mq.qinv}, n, C.logn, tid, NT, T.ntt_r);
      if (batched) {
        for (uint32_t j0 = tid; j0 < n; j0 += RA * NT) {
          uint64_t dv[RA];
#pragma unroll
          for (uint32_t u = 0; u < RA; ++u) dv[u] = dst[j0 + u * NT];
#pragma unroll
          for (uint32_t u = 0; u < RA; ++u) dst[j0 + u * NT] = add_q(dv[u], f_to_u64(f[PADX(j0 + u * NT)]), q);
        }
      } else {
        for (uint32_t j = tid; j < n; j += NT) dst[j] = add_q(dst[j], f_to_u64(f[PADX(j)]), q);
      }
    }
    return;
  }
  const int64_t bl = blockIdx.x >> 1, b = blk_lo + bl;
  const uint32_t comp = blockIdx.x & 1;
  const uint64_t* digits = digits_b + (size_t)blockIdx.z * dig_stride + (size_t)bl * L * k * n;
  uint64_t* dst = SP.p[blockIdx.z] + (((size_t)b * 2 + comp) * k + sg) * n;
  for (uint32_t j = tid; j < n; j += NT) {
    uint64_t acc = 0;
    for (uint32_t g = 0; g < L; ++g) {
      const size_t r = (((size_t)g * 2 + comp) * k + sg) * n + j;
      acc = add_q(acc, shoup_q(digits[((size_t)g * k + sg) * n + j], key[r], key_sh[r], q), q);
    }
    lds64[PADX(j)] = acc;
  }
  __syncthreads();
  ntt_inverse16(lds64, T.qitw + (size_t)sg * n, T.qitw_sh + (size_t)sg * n, C.q_ninv[sg], C.q_ninv_sh[sg],
                ModQ{q}, n, C.logn, tid, NT, T.ntt_r);
  for (uint32_t j = tid; j < n; j += NT) dst[j] = add_q(dst[j], lds64[PADX(j)], q);
}

// Fused relinearization / key switching: one workgroup per (block, residue
// sigma, request) of n / PER lanes, each owning PER coefficients.  For
// every gadget digit the digit polynomial mod q_sigma is transformed in LDS
// and multiplied into both key components, accumulated in registers; then
// the two sums are transformed back and added to c0, c1.  Same result as the
// digit transforms of k_ntt_q followed by k_relin_acc, without writing the
// transformed digits to memory.  PER 16: 512-lane workgroups (n = 8192),
// two waves per SIMD with room for the next digit's loads in registers;
// PER 8: 1024-lane workgroups, four waves per SIMD, no prefetch.
template <bool QF, int PER>
__global__ void __launch_bounds__(PER >= 16 ? 512 : 1024)
k_relin_fused(DevTabs T, const uint64_t* __restrict__ digits_b, int64_t blk_lo, ScorePtrs SP, uint64_t dig_stride,
              const uint64_t* __restrict__ key, const uint64_t* __restrict__ key_sh) {
  // QF: the key products (ModQF) and the transforms (balanced, ModQB) in
  // double precision on elements of type E, converted at the memory edges
  using E = typename std::conditional<QF, double, uint64_t>::type;
  using M = typename std::conditional<QF, ModQF, ModQ>::type;
  constexpr int RX = PER >= 16 ? 4 : 3;                 // radix-8 passes at most with 8 per lane (registers)
  extern __shared__ uint64_t lds64[];
  E* a = reinterpret_cast<E*>(lds64);
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = C.k, L = C.L, tid = threadIdx.x, nthr = blockDim.x;
  const int64_t bl = blockIdx.x, b = blk_lo + bl;
  const uint32_t sg = blockIdx.y;
  const uint64_t q = C.q[sg];
  M mod;
  const E *tw, *twsh, *itw, *itwsh;
  E ninv, ninv_sh;
  if constexpr (QF) {
    mod = ModQF{T.qf[sg], T.qf[HC_MAXQ + sg]};
    tw = twsh = T.qtw_f + (size_t)sg * n;
    itw = itwsh = T.qitw_f + (size_t)sg * n;
    ninv = ninv_sh = T.qf[2 * HC_MAXQ + sg];
  } else {
    mod = ModQ{q};
    tw = T.qtw + (size_t)sg * n;
    twsh = T.qtw_sh + (size_t)sg * n;
    itw = T.qitw + (size_t)sg * n;
    itwsh = T.qitw_sh + (size_t)sg * n;
    ninv = C.q_ninv[sg];
    ninv_sh = C.q_ninv_sh[sg];
  }
  auto in = [](uint64_t v) -> E { if constexpr (QF) return u64_to_f(v); else return v; };
  auto out = [](E v) -> uint64_t { if constexpr (QF) return f_to_u64(v); else return v; };
  // acc + D key mod q, both accumulators fully reduced
  auto mac = [&](E acc, E D, uint64_t kw, uint64_t ks) -> E {
    if constexpr (QF) {
      const E s = acc + mod.mul(D, u64_to_f(kw), 0.0);
      return s >= mod.q ? s - mod.q : s;
    } else {
      return add_q(acc, shoup_q(D, kw, ks, q), q);
    }
  };
  const uint64_t* digits = digits_b + (size_t)blockIdx.z * dig_stride + (size_t)bl * L * k * n;
  // a digit is stored once, as an integer (slot of residue 0): reduced mod q_sigma here
  const uint64_t qmu = C.q_mu64[sg];
  const bool one_sub = C.dig_one_sub != 0;
  auto red_dig = [&](uint64_t v) -> uint64_t { return one_sub ? (v >= q ? v - q : v) : red_q(v, q, qmu); };
  E acc0[PER], acc1[PER];
#pragma unroll PER
  for (uint32_t e = 0; e < PER; ++e) { acc0[e] = 0; acc1[e] = 0; }
  // f64 form with PER 16: digit g + 1 is loaded into registers while digit g
  // is transformed (the integer form has no registers to spare for it)
  constexpr bool PF = QF && PER >= 16;
  uint64_t pre[PF ? PER : 1];
  if constexpr (PF) {
#pragma unroll PER
    for (uint32_t e = 0; e < PER; ++e) pre[e] = tid + e * nthr < n ? digits[tid + e * nthr] : 0;
  }
  // double-precision form with the transforms' edge passes in registers: the
  // first forward pass on the digit as loaded, the last inverse pass on the
  // way out (a lane's PER coefficients tid + e n / PER are those passes'
  // elements when the workgroup has n / PER lanes and the passes may span
  // log2 PER stages)
  constexpr int LP = PER >= 16 ? 4 : 3;
  const bool edge_regs = QF && !PF && (nthr << LP) == n && C.logn > (uint32_t)LP && T.ntt_r >= (uint32_t)LP;
  for (uint32_t g = 0; g < L; ++g) {
    if constexpr (QF && !PF) {
      if (edge_regs) {
        const uint64_t* dg = digits + (size_t)g * k * n;
        double x[PER];
#pragma unroll PER
        for (uint32_t e = 0; e < PER; ++e) x[e] = in(red_dig(dg[tid + e * nthr]));
        const ModQB mb{mod.q, mod.qinv};
        ntt_fwd_first_regs_b<LP>(x, tw, mb);
        __syncthreads();                                // previous digit's products read
#pragma unroll PER
        for (uint32_t e = 0; e < PER; ++e) a[PADX(tid + e * nthr)] = x[e];
        __syncthreads();
        ntt_forward_b_from<RX>(a, tw, mb, n, C.logn, LP, tid, nthr, T.ntt_r);
        const size_t k0 = (((size_t)g * 2 + 0) * k + sg) * n, k1 = (((size_t)g * 2 + 1) * k + sg) * n;
#pragma unroll PER
        for (uint32_t e = 0; e < PER; ++e) {
          const uint32_t j = tid + e * nthr;
          const E D = a[PADX(j)];
          acc0[e] = mac(acc0[e], D, key[k0 + j], key_sh[k0 + j]);
          acc1[e] = mac(acc1[e], D, key[k1 + j], key_sh[k1 + j]);
        }
        continue;
      }
    }
    __syncthreads();                                    // previous digit's products read
    if constexpr (PF) {
#pragma unroll PER
      for (uint32_t e = 0; e < PER; ++e)                // reduced here, not at the load, which stays in flight
        if (tid + e * nthr < n) a[PADX(tid + e * nthr)] = in(red_dig(pre[e]));
    } else {
      const uint64_t* dg = digits + (size_t)g * k * n;
#pragma unroll PER
      for (uint32_t e = 0; e < PER; ++e)
        if (tid + e * nthr < n) a[PADX(tid + e * nthr)] = in(red_dig(dg[tid + e * nthr]));
    }
    __syncthreads();
    if constexpr (PF) {
      if (g + 1 < L) {
        const uint64_t* dn = digits + (size_t)(g + 1) * k * n;
#pragma unroll PER
        for (uint32_t e = 0; e < PER; ++e) pre[e] = tid + e * nthr < n ? dn[tid + e * nthr] : 0;
      }
    }
    if constexpr (QF)
      ntt_forward_b<RX>(a, tw, ModQB{mod.q, mod.qinv}, n, C.logn, tid, nthr, T.ntt_r);
    else
      ntt_forward16<RX>(a, tw, twsh, mod, n, C.logn, tid, nthr, T.ntt_r);
    const size_t k0 = (((size_t)g * 2 + 0) * k + sg) * n, k1 = (((size_t)g * 2 + 1) * k + sg) * n;
#pragma unroll PER
    for (uint32_t e = 0; e < PER; ++e) {
      const uint32_t j = tid + e * nthr;
      if (j >= n) break;                                // never on the GPU: n / PER lanes
      const E D = a[PADX(j)];
      acc0[e] = mac(acc0[e], D, key[k0 + j], key_sh[k0 + j]);
      acc1[e] = mac(acc1[e], D, key[k1 + j], key_sh[k1 + j]);
    }
  }
  for (uint32_t comp = 0; comp < 2; ++comp) {
    __syncthreads();
#pragma unroll PER
    for (uint32_t e = 0; e < PER; ++e)
      if (tid + e * nthr < n) a[PADX(tid + e * nthr)] = comp ? acc1[e] : acc0[e];
    __syncthreads();
    if constexpr (QF && !PF) {
      if (edge_regs) {
        const ModQB mb{mod.q, mod.qinv};
        ntt_inverse_b_upto<RX>(a, itw, mb, n, C.logn - LP, tid, nthr, T.ntt_r);
        double x[PER];
#pragma unroll PER
        for (uint32_t e = 0; e < PER; ++e) x[e] = a[PADX(tid + e * nthr)];
        ntt_inv_last_regs_b<LP>(x, itw, ninv, mb);
        uint64_t* dst = SP.p[blockIdx.z] + (((size_t)b * 2 + comp) * k + sg) * n;
#pragma unroll PER
        for (uint32_t e = 0; e < PER; ++e) {
          const uint32_t j = tid + e * nthr;
          dst[j] = add_q(dst[j], out(x[e]), q);
        }
        continue;
      }
    }
    if constexpr (QF)
      ntt_inverse_b<RX>(a, itw, ninv, ModQB{mod.q, mod.qinv}, n, C.logn, tid, nthr, T.ntt_r);
    else
      ntt_inverse16<RX>(a, itw, itwsh, ninv, ninv_sh, mod, n, C.logn, tid, nthr, T.ntt_r);
    uint64_t* dst = SP.p[blockIdx.z] + (((size_t)b * 2 + comp) * k + sg) * n;
#pragma unroll PER
    for (uint32_t e = 0; e < PER; ++e) {
      const uint32_t j = tid + e * nthr;
      if (j >= n) break;
      dst[j] = add_q(dst[j], out(a[PADX(j)]), q);
    }
  }
}

extern "C" __global__ void __launch_bounds__(WG)
k_sk_ntt(DevTabs T, const uint8_t* __restrict__ sk, uint64_t* __restrict__ S, uint64_t* __restrict__ Ssh) {
  // NTT of the secret key mod q_sigma with Shoup companions (decryption).
  extern __shared__ uint64_t lds64[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, tid = threadIdx.x, sg = blockIdx.x;
  const uint64_t q = C.q[sg];
  for (uint32_t j = tid; j < n; j += WG) lds64[PADX(j)] = sk[j] ? 1 : 0;
  __syncthreads();
  ntt_forward16(lds64, T.qtw + (size_t)sg * n, T.qtw_sh + (size_t)sg * n, ModQ{q}, n, C.logn, tid, WG, T.ntt_r);
  for (uint32_t j = tid; j < n; j += WG) {
    S[(size_t)sg * n + j] = lds64[PADX(j)];
    Ssh[(size_t)sg * n + j] = shoup_companion_q(lds64[PADX(j)], q, C.q_m128h[sg], C.q_m128l[sg]);
  }
}

template <bool QF, int NT>
__global__ void __launch_bounds__(NT)
k_dec_mul(DevTabs T, const uint64_t* __restrict__ scores, int64_t blk_lo, const uint64_t* __restrict__ S,
          const uint64_t* __restrict__ Ssh, uint64_t* __restrict__ xout) {
  // x = [c0 + c1 s]_q for block blk_lo + blockIdx.x, residue sigma; NT lanes
  // (512 at n = 8192, where a 256-lane workgroup's LDS share would leave two
  // waves per SIMD).
  extern __shared__ uint64_t lds64[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = C.k, tid = threadIdx.x, sg = blockIdx.y;
  const int64_t bl = blockIdx.x, b = blk_lo + bl;
  const uint64_t q = C.q[sg];
  const ModQ mq{q};
  const uint64_t* c0 = scores + (((size_t)b * 2 + 0) * k + sg) * n;
  const uint64_t* c1 = scores + (((size_t)b * 2 + 1) * k + sg) * n;
  if constexpr (QF) {
    // the same product in double precision: transforms balanced (ModQB), product by ModQF
    double* f = reinterpret_cast<double*>(lds64);
    const ModQF mf{T.qf[sg], T.qf[HC_MAXQ + sg]};
    const double* twf = T.qtw_f + (size_t)sg * n;
    const ModQB mb{mf.q, mf.qinv};
    if (n == 16u * NT && C.logn > 4 && T.ntt_r >= 4) {
      // 16 coefficients per lane, tid + e NT: the elements of the first
      // forward pass and of the last inverse pass, which run in registers on
      // c1 as loaded and on the way out (as in k_relin_fused)
      const double* itwf = T.qitw_f + (size_t)sg * n;
      double xr[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) xr[e] = u64_to_f(c1[tid + e * NT]);
      ntt_fwd_first_regs_b<4>(xr, twf, mb);
#pragma unroll
      for (int e = 0; e < 16; ++e) f[PADX(tid + e * NT)] = xr[e];
      __syncthreads();
      ntt_forward_b_from<4>(f, twf, mb, n, C.logn, 4, tid, NT, T.ntt_r);
      for_each_loaded(S + (size_t)sg * n, n, tid, NT,
                      [&](uint32_t j, uint64_t sv) { f[PADX(j)] = mf.mul(f[PADX(j)], u64_to_f(sv), 0.0); });
      __syncthreads();
      ntt_inverse_b_upto<4>(f, itwf, mb, n, C.logn - 4, tid, NT, T.ntt_r);
#pragma unroll
      for (int e = 0; e < 16; ++e) xr[e] = f[PADX(tid + e * NT)];
      ntt_inv_last_regs_b<4>(xr, itwf, T.qf[2 * HC_MAXQ + sg], mb);
      uint64_t* xo = xout + ((size_t)bl * k + sg) * n;
#pragma unroll
      for (int e = 0; e < 16; ++e) xo[tid + e * NT] = add_q(f_to_u64(xr[e]), c0[tid + e * NT], q);
      return;
    }
    load_padded(f, c1, n, tid, NT, [](uint64_t v) { return u64_to_f(v); });
    __syncthreads();
    ntt_forward_b(f, twf, mb, n, C.logn, tid, NT, T.ntt_r);
    for_each_loaded(S + (size_t)sg * n, n, tid, NT,
                    [&](uint32_t j, uint64_t sv) { f[PADX(j)] = mf.mul(f[PADX(j)], u64_to_f(sv), 0.0); });
    __syncthreads();
    const double* itwf = T.qitw_f + (size_t)sg * n;
    const double ninv = T.qf[2 * HC_MAXQ + sg];
    ntt_inverse_b(f, itwf, ninv, mb, n, C.logn, tid, NT, T.ntt_r);
    uint64_t* xo = xout + ((size_t)bl * k + sg) * n;
    for_each_loaded(c0, n, tid, NT, [&](uint32_t j, uint64_t v0) { xo[j] = add_q(f_to_u64(f[PADX(j)]), v0, q); });
    return;
  }
  load_padded(lds64, c1, n, tid, NT, [](uint64_t v) { return v; });
  __syncthreads();
  ntt_forward16(lds64, T.qtw + (size_t)sg * n, T.qtw_sh + (size_t)sg * n, mq, n, C.logn, tid, NT, T.ntt_r);
  for (uint32_t j = tid; j < n; j += NT)
    lds64[PADX(j)] = shoup_q(lds64[PADX(j)], S[(size_t)sg * n + j], Ssh[(size_t)sg * n + j], q);
  __syncthreads();
  ntt_inverse16(lds64, T.qitw + (size_t)sg * n, T.qitw_sh + (size_t)sg * n, C.q_ninv[sg], C.q_ninv_sh[sg], mq,
              n, C.logn, tid, NT, T.ntt_r);
  for (uint32_t j = tid; j < n; j += NT) xout[((size_t)bl * k + sg) * n + j] = add_q(lds64[PADX(j)], c0[j], q);
}

template <int KQ>
__global__ void __launch_bounds__(WG_DEC)
k_dec_decode(DevTabs T, const uint64_t* __restrict__ x, int64_t blk_lo, int64_t m, int32_t* __restrict__ out) {
  // pt = [round(t x / q)]_t coefficient-wise, then slot j = pt(psi^(2j+1))
  // (forward NTT mod t, read at brv(j)), centred into [-t/2, t/2).  KQ: the
  // number of q primes at compile time (0: read from C).
  extern __shared__ uint32_t lds32[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = KQ ? KQ : C.k, tid = threadIdx.x, t = C.t;
  const int64_t bl = blockIdx.x, b = blk_lo + bl;
  if (KQ && n % (4 * WG_DEC) == 0) {
    // four coefficients per lane, all their residues loaded before the Garner work
    for (uint32_t j0 = tid; j0 < n; j0 += 4 * WG_DEC) {
      uint64_t v[4][KQ ? KQ : 1];
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u)
#pragma unroll
        for (uint32_t i = 0; i < (KQ ? KQ : 1); ++i) v[u][i] = x[((size_t)bl * k + i) * n + j0 + u * WG_DEC];
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) lds32[PADX(j0 + u * WG_DEC)] = decrypt_coeff<KQ>(C, v[u]);
    }
  } else {
    for (uint32_t j = tid; j < n; j += WG_DEC) {
      uint64_t v[KQ ? KQ : HC_MAXQ];
      for (uint32_t i = 0; i < k; ++i) v[i] = x[((size_t)bl * k + i) * n + j];
      lds32[PADX(j)] = decrypt_coeff<KQ>(C, v);
    }
  }
  __syncthreads();
  ntt_forward16(lds32, T.ttw, T.ttw_sh, ModP{t}, n, C.logn, tid, WG_DEC, T.ntt_r);
  for (uint32_t s = tid; s < n; s += WG_DEC) {
    const int64_t item = b * n + s;
    if (item >= m) continue;
    const uint32_t z = lds32[PADX(bit_reverse(s, C.logn))];
    out[item] = z >= (t + 1) / 2 ? (int32_t)z - (int32_t)t : (int32_t)z;
  }
}

// Decryption and slot decoding of one block in one workgroup (App. A Alg.
// "Decryption", then the slot decode): for each q_sigma in turn,
// x_sigma = [c0 + c1 s]_{q_sigma} goes through LDS as in k_dec_mul's double-
// precision form (forward transform of c1, product by the key's transform,
// inverse transform, plus c0) and stays in registers, PER coefficients per
// lane; then each coefficient's scale as in k_dec_decode (decrypt_coeff), the
// forward transform mod t and the centred slots.  The same values as the two
// kernels, without x in memory.  Transform passes of at most RX stages (every
// lane busy at n = NT PER with PER = 8 and RX = 3).
template <int KQ, int NT, int PER, int RX>
__global__ void __launch_bounds__(NT)
k_dec_fused(DevTabs T, const uint64_t* __restrict__ scores, int64_t blk_lo, const uint64_t* __restrict__ S,
            int64_t m, int32_t* __restrict__ out) {
  extern __shared__ uint64_t lds64[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, tid = threadIdx.x;              // n == NT PER (checked at launch)
  const int64_t bl = blockIdx.x, b = blk_lo + bl;
  double* f = reinterpret_cast<double*>(lds64);
  uint32_t* l32 = reinterpret_cast<uint32_t*>(f + padded_len(n));
  uint64_t x[PER][KQ];
#pragma unroll
  for (int sg = 0; sg < KQ; ++sg) {
    const uint64_t q = C.q[sg];
    const ModQF mf{T.qf[sg], T.qf[HC_MAXQ + sg]};
    const ModQB mb{mf.q, mf.qinv};
    const uint64_t* c0 = scores + (((size_t)b * 2 + 0) * KQ + sg) * n;
    const uint64_t* c1 = scores + (((size_t)b * 2 + 1) * KQ + sg) * n;
    if (sg) __syncthreads();                                 // the previous prime's reads of f are done
    load_padded(f, c1, n, tid, NT, [](uint64_t v) { return u64_to_f(v); });
    __syncthreads();
    ntt_forward_b<RX>(f, T.qtw_f + (size_t)sg * n, mb, n, C.logn, tid, NT, T.ntt_r);
    for_each_loaded(S + (size_t)sg * n, n, tid, NT,
                    [&](uint32_t j, uint64_t sv) { f[PADX(j)] = mf.mul(f[PADX(j)], u64_to_f(sv), 0.0); });
    __syncthreads();
    ntt_inverse_b<RX>(f, T.qitw_f + (size_t)sg * n, T.qf[2 * HC_MAXQ + sg], mb, n, C.logn, tid, NT, T.ntt_r);
    uint64_t cv[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) cv[e] = c0[tid + e * NT];
#pragma unroll
    for (int e = 0; e < PER; ++e) x[e][sg] = add_q(f_to_u64(f[PADX(tid + e * NT)]), cv[e], q);
  }
#pragma unroll
  for (int e = 0; e < PER; ++e) l32[PADX(tid + e * NT)] = decrypt_coeff<KQ>(C, x[e]);
  __syncthreads();
  ntt_forward16<RX>(l32, T.ttw, T.ttw_sh, ModP{C.t}, n, C.logn, tid, NT, T.ntt_r);
  const uint32_t t = C.t;
  for (uint32_t sl = tid; sl < n; sl += NT) {
    const int64_t item = b * n + sl;
    if (item >= m) continue;
    const uint32_t z = l32[PADX(bit_reverse(sl, C.logn))];
    out[item] = z >= (t + 1) / 2 ? (int32_t)z - (int32_t)t : (int32_t)z;
  }
}

// ---------------------------------------------------------------- launchers

namespace hers {

static size_t lds_bytes(uint32_t n, int words64) { return (size_t)padded_len(n) * 8 * words64; }
static size_t lds_bytes32(uint32_t n) { return (size_t)padded_len(n) * 4; }

hipError_t launch_keygen(const DevTabs& T, uint32_t n, uint32_t k, uint32_t L, uint64_t seed, uint8_t* sk,
                         uint64_t* pk, uint64_t* rlk, hipStream_t s) {
  hipLaunchKernelGGL(k_keygen, dim3(1 + L, k), dim3(WG), lds_bytes(n, 2), s, T, seed, sk, pk, rlk);
  return hipGetLastError();
}

hipError_t launch_load_keys(const DevTabs& T, uint32_t n, uint32_t k, uint32_t L, const uint64_t* pk,
                            const uint64_t* rlk, hipStream_t s) {
  hipLaunchKernelGGL(k_load_keys, dim3(1 + L, 2 * k), dim3(WG), lds_bytes(n, 1), s, T, pk, rlk);
  return hipGetLastError();
}

hipError_t launch_encode(const DevTabs& T, uint32_t n, const int32_t* feats, int64_t ld, int64_t item_lo,
                         int64_t item_hi, int64_t fbase, int32_t d, int64_t block0, int64_t nblocks, uint32_t* pt,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_encode, dim3((uint32_t)(nblocks * d)), dim3(WG), lds_bytes32(n), s, T, feats, ld, item_lo,
                     item_hi, fbase, d, block0, pt);
  return hipGetLastError();
}

hipError_t launch_ct_add(const DevTabs& T, uint32_t n, uint32_t k, uint64_t* dst, const uint64_t* fresh, uint32_t nct,
                         int32_t d, int64_t block0, int64_t first_empty_block, hipStream_t s) {
  const uint64_t words = (uint64_t)nct * 2 * k * n;
  hipLaunchKernelGGL(k_ct_add, dim3((uint32_t)((words + WG - 1) / WG)), dim3(WG), 0, s, T, dst, fresh, nct, d, block0,
                     first_empty_block);
  return hipGetLastError();
}

hipError_t launch_encrypt(const DevTabs& T, uint32_t n, uint32_t k, uint32_t nct, const uint32_t* pt,
                          const int32_t* query, int32_t d, int64_t block0, uint64_t seed, uint32_t domain,
                          uint64_t* canon, hipStream_t s, int32_t qdim0) {
  const size_t lds = lds_bytes(n, 2);
  QueryVals qv;
  std::memset(&qv, 0, sizeof(qv));
  // a probe goes in launches of at most HERS_QCHUNK dimensions, its values in the arguments
  for (uint32_t c0 = 0; c0 < nct; c0 += (query ? HERS_QCHUNK : nct)) {
    const uint32_t cn = query ? (nct - c0 < HERS_QCHUNK ? nct - c0 : HERS_QCHUNK) : nct;
    if (query) std::memcpy(qv.v, query + c0, cn * sizeof(int32_t));
    uint64_t* out = canon + (size_t)c0 * 2 * k * n;
    if (T.qf_ok)
      hipLaunchKernelGGL(k_encrypt<true>, dim3(cn, k), dim3(WG_ENC), lds, s, T, query ? nullptr : pt, qv,
                         qdim0 + (int32_t)c0, d, block0, seed, domain, out);
    else
      hipLaunchKernelGGL(k_encrypt<false>, dim3(cn, k), dim3(WG_ENC), lds, s, T, query ? nullptr : pt, qv,
                         qdim0 + (int32_t)c0, d, block0, seed, domain, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_lift(const DevTabs& T, uint32_t n, const uint64_t* canon, uint32_t nct, int32_t d,
                       int64_t block0, uint32_t* out, hipStream_t s) {
  const dim3 grid((uint32_t)(((uint64_t)nct * n + WG - 1) / WG));
  switch (T.nq) {   // the prime counts of the parameter sets in use get unrolled bodies
    case 1: hipLaunchKernelGGL(k_lift<1>, grid, dim3(WG), 0, s, T, canon, nct, d, block0, out); break;
    case 2: hipLaunchKernelGGL(k_lift<2>, grid, dim3(WG), 0, s, T, canon, nct, d, block0, out); break;
    case 3: hipLaunchKernelGGL(k_lift<3>, grid, dim3(WG), 0, s, T, canon, nct, d, block0, out); break;
    case 5: hipLaunchKernelGGL(k_lift<5>, grid, dim3(WG), 0, s, T, canon, nct, d, block0, out); break;
    default: hipLaunchKernelGGL(k_lift<0>, grid, dim3(WG), 0, s, T, canon, nct, d, block0, out); break;
  }
  return hipGetLastError();
}

hipError_t launch_unlift(const DevTabs& T, uint32_t n, const uint32_t* coef, uint32_t nct, int32_t d,
                         uint64_t* canon, hipStream_t s) {
  const dim3 grid((uint32_t)(((uint64_t)nct * n + WG - 1) / WG));
  switch (T.nq) {
    case 3: hipLaunchKernelGGL(k_unlift<3>, grid, dim3(WG), 0, s, T, coef, nct, d, canon); break;
    case 5: hipLaunchKernelGGL(k_unlift<5>, grid, dim3(WG), 0, s, T, coef, nct, d, canon); break;
    default: hipLaunchKernelGGL(k_unlift<0>, grid, dim3(WG), 0, s, T, coef, nct, d, canon); break;
  }
  return hipGetLastError();
}

hipError_t launch_check_features(const int32_t* v, int64_t ld, int32_t rows, int64_t cols, int32_t bound,
                                 uint32_t* flag, uint32_t num_cus, hipStream_t s) {
  if (rows < 1 || cols < 1) return hipSuccess;
  uint64_t gx = ((uint64_t)cols + WG - 1) / WG;
  const uint64_t cap = (uint64_t)num_cus * 8 / (uint64_t)rows + 1;
  if (gx > cap) gx = cap;
  hipLaunchKernelGGL(k_check_features, dim3((uint32_t)gx, (uint32_t)rows), dim3(WG), 0, s, v, ld, cols, bound, flag);
  return hipGetLastError();
}

hipError_t launch_check_canon(const DevTabs& T, const uint64_t* canon, uint64_t words, uint32_t* flag,
                              uint32_t num_cus, hipStream_t s) {
  if (!words) return hipSuccess;
  uint64_t g = (words + WG - 1) / WG;
  if (g > (uint64_t)num_cus * 8) g = (uint64_t)num_cus * 8;
  hipLaunchKernelGGL(k_check_canon, dim3((uint32_t)g), dim3(WG), 0, s, T, canon, words, flag);
  return hipGetLastError();
}

hipError_t launch_ntt_p(const DevTabs& T, uint32_t n, uint32_t* polys, uint64_t npolys, uint32_t inner,
                        int inverse, hipStream_t s, uint32_t nsets, uint64_t set_stride) {
  hipLaunchKernelGGL(k_ntt_p, dim3((uint32_t)npolys, nsets), dim3(WG), lds_bytes32(n), s, T, polys, inner, inverse,
                     set_stride);
  return hipGetLastError();
}

hipError_t launch_mac(const DevTabs& T, uint32_t n, uint32_t K, const uint32_t* gallery, const uint32_t* probe,
                      int32_t d, int64_t blk_lo, int64_t blk_hi, uint32_t* acc, hipStream_t s, int variant,
                      uint32_t target_wgs, int32_t dim0, int32_t dcount) {
  if (dcount <= 0) dcount = d;
  if (dim0 < 0 || dim0 + dcount > d) return hipErrorInvalidValue;
  const int64_t nb = blk_hi - blk_lo;
  const uint32_t lanes = n / 4 < WG ? n / 4 : WG;          // 4 slots per lane
  const uint64_t tiles = n / 4 / lanes;
  static const int nb_of[12] = {1, 2, 1, 2, 1, 2, 1, 2, 4, 4, 2, 1};
  const int NB = variant >= 0 && variant < 12 ? nb_of[variant] : 1;
  // about target_wgs workgroups: groups of about bpg blocks, each taking its
  // steps of NB blocks interleaved with the other groups'
  uint64_t bpg = (uint64_t)nb * tiles * K / (target_wgs ? target_wgs : 2048);
  if (bpg < (uint64_t)NB) bpg = NB;
  bpg = (bpg + NB - 1) / NB * NB;
  const uint64_t groups = ((uint64_t)nb + bpg - 1) / bpg;
  dim3 grid((uint32_t)tiles, K, (uint32_t)groups);
#define MAC_CASE(V, NB_, U_, NT_)                                                                    \
  case V:                                                                                            \
    hipLaunchKernelGGL((k_mac<NB_, U_, NT_>), grid, dim3(lanes), 0, s, T, gallery, probe, d, dim0, dcount, \
                       blk_lo, blk_hi, acc);                                                         \
    break;
  switch (variant) {
    MAC_CASE(0, 1, 2, false)
    MAC_CASE(1, 2, 2, false)
    MAC_CASE(2, 1, 4, false)
    MAC_CASE(3, 2, 4, false)
    MAC_CASE(4, 1, 2, true)
    MAC_CASE(5, 2, 2, true)
    MAC_CASE(6, 1, 4, true)
    MAC_CASE(7, 2, 4, true)
    MAC_CASE(8, 4, 1, true)
    MAC_CASE(9, 4, 2, true)
    MAC_CASE(10, 2, 1, true)
    MAC_CASE(11, 1, 1, true)
    default: return hipErrorInvalidValue;
  }
#undef MAC_CASE
  return hipGetLastError();
}

hipError_t launch_mac_intt(const DevTabs& T, uint32_t n, uint32_t K, const uint32_t* gallery, const uint32_t* probe,
                           int32_t d, int64_t blk_lo, int64_t blk_hi, uint32_t* acc, hipStream_t s,
                           uint32_t target_wgs, int32_t dim0, int32_t dcount) {
  if (dcount <= 0) dcount = d;
  if (dim0 < 0 || dim0 + dcount > d) return hipErrorInvalidValue;
  const uint64_t items = (uint64_t)(blk_hi - blk_lo) * K;
  if (!items) return hipSuccess;
  // a grid that is a multiple of lcm(K, 8), so every workgroup keeps one prime
  uint64_t l = K;
  while (l % 8) l += K;
  uint64_t grid = target_wgs ? target_wgs : 512;
  grid = grid / l * l;
  if (grid < l) grid = l;
  if (grid > items) grid = items;
  const size_t lds = (size_t)3 * padded_len(n) * 4;
  const uint32_t lanes = n / 4;                            // one group of 4 slots per lane
  if (lanes > 1024) return hipErrorInvalidValue;           // n <= 4096
  if (lanes > 512)
    hipLaunchKernelGGL((k_mac_intt<1, 1024>), dim3((uint32_t)grid), dim3(lanes), lds, s, T, gallery, probe, d, dim0,
                       dcount, blk_lo, blk_hi, acc);
  else if (lanes > 256)
    hipLaunchKernelGGL((k_mac_intt<1, 512>), dim3((uint32_t)grid), dim3(lanes), lds, s, T, gallery, probe, d, dim0,
                       dcount, blk_lo, blk_hi, acc);
  else
    hipLaunchKernelGGL((k_mac_intt<1, 256>), dim3((uint32_t)grid), dim3(lanes), lds, s, T, gallery, probe, d, dim0,
                       dcount, blk_lo, blk_hi, acc);
  return hipGetLastError();
}

hipError_t launch_mac_multi(const DevTabs& T, const MacBatchArgs& A, uint32_t grid, hipStream_t s, int variant) {
  if (variant == MB_MFMA) {
    // the probes' digits stay in registers: d <= MF_DMAX (else the first schedule)
    bool fits = true;
    for (int g = 0; g < A.ngroups; ++g) fits &= A.g[g].d >= 1 && A.g[g].d <= MF_DMAX;
    if (fits) {
      hipLaunchKernelGGL(k_mac_mfma, dim3(grid), dim3(64 * MF_SLOTS), 0, s, T, A);
      return hipGetLastError();
    }
    variant = 0;
  }
  switch (variant) {
    case 1: hipLaunchKernelGGL((k_mac_multi<2, 4, 2>), dim3(grid), dim3(64 * MB_PROBES / 2), 0, s, T, A); break;
    case 2: hipLaunchKernelGGL((k_mac_multi<2, 8, 2>), dim3(grid), dim3(64 * MB_PROBES / 2), 0, s, T, A); break;
    case 3: hipLaunchKernelGGL((k_mac_multi<4, 4, 1>), dim3(grid), dim3(64 * MB_PROBES / 4), 0, s, T, A); break;
    default: hipLaunchKernelGGL((k_mac_multi<1, MB_DC, MB_BLOCKS>), dim3(grid), dim3(64 * MB_PROBES), 0, s, T, A);
  }
  return hipGetLastError();
}

hipError_t launch_rescale(const DevTabs& T, uint32_t n, const uint32_t* X, int64_t nblk, int64_t blk_lo,
                          const ScorePtrs& SP, uint32_t nreq, uint64_t* digits, uint64_t acc_stride,
                          uint64_t dig_stride, hipStream_t s, uint32_t k, uint32_t K, uint32_t W) {
  uint64_t total = (uint64_t)nblk * 3 * n;
  dim3 grid((uint32_t)((total + WG - 1) / WG), nreq);
  // the parameter sets in use get fully unrolled bodies; others use runtime bounds
  if (k == 3 && K == 8 && W == 3)
    hipLaunchKernelGGL((k_rescale<3, 8, 3>), grid, dim3(WG), 0, s, T, X, nblk, blk_lo, SP, digits, acc_stride,
                       dig_stride);
  else if (k == 5 && K == 16 && W == 4)
    hipLaunchKernelGGL((k_rescale<5, 16, 4>), grid, dim3(WG), 0, s, T, X, nblk, blk_lo, SP, digits, acc_stride,
                       dig_stride);
  else if (k == 2 && K == 8 && W == 3)
    hipLaunchKernelGGL((k_rescale<2, 8, 3>), grid, dim3(WG), 0, s, T, X, nblk, blk_lo, SP, digits, acc_stride,
                       dig_stride);
  else
    hipLaunchKernelGGL((k_rescale<0, 0, 0>), grid, dim3(WG), 0, s, T, X, nblk, blk_lo, SP, digits, acc_stride,
                       dig_stride);
  return hipGetLastError();
}

hipError_t launch_relin(const DevTabs& T, uint32_t n, uint32_t k, uint32_t L, uint64_t* digits, int64_t nblk,
                        int64_t blk_lo, const ScorePtrs& SP, uint32_t nreq, uint64_t dig_stride, hipStream_t s,
                        const uint64_t* key, const uint64_t* key_sh, uint32_t fuse_min_wgs) {
  if (!key) { key = T.rlk_ntt; key_sh = T.rlk_ntt_sh; }
  if ((uint64_t)nblk * k * nreq >= (uint64_t)fuse_min_wgs) {
    // many workgroups: one per (block, residue, request) does the digit
    // transforms, key products and both inverse transforms (no transformed
    // digits in memory)
    const dim3 grid((uint32_t)nblk, k, nreq);
    const size_t lds = lds_bytes(n, 1);
    if (T.rl_per == 8 && T.qf_ok && n / 8 <= 1024) {   // n >= 128: at least 16 lanes (the integer form
      hipLaunchKernelGGL((k_relin_fused<true, 8>), grid, dim3(n / 8), lds, s, T, digits, blk_lo, SP, dig_stride,
                         key, key_sh);                 // spills with 8 per lane: it keeps 16)
    } else {                                           // n >= 256: at least 16 lanes
      if (T.qf_ok)
        hipLaunchKernelGGL((k_relin_fused<true, 16>), grid, dim3(n / 16), lds, s, T, digits, blk_lo, SP, dig_stride,
                           key, key_sh);
      else
        hipLaunchKernelGGL((k_relin_fused<false, 16>), grid, dim3(n / 16), lds, s, T, digits, blk_lo, SP, dig_stride,
                           key, key_sh);
    }
    return hipGetLastError();
  }
  // few workgroups: the digit transforms (L per block, each for all k residues), then key products
  // and inverse transforms (2 k per block), as separate launches with more
  // workgroups each
  // (the double-precision key products take both components of a block in one workgroup)
  const dim3 g1((uint32_t)(nblk * L), nreq), g2((uint32_t)((T.qf_ok ? 1 : 2) * nblk), k, nreq);
  if (T.qf_ok)
    hipLaunchKernelGGL(k_ntt_q<true>, g1, dim3(WG), lds_bytes(n, 1), s, T, digits, dig_stride);
  else
    hipLaunchKernelGGL(k_ntt_q<false>, g1, dim3(WG), lds_bytes(n, 1), s, T, digits, dig_stride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // (512 lanes in double precision: its two LDS buffers leave room for two
  // workgroups per CU at n = 4096, one at 8192)
  if (T.qf_ok)
    hipLaunchKernelGGL((k_relin_acc<true, 512>), g2, dim3(512), 2 * lds_bytes(n, 1), s, T, digits, blk_lo, SP,
                       dig_stride, key, key_sh);
  else
    hipLaunchKernelGGL((k_relin_acc<false, WG>), g2, dim3(WG), lds_bytes(n, 1), s, T, digits, blk_lo, SP, dig_stride,
                       key, key_sh);
  return hipGetLastError();
}

hipError_t launch_encrypt_sk(const DevTabs& T, uint32_t n, uint32_t k, const int32_t* query, int32_t d, uint64_t seed,
                             const uint64_t* S, const uint64_t* Ssh, uint64_t* canon, hipStream_t s) {
  QueryVals qv;
  std::memset(&qv, 0, sizeof(qv));
  for (int32_t c0 = 0; c0 < d; c0 += HERS_QCHUNK) {
    const int32_t cn = d - c0 < HERS_QCHUNK ? d - c0 : HERS_QCHUNK;
    std::memcpy(qv.v, query + c0, cn * sizeof(int32_t));
    hipLaunchKernelGGL(k_encrypt_sk, dim3((uint32_t)cn, k), dim3(WG_ENC), lds_bytes(n, 1), s, T, qv, c0, seed, S, Ssh,
                       canon + (size_t)c0 * 2 * k * n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_sk_ntt(const DevTabs& T, uint32_t n, uint32_t k, const uint8_t* sk, uint64_t* S, uint64_t* Ssh,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_sk_ntt, dim3(k), dim3(WG), lds_bytes(n, 1), s, T, sk, S, Ssh);
  return hipGetLastError();
}

hipError_t launch_dec_mul(const DevTabs& T, uint32_t n, uint32_t k, const uint64_t* scores, int64_t nblk,
                          int64_t blk_lo, const uint64_t* S, const uint64_t* Ssh, uint64_t* x, hipStream_t s) {
  const dim3 grid((uint32_t)nblk, k);
  if (T.qf_ok && n >= 8192)
    hipLaunchKernelGGL((k_dec_mul<true, 512>), grid, dim3(512), lds_bytes(n, 1), s, T, scores, blk_lo, S, Ssh, x);
  else if (T.qf_ok)
    hipLaunchKernelGGL((k_dec_mul<true, WG>), grid, dim3(WG), lds_bytes(n, 1), s, T, scores, blk_lo, S, Ssh, x);
  else
    hipLaunchKernelGGL((k_dec_mul<false, WG>), grid, dim3(WG), lds_bytes(n, 1), s, T, scores, blk_lo, S, Ssh, x);
  return hipGetLastError();
}

bool dec_fused_fits(const DevTabs& T, uint32_t n) {
  // (five primes at n = 8192 would hold 80 registers of x per lane in 1024-lane
  // workgroups and spill: they keep the two kernels)
  return T.qf_ok && T.nq == 3 && n == 4096;
}

hipError_t launch_dec_fused(const DevTabs& T, uint32_t n, const uint64_t* scores, int64_t nblk, int64_t blk_lo,
                            const uint64_t* S, int64_t m, int32_t* out, hipStream_t s) {
  if (!dec_fused_fits(T, n)) return hipErrorInvalidValue;
  const dim3 grid((uint32_t)nblk);
  const size_t lds = lds_bytes(n, 1) + lds_bytes32(n);
  hipLaunchKernelGGL((k_dec_fused<3, 512, 8, 3>), grid, dim3(512), lds, s, T, scores, blk_lo, S, m, out);
  return hipGetLastError();
}

hipError_t launch_dec_decode(const DevTabs& T, uint32_t n, const uint64_t* x, int64_t nblk, int64_t blk_lo,
                             int64_t m, int32_t* out, hipStream_t s) {
  const dim3 grid((uint32_t)nblk);
  const size_t lds = lds_bytes32(n);
  switch (T.nq) {
    case 1: hipLaunchKernelGGL(k_dec_decode<1>, grid, dim3(WG_DEC), lds, s, T, x, blk_lo, m, out); break;
    case 2: hipLaunchKernelGGL(k_dec_decode<2>, grid, dim3(WG_DEC), lds, s, T, x, blk_lo, m, out); break;
    case 3: hipLaunchKernelGGL(k_dec_decode<3>, grid, dim3(WG_DEC), lds, s, T, x, blk_lo, m, out); break;
    case 5: hipLaunchKernelGGL(k_dec_decode<5>, grid, dim3(WG_DEC), lds, s, T, x, blk_lo, m, out); break;
    default: hipLaunchKernelGGL(k_dec_decode<0>, grid, dim3(WG_DEC), lds, s, T, x, blk_lo, m, out); break;
  }
  return hipGetLastError();
}

}  // namespace hers
