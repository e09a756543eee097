// rerank.hip -- second stage of the two-stage search (Sec. 4, "Two Stage
// Search"): packed 1:1 re-ranking of selected gallery items.
//
// S = n / W items share a ciphertext, one segment of W slots each; the probe
// is repeated in every segment.  Slot positions follow the orbit of 5 in
// (Z/2nZ)^*: position p of row r is slot j with 2j + 1 = (-1)^r 5^p mod 2n,
// and segment c of row r covers positions [W c, W c + W).  The automorphism
// x -> x^(5^s) then moves every segment's values s positions towards its
// start, so after one ciphertext product rotate-and-add with s = 1, 2, ...,
// W/2 leaves each item's inner product with the probe at its segment's first
// position.  A rotation is the automorphism of both components followed by
// key switching of the second from s(x^g) to s with a rotation key (RNS
// gadget digits, as the relinearization).
#include "kernels.h"

#include "ntt.h"

#define WG 256

// Slot of position p in row r: (e - 1) / 2 for e = (-1)^r 5^p mod 2n.
__device__ __forceinline__ uint32_t slot_of_position(uint32_t n, uint32_t r, uint32_t p) {
  const uint32_t mask = 2 * n - 1;                       // 2n is a power of two
  uint32_t e = 1, b = 5;
  for (uint32_t x = p; x; x >>= 1) {
    if (x & 1) e = (e * b) & mask;
    b = (b * b) & mask;
  }
  if (r) e = (2 * n - e) & mask;
  return (e - 1) >> 1;
}

extern "C" __global__ void __launch_bounds__(WG)
k_encode_packed(DevTabs T, const int32_t* __restrict__ feats, int64_t ld, int64_t count, int32_t D, int32_t W,
                int replicate, uint32_t* __restrict__ pt) {
  // Plaintext of ciphertext blockIdx.x: segment seg holds item
  // blockIdx.x * (n / W) + seg (features [D][ld], column = item), or with
  // `replicate` column 0 in every segment; positions past D and items past
  // `count` are 0.  Slots to coefficients as in k_encode (inverse NTT mod t).
  extern __shared__ uint32_t lds32[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, tid = threadIdx.x, t = C.t, half = n / 2;
  const uint32_t c = blockIdx.x;
  for (uint32_t pos = tid; pos < n; pos += WG) {
    const uint32_t r = pos / half, p = pos % half;
    const uint32_t seg = r * (half / W) + p / W, f = p % W;
    const int64_t x = replicate ? 0 : (int64_t)c * (n / W) + seg;
    int64_t v = 0;
    if ((int32_t)f < D && x < count) v = feats[(int64_t)f * ld + x];
    int64_t z = v % (int64_t)t;
    if (z < 0) z += t;
    lds32[PADX(bit_reverse(slot_of_position(n, r, p), C.logn))] = (uint32_t)z;
  }
  __syncthreads();
  ntt_inverse16(lds32, T.titw, T.titw_sh, C.t_ninv, C.t_ninv_sh, ModP{t}, n, C.logn, tid, WG, T.ntt_r);
  for (uint32_t j = tid; j < n; j += WG) pt[(size_t)c * n + j] = lds32[PADX(j)];
}

extern "C" __global__ void __launch_bounds__(WG)
k_rotkey(DevTabs T, uint64_t seed, uint64_t* __restrict__ rk, uint64_t* __restrict__ rk_ntt,
         uint64_t* __restrict__ rk_ntt_sh) {
  // Rotation key of step `st` (rotation by 2^st, g = 5^(2^st) mod 2n), gadget
  // digit gi, residue rho = blockIdx.y, blockIdx.x = st L + gi:
  // ([-(a s + e) + g_val s(x^g)]_q, a) -- Alg. "Key Generation"'s evaluation
  // key with s(x^g) in place of s^2.  Philox key (seed, KEYGEN), objects s
  // (0,0,0), a (5, gi, st), e (6, gi, st).  Canonical [steps][L][2][k][n]
  // to rk, NTT form and Shoup companions to rk_ntt, rk_ntt_sh.
  extern __shared__ uint64_t lds64[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = C.k, L = C.L, tid = threadIdx.x;
  const uint32_t st = blockIdx.x / L, gi = blockIdx.x % L, rho = blockIdx.y;
  const uint64_t q = C.q[rho];
  const ModQ mq{q};
  uint64_t* S = lds64;
  uint64_t* A = lds64 + padded_len(n);
  const uint64_t* tw = T.qtw + (size_t)rho * n;
  const uint64_t* twsh = T.qtw_sh + (size_t)rho * n;
  const size_t base = (size_t)blockIdx.x * 2 * k * n;
  for (uint32_t j = tid; j < n; j += WG)
    S[PADX(j)] = (philox_word(seed, HERS_DOMAIN_KEYGEN, 0, 0, 0, j >> 6) >> (j & 63)) & 1;
  for (uint32_t h = tid; h < n / 2; h += WG) {
    Philox4 b = philox4x64_10(((uint64_t)rho * n) / 2 + h, 5, gi, st, seed, HERS_DOMAIN_KEYGEN);
    for (int s = 0; s < 2; ++s) {
      const uint64_t lo = b.v[2 * s], hi = b.v[2 * s + 1];
      A[PADX(2 * h + s)] = add_q(shoup_q(red_q(hi, q, C.q_mu64[rho]), C.q_r64[rho], C.q_r64_sh[rho], q),
                                 red_q(lo, q, C.q_mu64[rho]), q);
    }
  }
  __syncthreads();
  for (uint32_t j = tid; j < n; j += WG) rk[base + ((size_t)k + rho) * n + j] = A[PADX(j)];
  ntt_forward16(S, tw, twsh, mq, n, C.logn, tid, WG, T.ntt_r);
  ntt_forward16(A, tw, twsh, mq, n, C.logn, tid, WG, T.ntt_r);
  for (uint32_t j = tid; j < n; j += WG) {
    const uint64_t a = A[PADX(j)];
    rk_ntt[base + ((size_t)k + rho) * n + j] = a;
    rk_ntt_sh[base + ((size_t)k + rho) * n + j] = shoup_companion_q(a, q, C.q_m128h[rho], C.q_m128l[rho]);
    A[PADX(j)] = sub_q(0, mul_q(a, S[PADX(j)], q, C.q_bar[rho], C.q_beta[rho]), q);     // -a s
  }
  __syncthreads();
  ntt_inverse16(A, T.qitw + (size_t)rho * n, T.qitw_sh + (size_t)rho * n, C.q_ninv[rho], C.q_ninv_sh[rho], mq, n,
                C.logn, tid, WG, T.ntt_r);
  // s(x^g) in coefficient form: x^i -> +-x^(i g mod n)
  const uint32_t mask = 2 * n - 1;
  uint32_t g = 5;
  for (uint32_t i = 0; i < st; ++i) g = (g * g) & mask;
  for (uint32_t i = tid; i < n; i += WG) {
    const uint64_t s = (philox_word(seed, HERS_DOMAIN_KEYGEN, 0, 0, 0, i >> 6) >> (i & 63)) & 1;
    const uint32_t e = (i * g) & mask;
    S[PADX(e & (n - 1))] = e < n ? s : (s ? q - 1 : 0);
  }
  __syncthreads();
  const uint64_t gv = C.g_val[gi][rho], gvsh = C.g_val_sh[gi][rho];
  for (uint32_t g4 = tid; g4 < n / 4; g4 += WG) {
    Philox4 b = philox4x64_10(g4, 6, gi, st, seed, HERS_DOMAIN_KEYGEN);
    for (int s = 0; s < 4; ++s) {
      const uint32_t j = 4 * g4 + s;
      const int e = cbd20(b.v[s]);
      const uint64_t em = e >= 0 ? (uint64_t)e : q - (uint64_t)(-e);
      const uint64_t v = add_q(sub_q(A[PADX(j)], em, q), shoup_q(S[PADX(j)], gv, gvsh, q), q);
      A[PADX(j)] = v;
      rk[base + (size_t)rho * n + j] = v;
    }
  }
  __syncthreads();
  ntt_forward16(A, tw, twsh, mq, n, C.logn, tid, WG, T.ntt_r);
  for (uint32_t j = tid; j < n; j += WG) {
    rk_ntt[base + (size_t)rho * n + j] = A[PADX(j)];
    rk_ntt_sh[base + (size_t)rho * n + j] = shoup_companion_q(A[PADX(j)], q, C.q_m128h[rho], C.q_m128l[rho]);
  }
}

extern "C" __global__ void __launch_bounds__(WG)
k_rot_digits(DevTabs T, const uint64_t* __restrict__ in, uint64_t* __restrict__ out, uint64_t* __restrict__ digits,
             uint32_t nct, uint32_t ginv) {
  // First half of rotate-and-add for ciphertexts [nct][2][k][n]: out =
  // (c0 + tau(c0), c1) and the gadget digits of tau(c1) ([nct][L][k][n],
  // each the integer it is, in the slot of residue 0), tau: x^i -> +-x^(i g mod 2n).  One workgroup
  // per (ciphertext blockIdx.x, residue r = blockIdx.y): residue r of c0 and
  // c1 is read once, coalesced, into LDS; the digits of q_r need only that
  // residue of tau(c1).  For destination coefficient dst, with ginv = g^-1
  // mod 2n, i = dst ginv mod 2n is the source if i < n (sign +), else i - n
  // is, with sign - (x^(i - n) maps to x^(dst + n) = -x^dst).
  extern __shared__ uint64_t lds64[];
  const HersConsts& C = *T.C;
  const uint32_t n = C.n, k = C.k, L = C.L, tid = threadIdx.x;
  const uint64_t c = blockIdx.x;
  const uint32_t r = blockIdx.y;
  const uint64_t q = C.q[r];
  const uint64_t* c0 = in + (c * 2 * k + r) * n;
  const uint64_t* c1 = in + (c * 2 * k + k + r) * n;
  uint64_t* o0 = out + (c * 2 * k + r) * n;
  uint64_t* o1 = out + (c * 2 * k + k + r) * n;
  uint64_t* s0 = lds64;
  uint64_t* s1 = lds64 + n;
  for (uint32_t j = tid; j < n; j += WG) {
    const uint64_t v1 = c1[j];
    s0[j] = c0[j];
    s1[j] = v1;
    o1[j] = v1;
  }
  __syncthreads();
  for (uint32_t dst = tid; dst < n; dst += WG) {
    const uint32_t e = (dst * ginv) & (2 * n - 1);
    const uint32_t i = e & (n - 1);
    uint64_t v0 = s0[i], v1 = s1[i];
    if (e >= n) { v0 = v0 ? q - v0 : 0; v1 = v1 ? q - v1 : 0; }
    o0[dst] = add_q(s0[dst], v0, q);
    const uint64_t y = shoup_q(v1, C.q_hatinv[r], C.q_hatinv_sh[r], q);
    for (uint32_t gi = 0; gi < L; ++gi) {
      if (C.g_rho[gi] != r) continue;
      // stored once, as an integer, in the slot of residue 0: the key switch reduces it per q_sigma
      digits[(c * L + gi) * k * n + dst] = C.w_bits ? (y >> C.g_shift[gi]) & ((1ULL << C.w_bits) - 1) : y;
    }
  }
}

extern "C" __global__ void __launch_bounds__(WG)
k_gather_cts(const uint32_t* __restrict__ items, uint64_t words, int64_t nct_total, const int64_t* __restrict__ ids,
             uint32_t* __restrict__ out) {
  // Ciphertext ids[blockIdx.y] of `items` (words u32 each) to out slot
  // blockIdx.y; an id outside [0, nct_total) gives zeros.
  const int64_t id = ids[blockIdx.y];
  const bool ok = id >= 0 && id < nct_total;
  uint32_t* o = out + (size_t)blockIdx.y * words;
  for (uint64_t w = (uint64_t)blockIdx.x * WG + threadIdx.x; w < words; w += (uint64_t)gridDim.x * WG)
    o[w] = ok ? items[(size_t)id * words + w] : 0u;
}

extern "C" __global__ void __launch_bounds__(WG)
k_rerank_pick(uint32_t n, const int32_t* __restrict__ slots, uint32_t nsel, int32_t W, int32_t* __restrict__ out) {
  // Client: the score of segment seg of ciphertext c is the first position
  // of the segment; slots [nsel][n] (decoded, slot order) -> out [nsel][n / W].
  const uint32_t S = n / (uint32_t)W, per_row = S / 2;
  const uint64_t idx = (uint64_t)blockIdx.x * WG + threadIdx.x;
  if (idx >= (uint64_t)nsel * S) return;
  const uint64_t c = idx / S;
  const uint32_t seg = (uint32_t)(idx % S);
  out[idx] = slots[c * n + slot_of_position(n, seg / per_row, (seg % per_row) * (uint32_t)W)];
}

namespace hers {

static size_t lds32_bytes(uint32_t n) { return (size_t)padded_len(n) * 4; }
static size_t lds64x2_bytes(uint32_t n) { return (size_t)padded_len(n) * 16; }

hipError_t launch_encode_packed(const DevTabs& T, uint32_t n, const int32_t* feats, int64_t ld, int64_t count,
                                int32_t D, int32_t W, int replicate, uint32_t nct, uint32_t* pt, hipStream_t s) {
  hipLaunchKernelGGL(k_encode_packed, dim3(nct), dim3(WG), lds32_bytes(n), s, T, feats, ld, count, D, W, replicate,
                     pt);
  return hipGetLastError();
}

hipError_t launch_rotkey(const DevTabs& T, uint32_t n, uint32_t k, uint32_t L, uint32_t nsteps, uint64_t seed,
                         uint64_t* rk, uint64_t* rk_ntt, uint64_t* rk_ntt_sh, hipStream_t s) {
  hipLaunchKernelGGL(k_rotkey, dim3(nsteps * L, k), dim3(WG), lds64x2_bytes(n), s, T, seed, rk, rk_ntt, rk_ntt_sh);
  return hipGetLastError();
}

hipError_t launch_rot_digits(const DevTabs& T, uint32_t n, uint32_t k, const uint64_t* ct_in, uint64_t* ct_out,
                             uint64_t* digits, uint32_t nct, uint32_t g, hipStream_t s) {
  // g^-1 mod 2n (g odd): the group has order n, so g^-1 = g^(n - 1)
  const uint32_t mask = 2 * n - 1;
  uint32_t ginv = 1, b = g;
  for (uint32_t x = n - 1; x; x >>= 1) {
    if (x & 1) ginv = (uint32_t)(((uint64_t)ginv * b) & mask);
    b = (uint32_t)(((uint64_t)b * b) & mask);
  }
  hipLaunchKernelGGL(k_rot_digits, dim3(nct, k), dim3(WG), (size_t)2 * n * 8, s, T, ct_in, ct_out, digits, nct,
                     ginv);
  return hipGetLastError();
}

hipError_t launch_gather_cts(const uint32_t* items, uint64_t words_per_ct, int64_t nct_total, const int64_t* ids,
                             uint32_t nsel, uint32_t* out, hipStream_t s) {
  uint64_t gx = (words_per_ct + WG - 1) / WG;
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(k_gather_cts, dim3((uint32_t)gx, nsel), dim3(WG), 0, s, items, words_per_ct, nct_total, ids, out);
  return hipGetLastError();
}

hipError_t launch_rerank_pick(uint32_t n, const int32_t* slot_scores, uint32_t nsel, int32_t W, int32_t* out,
                              hipStream_t s) {
  const uint64_t total = (uint64_t)nsel * (n / (uint32_t)W);
  hipLaunchKernelGGL(k_rerank_pick, dim3((uint32_t)((total + WG - 1) / WG)), dim3(WG), 0, s, n, slot_scores, nsel, W,
                     out);
  return hipGetLastError();
}

}  // namespace hers
