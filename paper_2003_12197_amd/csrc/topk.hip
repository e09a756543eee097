// topk.hip -- exact top-k of decrypted scores on the GPU.
//
// The client's last step (App. B, Alg. "HERS Search") ranks the gallery by
// decrypted score; the nearest neighbour is the argmax.  A key packs
// (score + 2^31) in its high word and the complement of the item index in its
// low word: keys are distinct, a larger key is a higher score or, for equal
// scores, a lower index, so the k largest keys are one well-defined answer.
//
// Selection through tile maxima.  Split the m scores into tiles of
// HERS_TOPK_TM and take each tile's largest key.  Let B be the k tiles with
// the largest maxima and tau the smallest of those k maxima.  A tile outside
// B has k tiles with larger maxima, so none of its keys is in the top k; and
// the k maxima of B are k keys >= tau, so every top-k key is >= tau.  Hence:
//   1. k_topk_tilemax   one maximum per tile (one streaming read of the scores);
//   2. top k of the tile maxima (generic passes);
//   3. k_topk_filter    each tile of B compacts its keys >= tau in LDS -- a
//                       handful unless scores tie massively -- sorts them and
//                       writes its best k;
//   4. top k of those k * k candidates, written as (index, score).
// With fewer than k tiles every tile is in B and tau = 0 (no filtering).
//
// Generic pass (k_topk_pass): each workgroup bitonic-sorts up to
// HERS_TOPK_TILE keys in LDS, descending, and keeps the first k; a pass with
// one workgroup sorts only the next power of two at or above its count.
#include "kernels.h"

#define TK_WG 256

__device__ __forceinline__ uint64_t score_key(int32_t s, uint64_t idx) {
  return ((uint64_t)((uint32_t)s ^ 0x80000000u) << 32) | (uint32_t)~(uint32_t)idx;
}
__device__ __forceinline__ uint32_t key_index(uint64_t key) { return ~(uint32_t)key; }
__device__ __forceinline__ int32_t key_score(uint64_t key) { return (int32_t)((uint32_t)(key >> 32) ^ 0x80000000u); }

// Sorts a[0, S) in LDS in descending order; S is a power of two.  Stage
// (size, stride) compares lo = 2t - (t mod stride) with lo + stride, in
// descending order where bit `size` of lo is clear.
__device__ void bitonic_desc(uint64_t* a, uint32_t S) {
  const uint32_t tid = threadIdx.x;
  for (uint32_t size = 2; size <= S; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t t = tid; t < S / 2; t += TK_WG) {
        const uint32_t lo = 2 * t - (t & (stride - 1)), hi = lo + stride;
        const bool desc = (lo & size) == 0;
        const uint64_t x = a[lo], y = a[hi];
        if ((x < y) == desc) { a[lo] = y; a[hi] = x; }
      }
      __syncthreads();
    }
  }
}

extern "C" __global__ void __launch_bounds__(TK_WG)
k_topk_pass(const int32_t* __restrict__ scores, const uint64_t* __restrict__ keys_in, uint64_t count, uint32_t k,
            uint64_t* __restrict__ keys_out, int64_t* __restrict__ idx_out, int32_t* __restrict__ val_out) {
  // keys come from scores (key of item i) or from keys_in; a workgroup takes
  // HERS_TOPK_TILE of them (zero keys past count) and writes its best k as keys
  // at keys_out[blockIdx.x * k ..], or decoded when idx_out is set (one-workgroup
  // final pass).
  __shared__ uint64_t tile[HERS_TOPK_TILE];
  const uint32_t tid = threadIdx.x;
  const uint64_t base = (uint64_t)blockIdx.x * HERS_TOPK_TILE;
  uint32_t S = HERS_TOPK_TILE;
  if (gridDim.x == 1) {
    S = 2;
    while (S < count) S <<= 1;
  }
  if (!scores && S % (4 * TK_WG) == 0 && base + S <= count) {
    // keys of a full tile: four per lane loaded before they are stored
    for (uint32_t j = tid; j < S; j += 4 * TK_WG) {
      uint64_t v[4];
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) v[u] = keys_in[base + j + u * TK_WG];
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) tile[j + u * TK_WG] = v[u];
    }
  } else {
    for (uint32_t j = tid; j < S; j += TK_WG) {
      const uint64_t i = base + j;
      uint64_t key = 0;
      if (i < count) key = scores ? score_key(scores[i], i) : keys_in[i];
      tile[j] = key;
    }
  }
  __syncthreads();
  bitonic_desc(tile, S);
  for (uint32_t j = tid; j < k; j += TK_WG) {
    const uint64_t key = tile[j];
    if (idx_out) {
      idx_out[j] = key_index(key);
      val_out[j] = key_score(key);
    } else {
      keys_out[(uint64_t)blockIdx.x * k + j] = key;
    }
  }
}

extern "C" __global__ void __launch_bounds__(TK_WG)
k_topk_tilemax(const int32_t* __restrict__ scores, uint64_t m, uint64_t* __restrict__ maxes) {
  __shared__ uint64_t red[TK_WG];
  const uint32_t tid = threadIdx.x;
  const uint64_t base = (uint64_t)blockIdx.x << HERS_TOPK_TM_LOG2;
  uint64_t best = 0;
#pragma unroll 16
  for (uint32_t j = tid; j < HERS_TOPK_TM; j += TK_WG) {
    const uint64_t i = base + j;
    if (i < m) {
      const uint64_t key = score_key(scores[i], i);
      best = key > best ? key : best;
    }
  }
  red[tid] = best;
  __syncthreads();
  for (uint32_t h = TK_WG / 2; h > 0; h >>= 1) {
    if (tid < h && red[tid + h] > red[tid]) red[tid] = red[tid + h];
    __syncthreads();
  }
  if (tid == 0) maxes[blockIdx.x] = red[0];
}

extern "C" __global__ void __launch_bounds__(TK_WG)
k_topk_filter(const int32_t* __restrict__ scores, uint64_t m, const uint64_t* __restrict__ best, uint32_t nbest,
              int use_tau, uint32_t k, uint64_t* __restrict__ cand) {
  // Workgroup w takes the tile holding the item of best[w] (a tile maximum).
  __shared__ uint64_t buf[HERS_TOPK_TM];
  __shared__ uint32_t cnt;
  const uint32_t tid = threadIdx.x;
  const uint64_t tile = (uint64_t)key_index(best[blockIdx.x]) >> HERS_TOPK_TM_LOG2;
  const uint64_t tau = use_tau ? best[nbest - 1] : 0;
  const uint64_t base = tile << HERS_TOPK_TM_LOG2;
  if (tid == 0) cnt = 0;
  __syncthreads();
  if (base + HERS_TOPK_TM <= m) {
    // full tile: four scores per lane loaded before they are compared
    for (uint32_t j = tid; j < HERS_TOPK_TM; j += 4 * TK_WG) {
      int32_t s[4];
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) s[u] = scores[base + j + u * TK_WG];
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) {
        const uint64_t key = score_key(s[u], base + j + u * TK_WG);
        if (key >= tau) buf[atomicAdd(&cnt, 1u)] = key;
      }
    }
  } else {
    for (uint32_t j = tid; j < HERS_TOPK_TM; j += TK_WG) {
      const uint64_t i = base + j;
      if (i < m) {
        const uint64_t key = score_key(scores[i], i);
        if (key >= tau) buf[atomicAdd(&cnt, 1u)] = key;
      }
    }
  }
  __syncthreads();
  const uint32_t c = cnt;
  if (c > k) {
    uint32_t S = 2;
    while (S < c) S <<= 1;
    for (uint32_t j = c + tid; j < S; j += TK_WG) buf[j] = 0;
    __syncthreads();
    bitonic_desc(buf, S);
  }
  for (uint32_t j = tid; j < k; j += TK_WG) cand[(uint64_t)blockIdx.x * k + j] = j < c ? buf[j] : 0;
}

// ---------------------------------------------------------------- large k (radix select)
// For k above the tile path's limit: the k-th largest key tau is found digit
// by digit from the top (digits of 11, 11, 11, 11, 11 and 9 bits): a pass
// histograms the current digit of the keys that agree with tau's digits
// found so far and picks the digit where the count from the top reaches the
// keys still missing.  Keys are distinct, so exactly k keys are >= tau; they
// are collected (any order) and each is written at its rank, the number of
// collected keys above it.
#define TK_RS_BINS 2048

struct RselState {
  uint64_t prefix;      // digits of tau found so far
  uint32_t need;        // keys still to place at or below the current prefix
  uint32_t count;       // collected keys
};

__device__ __forceinline__ bool rsel_match(uint64_t key, uint64_t prefix, uint32_t hi_shift) {
  return hi_shift >= 64 || (key >> hi_shift) == (prefix >> hi_shift);
}

extern "C" __global__ void __launch_bounds__(TK_WG)
k_rsel_hist(const int32_t* __restrict__ scores, uint64_t m, const RselState* __restrict__ st, uint32_t shift,
            uint32_t width, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[TK_RS_BINS];
  const uint32_t tid = threadIdx.x;
  for (uint32_t b = tid; b < TK_RS_BINS; b += TK_WG) h[b] = 0;
  __syncthreads();
  const uint64_t prefix = st->prefix;
  const uint32_t hi_shift = shift + width;
  const uint32_t lane = __lane_id();
  for (uint64_t i = (uint64_t)blockIdx.x * TK_WG + tid; i < m; i += (uint64_t)gridDim.x * TK_WG) {
    const uint64_t key = score_key(scores[i], i);
    const uint32_t bin =
        rsel_match(key, prefix, hi_shift) ? (uint32_t)(key >> shift) & ((1u << width) - 1) : 0xffffffffu;
    // Scores span few high digits, so most lanes of a wave share a bin: the
    // lanes in the first active lane's bin add their count with one atomic,
    // the others one each (same-address LDS atomics would serialize).
    const uint32_t b0 = __builtin_amdgcn_readfirstlane(bin);
    const uint64_t same = __ballot(bin == b0);
    if (bin == b0) {
      if (b0 != 0xffffffffu && lane == (uint32_t)(__ffsll((unsigned long long)same) - 1))
        atomicAdd(&h[b0], (uint32_t)__popcll(same));
    } else if (bin != 0xffffffffu) {
      atomicAdd(&h[bin], 1u);
    }
  }
  __syncthreads();
  for (uint32_t b = tid; b < TK_RS_BINS; b += TK_WG)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

extern "C" __global__ void __launch_bounds__(TK_WG)
k_rsel_choose(RselState* __restrict__ st, uint32_t shift, uint32_t width, uint32_t* __restrict__ hist) {
  // One workgroup: extend the prefix by the digit where the count from the
  // top reaches `need`, then clear the histogram for the next pass.
  // Thread j sums the j-th group of `per` bins counted from the top; one
  // lane scans the 256 group sums, then the bins of the group where the
  // count reaches `need`.
  __shared__ uint32_t h[TK_RS_BINS];
  __shared__ uint32_t gsum[TK_WG];
  const uint32_t tid = threadIdx.x, nb = 1u << width;
  const uint32_t per = (nb + TK_WG - 1) / TK_WG;
  for (uint32_t b = tid; b < TK_RS_BINS; b += TK_WG) {
    h[b] = b < nb ? hist[b] : 0;
    hist[b] = 0;
  }
  __syncthreads();
  uint32_t s = 0;
  for (uint32_t e = 0; e < per; ++e) {
    const uint32_t r = tid * per + e;                   // rank from the top
    if (r < nb) s += h[nb - 1 - r];
  }
  gsum[tid] = s;
  __syncthreads();
  if (tid == 0) {
    const uint32_t need = st->need;
    uint32_t cum = 0, g = 0;
    while (g + 1 < TK_WG && cum + gsum[g] < need) cum += gsum[g++];
    uint32_t r = g * per, b = nb - 1 - r;
    while (r + 1 < nb && cum + h[b] < need) {
      cum += h[b];
      ++r;
      b = nb - 1 - r;
    }
    st->prefix |= (uint64_t)b << shift;
    st->need = need - cum;
  }
}

extern "C" __global__ void __launch_bounds__(TK_WG)
k_rsel_collect(const int32_t* __restrict__ scores, uint64_t m, RselState* __restrict__ st, uint32_t k,
               uint64_t* __restrict__ out) {
  const uint64_t tau = st->prefix;
  for (uint64_t i = (uint64_t)blockIdx.x * TK_WG + threadIdx.x; i < m; i += (uint64_t)gridDim.x * TK_WG) {
    const uint64_t key = score_key(scores[i], i);
    if (key >= tau) {
      const uint32_t slot = atomicAdd(&st->count, 1u);
      if (slot < k) out[slot] = key;
    }
  }
}

extern "C" __global__ void __launch_bounds__(TK_WG)
k_rank_sort(const uint64_t* __restrict__ keys, uint32_t k, int64_t* __restrict__ idx_out,
            int32_t* __restrict__ val_out) {
  // Key keys[i] goes to position #{j : keys[j] > keys[i]} (keys distinct).
  __shared__ uint64_t tile[HERS_TOPK_TILE];
  const uint32_t i = blockIdx.x * TK_WG + threadIdx.x;
  const uint64_t key = i < k ? keys[i] : 0;
  uint32_t rank = 0;
  for (uint32_t base = 0; base < k; base += HERS_TOPK_TILE) {
    const uint32_t cnt = k - base < HERS_TOPK_TILE ? k - base : HERS_TOPK_TILE;
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < cnt; j += TK_WG) tile[j] = keys[base + j];
    __syncthreads();
    for (uint32_t j = 0; j < cnt; ++j) rank += tile[j] > key;
  }
  if (i < k) {
    idx_out[rank] = key_index(key);
    val_out[rank] = key_score(key);
  }
}

extern "C" __global__ void __launch_bounds__(TK_WG) k_rsel_init(RselState* st, uint32_t k, uint32_t* hist) {
  // state and histogram of the first pass (the workspace holds anything)
  for (uint32_t b = threadIdx.x; b < TK_RS_BINS; b += TK_WG) hist[b] = 0;
  if (threadIdx.x == 0) {
    st->prefix = 0;
    st->need = k;
    st->count = 0;
  }
}

namespace hers {

size_t topk_large_state_bytes() { return 256 + TK_RS_BINS * 4; }

hipError_t launch_topk_large(const int32_t* scores, uint64_t m, uint32_t k, void* work, uint64_t* keys,
                             int64_t* idx_out, int32_t* val_out, uint32_t num_cus, hipStream_t s) {
  RselState* st = (RselState*)work;
  uint32_t* hist = (uint32_t*)((char*)work + 256);
  // k_rsel_init clears the histogram for the first pass, k_rsel_choose after every pass
  hipLaunchKernelGGL(k_rsel_init, dim3(1), dim3(TK_WG), 0, s, st, k, hist);
  hipError_t e = hipGetLastError();
  uint64_t grid = (m + TK_WG - 1) / TK_WG;
  if (grid > (uint64_t)num_cus * 4) grid = (uint64_t)num_cus * 4;
  // histogram passes: one workgroup per CU, since every workgroup adds its
  // count of the few hot bins to the same global words
  const uint64_t hgrid = grid < num_cus ? grid : num_cus;
  static const uint32_t widths[6] = {11, 11, 11, 11, 11, 9};
  uint32_t shift = 64;
  for (int p = 0; p < 6 && e == hipSuccess; ++p) {
    shift -= widths[p];
    hipLaunchKernelGGL(k_rsel_hist, dim3((uint32_t)hgrid), dim3(TK_WG), 0, s, scores, m, st, shift, widths[p], hist);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_rsel_choose, dim3(1), dim3(TK_WG), 0, s, st, shift, widths[p], hist);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rsel_collect, dim3((uint32_t)grid), dim3(TK_WG), 0, s, scores, m, st, k, keys);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rank_sort, dim3((k + TK_WG - 1) / TK_WG), dim3(TK_WG), 0, s, keys, k, idx_out, val_out);
  return hipGetLastError();
}

hipError_t launch_topk_pass(const int32_t* scores, const uint64_t* keys_in, uint64_t count, uint32_t k,
                            uint64_t* keys_out, int64_t* idx_out, int32_t* val_out, hipStream_t s) {
  const uint64_t tiles = (count + HERS_TOPK_TILE - 1) / HERS_TOPK_TILE;
  if (idx_out && tiles != 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_topk_pass, dim3((uint32_t)tiles), dim3(TK_WG), 0, s, scores, keys_in, count, k, keys_out,
                     idx_out, val_out);
  return hipGetLastError();
}

hipError_t launch_topk_tilemax(const int32_t* scores, uint64_t m, uint64_t* maxes, hipStream_t s) {
  const uint64_t tiles = (m + HERS_TOPK_TM - 1) >> HERS_TOPK_TM_LOG2;
  hipLaunchKernelGGL(k_topk_tilemax, dim3((uint32_t)tiles), dim3(TK_WG), 0, s, scores, m, maxes);
  return hipGetLastError();
}

hipError_t launch_topk_filter(const int32_t* scores, uint64_t m, const uint64_t* best, uint32_t nbest, int use_tau,
                              uint32_t k, uint64_t* cand, hipStream_t s) {
  hipLaunchKernelGGL(k_topk_filter, dim3(nbest), dim3(TK_WG), 0, s, scores, m, best, nbest, use_tau, k, cand);
  return hipGetLastError();
}

}  // namespace hers
