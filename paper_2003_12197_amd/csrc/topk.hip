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
  for (uint32_t j = tid; j < S; j += TK_WG) {
    const uint64_t i = base + j;
    uint64_t key = 0;
    if (i < count) key = scores ? score_key(scores[i], i) : keys_in[i];
    tile[j] = key;
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
  for (uint32_t j = tid; j < HERS_TOPK_TM; j += TK_WG) {
    const uint64_t i = base + j;
    if (i < m) {
      const uint64_t key = score_key(scores[i], i);
      if (key >= tau) buf[atomicAdd(&cnt, 1u)] = key;
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

namespace hers {

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
