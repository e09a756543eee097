// kernels.h -- device table bundle and kernel launchers of libhers.
#pragma once
#include <hip/hip_runtime.h>

#include "hers_common.h"

// Device pointers handed to every kernel by value.
struct DevTabs {
  const HersConsts* C;
  const HersConsts* C_rare;   // == C; read by rarely taken paths, whose constant loads then stay apart
  const uint64_t *qtw, *qtw_sh, *qitw, *qitw_sh;   // [k][n]
  const uint32_t *ptw, *ptw_sh, *pitw, *pitw_sh;   // [K][n]
  const uint32_t *ttw, *ttw_sh, *titw, *titw_sh;   // [n]
  uint64_t *pk_ntt, *pk_ntt_sh;                    // [2][k][n] NTT domain
  uint64_t *rlk_ntt, *rlk_ntt_sh;                  // [L][2][k][n] NTT domain
  uint32_t ntt_r;                                  // stages per NTT pass (1..4: radix 2..16)
  uint32_t rl_per;                                 // coefficients per lane of the fused relinearization (8, 16)
  uint32_t nq;                                     // k, the number of q primes (host copy for launch choices)
  // double-precision arithmetic mod q (every q_i < 2^45): twiddles as
  // doubles [k][n], and qf[i] = q_i, qf[HC_MAXQ + i] = fl(1 / q_i),
  // qf[2 HC_MAXQ + i] = n^-1 mod q_i
  int qf_ok;
  const double *qtw_f, *qitw_f, *qf;
};

// Query values of a probe encryption, passed by value in the kernel arguments
// (no host-to-device copy): up to HERS_QCHUNK dimensions per launch.
#define HERS_QCHUNK 256
struct QueryVals {
  int32_t v[HERS_QCHUNK];
};

// Batched multiply-accumulate: up to MB_PROBES probes of one gallery per group.
#define MB_PROBES 16
#define MB_DC 8         // dimensions per register/LDS chunk
#define MB_BLOCKS 4     // blocks per work item
#define MB_MAXG 15      // groups per launch (kernel arguments stay below 4 KiB)

struct MacGroup {
  const uint32_t* gallery;            // search form [M][K][d][2][n]
  const uint32_t* probe[MB_PROBES];   // search forms [K][d][2][n]
  uint32_t* acc;                      // probe j's accumulators at acc + j * acc_stride: [blocks][3][K][n]
  uint64_t acc_stride;                // u32 words
  int64_t blk_lo, blk_hi;             // blocks of this round; accumulators indexed from blk_lo
  uint64_t item_begin;                // first work item of the group
  int32_t d, nprobe;
};

// Score-ciphertext pointers of the requests of one epilogue launch.
#define EP_MAXR 64
struct ScorePtrs {
  uint64_t* p[EP_MAXR];
};

struct MacBatchArgs {
  MacGroup g[MB_MAXG];
  uint64_t total_items;
  int32_t ngroups, pad;
};

namespace hers {
// variants as (probes per wave, dimensions per chunk, blocks per item):
// 0 (1, 8, 4) with 1024-lane workgroups; 1 (2, 4, 2), 2 (2, 8, 2) with 512
// lanes; 3 (4, 4, 1) with 256 lanes
#define MB_VARIANTS 5
#define MB_MFMA 4         // the schedule on the matrix cores (int8 digit products), d <= 128
hipError_t launch_mac_multi(const DevTabs& T, const MacBatchArgs& A, uint32_t grid, hipStream_t s, int variant = 0);
hipError_t launch_keygen(const DevTabs& T, uint32_t n, uint32_t k, uint32_t L, uint64_t seed, uint8_t* sk,
                         uint64_t* pk, uint64_t* rlk, hipStream_t s);
hipError_t launch_load_keys(const DevTabs& T, uint32_t n, uint32_t k, uint32_t L, const uint64_t* pk,
                            const uint64_t* rlk, hipStream_t s);
hipError_t launch_encode(const DevTabs& T, uint32_t n, const int32_t* feats, int64_t ld, int64_t item_lo,
                         int64_t item_hi, int64_t fbase, int32_t d, int64_t block0, int64_t nblocks, uint32_t* pt,
                         hipStream_t s);
hipError_t launch_ct_add(const DevTabs& T, uint32_t n, uint32_t k, uint64_t* dst, const uint64_t* fresh, uint32_t nct,
                         int32_t d, int64_t block0, int64_t first_empty_block, hipStream_t s);
// gallery (pt != NULL: nct plaintexts) or probe (query != NULL: host values of
// dimensions qdim0 .. qdim0 + nct - 1, canon at the first of them)
hipError_t launch_encrypt(const DevTabs& T, uint32_t n, uint32_t k, uint32_t nct, const uint32_t* pt,
                          const int32_t* query, int32_t d, int64_t block0, uint64_t seed, uint32_t domain,
                          uint64_t* canon, hipStream_t s, int32_t qdim0 = 0);
// probe dimensions 0 .. d - 1 from host query values
hipError_t launch_encrypt_sk(const DevTabs& T, uint32_t n, uint32_t k, const int32_t* query, int32_t d, uint64_t seed,
                             const uint64_t* S, const uint64_t* Ssh, uint64_t* canon, hipStream_t s);
hipError_t launch_lift(const DevTabs& T, uint32_t n, const uint64_t* canon, uint32_t nct, int32_t d,
                       int64_t block0, uint32_t* out, hipStream_t s);
hipError_t launch_unlift(const DevTabs& T, uint32_t n, const uint32_t* coef, uint32_t nct, int32_t d,
                         uint64_t* canon, hipStream_t s);
hipError_t launch_check_features(const int32_t* v, int64_t ld, int32_t rows, int64_t cols, int32_t bound,
                                 uint32_t* flag, uint32_t num_cus, hipStream_t s);
hipError_t launch_check_canon(const DevTabs& T, const uint64_t* canon, uint64_t words, uint32_t* flag,
                              uint32_t num_cus, hipStream_t s);
hipError_t launch_ntt_p(const DevTabs& T, uint32_t n, uint32_t* polys, uint64_t npolys, uint32_t inner,
                        int inverse, hipStream_t s, uint32_t nsets = 1, uint64_t set_stride = 0);
hipError_t launch_mac(const DevTabs& T, uint32_t n, uint32_t K, const uint32_t* gallery, const uint32_t* probe,
                      int32_t d, int64_t blk_lo, int64_t blk_hi, uint32_t* acc, hipStream_t s, int variant,
                      uint32_t target_wgs = 0, int32_t dim0 = 0, int32_t dcount = 0);
// one probe's multiply-accumulate with the inverse NTT of the accumulators
// fused in: writes them in the coefficient domain
hipError_t launch_mac_intt(const DevTabs& T, uint32_t n, uint32_t K, const uint32_t* gallery, const uint32_t* probe,
                           int32_t d, int64_t blk_lo, int64_t blk_hi, uint32_t* acc, hipStream_t s,
                           uint32_t target_wgs = 0, int32_t dim0 = 0, int32_t dcount = 0);
hipError_t launch_rescale(const DevTabs& T, uint32_t n, const uint32_t* X, int64_t nblk, int64_t blk_lo,
                          const ScorePtrs& SP, uint32_t nreq, uint64_t* digits, uint64_t acc_stride,
                          uint64_t dig_stride, hipStream_t s, uint32_t k, uint32_t K, uint32_t W);
hipError_t launch_relin(const DevTabs& T, uint32_t n, uint32_t k, uint32_t L, uint64_t* digits, int64_t nblk,
                        int64_t blk_lo, const ScorePtrs& SP, uint32_t nreq, uint64_t dig_stride, hipStream_t s,
                        const uint64_t* key = nullptr, const uint64_t* key_sh = nullptr,
                        uint32_t fuse_min_wgs = 2048);
// two-stage search, second stage (rerank.hip)
hipError_t launch_encode_packed(const DevTabs& T, uint32_t n, const int32_t* feats, int64_t ld, int64_t count,
                                int32_t D, int32_t W, int replicate, uint32_t nct, uint32_t* pt, hipStream_t s);
hipError_t launch_rotkey(const DevTabs& T, uint32_t n, uint32_t k, uint32_t L, uint32_t nsteps, uint64_t seed,
                         uint64_t* rk, uint64_t* rk_ntt, uint64_t* rk_ntt_sh, hipStream_t s);
hipError_t launch_rot_digits(const DevTabs& T, uint32_t n, uint32_t k, const uint64_t* ct_in, uint64_t* ct_out,
                             uint64_t* digits, uint32_t nct, uint32_t g, hipStream_t s);
hipError_t launch_gather_cts(const uint32_t* items, uint64_t words_per_ct, int64_t nct_total, const int64_t* ids,
                             uint32_t nsel, uint32_t* out, hipStream_t s);
hipError_t launch_rerank_pick(uint32_t n, const int32_t* slot_scores, uint32_t nsel, int32_t W, int32_t* out,
                              hipStream_t s);
hipError_t launch_sk_ntt(const DevTabs& T, uint32_t n, uint32_t k, const uint8_t* sk, uint64_t* S, uint64_t* Ssh,
                         hipStream_t s);
hipError_t launch_dec_mul(const DevTabs& T, uint32_t n, uint32_t k, const uint64_t* scores, int64_t nblk,
                          int64_t blk_lo, const uint64_t* S, const uint64_t* Ssh, uint64_t* x, hipStream_t s);
// Decryption and decoding in one kernel per block (the double-precision
// form at n = 4096 with three q primes); false / hipErrorInvalidValue
// elsewhere.
bool dec_fused_fits(const DevTabs& T, uint32_t n);
hipError_t launch_dec_fused(const DevTabs& T, uint32_t n, const uint64_t* scores, int64_t nblk, int64_t blk_lo,
                            const uint64_t* S, int64_t m, int32_t* out, hipStream_t s);
hipError_t launch_dec_decode(const DevTabs& T, uint32_t n, const uint64_t* x, int64_t nblk, int64_t blk_lo,
                             int64_t m, int32_t* out, hipStream_t s);
// top-k of decrypted scores (topk.hip): generic passes over tiles of
// HERS_TOPK_TILE keys, tile maxima over tiles of HERS_TOPK_TM scores
#define HERS_TOPK_TILE 2048
#define HERS_TOPK_TM_LOG2 12
#define HERS_TOPK_TM (1u << HERS_TOPK_TM_LOG2)
#define HERS_TOPK_TILE_K 512     // largest k of the tile path
#define HERS_TOPK_MAX_K 16384    // largest k (radix-select path above HERS_TOPK_TILE_K)
size_t topk_large_state_bytes();
hipError_t launch_topk_large(const int32_t* scores, uint64_t m, uint32_t k, void* work, uint64_t* keys,
                             int64_t* idx_out, int32_t* val_out, uint32_t num_cus, hipStream_t s);
hipError_t launch_topk_pass(const int32_t* scores, const uint64_t* keys_in, uint64_t count, uint32_t k,
                            uint64_t* keys_out, int64_t* idx_out, int32_t* val_out, hipStream_t s);
hipError_t launch_topk_tilemax(const int32_t* scores, uint64_t m, uint64_t* maxes, hipStream_t s);
hipError_t launch_topk_filter(const int32_t* scores, uint64_t m, const uint64_t* best, uint32_t nbest, int use_tau,
                              uint32_t k, uint64_t* cand, hipStream_t s);
}  // namespace hers
