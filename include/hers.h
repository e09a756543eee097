/*
 * hers.h -- C ABI of the MI355X HERS encrypted-search library (libhers.so).
 *
 * HERS (Engelsma, Jain, Boddeti, "HERS: Homomorphically Encrypted
 * Representation Search") scores a query q in Z^d against a gallery
 * P in Z^{d x m} under FV encryption: r(P, q) = P^T q computed on ciphertexts
 * (Sec. 3.1, Eq. 1).  Each gallery dimension of a block of n items is one FV
 * ciphertext with item j in slot j; each query dimension is one ciphertext with
 * its value in every slot (Sec. 3.2, Eq. 2-4).  The server multiplies the
 * ciphertexts dimension by dimension and sums over d (App. B, Alg. "HERS
 * Search"); the client decrypts one score ciphertext per block.
 *
 * Conventions for every call
 *   - Return value: HERS_OK (0) or a negative HERS_E* code; hers_last_error()
 *     returns a thread-local message for the last failure.
 *   - Pointers named *_dev are device pointers on the context's GPU; the caller
 *     allocates and owns them (sizes from the hers_*_words / hers_*_bytes
 *     queries) and must keep them alive until the work on `stream` completes.
 *     Pointers without the suffix are host pointers.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL = the
 *     default stream) and is complete when the stream is synchronised.
 *   - Canonical ciphertext layout (the exchange format, bit-comparable with
 *     the reference oracle): uint64 [2][k][n], component (ct[0], ct[1]),
 *     residue modulo q_i, coefficient j, every residue in [0, q_i).
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Search-form buffers are passed with their length in u32 words: a probe
 *     must be exactly hers_probe_words(d) long, a gallery a whole number of
 *     blocks of hers_gallery_words(n, d) words covering the m items; a buffer
 *     of another d is rejected with HERS_EDIM.
 *   - Calls that take device features or canonical ciphertexts check every
 *     value on the GPU first (HERS_ERANGE) and synchronise `stream` to read
 *     the result: they are not for stream capture.  A probe's query is a
 *     host array, checked on the host.
 *
 * Randomness: every random polynomial is drawn from Philox4x64-10 (Salmon et
 * al., SC'11) with key (seed, domain) and counter (w / 4, obj0, obj1, obj2);
 * binary polynomials take bit j mod 64 of word j / 64, errors are centred
 * binomial (eta = 20) from word j, uniform residues mod q_i come from words
 * 2(i n + j), 2(i n + j) + 1 read as a 128-bit integer reduced mod q_i.
 */
#ifndef HERS_H
#define HERS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HERS_OK 0
#define HERS_EINVAL (-1)   /* bad argument: null pointer, size, layout       */
#define HERS_EPARAM (-2)   /* unsupported or non NTT-friendly parameters     */
#define HERS_EDIM (-3)     /* dimension count out of range or mismatched     */
#define HERS_ESPACE (-4)   /* workspace too small                            */
#define HERS_EDEVICE (-5)  /* HIP runtime error                              */
#define HERS_ENOMEM (-6)   /* device allocation of library tables failed     */
#define HERS_ERANGE (-7)   /* input value out of range: a feature or query   */
                           /* beyond +-feature_bound, or a canonical residue */
                           /* not below its prime                            */

#define HERS_MAX_QPRIMES 8

/* Encryption parameters (App. A; Sec. 4.1 uses n = 4096, t = 1,032,193 and
 * three 36-bit primes in q).
 *   n          ring degree, a power of two in [256, 8192]; R = Z[x]/(x^n + 1)
 *   k, qbits   q is the product of k primes, the i-th being the largest prime
 *              below 2^qbits[i] that is 1 mod 2n and not yet taken (20..60 bits)
 *   t_bits     t is the largest prime below 2^t_bits that is 1 mod 2n (<= 22)
 *   w_bits     relinearization digit width: 0 = one digit per prime of q,
 *              else each residue digit is split into w_bits-bit digits
 *   d_max      largest number of dimensions a gallery may have; sizes the
 *              internal exact-product base
 *   feature_bound  largest |feature| of gallery and query; the context is
 *              rejected unless d_max * feature_bound^2 < t / 2, so that every
 *              score is recovered exactly modulo t (Sec. 3.2, "Encoding Scheme")
 */
typedef struct {
  uint32_t n;
  uint32_t k;
  uint32_t qbits[HERS_MAX_QPRIMES];
  uint32_t t_bits;
  uint32_t w_bits;
  uint32_t d_max;
  uint32_t feature_bound;
} hers_params;

/* Values derived from hers_params by the prime rule (no GPU needed). */
typedef struct {
  uint32_t n, k;
  uint64_t q[HERS_MAX_QPRIMES];   /* ciphertext primes q_0..q_{k-1}            */
  uint64_t t;                     /* plaintext modulus                          */
  uint32_t num_digits;            /* L: evaluation keys (gadget digits)         */
  uint32_t num_aux;               /* K: primes < 2^30 of the exact-product base */
  uint64_t aux[32];               /* those primes                               */
  double   log2_q, log2_aux;      /* log2 q and log2 of the product base        */
  uint32_t d_max, feature_bound;  /* as in hers_params                           */
} hers_info;

typedef struct hers_ctx hers_ctx;

const char* hers_last_error(void);

/* Resolve parameters on the host only (prime selection, digit counts). */
int hers_params_resolve(const hers_params* params, hers_info* out);

/* Create a context on HIP device `device`: precomputes NTT tables and the
 * constants of the exact base conversions and uploads them (library-owned
 * device memory, freed by hers_ctx_destroy). */
int hers_ctx_create(const hers_params* params, int device, hers_ctx** out);
void hers_ctx_destroy(hers_ctx* ctx);
int hers_ctx_info(const hers_ctx* ctx, hers_info* out);

/* ---- sizes (in elements of the stated type) ---------------------------- */
uint64_t hers_blocks(const hers_ctx* ctx, int64_t m);                 /* M = ceil(m / n)          */
uint64_t hers_ct_words(const hers_ctx* ctx);                          /* u64: 2 k n (one ct)      */
uint64_t hers_pk_words(const hers_ctx* ctx);                          /* u64: 2 k n               */
uint64_t hers_rlk_words(const hers_ctx* ctx);                         /* u64: L 2 k n             */
uint64_t hers_gallery_words(const hers_ctx* ctx, int64_t m, int32_t d); /* u32: M K d 2 n search form */
uint64_t hers_probe_words(const hers_ctx* ctx, int32_t d);            /* u32: K d 2 n search form */
/* workspace bytes for one call; `op` is 0 = encrypt_gallery (per block of
 * the chunk size given in `m` items), 1 = encrypt_probe, 2 = search over m
 * items, 3 = decrypt_scores over m items, 4 = enroll_append of a batch of
 * m items, 5 = search_literal over m items, 6 = rerank_encrypt of m
 * ciphertexts, 7 = rerank of m selected ciphertexts, 8 = rerank_decrypt of m
 * ciphertexts, 9 = export of the search form of m items (a probe: m = 1),
 * 10 = encrypt_probe_sk of d dimensions. */
uint64_t hers_workspace_bytes(const hers_ctx* ctx, int op, int64_t m, int32_t d);

/* ---- keys (App. A, Alg. "Key Generation") ------------------------------- */
/* theta_sk from R_2, pk = ([-(a s + e)]_q, a), and one evaluation key
 * ([-(a_g s + e_g) + g s^2]_q, a_g) per gadget digit g (the paper's base-w
 * decomposition generalised to RNS digits; w_bits above).  Philox key
 * (seed, 1); objects s (0,0,0), a (1,0,0), e (2,0,0), a_g (3,g,0), e_g (4,g,0).
 *   sk_dev  uint8 [n] in {0,1}; pk_dev canonical [2][k][n]; rlk_dev [L][2][k][n].
 * The public and evaluation keys are also loaded into the context. */
int hers_keygen(hers_ctx* ctx, uint64_t seed, uint8_t* sk_dev, uint64_t* pk_dev,
                uint64_t* rlk_dev, void* stream);

/* Load externally held keys (canonical layouts above) into the context. */
int hers_load_keys(hers_ctx* ctx, const uint64_t* pk_dev, const uint64_t* rlk_dev, void* stream);

/* ---- enrollment (Sec. 3.2 "Enrollment Protocol"; App. B Alg. "HERS Enrollment") ----
 * Encrypts gallery blocks [block0, block0 + nblocks) of a gallery of m_total
 * items and d dimensions.  feats_dev is int32 [d][ld] dimension-major
 * (Eq. 3: row i holds dimension i of every item) and holds items
 * block0*n .. block0*n + nblocks*n - 1 (those >= m_total are read as 0), ld
 * is its row stride in items (>= nblocks*n, or >= the remaining items).
 * Every feature of the range must lie in [-feature_bound, feature_bound]
 * (else HERS_ERANGE and nothing is encrypted).
 * Block b, dimension i is Encrypt(BatchEncode(row i of block b)) with Philox
 * key (seed, 2) and objects (b, i, 0|1|2) for u, e1, e2.
 *   gallery_dev  search form, u32 [M][K][d][2][n]; blocks outside the range
 *                are not touched.
 *   canon_dev    optional (NULL to skip): canonical cts [M][d][2][k][n].
 *   work_dev     workspace of hers_workspace_bytes(ctx, 0, nblocks*n, d).  */
int hers_encrypt_gallery(hers_ctx* ctx, const int32_t* feats_dev, int64_t ld, int64_t m_total,
                         int32_t d, int64_t block0, int64_t nblocks, uint64_t seed,
                         uint32_t* gallery_dev, uint64_t* canon_dev, void* work_dev,
                         size_t work_bytes, void* stream);

/* ---- online enrollment (App. B Alg. "HERS Enrollment", online form) ------
 * Appends c items (feats_dev int32 [d][ld], ld >= c: items k0 .. k0+c-1) to
 * a gallery that holds items 0 .. k0-1.  Client half: the batch is split at
 * block boundaries; for every block b it touches, dimension i is
 * Encrypt(BatchEncode(the batch's values of dimension i in their slots,
 * zero elsewhere)) with Philox key (seed, 4) and objects (b, i, 0|1|2)
 * (a seed must not be reused for another batch; features within
 * +-feature_bound, else HERS_ERANGE).  Server half: CipherAdd
 * into block b's running ciphertext; a block that held no item starts from
 * the trivial zero ciphertext (reading of the algorithm's Encrypt(0), whose
 * rollover branch also drops the incoming ciphertext -- here the batch is
 * split instead).  Touched blocks are lifted again into the search form.
 *   canon_dev    running canonical cts [M][d][2][k][n] (hers_encrypt_gallery's
 *                optional output, or earlier appends), updated in place;
 *                blocks past the last one holding an item may hold anything.
 *   gallery_dev  search form u32 [M][K][d][2][n], touched blocks rewritten.
 *   M must cover item k0 + c - 1.  work_dev: hers_workspace_bytes(ctx, 4, c, d). */
int hers_enroll_append(hers_ctx* ctx, const int32_t* feats_dev, int64_t ld, int64_t k0, int64_t c,
                       int32_t d, uint64_t seed, uint64_t* canon_dev, uint32_t* gallery_dev,
                       void* work_dev, size_t work_bytes, void* stream);

/* ---- query (App. B Alg. "HERS Search", client side) ---------------------
 * Dimension i is the constant plaintext [q_i]_t (Eq. 2), encrypted with the
 * public key (Philox key (seed, 3), objects (0, i, 0|1|2)).
 *   query int32 [d] in HOST memory, every value within +-feature_bound (else
 *   HERS_ERANGE, checked on the host); the values travel in the kernel
 *   arguments, so the call does not wait on the stream;
 *   probe_dev search form u32 [K][d][2][n];
 *   canon_dev optional canonical cts [d][2][k][n]. */
int hers_encrypt_probe(hers_ctx* ctx, const int32_t* query, int32_t d, uint64_t seed,
                       uint32_t* probe_dev, uint64_t* canon_dev, void* work_dev,
                       size_t work_bytes, void* stream);

/* The query encrypted under the client's secret key instead (Sec. 3.2,
 * "Search Protocol": the client encrypts the query "using the private key";
 * App. A defines only public-key encryption, which hers_encrypt_probe
 * follows): dimension i is ([Delta [q_i]_t - a s + e]_q, a), a uniform in R_q
 * (Philox key (seed, 7), object (0, i, 0): residue rho of coefficient j from
 * words 2(rho n + j), 2(rho n + j) + 1 as a 128-bit integer), e centred
 * binomial (object (0, i, 1)); so ct0 + ct1 s = Delta m + e, with less noise
 * than the public-key form.  Searched like any probe.
 *   sk_dev uint8 [n], or NULL for the key of hers_load_secret_key;
 *   query int32 [d] in host memory within +-feature_bound (else HERS_ERANGE);
 *   probe_dev search form u32 [K][d][2][n] of probe_words words (else HERS_EDIM);
 *   canon_dev optional canonical cts [d][2][k][n];
 *   work_dev hers_workspace_bytes(ctx, 10, 0, d) (less without a canon_dev
 *   or with sk_dev NULL: none when both are absent). */
int hers_encrypt_probe_sk(hers_ctx* ctx, const uint8_t* sk_dev, const int32_t* query, int32_t d, uint64_t seed,
                          uint32_t* probe_dev, uint64_t probe_words, uint64_t* canon_dev, void* work_dev,
                          size_t work_bytes, void* stream);

/* ---- canonical ciphertexts in and out (Sec. 3.2 "Enrollment Protocol" and
 * "Search Protocol": the client encrypts and sends ciphertexts, the server
 * stores and searches them without any plaintext) -------------------------
 * Import: canonical ciphertexts -> search form (exact centred lift to the
 * product base, forward NTT); every residue must be below its prime (else
 * HERS_ERANGE and nothing is written).
 *   hers_import_gallery: canon_dev holds blocks block0 .. block0 + nblocks - 1
 *     only, [nblocks][d][2][k][n] (so a large gallery is imported in chunks);
 *     gallery_dev is the whole gallery's search form (gallery_words long),
 *     blocks outside the range are not touched.
 *   hers_import_probe: canon_dev [d][2][k][n] -> probe_dev [K][d][2][n].
 * Export: search form -> canonical ciphertexts (inverse NTT, exact CRT over
 * the product base, residues mod q_i): the inverse of import, so an imported
 * or encrypted ciphertext comes back bit for bit.
 *   hers_export_gallery: blocks block0 .. block0 + nblocks - 1 into canon_dev
 *     [nblocks][d][2][k][n]; work_dev hers_workspace_bytes(ctx, 9, m, d) for
 *     the blocks of one pass (less: blocks in chunks, at least one block).
 *   hers_export_probe: probe_dev -> canon_dev [d][2][k][n]; work_dev
 *     hers_workspace_bytes(ctx, 9, 1, d). */
int hers_import_gallery(hers_ctx* ctx, const uint64_t* canon_dev, int64_t m_total, int32_t d, int64_t block0,
                        int64_t nblocks, uint32_t* gallery_dev, uint64_t gallery_words, void* stream);
int hers_import_probe(hers_ctx* ctx, const uint64_t* canon_dev, int32_t d, uint32_t* probe_dev,
                      uint64_t probe_words, void* stream);
int hers_export_gallery(hers_ctx* ctx, const uint32_t* gallery_dev, uint64_t gallery_words, int64_t m_total,
                        int32_t d, int64_t block0, int64_t nblocks, uint64_t* canon_dev, void* work_dev,
                        size_t work_bytes, void* stream);
int hers_export_probe(hers_ctx* ctx, const uint32_t* probe_dev, uint64_t probe_words, int32_t d,
                      uint64_t* canon_dev, void* work_dev, size_t work_bytes, void* stream);

/* ---- search (App. B Alg. "HERS Search", server side) --------------------
 * For every block b: X_0 = sum_i P_i0 G_bi0, X_1 = sum_i (P_i0 G_bi1 + P_i1 G_bi0),
 * X_2 = sum_i P_i1 G_bi1 over Z[x]/(x^n+1) (centred representatives), then
 * c_j = [round(t X_j / q)]_q (Alg. "Ciphertext Multiplication"), then one
 * relinearization with the context's evaluation keys.
 *   scores_dev canonical score cts [M][2][k][n].
 * Work is ordered on `stream`; with "overlap_chunks" it is split between
 * `stream` and the context's own stream and joined back into `stream`
 * (one context must not run two searches from different host threads). */
int hers_search(hers_ctx* ctx, const uint32_t* gallery_dev, uint64_t gallery_words, int64_t m,
                int32_t d, const uint32_t* probe_dev, uint64_t probe_words, uint64_t* scores_dev,
                void* work_dev, size_t work_bytes, void* stream);

/* For callers that cannot allocate device memory (code under stream or graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * search as hers_search, bit for bit, with its workspace (accumulators and
 * relinearization digits) in a static device array of HERS_SCRATCH_BYTES that
 * the library holds on each GPU it runs on until the process ends.  The call
 * allocates nothing; the blocks run in chunks that fit the array (never the
 * overlapped schedule).  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (two streams, two threads, two contexts)
 * race and must be serialised by the caller.  Every word the kernels read
 * from the array is written earlier in the same call, so no state carries
 * over between calls.  HERS_ESPACE if one block's workspace exceeds the
 * array (no shipped parameter set does: n = 8192, five primes and K = 16
 * need 3.2 MB). */
#define HERS_SCRATCH_BYTES (64ull << 20)
int hers_search_noalloc(hers_ctx* ctx, const uint32_t* gallery_dev, uint64_t gallery_words, int64_t m,
                        int32_t d, const uint32_t* probe_dev, uint64_t probe_words, uint64_t* scores_dev,
                        void* stream);

/* The paper-literal schedule (App. B Alg. "HERS Search" as printed): for
 * every dimension i, CipherMultiply(probe_i, gallery_i) -- tensor, rescale,
 * relinearization -- then CipherAdd into the block's score ciphertext.  The
 * same decrypted scores as hers_search (the plaintext products are summed
 * either way) from d times the rescales and relinearizations and other
 * ciphertext bits; kept as the timed comparison for the fused schedule.
 *   work_dev  hers_workspace_bytes(ctx, 5, m, d) (or less: blocks in chunks). */
int hers_search_literal(hers_ctx* ctx, const uint32_t* gallery_dev, uint64_t gallery_words,
                        int64_t m, int32_t d, const uint32_t* probe_dev, uint64_t probe_words,
                        uint64_t* scores_dev, void* work_dev, size_t work_bytes, void* stream);

/* Batched search: nreq independent (gallery, probe) requests in one
 * submission; request r reads galleries[r] (gallery_words[r] long, m[r]
 * items, d[r] dims) and probes[r] (probe_words[r] long) and writes scores[r].  Requests on the same gallery (same
 * pointer, m and d) are grouped, up to "mb_group" (16) per group: one persistent
 * multiply-accumulate launch streams each gallery block once for the whole
 * group, then every request gets its own rescale and relinearization.
 * Results are bit-identical to nreq calls of hers_search.  The workspace
 * holds at least one block per request; with W bytes, rounds of
 * floor(W / (nreq * hers_workspace_bytes(ctx, 2, n, 1))) blocks are used. */
int hers_search_batch(hers_ctx* ctx, int32_t nreq, const uint32_t* const* galleries,
                      const uint64_t* gallery_words, const int64_t* m, const int32_t* d,
                      const uint32_t* const* probes, const uint64_t* probe_words,
                      uint64_t* const* scores, void* work_dev, size_t work_bytes, void* stream);

/* Batched autotuner: times every multi-probe multiply-accumulate schedule
 * ("mb_variant") on the caller's batch -- the first round of blocks of
 * hers_search_batch with these arguments, reps launches each -- and keeps the
 * fastest in the context (another replaces the current one only if 3%
 * faster); the schedule in *chosen (may be NULL).  Overwrites the workspace;
 * synchronizes `stream`.  The schedules compute the same bits. */
int hers_autotune_batch(hers_ctx* ctx, int32_t nreq, const uint32_t* const* galleries,
                        const uint64_t* gallery_words, const int64_t* m, const int32_t* d,
                        const uint32_t* const* probes, const uint64_t* probe_words, uint64_t* const* scores,
                        void* work_dev, size_t work_bytes, int reps, void* stream, int64_t* chosen);

/* The same batch captured once as a HIP graph and replayed by
 * hers_plan_launch: the pointers are fixed at capture, so callers refill the
 * probe buffers (hers_encrypt_probe into the same probe_dev) and replay.
 * The plan keeps the context, galleries, probes, scores and workspace
 * pointers; they must stay valid until hers_plan_destroy. */
typedef struct hers_plan hers_plan;
int hers_plan_create(hers_ctx* ctx, int32_t nreq, const uint32_t* const* galleries,
                     const uint64_t* gallery_words, const int64_t* m, const int32_t* d,
                     const uint32_t* const* probes, const uint64_t* probe_words,
                     uint64_t* const* scores, void* work_dev, size_t work_bytes, hers_plan** out);
int hers_plan_launch(hers_plan* plan, void* stream);
void hers_plan_destroy(hers_plan* plan);

/* ---- decryption (App. B Alg. "HERS Search", client side) ----------------
 * pt = [round(t/q [c0 + c1 s]_q)]_t (Alg. "Decryption"), slot decode, centred
 * into [-t/2, t/2): scores_out_dev int32 [m], item b*n + j from slot j of block b.
 * sk_dev uint8 [n], or NULL to use the key of hers_load_secret_key (whose
 * transform is then not repeated per call); work_dev
 * hers_workspace_bytes(ctx, 3, m, 1) (blocks in chunks if smaller). */
/* Keeps the NTT form of a client's secret key in the context (stream-ordered
 * on `stream`; a later call replaces it). */
int hers_load_secret_key(hers_ctx* ctx, const uint8_t* sk_dev, void* stream);
int hers_decrypt_scores(hers_ctx* ctx, const uint8_t* sk_dev, const uint64_t* scores_dev,
                        int64_t m, int32_t* scores_out_dev, void* work_dev, size_t work_bytes,
                        void* stream);

/* ---- two-stage search, second stage (Sec. 4 "Two Stage Search") ----------
 * The first stage is a HERS search on a low-dimensional representation and
 * hers_topk of its decrypted scores; the second re-ranks the candidates with
 * the full representation under an encryption that addresses single items.
 * The paper names a 1:1 matcher for this stage without giving its steps;
 * this is a packed one:
 *   Packing: S = n / W items per ciphertext (W a power of two in [2, n/2],
 *   features D <= W, D <= d_max), item x in ciphertext x / S, segment x mod S
 *   of W slots; the probe is repeated in every segment.  Position p of row r
 *   is slot j with 2j + 1 = (-1)^r 5^p mod 2n; segment c of row r holds
 *   positions [W c, W c + W) (segment index r n / 2W + c).
 *   Score: one ciphertext product (tensor, rescale, relinearization), then
 *   for s = 1, 2, ..., W/2: ct += rotate(ct, 5^s), a rotation being the
 *   automorphism x -> x^(5^s) of both components and key switching from
 *   s(x^(5^s)) to s; each segment's first position then holds the item's
 *   inner product with the probe (|score| must stay below t/2).
 * Rotation keys: one per step, ([-(a s + e) + g_l s(x^(5^s))]_q, a) for every
 * gadget element g_l; Philox key (seed, 1), objects a (5, l, step), e (6, l,
 * step), s as in hers_keygen (same seed gives the same secret).
 *   rk_dev canonical [log2 W][L][2][k][n] (hers_rotation_key_words); the NTT
 *   form stays in the context. */
uint64_t hers_rotation_key_words(const hers_ctx* ctx, int32_t W);
int hers_rotation_keygen(hers_ctx* ctx, uint64_t seed, int32_t W, uint64_t* rk_dev, void* stream);

/* Encrypts items (replicate = 0: feats_dev int32 [D][ld], columns 0..count-1,
 * ceil(count / S) ciphertexts, Philox key (seed, 5), objects (c, 0, 0|1|2))
 * or a probe (replicate = 1, count = 1: column 0 in every segment, one
 * ciphertext, key (seed, 6), objects (0, 0, 0|1|2)); every feature within
 * +-feature_bound, else HERS_ERANGE.
 *   search_dev u32 [nct][K][2][n] (search form, d = 1); canon_dev optional
 *   canonical [nct][2][k][n]; work_dev hers_workspace_bytes(ctx, 6, nct, 0). */
int hers_rerank_encrypt(hers_ctx* ctx, const int32_t* feats_dev, int64_t ld, int64_t count, int32_t D,
                        int32_t W, int replicate, uint64_t seed, uint32_t* search_dev, uint64_t* canon_dev,
                        void* work_dev, size_t work_bytes, void* stream);

/* Server: scores the probe against the nsel ciphertexts ids_dev (device int64
 * [nsel], indices into items_search of nct_total ciphertexts; an index outside
 * [0, nct_total) selects an all-zero ciphertext, whose scores are 0).
 *   out_cts canonical [nsel][2][k][n]; work_dev hers_workspace_bytes(ctx, 7,
 *   nsel, 0) or less (ciphertexts in chunks).  Needs hers_rotation_keygen
 *   with this W (or a larger one) first. */
int hers_rerank(hers_ctx* ctx, const uint32_t* items_search, int64_t nct_total, const int64_t* ids_dev,
                int32_t nsel, const uint32_t* probe_search, int32_t W, uint64_t* out_cts, void* work_dev,
                size_t work_bytes, void* stream);

/* Client: decrypts the nsel re-rank ciphertexts and reads every segment's
 * score: scores_out int32 [nsel][n / W] (score of item ids[c] * S + seg at
 * [c][seg]); sk_dev as for hers_decrypt_scores (NULL: the loaded key);
 * work_dev hers_workspace_bytes(ctx, 8, nsel, 0). */
int hers_rerank_decrypt(hers_ctx* ctx, const uint8_t* sk_dev, const uint64_t* cts, int32_t nsel, int32_t W,
                        int32_t* scores_out, void* work_dev, size_t work_bytes, void* stream);

/* ---- tuning --------------------------------------------------------------
 * Kernel schedule knobs, normally chosen by hers_autotune.  Keys:
 *   "mac_variant"  fused multiply-accumulate schedule, 0..11, as (gallery
 *                  blocks per pass sharing one probe load, dimensions per
 *                  double-buffered load batch, non-temporal gallery loads):
 *                  0 (1,2,no) 1 (2,2,no) 2 (1,4,no) 3 (2,4,no) 4 (1,2,yes)
 *                  5 (2,2,yes) 6 (1,4,yes) 7 (2,4,yes) 8 (4,1,yes)
 *                  9 (4,2,yes) 10 (2,1,yes) 11 (1,1,yes); 12 (n <= 4096 only):
 *                  one workgroup per (block, prime) over the whole ring,
 *                  with the inverse NTT of the accumulators fused in (no
 *                  separate transform launch or round trip through memory).
 *   "ntt_radix_log2" stages per NTT pass, 1..4 (radix 2, 4, 8, 16; default 4):
 *                  each pass keeps 2^r elements per lane in registers and
 *                  costs one barrier.
 *   "overlap_chunks" hers_search in this many block chunks, 0..256 (0 =
 *                  automatic: 8 from 4096 blocks up, else off; 1 = off):
 *                  each chunk's rescale and relinearization run on the
 *                  context's own stream beside the next chunk's
 *                  multiply-accumulate.  The caller's stream waits for that
 *                  stream before hers_search returns, so stream order holds.
 *   "mac_wgs_per_cu" workgroups per compute unit of a hers_search
 *                  multiply-accumulate launch, 0..64 (0 = 8, for schedule
 *                  12 the n/4-lane workgroups that fill a CU: 2 at n = 4096);
 *                  fewer leave room on each CU for an overlapped epilogue.
 *   "relin_fuse_min_wgs" relinearizations (and rotations) launched with at
 *                  least this many workgroups (blocks x primes x requests)
 *                  run as one fused kernel per (block, prime): digit
 *                  transforms, key products, inverse transforms without the
 *                  transformed digits in memory; smaller ones as two kernels
 *                  with more workgroups.  0 = 8 per compute unit at
 *                  n >= 8192; below n = 8192 always where every q_i <
 *                  2^45, "relin_lane_coeffs" is 8 and "ntt_radix_log2" is at
 *                  least 3, else never; 1 = always.
 *   "dec_fused"    1 (default): hers_decrypt_scores in one kernel per block
 *                  where it fits (double-precision arithmetic, n = 4096,
 *                  three q primes), [c0 + c1 s]_q kept in registers; 0: the
 *                  product and the decoding as two kernels through the
 *                  workspace.  The same scores either way.
 *   "relin_lane_coeffs" coefficients per lane of the fused form, 8 (default:
 *                  n / 8 lanes, four waves per SIMD) or 16 (n / 16 lanes,
 *                  two waves per SIMD, the next digit's loads held in
 *                  registers); 8 applies where every q_i < 2^45 (the
 *                  double-precision form) and n <= 8192, else 16.
 *   "mb_variant"   multi-probe multiply-accumulate schedule of
 *                  hers_search_batch, 0..4; 0..3 as (probes per wave, dimensions
 *                  per staged chunk, blocks per item): 0 (1, 8, 4) in
 *                  1024-lane workgroups, 1 (2, 4, 2), 2 (2, 8, 2) in 512-lane
 *                  workgroups, 3 (4, 4, 1) in 256-lane workgroups.  More
 *                  probes per wave read each staged gallery word from LDS
 *                  once for all of them.  4: on the matrix cores -- the
 *                  residues as four balanced base-256 digits, the sums over
 *                  the dimensions as int8 matrix products per slot (MFMA),
 *                  recombined exactly mod p; for d <= 128 (a batch with a
 *                  larger d runs schedule 0).
 *   "mb_group"     most probes of one gallery grouped into one multi-probe
 *                  pass, 1..16 (default 16).
 * Every schedule computes the same bits.  Returns HERS_EINVAL for an unknown
 * key or value. */
int hers_set_option(hers_ctx* ctx, const char* key, int64_t value);

/* Autotuner: times every "mac_variant" schedule together with the inverse
 * NTT of the accumulators (which schedule 12 does itself) on the caller's
 * gallery and probe (reps launches each, over as many leading blocks as the
 * search workspace holds; another schedule replaces the current one only if
 * 3% faster), then the search epilogue's transforms under NTT pass radix 4,
 * 8 and 16, then -- when scores_dev (score cts [M][2][k][n]) is not NULL --
 * whole hers_search calls over "overlap_chunks" 1, 2, 4, ..., 64 (chunks of
 * at least 16 blocks) x "mac_wgs_per_cu" 0, 1, 2 x the schedule found first,
 * schedule 8, schedule 9, schedule 10 or schedule 12, and -- where the default
 * relinearization is the two-kernel form -- over chunk counts 1, 4, 16, 64 x
 * "mac_wgs_per_cu" 0, 1 with the relinearization fused ("relin_fuse_min_wgs"
 * 1) and the best schedule; the plain combination (no chunks, default grid,
 * schedule found first) and the four fastest others are then timed again in
 * turn, one search each over 2 reps rounds, and another than the plain one
 * must be 3% faster by those sums to be kept.  Keeps the fastest of each in
 * the context and returns the schedule in *chosen (may be NULL).  The
 * workspace and scores_dev contents are overwritten; the call synchronizes
 * `stream`. */
int hers_autotune(hers_ctx* ctx, const uint32_t* gallery_dev, uint64_t gallery_words, int64_t m, int32_t d,
                  const uint32_t* probe_dev, uint64_t probe_words, uint64_t* scores_dev, void* work_dev,
                  size_t work_bytes, int reps, void* stream, int64_t* chosen);
int hers_get_option(const hers_ctx* ctx, const char* key, int64_t* value);

/* ---- nearest neighbours (App. B, Alg. "HERS Search": argmax of the decrypted scores) ----
 * The k highest of scores_dev (int32 [m], as written by hers_decrypt_scores),
 * highest first; equal scores are ordered by lower item index.
 * idx_dev int64 [k], val_dev int32 [k]; 1 <= k <= 16384 (and k <= m),
 * m <= 2^32; workspace of hers_topk_workspace_bytes(m, k).  Up to k = 512
 * the k tiles of 4096 scores with the largest maxima are filtered and
 * sorted; above, the k-th largest (score, index) key is found by radix
 * select and the k keys at or above it are ranked. */
uint64_t hers_topk_workspace_bytes(int64_t m, int32_t k);
int hers_topk(hers_ctx* ctx, const int32_t* scores_dev, int64_t m, int32_t k, int64_t* idx_dev, int32_t* val_dev,
              void* work_dev, size_t work_bytes, void* stream);

/* ---- serving ---------------------------------------------------------------
 * A request loop over one context (the context then belongs to the server's
 * worker thread until hers_server_destroy).  Galleries (search form, caller
 * memory) and the evaluation key stay resident.  A query submitted with
 * hers_server_submit is, on the GPU, encrypted (hers_encrypt_probe with the
 * given seed), searched against its gallery and decrypted with sk_dev.
 *   Admission: every request needs probe + score ciphertexts +
 *   decrypted scores, and each wave a workspace, all carved from arena_dev
 *   (arena_bytes of device memory owned by the caller) by a first-fit
 *   allocator; a request that does not fit waits (counted in deferrals) until
 *   results are collected with hers_server_wait, which frees its memory.
 *   Batching: a wave is the oldest queued request and the later queued
 *   requests on the same gallery (up to max_batch, arrival order), which
 *   share one pass over the gallery; requests on other galleries form waves
 *   of their own, so a short search never waits for a long one in its wave.
 *   Up to four waves run at once, each on its own stream.  Each result is
 *   bit-identical to the same request served alone.
 * hers_server_add_gallery takes the gallery's search form and its length in
 * u32 words (whole blocks of d dimensions covering m items, else HERS_EDIM).
 * hers_server_submit copies the query (host int32 [d] of the gallery, every
 * value within +-feature_bound, else HERS_ERANGE) and returns a ticket, or
 * HERS_ENOMEM if one request alone exceeds the arena.
 * hers_server_wait blocks until the ticket's scores are ready, optionally
 * copies the decrypted scores (host int32 [m]) and the score ciphertexts
 * (host u64 [M][2][k][n]) out, reports the latency from submission to scores
 * ready on the GPU, and releases the ticket.  A worker short of arena
 * memory sleeps until a result is collected or a request arrives.
 * hers_server_destroy lets the waves on the GPU finish; requests still
 * queued are dropped.  Every hers_server_wait must have returned first. */
typedef struct hers_server hers_server;
typedef struct {
  int64_t submitted, completed, deferrals, waves, max_wave, queued, in_flight;
  uint64_t arena_peak;
  uint64_t gallery_bytes;   /* search-form bytes streamed: once per gallery group of a wave */
} hers_server_stats;
int hers_server_create(hers_ctx* ctx, const uint8_t* sk_dev, void* arena_dev, size_t arena_bytes,
                       int32_t max_batch, hers_server** out);
int hers_server_add_gallery(hers_server* srv, const uint32_t* gallery_dev, uint64_t gallery_words,
                            int64_t m, int32_t d, int32_t* gallery_id);
int hers_server_submit(hers_server* srv, int32_t gallery_id, const int32_t* query, uint64_t seed,
                       int64_t* ticket);
int hers_server_wait(hers_server* srv, int64_t ticket, int32_t* scores_out, uint64_t* ct_out,
                     double* latency_ms);
int hers_server_stats_get(hers_server* srv, hers_server_stats* out);
void hers_server_destroy(hers_server* srv);

/* ---- per-stage timing ---------------------------------------------------
 * While enabled, every kernel launch of the library is bracketed by HIP events
 * recorded on the stream it is launched on.  hers_profile_enable clears the
 * records.  hers_profile_read waits for the recorded events and returns the
 * summed duration (ms) and launch count of one stage: "mac" (the fused
 * multiply-accumulate), "mac_multi" (its batched form), "topk", "intt_acc", "rescale", "relin", "encrypt", "lift",
 * "ntt_fwd", "encode", "keygen", "sk_ntt", "dec_mul", "dec_decode". */
int hers_profile_enable(hers_ctx* ctx, int on);
/* Restricts the timing to the stages named in `stages`, a comma-separated
 * list of the names above (e.g. "mac"); NULL or "" times every stage.  Each
 * timed launch costs two event records on its stream, a few microseconds of
 * GPU time, so a caller timing a whole query times only the stage it needs. */
int hers_profile_select(hers_ctx* ctx, const char* stages);
int hers_profile_read(hers_ctx* ctx, const char* stage, double* total_ms, uint64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* HERS_H */
