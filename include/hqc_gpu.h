/*
 * hqc_gpu.h -- C ABI of the gfx950 HQC decryption library (libhqc_gpu.so).
 *
 * What it computes: HQC.PKE.Decrypt (Alg. 2 of the OptHQC paper, arXiv
 * 2512.12904) in batches, with the secret key y:
 *     m = C.Decode(v + (u * y) restricted to its first n1*n2 bits)
 * where u * y is the product in GF(2)[X]/(X^n - 1) of Eq. (1), computed as
 * the XOR of the rotations of u by the support indices of y, and C.Decode
 * is the concatenated decoder of Sec. II-A: each of the n1 blocks of n2 bits
 * is decoded as a duplicated RM(1,7) codeword (maximum likelihood, by a
 * 128-point Walsh-Hadamard transform), then the n1 symbols are decoded as a
 * shortened Reed-Solomon codeword over GF(2^8) (syndromes, Berlekamp-Massey,
 * Chien search, Forney) and the k message bytes are returned.  Parameter
 * sets: Table I (HQC-1, HQC-3, HQC-5).
 *
 * Conventions (fixed so that every input, also one beyond the decoding
 * radius, has one defined output):
 *   - bit t of a polynomial is bit (t & 63) of 64-bit word (t >> 6);
 *   - u: ceil(n/64) words per item; bits >= n are ignored;
 *   - v: n1*n2/64 words per item (v is truncated to n1*n2 bits);
 *   - y: w uint32 support indices per item, read as the polynomial
 *     sum_k X^(y_k mod n) (repeated indices cancel);
 *   - RM block j of the received word is bits [j*n2, (j+1)*n2); copy q of
 *     the 128-bit RM(1,7) word sits at offset 128*q; byte b encodes as
 *     bit i = b7 ^ parity(b & i & 0x7F); the decoder takes the smallest
 *     index among equal-magnitude Hadamard peaks;
 *   - RS: narrow-sense (roots alpha^1..alpha^2delta, alpha = x, field
 *     polynomial x^8+x^4+x^3+x^2+1), parity symbols first, message byte t
 *     at symbol 2*delta + t; corrections are applied without a failure
 *     check (PKE decryption has no failure output).
 *   - m_out: k bytes per item.
 *
 * Memory: every array argument is DEVICE memory (hipMalloc'd or a torch
 * CUDA/HIP tensor), except y_host in hqc_keystore_put* and the hqc_params_t /
 * hqc_segment_t structs themselves, which are host memory read during the
 * call and not retained.  The caller owns all buffers.  u, v, r must be
 * 8-byte aligned, y, key_ids and m_out 4-byte aligned (m_out is written a
 * dword at a time).
 *
 * Execution: calls enqueue work on params->stream (a hipStream_t; NULL means
 * the null stream) and return; outputs are valid once that stream is
 * synchronised.  Kernels never branch on or index by secret data except
 * through data-independent primitives (see the library's design notes).
 *
 * Errors: every int-returning call returns HQC_OK or a negative code; on an
 * error detected before launch nothing is enqueued and nothing is written.
 * count == 0 is a successful no-op.  HQC_EHIP reports a HIP runtime error,
 * whose hipError_t is then available from hqc_last_hip_error().
 */
#ifndef HQC_GPU_H
#define HQC_GPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HQC_OK 0
#define HQC_EINVAL (-1)   /* bad pointer, alignment, parameter id, flags  */
#define HQC_ERANGE (-2)   /* count or key id beyond what the call supports */
#define HQC_EHIP (-3)     /* HIP runtime error (see hqc_last_hip_error)    */
#define HQC_ENOMEM (-4)   /* device or host allocation failed              */

/* params->flags */
#define HQC_F_PER_ITEM_LAUNCH 0x1u /* baseline: one kernel launch per item   */
#define HQC_F_GRAPH 0x2u           /* launch through a cached hipGraph        */

/* Largest count of one call (items are indexed with 32-bit integers). */
#define HQC_MAX_COUNT ((size_t)1 << 31)

/* Sizes of one parameter set (Table I plus derived word counts). */
typedef struct hqc_sizes {
  int32_t param_id; /* 1, 3 or 5 */
  int32_t n;        /* ring length */
  int32_t n1, k;    /* RS length and dimension (k = message bytes) */
  int32_t delta;    /* RS correction radius */
  int32_t n2;       /* duplicated RM length = 128 * mult */
  int32_t mult;     /* RM(1,7) copies per block */
  int32_t w;        /* weight of y */
  int32_t wr, we;   /* weights of r1, r2 and e (encryption side) */
  int32_t u_words;  /* uint64 words of u per item = ceil(n / 64) */
  int32_t v_words;  /* uint64 words of v (or r) per item = n1 * n2 / 64 */
} hqc_sizes_t;

/* Per-call launch options (host struct, read during the call only). */
typedef struct hqc_params {
  int32_t param_id; /* 1, 3 or 5; ignored by the *_mixed calls */
  uint32_t flags;   /* HQC_F_* */
  void *stream;     /* hipStream_t, or NULL for the null stream */
  int32_t grid;     /* persistent workgroups; 0 = chosen by the library */
  int32_t tile;     /* items per workgroup tile, 1..64; 0 = chosen by the library.
                       In a launch over several sets this is the HQC-1
                       tile, and the other sets' tiles are that divided by
                       their relative time per item (HQC-3 about 1.5-2x,
                       HQC-5 3-4x) and rounded to a power of two, but not
                       below min(tile, 4), so that the tiles take about as
                       long.  Results never depend on grid or tile. */
  int32_t shape;    /* kernel shape: 0 = chosen by the library, 1 = shape A, 2 =
                       shape B (single-set HQC-1 or HQC-3 decryption, decoding
                       and keyed decryption only; HQC_EINVAL elsewhere).
                       A: every set's default, two wavefronts per SIMD.
                       B: three wavefronts per SIMD, built for the smaller
                       register budget (HQC-3: with its received word over
                       the doubled u, for less LDS per wavefront).  Results
                       never depend on it. */
} hqc_params_t;

/* One homogeneous part of a mixed-parameter batch (host struct). */
typedef struct hqc_segment {
  int32_t param_id;        /* 1, 3 or 5 */
  int32_t reserved;        /* must be 0 */
  size_t count;            /* items in this segment */
  const uint64_t *u;       /* decrypt: count * u_words; decode: r, count * v_words */
  const uint64_t *v;       /* decrypt: count * v_words; decode: NULL */
  const uint32_t *y;       /* decrypt: count * w; decode: NULL;
                              hqc_decrypt_mixed_keyed: count key ids */
  uint8_t *m_out;          /* count * k bytes */
} hqc_segment_t;

typedef struct hqc_keystore hqc_keystore_t;

/* Fills *out for param_id 1, 3 or 5.  HQC_EINVAL for another id or NULL. */
int hqc_sizes(int param_id, hqc_sizes_t *out);

/* Alg. 2 on count items of one parameter set: m_out[i] = Decrypt(y[i],
 * (u[i], v[i])).  The whole batch is one persistent kernel launch (or one
 * hipGraph launch with HQC_F_GRAPH, or count launches with
 * HQC_F_PER_ITEM_LAUNCH).  Precondition (not checked on the device): the
 * arrays hold count items. */
int hqc_decrypt_batch(const hqc_params_t *params, const uint64_t *u,
                      const uint64_t *v, const uint32_t *y, uint8_t *m_out,
                      size_t count);

/* C.Decode only (Sec. II-A): m_out[i] = Decode(r[i]), r: count * v_words.
 * Equals hqc_decrypt_batch with u = 0. */
int hqc_decode_batch(const hqc_params_t *params, const uint64_t *r,
                     uint8_t *m_out, size_t count);

/* Mixed HQC-1/3/5 batches: up to 3 segments (at most one per parameter
 * set), processed by one persistent launch.  Results are identical to
 * per-segment hqc_decrypt_batch / hqc_decode_batch calls. */
int hqc_decrypt_mixed(const hqc_params_t *params, const hqc_segment_t *segs,
                      int nseg);
int hqc_decode_mixed(const hqc_params_t *params, const hqc_segment_t *segs,
                     int nseg);

/* Device-resident secret keys (the y of Alg. 3) for serving.  cap[i] is the
 * number of key slots for HQC-1, HQC-3, HQC-5 (i = 0, 1, 2).  Slots start
 * zero (an all-zero y).  The store owns its device memory until destroy. */
int hqc_keystore_create(hqc_keystore_t **ks, const size_t cap[3]);
/* Copies w indices from host memory into slot key_id; every index must be
 * < n and the indices distinct (HQC_EINVAL otherwise; HQC_ERANGE when
 * key_id >= capacity).  Synchronous. */
int hqc_keystore_put(hqc_keystore_t *ks, int param_id, uint32_t key_id,
                     const uint32_t *y_host);
/* The same for count consecutive slots from key_id0 (y_host: count * w). */
int hqc_keystore_put_many(hqc_keystore_t *ks, int param_id, uint32_t key_id0,
                          size_t count, const uint32_t *y_host);
int hqc_keystore_destroy(hqc_keystore_t *ks);
/* Items whose device key id was out of range since creation (they decrypt
 * to zero bytes).  Synchronous. */
int hqc_keystore_bad_ids(const hqc_keystore_t *ks, uint64_t *out);

/* hqc_decrypt_batch with y taken from the keystore: item i uses slot
 * key_ids[i] (device array of count uint32) of params->param_id. */
int hqc_decrypt_batch_keyed(const hqc_params_t *params, const hqc_keystore_t *ks,
                            const uint64_t *u, const uint64_t *v,
                            const uint32_t *key_ids, uint8_t *m_out, size_t count);

/* Mixed HQC-1/3/5 batch with keys from the keystore, as one persistent
 * launch (Alg. 2 per item; the serving loop's batches): up to 3 segments,
 * at most one per parameter set.  In each segment, y holds count uint32 key
 * ids (device, 4-byte aligned) into that set's slots instead of keys; u, v
 * and m_out are as for hqc_decrypt_mixed.  Out-of-range ids decrypt to zero
 * bytes and are counted as in hqc_decrypt_batch_keyed.  Results equal one
 * hqc_decrypt_batch_keyed call per segment.  HQC_EINVAL for a NULL keystore
 * or as hqc_decrypt_mixed. */
int hqc_decrypt_mixed_keyed(const hqc_params_t *params, const hqc_keystore_t *ks,
                            const hqc_segment_t *segs, int nseg);

/* Key generation, Alg. 3 (the randomness is an input): s[i] = x[i] + h[i]*y[i]
 * in GF(2)[X]/(X^n - 1).  h, s_out: count * u_words; x, y: count * w.
 * Indices are taken mod n; s_out bits >= n are zero. */
int hqc_keygen_batch(const hqc_params_t *params, const uint64_t *h, const uint32_t *x,
                     const uint32_t *y, uint64_t *s_out, size_t count);

/* Encryption, Alg. 1, with the public key (h[i], s[i]) of item i and the
 * randomness as input: u = r1 + h*r2, v = the first n1*n2 bits of
 * mG + s*r2 + e, mG the concatenated code of m (Sec. II-A).
 * h, s, u_out: count * u_words; m: count * k; r1, r2: count * wr;
 * e: count * we; v_out: count * v_words. */
int hqc_encrypt_batch(const hqc_params_t *params, const uint64_t *h, const uint64_t *s,
                      const uint8_t *m, const uint32_t *r1, const uint32_t *r2,
                      const uint32_t *e, uint64_t *u_out, uint64_t *v_out, size_t count);

/* The concatenated code of Sec. II-A (the mG of Alg. 1) with an optional
 * symbol-error pattern between the outer and the inner code:
 *     r_out[i] = the n1 duplicated RM(1,7) blocks of c + sym_err[i],
 *     c = the systematic RS codeword of m[i] (parity at symbols 0 .. 2 delta - 1,
 *         m[i][t] at symbol 2 delta + t),
 * i.e. C.Encode(m[i]) when sym_err is NULL.  A nonzero byte e at symbol j
 * replaces RM block j by the codeword of c_j + e, so that the block decodes
 * to a wrong symbol whatever noise within the RM radius is added: the
 * decoder-stress words are r_out plus such noise.  m: count * k bytes;
 * sym_err: NULL or count * n1 bytes; r_out: count * v_words words, 8-byte
 * aligned; all device memory.  params->flags must be 0. */
int hqc_code_encode_batch(const hqc_params_t *params, const uint8_t *m, const uint8_t *sym_err,
                          uint64_t *r_out, size_t count);

/* ---- KEM (Sec. II-A: the PKE wrapped by the HHK transform with implicit
 * rejection; domain-separated SHAKE256 for seed formation and key
 * derivation).  The paper does not fix the byte-level construction; this
 * library uses, per item:
 *   draws(m) = SHAKE256(m || 0x03) as little-endian 32-bit words: wr for r1,
 *              wr for r2, we for e, each turned into distinct positions by
 *              Floyd's sampling (p_i = i + floor(a_i (n - i) / 2^32), then
 *              for i = w-1 down to 0, p_i <- i if a later p_j equals it);
 *   Encaps:    (u, v) = Encrypt(pk, m; draws(m)),
 *              K = SHAKE256(m || u || v || 0x04)[0, 32);
 *   Decaps:    m' = Decrypt(y, (u, v)); ok = [Encrypt(pk, m'; draws(m'))
 *              equals (u, v) in every word, padding bits of u included];
 *              K = SHAKE256((ok ? m' : sigma) || u || v || 0x04)[0, 32),
 *              the choice a select, not a branch.
 * u and v enter the hash as their 64-bit words, little-endian.  Message m
 * and sigma (the secret k-byte string of sk, Alg. 3) are inputs: the caller
 * draws them.  Decapsulation has no error output for a bad ciphertext
 * (implicit rejection); keys are HQC_KEM_KEY_BYTES bytes per item.
 *
 * Buffers: h, s, u, v, m, sigma, key_out 8-byte aligned, y 4-byte aligned;
 * per item: h, s, u: u_words words; v: v_words; y: w indices; m, sigma: k
 * bytes; key_out: 32 bytes.  workspace: device memory of at least
 * hqc_kem_workspace_bytes(param_id, count) bytes, 8-byte aligned, owned by
 * the caller, overwritten by the call and free again once the stream has
 * passed it.  params->flags must be 0. */
#define HQC_KEM_KEY_BYTES 32
/* The KEM's fixed-weight sampling alone: for each item, 2 wr + we draws
 * (32-bit words; rows of 2 wr + we words) become the supports of r1, r2 and e
 * (rows of 2 wr + we indices in [0, n), each vector's indices distinct, in
 * index order i) by Floyd's sampling as above.  draws, supp_out 4-byte
 * aligned device memory; params->flags must be 0. */
int hqc_fixed_weight_batch(const hqc_params_t *params, const uint32_t *draws, uint32_t *supp_out,
                           size_t count);
/* Workspace size for count items of one parameter set (0 for a bad id). */
size_t hqc_kem_workspace_bytes(int param_id, size_t count);
int hqc_kem_encaps_batch(const hqc_params_t *params, const uint64_t *h, const uint64_t *s,
                         const uint8_t *m, uint64_t *u_out, uint64_t *v_out, uint8_t *key_out,
                         void *workspace, size_t workspace_bytes, size_t count);
int hqc_kem_decaps_batch(const hqc_params_t *params, const uint64_t *h, const uint64_t *s,
                         const uint32_t *y, const uint8_t *sigma, const uint64_t *u,
                         const uint64_t *v, uint8_t *key_out, void *workspace,
                         size_t workspace_bytes, size_t count);

/* ---- Allocation-free decapsulation ----------------------------------------
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * hqc_kem_decaps_batch with its workspace taken from a fixed array of
 * HQC_NOALLOC_SCRATCH_BYTES bytes that the library's code object holds on
 * every device it runs on, until the process ends.  The call allocates
 * nothing.  count is limited by that size: HQC_ERANGE unless
 * hqc_kem_workspace_bytes(param_id, count) <= HQC_NOALLOC_SCRATCH_BYTES
 * (69,041 HQC-1, 44,034 HQC-3 or 34,592 HQC-5 items).  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (on different streams, or from
 * different threads, before the earlier call's stream has passed it) race
 * and give undefined keys; calls ordered on one stream are safe.  Nothing
 * in the array needs to start at zero (every call writes what it reads).
 * Other arguments, errors and results as hqc_kem_decaps_batch. */
#define HQC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int hqc_kem_decaps_batch_noalloc(const hqc_params_t *params, const uint64_t *h,
                                 const uint64_t *s, const uint32_t *y, const uint8_t *sigma,
                                 const uint64_t *u, const uint64_t *v, uint8_t *key_out,
                                 size_t count);

/* ---- Adaptive ring multiplication (Sec. III-B, threshold-aware
 * scheduling): out[i] = a[i] * b[i] in GF(2)[X]/(X^n - 1) for dense n-bit
 * rows (u_words words each; bits >= n of a and b ignored, of out zero).
 * Item i takes the sparse path of Eq. (1) (XOR of rotations of b[i] by the
 * support of a[i]) when weight(a[i]) <= threshold and <= HQC_RING_SPARSE_MAX,
 * else the dense path (Karatsuba over 64-bit words, then reduction mod
 * X^n - 1).  Both give the same product.  path_out (nullable, count bytes):
 * 0 sparse, 1 dense.  The path depends on the weight of a and the sparse
 * path's timing on its support: for operands whose weight and support are
 * public (the PKE and KEM entry points take supports directly and run in
 * constant time).
 *
 * a, b, out 8-byte aligned.  workspace: device memory, 8-byte aligned, of at
 * least hqc_ring_workspace_bytes(param_id, count, 1) bytes; with
 * hqc_ring_workspace_bytes(param_id, count, count) bytes every dense item
 * is processed in one pass, with less in chunks.  params->flags must be 0;
 * params->grid sets the sparse kernel's persistent grid (0 = occupancy). */
#define HQC_RING_SPARSE_MAX 4096
size_t hqc_ring_workspace_bytes(int param_id, size_t count, size_t chunk_items);
/* The weight threshold calibrated for the parameter set (the measured
 * cross-over of the two paths on MI355X); 0 for a bad id. */
uint32_t hqc_ring_default_threshold(int param_id);
int hqc_ring_mul_batch(const hqc_params_t *params, const uint64_t *a, const uint64_t *b,
                       uint64_t *out, uint8_t *path_out, uint32_t threshold, void *workspace,
                       size_t workspace_bytes, size_t count);

/* ---- Intermediates (debugging and stage-by-stage parity) ---------------
 * Bytes of one item's record for hqc_decrypt_debug (0 for a bad id).  The
 * record holds, at increasing offsets: the received word v + (u*y) on its
 * first n1*n2 bits (4*n1*n2/32 bytes, little-endian dwords), the n1 RM
 * symbols, the syndromes S_1 .. S_2delta, the error locator Lambda
 * (2 delta + 1 coefficients, Lambda_0 = 1: Massey's error locator
 * exactly), and the error values at
 * the k message positions; then zero to three padding bytes. */
size_t hqc_debug_bytes(int param_id);
/* hqc_decrypt_batch that also writes each item's record to dbg_out (device,
 * count * hqc_debug_bytes(param_id) bytes, 4-byte aligned).  The same
 * kernels run; the records only add stores.  Messages are identical to
 * hqc_decrypt_batch's.  HQC_EINVAL as there, or for a bad dbg_out or the
 * per-item launch flag. */
int hqc_decrypt_debug(const hqc_params_t *params, const uint64_t *u, const uint64_t *v,
                      const uint32_t *y, uint8_t *m_out, uint8_t *dbg_out, size_t count);

/* Static text for an HQC_* code. */
const char *hqc_strerror(int code);
/* hipError_t of the last HQC_EHIP on this thread (0 if none). */
int hqc_last_hip_error(void);
/* Number of persistent workgroups the library would launch for param_id
 * (0 = mixed) on the current device; HQC_EINVAL / HQC_EHIP on error. */
int hqc_default_grid(int param_id);
/* Releases cached graphs.  Keystores stay valid. */
void hqc_shutdown(void);

/* ---- Launch-configuration autotuner ------------------------------------
 * The decryption kernels take three launch parameters that never change the
 * results: the kernel shape (params->shape: register budget and LDS layout
 * for two or three wavefronts per SIMD), the persistent grid (workgroups)
 * and the tile (ciphertexts per workgroup tile; a workgroup decodes the
 * Reed-Solomon words of consecutive tiles together, two lanes per word in
 * passes of up to 32 words, one lane per word in larger ones).  The library
 * keeps a table, per device, parameter set and batch-size bucket (the power
 * of two at or above count), of the configuration to use when a single-set
 * call leaves params->grid, params->tile and params->shape at 0.  Without an
 * entry such a call uses the library's built-in table (the autotuner's
 * choices on MI355X at each power-of-two batch from 2^8 to 2^20 items).
 * Other calls (mixed sets, decoding, some knobs given) get what the caller
 * left open by rule: shape B for single-set HQC-3 once count gives B's
 * occupancy grid 16 items per workgroup, else shape A; the occupancy grid
 * of the shape; and the largest power-of-two tile not above count / grid
 * (at most 64).  Because the kernels' time does not depend
 * on the data (constant time), configurations can be timed on random
 * inputs. */
typedef struct hqc_tune_report {
  int32_t param_id;
  int32_t tile, grid;            /* chosen configuration (now in the table) */
  float ms;                      /* its median launch time */
  int32_t heuristic_tile, heuristic_grid;
  float heuristic_ms;            /* median time of the built-in default */
  int32_t candidates;            /* configurations timed */
  int32_t identical;             /* 1: every configuration gave byte-identical messages */
  uint64_t count;
  int32_t shape;                 /* chosen shape (1 = A, 2 = B) */
  int32_t heuristic_shape;       /* the built-in default's shape */
} hqc_tune_report_t;

/* Times candidate (shape, tile, grid) triples of the decryption kernel for param_id
 * (1, 3 or 5) on count random ciphertexts (count in 1 .. 2^20): one untimed
 * launch each, whose messages must all be byte-identical, then reps rounds
 * that time every candidate once, in a freshly shuffled order per round
 * (each sample four back-to-back hipGraph launches behind two untimed
 * ones), on `stream` (NULL: null stream).  The candidate with the lowest
 * median per launch is stored in the table if it beats the built-in default
 * by more than 1 %, else the default is (nothing is
 * stored if any candidate's messages differed: out->identical = 0); *out
 * gets the choice and both medians.  Allocates and frees its own device buffers
 * (u, v, y, m: count * (8 u_words + 8 v_words + 4 w + k) bytes); blocks
 * until done.  HQC_EINVAL: bad id, count 0, reps < 1 or out NULL;
 * HQC_ERANGE: count > 2^20; HQC_ENOMEM / HQC_EHIP: allocation or HIP
 * failure (the table is then unchanged). */
int hqc_autotune_decrypt(int param_id, size_t count, int reps, void *stream,
                         hqc_tune_report_t *out);
/* Sets the table entry of count's bucket on the current device (tile 1..64,
 * grid >= 1, shape 1 (A) or 2 (B, HQC-1 and HQC-3 only)); tile = grid =
 * shape = 0 removes it.  HQC_EINVAL otherwise. */
int hqc_tune_set(int param_id, size_t count, int tile, int grid, int shape);
/* The entry used for a call of count items: *tile, *grid and *shape, or 0, 0
 * and 0 when there is none.  HQC_EINVAL for a bad id or NULL pointers. */
int hqc_tune_get(int param_id, size_t count, int *tile, int *grid, int *shape);
/* Empties the table (all devices). */
void hqc_tune_clear(void);
/* The launch that hqc_decrypt_batch(params, ..., count) makes on the current
 * device: *shape (1 = A, 2 = B), *tile (items per tile) and *grid (persistent
 * workgroups, at most the number of tiles) -- params' own values where set,
 * else the table's entry, else the built-in choice.  Launches nothing.
 * HQC_EINVAL: bad params or id, NULL pointers, count 0 or above
 * HQC_MAX_COUNT, or shape B for a set without it; HQC_EHIP: no device. */
int hqc_launch_config(const hqc_params_t *params, size_t count, int *shape, int *tile,
                      int *grid);

#ifdef __cplusplus
}
#endif
#endif /* HQC_GPU_H */
