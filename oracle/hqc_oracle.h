/*
 * hqc_oracle.h -- plain CPU model of HQC.PKE (KeyGen, Encrypt, Decrypt) and of
 * the concatenated code it decodes with.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code.  It exists so that tests, the smoke check and the CPU
 * baseline timing can compare the GPU path against an independent, slow,
 * obviously correct implementation.  It shares no source with the GPU path.
 *
 * Paper: "OptHQC: Optimize HQC for High-Performance Post-Quantum
 * Cryptography" (Dong, Feng, Wang; arXiv 2512.12904).
 *   - parameter sets: Table I
 *   - ring product in GF(2)[X]/(X^N - 1): Eq. (1), Sec. III-B
 *   - PKE.Encrypt / PKE.Decrypt / KEM.KeyGen: Alg. 1, Alg. 2, Alg. 3, Sec. II-A
 *   - concatenated code (shortened Reed-Solomon outer, duplicated Reed-Muller
 *     inner): Sec. II-A and Sec. III-A
 *   - Reed-Solomon over GF(2^8), syndromes: Sec. III-D
 * The paper does not spell out the decoders; the readings used here (RM(1,7)
 * maximum-likelihood decoding by Walsh-Hadamard transform, Berlekamp-Massey,
 * Chien search, Forney) are textbook algorithms and every convention is
 * stated next to the function that fixes it.
 *
 * Parity status of each function (what pins it, checked by tests marked
 * "not gpu"):
 *   hqco_gf_*          field axioms, primitive-element order, brute force
 *   hqco_mul_sparse    schoolbook product mod X^n - 1 (numpy), identities
 *   hqco_fht128        brute-force correlation, Parseval, H*H = 128 I
 *   hqco_rm_*          Table I minimum distances, brute-force nearest codeword
 *   hqco_rs_*          g(alpha^i) = 0, zero syndromes of codewords, exact
 *                      recovery within the radius, brute force on a tiny code,
 *                      the Sec. III-D multiplication count
 *   hqco_pke_*         Decrypt(Encrypt(m)) = m (ground truth m)
 *   beyond-radius decoder output (more than delta symbol errors, RM ties):
 *                      parity unpinned -- fixed only by the conventions below
 *
 * All buffers are caller-owned.  Bit t of a polynomial is bit (t & 63) of
 * 64-bit word (t >> 6).  Functions never fail on well-formed sizes; the
 * batch helpers return 0 on success and -1 on a bad parameter id.
 */
#ifndef HQC_ORACLE_H
#define HQC_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hqco_param {
  int32_t id;        /* 1, 3 or 5 (HQC-1, HQC-3, HQC-5) */
  int32_t n;         /* ring length N */
  int32_t n1;        /* RS length */
  int32_t k;         /* RS dimension = message bytes */
  int32_t rs_d;      /* RS minimum distance (Table I) */
  int32_t delta;     /* RS correction radius (rs_d - 1) / 2 */
  int32_t n2;        /* duplicated RM length */
  int32_t rm_d;      /* duplicated RM minimum distance (Table I) */
  int32_t mult;      /* RM(1,7) copies per block = n2 / 128 */
  int32_t w;         /* weight of x and y */
  int32_t wr;        /* weight of r1 and r2 */
  int32_t we;        /* weight of e */
  int32_t nwords;    /* 64-bit words of an n-bit polynomial: ceil(n / 64) */
  int32_t vwords;    /* 64-bit words of a codeword: n1 * n2 / 64 */
} hqco_param_t;

/* Table I.  Returns 0, or -1 for an unknown id. */
int hqco_param(int id, hqco_param_t *out);

/* ---- GF(2^8), modulus x^8 + x^4 + x^3 + x^2 + 1 ---------------------- */
uint8_t hqco_gf_mul(uint8_t a, uint8_t b);      /* carry-less product, reduced */
uint8_t hqco_gf_pow(uint8_t a, uint32_t e);     /* a^e, 0^0 = 1 */
uint8_t hqco_gf_inv(uint8_t a);                 /* a^254; inv(0) = 0 */
/* exp[i] = alpha^i (i < 255) and log[alpha^i] = i, alpha = 0x02; log[0] = 0 */
void hqco_gf_tables(uint8_t exp_out[255], uint8_t log_out[256]);

/* ---- ring product, Eq. (1) ------------------------------------------ */
/* out = (sum over k of X^(supp[k] mod n)) * a  mod (X^n - 1).
 * a: ceil(n/64) words; bits >= n of a are ignored.  supp: w indices
 * (a multiset: repeated indices cancel).  out: ceil(n/64) words. */
void hqco_mul_sparse(int n, const uint64_t *a, const uint32_t *supp, int w,
                     uint64_t *out);

/* ---- duplicated RM(1,7) ------------------------------------------------ */
/* Codeword of byte b: bit i (0..127) = b7 ^ XOR_l (b_l & i_l), l = 0..6,
 * repeated mult times: copy q occupies bits 128q .. 128q+127 of out. */
void hqco_rm_encode(int mult, uint8_t b, uint64_t *out /* 2*mult words */);
/* Natural-order Walsh-Hadamard transform:
 * out[u] = sum_i in[i] * (-1)^popcount(u & i). */
void hqco_fht128(const int32_t in[128], int32_t out[128]);
/* Maximum-likelihood decode of one block of 128*mult bits: with
 * t_i = mult - 2 * (number of copies whose bit i is set), T = FHT(t),
 * u* = the smallest u maximising |T(u)|, result = u* | 128 * [T(u*) < 0].
 * T_out (nullable) receives T. */
uint8_t hqco_rm_decode(int mult, const uint64_t *blk, int32_t *T_out);

/* ---- shortened narrow-sense Reed-Solomon over GF(2^8) ------------------- */
/* Generator g(x) = prod_{i=1}^{2d} (x - alpha^i), two_delta + 1 coefficients,
 * g[i] the coefficient of x^i (monic). */
void hqco_rs_generator(int two_delta, uint8_t *g);
/* Systematic encoding: c(x) = x^(2d) m(x) + (x^(2d) m(x) mod g(x)),
 * i.e. parity in c[0 .. 2d), m[t] at c[2d + t].  2d = n1 - k. */
void hqco_rs_encode(int n1, int k, const uint8_t *m, uint8_t *c);
/* S[i-1] = c(alpha^i), i = 1 .. 2d. */
void hqco_rs_syndromes(int n1, int two_delta, const uint8_t *c, uint8_t *S);
/* Berlekamp-Massey (Massey 1969) from S_1..S_2d; lambda gets 2d+1
 * coefficients; returns L. */
int hqco_rs_berlekamp_massey(int two_delta, const uint8_t *S, uint8_t *lambda);

typedef struct hqco_rs_trace {
  uint8_t S[64];        /* syndromes S_1 .. S_2d */
  uint8_t lambda[65];   /* error locator, 2d + 1 coefficients */
  int32_t L;            /* BM register length */
  uint8_t omega[64];    /* error evaluator, 2d coefficients */
  uint8_t located[256]; /* 1 where lambda(alpha^-j) = 0, j < n1 */
  uint8_t err[256];     /* Forney error values e_j, j < n1 */
} hqco_rs_trace_t;
/* Full decode: syndromes, BM, Chien, Forney, correct, extract m (k bytes).
 * No failure detection: the corrections are applied whatever L is. */
void hqco_rs_decode(int n1, int k, const uint8_t *c, uint8_t *m,
                    hqco_rs_trace_t *trace /* nullable */);

/* ---- concatenated code ------------------------------------------------- */
/* RS symbol j occupies bits [j*n2, (j+1)*n2) as its duplicated RM codeword. */
void hqco_code_encode(int id, const uint8_t *m, uint64_t *cw /* vwords */);
/* symbols_out (nullable, n1 bytes), trace (nullable). */
void hqco_code_decode(int id, const uint64_t *r /* vwords */, uint8_t *m,
                      uint8_t *symbols_out, hqco_rs_trace_t *trace);

/* ---- HQC.PKE, Alg. 1-3 --------------------------------------------------- */
/* s = x + h*y (Alg. 3).  h, s: nwords; x, y: w indices each. */
void hqco_keygen(int id, const uint64_t *h, const uint32_t *x,
                 const uint32_t *y, uint64_t *s);
/* u = r1 + h*r2; v = first n1*n2 bits of (mG + s*r2 + e)  (Alg. 1).
 * r1, r2: wr indices; e: we indices; u: nwords; v: vwords. */
void hqco_encrypt(int id, const uint64_t *h, const uint64_t *s,
                  const uint8_t *m, const uint32_t *r1, const uint32_t *r2,
                  const uint32_t *e, uint64_t *u, uint64_t *v);
/* m = C.Decode(v + (u*y) restricted to [0, n1*n2))  (Alg. 2, secret y). */
void hqco_decrypt(int id, const uint32_t *y, const uint64_t *u,
                  const uint64_t *v, uint8_t *m);

/* ---- decoder stress words ----------------------------------------------- */
/* r = C.Encode(m); block bad[l] (l < nbad) is XORed with the duplicated RM
 * codeword of dval[l]; then the random noise vector (vwords words, drawn by
 * the caller) is XORed in.  r may alias noise. */
void hqco_stress_word(int id, const uint8_t *m, int nbad, const uint32_t *bad,
                      const uint8_t *dval, const uint64_t *noise, uint64_t *r);

/* ---- batch helpers (threads across items only) -------------------------- */
int hqco_keygen_batch(int id, size_t count, const uint64_t *h,
                      const uint32_t *x, const uint32_t *y, uint64_t *s,
                      int nthreads);
/* key_of[i] (nullable) selects the key row of item i (else row i). */
int hqco_encrypt_batch(int id, size_t count, const uint64_t *h,
                       const uint64_t *s, const int64_t *key_of,
                       const uint8_t *m, const uint32_t *r1,
                       const uint32_t *r2, const uint32_t *e, uint64_t *u,
                       uint64_t *v, int nthreads);
int hqco_decrypt_batch(int id, size_t count, const uint32_t *y,
                       const int64_t *key_of, const uint64_t *u,
                       const uint64_t *v, uint8_t *m, int nthreads);
int hqco_decode_batch(int id, size_t count, const uint64_t *r, uint8_t *m,
                      int nthreads);
/* Stress words in bulk: item i uses m + i*k, bad + i*delta, dval + i*delta,
 * noise + i*vwords and writes r + i*vwords (r may alias noise). */
int hqco_stress_batch(int id, size_t count, const uint8_t *m, const uint32_t *bad,
                      const uint8_t *dval, const uint64_t *noise, uint64_t *r,
                      int nthreads);

#ifdef __cplusplus
}
#endif
#endif /* HQC_ORACLE_H */
