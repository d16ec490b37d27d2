/*
 * kem_oracle.h -- plain CPU model of HQC.KEM encapsulation and decapsulation
 * (the HHK transform with implicit rejection that Sec. II-A describes around
 * the PKE), with SHAKE256 written from FIPS 202.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; it shares no source with the GPU path.
 *
 * The paper names the ingredients (domain-separated SHAKE-derived G, H and K
 * for seed formation and key derivation; Decaps decrypts, re-encrypts,
 * compares and rejects implicitly) but not their byte-level form, and the
 * specification is not available here.  The construction fixed below is
 * one reading of the paper; it is self-consistent, and its SHAKE256 agrees with
 * an independent implementation (Python's hashlib), but interoperability
 * with the official HQC byte strings is parity unpinned.
 *
 *   SHAKE256(M, d)  FIPS 202: Keccak-f[1600] (theta, rho, pi, chi, iota,
 *                   24 rounds), rate 136 bytes, M || 1111 then pad10*1.
 *   Z(m)            = SHAKE256(m || 0x03) read as little-endian 32-bit words
 *                     a_0, a_1, ...: wr words for r1, wr for r2, we for e.
 *   FixedWeight(n, w, a_0..a_{w-1}): p_i = i + floor(a_i (n - i) / 2^32);
 *                   then for i = w-1 down to 0, p_i <- i if p_i equals a
 *                   later p_j.  This is Floyd's sampling (Bentley & Floyd,
 *                   CACM 1987) with the positions reflected; every w-subset
 *                   is equally likely for uniform draws in [i, n), and the
 *                   loop has a fixed length.
 *   Encaps(pk; m)   (r1, r2, e) = FixedWeight on Z(m);
 *                   (u, v) = PKE.Encrypt(pk, m; r1, r2, e)      (Alg. 1)
 *                   K = first 32 bytes of SHAKE256(m || u || v || 0x04),
 *                   u and v as their 64-bit words, little-endian.
 *   Decaps(sk, pk, (u, v))
 *                   m' = PKE.Decrypt(y, (u, v))                  (Alg. 2)
 *                   (u', v') = Encrypt(pk, m'; FixedWeight on Z(m'))
 *                   ok = [u' == u and v' == v] over every word (bits >= n of
 *                   u included, so a nonzero padding bit rejects)
 *                   K = first 32 bytes of SHAKE256((ok ? m' : sigma) || u ||
 *                   v || 0x04); sigma is the k-byte secret of sk (Alg. 3).
 */
#ifndef HQC_KEM_ORACLE_H
#define HQC_KEM_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HQCO_KEM_KEY_BYTES 32

/* Keccak-f[1600] on 25 lanes, lane x + 5y = A[x, y] (FIPS 202, Sec. 3). */
void hqco_keccak_f1600(uint64_t A[25]);
/* SHAKE256(in, 8 * outlen) (FIPS 202, Sec. 6.2). */
void hqco_shake256(const uint8_t *in, size_t inlen, uint8_t *out, size_t outlen);
/* Floyd's fixed-weight sampling as above: w draws a[0..w) -> w distinct
 * indices in [0, n), in index order i. */
void hqco_fixed_weight(int n, int w, const uint32_t *a, uint32_t *supp);
/* The 2 wr + we words of Z(m) for parameter set id. */
void hqco_kem_seed_words(int id, const uint8_t *m, uint32_t *words);
/* Encaps; u: nwords, v: vwords, key: 32 bytes. */
void hqco_kem_encaps(int id, const uint64_t *h, const uint64_t *s, const uint8_t *m,
                     uint64_t *u, uint64_t *v, uint8_t *key);
/* Decaps; returns ok (1 = the re-encryption matched, 0 = rejected). */
int hqco_kem_decaps(int id, const uint64_t *h, const uint64_t *s, const uint32_t *y,
                    const uint8_t *sigma, const uint64_t *u, const uint64_t *v,
                    uint8_t *key);

/* Batches, threads across items only; item i uses row i of every array.
 * Return 0, or -1 for a bad parameter id.  ok may be NULL. */
int hqco_kem_encaps_batch(int id, size_t count, const uint64_t *h, const uint64_t *s,
                          const uint8_t *m, uint64_t *u, uint64_t *v, uint8_t *key,
                          int nthreads);
int hqco_kem_decaps_batch(int id, size_t count, const uint64_t *h, const uint64_t *s,
                          const uint32_t *y, const uint8_t *sigma, const uint64_t *u,
                          const uint64_t *v, uint8_t *key, int32_t *ok, int nthreads);

#ifdef __cplusplus
}
#endif
#endif /* HQC_KEM_ORACLE_H */
