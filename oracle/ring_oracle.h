/*
 * ring_oracle.h -- plain CPU model of the adaptive ring multiplication of
 * Sec. III-B: a product in GF(2)[X]/(X^n - 1) that takes the sparse path of
 * Eq. (1) (XOR of rotations of the dense operand by the support of the
 * other) when the first operand's Hamming weight is at most a threshold,
 * and otherwise a dense Karatsuba product followed by reduction mod X^n - 1.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; it shares no source with the GPU path.
 *
 * Dense path (the paper names Toom-Cook; this oracle uses its two-way case,
 * Karatsuba, over 64-bit words): operands zero-padded to 2^L * M words,
 * M = ceil(U / 2^L), L = hqco_ring_levels(U); a split at h words gives
 *   A = A0 + X^(64h) A1,  P0 = A0 B0,  P1 = A1 B1,  P2 = (A0 + A1)(B0 + B1),
 *   A B = P0 + X^(64h) (P0 + P1 + P2) + X^(128h) P1,
 * recursively down to M-word blocks multiplied bit by bit; then
 * r_t = c_t + c_(t+n) for t < n.
 *
 * Pins (tests/test_oracle_ring.py): both paths equal numpy's convolution of
 * the bit vectors mod 2 folded mod X^n - 1 (tiny n exhaustively, HQC sizes
 * at random); the threshold only selects the path.
 */
#ifndef HQC_RING_ORACLE_H
#define HQC_RING_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Karatsuba depth for a U-word operand: the smallest L >= 0 with
 * ceil(U / 2^L) <= 8 (leaf blocks of 5 to 8 words for the HQC sizes). */
int hqco_ring_levels(int uwords);
/* Dense path: out = a * b mod (X^n - 1); a, b, out: ceil(n/64) words, bits
 * >= n of a and b ignored, of out zero. */
void hqco_ring_mul_dense(int n, const uint64_t *a, const uint64_t *b, uint64_t *out);
/* Sparse path (Eq. (1)) on the support of a. */
void hqco_ring_mul_sparse(int n, const uint64_t *a, const uint64_t *b, uint64_t *out);
/* Adaptive: the sparse path iff weight(a) <= threshold; returns 0 (sparse)
 * or 1 (dense). */
int hqco_ring_mul(int n, const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t threshold);

#ifdef __cplusplus
}
#endif
#endif /* HQC_RING_ORACLE_H */
