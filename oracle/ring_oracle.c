/*
 * ring_oracle.c -- plain CPU model of the adaptive ring multiplication
 * (Sec. III-B).  TEST INFRASTRUCTURE ONLY; see ring_oracle.h.
 */
#include "ring_oracle.h"

#include <stdlib.h>
#include <string.h>

#include "hqc_oracle.h"

int hqco_ring_levels(int uwords) {
  int L = 0;
  while ((uwords + (1 << L) - 1) >> L > 8) L++;
  return L;
}

static int bit(const uint64_t *a, long t) { return (int)((a[t >> 6] >> (t & 63)) & 1u); }
static void flip(uint64_t *a, long t) { a[t >> 6] ^= (uint64_t)1 << (t & 63); }

/* c (2m words) = a * b, a and b m words: for every set bit i of a, add b
 * shifted up by i bits */
static void block_mul(const uint64_t *a, const uint64_t *b, int m, uint64_t *c) {
  memset(c, 0, sizeof(uint64_t) * 2 * (size_t)m);
  for (long i = 0; i < 64L * m; i++) {
    if (!bit(a, i)) continue;
    const long s = i / 64;
    const int r = (int)(i % 64);
    for (int j = 0; j < m; j++) {
      c[s + j] ^= b[j] << r;
      if (r) c[s + j + 1] ^= b[j] >> (64 - r);
    }
  }
}

/* c (2w words) = a * b by Karatsuba, a and b w words, w = 2^l * leaf */
static void karatsuba(const uint64_t *a, const uint64_t *b, int w, int leaf, uint64_t *c) {
  if (w <= leaf) {
    block_mul(a, b, w, c);
    return;
  }
  const int h = w / 2;
  uint64_t *p0 = calloc((size_t)2 * h, 8), *p1 = calloc((size_t)2 * h, 8),
           *p2 = calloc((size_t)2 * h, 8), *sa = calloc((size_t)h, 8), *sb = calloc((size_t)h, 8);
  for (int i = 0; i < h; i++) {
    sa[i] = a[i] ^ a[h + i];
    sb[i] = b[i] ^ b[h + i];
  }
  karatsuba(a, b, h, leaf, p0);
  karatsuba(a + h, b + h, h, leaf, p1);
  karatsuba(sa, sb, h, leaf, p2);
  memset(c, 0, sizeof(uint64_t) * 2 * (size_t)w);
  for (int i = 0; i < 2 * h; i++) {
    c[i] ^= p0[i];
    c[h + i] ^= p0[i] ^ p1[i] ^ p2[i];
    c[2 * h + i] ^= p1[i];
  }
  free(p0);
  free(p1);
  free(p2);
  free(sa);
  free(sb);
}

void hqco_ring_mul_dense(int n, const uint64_t *a, const uint64_t *b, uint64_t *out) {
  const int U = (n + 63) / 64, L = hqco_ring_levels(U);
  const int M = (U + (1 << L) - 1) >> L, W = M << L;
  uint64_t *pa = calloc((size_t)W, 8), *pb = calloc((size_t)W, 8), *c = calloc((size_t)2 * W, 8);
  for (long t = 0; t < n; t++) {
    if (bit(a, t)) flip(pa, t);
    if (bit(b, t)) flip(pb, t);
  }
  karatsuba(pa, pb, W, M, c);
  memset(out, 0, sizeof(uint64_t) * (size_t)U);
  for (long t = 0; t < n; t++)
    if (bit(c, t) ^ bit(c, t + n)) flip(out, t);
  free(pa);
  free(pb);
  free(c);
}

void hqco_ring_mul_sparse(int n, const uint64_t *a, const uint64_t *b, uint64_t *out) {
  uint32_t *supp = malloc(sizeof(uint32_t) * (size_t)n);
  int w = 0;
  for (long t = 0; t < n; t++)
    if (bit(a, t)) supp[w++] = (uint32_t)t;
  hqco_mul_sparse(n, b, supp, w, out);
  free(supp);
}

int hqco_ring_mul(int n, const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t threshold) {
  uint32_t w = 0;
  for (long t = 0; t < n; t++) w += (uint32_t)bit(a, t);
  if (w <= threshold) {
    hqco_ring_mul_sparse(n, a, b, out);
    return 0;
  }
  hqco_ring_mul_dense(n, a, b, out);
  return 1;
}
