/* Host-side exercise of the oracle's C code under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built and run by tests/test_sanitize.py with
 * gcc -fsanitize=address,undefined -fno-sanitize-recover=all).  For each
 * parameter set: key generation, encryption and decryption round trips,
 * decoding with symbol errors up to the radius and beyond it, the KEM
 * (encapsulation, decapsulation of honest and tampered ciphertexts), the
 * 128-point transform, and the ring multiplications.  Inputs are seeded
 * (SplitMix64); exit status 0 when every round trip holds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/hqc_oracle.h"
#include "../oracle/kem_oracle.h"
#include "../oracle/ring_oracle.h"

static uint64_t g_state = 0x5A17;

static uint64_t next64(void) {  /* SplitMix64 (Steele, Lea, Flood 2014) */
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* w distinct indices in [0, n) by rejection */
static void support(int n, int w, uint32_t *out) {
  for (int i = 0; i < w; ++i) {
    for (;;) {
      uint32_t c = (uint32_t)(next64() % (uint64_t)n);
      int seen = 0;
      for (int j = 0; j < i; ++j) seen |= out[j] == c;
      if (!seen) {
        out[i] = c;
        break;
      }
    }
  }
}

static void dense(int n, int nwords, uint64_t *out) {
  for (int i = 0; i < nwords; ++i) out[i] = next64();
  if (n % 64) out[nwords - 1] &= (1ull << (n % 64)) - 1ull;
}

#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      return 1;                                                     \
    }                                                               \
  } while (0)

static int run_set(int id) {
  hqco_param_t p;
  CHECK(hqco_param(id, &p) == 0);
  const int nw = p.nwords, vw = p.vwords, k = p.k;
  uint64_t *h = calloc((size_t)nw, 8), *s = calloc((size_t)nw, 8), *u = calloc((size_t)nw, 8);
  uint64_t *v = calloc((size_t)vw, 8), *r = calloc((size_t)vw, 8), *rr = calloc((size_t)nw, 8);
  uint32_t *x = calloc((size_t)p.w, 4), *y = calloc((size_t)p.w, 4);
  uint32_t *r1 = calloc((size_t)p.wr, 4), *r2 = calloc((size_t)p.wr, 4), *e = calloc((size_t)p.we, 4);
  uint8_t m[64], m2[64], sigma[64], key[32], key2[32], sym[256], c[256], cm[64];
  CHECK(h && s && u && v && r && rr && x && y && r1 && r2 && e);

  for (int it = 0; it < 3; ++it) {
    /* PKE round trip (Alg. 1-3) */
    dense(p.n, nw, h);
    support(p.n, p.w, x);
    support(p.n, p.w, y);
    hqco_keygen(id, h, x, y, s);
    for (int i = 0; i < k; ++i) m[i] = (uint8_t)next64();
    support(p.n, p.wr, r1);
    support(p.n, p.wr, r2);
    support(p.n, p.we, e);
    hqco_encrypt(id, h, s, m, r1, r2, e, u, v);
    hqco_decrypt(id, y, u, v, m2);
    CHECK(memcmp(m, m2, (size_t)k) == 0);

    /* decoding: a codeword with delta symbol errors (inside the radius),
     * then with 2 delta (beyond it: any output, no memory error) */
    hqco_code_encode(id, m, r);
    hqco_rs_trace_t tr;
    memcpy(v, r, (size_t)vw * 8);
    for (int j = 0; j < p.delta; ++j) {
      const int blk = (j * 7 + it) % p.n1, words = p.n2 / 64;
      for (int q = 0; q < words; ++q) v[blk * words + q] ^= next64();
    }
    hqco_code_decode(id, v, m2, sym, &tr);
    CHECK(memcmp(m, m2, (size_t)k) == 0);
    for (int j = 0; j < 2 * p.delta; ++j) {
      const int blk = (int)(next64() % (uint64_t)p.n1), words = p.n2 / 64;
      for (int q = 0; q < words; ++q) v[blk * words + q] ^= next64();
    }
    hqco_code_decode(id, v, m2, sym, &tr);

    /* Reed-Solomon alone: encode, delta errors at distinct positions, decode */
    hqco_rs_encode(p.n1, k, m, c);
    for (int j = 0; j < p.delta; ++j) c[(j * 3 + it) % p.n1] ^= (uint8_t)(1 + next64() % 255);
    hqco_rs_decode(p.n1, k, c, cm, &tr);
    CHECK(memcmp(cm, m, (size_t)k) == 0);

    /* KEM: honest and tampered ciphertexts */
    for (int i = 0; i < k; ++i) sigma[i] = (uint8_t)next64();
    hqco_kem_encaps(id, h, s, m, u, v, key);
    CHECK(hqco_kem_decaps(id, h, s, y, sigma, u, v, key2) == 1);
    CHECK(memcmp(key, key2, 32) == 0);
    v[vw - 1] ^= 1ull << 63;
    CHECK(hqco_kem_decaps(id, h, s, y, sigma, u, v, key2) == 0);

    /* ring multiplication, both paths and the dispatcher */
    dense(p.n, nw, u);
    hqco_ring_mul_dense(p.n, h, u, rr);
    hqco_ring_mul_sparse(p.n, h, u, s);
    CHECK(memcmp(rr, s, (size_t)nw * 8) == 0);
    CHECK(hqco_ring_mul(p.n, h, u, s, 4096) >= 0);
  }
  int32_t t[128], T[128];
  for (int i = 0; i < 128; ++i) t[i] = (int32_t)(next64() % 7) - 3;
  hqco_fht128(t, T);

  free(h); free(s); free(u); free(v); free(r); free(rr);
  free(x); free(y); free(r1); free(r2); free(e);
  return 0;
}

int main(void) {
  const int ids[3] = {1, 3, 5};
  for (int i = 0; i < 3; ++i) {
    if (run_set(ids[i]) != 0) return 1;
    printf("set %d ok\n", ids[i]);
  }
  return 0;
}
