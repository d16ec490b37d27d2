/* Host-side exercise of the seeded input generator (the product package's
 * csrc/hqc_synth.c) under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built and run by tests/test_sanitize.py).  For each parameter set and
 * thread counts 1, 3 and 16: keys, encryption randomness and decoder-stress
 * draws, checked for their documented structure (supports distinct and below
 * their bound, bits >= n of h clear, delta distinct bad blocks with nonzero
 * values, noise only in clean blocks and at most rho bits per block) and for
 * equality across thread counts; invalid sizes are refused.  Exit status 0
 * when every check holds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct synth_sizes {
  int32_t param_id;
  int32_t n, n1, n2, k, delta, w, wr, we;
  int32_t rho;
} synth_sizes_t;

int synth_keys(uint64_t master, const synth_sizes_t *sz, size_t count, uint64_t key_id0,
               uint64_t *h, uint32_t *x, uint32_t *y, int nthreads);
int synth_encryptions(uint64_t master, const synth_sizes_t *sz, size_t count,
                      const int64_t *key_of, uint64_t ct_id0, uint8_t *m, uint32_t *r1,
                      uint32_t *r2, uint32_t *e, int nthreads);
int synth_stress(uint64_t master, const synth_sizes_t *sz, size_t count, uint64_t word_id0,
                 uint8_t *m, uint32_t *bad, uint8_t *dval, uint64_t *noise, int nthreads);
void synth_fill_words(uint64_t seed, size_t nwords, uint64_t *out);
void synth_fixed_weight(uint64_t seed, uint32_t bound, int w, uint32_t *out);

static int fail(const char *what, int set) {
  printf("FAIL set %d: %s\n", set, what);
  return 1;
}

static int distinct_below(const uint32_t *a, int w, uint32_t bound) {
  for (int i = 0; i < w; ++i) {
    if (a[i] >= bound) return 0;
    for (int j = 0; j < i; ++j)
      if (a[i] == a[j]) return 0;
  }
  return 1;
}

static int popcount64(uint64_t x) {
  int c = 0;
  for (; x; x &= x - 1) ++c;
  return c;
}

static int check_set(const synth_sizes_t *sz) {
  const int set = sz->param_id;
  const size_t cnt = 37;
  const int nw = (sz->n + 63) / 64, vw = sz->n1 * sz->n2 / 64;
  const int threads[3] = {1, 3, 16};
  uint64_t *h[3];
  uint32_t *x[3], *y[3], *r1[3], *r2[3], *e[3], *bad[3];
  uint8_t *m[3], *sm[3], *dval[3];
  uint64_t *noise[3];
  int64_t key_of[37];
  for (size_t i = 0; i < cnt; ++i) key_of[i] = (int64_t)(i % 5);
  for (int t = 0; t < 3; ++t) {
    h[t] = malloc(cnt * nw * 8);
    x[t] = malloc(cnt * sz->w * 4);
    y[t] = malloc(cnt * sz->w * 4);
    m[t] = malloc(cnt * sz->k);
    r1[t] = malloc(cnt * sz->wr * 4);
    r2[t] = malloc(cnt * sz->wr * 4);
    e[t] = malloc(cnt * sz->we * 4);
    sm[t] = malloc(cnt * sz->k);
    bad[t] = malloc(cnt * sz->delta * 4);
    dval[t] = malloc(cnt * sz->delta);
    noise[t] = malloc(cnt * vw * 8);
    if (synth_keys(0x5A, sz, cnt, 7, h[t], x[t], y[t], threads[t])) return fail("keys rc", set);
    if (synth_encryptions(0x5B, sz, cnt, key_of, 3, m[t], r1[t], r2[t], e[t], threads[t]))
      return fail("encryptions rc", set);
    if (synth_stress(0x5C, sz, cnt, 11, sm[t], bad[t], dval[t], noise[t], threads[t]))
      return fail("stress rc", set);
  }
  for (int t = 1; t < 3; ++t) {
    if (memcmp(h[0], h[t], cnt * nw * 8) || memcmp(x[0], x[t], cnt * sz->w * 4) ||
        memcmp(y[0], y[t], cnt * sz->w * 4))
      return fail("keys differ across thread counts", set);
    if (memcmp(m[0], m[t], cnt * sz->k) || memcmp(r1[0], r1[t], cnt * sz->wr * 4) ||
        memcmp(r2[0], r2[t], cnt * sz->wr * 4) || memcmp(e[0], e[t], cnt * sz->we * 4))
      return fail("encryption draws differ across thread counts", set);
    if (memcmp(sm[0], sm[t], cnt * sz->k) || memcmp(bad[0], bad[t], cnt * sz->delta * 4) ||
        memcmp(dval[0], dval[t], cnt * sz->delta) || memcmp(noise[0], noise[t], cnt * vw * 8))
      return fail("stress draws differ across thread counts", set);
  }
  for (size_t i = 0; i < cnt; ++i) {
    if (sz->n % 64 && (h[0][i * nw + nw - 1] >> (sz->n % 64)) != 0) return fail("h bits >= n", set);
    if (!distinct_below(x[0] + i * sz->w, sz->w, (uint32_t)sz->n) ||
        !distinct_below(y[0] + i * sz->w, sz->w, (uint32_t)sz->n) ||
        !distinct_below(r1[0] + i * sz->wr, sz->wr, (uint32_t)sz->n) ||
        !distinct_below(r2[0] + i * sz->wr, sz->wr, (uint32_t)sz->n) ||
        !distinct_below(e[0] + i * sz->we, sz->we, (uint32_t)sz->n))
      return fail("support", set);
    const uint32_t *b = bad[0] + i * sz->delta;
    if (!distinct_below(b, sz->delta, (uint32_t)sz->n1)) return fail("bad blocks", set);
    for (int l = 0; l < sz->delta; ++l)
      if (dval[0][i * sz->delta + l] == 0) return fail("zero symbol error", set);
    const uint64_t *nz = noise[0] + i * vw;
    const int bw = sz->n2 / 64;
    for (int j = 0; j < sz->n1; ++j) {
      int is_bad = 0, wt = 0;
      for (int l = 0; l < sz->delta; ++l) is_bad |= b[l] == (uint32_t)j;
      for (int q = 0; q < bw; ++q) wt += popcount64(nz[j * bw + q]);
      if ((is_bad && wt) || wt > sz->rho) return fail("noise", set);
    }
  }
  /* sizes whose draws could not finish are refused */
  synth_sizes_t b = *sz;
  b.delta = b.n1 + 1;
  if (synth_stress(1, &b, 1, 0, sm[0], bad[0], dval[0], noise[0], 1) != -1)
    return fail("delta > n1 accepted", set);
  b = *sz;
  b.rho = b.n2 + 1;
  if (synth_stress(1, &b, 1, 0, sm[0], bad[0], dval[0], noise[0], 1) != -1)
    return fail("rho > n2 accepted", set);
  b = *sz;
  b.w = b.n + 1;
  if (synth_keys(1, &b, 1, 0, h[0], x[0], y[0], 1) != -1) return fail("w > n accepted", set);
  for (int t = 0; t < 3; ++t) {
    free(h[t]); free(x[t]); free(y[t]); free(m[t]); free(r1[t]); free(r2[t]); free(e[t]);
    free(sm[t]); free(bad[t]); free(dval[t]); free(noise[t]);
  }
  uint64_t words[5];
  synth_fill_words(3, 5, words);
  uint32_t fw[4];
  synth_fixed_weight(9, 4, 4, fw);  /* every index of a tiny bound */
  if (!distinct_below(fw, 4, 4)) return fail("fixed weight w = bound", set);
  printf("set %d ok\n", set);
  return 0;
}

int main(void) {
  const synth_sizes_t sets[3] = {
      {1, 17669, 46, 384, 16, 15, 66, 75, 75, 95},
      {3, 35851, 56, 640, 24, 16, 100, 114, 114, 159},
      {5, 57637, 90, 640, 32, 29, 131, 149, 149, 159},
  };
  int bad = 0;
  for (int i = 0; i < 3; ++i) bad |= check_set(&sets[i]);
  return bad;
}
