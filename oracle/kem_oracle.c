/*
 * kem_oracle.c -- plain CPU model of the KEM around HQC.PKE and of SHAKE256.
 * TEST INFRASTRUCTURE ONLY; see kem_oracle.h for the construction and what
 * pins each function.
 */
#include "kem_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#include "hqc_oracle.h"

/* ---- Keccak-f[1600], FIPS 202 Sec. 3.2 ------------------------------------ */

static uint64_t rotl64(uint64_t x, unsigned r) {
  r &= 63u;
  return r ? (x << r) | (x >> (64u - r)) : x;
}

/* rc(t), FIPS 202 Algorithm 5: an LFSR over GF(2) read one bit per step.
 * R[i] is bit i of the integer R. */
static int rc_bit(int t) {
  if (t % 255 == 0) return 1;
  unsigned R = 1u; /* "10000000": R[0] = 1 */
  for (int i = 1; i <= t % 255; i++) {
    R <<= 1;                       /* R = 0 || R */
    unsigned b8 = (R >> 8) & 1u;   /* R[8] */
    R ^= b8 | b8 << 4 | b8 << 5 | b8 << 6;
    R &= 0xFFu;                    /* Trunc8 */
  }
  return (int)(R & 1u);
}

static uint64_t round_constant(int ir) {
  uint64_t rc = 0;
  for (int j = 0; j <= 6; j++)
    if (rc_bit(j + 7 * ir)) rc |= (uint64_t)1 << ((1u << j) - 1u);
  return rc;
}

void hqco_keccak_f1600(uint64_t A[25]) {
#define L(x, y) A[(x) + 5 * (y)]
  for (int ir = 0; ir < 24; ir++) {
    /* theta */
    uint64_t C[5], D[5];
    for (int x = 0; x < 5; x++) C[x] = L(x, 0) ^ L(x, 1) ^ L(x, 2) ^ L(x, 3) ^ L(x, 4);
    for (int x = 0; x < 5; x++) D[x] = C[(x + 4) % 5] ^ rotl64(C[(x + 1) % 5], 1);
    for (int y = 0; y < 5; y++)
      for (int x = 0; x < 5; x++) L(x, y) ^= D[x];
    /* rho: offsets (t + 1)(t + 2) / 2 along the walk (x, y) <- (y, 2x + 3y) */
    {
      int x = 1, y = 0;
      for (int t = 0; t < 24; t++) {
        L(x, y) = rotl64(L(x, y), (unsigned)(((t + 1) * (t + 2) / 2) % 64));
        int nx = y, ny = (2 * x + 3 * y) % 5;
        x = nx;
        y = ny;
      }
    }
    /* pi: A'[x, y] = A[x + 3y, x] */
    uint64_t B[25];
    for (int y = 0; y < 5; y++)
      for (int x = 0; x < 5; x++) B[x + 5 * y] = L((x + 3 * y) % 5, x);
    /* chi */
    for (int y = 0; y < 5; y++)
      for (int x = 0; x < 5; x++)
        L(x, y) = B[x + 5 * y] ^ (~B[(x + 1) % 5 + 5 * y] & B[(x + 2) % 5 + 5 * y]);
    /* iota */
    L(0, 0) ^= round_constant(ir);
  }
#undef L
}

/* ---- SHAKE256, FIPS 202 Sec. 6.2 and 4 -------------------------------------- */

#define RATE 136

void hqco_shake256(const uint8_t *in, size_t inlen, uint8_t *out, size_t outlen) {
  uint64_t A[25];
  memset(A, 0, sizeof A);
  /* padded input: in || 0x1F || 0 ... || 0x80 (the last byte ORed), whole blocks */
  size_t blocks = inlen / RATE + 1;
  for (size_t b = 0; b < blocks; b++) {
    uint8_t blk[RATE];
    memset(blk, 0, RATE);
    size_t off = b * RATE;
    size_t take = off < inlen ? (inlen - off < RATE ? inlen - off : RATE) : 0;
    memcpy(blk, in + off, take);
    if (b == blocks - 1) {
      blk[inlen - off] ^= 0x1F;
      blk[RATE - 1] ^= 0x80;
    }
    for (int i = 0; i < RATE; i++) A[i / 8] ^= (uint64_t)blk[i] << (8 * (i % 8));
    hqco_keccak_f1600(A);
  }
  size_t done = 0;
  for (;;) {
    for (int i = 0; i < RATE && done < outlen; i++, done++)
      out[done] = (uint8_t)(A[i / 8] >> (8 * (i % 8)));
    if (done == outlen) break;
    hqco_keccak_f1600(A);
  }
}

/* ---- fixed-weight sampling (Floyd) ------------------------------------------ */

void hqco_fixed_weight(int n, int w, const uint32_t *a, uint32_t *supp) {
  for (int i = 0; i < w; i++)
    supp[i] = (uint32_t)i + (uint32_t)(((uint64_t)a[i] * (uint64_t)(n - i)) >> 32);
  for (int i = w - 1; i >= 0; i--) {
    int dup = 0;
    for (int j = i + 1; j < w; j++) dup |= supp[j] == supp[i];
    if (dup) supp[i] = (uint32_t)i;
  }
}

/* ---- the KEM ------------------------------------------------------------------ */

void hqco_kem_seed_words(int id, const uint8_t *m, uint32_t *words) {
  hqco_param_t p;
  if (hqco_param(id, &p)) return;
  uint8_t in[65];
  memcpy(in, m, (size_t)p.k);
  in[p.k] = 0x03;
  size_t nw = (size_t)(2 * p.wr + p.we);
  uint8_t *buf = malloc(4 * nw);
  hqco_shake256(in, (size_t)p.k + 1, buf, 4 * nw);
  for (size_t i = 0; i < nw; i++)
    words[i] = (uint32_t)buf[4 * i] | (uint32_t)buf[4 * i + 1] << 8 |
               (uint32_t)buf[4 * i + 2] << 16 | (uint32_t)buf[4 * i + 3] << 24;
  free(buf);
}

static void encrypt_from_m(const hqco_param_t *p, const uint64_t *h, const uint64_t *s,
                           const uint8_t *m, uint64_t *u, uint64_t *v) {
  size_t nw = (size_t)(2 * p->wr + p->we);
  uint32_t *a = malloc(4 * nw), *supp = malloc(4 * nw);
  hqco_kem_seed_words(p->id, m, a);
  hqco_fixed_weight(p->n, p->wr, a, supp);
  hqco_fixed_weight(p->n, p->wr, a + p->wr, supp + p->wr);
  hqco_fixed_weight(p->n, p->we, a + 2 * p->wr, supp + 2 * p->wr);
  hqco_encrypt(p->id, h, s, m, supp, supp + p->wr, supp + 2 * p->wr, u, v);
  free(a);
  free(supp);
}

/* first 32 bytes of SHAKE256(prefix || u || v || 0x04) */
static void derive_key(const hqco_param_t *p, const uint8_t *prefix, const uint64_t *u,
                       const uint64_t *v, uint8_t *key) {
  size_t len = (size_t)p->k + 8 * (size_t)p->nwords + 8 * (size_t)p->vwords + 1;
  uint8_t *in = malloc(len), *q = in;
  memcpy(q, prefix, (size_t)p->k);
  q += p->k;
  for (int i = 0; i < p->nwords; i++)
    for (int b = 0; b < 8; b++) *q++ = (uint8_t)(u[i] >> (8 * b));
  for (int i = 0; i < p->vwords; i++)
    for (int b = 0; b < 8; b++) *q++ = (uint8_t)(v[i] >> (8 * b));
  *q = 0x04;
  hqco_shake256(in, len, key, HQCO_KEM_KEY_BYTES);
  free(in);
}

void hqco_kem_encaps(int id, const uint64_t *h, const uint64_t *s, const uint8_t *m,
                     uint64_t *u, uint64_t *v, uint8_t *key) {
  hqco_param_t p;
  if (hqco_param(id, &p)) return;
  encrypt_from_m(&p, h, s, m, u, v);
  derive_key(&p, m, u, v, key);
}

int hqco_kem_decaps(int id, const uint64_t *h, const uint64_t *s, const uint32_t *y,
                    const uint8_t *sigma, const uint64_t *u, const uint64_t *v,
                    uint8_t *key) {
  hqco_param_t p;
  if (hqco_param(id, &p)) return 0;
  uint8_t m[64];
  hqco_decrypt(id, y, u, v, m);
  uint64_t *u2 = malloc(8 * (size_t)p.nwords), *v2 = malloc(8 * (size_t)p.vwords);
  encrypt_from_m(&p, h, s, m, u2, v2);
  int ok = memcmp(u, u2, 8 * (size_t)p.nwords) == 0 && memcmp(v, v2, 8 * (size_t)p.vwords) == 0;
  derive_key(&p, ok ? m : sigma, u, v, key);
  free(u2);
  free(v2);
  return ok;
}

/* ---- batches ------------------------------------------------------------------ */

typedef struct kjob {
  int id, decaps;
  size_t lo, hi;
  const uint64_t *h, *s, *u_in, *v_in;
  const uint32_t *y;
  const uint8_t *m, *sigma;
  uint64_t *u, *v;
  uint8_t *key;
  int32_t *ok;
} kjob_t;

static void *run_kjob(void *arg) {
  kjob_t *j = arg;
  hqco_param_t p;
  hqco_param(j->id, &p);
  const size_t U = (size_t)p.nwords, V = (size_t)p.vwords, K = (size_t)p.k;
  for (size_t i = j->lo; i < j->hi; i++) {
    if (j->decaps) {
      int ok = hqco_kem_decaps(j->id, j->h + i * U, j->s + i * U, j->y + i * (size_t)p.w,
                               j->sigma + i * K, j->u_in + i * U, j->v_in + i * V,
                               j->key + i * HQCO_KEM_KEY_BYTES);
      if (j->ok) j->ok[i] = ok;
    } else {
      hqco_kem_encaps(j->id, j->h + i * U, j->s + i * U, j->m + i * K, j->u + i * U,
                      j->v + i * V, j->key + i * HQCO_KEM_KEY_BYTES);
    }
  }
  return NULL;
}

static int run_kem(kjob_t tmpl, size_t count, int nthreads) {
  hqco_param_t p;
  if (hqco_param(tmpl.id, &p)) return -1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if ((size_t)nthreads > count) nthreads = count ? (int)count : 1;
  pthread_t th[256];
  kjob_t jobs[256];
  for (int t = 0; t < nthreads; t++) {
    jobs[t] = tmpl;
    jobs[t].lo = count * (size_t)t / (size_t)nthreads;
    jobs[t].hi = count * (size_t)(t + 1) / (size_t)nthreads;
  }
  for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, run_kjob, &jobs[t]);
  for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
  return 0;
}

int hqco_kem_encaps_batch(int id, size_t count, const uint64_t *h, const uint64_t *s,
                          const uint8_t *m, uint64_t *u, uint64_t *v, uint8_t *key,
                          int nthreads) {
  kjob_t t = {0};
  t.id = id;
  t.h = h;
  t.s = s;
  t.m = m;
  t.u = u;
  t.v = v;
  t.key = key;
  return run_kem(t, count, nthreads);
}

int hqco_kem_decaps_batch(int id, size_t count, const uint64_t *h, const uint64_t *s,
                          const uint32_t *y, const uint8_t *sigma, const uint64_t *u,
                          const uint64_t *v, uint8_t *key, int32_t *ok, int nthreads) {
  kjob_t t = {0};
  t.id = id;
  t.decaps = 1;
  t.h = h;
  t.s = s;
  t.y = y;
  t.sigma = sigma;
  t.u_in = u;
  t.v_in = v;
  t.key = key;
  t.ok = ok;
  return run_kem(t, count, nthreads);
}
