/*
 * hqc_synth.c -- seeded synthetic inputs for HQC decryption workloads.
 *
 * This module only draws random numbers: uniform dense bit vectors, uniform
 * bytes, and uniform fixed-weight support sets.  It contains none of the
 * scheme's arithmetic (no ring product, no encoding, no decoding); the draws
 * are handed to whichever side computes with them.  The paper's SHAKE-based
 * sampling (Sec. II-A) is replaced by SplitMix64 streams, so the bytes differ
 * from the official scheme while the distributions are the same: h uniform
 * over n-bit vectors, x, y, r1, r2, e uniform over vectors of their weight
 * (Alg. 1 and Alg. 3), m uniform.
 *
 * SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15, output = the
 * state passed through the two xor-shift-multiply rounds of the published
 * finaliser.
 *
 * Streams (frozen: changing anything here changes every dataset):
 *   seed(parent, salt)   = first output of the stream whose state is parent ^ salt
 *   key stream           = seed(master, param_id << 56 ^ key_id)
 *       draws, in order: h (ceil(n/64) words, bits >= n cleared), x (w), y (w)
 *   encryption stream    = seed(key stream seed, 1 << 55 ^ ct_id)
 *       draws, in order: m (k bytes), r1 (wr), r2 (wr), e (we)
 *   stress-word stream   = seed(master, param_id << 56 ^ 1 << 54 ^ word_id)
 *       draws, in order: m (k bytes), delta distinct block indices < n1,
 *       delta values in [1, 255], then for each block not drawn, in block
 *       order: tau uniform in [0, rho], then tau distinct bit positions < n2
 *       of that block, set in the noise vector.
 *   bytes: each output gives 8 bytes, least significant first.
 *   index in [0, bound): c = output >> 32; c is rejected when
 *       c >= 2^32 - (2^32 mod bound); the index is c mod bound.
 *   fixed weight w: indices drawn as above, a repeat of an index already
 *       taken is rejected, until w distinct ones; kept in draw order.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct synth_sizes {
  int32_t param_id; /* 1, 3 or 5: only salts the streams */
  int32_t n, n1, n2, k, delta, w, wr, we;
  int32_t rho; /* largest noise weight per clean block */
} synth_sizes_t;

static const uint64_t GAMMA = 0x9E3779B97F4A7C15ull;

uint64_t synth_splitmix64_next(uint64_t *state) {
  uint64_t z = (*state += GAMMA);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t synth_seed(uint64_t parent, uint64_t salt) {
  uint64_t st = parent ^ salt;
  return synth_splitmix64_next(&st);
}

static uint32_t draw_below(uint64_t *st, uint32_t bound) {
  uint64_t lim = (1ull << 32) - ((1ull << 32) % bound);
  for (;;) {
    uint64_t c = synth_splitmix64_next(st) >> 32;
    if (c < lim) return (uint32_t)(c % bound);
  }
}

static void draw_bytes(uint64_t *st, int nbytes, uint8_t *out) {
  uint64_t z = 0;
  for (int i = 0; i < nbytes; i++) {
    if ((i & 7) == 0) z = synth_splitmix64_next(st);
    out[i] = (uint8_t)(z >> (8 * (i & 7)));
  }
}

static void draw_dense(uint64_t *st, int nbits, uint64_t *out) {
  int words = (nbits + 63) / 64;
  for (int i = 0; i < words; i++) out[i] = synth_splitmix64_next(st);
  if (nbits & 63) out[words - 1] &= (1ull << (nbits & 63)) - 1;
}

static void draw_fixed_weight(uint64_t *st, uint32_t bound, int w, uint32_t *out) {
  int have = 0;
  while (have < w) {
    uint32_t c = draw_below(st, bound);
    int dup = 0;
    for (int i = 0; i < have; i++) dup |= (out[i] == c);
    if (!dup) out[have++] = c;
  }
}

/* Exported single-stream draws (used by tests of this module). */
void synth_fixed_weight(uint64_t seed, uint32_t bound, int w, uint32_t *out) {
  uint64_t st = seed;
  draw_fixed_weight(&st, bound, w, out);
}
void synth_dense(uint64_t seed, int nbits, uint64_t *out) {
  uint64_t st = seed;
  draw_dense(&st, nbits, out);
}

/* ---------------------------------------------------------------------- */
typedef struct task {
  int op;
  uint64_t master;
  synth_sizes_t sz;
  size_t lo, hi;
  uint64_t id0;
  const int64_t *key_of;
  uint64_t *h;
  uint32_t *x, *y;
  uint8_t *m;
  uint32_t *r1, *r2, *e;
  uint32_t *bad;
  uint8_t *dval;
  uint64_t *noise;
} task_t;

static uint64_t key_seed(const task_t *t, uint64_t key_id) {
  return synth_seed(t->master, ((uint64_t)t->sz.param_id << 56) ^ key_id);
}

static void *run_task(void *arg) {
  task_t *t = arg;
  const synth_sizes_t *s = &t->sz;
  int nwords = (s->n + 63) / 64;
  int vwords = s->n1 * s->n2 / 64;
  for (size_t i = t->lo; i < t->hi; i++) {
    if (t->op == 0) { /* keys */
      uint64_t st = key_seed(t, t->id0 + i);
      draw_dense(&st, s->n, t->h + i * nwords);
      draw_fixed_weight(&st, (uint32_t)s->n, s->w, t->x + i * s->w);
      draw_fixed_weight(&st, (uint32_t)s->n, s->w, t->y + i * s->w);
    } else if (t->op == 1) { /* encryption randomness */
      uint64_t kid = t->key_of ? (uint64_t)t->key_of[i] : 0;
      uint64_t st = synth_seed(key_seed(t, kid), (1ull << 55) ^ (t->id0 + i));
      draw_bytes(&st, s->k, t->m + i * s->k);
      draw_fixed_weight(&st, (uint32_t)s->n, s->wr, t->r1 + i * s->wr);
      draw_fixed_weight(&st, (uint32_t)s->n, s->wr, t->r2 + i * s->wr);
      draw_fixed_weight(&st, (uint32_t)s->n, s->we, t->e + i * s->we);
    } else { /* stress words */
      uint64_t st = synth_seed(t->master, ((uint64_t)s->param_id << 56) ^ (1ull << 54) ^
                                              (t->id0 + i));
      uint32_t *bad = t->bad + i * s->delta;
      uint8_t *dval = t->dval + i * s->delta;
      uint64_t *noise = t->noise + i * vwords;
      draw_bytes(&st, s->k, t->m + i * s->k);
      draw_fixed_weight(&st, (uint32_t)s->n1, s->delta, bad);
      for (int l = 0; l < s->delta; l++) dval[l] = (uint8_t)(1 + draw_below(&st, 255));
      memset(noise, 0, sizeof(uint64_t) * vwords);
      uint32_t pos[1024];
      for (int j = 0; j < s->n1; j++) {
        int is_bad = 0;
        for (int l = 0; l < s->delta; l++) is_bad |= (bad[l] == (uint32_t)j);
        if (is_bad) continue;
        int tau = (int)draw_below(&st, (uint32_t)s->rho + 1);
        draw_fixed_weight(&st, (uint32_t)s->n2, tau, pos);
        for (int f = 0; f < tau; f++) {
          long b = (long)j * s->n2 + pos[f];
          noise[b >> 6] |= 1ull << (b & 63);
        }
      }
    }
  }
  return NULL;
}

static int run(task_t tmpl, size_t count, int nthreads) {
  const synth_sizes_t *s = &tmpl.sz;
  /* every fixed-weight draw must be able to finish: weights at most their
     bound, noise weights within one block and the position buffer */
  if (s->n <= 0 || s->n1 <= 0 || s->n2 <= 0 || s->k < 0 || s->rho < 0 || s->rho >= 1024 ||
      s->rho > s->n2 || s->delta < 0 || s->delta > s->n1 || s->w < 0 || s->w > s->n ||
      s->wr < 0 || s->wr > s->n || s->we < 0 || s->we > s->n || (s->n1 * s->n2) % 64 != 0)
    return -1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if ((size_t)nthreads > count) nthreads = count ? (int)count : 1;
  task_t tasks[256];
  pthread_t th[256];
  for (int i = 0; i < nthreads; i++) {
    tasks[i] = tmpl;
    tasks[i].lo = count * i / nthreads;
    tasks[i].hi = count * (i + 1) / nthreads;
  }
  if (nthreads == 1) {
    run_task(&tasks[0]);
    return 0;
  }
  for (int i = 0; i < nthreads; i++) pthread_create(&th[i], NULL, run_task, &tasks[i]);
  for (int i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
  return 0;
}

/* Keys key_id0 .. key_id0 + count - 1: h (count x ceil(n/64) words),
 * x and y (count x w indices each). */
int synth_keys(uint64_t master, const synth_sizes_t *sz, size_t count, uint64_t key_id0,
               uint64_t *h, uint32_t *x, uint32_t *y, int nthreads) {
  task_t t;
  memset(&t, 0, sizeof t);
  t.op = 0;
  t.master = master;
  t.sz = *sz;
  t.id0 = key_id0;
  t.h = h;
  t.x = x;
  t.y = y;
  return run(t, count, nthreads);
}

/* Encryption randomness for ciphertexts ct_id0 + i under key key_of[i]
 * (key 0 when key_of is NULL): m (k bytes), r1, r2 (wr), e (we). */
int synth_encryptions(uint64_t master, const synth_sizes_t *sz, size_t count,
                      const int64_t *key_of, uint64_t ct_id0, uint8_t *m, uint32_t *r1,
                      uint32_t *r2, uint32_t *e, int nthreads) {
  task_t t;
  memset(&t, 0, sizeof t);
  t.op = 1;
  t.master = master;
  t.sz = *sz;
  t.id0 = ct_id0;
  t.key_of = key_of;
  t.m = m;
  t.r1 = r1;
  t.r2 = r2;
  t.e = e;
  return run(t, count, nthreads);
}

/* Stress-word draws for words word_id0 + i: m (k bytes), bad (delta block
 * indices), dval (delta nonzero bytes), noise (n1*n2/64 words). */
int synth_stress(uint64_t master, const synth_sizes_t *sz, size_t count, uint64_t word_id0,
                 uint8_t *m, uint32_t *bad, uint8_t *dval, uint64_t *noise, int nthreads) {
  task_t t;
  memset(&t, 0, sizeof t);
  t.op = 2;
  t.master = master;
  t.sz = *sz;
  t.id0 = word_id0;
  t.m = m;
  t.bad = bad;
  t.dval = dval;
  t.noise = noise;
  return run(t, count, nthreads);
}

/* Uniform random bytes / words from one stream (filler for inputs whose
 * content does not matter, e.g. beyond-radius parity cases). */
void synth_fill_words(uint64_t seed, size_t nwords, uint64_t *out) {
  uint64_t st = seed;
  for (size_t i = 0; i < nwords; i++) out[i] = synth_splitmix64_next(&st);
}
