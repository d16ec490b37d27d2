/*
 * hqc_oracle.c -- plain CPU model of HQC.PKE and its concatenated code.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline timing, never by the product library.  Written for clarity, not
 * speed: no SIMD, no bit tricks beyond word shifts, threads only across
 * independent items in the *_batch helpers.  See hqc_oracle.h for the
 * paper passages and for what pins each function.
 */
#include "hqc_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Parameters: Table I.  Columns: N, omega, omega_e = omega_r, RS [n1,k,d],  */
/* RM [n2, 8, d2].                                                           */
/* ------------------------------------------------------------------------ */
static const struct {
  int id, n, w, wre, n1, k, rs_d, n2, rm_d;
} TABLE_I[3] = {
    {1, 17669, 66, 75, 46, 16, 31, 384, 192},
    {3, 35851, 100, 114, 56, 24, 33, 640, 320},
    {5, 57637, 131, 149, 90, 32, 59, 640, 320},
};

int hqco_param(int id, hqco_param_t *out) {
  for (int i = 0; i < 3; i++) {
    if (TABLE_I[i].id != id) continue;
    hqco_param_t p;
    p.id = id;
    p.n = TABLE_I[i].n;
    p.n1 = TABLE_I[i].n1;
    p.k = TABLE_I[i].k;
    p.rs_d = TABLE_I[i].rs_d;
    p.delta = (TABLE_I[i].rs_d - 1) / 2;
    p.n2 = TABLE_I[i].n2;
    p.rm_d = TABLE_I[i].rm_d;
    p.mult = TABLE_I[i].n2 / 128;
    p.w = TABLE_I[i].w;
    p.wr = TABLE_I[i].wre;
    p.we = TABLE_I[i].wre;
    p.nwords = (p.n + 63) / 64;
    p.vwords = p.n1 * p.n2 / 64;
    *out = p;
    return 0;
  }
  return -1;
}

/* ------------------------------------------------------------------------ */
/* GF(2^8) with modulus x^8 + x^4 + x^3 + x^2 + 1 (0x11D), alpha = x.        */
/* ------------------------------------------------------------------------ */
#define GF_MODULUS 0x11Du

uint8_t hqco_gf_mul(uint8_t a, uint8_t b) {
  /* schoolbook carry-less product (degree <= 14) ... */
  uint32_t p = 0;
  for (int i = 0; i < 8; i++)
    if ((b >> i) & 1u) p ^= (uint32_t)a << i;
  /* ... then reduce the terms of degree 14 .. 8 by the modulus */
  for (int d = 14; d >= 8; d--)
    if ((p >> d) & 1u) p ^= GF_MODULUS << (d - 8);
  return (uint8_t)p;
}

uint8_t hqco_gf_pow(uint8_t a, uint32_t e) {
  uint8_t r = 1, b = a;
  while (e) {
    if (e & 1u) r = hqco_gf_mul(r, b);
    b = hqco_gf_mul(b, b);
    e >>= 1;
  }
  return r;
}

/* a^254 = a^-1 for a != 0 (the multiplicative group has order 255); 0 -> 0 */
uint8_t hqco_gf_inv(uint8_t a) { return hqco_gf_pow(a, 254); }

/* Full multiplication table filled from hqco_gf_mul, plus the powers of
 * alpha; built once, read-only afterwards. */
static uint8_t MUL[256][256];
static uint8_t ALPHA_POW[255];
static uint8_t LOG_OF[256];
static pthread_once_t tables_once = PTHREAD_ONCE_INIT;

static void build_tables(void) {
  for (int a = 0; a < 256; a++)
    for (int b = 0; b < 256; b++) MUL[a][b] = hqco_gf_mul((uint8_t)a, (uint8_t)b);
  uint8_t x = 1;
  memset(LOG_OF, 0, sizeof LOG_OF);
  for (int i = 0; i < 255; i++) {
    ALPHA_POW[i] = x;
    LOG_OF[x] = (uint8_t)i;
    x = hqco_gf_mul(x, 0x02);
  }
}
static void tables(void) { pthread_once(&tables_once, build_tables); }

static inline uint8_t gmul(uint8_t a, uint8_t b) { return MUL[a][b]; }
/* alpha^e for any integer e (negative allowed) */
static inline uint8_t apow(long e) {
  long r = e % 255;
  if (r < 0) r += 255;
  return ALPHA_POW[r];
}

void hqco_gf_tables(uint8_t exp_out[255], uint8_t log_out[256]) {
  tables();
  memcpy(exp_out, ALPHA_POW, 255);
  memcpy(log_out, LOG_OF, 256);
}

/* ------------------------------------------------------------------------ */
/* Ring product in GF(2)[X]/(X^n - 1), Eq. (1):                              */
/*   a1 * a2 = XOR over i in Supp(a1) of X^i * a2.                           */
/* X^s * a is the cyclic rotation of the n-bit vector a by s places; it is  */
/* formed here as (a << s, truncated to n bits) XOR (a >> (n - s)).          */
/* ------------------------------------------------------------------------ */
static void clear_above(uint64_t *a, int words, int nbits) {
  for (int i = 0; i < words; i++) {
    int lo = 64 * i;
    if (lo >= nbits)
      a[i] = 0;
    else if (nbits - lo < 64)
      a[i] &= (1ull << (nbits - lo)) - 1;
  }
}

/* out = a << s within a words-long array (bits shifted past the end drop) */
static void shift_up(const uint64_t *a, int words, int s, uint64_t *out) {
  int ws = s / 64, bs = s % 64;
  for (int i = words - 1; i >= 0; i--) {
    uint64_t v = 0;
    int j = i - ws;
    if (j >= 0) {
      v = a[j] << bs;
      if (bs && j - 1 >= 0) v |= a[j - 1] >> (64 - bs);
    }
    out[i] = v;
  }
}

/* out = a >> s */
static void shift_down(const uint64_t *a, int words, int s, uint64_t *out) {
  int ws = s / 64, bs = s % 64;
  for (int i = 0; i < words; i++) {
    uint64_t v = 0;
    int j = i + ws;
    if (j < words) {
      v = a[j] >> bs;
      if (bs && j + 1 < words) v |= a[j + 1] << (64 - bs);
    }
    out[i] = v;
  }
}

void hqco_mul_sparse(int n, const uint64_t *a, const uint32_t *supp, int w,
                     uint64_t *out) {
  int words = (n + 63) / 64;
  uint64_t *am = malloc(sizeof(uint64_t) * words);
  uint64_t *t1 = malloc(sizeof(uint64_t) * words);
  uint64_t *t2 = malloc(sizeof(uint64_t) * words);
  memcpy(am, a, sizeof(uint64_t) * words);
  clear_above(am, words, n);
  memset(out, 0, sizeof(uint64_t) * words);
  for (int k = 0; k < w; k++) {
    int s = (int)(supp[k] % (uint32_t)n);
    if (s == 0) {
      for (int i = 0; i < words; i++) out[i] ^= am[i];
      continue;
    }
    shift_up(am, words, s, t1);
    clear_above(t1, words, n); /* bits that pass X^n wrap around ... */
    shift_down(am, words, n - s, t2); /* ... and re-enter at the bottom */
    for (int i = 0; i < words; i++) out[i] ^= t1[i] ^ t2[i];
  }
  free(am);
  free(t1);
  free(t2);
}

/* ------------------------------------------------------------------------ */
/* Duplicated first-order Reed-Muller code RM(1,7), n2 = 128 * mult.         */
/* ------------------------------------------------------------------------ */
static inline int get_bit(const uint64_t *a, long t) { return (int)((a[t >> 6] >> (t & 63)) & 1u); }
static inline void flip_bit(uint64_t *a, long t) { a[t >> 6] ^= 1ull << (t & 63); }

static int parity7(int x) {
  int p = 0;
  for (int l = 0; l < 7; l++) p ^= (x >> l) & 1;
  return p;
}

void hqco_rm_encode(int mult, uint8_t b, uint64_t *out) {
  memset(out, 0, sizeof(uint64_t) * 2 * mult);
  for (int i = 0; i < 128; i++) {
    /* affine Boolean function: constant term b7, linear part b0..b6 */
    int bit = ((b >> 7) & 1) ^ parity7(b & i & 0x7F);
    if (bit)
      for (int q = 0; q < mult; q++) flip_bit(out, 128L * q + i);
  }
}

void hqco_fht128(const int32_t in[128], int32_t out[128]) {
  int32_t x[128];
  memcpy(x, in, sizeof x);
  for (int h = 1; h < 128; h *= 2)
    for (int i = 0; i < 128; i += 2 * h)
      for (int j = i; j < i + h; j++) {
        int32_t a = x[j], c = x[j + h];
        x[j] = a + c;
        x[j + h] = a - c;
      }
  memcpy(out, x, sizeof x);
}

uint8_t hqco_rm_decode(int mult, const uint64_t *blk, int32_t *T_out) {
  int32_t t[128], T[128];
  for (int i = 0; i < 128; i++) {
    int ones = 0;
    for (int q = 0; q < mult; q++) ones += get_bit(blk, 128L * q + i);
    /* sum over the copies of (-1)^bit */
    t[i] = mult - 2 * ones;
  }
  hqco_fht128(t, T);
  int best = 0;
  for (int u = 1; u < 128; u++)
    if (abs(T[u]) > abs(T[best])) best = u; /* strict: smallest u wins ties */
  if (T_out) memcpy(T_out, T, sizeof T);
  return (uint8_t)(best | (T[best] < 0 ? 0x80 : 0));
}

/* ------------------------------------------------------------------------ */
/* Reed-Solomon over GF(2^8): narrow-sense (roots alpha^1 .. alpha^2d),      */
/* shortened to length n1, systematic.                                       */
/* ------------------------------------------------------------------------ */
void hqco_rs_generator(int two_delta, uint8_t *g) {
  tables();
  memset(g, 0, (size_t)two_delta + 1);
  g[0] = 1; /* g = 1, degree 0 */
  for (int i = 1; i <= two_delta; i++) {
    /* g <- g * (x + alpha^i)   (characteristic 2: minus is plus) */
    uint8_t r = apow(i);
    for (int d = i; d >= 0; d--) {
      uint8_t shifted = d > 0 ? g[d - 1] : 0; /* coefficient of x * g */
      g[d] = shifted ^ gmul(r, g[d]);
    }
  }
}

void hqco_rs_encode(int n1, int k, const uint8_t *m, uint8_t *c) {
  tables();
  int td = n1 - k;
  uint8_t g[256];
  hqco_rs_generator(td, g);
  /* A(x) = x^td * m(x), then reduce mod the monic g by long division */
  uint8_t A[256];
  memset(A, 0, sizeof A);
  for (int t = 0; t < k; t++) A[td + t] = m[t];
  for (int d = n1 - 1; d >= td; d--) {
    uint8_t q = A[d];
    if (!q) continue;
    for (int i = 0; i <= td; i++) A[d - td + i] ^= gmul(q, g[i]);
  }
  for (int j = 0; j < td; j++) c[j] = A[j];     /* parity = remainder */
  for (int t = 0; t < k; t++) c[td + t] = m[t]; /* message, unchanged */
}

void hqco_rs_syndromes(int n1, int two_delta, const uint8_t *c, uint8_t *S) {
  tables();
  for (int i = 1; i <= two_delta; i++) {
    uint8_t s = 0;
    for (int j = 0; j < n1; j++) s ^= gmul(c[j], apow((long)i * j));
    S[i - 1] = s;
  }
}

int hqco_rs_berlekamp_massey(int two_delta, const uint8_t *S, uint8_t *lambda) {
  tables();
  int td = two_delta;
  uint8_t C[65], B[65], T[65];
  memset(C, 0, sizeof C);
  memset(B, 0, sizeof B);
  C[0] = 1;
  B[0] = 1;
  int L = 0, shift = 1;
  uint8_t b = 1;
  for (int r = 1; r <= td; r++) {
    /* discrepancy of the current connection polynomial at step r */
    uint8_t delta = S[r - 1];
    for (int i = 1; i <= td; i++)
      if (r - i >= 1) delta ^= gmul(C[i], S[r - i - 1]);
    if (delta == 0) {
      shift++;
      continue;
    }
    uint8_t coef = gmul(delta, hqco_gf_inv(b));
    memcpy(T, C, sizeof C);
    for (int i = shift; i <= td; i++) C[i] ^= gmul(coef, B[i - shift]); /* terms above 2d dropped */
    if (2 * L <= r - 1) {
      L = r - L;
      memcpy(B, T, sizeof B);
      b = delta;
      shift = 1;
    } else {
      shift++;
    }
  }
  memcpy(lambda, C, (size_t)td + 1);
  return L;
}

void hqco_rs_decode(int n1, int k, const uint8_t *c, uint8_t *m,
                    hqco_rs_trace_t *trace) {
  tables();
  int td = n1 - k;
  uint8_t S[64], lambda[65], omega[64], located[256], err[256];
  hqco_rs_syndromes(n1, td, c, S);
  int L = hqco_rs_berlekamp_massey(td, S, lambda);

  /* Omega(x) = S(x) Lambda(x) mod x^2d with S(x) = sum_i S_i x^(i-1) */
  for (int e = 0; e < td; e++) {
    uint8_t o = 0;
    for (int i = 0; i <= e; i++) o ^= gmul(lambda[i], S[e - i]);
    omega[e] = o;
  }
  for (int j = 0; j < n1; j++) {
    /* Chien: position j is in error iff Lambda(alpha^-j) = 0 */
    uint8_t lam = 0, dlam = 0, om = 0;
    for (int i = 0; i <= td; i++) {
      uint8_t term = gmul(lambda[i], apow(-(long)i * j));
      lam ^= term;
    }
    /* formal derivative: Lambda'(x) = sum over odd i of Lambda_i x^(i-1) */
    for (int i = 1; i <= td; i += 2) dlam ^= gmul(lambda[i], apow(-(long)(i - 1) * j));
    for (int e = 0; e < td; e++) om ^= gmul(omega[e], apow(-(long)e * j));
    located[j] = (uint8_t)(lam == 0);
    /* Forney (first consecutive root alpha^1): e_j = Omega(X^-1) / Lambda'(X^-1) */
    err[j] = located[j] ? gmul(om, hqco_gf_inv(dlam)) : 0;
  }
  for (int t = 0; t < k; t++) m[t] = c[td + t] ^ err[td + t];

  if (trace) {
    memset(trace, 0, sizeof *trace);
    memcpy(trace->S, S, (size_t)td);
    memcpy(trace->lambda, lambda, (size_t)td + 1);
    trace->L = L;
    memcpy(trace->omega, omega, (size_t)td);
    memcpy(trace->located, located, (size_t)n1);
    memcpy(trace->err, err, (size_t)n1);
  }
}

/* ------------------------------------------------------------------------ */
/* Concatenated code: RS outer, duplicated RM inner.                         */
/* ------------------------------------------------------------------------ */
void hqco_code_encode(int id, const uint8_t *m, uint64_t *cw) {
  hqco_param_t p;
  if (hqco_param(id, &p)) return;
  uint8_t c[256];
  hqco_rs_encode(p.n1, p.k, m, c);
  int bw = p.n2 / 64; /* words per RM block */
  for (int j = 0; j < p.n1; j++) hqco_rm_encode(p.mult, c[j], cw + (long)j * bw);
}

void hqco_code_decode(int id, const uint64_t *r, uint8_t *m, uint8_t *symbols_out,
                      hqco_rs_trace_t *trace) {
  hqco_param_t p;
  if (hqco_param(id, &p)) return;
  uint8_t c[256];
  int bw = p.n2 / 64;
  for (int j = 0; j < p.n1; j++) c[j] = hqco_rm_decode(p.mult, r + (long)j * bw, NULL);
  if (symbols_out) memcpy(symbols_out, c, (size_t)p.n1);
  hqco_rs_decode(p.n1, p.k, c, m, trace);
}

/* ------------------------------------------------------------------------ */
/* HQC.PKE (Alg. 1-3).                                                       */
/* ------------------------------------------------------------------------ */
static uint64_t *support_to_dense(const hqco_param_t *p, const uint32_t *supp, int w) {
  uint64_t *d = calloc((size_t)p->nwords, sizeof(uint64_t));
  for (int i = 0; i < w; i++) flip_bit(d, supp[i] % (uint32_t)p->n);
  return d;
}

void hqco_keygen(int id, const uint64_t *h, const uint32_t *x, const uint32_t *y,
                 uint64_t *s) {
  hqco_param_t p;
  if (hqco_param(id, &p)) return;
  uint64_t *hy = malloc(sizeof(uint64_t) * p.nwords);
  hqco_mul_sparse(p.n, h, y, p.w, hy);
  uint64_t *xd = support_to_dense(&p, x, p.w);
  for (int i = 0; i < p.nwords; i++) s[i] = xd[i] ^ hy[i];
  free(hy);
  free(xd);
}

void hqco_encrypt(int id, const uint64_t *h, const uint64_t *s, const uint8_t *m,
                  const uint32_t *r1, const uint32_t *r2, const uint32_t *e,
                  uint64_t *u, uint64_t *v) {
  hqco_param_t p;
  if (hqco_param(id, &p)) return;
  uint64_t *hr2 = malloc(sizeof(uint64_t) * p.nwords);
  uint64_t *sr2 = malloc(sizeof(uint64_t) * p.nwords);
  uint64_t *mg = calloc((size_t)p.nwords, sizeof(uint64_t));
  uint64_t *r1d = support_to_dense(&p, r1, p.wr);
  uint64_t *ed = support_to_dense(&p, e, p.we);
  hqco_mul_sparse(p.n, h, r2, p.wr, hr2);
  hqco_mul_sparse(p.n, s, r2, p.wr, sr2);
  hqco_code_encode(id, m, mg); /* n1*n2 bits, zero above */
  for (int i = 0; i < p.nwords; i++) u[i] = r1d[i] ^ hr2[i];
  /* v keeps the first n1*n2 bits (a whole number of words) */
  for (int i = 0; i < p.vwords; i++) v[i] = mg[i] ^ sr2[i] ^ ed[i];
  free(hr2);
  free(sr2);
  free(mg);
  free(r1d);
  free(ed);
}

void hqco_decrypt(int id, const uint32_t *y, const uint64_t *u, const uint64_t *v,
                  uint8_t *m) {
  hqco_param_t p;
  if (hqco_param(id, &p)) return;
  uint64_t *uy = malloc(sizeof(uint64_t) * p.nwords);
  uint64_t *r = malloc(sizeof(uint64_t) * p.vwords);
  hqco_mul_sparse(p.n, u, y, p.w, uy);
  for (int i = 0; i < p.vwords; i++) r[i] = v[i] ^ uy[i];
  hqco_code_decode(id, r, m, NULL, NULL);
  free(uy);
  free(r);
}

void hqco_stress_word(int id, const uint8_t *m, int nbad, const uint32_t *bad,
                      const uint8_t *dval, const uint64_t *noise, uint64_t *r) {
  hqco_param_t p;
  if (hqco_param(id, &p)) return;
  uint64_t *cw = malloc(sizeof(uint64_t) * p.vwords);
  hqco_code_encode(id, m, cw);
  int bw = p.n2 / 64;
  uint64_t blk[10];
  for (int l = 0; l < nbad; l++) {
    hqco_rm_encode(p.mult, dval[l], blk);
    for (int i = 0; i < bw; i++) cw[(long)bad[l] * bw + i] ^= blk[i];
  }
  for (int i = 0; i < p.vwords; i++) r[i] = cw[i] ^ noise[i];
  free(cw);
}

/* ------------------------------------------------------------------------ */
/* Batch helpers: a static split of the items over nthreads workers.         */
/* ------------------------------------------------------------------------ */
typedef struct job {
  int op, id;
  size_t lo, hi;
  const uint64_t *h, *s_in, *u_in, *v_in;
  const uint32_t *x, *y, *r1, *r2, *e;
  const int64_t *key_of;
  const uint8_t *m_in, *dval;
  const uint32_t *bad;
  uint64_t *s_out, *u_out, *v_out;
  uint8_t *m_out;
} job_t;

static void *run_job(void *arg) {
  job_t *j = arg;
  hqco_param_t p;
  hqco_param(j->id, &p);
  for (size_t i = j->lo; i < j->hi; i++) {
    size_t kr = j->key_of ? (size_t)j->key_of[i] : i;
    switch (j->op) {
      case 0:
        hqco_keygen(j->id, j->h + i * p.nwords, j->x + i * p.w, j->y + i * p.w,
                    j->s_out + i * p.nwords);
        break;
      case 1:
        hqco_encrypt(j->id, j->h + kr * p.nwords, j->s_in + kr * p.nwords,
                     j->m_in + i * p.k, j->r1 + i * p.wr, j->r2 + i * p.wr,
                     j->e + i * p.we, j->u_out + i * p.nwords, j->v_out + i * p.vwords);
        break;
      case 2:
        hqco_decrypt(j->id, j->y + kr * p.w, j->u_in + i * p.nwords,
                     j->v_in + i * p.vwords, j->m_out + i * p.k);
        break;
      case 3:
        hqco_code_decode(j->id, j->u_in + i * p.vwords, j->m_out + i * p.k, NULL, NULL);
        break;
      case 4:
        hqco_stress_word(j->id, j->m_in + i * p.k, p.delta, j->bad + i * p.delta,
                         j->dval + i * p.delta, j->u_in + i * p.vwords,
                         j->u_out + i * p.vwords);
        break;
    }
  }
  return NULL;
}

static int run_batch(job_t tmpl, size_t count, int nthreads) {
  hqco_param_t p;
  if (hqco_param(tmpl.id, &p)) return -1;
  tables();
  if (nthreads < 1) nthreads = 1;
  if ((size_t)nthreads > count) nthreads = count ? (int)count : 1;
  pthread_t th[256];
  job_t jobs[256];
  if (nthreads > 256) nthreads = 256;
  for (int t = 0; t < nthreads; t++) {
    jobs[t] = tmpl;
    jobs[t].lo = count * t / nthreads;
    jobs[t].hi = count * (t + 1) / nthreads;
  }
  if (nthreads == 1) {
    run_job(&jobs[0]);
    return 0;
  }
  for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, run_job, &jobs[t]);
  for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
  return 0;
}

int hqco_keygen_batch(int id, size_t count, const uint64_t *h, const uint32_t *x,
                      const uint32_t *y, uint64_t *s, int nthreads) {
  job_t j;
  memset(&j, 0, sizeof j);
  j.op = 0;
  j.id = id;
  j.h = h;
  j.x = x;
  j.y = y;
  j.s_out = s;
  return run_batch(j, count, nthreads);
}

int hqco_encrypt_batch(int id, size_t count, const uint64_t *h, const uint64_t *s,
                       const int64_t *key_of, const uint8_t *m, const uint32_t *r1,
                       const uint32_t *r2, const uint32_t *e, uint64_t *u, uint64_t *v,
                       int nthreads) {
  job_t j;
  memset(&j, 0, sizeof j);
  j.op = 1;
  j.id = id;
  j.h = h;
  j.s_in = s;
  j.key_of = key_of;
  j.m_in = m;
  j.r1 = r1;
  j.r2 = r2;
  j.e = e;
  j.u_out = u;
  j.v_out = v;
  return run_batch(j, count, nthreads);
}

int hqco_decrypt_batch(int id, size_t count, const uint32_t *y, const int64_t *key_of,
                       const uint64_t *u, const uint64_t *v, uint8_t *m, int nthreads) {
  job_t j;
  memset(&j, 0, sizeof j);
  j.op = 2;
  j.id = id;
  j.y = y;
  j.key_of = key_of;
  j.u_in = u;
  j.v_in = v;
  j.m_out = m;
  return run_batch(j, count, nthreads);
}

int hqco_decode_batch(int id, size_t count, const uint64_t *r, uint8_t *m, int nthreads) {
  job_t j;
  memset(&j, 0, sizeof j);
  j.op = 3;
  j.id = id;
  j.u_in = r;
  j.m_out = m;
  return run_batch(j, count, nthreads);
}

int hqco_stress_batch(int id, size_t count, const uint8_t *m, const uint32_t *bad,
                      const uint8_t *dval, const uint64_t *noise, uint64_t *r,
                      int nthreads) {
  job_t j;
  memset(&j, 0, sizeof j);
  j.op = 4;
  j.id = id;
  j.m_in = m;
  j.bad = bad;
  j.dval = dval;
  j.u_in = noise;
  j.u_out = r;
  return run_batch(j, count, nthreads);
}
