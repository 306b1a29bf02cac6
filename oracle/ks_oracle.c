/*
 * ks_oracle.c -- plain, slow CPU oracle for CKKS hybrid key switching.
 *
 * TEST INFRASTRUCTURE ONLY (see ks_oracle.h).  Every reduction is a plain
 * uint64 '%'; there is no Montgomery, Shoup or Barrett arithmetic, no lazy
 * range, no fusion and no reordering beyond what each function's definition
 * states.  The HIP library must never include or link this file.
 *
 * Readings of the paper taken here (the paper is silent on them):
 *  - moduli: 2^30 - t*2N + 1 for t = 1, 2, ...; first K primes form P,
 *    the next L+1 form Q (P > Q_j so the ModDown error stays small);
 *  - psi: the smallest primitive 2N-th root of unity;
 *  - evaluation domain: NTT(a)[j] = a(psi^(2*brv(j)+1));
 *  - digits are the raw limbs (Sec. III-A decomposition); the gadget factor
 *    lives in the key, [P]_m on the digit's own q-limbs and 0 elsewhere;
 *  - basis conversion is the fast (approximate) one, with no correction,
 *    in both ModUp P2 and ModDown P2;
 *  - ModDown P4 computes (acc - w_hat) * [P^-1]_{q_i}; outputs canonical.
 */
#include "ks_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static int g_fault = 0;
void oracle_set_fault(int fault) { g_fault = fault; }
/* Planted mistakes (for tests of the checks, never set otherwise):
 *  1: ModUp P5 drops the last digit's contribution
 *  2: ModDown P4 adds w_hat instead of subtracting it
 *  3: ModUp P2 uses the wrong target constant (index off by one)
 *  4: ModUp P3 bypass takes the limb from the neighbouring digit
 *  5: hoisted rotations (single and summed) permute the digits with the
 *     inverse map */

/* ------------------------------------------------------------------ */
/* integers                                                             */
/* ------------------------------------------------------------------ */

static uint32_t mulmod(uint32_t a, uint32_t b, uint32_t q) {
  return (uint32_t)(((uint64_t)a * (uint64_t)b) % q);
}
static uint32_t addmod(uint32_t a, uint32_t b, uint32_t q) {
  return (uint32_t)(((uint64_t)a + (uint64_t)b) % q);
}
static uint32_t submod(uint32_t a, uint32_t b, uint32_t q) {
  return (uint32_t)(((uint64_t)a + (uint64_t)q - (uint64_t)(b % q)) % q);
}

uint32_t oracle_powmod(uint32_t b, uint64_t e, uint32_t q) {
  uint64_t r = 1 % q, x = b % q;
  while (e) {
    if (e & 1) r = (r * x) % q;
    x = (x * x) % q;
    e >>= 1;
  }
  return (uint32_t)r;
}

/* q prime: a^(q-2) is the inverse of a (Fermat). */
uint32_t oracle_invmod(uint32_t a, uint32_t q) { return oracle_powmod(a, (uint64_t)q - 2, q); }

uint32_t oracle_bitrev(uint32_t x, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

int oracle_is_prime(uint64_t n) {
  if (n < 2) return 0;
  for (uint64_t d = 2; d * d <= n; d++)
    if (n % d == 0) return 0;
  return 1;
}

int oracle_gen_primes(uint32_t log_n, uint32_t count, uint32_t *out) {
  const uint64_t two_n = 2ull << log_n;
  uint32_t found = 0;
  for (uint64_t t = 1; found < count; t++) {
    if (t * two_n >= (1ull << 29)) return -1; /* stay above 2^29 */
    uint64_t c = (1ull << 30) - t * two_n + 1;
    if (oracle_is_prime(c)) out[found++] = (uint32_t)c;
  }
  return 0;
}

int oracle_moduli(const oracle_params *p, uint32_t *out) {
  uint32_t total = p->num_q + p->num_p;
  uint32_t *pr = (uint32_t *)malloc(sizeof(uint32_t) * total);
  if (!pr) return -1;
  if (oracle_gen_primes(p->log_n, total, pr) != 0) { free(pr); return -1; }
  for (uint32_t i = 0; i < p->num_q; i++) out[i] = pr[p->num_p + i];
  for (uint32_t k = 0; k < p->num_p; k++) out[p->num_q + k] = pr[k];
  free(pr);
  return 0;
}

static uint32_t min_psi_search(uint32_t q, uint32_t log_n) {
  const uint64_t n = 1ull << log_n;
  for (uint32_t x = 2; x < q; x++)
    if (oracle_powmod(x, n, q) == q - 1) return x;
  return 0;
}

/* The search is slow for small N, so results are remembered per (q, log_n). */
uint32_t oracle_min_psi(uint32_t q, uint32_t log_n) {
  static uint32_t cq[512], cl[512], cv[512];
  static unsigned used = 0;
  for (unsigned i = 0; i < used; i++)
    if (cq[i] == q && cl[i] == log_n) return cv[i];
  uint32_t v = min_psi_search(q, log_n);
  if (used < 512) { cq[used] = q; cl[used] = log_n; cv[used] = v; used++; }
  return v;
}

/* ------------------------------------------------------------------ */
/* NTT                                                                  */
/* ------------------------------------------------------------------ */

/* Definition: evaluation of a(X) at psi^(2*brv(j)+1), by Horner's rule. */
void oracle_ntt_direct(const uint32_t *a, uint32_t *out, uint32_t log_n, uint32_t q, uint32_t psi) {
  const uint32_t n = 1u << log_n;
  for (uint32_t j = 0; j < n; j++) {
    uint32_t x = oracle_powmod(psi, 2ull * oracle_bitrev(j, log_n) + 1, q);
    uint32_t acc = 0;
    for (uint32_t i = n; i-- > 0;) acc = addmod(mulmod(acc, x, q), a[i], q);
    out[j] = acc;
  }
}

/* Textbook cyclic DFT over Z_q, radix-2 decimation in time:
 * A[k] = sum_i a[i] * w^(i*k), natural order in and out. */
static void cyclic_dft(uint32_t *a, uint32_t log_n, uint32_t q, uint32_t w) {
  const uint32_t n = 1u << log_n;
  for (uint32_t i = 0; i < n; i++) {
    uint32_t r = oracle_bitrev(i, log_n);
    if (i < r) { uint32_t t = a[i]; a[i] = a[r]; a[r] = t; }
  }
  for (uint32_t len = 2; len <= n; len <<= 1) {
    uint32_t wl = oracle_powmod(w, n / len, q);
    for (uint32_t s = 0; s < n; s += len) {
      uint32_t wk = 1;
      for (uint32_t k = 0; k < len / 2; k++) {
        uint32_t u = a[s + k];
        uint32_t v = mulmod(a[s + k + len / 2], wk, q);
        a[s + k] = addmod(u, v, q);
        a[s + k + len / 2] = submod(u, v, q);
        wk = mulmod(wk, wl, q);
      }
    }
  }
}

/* a(psi^(2b+1)) = sum_i (a_i psi^i) (psi^2)^(b i): twist by psi^i, take the
 * cyclic DFT with w = psi^2, and list entry brv(j) at position j. */
void oracle_ntt(uint32_t *a, uint32_t log_n, uint32_t q, uint32_t psi) {
  const uint32_t n = 1u << log_n;
  uint32_t *t = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t pw = 1;
  for (uint32_t i = 0; i < n; i++) { t[i] = mulmod(a[i], pw, q); pw = mulmod(pw, psi, q); }
  cyclic_dft(t, log_n, q, mulmod(psi, psi, q));
  for (uint32_t j = 0; j < n; j++) a[j] = t[oracle_bitrev(j, log_n)];
  free(t);
}

/* Inverse of oracle_ntt: undo the listing order, inverse cyclic DFT
 * (w^-1 and a factor N^-1), then untwist by psi^-i. */
void oracle_intt(uint32_t *a, uint32_t log_n, uint32_t q, uint32_t psi) {
  const uint32_t n = 1u << log_n;
  uint32_t *t = (uint32_t *)malloc(sizeof(uint32_t) * n);
  for (uint32_t k = 0; k < n; k++) t[k] = a[oracle_bitrev(k, log_n)];
  uint32_t psi_inv = oracle_invmod(psi, q);
  cyclic_dft(t, log_n, q, mulmod(psi_inv, psi_inv, q));
  uint32_t n_inv = oracle_invmod(n % q, q), pw = 1;
  for (uint32_t i = 0; i < n; i++) {
    a[i] = mulmod(mulmod(t[i], n_inv, q), pw, q);
    pw = mulmod(pw, psi_inv, q);
  }
  free(t);
}

void oracle_negacyclic_mul(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t log_n, uint32_t q) {
  const uint32_t n = 1u << log_n;
  for (uint32_t k = 0; k < n; k++) c[k] = 0;
  for (uint32_t i = 0; i < n; i++)
    for (uint32_t j = 0; j < n; j++) {
      uint32_t prod = mulmod(a[i], b[j], q);
      if (i + j < n) c[i + j] = addmod(c[i + j], prod, q);
      else c[i + j - n] = submod(c[i + j - n], prod, q); /* X^N = -1 */
    }
}

/* ------------------------------------------------------------------ */
/* basis conversion                                                     */
/* ------------------------------------------------------------------ */

/* [prod_{i != skip} src_i]_m */
static uint32_t prod_except(const uint32_t *src, uint32_t ns, uint32_t skip, uint32_t m) {
  uint32_t r = 1 % m;
  for (uint32_t i = 0; i < ns; i++)
    if (i != skip) r = mulmod(r, src[i] % m, m);
  return r;
}

void oracle_bconv(const uint32_t *x, const uint32_t *src, uint32_t ns,
                  uint32_t *y, const uint32_t *dst, uint32_t nt, uint32_t n) {
  uint32_t *xt = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)ns * n);
  /* [x_i * (S/s_i)^-1]_{s_i} */
  for (uint32_t i = 0; i < ns; i++) {
    uint32_t c = oracle_invmod(prod_except(src, ns, i, src[i]), src[i]);
    for (uint32_t z = 0; z < n; z++) xt[(size_t)i * n + z] = mulmod(x[(size_t)i * n + z], c, src[i]);
  }
  for (uint32_t t = 0; t < nt; t++) {
    const uint32_t m = dst[t];
    for (uint32_t z = 0; z < n; z++) y[(size_t)t * n + z] = 0;
    for (uint32_t i = 0; i < ns; i++) {
      uint32_t ii = (g_fault == 3 && ns > 1) ? (i + 1) % ns : i;
      uint32_t c = prod_except(src, ns, ii, m);
      for (uint32_t z = 0; z < n; z++)
        y[(size_t)t * n + z] = addmod(y[(size_t)t * n + z], mulmod(xt[(size_t)i * n + z], c, m), m);
    }
  }
  free(xt);
}

/* ------------------------------------------------------------------ */
/* hybrid key switching                                                 */
/* ------------------------------------------------------------------ */

uint64_t oracle_evk_words(uint32_t log_n, uint32_t num_q, uint32_t num_p, uint32_t dnum) {
  return (uint64_t)dnum * 2ull * (uint64_t)(num_q + num_p) << log_n;
}

typedef struct {
  uint32_t n, log_n, L1, K, dnum, alpha, level, ntow, ndig;
  uint32_t q[160];    /* extended basis D_l: q_0..q_l, p_0..p_{K-1} */
  uint32_t evk_limb[160]; /* limb index of D_l tower t inside the evk */
  uint32_t psi[160];
} ks_ctx;

static int ctx_init(ks_ctx *c, const oracle_params *p, const uint32_t *moduli, uint32_t level) {
  if (p->log_n < 1 || p->log_n > 17 || p->num_q == 0 || p->dnum == 0 || p->dnum > p->num_q ||
      p->num_p == 0 || level >= p->num_q || p->num_q + p->num_p > 160)
    return -1;
  c->log_n = p->log_n;
  c->n = 1u << p->log_n;
  c->L1 = p->num_q;
  c->K = p->num_p;
  c->dnum = p->dnum;
  c->alpha = (p->num_q + p->dnum - 1) / p->dnum;  /* Table I: ceil((L+1)/dnum) */
  c->level = level;
  c->ntow = level + 1 + p->num_p;
  c->ndig = (level + 1 + c->alpha - 1) / c->alpha; /* digits holding a live tower */
  for (uint32_t i = 0; i <= level; i++) { c->q[i] = moduli[i]; c->evk_limb[i] = i; }
  for (uint32_t k = 0; k < p->num_p; k++) {
    c->q[level + 1 + k] = moduli[p->num_q + k];
    c->evk_limb[level + 1 + k] = p->num_q + k;
  }
  for (uint32_t t = 0; t < c->ntow; t++) c->psi[t] = oracle_min_psi(c->q[t], c->log_n);
  return 0;
}

static void digit_range(const ks_ctx *c, uint32_t j, uint32_t *lo, uint32_t *hi) {
  *lo = j * c->alpha;
  *hi = (j + 1) * c->alpha;
  if (*hi > c->level + 1) *hi = c->level + 1;
}

#define LIMB(buf, idx, n) ((buf) + (size_t)(idx) * (n))

/* ModDown, Sec. III-C, for one polynomial t: acc holds [ntow][N] (evaluation
 * domain, towers of D_l), out receives [level+1][N]. */
static void moddown(const ks_ctx *c, const uint32_t *acc, uint32_t *out) {
  const uint32_t n = c->n, l1 = c->level + 1, K = c->K;
  uint32_t *a = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)K * n);
  uint32_t *w = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)l1 * n);
  /* P1: INTT of the last K towers */
  for (uint32_t k = 0; k < K; k++) {
    memcpy(LIMB(a, k, n), LIMB(acc, l1 + k, n), sizeof(uint32_t) * n);
    oracle_intt(LIMB(a, k, n), c->log_n, c->q[l1 + k], c->psi[l1 + k]);
  }
  /* P2: basis conversion P -> Q_l */
  oracle_bconv(a, &c->q[l1], K, w, c->q, l1, n);
  /* P3: NTT of the l+1 converted towers; P4: subtract, times P^-1 */
  for (uint32_t i = 0; i < l1; i++) {
    const uint32_t qi = c->q[i];
    oracle_ntt(LIMB(w, i, n), c->log_n, qi, c->psi[i]);
    uint32_t p_mod = 1;
    for (uint32_t k = 0; k < K; k++) p_mod = mulmod(p_mod, c->q[l1 + k] % qi, qi);
    uint32_t p_inv = oracle_invmod(p_mod, qi);
    for (uint32_t z = 0; z < n; z++) {
      uint32_t diff = (g_fault == 2) ? addmod(LIMB(acc, i, n)[z], LIMB(w, i, n)[z], qi)
                                     : submod(LIMB(acc, i, n)[z], LIMB(w, i, n)[z], qi);
      LIMB(out, i, n)[z] = mulmod(diff, p_inv, qi);
    }
  }
  free(a);
  free(w);
}

/* ModUp P1-P3 (Sec. III-B) of d [level+1][N]: x receives the INTT of
 * every input tower, y[j][t] ([D][T][N], evaluation domain) digit j
 * extended to every tower of D_l, the digit's own towers copied from d.
 * tgt [T][N] and tq [T] are scratch. */
static void modup(const ks_ctx *cc, const uint32_t *d, uint32_t *x, uint32_t *y, uint32_t *tgt, uint32_t *tq) {
  const ks_ctx c = *cc;
  const uint32_t n = c.n, l1 = c.level + 1, T = c.ntow, D = c.ndig;
  memcpy(x, d, sizeof(uint32_t) * (size_t)l1 * n);
  for (uint32_t i = 0; i < l1; i++) oracle_intt(LIMB(x, i, n), c.log_n, c.q[i], c.psi[i]);
  for (uint32_t j = 0; j < D; j++) {
    uint32_t lo, hi;
    digit_range(&c, j, &lo, &hi);
    /* P2: extend digit j from its towers S_j to every other tower of D_l */
    uint32_t nt = 0;
    for (uint32_t t = 0; t < T; t++)
      if (t < lo || t >= hi) tq[nt++] = c.q[t];
    oracle_bconv(LIMB(x, lo, n), &c.q[lo], hi - lo, tgt, tq, nt, n);
    /* P3: NTT of the extended towers, concatenated with the digit itself */
    uint32_t u = 0;
    for (uint32_t t = 0; t < T; t++) {
      uint32_t *dst = LIMB(y, (size_t)j * T + t, n);
      if (t >= lo && t < hi) {
        uint32_t src = t;
        if (g_fault == 4 && D > 1) src = (t + c.alpha) % l1;
        memcpy(dst, LIMB(d, src, n), sizeof(uint32_t) * n);
      } else {
        memcpy(dst, LIMB(tgt, u, n), sizeof(uint32_t) * n);
        oracle_ntt(dst, c.log_n, c.q[t], c.psi[t]);
        u++;
      }
    }
  }
}

int oracle_keyswitch(const oracle_params *p, const uint32_t *moduli, uint32_t level,
                     const uint32_t *evk, const uint32_t *d, uint32_t *out) {
  ks_ctx c;
  if (ctx_init(&c, p, moduli, level) != 0) return -1;
  const uint32_t n = c.n, l1 = level + 1, T = c.ntow, D = c.ndig, EL = c.L1 + c.K;
  /* ModUp P1: INTT of every input tower */
  uint32_t *x = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)l1 * n);
  /* ModUp P2/P3 output, one [T][N] block per digit: y[j][t] */
  uint32_t *y = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)D * T * n);
  uint32_t *acc = (uint32_t *)calloc((size_t)2 * T * n, sizeof(uint32_t));
  uint32_t *tgt = (uint32_t *)malloc(sizeof(uint32_t) * T * n);
  uint32_t *tq = (uint32_t *)malloc(sizeof(uint32_t) * T);
  if (!x || !y || !acc || !tgt || !tq) { free(x); free(y); free(acc); free(tgt); free(tq); return -1; }

  modup(&c, d, x, y, tgt, tq);
  /* P4: apply the key, P5: sum over digits */
  for (uint32_t j = 0; j < D; j++) {
    if (g_fault == 1 && j == D - 1 && D > 1) continue;
    for (uint32_t s = 0; s < 2; s++)
      for (uint32_t t = 0; t < T; t++) {
        const uint32_t *ek = evk + (((size_t)j * 2 + s) * EL + c.evk_limb[t]) * n;
        const uint32_t *yy = LIMB(y, (size_t)j * T + t, n);
        uint32_t *aa = LIMB(acc, (size_t)s * T + t, n);
        for (uint32_t z = 0; z < n; z++) aa[z] = addmod(aa[z], mulmod(yy[z], ek[z], c.q[t]), c.q[t]);
      }
  }
  /* ModDown P1-P4 for both polynomials */
  for (uint32_t s = 0; s < 2; s++) moddown(&c, LIMB(acc, (size_t)s * T, n), LIMB(out, (size_t)s * l1, n));
  free(x); free(y); free(acc); free(tgt); free(tq);
  return 0;
}
/* Output-Centric order (Sec. IV-C): INTT outputs kept, then one output tower
 * at a time.  Section 2 (the P towers, every digit extended) comes first so
 * their INTT (ModDown P1) is available; then each Q tower takes the other
 * digits through P2/P3, bypasses its own digit, accumulates P4/P5, and goes
 * through ModDown P2-P4 for that single tower. */
int oracle_keyswitch_oc(const oracle_params *p, const uint32_t *moduli, uint32_t level,
                        const uint32_t *evk, const uint32_t *d, uint32_t *out) {
  ks_ctx c;
  if (ctx_init(&c, p, moduli, level) != 0) return -1;
  const uint32_t n = c.n, l1 = level + 1, K = c.K, D = c.ndig, EL = c.L1 + c.K;
  uint32_t *x = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)l1 * n);
  uint32_t *ap = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)2 * K * n); /* ModDown P1 output */
  uint32_t *one = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t *acc = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)2 * n);
  if (!x || !ap || !one || !acc) { free(x); free(ap); free(one); free(acc); return -1; }
  memcpy(x, d, sizeof(uint32_t) * (size_t)l1 * n);
  for (uint32_t i = 0; i < l1; i++) oracle_intt(LIMB(x, i, n), c.log_n, c.q[i], c.psi[i]);

  for (uint32_t pass = 0; pass < 2; pass++) {           /* 0: P towers, 1: Q towers */
    uint32_t t0 = pass == 0 ? l1 : 0, t1 = pass == 0 ? l1 + K : l1;
    for (uint32_t t = t0; t < t1; t++) {
      const uint32_t m = c.q[t];
      memset(acc, 0, sizeof(uint32_t) * 2 * n);
      for (uint32_t j = 0; j < D; j++) {
        uint32_t lo, hi;
        digit_range(&c, j, &lo, &hi);
        if (t >= lo && t < hi) memcpy(one, LIMB(d, t, n), sizeof(uint32_t) * n); /* bypass */
        else {
          oracle_bconv(LIMB(x, lo, n), &c.q[lo], hi - lo, one, &m, 1, n);
          oracle_ntt(one, c.log_n, m, c.psi[t]);
        }
        for (uint32_t s = 0; s < 2; s++) {
          const uint32_t *ek = evk + (((size_t)j * 2 + s) * EL + c.evk_limb[t]) * n;
          for (uint32_t z = 0; z < n; z++) acc[s * n + z] = addmod(acc[s * n + z], mulmod(one[z], ek[z], m), m);
        }
      }
      for (uint32_t s = 0; s < 2; s++) {
        if (pass == 0) {
          memcpy(LIMB(ap, (size_t)s * K + (t - l1), n), acc + s * n, sizeof(uint32_t) * n);
          oracle_intt(LIMB(ap, (size_t)s * K + (t - l1), n), c.log_n, m, c.psi[t]);
        } else {
          oracle_bconv(LIMB(ap, (size_t)s * K, n), &c.q[l1], K, one, &m, 1, n);
          oracle_ntt(one, c.log_n, m, c.psi[t]);
          uint32_t p_mod = 1;
          for (uint32_t k = 0; k < K; k++) p_mod = mulmod(p_mod, c.q[l1 + k] % m, m);
          uint32_t p_inv = oracle_invmod(p_mod, m);
          uint32_t *o = LIMB(out, (size_t)s * l1 + t, n);
          for (uint32_t z = 0; z < n; z++) o[z] = mulmod(submod(acc[s * n + z], one[z], m), p_inv, m);
        }
      }
    }
  }
  free(x); free(ap); free(one); free(acc);
  return 0;
}

/* ------------------------------------------------------------------ */
/* key generation                                                       */
/* ------------------------------------------------------------------ */

/* xoshiro256** (Blackman & Vigna), seeded through splitmix64. */
typedef struct { uint64_t s[4]; } rng_t;
static uint64_t splitmix64(uint64_t *x) {
  uint64_t z = (*x += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static uint64_t rng_next(rng_t *r) {
  uint64_t res = rotl(r->s[1] * 5, 7) * 9, t = r->s[1] << 17;
  r->s[2] ^= r->s[0]; r->s[3] ^= r->s[1]; r->s[1] ^= r->s[2]; r->s[0] ^= r->s[3];
  r->s[2] ^= t; r->s[3] = rotl(r->s[3], 45);
  return res;
}
static void rng_seed(rng_t *r, uint64_t seed) { for (int i = 0; i < 4; i++) r->s[i] = splitmix64(&seed); }
/* uniform in [0, m) by rejection */
static uint32_t rng_below(rng_t *r, uint32_t m) {
  uint64_t lim = (UINT64_MAX / m) * m;
  for (;;) { uint64_t v = rng_next(r); if (v < lim) return (uint32_t)(v % m); }
}
static double rng_unit(rng_t *r) { return ((rng_next(r) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
static int32_t rng_gauss(rng_t *r) { /* Box-Muller, sigma 3.2, clamp 19 */
  double u1 = rng_unit(r), u2 = rng_unit(r);
  double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  long e = lround(3.2 * z);
  if (e > 19) e = 19;
  if (e < -19) e = -19;
  return (int32_t)e;
}
static uint32_t signed_mod(int32_t v, uint32_t m) { return v >= 0 ? (uint32_t)v % m : m - ((uint32_t)(-v) % m); }

/* Seeded key halves (key compression, Sec. IV-D): the a half of every evk
 * pair comes from a counter-based generator instead of being stored.  The
 * generator is SplitMix64 (Steele, Lea and Flood 2014) used at a counter:
 * output t of seed s is the SplitMix64 output mix of s + (t + 1) * gamma.
 * Word (j, g, k) of the a halves is a = x * 2^-32 mod m_g, x the output at
 * t = (j * (L+1+K) + g) * N + k. */
uint64_t oracle_splitmix_at(uint64_t seed, uint64_t t) {
  uint64_t x = seed + t * 0x9e3779b97f4a7c15ull;
  return splitmix64(&x);
}

int oracle_seeded_a(const oracle_params *p, const uint32_t *moduli, uint64_t a_seed, uint32_t *evk) {
  if (!p || !moduli || !evk) return -1;
  const uint32_t n = 1u << p->log_n;
  const uint32_t alpha = (p->num_q + p->dnum - 1) / p->dnum;
  const uint32_t K = p->num_p ? p->num_p : alpha, EL = p->num_q + K;
  for (uint32_t j = 0; j < p->dnum; j++)
    for (uint32_t g = 0; g < EL; g++) {
      const uint32_t m = moduli[g]; /* moduli[] and the key rows share the order q_0..q_L, p_0..p_{K-1} */
      const uint32_t inv32 = oracle_invmod((uint32_t)((1ull << 32) % m), m);
      uint32_t *a = evk + (((size_t)j * 2 + 1) * EL + g) * n;
      for (uint32_t k = 0; k < n; k++) {
        const uint64_t x = oracle_splitmix_at(a_seed, ((uint64_t)j * EL + g) * n + k);
        a[k] = mulmod((uint32_t)(x % m), inv32, m);
      }
    }
  return 0;
}

/* s2 of a key: KG_RANDOM a fresh ternary secret, KG_ROTATE sigma_k(s) (the
 * key of a rotation), KG_RELIN s^2 (the key of a multiplication). */
enum { KG_RANDOM = 0, KG_ROTATE = 1, KG_RELIN = 2 };
static int keygen_impl(const oracle_params *p, const uint32_t *moduli, uint64_t seed, int seeded, int mode,
                       uint32_t galois, int8_t *s, int8_t *s2, uint32_t *evk);

int oracle_keygen(const oracle_params *p, const uint32_t *moduli, uint64_t seed,
                  int8_t *s, int8_t *s2, uint32_t *evk) {
  return keygen_impl(p, moduli, seed, 0, KG_RANDOM, 0, s, s2, evk);
}

int oracle_keygen_rotation(const oracle_params *p, const uint32_t *moduli, uint64_t seed, uint32_t galois,
                           int8_t *s, int8_t *s2, uint32_t *evk) {
  const uint32_t two_n = 2u << p->log_n;
  if ((galois & 1u) == 0 || galois >= two_n) return -1;
  return keygen_impl(p, moduli, seed, 0, KG_ROTATE, galois, s, s2, evk);
}

int oracle_keygen_relin(const oracle_params *p, const uint32_t *moduli, uint64_t seed, int8_t *s, uint32_t *evk) {
  int8_t *s2 = (int8_t *)malloc((size_t)1 << p->log_n);
  if (!s2) return -1;
  const int h = keygen_impl(p, moduli, seed, 0, KG_RELIN, 0, s, s2, evk);
  free(s2);
  return h;
}

int oracle_keygen_seeded(const oracle_params *p, const uint32_t *moduli, uint64_t seed, uint64_t a_seed,
                         int8_t *s, int8_t *s2, uint32_t *evk) {
  if (oracle_seeded_a(p, moduli, a_seed, evk) != 0) return -1;
  return keygen_impl(p, moduli, seed, 1, KG_RANDOM, 0, s, s2, evk);
}

/* ------------------------------------------------------------------ */
/* callers of the key switch: rotation and multiplication (Sec. II)     */
/* ------------------------------------------------------------------ */

/* The CKKS automorphism a(X) -> a(X^k), k odd (rotation by r slots uses
 * k = 5^r mod 2N, conjugation k = 2N - 1; Cheon, Kim, Kim and Song 2017).
 * Coefficient domain: X^i maps to X^(i k mod 2N) = -X^(i k mod 2N - N)
 * past N, since X^N = -1. */
int oracle_automorphism_coeff(const uint32_t *a, uint32_t log_n, uint32_t galois, uint32_t q, uint32_t *out) {
  const uint32_t n = 1u << log_n, two_n = 2 * n;
  if ((galois & 1u) == 0 || galois >= two_n) return -1;
  for (uint32_t i = 0; i < n; i++) {
    const uint32_t e = (uint32_t)(((uint64_t)i * galois) % two_n);
    if (e < n) out[e] = a[i];
    else out[e - n] = a[i] ? q - a[i] : 0;
  }
  return 0;
}

/* Evaluation domain: slot j holds a(psi^(2 brv(j) + 1)), so the slot of
 * a(X^k) at that point holds a at psi^(k (2 brv(j) + 1)), i.e. slot j' with
 * 2 brv(j') + 1 = k (2 brv(j) + 1) mod 2N: a permutation, the same for
 * every modulus. */
int oracle_automorphism_eval(const uint32_t *a, uint32_t log_n, uint32_t galois, uint32_t *out) {
  const uint32_t n = 1u << log_n, two_n = 2 * n;
  if ((galois & 1u) == 0 || galois >= two_n) return -1;
  for (uint32_t j = 0; j < n; j++) {
    const uint32_t e = 2 * oracle_bitrev(j, log_n) + 1;
    const uint32_t e2 = (uint32_t)(((uint64_t)galois * e) % two_n);
    out[j] = a[oracle_bitrev((e2 - 1) / 2, log_n)];
  }
  return 0;
}

/* Rotations of one ciphertext (c0, c1) at `level` (evaluation domain) by
 * `count` Galois elements, sharing one ModUp (hoisting: the automorphism is
 * a permutation of the evaluation domain that commutes with the key
 * product, so the extended digits of c1 are computed once and permuted per
 * rotation; double hoisting is named in Sec. VII).  Rotation r:
 *   acc_s = sum_j sigma_r(y_j) * evk_r[j][s]   (ModUp P4/P5 on permuted digits)
 *   out_r = (ModDown(acc_0) + sigma_r(c0), ModDown(acc_1))
 * where y_j are the ModUp P1-P3 outputs of c1.  evk_r switches from
 * sigma_r(s) to s.  evks: count keys one after the other; outs: count
 * outputs [2][level+1][N]. */
int oracle_rotate_hoisted(const oracle_params *p, const uint32_t *moduli, uint32_t level, const uint32_t *c0,
                          const uint32_t *c1, uint32_t count, const uint32_t *galois, const uint32_t *evks,
                          uint32_t *outs) {
  ks_ctx c;
  if (ctx_init(&c, p, moduli, level) != 0) return -1;
  const uint32_t n = c.n, l1 = level + 1, T = c.ntow, D = c.ndig, EL = c.L1 + c.K;
  const size_t evk_words = (size_t)p->dnum * 2 * EL * n;
  for (uint32_t r = 0; r < count; r++)
    if ((galois[r] & 1u) == 0 || galois[r] >= 2 * n) return -1;
  uint32_t *x = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)l1 * n);
  uint32_t *y = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)D * T * n);
  uint32_t *acc = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)2 * T * n);
  uint32_t *tgt = (uint32_t *)malloc(sizeof(uint32_t) * T * n);
  uint32_t *tq = (uint32_t *)malloc(sizeof(uint32_t) * T);
  uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * n);
  if (!x || !y || !acc || !tgt || !tq || !perm) {
    free(x); free(y); free(acc); free(tgt); free(tq); free(perm);
    return -1;
  }
  modup(&c, c1, x, y, tgt, tq);
  for (uint32_t r = 0; r < count; r++) {
    const uint32_t *evk = evks + r * evk_words;
    uint32_t *out = outs + (size_t)r * 2 * l1 * n;
    memset(acc, 0, sizeof(uint32_t) * (size_t)2 * T * n);
    for (uint32_t j = 0; j < D; j++)
      for (uint32_t t = 0; t < T; t++) {
        if (g_fault == 1 && j == D - 1 && D > 1) continue;
        oracle_automorphism_eval(LIMB(y, (size_t)j * T + t, n), c.log_n, galois[r], perm);
        if (g_fault == 5) { /* the inverse permutation: scatter where a gather belongs */
          for (uint32_t z = 0; z < n; z++) perm[z] = 0;
          for (uint32_t z = 0; z < n; z++) {
            const uint32_t e2 = (uint32_t)(((uint64_t)galois[r] * (2 * oracle_bitrev(z, c.log_n) + 1)) % (2 * n));
            perm[oracle_bitrev((e2 - 1) / 2, c.log_n)] = LIMB(y, (size_t)j * T + t, n)[z];
          }
        }
        for (uint32_t s = 0; s < 2; s++) {
          const uint32_t *ek = evk + (((size_t)j * 2 + s) * EL + c.evk_limb[t]) * n;
          uint32_t *aa = LIMB(acc, (size_t)s * T + t, n);
          for (uint32_t z = 0; z < n; z++) aa[z] = addmod(aa[z], mulmod(perm[z], ek[z], c.q[t]), c.q[t]);
        }
      }
    for (uint32_t s = 0; s < 2; s++) moddown(&c, LIMB(acc, (size_t)s * T, n), LIMB(out, (size_t)s * l1, n));
    for (uint32_t i = 0; i < l1; i++) {
      oracle_automorphism_eval(LIMB(c0, i, n), c.log_n, galois[r], perm);
      for (uint32_t z = 0; z < n; z++) LIMB(out, i, n)[z] = addmod(LIMB(out, i, n)[z], perm[z], c.q[i]);
    }
  }
  free(x); free(y); free(acc); free(tgt); free(tq); free(perm);
  return 0;
}

/* Double hoisting (named in Sec. VII): a sum of rotations, each optionally
 * times a plaintext diagonal p_r, with one ModUp of c1 and one ModDown for
 * the whole sum:
 *   ACC_s = sum_r p_r * sum_j sigma_r(y_j) * evk_r[j][s]   (extended basis)
 *   out   = (ModDown(ACC_0) + sum_r p_r * sigma_r(c0), ModDown(ACC_1))
 * diags: null (every p_r = 1) or [count][L+1+K][N] in key-row order
 * (q_0..q_L, p_0..p_{K-1}; evaluation domain). */
int oracle_rotate_sum_hoisted(const oracle_params *p, const uint32_t *moduli, uint32_t level, const uint32_t *c0,
                              const uint32_t *c1, uint32_t count, const uint32_t *galois, const uint32_t *evks,
                              const uint32_t *diags, uint32_t *out) {
  ks_ctx c;
  if (ctx_init(&c, p, moduli, level) != 0) return -1;
  const uint32_t n = c.n, l1 = level + 1, T = c.ntow, D = c.ndig, EL = c.L1 + c.K;
  const size_t evk_words = (size_t)p->dnum * 2 * EL * n, diag_words = (size_t)EL * n;
  for (uint32_t r = 0; r < count; r++)
    if ((galois[r] & 1u) == 0 || galois[r] >= 2 * n) return -1;
  uint32_t *x = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)l1 * n);
  uint32_t *y = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)D * T * n);
  uint32_t *acc = (uint32_t *)calloc((size_t)2 * T * n, sizeof(uint32_t));
  uint32_t *tgt = (uint32_t *)malloc(sizeof(uint32_t) * T * n);
  uint32_t *tq = (uint32_t *)malloc(sizeof(uint32_t) * T);
  uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t *one = (uint32_t *)malloc(sizeof(uint32_t) * n);
  if (!x || !y || !acc || !tgt || !tq || !perm || !one) {
    free(x); free(y); free(acc); free(tgt); free(tq); free(perm); free(one);
    return -1;
  }
  modup(&c, c1, x, y, tgt, tq);
  for (uint32_t r = 0; r < count; r++) {
    const uint32_t *evk = evks + r * evk_words;
    for (uint32_t t = 0; t < T; t++) {
      const uint32_t m = c.q[t];
      const uint32_t *pr = diags ? diags + r * diag_words + (size_t)c.evk_limb[t] * n : NULL;
      for (uint32_t s = 0; s < 2; s++) {
        memset(one, 0, sizeof(uint32_t) * n); /* this rotation's key product, tower t */
        for (uint32_t j = 0; j < D; j++) {
          if (g_fault == 1 && j == D - 1 && D > 1) continue;
          oracle_automorphism_eval(LIMB(y, (size_t)j * T + t, n), c.log_n, galois[r], perm);
          if (g_fault == 5) /* the inverse permutation: scatter where a gather belongs */
            for (uint32_t z = 0; z < n; z++) {
              const uint32_t e2 = (uint32_t)(((uint64_t)galois[r] * (2 * oracle_bitrev(z, c.log_n) + 1)) % (2 * n));
              perm[oracle_bitrev((e2 - 1) / 2, c.log_n)] = LIMB(y, (size_t)j * T + t, n)[z];
            }
          const uint32_t *ek = evk + (((size_t)j * 2 + s) * EL + c.evk_limb[t]) * n;
          for (uint32_t z = 0; z < n; z++) one[z] = addmod(one[z], mulmod(perm[z], ek[z], m), m);
        }
        uint32_t *aa = LIMB(acc, (size_t)s * T + t, n);
        for (uint32_t z = 0; z < n; z++) aa[z] = addmod(aa[z], pr ? mulmod(pr[z], one[z], m) : one[z], m);
      }
    }
  }
  for (uint32_t s = 0; s < 2; s++) moddown(&c, LIMB(acc, (size_t)s * T, n), LIMB(out, (size_t)s * l1, n));
  for (uint32_t r = 0; r < count; r++)
    for (uint32_t i = 0; i < l1; i++) {
      const uint32_t *pr = diags ? diags + r * diag_words + (size_t)i * n : NULL;
      oracle_automorphism_eval(LIMB(c0, i, n), c.log_n, galois[r], perm);
      for (uint32_t z = 0; z < n; z++)
        LIMB(out, i, n)[z] = addmod(LIMB(out, i, n)[z], pr ? mulmod(pr[z], perm[z], c.q[i]) : perm[z], c.q[i]);
    }
  free(x); free(y); free(acc); free(tgt); free(tq); free(perm); free(one);
  return 0;
}

/* One rotation without hoisting: permute c0 and c1, key-switch sigma(c1),
 * add sigma(c0).  A different, equally valid result (the ModUp of sigma(c1)
 * differs from sigma of the ModUp of c1 by multiples of Q_j). */
int oracle_rotate(const oracle_params *p, const uint32_t *moduli, uint32_t level, const uint32_t *c0,
                  const uint32_t *c1, uint32_t galois, const uint32_t *evk, uint32_t *out) {
  const uint32_t n = 1u << p->log_n, l1 = level + 1;
  if ((galois & 1u) == 0 || galois >= 2 * n || level >= p->num_q) return -1;
  uint32_t *sc1 = (uint32_t *)calloc((size_t)l1 * n, sizeof(uint32_t));
  uint32_t *sc0 = (uint32_t *)calloc((size_t)l1 * n, sizeof(uint32_t));
  if (!sc1 || !sc0) { free(sc1); free(sc0); return -1; }
  int rc = 0;
  for (uint32_t i = 0; i < l1; i++) {
    rc |= oracle_automorphism_eval(LIMB(c1, i, n), p->log_n, galois, LIMB(sc1, i, n));
    rc |= oracle_automorphism_eval(LIMB(c0, i, n), p->log_n, galois, LIMB(sc0, i, n));
  }
  if (rc == 0) rc = oracle_keyswitch(p, moduli, level, evk, sc1, out);
  for (uint32_t i = 0; rc == 0 && i < l1; i++)
    for (uint32_t z = 0; z < n; z++) LIMB(out, i, n)[z] = addmod(LIMB(out, i, n)[z], LIMB(sc0, i, n)[z], moduli[i]);
  free(sc1); free(sc0);
  return rc;
}

/* Multiplication with relinearisation: the tensor product of (a0, a1) and
 * (b0, b1) (pointwise in the evaluation domain) is d0 = a0 b0,
 * d1 = a0 b1 + a1 b0, d2 = a1 b1, decryptable with (1, s, s^2); the key
 * switch of d2 with a key from s^2 to s brings it back:
 * out = (d0 + KS(d2)_0, d1 + KS(d2)_1). */
int oracle_mult_relin(const oracle_params *p, const uint32_t *moduli, uint32_t level, const uint32_t *a0,
                      const uint32_t *a1, const uint32_t *b0, const uint32_t *b1, const uint32_t *evk, uint32_t *out) {
  const uint32_t n = 1u << p->log_n, l1 = level + 1;
  if (level >= p->num_q) return -1;
  uint32_t *d = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)3 * l1 * n);
  if (!d) return -1;
  for (uint32_t i = 0; i < l1; i++) {
    const uint32_t q = moduli[i];
    for (uint32_t z = 0; z < n; z++) {
      const size_t w = (size_t)i * n + z;
      d[w] = mulmod(a0[w], b0[w], q);
      d[(size_t)l1 * n + w] = addmod(mulmod(a0[w], b1[w], q), mulmod(a1[w], b0[w], q), q);
      d[(size_t)2 * l1 * n + w] = mulmod(a1[w], b1[w], q);
    }
  }
  int rc = oracle_keyswitch(p, moduli, level, evk, d + (size_t)2 * l1 * n, out);
  for (uint32_t h = 0; rc == 0 && h < 2; h++)
    for (uint32_t i = 0; i < l1; i++)
      for (uint32_t z = 0; z < n; z++) {
        const size_t w = ((size_t)h * l1 + i) * n + z;
        out[w] = addmod(out[w], d[w], moduli[i]);
      }
  free(d);
  return rc;
}

static int keygen_impl(const oracle_params *p, const uint32_t *moduli, uint64_t seed, int seeded, int mode,
                       uint32_t galois, int8_t *s, int8_t *s2, uint32_t *evk) {
  ks_ctx c;
  if (ctx_init(&c, p, moduli, p->num_q - 1) != 0) return -1;
  const uint32_t n = c.n, EL = c.L1 + c.K;
  rng_t r;
  rng_seed(&r, seed);
  int h = 0;
  for (uint32_t z = 0; z < n; z++) { s[z] = (int8_t)((int)rng_below(&r, 3) - 1); h += s[z] != 0; }
  for (uint32_t z = 0; z < n; z++) s2[z] = (int8_t)((int)rng_below(&r, 3) - 1);
  if (mode == KG_ROTATE) { /* s2 = s(X^k): coefficient i moves to i k mod 2N, negated past N */
    const uint32_t two_n = 2 * n;
    for (uint32_t i = 0; i < n; i++) {
      const uint32_t e = (uint32_t)(((uint64_t)i * galois) % two_n);
      if (e < n) s2[e] = s[i]; else s2[e - n] = (int8_t)-s[i];
    }
  }
  uint32_t *sh = (uint32_t *)malloc(sizeof(uint32_t) * n), *s2h = (uint32_t *)malloc(sizeof(uint32_t) * n);
  uint32_t *eh = (uint32_t *)malloc(sizeof(uint32_t) * n);
  int32_t *e = (int32_t *)malloc(sizeof(int32_t) * n);
  for (uint32_t j = 0; j < p->dnum; j++) {
    uint32_t lo = j * c.alpha, hi = (j + 1) * c.alpha;
    if (hi > c.L1) hi = c.L1;
    for (uint32_t z = 0; z < n; z++) e[z] = rng_gauss(&r);
    for (uint32_t g = 0; g < EL; g++) {
      const uint32_t m = c.q[g]; /* at level L the D_L order equals the evk order */
      for (uint32_t z = 0; z < n; z++) { sh[z] = signed_mod(s[z], m); s2h[z] = signed_mod(s2[z], m); eh[z] = signed_mod(e[z], m); }
      oracle_ntt(sh, c.log_n, m, c.psi[g]);
      oracle_ntt(s2h, c.log_n, m, c.psi[g]);
      if (mode == KG_RELIN) /* s^2 in the evaluation domain is the pointwise square */
        for (uint32_t z = 0; z < n; z++) s2h[z] = mulmod(sh[z], sh[z], m);
      oracle_ntt(eh, c.log_n, m, c.psi[g]);
      uint32_t gad = 0; /* [P]_m on digit j's own q-limbs */
      if (g >= lo && g < hi) {
        gad = 1;
        for (uint32_t k = 0; k < c.K; k++) gad = mulmod(gad, moduli[c.L1 + k] % m, m);
      }
      uint32_t *b = evk + (((size_t)j * 2 + 0) * EL + g) * n;
      uint32_t *a = evk + (((size_t)j * 2 + 1) * EL + g) * n;
      for (uint32_t z = 0; z < n; z++) {
        if (!seeded) a[z] = rng_below(&r, m); /* seeded: a already holds the generator's words */
        uint32_t v = submod(eh[z], mulmod(a[z], sh[z], m), m);
        b[z] = addmod(v, mulmod(gad, s2h[z], m), m);
      }
    }
  }
  free(sh); free(s2h); free(eh); free(e);
  return h;
}
