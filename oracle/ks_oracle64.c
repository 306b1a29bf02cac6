/*
 * ks_oracle64.c -- plain, slow CPU oracle for hybrid key switching with
 * 64-bit machine words (towers of ~60-bit primes, Sec. II word-size moduli).
 *
 * TEST INFRASTRUCTURE ONLY (see ks_oracle.h).  Residues are uint64 in
 * [0, m); every product is an exact unsigned __int128 followed by a plain
 * '%'.  There is no Montgomery, Shoup or Barrett arithmetic, no lazy range,
 * no fusion and no reordering beyond what each function's definition
 * states.  The HIP library must never include or link this file.
 *
 * Readings for 64-bit words (the paper names the word size only):
 *  - moduli: 2^60 - t*2N + 1 for t = 1, 2, ...; first K primes form P, the
 *    next L+1 form Q (as for the 30-bit towers);
 *  - psi: the smallest x with x^N = -1 (mod q).  The solutions of
 *    x^N = -1 are exactly the N odd powers of any one of them, so the
 *    smallest is found by listing those N powers: a search from 2 upward
 *    would take about q/N steps;
 *  - everything else as in ks_oracle.c: evaluation domain a(psi^(2brv(j)+1)),
 *    raw-limb digits with the gadget [P]_m in the key, fast basis conversion
 *    without correction, ModDown P4 as (acc - w_hat) * [P^-1]_{q_i}.
 */
#include "ks_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

static int g_fault64 = 0;
void oracle64_set_fault(int fault) { g_fault64 = fault; }
/* Planted mistakes (for tests of the checks, never set otherwise):
 *  1: ModUp P5 drops the last digit's contribution
 *  2: ModDown P4 adds w_hat instead of subtracting it
 *  3: ModUp P2 uses the wrong target constant (index off by one)
 *  4: ModUp P3 bypass takes the limb from the neighbouring digit */

/* ------------------------------------------------------------------ */
/* integers                                                             */
/* ------------------------------------------------------------------ */

static uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
static uint64_t addmod64(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + b) % q); }
static uint64_t submod64(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + q - (b % q)) % q); }

uint64_t oracle64_powmod(uint64_t b, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q, x = b % q;
  while (e) {
    if (e & 1) r = mulmod64(r, x, q);
    x = mulmod64(x, x, q);
    e >>= 1;
  }
  return r;
}

/* q prime: a^(q-2) is the inverse of a (Fermat). */
uint64_t oracle64_invmod(uint64_t a, uint64_t q) { return oracle64_powmod(a, q - 2, q); }

/* Miller-Rabin with the first twelve primes as bases: exact for every n
 * below 3.3e24, so for every 64-bit n. */
int oracle64_is_prime(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; i++) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; s++; }
  for (int i = 0; i < 12; i++) {
    uint64_t x = oracle64_powmod(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int witness = 1;
    for (int r = 1; r < s; r++) {
      x = mulmod64(x, x, n);
      if (x == n - 1) { witness = 0; break; }
    }
    if (witness) return 0;
  }
  return 1;
}

int oracle64_gen_primes(uint32_t log_n, uint32_t count, uint64_t *out) {
  const uint64_t two_n = 2ull << log_n;
  uint32_t found = 0;
  for (uint64_t t = 1; found < count; t++) {
    if (t * two_n >= (1ull << 59)) return -1; /* stay above 2^59 */
    const uint64_t c = (1ull << 60) - t * two_n + 1;
    if (oracle64_is_prime(c)) out[found++] = c;
  }
  return 0;
}

int oracle64_moduli(const oracle_params *p, uint64_t *out) {
  const uint32_t total = p->num_q + p->num_p;
  uint64_t *pr = (uint64_t *)malloc(sizeof(uint64_t) * total);
  if (!pr) return -1;
  if (oracle64_gen_primes(p->log_n, total, pr) != 0) { free(pr); return -1; }
  for (uint32_t i = 0; i < p->num_q; i++) out[i] = pr[p->num_p + i];
  for (uint32_t k = 0; k < p->num_p; k++) out[p->num_q + k] = pr[k];
  free(pr);
  return 0;
}

/* Smallest x with x^N = -1 (mod q).  c^((q-1)/2N) has order 2N exactly when
 * c^((q-1)/2) = -1 (c a quadratic non-residue, Euler's criterion); its odd
 * powers are all N solutions; the smallest of them is returned. */
uint64_t oracle64_min_psi(uint64_t q, uint32_t log_n) {
  const uint64_t n = 1ull << log_n, two_n = 2 * n;
  if ((q - 1) % two_n) return 0;
  uint64_t c = 2;
  while (oracle64_powmod(c, (q - 1) / 2, q) != q - 1) c++;
  const uint64_t root = oracle64_powmod(c, (q - 1) / two_n, q);
  const uint64_t sq = mulmod64(root, root, q);
  uint64_t best = root, x = root;
  for (uint64_t i = 1; i < n; i++) {
    x = mulmod64(x, sq, q);
    if (x < best) best = x;
  }
  return best;
}

/* ------------------------------------------------------------------ */
/* NTT                                                                  */
/* ------------------------------------------------------------------ */

/* Definition: evaluation of a(X) at psi^(2*brv(j)+1), by Horner's rule. */
void oracle64_ntt_direct(const uint64_t *a, uint64_t *out, uint32_t log_n, uint64_t q, uint64_t psi) {
  const uint32_t n = 1u << log_n;
  for (uint32_t j = 0; j < n; j++) {
    const uint64_t x = oracle64_powmod(psi, 2ull * oracle_bitrev(j, log_n) + 1, q);
    uint64_t acc = 0;
    for (uint32_t i = n; i-- > 0;) acc = addmod64(mulmod64(acc, x, q), a[i], q);
    out[j] = acc;
  }
}

/* Textbook cyclic DFT over Z_q, radix-2 decimation in time:
 * A[k] = sum_i a[i] * w^(i*k), natural order in and out. */
static void cyclic_dft64(uint64_t *a, uint32_t log_n, uint64_t q, uint64_t w) {
  const uint32_t n = 1u << log_n;
  for (uint32_t i = 0; i < n; i++) {
    const uint32_t r = oracle_bitrev(i, log_n);
    if (i < r) { const uint64_t t = a[i]; a[i] = a[r]; a[r] = t; }
  }
  for (uint32_t len = 2; len <= n; len <<= 1) {
    const uint64_t wl = oracle64_powmod(w, n / len, q);
    for (uint32_t s = 0; s < n; s += len) {
      uint64_t wk = 1;
      for (uint32_t k = 0; k < len / 2; k++) {
        const uint64_t u = a[s + k], v = mulmod64(a[s + k + len / 2], wk, q);
        a[s + k] = addmod64(u, v, q);
        a[s + k + len / 2] = submod64(u, v, q);
        wk = mulmod64(wk, wl, q);
      }
    }
  }
}

/* a(psi^(2b+1)) = sum_i (a_i psi^i) (psi^2)^(b i): twist by psi^i, cyclic
 * DFT with w = psi^2, entry brv(j) listed at position j. */
void oracle64_ntt(uint64_t *a, uint32_t log_n, uint64_t q, uint64_t psi) {
  const uint32_t n = 1u << log_n;
  uint64_t *t = (uint64_t *)malloc(sizeof(uint64_t) * n);
  uint64_t pw = 1;
  for (uint32_t i = 0; i < n; i++) { t[i] = mulmod64(a[i], pw, q); pw = mulmod64(pw, psi, q); }
  cyclic_dft64(t, log_n, q, mulmod64(psi, psi, q));
  for (uint32_t j = 0; j < n; j++) a[j] = t[oracle_bitrev(j, log_n)];
  free(t);
}

/* Inverse of oracle64_ntt: undo the listing order, inverse cyclic DFT (w^-1
 * and a factor N^-1), then untwist by psi^-i. */
void oracle64_intt(uint64_t *a, uint32_t log_n, uint64_t q, uint64_t psi) {
  const uint32_t n = 1u << log_n;
  uint64_t *t = (uint64_t *)malloc(sizeof(uint64_t) * n);
  for (uint32_t k = 0; k < n; k++) t[k] = a[oracle_bitrev(k, log_n)];
  const uint64_t psi_inv = oracle64_invmod(psi, q);
  cyclic_dft64(t, log_n, q, mulmod64(psi_inv, psi_inv, q));
  const uint64_t n_inv = oracle64_invmod(n % q, q);
  uint64_t pw = 1;
  for (uint32_t i = 0; i < n; i++) {
    a[i] = mulmod64(mulmod64(t[i], n_inv, q), pw, q);
    pw = mulmod64(pw, psi_inv, q);
  }
  free(t);
}

void oracle64_negacyclic_mul(const uint64_t *a, const uint64_t *b, uint64_t *c, uint32_t log_n, uint64_t q) {
  const uint32_t n = 1u << log_n;
  for (uint32_t k = 0; k < n; k++) c[k] = 0;
  for (uint32_t i = 0; i < n; i++)
    for (uint32_t j = 0; j < n; j++) {
      const uint64_t prod = mulmod64(a[i], b[j], q);
      if (i + j < n) c[i + j] = addmod64(c[i + j], prod, q);
      else c[i + j - n] = submod64(c[i + j - n], prod, q); /* X^N = -1 */
    }
}

/* ------------------------------------------------------------------ */
/* basis conversion                                                     */
/* ------------------------------------------------------------------ */

/* [prod_{i != skip} src_i]_m */
static uint64_t prod_except64(const uint64_t *src, uint32_t ns, uint32_t skip, uint64_t m) {
  uint64_t r = 1 % m;
  for (uint32_t i = 0; i < ns; i++)
    if (i != skip) r = mulmod64(r, src[i] % m, m);
  return r;
}

/* Fast basis conversion (Sec. III-B P2): y_t = sum_i [x_i (S/s_i)^-1]_{s_i}
 * [(S/s_i)]_{d_t} mod d_t, for x [ns][n] over src and y [nt][n] over dst. */
void oracle64_bconv(const uint64_t *x, const uint64_t *src, uint32_t ns, uint64_t *y, const uint64_t *dst,
                    uint32_t nt, uint32_t n) {
  uint64_t *xt = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)ns * n);
  for (uint32_t i = 0; i < ns; i++) {
    const uint64_t c = oracle64_invmod(prod_except64(src, ns, i, src[i]), src[i]);
    for (uint32_t z = 0; z < n; z++) xt[(size_t)i * n + z] = mulmod64(x[(size_t)i * n + z], c, src[i]);
  }
  for (uint32_t t = 0; t < nt; t++) {
    const uint64_t m = dst[t];
    for (uint32_t z = 0; z < n; z++) y[(size_t)t * n + z] = 0;
    for (uint32_t i = 0; i < ns; i++) {
      const uint32_t ii = (g_fault64 == 3 && ns > 1) ? (i + 1) % ns : i;
      const uint64_t c = prod_except64(src, ns, ii, m);
      for (uint32_t z = 0; z < n; z++)
        y[(size_t)t * n + z] = addmod64(y[(size_t)t * n + z], mulmod64(xt[(size_t)i * n + z], c, m), m);
    }
  }
  free(xt);
}

/* ------------------------------------------------------------------ */
/* hybrid key switching, Max-Parallel order (Sec. III)                  */
/* ------------------------------------------------------------------ */

typedef struct {
  uint32_t n, log_n, L1, K, dnum, alpha, level, ntow, ndig;
  uint64_t q[160];        /* extended basis D_l: q_0..q_l, p_0..p_{K-1} */
  uint32_t evk_limb[160]; /* limb index of D_l tower t inside the evk */
  uint64_t psi[160];
} ks64_ctx;

static int ctx64_init(ks64_ctx *c, const oracle_params *p, const uint64_t *moduli, uint32_t level) {
  if (p->log_n < 1 || p->log_n > 17 || p->num_q == 0 || p->dnum == 0 || p->dnum > p->num_q ||
      p->num_p == 0 || level >= p->num_q || p->num_q + p->num_p > 160)
    return -1;
  c->log_n = p->log_n;
  c->n = 1u << p->log_n;
  c->L1 = p->num_q;
  c->K = p->num_p;
  c->dnum = p->dnum;
  c->alpha = (p->num_q + p->dnum - 1) / p->dnum; /* Table I: ceil((L+1)/dnum) */
  c->level = level;
  c->ntow = level + 1 + p->num_p;
  c->ndig = (level + 1 + c->alpha - 1) / c->alpha; /* digits holding a live tower */
  for (uint32_t i = 0; i <= level; i++) { c->q[i] = moduli[i]; c->evk_limb[i] = i; }
  for (uint32_t k = 0; k < p->num_p; k++) {
    c->q[level + 1 + k] = moduli[p->num_q + k];
    c->evk_limb[level + 1 + k] = p->num_q + k;
  }
  for (uint32_t t = 0; t < c->ntow; t++) c->psi[t] = oracle64_min_psi(c->q[t], c->log_n);
  return 0;
}

#define LIMB64(buf, idx, n) ((buf) + (size_t)(idx) * (n))

/* ModDown, Sec. III-C, for one polynomial: acc [ntow][N] (evaluation domain,
 * towers of D_l) -> out [level+1][N]. */
static void moddown64(const ks64_ctx *c, const uint64_t *acc, uint64_t *out) {
  const uint32_t n = c->n, l1 = c->level + 1, K = c->K;
  uint64_t *a = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)K * n);
  uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)l1 * n);
  /* P1: INTT of the last K towers */
  for (uint32_t k = 0; k < K; k++) {
    memcpy(LIMB64(a, k, n), LIMB64(acc, l1 + k, n), sizeof(uint64_t) * n);
    oracle64_intt(LIMB64(a, k, n), c->log_n, c->q[l1 + k], c->psi[l1 + k]);
  }
  /* P2: basis conversion P -> Q_l */
  oracle64_bconv(a, &c->q[l1], K, w, c->q, l1, n);
  /* P3: NTT of the converted towers; P4: subtract, times P^-1 */
  for (uint32_t i = 0; i < l1; i++) {
    const uint64_t qi = c->q[i];
    oracle64_ntt(LIMB64(w, i, n), c->log_n, qi, c->psi[i]);
    uint64_t p_mod = 1;
    for (uint32_t k = 0; k < K; k++) p_mod = mulmod64(p_mod, c->q[l1 + k] % qi, qi);
    const uint64_t p_inv = oracle64_invmod(p_mod, qi);
    for (uint32_t z = 0; z < n; z++) {
      const uint64_t diff = (g_fault64 == 2) ? addmod64(LIMB64(acc, i, n)[z], LIMB64(w, i, n)[z], qi)
                                             : submod64(LIMB64(acc, i, n)[z], LIMB64(w, i, n)[z], qi);
      LIMB64(out, i, n)[z] = mulmod64(diff, p_inv, qi);
    }
  }
  free(a);
  free(w);
}

int oracle64_keyswitch(const oracle_params *p, const uint64_t *moduli, uint32_t level, const uint64_t *evk,
                       const uint64_t *d, uint64_t *out) {
  ks64_ctx c;
  if (ctx64_init(&c, p, moduli, level) != 0) return -1;
  const uint32_t n = c.n, l1 = level + 1, T = c.ntow, D = c.ndig, EL = c.L1 + c.K;
  uint64_t *x = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)l1 * n);   /* ModUp P1 */
  uint64_t *y = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)T * n);    /* one digit extended */
  uint64_t *tgt = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)T * n);
  uint64_t *tq = (uint64_t *)malloc(sizeof(uint64_t) * T);
  uint64_t *acc = (uint64_t *)calloc((size_t)2 * T * n, sizeof(uint64_t));
  if (!x || !y || !tgt || !tq || !acc) { free(x); free(y); free(tgt); free(tq); free(acc); return -1; }
  /* ModUp P1: INTT of every input tower */
  memcpy(x, d, sizeof(uint64_t) * (size_t)l1 * n);
  for (uint32_t i = 0; i < l1; i++) oracle64_intt(LIMB64(x, i, n), c.log_n, c.q[i], c.psi[i]);
  for (uint32_t j = 0; j < D; j++) {
    const uint32_t lo = j * c.alpha, hi = (j + 1) * c.alpha < l1 ? (j + 1) * c.alpha : l1;
    /* P2: digit j converted from S_j to every other tower of D_l */
    uint32_t nt = 0;
    for (uint32_t t = 0; t < T; t++)
      if (t < lo || t >= hi) tq[nt++] = c.q[t];
    oracle64_bconv(LIMB64(x, lo, n), &c.q[lo], hi - lo, tgt, tq, nt, n);
    /* P3: NTT of the converted towers; the digit's own towers are d itself */
    uint32_t u = 0;
    for (uint32_t t = 0; t < T; t++) {
      uint64_t *dst = LIMB64(y, t, n);
      if (t >= lo && t < hi) {
        uint32_t src = t;
        if (g_fault64 == 4 && D > 1) src = (t + c.alpha) % l1;
        memcpy(dst, LIMB64(d, src, n), sizeof(uint64_t) * n);
      } else {
        memcpy(dst, LIMB64(tgt, u, n), sizeof(uint64_t) * n);
        oracle64_ntt(dst, c.log_n, c.q[t], c.psi[t]);
        u++;
      }
    }
    /* P4: apply the key, P5: sum over digits */
    if (g_fault64 == 1 && j == D - 1 && D > 1) continue;
    for (uint32_t s = 0; s < 2; s++)
      for (uint32_t t = 0; t < T; t++) {
        const uint64_t *ek = evk + (((size_t)j * 2 + s) * EL + c.evk_limb[t]) * n;
        const uint64_t *yy = LIMB64(y, t, n);
        uint64_t *aa = LIMB64(acc, (size_t)s * T + t, n);
        for (uint32_t z = 0; z < n; z++) aa[z] = addmod64(aa[z], mulmod64(yy[z], ek[z], c.q[t]), c.q[t]);
      }
  }
  /* ModDown P1-P4 for both polynomials */
  for (uint32_t s = 0; s < 2; s++) moddown64(&c, LIMB64(acc, (size_t)s * T, n), LIMB64(out, (size_t)s * l1, n));
  free(x); free(y); free(tgt); free(tq); free(acc);
  return 0;
}

/* ------------------------------------------------------------------ */
/* key generation (the generator and distributions of ks_oracle.c)      */
/* ------------------------------------------------------------------ */

typedef struct { uint64_t s[4]; } rng64_t;
static uint64_t splitmix64_next(uint64_t *x) {
  uint64_t z = (*x += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static uint64_t rng64_next(rng64_t *r) { /* xoshiro256** (Blackman & Vigna) */
  const uint64_t res = rotl64(r->s[1] * 5, 7) * 9, t = r->s[1] << 17;
  r->s[2] ^= r->s[0]; r->s[3] ^= r->s[1]; r->s[1] ^= r->s[2]; r->s[0] ^= r->s[3];
  r->s[2] ^= t; r->s[3] = rotl64(r->s[3], 45);
  return res;
}
static void rng64_seed(rng64_t *r, uint64_t seed) { for (int i = 0; i < 4; i++) r->s[i] = splitmix64_next(&seed); }
static uint64_t rng64_below(rng64_t *r, uint64_t m) { /* uniform in [0, m) by rejection */
  const uint64_t lim = (UINT64_MAX / m) * m;
  for (;;) { const uint64_t v = rng64_next(r); if (v < lim) return v % m; }
}
static double rng64_unit(rng64_t *r) { return ((rng64_next(r) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
static int32_t rng64_gauss(rng64_t *r) { /* Box-Muller, sigma 3.2, clamp 19 */
  const double u1 = rng64_unit(r), u2 = rng64_unit(r);
  const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  long e = lround(3.2 * z);
  if (e > 19) e = 19;
  if (e < -19) e = -19;
  return (int32_t)e;
}
static uint64_t signed_mod64(int32_t v, uint64_t m) { return v >= 0 ? (uint64_t)v % m : m - ((uint64_t)(-(int64_t)v) % m); }

/* s, s2 ternary; evk[j] = (b_j, a_j) with b_j = e_j - a_j s + g_j s2, g_j =
 * [P]_m on digit j's own q-limbs and 0 elsewhere (evaluation domain).
 * Returns h = the Hamming weight of s. */
/* seeded: the a halves already hold the generator's words (oracle64_seeded_a) */
static int keygen64_impl(const oracle_params *p, const uint64_t *moduli, uint64_t seed, int seeded, int8_t *s,
                         int8_t *s2, uint64_t *evk) {
  ks64_ctx c;
  if (ctx64_init(&c, p, moduli, p->num_q - 1) != 0) return -1;
  const uint32_t n = c.n, EL = c.L1 + c.K;
  rng64_t r;
  rng64_seed(&r, seed);
  int h = 0;
  for (uint32_t z = 0; z < n; z++) { s[z] = (int8_t)((int)rng64_below(&r, 3) - 1); h += s[z] != 0; }
  for (uint32_t z = 0; z < n; z++) s2[z] = (int8_t)((int)rng64_below(&r, 3) - 1);
  uint64_t *sh = (uint64_t *)malloc(sizeof(uint64_t) * n), *s2h = (uint64_t *)malloc(sizeof(uint64_t) * n);
  uint64_t *eh = (uint64_t *)malloc(sizeof(uint64_t) * n);
  int32_t *e = (int32_t *)malloc(sizeof(int32_t) * n);
  for (uint32_t j = 0; j < p->dnum; j++) {
    const uint32_t lo = j * c.alpha, hi = (j + 1) * c.alpha < c.L1 ? (j + 1) * c.alpha : c.L1;
    for (uint32_t z = 0; z < n; z++) e[z] = rng64_gauss(&r);
    for (uint32_t g = 0; g < EL; g++) {
      const uint64_t m = c.q[g]; /* at level L the D_L order equals the evk order */
      for (uint32_t z = 0; z < n; z++) {
        sh[z] = signed_mod64(s[z], m);
        s2h[z] = signed_mod64(s2[z], m);
        eh[z] = signed_mod64(e[z], m);
      }
      oracle64_ntt(sh, c.log_n, m, c.psi[g]);
      oracle64_ntt(s2h, c.log_n, m, c.psi[g]);
      oracle64_ntt(eh, c.log_n, m, c.psi[g]);
      uint64_t gad = 0; /* [P]_m on digit j's own q-limbs */
      if (g >= lo && g < hi) {
        gad = 1;
        for (uint32_t k = 0; k < c.K; k++) gad = mulmod64(gad, moduli[c.L1 + k] % m, m);
      }
      uint64_t *b = evk + (((size_t)j * 2 + 0) * EL + g) * n;
      uint64_t *a = evk + (((size_t)j * 2 + 1) * EL + g) * n;
      for (uint32_t z = 0; z < n; z++) {
        if (!seeded) a[z] = rng64_below(&r, m);
        b[z] = addmod64(submod64(eh[z], mulmod64(a[z], sh[z], m), m), mulmod64(gad, s2h[z], m), m);
      }
    }
  }
  free(sh); free(s2h); free(eh); free(e);
  return h;
}

int oracle64_keygen(const oracle_params *p, const uint64_t *moduli, uint64_t seed, int8_t *s, int8_t *s2,
                    uint64_t *evk) {
  return keygen64_impl(p, moduli, seed, 0, s, s2, evk);
}

/* Key compression (Sec. IV-D) with 64-bit words: word (j, g, k) of the a
 * halves is X 2^-64 mod m_g for the 123-bit integer X = (x1 >> 5) 2^64 + x0,
 * where x0 and x1 are the SplitMix64 outputs (oracle_splitmix_at, the 32-bit
 * oracle's generator) at counters 2t and 2t + 1, t = (j (L+1+K) + g) N + k.
 * One 64-bit output reduced mod a 60-bit prime would sit up to 2^-6 from
 * uniform; X, uniform on [0, 2^123), sits below m / 2^125 < 2^-65.  Computed
 * here as (X mod m) times the inverse of 2^64 mod m. */
int oracle64_seeded_a(const oracle_params *p, const uint64_t *moduli, uint64_t a_seed, uint64_t *evk) {
  if (!p || !moduli || !evk || p->num_q == 0 || p->dnum == 0 || p->num_p == 0) return -1;
  const uint32_t n = 1u << p->log_n, EL = p->num_q + p->num_p;
  for (uint32_t g = 0; g < EL; g++) {
    const uint64_t m = moduli[g];
    const uint64_t r64 = (uint64_t)(((u128)1 << 64) % m), inv = oracle64_invmod(r64, m);
    for (uint32_t j = 0; j < p->dnum; j++) {
      uint64_t *a = evk + (((size_t)j * 2 + 1) * EL + g) * n;
      for (uint32_t k = 0; k < n; k++) {
        const uint64_t t = ((uint64_t)j * EL + g) * n + k;
        const u128 X = ((u128)(oracle_splitmix_at(a_seed, 2 * t + 1) >> 5) << 64) | oracle_splitmix_at(a_seed, 2 * t);
        a[k] = mulmod64((uint64_t)(X % m), inv, m);
      }
    }
  }
  return 0;
}

int oracle64_keygen_seeded(const oracle_params *p, const uint64_t *moduli, uint64_t seed, uint64_t a_seed,
                           int8_t *s, int8_t *s2, uint64_t *evk) {
  if (oracle64_seeded_a(p, moduli, a_seed, evk) != 0) return -1;
  return keygen64_impl(p, moduli, seed, 1, s, s2, evk);
}
