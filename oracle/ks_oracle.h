/*
 * ks_oracle.h -- plain, slow CPU oracle for CKKS hybrid key switching.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code,
 * header, table or constant generator with the HIP library under
 * paper_2311_01598_amd/; it re-derives every modulus, root and constant from
 * the definitions with plain uint64 '%' arithmetic.
 *
 * Notation follows the paper (CiFlow, Sec. II Table I and Sec. III):
 *   N = 2^log_n ring degree; q_0..q_L the Q moduli (num_q = L+1 of them);
 *   p_0..p_{K-1} the special moduli of P (num_p = K); dnum digits of
 *   alpha = ceil((L+1)/dnum) towers each; level l means l+1 towers q_0..q_l.
 *
 * Layouts (all uint32, limb-major, every residue canonical in [0, m)):
 *   polynomial at level l  : [l+1][N]
 *   evaluation key (evk)   : [dnum][2][L+1+K][N]; limb g < L+1 is q_g,
 *                            limb L+1+k is p_k (Sec. III-B, ModUp P4 shape)
 *   key-switch output      : [2][l+1][N]
 *   moduli array           : [L+1+K] = q_0..q_L, p_0..p_{K-1}
 */
#ifndef KS_ORACLE_H
#define KS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  uint32_t log_n;  /* ring degree N = 2^log_n */
  uint32_t num_q;  /* L+1 */
  uint32_t dnum;   /* number of digits */
  uint32_t num_p;  /* K */
} oracle_params;

/* Number theory (Sec. II: RNS with word-size NTT-friendly moduli). */
int oracle_is_prime(uint64_t n);                 /* trial division */
/* Candidates 2^30 - t*2N + 1, t = 1, 2, ...; the first `count` primes in
 * that order.  Returns 0 on success, -1 if fewer than `count` exist. */
int oracle_gen_primes(uint32_t log_n, uint32_t count, uint32_t *out);
/* Moduli of a parameter set: the first K primes are p_0..p_{K-1}, the next
 * L+1 are q_0..q_L; written out as q_0..q_L, p_0..p_{K-1}. */
int oracle_moduli(const oracle_params *p, uint32_t *out);
/* Smallest x in [2, q) with x^N = -1 (mod q): the 2N-th root that fixes the
 * evaluation points of the NTT. */
uint32_t oracle_min_psi(uint32_t q, uint32_t log_n);
uint32_t oracle_powmod(uint32_t b, uint64_t e, uint32_t q);
uint32_t oracle_invmod(uint32_t a, uint32_t q);
uint32_t oracle_bitrev(uint32_t x, uint32_t bits);

/* Negacyclic NTT into the evaluation domain (Sec. II/III-B "evaluation
 * domain"): out[j] = a(psi^(2*brv(j)+1)) mod q, i.e. evaluation of a(X) at
 * the N roots of X^N+1 listed in bit-reversed order. */
void oracle_ntt_direct(const uint32_t *a, uint32_t *out, uint32_t log_n, uint32_t q, uint32_t psi);
void oracle_ntt(uint32_t *a, uint32_t log_n, uint32_t q, uint32_t psi);   /* in place */
void oracle_intt(uint32_t *a, uint32_t log_n, uint32_t q, uint32_t psi);  /* in place */
/* c = a*b in Z_q[X]/(X^N+1), schoolbook O(N^2). */
void oracle_negacyclic_mul(const uint32_t *a, const uint32_t *b, uint32_t *c, uint32_t log_n, uint32_t q);

/* Fast basis conversion (ModUp P2 / ModDown P2): x holds `ns` source limbs
 * (coefficient domain) modulo src[0..ns); y receives `nt` limbs modulo
 * dst[0..nt):  y_m = sum_i [x_i * (S/s_i)^-1]_{s_i} * [S/s_i]_m  mod m. */
void oracle_bconv(const uint32_t *x, const uint32_t *src, uint32_t ns,
                  uint32_t *y, const uint32_t *dst, uint32_t nt, uint32_t n);

/* Hybrid key switching, Sec. III (ModUp P1-P5, ModDown P1-P4), executed in
 * the Max-Parallel order of Sec. IV-A: every stage over all towers before the
 * next.  d: [level+1][N] evaluation domain; evk: [dnum][2][L+1+K][N];
 * out: [2][level+1][N].  Returns 0, or -1 on bad arguments / allocation. */
int oracle_keyswitch(const oracle_params *p, const uint32_t *moduli, uint32_t level,
                     const uint32_t *evk, const uint32_t *d, uint32_t *out);
/* The same computation in the Output-Centric order of Sec. IV-C: one output
 * tower at a time (P towers first, then each Q tower through ModDown). */
int oracle_keyswitch_oc(const oracle_params *p, const uint32_t *moduli, uint32_t level,
                        const uint32_t *evk, const uint32_t *d, uint32_t *out);

/* Seeded key generation (RLWE, Sec. III): s, s2 ternary in {-1,0,1} (s2 is
 * the key the input is decryptable under, s the target key); for digit j the
 * evk pair is (b_j, a_j), b_j = -a_j*s + e_j + g_j*s2 with g_j = [P]_m on the
 * q-limbs of digit j and 0 on every other limb; e_j rounded Gaussian,
 * sigma = 3.2, clamped to |e| <= 19.  Returns h = ||s||_1, or -1. */
int oracle_keygen(const oracle_params *p, const uint32_t *moduli, uint64_t seed,
                  int8_t *s, int8_t *s2, uint32_t *evk);

/* Key compression (Sec. IV-D): a halves regenerated from a seed.
 * oracle_splitmix_at: output t of the counter-based SplitMix64 generator
 * (Steele, Lea and Flood 2014) for `seed`: the SplitMix64 mix of
 * seed + (t + 1) * 0x9e3779b97f4a7c15.
 * oracle_seeded_a: writes the a half of every pair of a full-layout evk,
 * word (j, g, k) = x * 2^-32 mod m_g with x the output at
 * t = (j * (L+1+K) + g) * N + k (g in evk order q_0..q_L, p_0..p_{K-1}).
 * oracle_keygen_seeded: oracle_keygen with those a halves (the b halves
 * computed from them), so the b halves plus a_seed are the whole key. */
uint64_t oracle_splitmix_at(uint64_t seed, uint64_t t);
int oracle_seeded_a(const oracle_params *p, const uint32_t *moduli, uint64_t a_seed, uint32_t *evk);
int oracle_keygen_seeded(const oracle_params *p, const uint32_t *moduli, uint64_t seed, uint64_t a_seed,
                         int8_t *s, int8_t *s2, uint32_t *evk);

/* Callers of the key switch (Sec. II: rotations and multiplications need
 * it).  Galois element k: odd, below 2N.
 * oracle_automorphism_coeff: a(X^k) of a coefficient-domain limb.
 * oracle_automorphism_eval: the same map on an evaluation-domain limb, a
 * permutation of the slots (modulus-independent).
 * oracle_keygen_rotation: key switching from s(X^k) to s (s2 returns s(X^k)).
 * oracle_keygen_relin: key switching from s^2 to s.
 * oracle_rotate_hoisted: count rotations of (c0, c1) sharing one ModUp of
 * c1; evks [count][dnum][2][L+1+K][N], outs [count][2][level+1][N].
 * oracle_rotate: one rotation, permute then key-switch (cross-check).
 * oracle_mult_relin: tensor product then key switch of d2, out [2][l+1][N].
 * All return 0 (keygen: the Hamming weight of s) or -1 on bad arguments. */
int oracle_automorphism_coeff(const uint32_t *a, uint32_t log_n, uint32_t galois, uint32_t q, uint32_t *out);
int oracle_automorphism_eval(const uint32_t *a, uint32_t log_n, uint32_t galois, uint32_t *out);
int oracle_keygen_rotation(const oracle_params *p, const uint32_t *moduli, uint64_t seed, uint32_t galois,
                           int8_t *s, int8_t *s2, uint32_t *evk);
int oracle_keygen_relin(const oracle_params *p, const uint32_t *moduli, uint64_t seed, int8_t *s, uint32_t *evk);
int oracle_rotate_hoisted(const oracle_params *p, const uint32_t *moduli, uint32_t level, const uint32_t *c0,
                          const uint32_t *c1, uint32_t count, const uint32_t *galois, const uint32_t *evks,
                          uint32_t *outs);
/* oracle_rotate_sum_hoisted: double hoisting, sum_r p_r sigma_r(c0, c1)
 * with one ModUp and one ModDown; diags null (all p_r = 1) or
 * [count][L+1+K][N] (key-row order, evaluation domain); out [2][l+1][N]. */
int oracle_rotate_sum_hoisted(const oracle_params *p, const uint32_t *moduli, uint32_t level, const uint32_t *c0,
                              const uint32_t *c1, uint32_t count, const uint32_t *galois, const uint32_t *evks,
                              const uint32_t *diags, uint32_t *out);
int oracle_rotate(const oracle_params *p, const uint32_t *moduli, uint32_t level, const uint32_t *c0,
                  const uint32_t *c1, uint32_t galois, const uint32_t *evk, uint32_t *out);
int oracle_mult_relin(const oracle_params *p, const uint32_t *moduli, uint32_t level, const uint32_t *a0,
                      const uint32_t *a1, const uint32_t *b0, const uint32_t *b1, const uint32_t *evk, uint32_t *out);

/* Test hook: plant a deliberate mistake in the oracle's key switch so tests
 * can show their checks catch it.  0 = none; see ks_oracle.c for the list. */
void oracle_set_fault(int fault);

/* Evaluation-key size in words for a parameter set (Sec. III-B P4 shape). */
uint64_t oracle_evk_words(uint32_t log_n, uint32_t num_q, uint32_t num_p, uint32_t dnum);

/* ---- 64-bit words (ks_oracle64.c): towers of ~60-bit primes in uint64
 * words, every product an exact unsigned __int128 reduced with '%'.  Same
 * layouts and conventions as above with uint64 residues; moduli
 * 2^60 - t*2N + 1; psi the smallest x with x^N = -1 (mod q). */
int oracle64_is_prime(uint64_t n);               /* Miller-Rabin, 12 prime bases */
int oracle64_gen_primes(uint32_t log_n, uint32_t count, uint64_t *out);
int oracle64_moduli(const oracle_params *p, uint64_t *out);
uint64_t oracle64_min_psi(uint64_t q, uint32_t log_n);
uint64_t oracle64_powmod(uint64_t b, uint64_t e, uint64_t q);
uint64_t oracle64_invmod(uint64_t a, uint64_t q);
void oracle64_ntt_direct(const uint64_t *a, uint64_t *out, uint32_t log_n, uint64_t q, uint64_t psi);
void oracle64_ntt(uint64_t *a, uint32_t log_n, uint64_t q, uint64_t psi);
void oracle64_intt(uint64_t *a, uint32_t log_n, uint64_t q, uint64_t psi);
void oracle64_negacyclic_mul(const uint64_t *a, const uint64_t *b, uint64_t *c, uint32_t log_n, uint64_t q);
void oracle64_bconv(const uint64_t *x, const uint64_t *src, uint32_t ns, uint64_t *y, const uint64_t *dst,
                    uint32_t nt, uint32_t n);
int oracle64_keyswitch(const oracle_params *p, const uint64_t *moduli, uint32_t level, const uint64_t *evk,
                       const uint64_t *d, uint64_t *out);
int oracle64_keygen(const oracle_params *p, const uint64_t *moduli, uint64_t seed, int8_t *s, int8_t *s2,
                    uint64_t *evk);
/* Key compression (Sec. IV-D) with 64-bit words: the a halves are
 * x 2^-64 mod m_g for the SplitMix64 output x at the counter of
 * oracle_seeded_a (t = (j (L+1+K) + g) N + k); keygen_seeded computes the b
 * halves from them. */
int oracle64_seeded_a(const oracle_params *p, const uint64_t *moduli, uint64_t a_seed, uint64_t *evk);
int oracle64_keygen_seeded(const oracle_params *p, const uint64_t *moduli, uint64_t seed, uint64_t a_seed,
                           int8_t *s, int8_t *s2, uint64_t *evk);
void oracle64_set_fault(int fault);

#ifdef __cplusplus
}
#endif
#endif
