// ks64.hip -- hybrid key switching with 64-bit words: towers of ~60-bit
// primes (Sec. II word-size moduli, 36-64 bits; Table III's evk sizes count
// 8-byte words), the Max-Parallel order of Sec. IV-A: every stage over all
// towers, each stage's output in device memory.
//
// Arithmetic on uint64 residues below 2^60:
//  - products with a constant (conversion prescales, P^-1, N^-1): Shoup's
//    method with the precomputed floor(w 2^64 / q), one 64-bit high product
//    and two low products, result in [0, 2q) then one conditional
//    subtraction; the transforms' twiddle products take the high product
//    without its lowest partial product and carries, result in [0, 4q);
//  - sums of products (conversion, key multiply-accumulate): exact
//    accumulation of at most 16 products of canonical residues (each below
//    2^60 m, so the sum stays below m 2^64), then one Montgomery reduction
//    REDC(T) = (T + ((T mod 2^64)(-m^-1) mod 2^64) m) / 2^64 < 2m.  The
//    2^-64 it leaves is cancelled by constants kept in Montgomery form
//    (c 2^64 mod m), or by one Shoup product with 2^64 mod m.  Each operand
//    is split into 30-bit halves, a = a1 2^30 + a0, so a product is four
//    32 x 32 -> 64-bit products a1 b1 2^60 + (a1 b0 + a0 b1) 2^30 + a0 b0,
//    each below 2^60: four 64-bit sums (one multiply-add per partial
//    product) hold 16 products without overflow, and are combined into
//    the 128-bit sum once per chunk.
//  - every stage leaves canonical residues, except inside a transform: a
//    pass hands its next pass words in [0, 8q) (forward) or [0, 4q)
//    (inverse), and the last pass makes them canonical.
// The forward transform is the Cooley-Tukey network that lists a(psi^(2
// brv(j)+1)) at position j; the inverse is the Gentleman-Sande network and
// N^-1.  A transform of N = R x 256 words is a column pass (stages with
// butterfly distance >= 256) and a row pass (distance < 256), each staged
// through LDS.  Where a transform feeds an element-wise step, its row pass
// runs inside that step's kernel: the forward row pass of the converted
// towers with the key multiply-accumulate (and, for the special towers, the
// inverse row pass of ModDown), the forward row pass of ModDown's converted
// towers with the final subtraction and P^-1.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include <hip/hip_runtime.h>

#include "ks.h"
#include "numtheory.h"
#include "range_check.h"

namespace ks64 {

typedef unsigned __int128 u128;

constexpr uint32_t kMaxTowers = 128;
constexpr uint32_t kList = 96;  // towers per transform launch
constexpr uint32_t kRowWords = 256;
constexpr uint32_t kRowsPerTile = 4;
constexpr uint32_t kColsPerTile = 4;

struct Mod64 {
  uint64_t q, qneg;   // modulus, -q^-1 mod 2^64
  uint64_t r64, r64s; // 2^64 mod q and its Shoup companion
  uint64_t ninv, ninvs;
};

// Device view of a plan.
struct Dev64 {
  uint32_t log_n, num_q, num_p, dnum, alpha, ntot;
  const Mod64 *mods;      // [ntot], order q_0..q_L, p_0..p_{K-1}
  const uint4 *tw_fwd;    // [ntot][N]: (w, w') as two little-endian uint64 per entry
  const uint4 *tw_inv;
  const uint64_t *up_pre; // [num_q][dnum][alpha][2]: [q^_{j,s}^-1]_{q_s} and Shoup companion
  const uint64_t *up_cst; // [num_q][dnum][ntot][alpha] + 32 zero words: [q^_{j,s}]_{m_g} 2^64 mod m_g
  const uint64_t *dn_pre; // [K][2]: [p^_k^-1]_{p_k} and companion
  const uint64_t *dn_cst; // [num_q][K] + 32 zero words: [p^_k]_{q_i} 2^64 mod q_i
  const uint64_t *pinv;   // [num_q][2]: [P^-1]_{q_i} and companion
};

struct List64 {
  uint32_t count;
  uint32_t src[kList];
  uint32_t dst[kList];
  uint16_t g[kList];
};

// ------------------------------------------------------------ arithmetic
__device__ __forceinline__ uint64_t csub(uint64_t x, uint64_t q) { return x >= q ? x - q : x; }
__device__ __forceinline__ uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) { return csub(a + b, q); }
__device__ __forceinline__ uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }
// a < 2^64, w < q < 2^62, ws = floor(w 2^64 / q): a w mod q in [0, 2q)
__device__ __forceinline__ uint64_t shoup_lazy(uint64_t a, uint64_t w, uint64_t ws, uint64_t q) {
  const uint64_t h = __umul64hi(a, ws);
  const uint64_t r = a * w - h * q;
  KS_RANGE(r < 2 * q, KS_RC64_SHOUP);
  return r;
}
// the same, canonical
__device__ __forceinline__ uint64_t shoup(uint64_t a, uint64_t w, uint64_t ws, uint64_t q) {
  return csub(shoup_lazy(a, w, ws, q), q);
}
// Shoup's product with an estimate of the quotient h = floor(a ws / 2^64):
// with a = a1 2^32 + a0 and ws = s1 2^32 + s0, a ws / 2^64 equals
// a1 s1 + floor(a1 s0 / 2^32) + floor(a0 s1 / 2^32) plus a fraction below
// 3 (the two dropped low halves and a0 s0 / 2^64), so the estimate is h,
// h - 1 or h - 2 and a w - estimate q lies in [0, 4q).  Two 32-bit high
// products and one multiply-add instead of the exact high product's three
// multiply-adds.
__device__ __forceinline__ uint64_t shoup_lazy4(uint64_t a, uint64_t w, uint64_t ws, uint64_t q) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), s0 = (uint32_t)ws, s1 = (uint32_t)(ws >> 32);
  const uint64_t h = (uint64_t)a1 * s1 + __umulhi(a1, s0) + __umulhi(a0, s1);
  const uint64_t r = a * w - h * q;
  KS_RANGE(r < 4 * q, KS_RC64_SHOUP4);
  return r;
}
// A 128-bit value, (hi, lo).
struct Acc128 {
  uint64_t lo = 0, hi = 0;
};
// Sum of at most 16 products of values below 2^60 as 30-bit halves.
constexpr uint64_t kLo30 = (1ull << 30) - 1;
struct Acc4 {
  uint64_t s0 = 0, s1a = 0, s1b = 0, s2 = 0;
  __device__ __forceinline__ void mac(uint32_t a0, uint32_t a1, uint32_t b0, uint32_t b1) {
    KS_RANGE((a0 | a1 | b0 | b1) < (1u << 30), KS_RC64_MAC_OPND);
#ifdef KS_CHECK_RANGES
    const uint64_t p0 = s0, p1 = s1a, p2 = s1b, p3 = s2;
#endif
    s0 += (uint64_t)a0 * b0;
    s1a += (uint64_t)a1 * b0;
    s1b += (uint64_t)a0 * b1;
    s2 += (uint64_t)a1 * b1;
    KS_RANGE(s0 >= p0 && s1a >= p1 && s1b >= p2 && s2 >= p3, KS_RC64_MAC_WRAP);
  }
  __device__ __forceinline__ void mac(uint32_t a0, uint32_t a1, uint64_t b) {
    mac(a0, a1, (uint32_t)(b & kLo30), (uint32_t)(b >> 30));
  }
  __device__ __forceinline__ Acc128 sum() const {
    const u128 t = (u128)s0 + ((u128)s1a << 30) + ((u128)s1b << 30) + ((u128)s2 << 60);
    Acc128 r;
    r.lo = (uint64_t)t;
    r.hi = (uint64_t)(t >> 64);
    return r;
  }
};
// T < q 2^64: (T + m q) / 2^64 with m = T_lo (-q^-1) mod 2^64, canonical
__device__ __forceinline__ uint64_t redc(const Acc128 &t, const Mod64 &m) {
  KS_RANGE(t.hi < m.q, KS_RC64_REDC_IN);
  const uint64_t u = t.lo * m.qneg;
  const uint64_t lo = t.lo + u * m.q;  // 0 mod 2^64 by the choice of u
  return csub(t.hi + __umul64hi(u, m.q) + (lo < t.lo ? 1u : 0u), m.q);
}

// Compressed keys (Sec. IV-D): the a half of digit j's key row g is
// regenerated where it is consumed.  Word k is X 2^-64 mod m for the 123-bit
// integer X = (x1 >> 5) 2^64 + x0, x0 and x1 the SplitMix64 outputs
// (Steele, Lea and Flood 2014) at counters 2t and 2t + 1 of the word's
// counter t = (j ntot + g) N + k; output c of seed s is the mix of
// s + (c + 1) gamma.  X is below 2^123 < m 2^64, so one Montgomery reduction
// gives the canonical residue; X's 123 bits keep the words below 2^-65 from
// uniform (one 64-bit output would leave up to 2^-6 for a 60-bit prime).
// The pre-mix state of output c is s + (c + 1) gamma, so consecutive
// outputs step it by gamma and a thread's words (counters 512 apart) by
// 512 gamma: no counter multiplies per word.
constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;
__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
// z0: the state of output 2t, seed + (2t + 1) gamma.
__device__ __forceinline__ uint64_t seeded_a64(uint64_t z0, const Mod64 &m) {
  Acc128 x;
  x.lo = splitmix_mix(z0);
  x.hi = splitmix_mix(z0 + kGamma) >> 5;
  return redc(x, m);
}

// ------------------------------------------------------------ transforms
// The twiddle of the butterfly (j, j + t) is entry N / (2t) + j / (2t) of the
// table.  A pass transforms sequences of M words (M = 256 in the row pass,
// M = R = N / 256 in the column pass) held in LDS; within a sequence the
// butterflies at distance t come in h = M / (2t) groups, and group k takes
// the twiddle the tile stages at [h + k] (one round of loads per tile, so
// the stages read no global memory).  Stages run two at a time (radix 4:
// four words per thread, one LDS round trip and one barrier per two
// stages); an odd stage count ends with one radix-2 stage.

__device__ __forceinline__ void tw_of(const uint4 v, uint64_t *w, uint64_t *ws) {
  *w = ((uint64_t)v.y << 32) | v.x;
  *ws = ((uint64_t)v.w << 32) | v.z;
}
// Harvey's lazy butterflies, widened for twiddle products in [0, 4q)
// (q < 2^60, so 8q < 2^63 fits a word).  Cooley-Tukey (a, b) ->
// (a + b w, a - b w) on inputs in [0, 8q), outputs in [0, 8q): one
// conditional subtraction of 4q per butterfly.
__device__ __forceinline__ void ct(uint64_t &a, uint64_t &b, const uint4 tv, uint64_t q) {
  KS_RANGE(a < 8 * q && b < 8 * q, KS_RC64_CT_IN);
  uint64_t w, ws;
  tw_of(tv, &w, &ws);
  const uint64_t q4 = 4 * q, x = csub(a, q4), v = shoup_lazy4(b, w, ws, q);
  a = x + v;
  b = x - v + q4;
}
// Gentleman-Sande (a, b) -> (a + b, (a - b) w) on inputs in [0, 4q),
// outputs in [0, 4q).
__device__ __forceinline__ void gs(uint64_t &a, uint64_t &b, const uint4 tv, uint64_t q) {
  KS_RANGE(a < 4 * q && b < 4 * q, KS_RC64_GS_IN);
  uint64_t w, ws;
  tw_of(tv, &w, &ws);
  const uint64_t q4 = 4 * q, d = a - b + q4;
  a = csub(a + b, q4);
  b = shoup_lazy4(d, w, ws, q);
}
// A forward transform's word in [0, 8q) made canonical.
__device__ __forceinline__ uint64_t fwd_canon(uint64_t x, uint64_t q) {
  KS_RANGE(x < 8 * q, KS_RC64_FWD_IN);
  return csub(csub(csub(x, 4 * q), 2 * q), q);
}

// One step over `nseq` sequences of M words in LDS (word p of sequence c
// at s[p * ps + c * cs]) with twiddles at tw + c * ts.  Forward: the
// stages at distances t and t / 2 (t >= 2), or t alone when R2; inverse:
// distances t and 2t, or t alone when R2.  Consecutive threads take
// consecutive units of one sequence when SEQ (rows: contiguous words), of
// consecutive sequences otherwise (columns: words of a row are adjacent).
template <bool INV, bool R2, bool SEQ>
__device__ __forceinline__ void nstep(uint64_t *s, const uint4 *tw, uint32_t M, uint32_t nseq, uint32_t ps,
                                      uint32_t cs, uint32_t ts, uint32_t tmask, uint32_t t, uint64_t q) {
  const uint32_t per = R2 ? M / 2 : M / 4;
  for (uint32_t u = threadIdx.x; u < per * nseq; u += 256) {
    const uint32_t c = SEQ ? u / per : u % nseq, k = SEQ ? u % per : u / nseq;
    uint64_t *x = s + c * cs;
    const uint4 *w = tw + (c & tmask) * ts;
    if (R2) {
      const uint32_t grp = k / t, p0 = grp * 2 * t + k % t;
      uint64_t a = x[p0 * ps], b = x[(p0 + t) * ps];
      if (!INV) ct(a, b, w[M / (2 * t) + grp], q);
      else gs(a, b, w[M / (2 * t) + grp], q);
      x[p0 * ps] = a;
      x[(p0 + t) * ps] = b;
    } else if (!INV) {
      const uint32_t half = t / 2, grp = k / half, p0 = grp * 2 * t + k % half, h1 = M / (2 * t);
      uint64_t x0 = x[p0 * ps], x1 = x[(p0 + half) * ps], x2 = x[(p0 + t) * ps], x3 = x[(p0 + t + half) * ps];
      const uint4 w1 = w[h1 + grp];
      ct(x0, x2, w1, q);
      ct(x1, x3, w1, q);
      ct(x0, x1, w[2 * h1 + 2 * grp], q);
      ct(x2, x3, w[2 * h1 + 2 * grp + 1], q);
      x[p0 * ps] = x0;
      x[(p0 + half) * ps] = x1;
      x[(p0 + t) * ps] = x2;
      x[(p0 + t + half) * ps] = x3;
    } else {
      const uint32_t grp = k / t, p0 = grp * 4 * t + k % t, h1 = M / (2 * t);
      uint64_t x0 = x[p0 * ps], x1 = x[(p0 + t) * ps], x2 = x[(p0 + 2 * t) * ps], x3 = x[(p0 + 3 * t) * ps];
      gs(x0, x1, w[h1 + 2 * grp], q);
      gs(x2, x3, w[h1 + 2 * grp + 1], q);
      const uint4 w2 = w[h1 / 2 + grp];
      gs(x0, x2, w2, q);
      gs(x1, x3, w2, q);
      x[p0 * ps] = x0;
      x[(p0 + t) * ps] = x1;
      x[(p0 + 2 * t) * ps] = x2;
      x[(p0 + 3 * t) * ps] = x3;
    }
  }
}

// All stages of a pass over sequences of M = 2^lm words; sequence c takes
// the twiddles of sequence c & tmask.
template <bool INV, bool SEQ>
__device__ __forceinline__ void npass(uint64_t *s, const uint4 *tw, uint32_t lm, uint32_t nseq, uint32_t ps,
                                      uint32_t cs, uint32_t ts, uint32_t tmask, uint64_t q) {
  const uint32_t M = 1u << lm;
  if (!INV) {
    uint32_t t = M / 2;
    for (; t >= 2; t /= 4) {
      nstep<false, false, SEQ>(s, tw, M, nseq, ps, cs, ts, tmask, t, q);
      __syncthreads();
    }
    if (t == 1) {
      nstep<false, true, SEQ>(s, tw, M, nseq, ps, cs, ts, tmask, 1, q);
      __syncthreads();
    }
  } else {
    uint32_t t = 1;
    for (; 2 * t < M; t *= 4) {
      nstep<true, false, SEQ>(s, tw, M, nseq, ps, cs, ts, tmask, t, q);
      __syncthreads();
    }
    if (t < M) {
      nstep<true, true, SEQ>(s, tw, M, nseq, ps, cs, ts, tmask, t, q);
      __syncthreads();
    }
  }
}

// Row pass: tiles of kRowsPerTile rows of 256 words (a block reads its whole
// tile before writing it, so src may equal dst).  Forward: stages with
// butterfly distance t = 128 .. 1 (Cooley-Tukey); inverse: t = 1 .. 128
// (Gentleman-Sande).  Row r at distance t (h = 128 / t groups) uses table
// entries h (N / 256 + r) + k, k < h, kept at [row][h + k].
__device__ __forceinline__ void stage_row_tw(uint4 *tws, const uint4 *tab, uint32_t N, uint32_t row0) {
  for (uint32_t e = threadIdx.x; e < kRowsPerTile * kRowWords; e += 256) {
    const uint32_t rr = e / kRowWords, k = e % kRowWords;
    if (k == 0) continue;
    const uint32_t h = 1u << (31 - __clz(k));
    tws[e] = tab[(size_t)h * (N / kRowWords + row0 + rr) + (k - h)];
  }
}

template <bool INV>
__global__ __launch_bounds__(256) void k_row(Dev64 P, List64 L, const uint64_t *src, uint64_t *dst) {
  __shared__ uint64_t s[kRowsPerTile * kRowWords];
  __shared__ uint4 tws[kRowsPerTile * kRowWords];
  const uint32_t N = 1u << P.log_n, c = blockIdx.y;
  const uint32_t g = L.g[c];
  const Mod64 m = P.mods[g];
  const uint4 *tab = (INV ? P.tw_inv : P.tw_fwd) + (size_t)g * N;
  const size_t base = (size_t)blockIdx.x * kRowsPerTile * kRowWords;
  const uint64_t *in = src + (size_t)L.src[c] * N + base;
  uint64_t *out = dst + (size_t)L.dst[c] * N + base;
  const uint32_t row0 = blockIdx.x * kRowsPerTile;
  for (uint32_t i = threadIdx.x; i < kRowsPerTile * kRowWords; i += 256) s[i] = in[i];
  stage_row_tw(tws, tab, N, row0);
  __syncthreads();
  npass<INV, true>(s, tws, 8, kRowsPerTile, 1, kRowWords, kRowWords, ~0u, m.q);
  // forward: the transform's last pass, words [0, 8q) -> canonical; inverse:
  // the first pass, words left in [0, 4q) for the column pass
  for (uint32_t i = threadIdx.x; i < kRowsPerTile * kRowWords; i += 256)
    out[i] = INV ? s[i] : fwd_canon(s[i], m.q);
}

// Column pass: tiles of kColsPerTile columns of R = N / 256 rows.  Forward:
// row distance R/2 .. 1 (butterfly distance t = 256 x that); inverse: 1 ..
// R/2, then N^-1.  Every stage uses entries [1, R) of the table, staged
// once per tile.  Blocks are dealt to the 8 XCDs in turn; block x of the
// B = 256 / kColsPerTile column tiles takes tile (x % 8) * (B / 8) + x / 8,
// so each XCD's L2 holds 32 whole columns (256-byte row segments) of the
// limb.  Four columns per tile (32-byte segments, 24 KB of LDS, six blocks
// per CU) ran faster than two, eight or sixteen.
template <bool INV>
__global__ __launch_bounds__(256) void k_col(Dev64 P, List64 L, const uint64_t *src, uint64_t *dst) {
  __shared__ uint64_t s[512 * kColsPerTile];
  __shared__ uint4 tws[512];
  const uint32_t N = 1u << P.log_n, R = N / kRowWords, c = blockIdx.y;
  const uint32_t g = L.g[c];
  const Mod64 m = P.mods[g];
  const uint4 *tab = (INV ? P.tw_inv : P.tw_fwd) + (size_t)g * N;
  const uint32_t x = blockIdx.x, col0 = ((x % 8) * (gridDim.x / 8) + x / 8) * kColsPerTile;
  const uint64_t *in = src + (size_t)L.src[c] * N;
  uint64_t *out = dst + (size_t)L.dst[c] * N;
  for (uint32_t i = threadIdx.x; i < R * kColsPerTile; i += 256)
    s[i] = in[(size_t)(i / kColsPerTile) * kRowWords + col0 + i % kColsPerTile];
  for (uint32_t e = threadIdx.x; e < R; e += 256) tws[e] = tab[e];
  __syncthreads();
  npass<INV, false>(s, tws, P.log_n - 8, kColsPerTile, kColsPerTile, 1, 0, 0, m.q);
  for (uint32_t i = threadIdx.x; i < R * kColsPerTile; i += 256) {
    uint64_t v = s[i];
    if (INV) v = shoup(v, m.ninv, m.ninvs, m.q);
    out[(size_t)(i / kColsPerTile) * kRowWords + col0 + i % kColsPerTile] = v;
  }
}

// ------------------------------------------------------------ ModUp P2
// Digit j of the input (X, coefficient domain) converted to every tower of
// D_l outside the digit: y_{j,t} = sum_s [x_s q^_{j,s}^-1]_{q_s} [q^_{j,s}]_{m_t}.
// grid (N / 256, digits, target groups of kTgtGroup towers); each thread one
// coefficient.
__device__ __forceinline__ uint32_t gidx(const Dev64 &P, uint32_t level, uint32_t t) {
  return t <= level ? t : P.num_q + (t - level - 1);
}

// Each block converts 256 coefficients of one digit to one group of
// kTgtGroup consecutive towers of D_l (grid z), two targets at a time so
// that the two 128-bit sums are independent chains.  Groups of 32 reuse the
// loaded and prescaled sources for more targets than groups of 8 or 16 (at
// Table III's sets the conversions ran 20-30 % faster); 64 was no faster.
constexpr uint32_t kTgtGroup = 32;

// sum_{s < ns} x[s] c[s] reduced mod m for two targets, the sources as
// 30-bit halves (x0, x1) and zero from ns on: chunks of 16 products, each
// chunk one REDC (its 2^-64 cancelled by constants in Montgomery form).
// The constants of a chunk are read without a bound (the tables are padded
// by 32 entries), so they load as wide scalar reads.
template <int MAXS>
__device__ __forceinline__ void conv2(const uint32_t (&x0)[MAXS], const uint32_t (&x1)[MAXS], uint32_t ns,
                                      const uint64_t *c0, const uint64_t *c1, const Mod64 &m0, const Mod64 &m1,
                                      uint64_t *y0, uint64_t *y1) {
  uint64_t r0 = 0, r1 = 0;
#pragma unroll
  for (int k0 = 0; k0 < MAXS; k0 += 16) {
    if ((uint32_t)k0 < ns) {
      Acc4 a0, a1;
#pragma unroll
      for (int k = k0; k < k0 + 16 && k < MAXS; k++) {
        a0.mac(x0[k], x1[k], c0[k]);
        a1.mac(x0[k], x1[k], c1[k]);
      }
      r0 = add_mod(r0, redc(a0.sum(), m0), m0.q);
      r1 = add_mod(r1, redc(a1.sum(), m1), m1.q);
    }
  }
  *y0 = r0;
  *y1 = r1;
}

template <int MAXA>
__global__ __launch_bounds__(256) void k_bconv_up(Dev64 P, uint32_t level, const uint64_t *__restrict__ X,
                                                  uint64_t *__restrict__ Y) {
  const uint32_t N = 1u << P.log_n, j = blockIdx.y, l1 = level + 1, T = l1 + P.num_p;
  const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t lo = j * P.alpha, hi = min(lo + P.alpha, l1), ns = hi - lo;
  const uint32_t t0 = blockIdx.z * kTgtGroup, t1 = min(t0 + kTgtGroup, T);
  const size_t crow = (size_t)level * P.dnum + j, cbase = crow * P.alpha;
  uint32_t x0[MAXA], x1[MAXA];
#pragma unroll
  for (int s = 0; s < MAXA; s++) {
    x0[s] = x1[s] = 0;
    if ((uint32_t)s < ns) {
      const uint64_t *pre = P.up_pre + (cbase + s) * 2;
      const uint64_t v = shoup(X[(size_t)(lo + s) * N + c], pre[0], pre[1], P.mods[lo + s].q);
      x0[s] = (uint32_t)(v & kLo30);
      x1[s] = (uint32_t)(v >> 30);
    }
  }
  // the group's targets outside the digit, in pairs (an odd count repeats
  // the last target, written twice with the same value)
  auto skip = [&](uint32_t t) { return (t >= lo && t < hi) ? hi : t; };
  for (uint32_t t = skip(t0); t < t1;) {
    const uint32_t tn = skip(t + 1), ta = t, tb = tn < t1 ? tn : t;
    t = tn < t1 ? skip(tn + 1) : t1;
    const uint32_t ga = gidx(P, level, ta), gb = gidx(P, level, tb);
    uint64_t ya, yb;
    conv2<MAXA>(x0, x1, ns, P.up_cst + (crow * P.ntot + ga) * P.alpha, P.up_cst + (crow * P.ntot + gb) * P.alpha,
                P.mods[ga], P.mods[gb], &ya, &yb);
    Y[((size_t)j * T + ta) * N + c] = ya;
    Y[((size_t)j * T + tb) * N + c] = yb;
  }
}

// ------------------------------------------------------------ ModUp P3-P5
// For target tower t of D_l and a tile of kRowsPerTile rows: the forward
// row pass of every digit's converted tower (its column pass done before),
// then acc_s[t] = sum_j yhat_{j,t} evk[j][s][t] over the live digits, where
// yhat_{j,t} is the input tower itself when t is one of digit j's own towers
// (Sec. IV-C bypass: NTT(INTT(d_t)) = d_t).  Q targets write acc_s[t]; for a
// P target the inverse row pass of both accumulators follows (ModDown P1,
// first pass), written to XP[s][t - l - 1] for the inverse column pass.
// grid (R / kRowsPerTile, T); each thread owns kRowWords * kRowsPerTile /
// 256 words of the tile.
constexpr uint32_t kTileWords = kRowsPerTile * kRowWords, kPerThread = kTileWords / 256;
// SEEDED: evk holds the b halves only, [dnum][ntot][N], and the a halves are
// regenerated from a_seed (seeded_a64).
template <bool SEEDED>
__global__ __launch_bounds__(256) void k_row_mac(Dev64 P, uint32_t level, const uint64_t *__restrict__ d,
                                                 const uint64_t *__restrict__ Y, const uint64_t *__restrict__ evk,
                                                 uint64_t a_seed, uint64_t *__restrict__ acc,
                                                 uint64_t *__restrict__ XP) {
  __shared__ uint64_t s[2 * kTileWords];
  __shared__ uint4 tws[kTileWords];
  const uint32_t N = 1u << P.log_n, t = blockIdx.y, l1 = level + 1, T = l1 + P.num_p;
  const uint32_t g = gidx(P, level, t), D = (l1 + P.alpha - 1) / P.alpha;
  const Mod64 m = P.mods[g];
  const uint32_t row0 = blockIdx.x * kRowsPerTile;
  const size_t base = (size_t)row0 * kRowWords;
  stage_row_tw(tws, P.tw_fwd + (size_t)g * N, N, row0);
  Acc4 a0[kPerThread], a1[kPerThread];
  for (uint32_t j = 0; j < D; j++) {
    const uint32_t lo = j * P.alpha, hi = min(lo + P.alpha, l1);
    uint64_t y[kPerThread];
    if (t >= lo && t < hi) {  // the own digit: the input tower
#pragma unroll
      for (uint32_t i = 0; i < kPerThread; i++) y[i] = d[(size_t)t * N + base + threadIdx.x + 256 * i];
    } else {
      const uint64_t *src = Y + ((size_t)j * T + t) * N + base;
      __syncthreads();  // the previous digit's words are read
      for (uint32_t e = threadIdx.x; e < kTileWords; e += 256) s[e] = src[e];
      __syncthreads();
      npass<false, true>(s, tws, 8, kRowsPerTile, 1, kRowWords, kRowWords, ~0u, m.q);
#pragma unroll
      for (uint32_t i = 0; i < kPerThread; i++) y[i] = fwd_canon(s[threadIdx.x + 256 * i], m.q);
    }
    const size_t row = (size_t)j * (SEEDED ? 1 : 2) * P.ntot + g;  // b half of digit j, key row g
    const uint64_t *e0 = evk + row * N + base;
    const uint64_t *e1 = SEEDED ? nullptr : evk + (row + P.ntot) * N + base;  // a half (full keys)
    // generator state of word (j, g, base + threadIdx.x), compressed keys
    const uint64_t z0 = a_seed + (2 * (((uint64_t)j * P.ntot + g) * N + base + threadIdx.x) + 1) * kGamma;
#pragma unroll
    for (uint32_t i = 0; i < kPerThread; i++) {
      const uint32_t y0 = (uint32_t)(y[i] & kLo30), y1 = (uint32_t)(y[i] >> 30);
      const uint64_t ak = SEEDED ? seeded_a64(z0 + (uint64_t)(512 * i) * kGamma, m) : e1[threadIdx.x + 256 * i];
      a0[i].mac(y0, y1, e0[threadIdx.x + 256 * i]);
      a1[i].mac(y0, y1, ak);
    }
  }
  uint64_t v0[kPerThread], v1[kPerThread];
#pragma unroll
  for (uint32_t i = 0; i < kPerThread; i++) {
    v0[i] = shoup(redc(a0[i].sum(), m), m.r64, m.r64s, m.q);
    v1[i] = shoup(redc(a1[i].sum(), m), m.r64, m.r64s, m.q);
  }
  if (t < l1) {
#pragma unroll
    for (uint32_t i = 0; i < kPerThread; i++) {
      acc[((size_t)0 * T + t) * N + base + threadIdx.x + 256 * i] = v0[i];
      acc[((size_t)1 * T + t) * N + base + threadIdx.x + 256 * i] = v1[i];
    }
    return;
  }
  __syncthreads();  // every read of s and of the forward twiddles is done
#pragma unroll
  for (uint32_t i = 0; i < kPerThread; i++) {
    s[threadIdx.x + 256 * i] = v0[i];
    s[kTileWords + threadIdx.x + 256 * i] = v1[i];
  }
  stage_row_tw(tws, P.tw_inv + (size_t)g * N, N, row0);
  __syncthreads();
  npass<true, true>(s, tws, 8, 2 * kRowsPerTile, 1, kRowWords, kRowWords, kRowsPerTile - 1, m.q);
  const uint32_t k = t - l1, K = P.num_p;
  for (uint32_t e = threadIdx.x; e < 2 * kTileWords; e += 256) {
    const uint32_t h = e / kTileWords;
    XP[((size_t)h * K + k) * N + base + (e - h * kTileWords)] = s[e];  // [0, 4q): the column pass finishes
  }
}

// ------------------------------------------------------------ ModDown P2
// w_{s,i} = sum_k [a_{s,k} p^_k^-1]_{p_k} [p^_k]_{q_i}, i <= level.
// grid (N / 256, 2, target groups of kTgtGroup towers).
template <int MAXK>
__global__ __launch_bounds__(256) void k_bconv_down(Dev64 P, uint32_t level, const uint64_t *__restrict__ XP,
                                                    uint64_t *__restrict__ W) {
  const uint32_t N = 1u << P.log_n, s = blockIdx.y, K = P.num_p, l1 = level + 1;
  const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t i0 = blockIdx.z * kTgtGroup, i1 = min(i0 + kTgtGroup, l1);
  uint32_t x0[MAXK], x1[MAXK];
#pragma unroll
  for (int k = 0; k < MAXK; k++) {
    x0[k] = x1[k] = 0;
    if ((uint32_t)k < K) {
      const uint64_t v =
          shoup(XP[((size_t)s * K + k) * N + c], P.dn_pre[2 * k], P.dn_pre[2 * k + 1], P.mods[P.num_q + k].q);
      x0[k] = (uint32_t)(v & kLo30);
      x1[k] = (uint32_t)(v >> 30);
    }
  }
  for (uint32_t i = i0; i < i1; i += 2) {
    const uint32_t ia = i, ib = min(i + 1, i1 - 1);
    uint64_t wa, wb;
    conv2<MAXK>(x0, x1, K, P.dn_cst + (size_t)ia * K, P.dn_cst + (size_t)ib * K, P.mods[ia], P.mods[ib], &wa, &wb);
    W[((size_t)s * l1 + ia) * N + c] = wa;
    W[((size_t)s * l1 + ib) * N + c] = wb;
  }
}

// ------------------------------------------------------------ ModDown P3-P4
// For Q tower i and a tile of rows: the forward row pass of both converted
// polynomials w_s (column pass done before), then
// out_s[i] = (acc_s[i] - w_s[i]) [P^-1]_{q_i}.  grid (R / kRowsPerTile, l+1).
__global__ __launch_bounds__(256) void k_row_moddown(Dev64 P, uint32_t level, const uint64_t *__restrict__ acc,
                                                     const uint64_t *__restrict__ W, uint64_t *__restrict__ out) {
  __shared__ uint64_t s[2 * kTileWords];
  __shared__ uint4 tws[kTileWords];
  const uint32_t N = 1u << P.log_n, i = blockIdx.y, l1 = level + 1, T = l1 + P.num_p;
  const Mod64 m = P.mods[i];
  const uint32_t row0 = blockIdx.x * kRowsPerTile;
  const size_t base = (size_t)row0 * kRowWords;
  stage_row_tw(tws, P.tw_fwd + (size_t)i * N, N, row0);
  for (uint32_t e = threadIdx.x; e < 2 * kTileWords; e += 256) {
    const uint32_t h = e / kTileWords;
    s[e] = W[((size_t)h * l1 + i) * N + base + (e - h * kTileWords)];
  }
  __syncthreads();
  npass<false, true>(s, tws, 8, 2 * kRowsPerTile, 1, kRowWords, kRowWords, kRowsPerTile - 1, m.q);
  const uint64_t pi = P.pinv[2 * i], pis = P.pinv[2 * i + 1];
  for (uint32_t e = threadIdx.x; e < 2 * kTileWords; e += 256) {
    const uint32_t h = e / kTileWords;
    const size_t o = base + (e - h * kTileWords);
    const uint64_t w = fwd_canon(s[e], m.q);
    out[((size_t)h * l1 + i) * N + o] = shoup(sub_mod(acc[((size_t)h * T + i) * N + o], w, m.q), pi, pis, m.q);
  }
}

// ------------------------------------------------------------ arithmetic probe
// The primitives above applied element-wise to caller arrays, for a test
// that compares each with a b mod q directly (not part of the method).
// Element i: a = a[i], b = b[i] (any words), the twiddle (w, ws); each
// primitive gets its operands reduced into the range it is specified for.
constexpr uint32_t kProbe64Out = 9;
__global__ __launch_bounds__(256) void k_arith_probe64(Mod64 m, uint4 tv, uint32_t n, const uint64_t *a,
                                                       const uint64_t *b, uint64_t *out) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint64_t q = m.q, ai = a[i], bi = b[i];
  uint64_t w, ws;
  tw_of(tv, &w, &ws);
  uint64_t *o = out + (size_t)i * kProbe64Out;
  o[0] = shoup(ai, w, ws, q);        // a w mod q
  o[1] = shoup_lazy4(ai, w, ws, q);  // a w mod q, in [0, 4q)
  const uint64_t ac = ai % q, bc = bi % q;
  Acc4 one;
  one.mac((uint32_t)(ac & kLo30), (uint32_t)(ac >> 30), bc);
  o[2] = redc(one.sum(), m);  // a b 2^-64 mod q
  Acc4 sum;  // the 16 products from element i on (cyclically), 2^-64
  for (uint32_t k = 0; k < 16; k++) {
    const uint32_t j = (i + k) % n;
    const uint64_t x = a[j] % q;
    sum.mac((uint32_t)(x & kLo30), (uint32_t)(x >> 30), b[j] % q);
  }
  o[3] = redc(sum.sum(), m);
  uint64_t x = ai % (8 * q), y = bi % (8 * q);
  ct(x, y, tv, q);  // (x + w y, x - w y), [0, 8q)
  o[4] = x;
  o[5] = y;
  uint64_t u = ai % (4 * q), v = bi % (4 * q);
  gs(u, v, tv, q);  // (u + v, (u - v) w), [0, 4q)
  o[6] = u;
  o[7] = v;
  o[8] = fwd_canon(ai % (8 * q), q);
}

// ------------------------------------------------------------ host side
namespace {

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return ks::mulmod64(a, b, q); }
uint64_t invmod(uint64_t a, uint64_t q) { return ks::invmod64(a, q); }
uint64_t shoup_of(uint64_t w, uint64_t q) { return ks::shoup64(w, q); }
uint64_t mont_of(uint64_t w, uint64_t q) { return ks::mont64(w, q); }

uint32_t bitrev(uint32_t x, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

ks_status_t default_moduli(uint32_t log_n, uint32_t num_q, uint32_t K, uint64_t *out) {
  std::vector<uint64_t> pr(num_q + K);
  if (ks::ntt_primes64(log_n, num_q + K, pr.data()) != 0) return KS_ERR_UNSUPPORTED;
  for (uint32_t i = 0; i < num_q; i++) out[i] = pr[K + i];
  for (uint32_t k = 0; k < K; k++) out[num_q + k] = pr[k];
  return KS_OK;
}

ks_status_t validate(const ks64_params_t *p, uint32_t *K_out) {
  if (!p) return KS_ERR_INVALID_ARG;
  if (p->log_n < 12 || p->log_n > 17) return KS_ERR_UNSUPPORTED;
  if (p->num_q == 0 || p->dnum == 0 || p->dnum > p->num_q) return KS_ERR_INVALID_ARG;
  const uint32_t alpha = (p->num_q + p->dnum - 1) / p->dnum, K = p->num_p ? p->num_p : alpha;
  if (p->num_q + K > kMaxTowers || alpha > 32 || K > 32 || p->dnum > 16) return KS_ERR_UNSUPPORTED;
  if (p->moduli) {
    const uint64_t two_n = 2ull << p->log_n;
    for (uint32_t i = 0; i < p->num_q + K; i++) {
      const uint64_t m = p->moduli[i];
      if (m <= (1ull << 59) || m >= (1ull << 60) || m % two_n != 1 || !ks::is_prime64(m)) return KS_ERR_INVALID_ARG;
      for (uint32_t j = 0; j < i; j++)
        if (p->moduli[j] == m) return KS_ERR_INVALID_ARG;
    }
  }
  *K_out = K;
  return KS_OK;
}

}  // namespace
}  // namespace ks64

using namespace ks64;

struct ks64_plan {
  uint32_t log_n = 0, n = 0, num_q = 0, num_p = 0, dnum = 0, alpha = 0, ntot = 0;
  int device = -1;
  std::vector<uint64_t> mod;
  Dev64 dev{};
  std::vector<void *> allocs;
};

namespace {

template <class T>
ks_status_t upload64(ks64_plan *pl, const std::vector<T> &h, const T **dst) {
  void *p = nullptr;
  const size_t bytes = std::max<size_t>(h.size() * sizeof(T), 256);
  if (hipMalloc(&p, bytes) != hipSuccess) return KS_ERR_NOMEM;
  pl->allocs.push_back(p);
  if (!h.empty() && hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return KS_ERR_DEVICE;
  *dst = (const T *)p;
  return KS_OK;
}

ks_status_t build(ks64_plan *pl, const ks64_params_t *p, uint32_t K) {
  pl->log_n = p->log_n;
  pl->n = 1u << p->log_n;
  pl->num_q = p->num_q;
  pl->num_p = K;
  pl->dnum = p->dnum;
  pl->alpha = (p->num_q + p->dnum - 1) / p->dnum;
  pl->ntot = p->num_q + K;
  if (hipGetDevice(&pl->device) != hipSuccess) return KS_ERR_DEVICE;
  pl->mod.resize(pl->ntot);
  if (p->moduli) std::copy(p->moduli, p->moduli + pl->ntot, pl->mod.begin());
  else if (default_moduli(p->log_n, p->num_q, K, pl->mod.data()) != KS_OK) return KS_ERR_UNSUPPORTED;
  const uint32_t N = pl->n, L1 = pl->num_q, T = pl->ntot, A = pl->alpha, D = pl->dnum;
  std::vector<Mod64> mods(T);
  std::vector<uint64_t> twf((size_t)T * N * 2), twi((size_t)T * N * 2);
  for (uint32_t g = 0; g < T; g++) {
    const uint64_t q = pl->mod[g];
    uint64_t inv = 1;  // q^-1 mod 2^64 by Newton's iteration
    for (int i = 0; i < 7; i++) inv *= 2 - q * inv;
    Mod64 &m = mods[g];
    m.q = q;
    m.qneg = (uint64_t)0 - inv;
    m.r64 = (uint64_t)(((u128)1 << 64) % q);
    m.r64s = shoup_of(m.r64, q);
    m.ninv = invmod(N % q, q);
    m.ninvs = shoup_of(m.ninv, q);
    const uint64_t psi = ks::min_root64(q, p->log_n), psi_inv = invmod(psi, q);
    uint64_t pw = 1, pwi = 1;
    std::vector<uint64_t> pows(N), powsi(N);
    for (uint32_t i = 0; i < N; i++) {
      pows[i] = pw;
      powsi[i] = pwi;
      pw = mulmod(pw, psi, q);
      pwi = mulmod(pwi, psi_inv, q);
    }
    for (uint32_t k = 0; k < N; k++) {
      const uint32_t e = bitrev(k, p->log_n);
      twf[((size_t)g * N + k) * 2] = pows[e];
      twf[((size_t)g * N + k) * 2 + 1] = shoup_of(pows[e], q);
      twi[((size_t)g * N + k) * 2] = powsi[e];
      twi[((size_t)g * N + k) * 2 + 1] = shoup_of(powsi[e], q);
    }
  }
  // ModUp conversion constants per level (the last live digit is partial)
  std::vector<uint64_t> up_pre((size_t)L1 * D * A * 2, 0), up_cst((size_t)L1 * D * A * T + 32, 0);
  for (uint32_t lv = 0; lv < L1; lv++)
    for (uint32_t j = 0; j < D; j++) {
      const uint32_t lo = j * A;
      if (lo > lv) break;
      const uint32_t hi = std::min(lo + A, lv + 1);
      for (uint32_t s = lo; s < hi; s++) {
        const size_t ix = ((size_t)lv * D + j) * A + (s - lo);
        const uint64_t qs = pl->mod[s];
        uint64_t qhat_s = 1;
        for (uint32_t u = lo; u < hi; u++)
          if (u != s) qhat_s = mulmod(qhat_s, pl->mod[u] % qs, qs);
        up_pre[ix * 2] = invmod(qhat_s, qs);
        up_pre[ix * 2 + 1] = shoup_of(up_pre[ix * 2], qs);
        for (uint32_t g = 0; g < T; g++) {
          const uint64_t mg = pl->mod[g];
          uint64_t qh = 1;
          for (uint32_t u = lo; u < hi; u++)
            if (u != s) qh = mulmod(qh, pl->mod[u] % mg, mg);
          up_cst[(((size_t)lv * D + j) * T + g) * A + (s - lo)] = mont_of(qh, mg);
        }
      }
    }
  // ModDown constants
  std::vector<uint64_t> dn_pre((size_t)K * 2), dn_cst((size_t)K * L1 + 32, 0), pinv((size_t)L1 * 2);
  for (uint32_t k = 0; k < K; k++) {
    const uint64_t pk = pl->mod[L1 + k];
    uint64_t ph = 1;
    for (uint32_t u = 0; u < K; u++)
      if (u != k) ph = mulmod(ph, pl->mod[L1 + u] % pk, pk);
    dn_pre[2 * k] = invmod(ph, pk);
    dn_pre[2 * k + 1] = shoup_of(dn_pre[2 * k], pk);
    for (uint32_t i = 0; i < L1; i++) {
      const uint64_t qi = pl->mod[i];
      uint64_t h = 1;
      for (uint32_t u = 0; u < K; u++)
        if (u != k) h = mulmod(h, pl->mod[L1 + u] % qi, qi);
      dn_cst[(size_t)i * K + k] = mont_of(h, qi);
    }
  }
  for (uint32_t i = 0; i < L1; i++) {
    const uint64_t qi = pl->mod[i];
    uint64_t P = 1;
    for (uint32_t k = 0; k < K; k++) P = mulmod(P, pl->mod[L1 + k] % qi, qi);
    pinv[2 * i] = invmod(P, qi);
    pinv[2 * i + 1] = shoup_of(pinv[2 * i], qi);
  }
  Dev64 &d = pl->dev;
  d.log_n = pl->log_n;
  d.num_q = L1;
  d.num_p = K;
  d.dnum = D;
  d.alpha = A;
  d.ntot = T;
  ks_status_t st;
  if ((st = upload64(pl, mods, &d.mods)) != KS_OK) return st;
  const uint64_t *tf = nullptr, *ti = nullptr;
  if ((st = upload64(pl, twf, &tf)) != KS_OK) return st;
  if ((st = upload64(pl, twi, &ti)) != KS_OK) return st;
  d.tw_fwd = (const uint4 *)tf;
  d.tw_inv = (const uint4 *)ti;
  if ((st = upload64(pl, up_pre, &d.up_pre)) != KS_OK) return st;
  if ((st = upload64(pl, up_cst, &d.up_cst)) != KS_OK) return st;
  if ((st = upload64(pl, dn_pre, &d.dn_pre)) != KS_OK) return st;
  if ((st = upload64(pl, dn_cst, &d.dn_cst)) != KS_OK) return st;
  if ((st = upload64(pl, pinv, &d.pinv)) != KS_OK) return st;
  return KS_OK;
}

void free_plan(ks64_plan *pl) {
  for (void *p : pl->allocs) (void)hipFree(p);
  pl->allocs.clear();
}

// One transform direction over a list of towers, split into launches of
// kList.  col_only: the column pass alone (forward: its first pass, words
// left in [0, 8q) for a fused row pass; inverse: its second pass, reading
// words in [0, 4q) that a fused row pass wrote).
hipError_t transform(const ks64_plan *pl, bool inverse, const uint64_t *src, uint64_t *dst,
                     const std::vector<uint32_t> &so, const std::vector<uint32_t> &dof,
                     const std::vector<uint32_t> &g, hipStream_t st, bool col_only = false) {
  const uint32_t N = pl->n, R = N / kRowWords;
  for (size_t b = 0; b < so.size(); b += kList) {
    List64 L{};
    L.count = (uint32_t)std::min<size_t>(kList, so.size() - b);
    for (uint32_t i = 0; i < L.count; i++) {
      L.src[i] = so[b + i];
      L.dst[i] = dof[b + i];
      L.g[i] = (uint16_t)g[b + i];
    }
    const dim3 grow(R / kRowsPerTile, L.count), gcol(kRowWords / kColsPerTile, L.count);
    if (col_only) {
      if (!inverse) hipLaunchKernelGGL(k_col<false>, gcol, dim3(256), 0, st, pl->dev, L, src, dst);
      else hipLaunchKernelGGL(k_col<true>, gcol, dim3(256), 0, st, pl->dev, L, src, dst);
    } else if (!inverse) {  // column pass (large distances) first, in place into dst
      hipLaunchKernelGGL(k_col<false>, gcol, dim3(256), 0, st, pl->dev, L, src, dst);
      List64 L2 = L;
      for (uint32_t i = 0; i < L.count; i++) L2.src[i] = L.dst[i];
      hipLaunchKernelGGL(k_row<false>, grow, dim3(256), 0, st, pl->dev, L2, dst, dst);
    } else {
      hipLaunchKernelGGL(k_row<true>, grow, dim3(256), 0, st, pl->dev, L, src, dst);
      List64 L2 = L;
      for (uint32_t i = 0; i < L.count; i++) L2.src[i] = L.dst[i];
      hipLaunchKernelGGL(k_col<true>, gcol, dim3(256), 0, st, pl->dev, L2, dst, dst);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

size_t ws_words(const ks64_plan *pl, uint32_t level) {
  const size_t L1 = level + 1, K = pl->num_p, T = L1 + K, D = (L1 + pl->alpha - 1) / pl->alpha;
  return (L1 + D * T + 2 * T + 2 * K + 2 * L1) * (size_t)pl->n;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + nb && y < x + na;
}

}  // namespace

extern "C" {

uint64_t ks64_root_of_unity(uint64_t q, uint32_t log_n) {
  if (log_n < 1 || log_n > 20) return 0;
  return ks::min_root64(q, log_n);
}

ks_status_t ks64_params_moduli(const ks64_params_t *p, uint64_t *host_out) {
  uint32_t K = 0;
  const ks_status_t st = validate(p, &K);
  if (st != KS_OK) return st;
  if (!host_out) return KS_ERR_INVALID_ARG;
  if (p->moduli) {
    std::copy(p->moduli, p->moduli + p->num_q + K, host_out);
    return KS_OK;
  }
  return default_moduli(p->log_n, p->num_q, K, host_out);
}

ks_status_t ks64_plan_create(const ks64_params_t *p, ks64_plan_t *out) {
  if (!out) return KS_ERR_INVALID_ARG;
  *out = nullptr;
  uint32_t K = 0;
  ks_status_t st = validate(p, &K);
  if (st != KS_OK) return st;
  ks64_plan *pl = new (std::nothrow) ks64_plan();
  if (!pl) return KS_ERR_NOMEM;
  st = build(pl, p, K);
  if (st != KS_OK) {
    free_plan(pl);
    delete pl;
    return st;
  }
  *out = pl;
  return KS_OK;
}

ks_status_t ks64_plan_destroy(ks64_plan_t plan) {
  if (!plan) return KS_ERR_INVALID_ARG;
  free_plan(plan);
  delete plan;
  return KS_OK;
}

ks_status_t ks64_plan_moduli(ks64_plan_t plan, uint64_t *host_out) {
  if (!plan || !host_out) return KS_ERR_INVALID_ARG;
  std::copy(plan->mod.begin(), plan->mod.end(), host_out);
  return KS_OK;
}

ks_status_t ks64_workspace_size(ks64_plan_t plan, uint32_t level, size_t *bytes) {
  if (!plan || !bytes || level >= plan->num_q) return KS_ERR_INVALID_ARG;
  *bytes = ws_words(plan, level) * sizeof(uint64_t);
  return KS_OK;
}

ks_status_t ks64_ntt(ks64_plan_t plan, uint32_t count, const uint32_t *g, int inverse, uint64_t *data,
                     void *stream) {
  if (!plan || (count && (!g || !data))) return KS_ERR_INVALID_ARG;
  if ((uintptr_t)data & 15) return KS_ERR_INVALID_ARG;
  std::vector<uint32_t> so(count), gg(count);
  for (uint32_t i = 0; i < count; i++) {
    if (g[i] >= plan->ntot) return KS_ERR_INVALID_ARG;
    so[i] = i;
    gg[i] = g[i];
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) return KS_ERR_INVALID_ARG;
  return transform(plan, inverse != 0, data, data, so, so, gg, (hipStream_t)stream) == hipSuccess ? KS_OK
                                                                                                     : KS_ERR_DEVICE;
}

}  // extern "C"

namespace {

// The key switch with a full key (seeded = false, evk [dnum][2][L+1+K][N])
// or a compressed one (evk the b halves [dnum][L+1+K][N], a halves from
// a_seed).
ks_status_t keyswitch64(ks64_plan_t plan, const uint64_t *evk, bool seeded, uint64_t a_seed, uint32_t level,
                        const uint64_t *in, uint64_t *out, void *workspace, size_t workspace_bytes, void *stream) {
  if (!plan || !evk || !in || !out || !workspace) return KS_ERR_INVALID_ARG;
  const ks64_plan *pl = plan;
  if (level >= pl->num_q) return KS_ERR_INVALID_ARG;
  if (((uintptr_t)evk | (uintptr_t)in | (uintptr_t)out) & 15) return KS_ERR_INVALID_ARG;
  if ((uintptr_t)workspace & 255) return KS_ERR_INVALID_ARG;
  const size_t need = ws_words(pl, level) * sizeof(uint64_t);
  if (workspace_bytes < need) return KS_ERR_BUDGET;
  const uint32_t N = pl->n, L1 = level + 1, K = pl->num_p, T = L1 + K, D = (L1 + pl->alpha - 1) / pl->alpha;
  const size_t lb = (size_t)N * sizeof(uint64_t);
  const size_t evk_b = (size_t)pl->dnum * (seeded ? 1 : 2) * pl->ntot * lb;
  if (overlaps(out, 2 * L1 * lb, in, L1 * lb) || overlaps(out, 2 * L1 * lb, evk, evk_b) ||
      overlaps(out, 2 * L1 * lb, workspace, workspace_bytes) || overlaps(workspace, workspace_bytes, in, L1 * lb) ||
      overlaps(workspace, workspace_bytes, evk, evk_b))
    return KS_ERR_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl->device) return KS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  uint64_t *X = (uint64_t *)workspace, *Y = X + (size_t)L1 * N, *ACC = Y + (size_t)D * T * N;
  uint64_t *XP = ACC + (size_t)2 * T * N, *W = XP + (size_t)2 * K * N;
  const uint32_t blocks = N / 256;
  std::vector<uint32_t> so, dof, g;
  // ModUp P1: INTT of every input tower
  for (uint32_t i = 0; i < L1; i++) { so.push_back(i); dof.push_back(i); g.push_back(i); }
  if (transform(pl, true, in, X, so, dof, g, st) != hipSuccess) return KS_ERR_DEVICE;
  // P2: every digit converted to the other towers of D_l
  const dim3 gup(blocks, D, (T + kTgtGroup - 1) / kTgtGroup);
  if (pl->alpha <= 8) hipLaunchKernelGGL(k_bconv_up<8>, gup, dim3(256), 0, st, pl->dev, level, X, Y);
  else if (pl->alpha <= 16) hipLaunchKernelGGL(k_bconv_up<16>, gup, dim3(256), 0, st, pl->dev, level, X, Y);
  else if (pl->alpha <= 24) hipLaunchKernelGGL(k_bconv_up<24>, gup, dim3(256), 0, st, pl->dev, level, X, Y);
  else hipLaunchKernelGGL(k_bconv_up<32>, gup, dim3(256), 0, st, pl->dev, level, X, Y);
  if (hipGetLastError() != hipSuccess) return KS_ERR_DEVICE;
  // P3: NTT of the converted towers (a digit's own towers are never read from Y)
  so.clear(); dof.clear(); g.clear();
  for (uint32_t j = 0; j < D; j++) {
    const uint32_t lo = j * pl->alpha, hi = std::min(lo + pl->alpha, L1);
    for (uint32_t t = 0; t < T; t++) {
      if (t >= lo && t < hi) continue;
      so.push_back(j * T + t); dof.push_back(j * T + t);
      g.push_back(t <= level ? t : pl->num_q + (t - L1));
    }
  }
  if (transform(pl, false, Y, Y, so, dof, g, st, true) != hipSuccess) return KS_ERR_DEVICE;
  // P3 row pass, P4/P5 key multiply-accumulate over the digits; for the K
  // special towers also ModDown P1's inverse row pass (into XP)
  const uint32_t rtiles = N / kRowWords / kRowsPerTile;
  if (seeded)
    hipLaunchKernelGGL(k_row_mac<true>, dim3(rtiles, T), dim3(256), 0, st, pl->dev, level, in, Y, evk, a_seed, ACC, XP);
  else
    hipLaunchKernelGGL(k_row_mac<false>, dim3(rtiles, T), dim3(256), 0, st, pl->dev, level, in, Y, evk, a_seed, ACC,
                       XP);
  if (hipGetLastError() != hipSuccess) return KS_ERR_DEVICE;
  // ModDown P1: the inverse column pass of the K special towers of both polynomials
  so.clear(); dof.clear(); g.clear();
  for (uint32_t s = 0; s < 2; s++)
    for (uint32_t k = 0; k < K; k++) { so.push_back(s * K + k); dof.push_back(s * K + k); g.push_back(pl->num_q + k); }
  if (transform(pl, true, XP, XP, so, dof, g, st, true) != hipSuccess) return KS_ERR_DEVICE;
  // P2: conversion P -> Q_l
  const dim3 gdn(blocks, 2, (L1 + kTgtGroup - 1) / kTgtGroup);
  if (K <= 8) hipLaunchKernelGGL(k_bconv_down<8>, gdn, dim3(256), 0, st, pl->dev, level, XP, W);
  else if (K <= 16) hipLaunchKernelGGL(k_bconv_down<16>, gdn, dim3(256), 0, st, pl->dev, level, XP, W);
  else if (K <= 24) hipLaunchKernelGGL(k_bconv_down<24>, gdn, dim3(256), 0, st, pl->dev, level, XP, W);
  else hipLaunchKernelGGL(k_bconv_down<32>, gdn, dim3(256), 0, st, pl->dev, level, XP, W);
  if (hipGetLastError() != hipSuccess) return KS_ERR_DEVICE;
  // P3: NTT; P4: subtract, times P^-1
  so.clear(); dof.clear(); g.clear();
  for (uint32_t s = 0; s < 2; s++)
    for (uint32_t i = 0; i < L1; i++) { so.push_back(s * L1 + i); dof.push_back(s * L1 + i); g.push_back(i); }
  if (transform(pl, false, W, W, so, dof, g, st, true) != hipSuccess) return KS_ERR_DEVICE;
  hipLaunchKernelGGL(k_row_moddown, dim3(rtiles, L1), dim3(256), 0, st, pl->dev, level, ACC, W, out);
  return hipGetLastError() == hipSuccess ? KS_OK : KS_ERR_DEVICE;
}

}  // namespace

extern "C" {

ks_status_t ks64_keyswitch(ks64_plan_t plan, const uint64_t *evk, uint32_t level, const uint64_t *in,
                           uint64_t *out, void *workspace, size_t workspace_bytes, void *stream) {
  return keyswitch64(plan, evk, false, 0, level, in, out, workspace, workspace_bytes, stream);
}

ks_status_t ks64_keyswitch_seeded(ks64_plan_t plan, const uint64_t *evk_b, uint64_t a_seed, uint32_t level,
                                  const uint64_t *in, uint64_t *out, void *workspace, size_t workspace_bytes,
                                  void *stream) {
  return keyswitch64(plan, evk_b, true, a_seed, level, in, out, workspace, workspace_bytes, stream);
}

ks_status_t ks64_arith_probe(uint64_t q, uint64_t w, uint32_t n, const uint64_t *a, const uint64_t *b, uint64_t *out,
                             void *stream) {
  if (!a || !b || !out || n == 0) return KS_ERR_INVALID_ARG;
  if (!(q & 1u) || q <= (1ull << 59) || q >= (1ull << 60) || w >= q) return KS_ERR_INVALID_ARG;
  uint64_t inv = 1;  // q^-1 mod 2^64 by Newton's iteration
  for (int i = 0; i < 7; i++) inv *= 2 - q * inv;
  Mod64 m{};
  m.q = q;
  m.qneg = (uint64_t)0 - inv;
  const uint64_t ws = shoup_of(w, q);
  const uint4 tv = make_uint4((uint32_t)w, (uint32_t)(w >> 32), (uint32_t)ws, (uint32_t)(ws >> 32));
  hipLaunchKernelGGL(k_arith_probe64, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, m, tv, n, a, b, out);
  return hipGetLastError() == hipSuccess ? KS_OK : KS_ERR_DEVICE;
}

}  // extern "C"
