// modarith.h -- exact uint32 modular arithmetic for 30-bit NTT primes on gfx950.
//
// All moduli satisfy 2^29 < q < 2^30, so 4q < 2^32: lazy values in [0, 4q)
// fit a 32-bit lane.  Three reductions are used:
//   * Shoup multiplication by a precomputed constant w (companion
//     w' = floor(w * 2^32 / q)): a*w mod q in [0, 2q) for any a < 2^32,
//     one mul_hi and two mul_lo;
//   * REDC of a 64-bit accumulator T (sum of at most 16 products of values
//     below 2^30): returns T * 2^-32 mod q, canonical.  The high word is first
//     brought below 2q with a one-word Barrett step (mu = floor(2^32/q)), so
//     T' = hi*2^32 + lo < 2q*2^32 and (T' + u q)/2^32 < 3q;
//   * conditional subtraction csub(a, m) = min(a, a - m) (unsigned).
// Constants that meet a REDC carry the factor 2^32 (Montgomery form), so a
// dot product followed by one REDC yields the plain residue.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "range_check.h"

namespace ks {

// Global-memory views of generic pointers.  Buffers reached through a job
// table or a plan struct are generic (flat) pointers to the compiler; a flat
// access counts against both the memory and the LDS wait counters, so an LDS
// wait would also wait for every outstanding HBM load.  Every HBM access of
// the kernels goes through one of these casts instead.
#define KS_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const KS_GLOBAL T *gp(const T *p) {
  return (const KS_GLOBAL T *)p;
}
template <class T>
__device__ __forceinline__ KS_GLOBAL T *gp(T *p) {
  return (KS_GLOBAL T *)p;
}
// Vector loads and stores through native vector types (HIP's uint2 / uint4
// classes cannot be copied out of another address space).
typedef uint32_t ks_v2u __attribute__((ext_vector_type(2)));
typedef uint32_t ks_v4u __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint2 ldg2(const uint2 *p) {
  const ks_v2u v = *(const KS_GLOBAL ks_v2u *)p;
  return make_uint2(v.x, v.y);
}
__device__ __forceinline__ uint4 ldg4(const void *p) {
  const ks_v4u v = *(const KS_GLOBAL ks_v4u *)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}
// Uniform reads of read-only plan tables through the scalar data cache (the
// constant address space): the value lands in SGPRs instead of occupying a
// VGPR in every lane.  Only for addresses that are the same across the wave
// and tables that no kernel writes.
#define KS_CONST __attribute__((address_space(4)))
__device__ __forceinline__ uint32_t ldc(const uint32_t *p) { return *(const KS_CONST uint32_t *)p; }
__device__ __forceinline__ uint2 ldc2(const uint2 *p) {
  const KS_CONST uint32_t *w = (const KS_CONST uint32_t *)p;
  return make_uint2(w[0], w[1]);
}
__device__ __forceinline__ double ldcd(const double *p) { return *(const KS_CONST double *)p; }

// Raw buffer access: one 128-bit resource (base, size in bytes) in SGPRs, a
// per-thread byte offset in a VGPR and a uniform byte offset in an SGPR, so
// a strided walk over a limb costs no vector address arithmetic.  Accesses
// past the size read 0 / are dropped by the hardware bounds check.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ uint32_t buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)voff, (int)soff, 0);
}
// The same store with the non-temporal cache policy (bit 1 of the buffer
// instruction's cache-policy operand), for data written once and read once
// by a later launch: the basis-conversion outputs.
__device__ __forceinline__ void buf_st_nt(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)voff, (int)soff, 2);
}
// Streaming variants for data touched once per key switch (the key words,
// the output): non-temporal hints, so that they do not push the reused
// tables and intermediates out of the caches.
__device__ __forceinline__ uint4 ldg4_nt(const void *p) {
  const ks_v4u v = __builtin_nontemporal_load((const KS_GLOBAL ks_v4u *)p);
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void stg4_nt(void *p, uint4 v) {
  ks_v4u t;
  t.x = v.x; t.y = v.y; t.z = v.z; t.w = v.w;
  __builtin_nontemporal_store(t, (KS_GLOBAL ks_v4u *)p);
}
__device__ __forceinline__ void stg4(void *p, uint4 v) {
  ks_v4u t;
  t.x = v.x; t.y = v.y; t.z = v.z; t.w = v.w;
  *(KS_GLOBAL ks_v4u *)p = t;
}

struct ModQ {
  uint32_t q;        // modulus
  uint32_t qinv;     // -q^-1 mod 2^32
  uint32_t mu;       // floor(2^32 / q)
  uint32_t pad;
};
// Shoup companion floor(w 2^32 / q) of w < q from qrecip = 2^32 / q (double):
// the double product is within 2^-20 of the exact quotient, so its floor r
// is off by at most one; the remainder w 2^32 - r q (exact modulo 2^32,
// and within (-2^31, 2^31) because it lies in [-q, 2q)) tells which way.
__device__ __forceinline__ uint32_t shoup_companion(uint32_t w, uint32_t q, double qrecip) {
  uint32_t r = (uint32_t)((double)w * qrecip);
  const int32_t t = (int32_t)(0u - r * q);
  r = t < 0 ? r - 1u : r;
  r = t >= (int32_t)q ? r + 1u : r;
  return r;
}
__device__ __forceinline__ ModQ ldmodc(const ModQ *p) {  // uniform address (see ldc)
  const KS_CONST uint32_t *w = (const KS_CONST uint32_t *)p;
  ModQ m;
  m.q = w[0]; m.qinv = w[1]; m.mu = w[2]; m.pad = w[3];
  return m;
}
__device__ __forceinline__ ModQ ldmod(const ModQ *p) {
  const ks_v4u v = *(const KS_GLOBAL ks_v4u *)p;
  ModQ m;
  m.q = v.x; m.qinv = v.y; m.mu = v.z; m.pad = v.w;
  return m;
}

__device__ __forceinline__ uint32_t csub(uint32_t a, uint32_t m) {
  uint32_t d = a - m;
  return d < a ? d : a;  // a >= m ? a - m : a
}

// -q mod 2^32, hidden from the optimiser (which would otherwise turn
// h * (-q) back into a subtraction of h * q) so a w - h q folds into one
// multiply-add.  The empty asm emits nothing and is shared between uses.
__device__ __forceinline__ uint32_t neg_mod(uint32_t q) {
  uint32_t nq = 0u - q;
  asm("" : "+v"(nq));
  return nq;
}

// a * w mod q in [0, 2q), any a < 2^32.
__device__ __forceinline__ uint32_t mul_shoup(uint32_t a, uint32_t w, uint32_t wp, uint32_t q) {
  const uint32_t h = __umulhi(a, wp);
  const uint32_t r = a * w + h * neg_mod(q);
  KS_RANGE(r < 2 * q, KS_RC_SHOUP_OUT);
  return r;
}

// One term of a sum of at most 16 products of values below 2^30.
__device__ __forceinline__ uint64_t mad64(uint32_t a, uint32_t b, uint64_t c) {
  KS_RANGE((a | b) < (1u << 30), KS_RC_MAC_OPND);
  const uint64_t r = (uint64_t)a * (uint64_t)b + c;
  KS_RANGE(r >= c, KS_RC_MAC_WRAP);
  return r;
}

// T * 2^-32 mod q in [0, 3q), for any T < 2^64: REDC without its final
// conditional subtractions, for consumers that take lazy words (a forward
// transform, a Shoup product).
__device__ __forceinline__ uint32_t redc64_lazy(uint64_t T, const ModQ &m) {
  uint32_t hi = (uint32_t)(T >> 32), lo = (uint32_t)T;
  hi += __umulhi(hi, m.mu) * neg_mod(m.q);  // hi - floor(hi mu / 2^32) q, in [0, 2q)
  uint32_t u = lo * m.qinv;
  uint64_t s = (uint64_t)u * m.q + (((uint64_t)hi << 32) | lo);
  const uint32_t r = (uint32_t)(s >> 32);
  KS_RANGE(r < 3 * m.q, KS_RC_REDC_OUT);
  return r;
}

// T * 2^-32 mod q, canonical, for any T < 2^64.
__device__ __forceinline__ uint32_t redc64(uint64_t T, const ModQ &m) {
  uint32_t hi = (uint32_t)(T >> 32), lo = (uint32_t)T;
  hi += __umulhi(hi, m.mu) * neg_mod(m.q);  // hi - floor(hi mu / 2^32) q, in [0, 2q)
  uint32_t u = lo * m.qinv;
  uint64_t s = (uint64_t)u * m.q + (((uint64_t)hi << 32) | lo);
  uint32_t r = (uint32_t)(s >> 32);      // [0, 3q)
  r = csub(r, m.q);
  r = csub(r, m.q);
  KS_RANGE(r < (KS_RANGE_STRICT() ? m.q / 2 : m.q), KS_RC_REDC_OUT);
  return r;
}

// Compressed keys (Sec. IV-D): the a half of a key pair is regenerated where
// it is consumed instead of read.  The generator is SplitMix64 (Steele, Lea
// and Flood 2014) evaluated at a counter: output t of seed s mixes
// s + (t + 1) gamma.  Word k of row g of digit j's a half uses the counter
// t = (j (L+1+K) + g) N + k, which is the word's position in the b halves;
// the word is x 2^-32 mod m_g (one REDC of the 64-bit output, canonical).
// Four consecutive counters from t.
__device__ __forceinline__ void seeded_a4(uint32_t (&a)[4], uint64_t seed, uint32_t t, const ModQ &m) {
  constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;
  uint64_t z = seed + ((uint64_t)t + 1) * kGamma;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    uint64_t x = z;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    x ^= x >> 31;
    a[i] = redc64(x, m);
    z += kGamma;
  }
}

// The automorphism X -> X^k (k odd) in the evaluation domain: slot j holds
// the value at psi^(2 brv(j) + 1), so the slot of a(X^k) takes a's slot
// pi(j) with 2 brv(pi(j)) + 1 = k (2 brv(j) + 1) mod 2N.  (The product is
// only needed modulo 2N, a power of two, so 32-bit wrap-around is exact.)
// pi maps every aligned block of 2^b slots onto one aligned block.
__device__ __forceinline__ uint32_t galois_perm(uint32_t j, uint32_t k, uint32_t log_n) {
  const uint32_t e = 2u * (__brev(j) >> (32 - log_n)) + 1u;
  const uint32_t e2 = (k * e) & ((2u << log_n) - 1u);
  return __brev((e2 - 1u) >> 1) >> (32 - log_n);
}

// Harvey forward (Cooley-Tukey) butterfly, inputs and outputs in [0, 4q).
// The forward twiddle tables hold (-w mod 2^32, w') so that the Shoup
// product comes out negated: nt = h q + y (-w) = -(y w - h q) = -t mod 2^32
// with t in [0, 2q); then x' = a + t = a - nt and y' = a + 2q - t =
// a + 2q + nt, a single three-input add.
__device__ __forceinline__ void bfly_ct(uint32_t &x, uint32_t &y, uint32_t wneg, uint32_t wp, uint32_t q) {
  KS_RANGE(x < 4 * q && y < 4 * q, KS_RC_CT_IN);
  const uint32_t two_q = q << 1;
  const uint32_t a = csub(x, two_q);
  const uint32_t h = __umulhi(y, wp);
  const uint32_t nt = h * q + y * wneg;
  x = a - nt;
  y = a + two_q + nt;
}

// Harvey inverse (Gentleman-Sande) butterfly, inputs and outputs in [0, 2q);
// inverse tables hold (w, w').
__device__ __forceinline__ void bfly_gs(uint32_t &x, uint32_t &y, uint32_t w, uint32_t wp, uint32_t q) {
  KS_RANGE(x < 2 * q && y < 2 * q, KS_RC_GS_IN);
  const uint32_t two_q = q << 1;
  const uint32_t a = x, b = y;
  x = csub(a + b, two_q);
  y = mul_shoup(a + two_q - b, w, wp, q);
}

// [0, 4q) -> [0, q)
__device__ __forceinline__ uint32_t canon4(uint32_t a, uint32_t q) {
  KS_RANGE(a < 4 * q, KS_RC_CANON4_IN);
  return csub(csub(a, q << 1), q);
}

}  // namespace ks
