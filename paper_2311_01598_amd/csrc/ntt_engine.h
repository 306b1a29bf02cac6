// ntt_engine.h -- register/LDS building blocks of the two-pass negacyclic NTT.
//
// The length-N transform (N = 2^log_n, evaluation order a(psi^(2 brv(j)+1)))
// is the in-place Cooley-Tukey network whose stage s (1..log_n) pairs
// j and j + N/2^s with twiddle psi^brv(2^(s-1) + (j >> (log_n+1-s))).
// Write N = 2^a * 2^b and view the array as 2^a rows of 2^b words:
//   * stages 1..a pair words of one column -> "column pass": 2^b independent
//     length-2^a sub-transforms with twiddle node M = 1;
//   * stages a+1..a+b stay inside one row -> "row pass": row r is a
//     length-2^b sub-transform with twiddle node M = 2^a + r.
// A sub-transform of length 2^A at node M uses, at its stage s (1..A) and
// element k, the twiddle index M*2^(s-1) + (k >> (A+1-s)).
// The inverse runs the same network backwards with Gentleman-Sande
// butterflies and psi^-brv twiddles, without the N^-1 factor.
//
// A sub-transform is computed in phases of R consecutive stages; in a phase
// each thread holds a group of 2^R elements in registers,
//   k = hi * 2^(A-S0+1) + u * 2^LOB + lo,   LOB = A-S0-R+1, u < 2^R,
// and the phase's twiddles are M*2^(s-1) + hi*2^t + (u >> (R-t)).
#pragma once
#include "modarith.h"

namespace ks {

template <int A, int S0, int R>
struct Phase {
  static constexpr int LOB = A - S0 - R + 1;
  static constexpr int GROUPS = 1 << (A - R);
  __device__ static __forceinline__ int hi(int g) { return g >> LOB; }
  __device__ static __forceinline__ int base(int g) { return ((g >> LOB) << (LOB + R)) | (g & ((1 << LOB) - 1)); }
  __device__ static __forceinline__ int elem(int g, int u) { return base(g) + (u << LOB); }
};

// Twiddle sources: a global table (entries read with a global load) or a
// copy of its first entries staged in LDS.
struct LdsTw {
  const uint2 *p;
};
__device__ __forceinline__ uint2 tw_at(const uint2 *tw, uint32_t i) { return ldg2(tw + i); }
__device__ __forceinline__ uint2 tw_at(LdsTw tw, uint32_t i) { return tw.p[i]; }

// Forward stages S0..S0+R-1 on one register group.
template <int A, int S0, int R, class TW>
__device__ __forceinline__ void ct_group(uint32_t (&x)[1 << R], int g, uint32_t M, TW tw, uint32_t q) {
  const uint32_t hi = (uint32_t)Phase<A, S0, R>::hi(g);
#pragma unroll
  for (int t = 0; t < R; t++) {
    const int half = 1 << (R - 1 - t);
    const uint32_t node = (M << (S0 + t - 1)) + (hi << t);
#pragma unroll
    for (int u = 0; u < (1 << R); u++) {
      if (u & half) continue;
      const uint2 w = tw_at(tw, node + (uint32_t)(u >> (R - t)));
      bfly_ct(x[u], x[u + half], w.x, w.y, q);
    }
  }
}

// Inverse stages S0+R-1..S0 on one register group.
template <int A, int S0, int R, class TW>
__device__ __forceinline__ void gs_group(uint32_t (&x)[1 << R], int g, uint32_t M, TW tw, uint32_t q) {
  const uint32_t hi = (uint32_t)Phase<A, S0, R>::hi(g);
#pragma unroll
  for (int t = R - 1; t >= 0; t--) {
    const int half = 1 << (R - 1 - t);
    const uint32_t node = (M << (S0 + t - 1)) + (hi << t);
#pragma unroll
    for (int u = 0; u < (1 << R); u++) {
      if (u & half) continue;
      const uint2 w = tw_at(tw, node + (uint32_t)(u >> (R - t)));
      bfly_gs(x[u], x[u + half], w.x, w.y, q);
    }
  }
}

// One phase over LDS: groups tig, tig+TPS, ... of the sub-transform whose
// element k lives at lds[addr(k)].
template <int A, int S0, int R, int TPS, bool INV, class Addr>
__device__ __forceinline__ void lds_phase(uint32_t *lds, const Addr &addr, int tig, uint32_t M,
                                          const uint2 *__restrict__ tw, uint32_t q) {
  using Ph = Phase<A, S0, R>;
  static_assert(Ph::GROUPS % TPS == 0, "groups must divide evenly among threads");
#pragma unroll
  for (int gi = 0; gi < Ph::GROUPS / TPS; gi++) {
    const int g = tig + gi * TPS;
    uint32_t x[1 << R];
#pragma unroll
    for (int u = 0; u < (1 << R); u++) x[u] = lds[addr(Ph::elem(g, u))];
    if (INV) gs_group<A, S0, R>(x, g, M, tw, q);
    else ct_group<A, S0, R>(x, g, M, tw, q);
#pragma unroll
    for (int u = 0; u < (1 << R); u++) lds[addr(Ph::elem(g, u))] = x[u];
  }
}

// Phase split of a length-2^A sub-transform: R1 stages then R2 stages.
template <int A> struct Split;
template <> struct Split<4> { static constexpr int R1 = 4, R2 = 0; };
template <> struct Split<5> { static constexpr int R1 = 5, R2 = 0; };
template <> struct Split<6> { static constexpr int R1 = 3, R2 = 3; };
template <> struct Split<7> { static constexpr int R1 = 4, R2 = 3; };
template <> struct Split<8> { static constexpr int R1 = 4, R2 = 4; };
template <> struct Split<9> { static constexpr int R1 = 5, R2 = 4; };

template <int A>
struct SubNtt {
  static constexpr int R1 = Split<A>::R1, R2 = Split<A>::R2;
  static constexpr int RMAX = R1 > R2 ? R1 : R2;
  static constexpr int TPS = 1 << (A - RMAX);  // threads per sub-transform

  // Whole sub-transform in LDS; the caller synchronises before and after.
  template <bool INV, class Addr>
  __device__ static __forceinline__ void run(uint32_t *lds, const Addr &addr, int tig, uint32_t M,
                                             const uint2 *__restrict__ tw, uint32_t q) {
    if constexpr (!INV) {
      lds_phase<A, 1, R1, TPS, false>(lds, addr, tig, M, tw, q);
      if constexpr (R2 > 0) {
        __syncthreads();
        lds_phase<A, 1 + R1, R2, TPS, false>(lds, addr, tig, M, tw, q);
      }
    } else {
      if constexpr (R2 > 0) {
        lds_phase<A, 1 + R1, R2, TPS, true>(lds, addr, tig, M, tw, q);
        __syncthreads();
      }
      lds_phase<A, 1, R1, TPS, true>(lds, addr, tig, M, tw, q);
    }
  }
};

}  // namespace ks
