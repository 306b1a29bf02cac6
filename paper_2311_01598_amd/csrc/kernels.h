// kernels.h -- host launchers of the key-switching kernels.
#pragma once
#include "plan.h"

namespace ks {

constexpr uint32_t kMaxList = 96;

// A list of limbs for the generic NTT passes: limb c is read from
// src + src_off[c]*N, written to dst + dst_off[c]*N, modulus number g[c].
struct LimbList {
  uint32_t count;
  uint32_t src_off[kMaxList];
  uint32_t dst_off[kMaxList];
  uint16_t g[kMaxList];
};

// Generic column / row passes (forward = stages 1..a then a+1..log_n;
// inverse = the reverse, unscaled).  Lists longer than kMaxList are split.
hipError_t launch_ntt(const Plan &pl, bool inverse, const uint32_t *src, uint32_t *dst,
                      const std::vector<uint32_t> &src_off, const std::vector<uint32_t> &dst_off,
                      const std::vector<uint32_t> &g, hipStream_t st);
hipError_t launch_col(const Plan &pl, bool inverse, const uint32_t *src, uint32_t *dst, const LimbList &L,
                      hipStream_t st);
hipError_t launch_row(const Plan &pl, bool inverse, const uint32_t *src, uint32_t *dst, const LimbList &L,
                      hipStream_t st);
// data[c] *= N^-1 and canonicalise (forward: canonicalise only).
hipError_t launch_finish_ntt(const Plan &pl, bool inverse, uint32_t *data, const LimbList &L, hipStream_t st);

// ModUp P2 for digits j0..j0+nd-1 at `level`.  x holds the unscaled INTT
// output: [l+1][N], or only the digit's towers [s][N] when digit_rel.  y
// receives [nd][T][N] ([T][N] when digit_rel); own-digit slots untouched.
hipError_t launch_bconv_up(const Plan &pl, uint32_t level, uint32_t j0, uint32_t nd, bool digit_rel,
                           const uint32_t *x, uint32_t *y, hipStream_t st);
// ModUp P4 (Max-Parallel): z[j][s][t] = REDC(yhat[j][t] * evk[j][s][g(t)]);
// yhat is y (lazy, NTT domain) except on digit j's own towers where it is d.
hipError_t launch_keymul(const Plan &pl, uint32_t level, const uint32_t *d, const uint32_t *y, const uint32_t *evk,
                         uint32_t *z, hipStream_t st);
// ModUp P5 (Max-Parallel): acc[s][t] = sum_j z[j][s][t].
hipError_t launch_reduce_digits(const Plan &pl, uint32_t level, const uint32_t *z, uint32_t *acc, hipStream_t st);
// ModUp P4+P5 for one digit (Digit-Centric): acc[s][t] (+)= REDC(yhat * evk).
hipError_t launch_keymac_digit(const Plan &pl, uint32_t level, uint32_t j, const uint32_t *d, const uint32_t *yj,
                               const uint32_t *evk, uint32_t *acc, hipStream_t st);
// ModDown P2: xp [2][K][N] unscaled INTT of acc's P towers -> w [2][l+1][N].
hipError_t launch_bconv_down(const Plan &pl, uint32_t level, const uint32_t *xp, uint32_t *w, hipStream_t st);
// ModDown P4: out[s][i] = (acc[s][i] - what[s][i]) * P^-1 (with the 2^32 fold).
hipError_t launch_moddown_final(const Plan &pl, uint32_t level, const uint32_t *acc, const uint32_t *what,
                                uint32_t *out, hipStream_t st);

// Output-Centric fused kernels, see kernels.hip.
struct OcArgs {
  const uint32_t *d;     // [l+1][N] input
  const uint32_t *evk;   // [dnum][2][L+1+K][N]
  uint32_t *out;         // [2][l+1][N]
  uint32_t *xt;          // [l+1][N]   ModUp P1 output (unscaled INTT, lazy)
  uint32_t *ycol;        // [ndig][T][N] column-pass output of ModUp P2/P3
  uint32_t *zp;          // [2][K][N]  ModDown P1 row-pass output
  uint32_t *wcol;        // [2][l+1][N] column-pass output of ModDown P2/P3
  uint32_t level;
};
hipError_t launch_oc(const Plan &pl, const OcArgs &a, hipStream_t st);
// Steps 2-7 of the Output-Centric order for a column pass of length 2^A
// (explicitly instantiated in oc_a<A>.hip).
template <int A>
hipError_t oc_cols(const Plan &pl, const OcArgs &a, hipStream_t st);

}  // namespace ks
