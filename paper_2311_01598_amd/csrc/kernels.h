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

// Compressed keys: writes the a half of every pair of the full-layout key evk
// [dnum][2][L+1+K][N] from the seed (the b halves are left as they are).
hipError_t launch_expand_a(const Plan &pl, uint64_t seed, uint32_t *evk, hipStream_t st);
// out[c][j] = in[c][pi(j)] for `count` limbs [count][N]: the automorphism
// X -> X^galois in the evaluation domain.
hipError_t launch_automorphism(const Plan &pl, uint32_t galois, uint32_t count, const uint32_t *in, uint32_t *out,
                               hipStream_t st);
// One term of a double-hoisted rotation sum: the rotation's key (full
// layout), its plaintext diagonal ([L+1+K][N] in key-row order, or null for
// 1) and its Galois element.
struct RotTerm {
  const uint32_t *evk;
  const uint32_t *diag;
  uint32_t galois, pad;
};
// ACC [2][T] (carrying 2^-32, as the MP ModDown expects) = sum over the terms
// of diag * sum_j sigma(yhat_j) * evk[j]; yhat_j is Y's digit j with the
// digit's own towers read from d.
hipError_t launch_rotsum_keymul(const Plan &pl, uint32_t level, const uint32_t *d, const uint32_t *y,
                                const RotTerm *terms, uint32_t nterm, uint32_t *acc, hipStream_t st);
// out[0][i] += sum over the terms of diag * sigma(c0[i]).
hipError_t launch_rotsum_c0(const Plan &pl, uint32_t level, const uint32_t *c0, const RotTerm *terms, uint32_t nterm,
                            uint32_t *out, hipStream_t st);
// Tensor product of (a0, a1) and (b0, b1) at `level`: d [3][l+1][N] =
// (a0 b0, a0 b1 + a1 b0, a1 b1), pointwise, canonical.
hipError_t launch_tensor(const Plan &pl, uint32_t level, const uint32_t *a0, const uint32_t *a1, const uint32_t *b0,
                         const uint32_t *b1, uint32_t *d, hipStream_t st);

// ------------------------------------------------------------ Output-Centric
// Phases in issue order (see oc_kernels.h).
enum OcPhase : uint32_t {
  OC_INTT_ROW = 0, OC_INTT_COL, OC_UP_P, OC_ROW_P, OC_UP_Q, OC_INTT_COL_DN, OC_DN, OC_ROW_Q, OC_NPHASE
};
// Launch-only phase: the UP_P and UP_Q tiles of a job in one grid (UP_P
// first).  Both depend only on INTT_COL, so one launch fills the device with
// both instead of running them one after the other.
constexpr uint32_t OC_UP_PQ = OC_NPHASE;
// Launch-only phases: ROW_P / ROW_Q for compressed keys (Sec. IV-D), which
// read only the b halves and regenerate the a halves from the job's seed.
constexpr uint32_t OC_ROW_P_SEEDED = OC_NPHASE + 1;
constexpr uint32_t OC_ROW_Q_SEEDED = OC_NPHASE + 2;
// Launch-only phases: ROW_P / ROW_Q for the callers of the key switch
// (rotation, multiplication): the digits are read through the job's
// automorphism and ROW_Q adds the job's addends to its output.
constexpr uint32_t OC_ROW_P_EXT = OC_NPHASE + 3;
constexpr uint32_t OC_ROW_Q_EXT = OC_NPHASE + 4;
// Both: extended row stages with compressed keys (rotation keys stored as
// their b halves and a seed).
constexpr uint32_t OC_ROW_P_SEEDED_EXT = OC_NPHASE + 5;
constexpr uint32_t OC_ROW_Q_SEEDED_EXT = OC_NPHASE + 6;
// Double hoisting: ROW_P / ROW_Q summing the job's rotation terms before one
// ModDown.
constexpr uint32_t OC_ROW_P_SUM = OC_NPHASE + 7;
constexpr uint32_t OC_ROW_Q_SUM = OC_NPHASE + 8;
// Flag on a row phase's launch id: every job of the launch has at most 4
// transforms per round loop of a row tile (ROW_P: ndig, ROW_Q: ndig + 1, the
// summing ROW_Q: ndig - 1 per term), so the tiles run one round, compiled
// without the loop (far fewer live registers).
constexpr uint32_t OC_ONE_ROUND = 64;
// Flag on the summing ROW_Q launch id (with OC_ONE_ROUND): every term has at
// most 2 foreign digits, so a round transforms two terms' digits at once.
constexpr uint32_t OC_PAIR_TERMS = 128;
// The phase a launch id runs (launch ids carry the flags above).
constexpr uint32_t OC_PHASE_BITS = 63;

// Which row-stage kernels a launch uses.
enum OcRowVariant : uint32_t { OC_ROWS_PLAIN = 0, OC_ROWS_SEEDED, OC_ROWS_EXT, OC_ROWS_SEEDED_EXT, OC_ROWS_SUM };
// Which phases a launch sequence runs: all, ModUp only (INTT_ROW .. UP_PQ),
// or the rest (ROW_P .. ROW_Q) on the ModUp output of an earlier launch.
enum OcPart : uint32_t { OC_PART_ALL = 0, OC_PART_MODUP, OC_PART_REST };

// One key switch as the OC kernels see it (device-visible, by value or in a
// job table).  Workspace regions: xt [l+1][N] ModUp P1 output, ycol
// [ndig][T][N] column-pass output of ModUp P2/P3, zp [2][K][N] ModDown P1,
// wcol [2][l+1][N] column-pass output of ModDown P2/P3.  evk is the full key
// [dnum][2][L+1+K][N], or for a compressed key its b halves [dnum][L+1+K][N]
// with a_seed regenerating the a halves (the seeded row phases).  The
// extended row phases read digit word j of a row at the automorphism's
// pi(j) (galois = k of X -> X^k, 1 = none) and add add0[t][pi(j)] and
// add1[t][pi(j)] ([l+1][N] each, either may be null) to the two outputs.
// The summing row phases take the rotation terms terms[0..nterm) instead of
// evk and galois, and add0 = c0.
struct OcJob {
  const uint32_t *d;
  const uint32_t *evk;
  uint32_t *out;
  uint32_t *xt, *ycol, *zp, *wcol;
  const uint32_t *add0, *add1;
  const RotTerm *terms;
  uint64_t a_seed;
  uint32_t level, ttu, ttd, galois, nterm, pad;
  uint32_t tiles[OC_NPHASE];  // tile count of every phase for this job
};

// Segment of the persistent work queue: items [start, next.start) are the
// tiles of `phase` for job `job`.
struct OcSeg {
  uint32_t start, job, phase, pad;
};

constexpr int kRB = 16;   // rows per OC inverse-row tile (one transform per row)
constexpr int kRBQ = 4;   // rows per OC ROW_P / ROW_Q tile (four transforms per row in parallel)

__host__ __device__ __forceinline__ uint32_t oc_gidx(uint32_t num_q, uint32_t level, uint32_t t) {
  return t <= level ? t : num_q + (t - level - 1);
}
__host__ __device__ __forceinline__ uint32_t cdiv(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

// Phases each phase waits for in the persistent launch (bit q = phase q
// complete for the same job).
__host__ __device__ constexpr uint32_t oc_deps(uint32_t phase) {
  return phase == OC_INTT_COL      ? (1u << OC_INTT_ROW)
         : phase == OC_UP_P        ? (1u << OC_INTT_COL)
         : phase == OC_ROW_P       ? (1u << OC_UP_P)
         : phase == OC_UP_Q        ? (1u << OC_INTT_COL)
         : phase == OC_INTT_COL_DN ? (1u << OC_ROW_P)
         : phase == OC_DN          ? (1u << OC_INTT_COL_DN)
         : phase == OC_ROW_Q       ? ((1u << OC_DN) | (1u << OC_UP_Q))
                                   : 0u;
}

// Tile counts of every phase for a job at `level`.
__host__ __device__ inline void oc_phase_tiles(uint32_t loga, uint32_t cb, uint32_t alpha, uint32_t K,
                                               uint32_t level, uint32_t ttu, uint32_t ttd, uint32_t *n) {
  const uint32_t L1 = level + 1, rbk = (1u << loga) / kRB, rbq = (1u << loga) / kRBQ, ndig = cdiv(L1, alpha);
  uint32_t upq = 0;
  for (uint32_t j = 0; j < ndig; j++) {
    const uint32_t lo = j * alpha, s = (lo + alpha < L1 ? lo + alpha : L1) - lo;
    upq += cdiv(L1 - s, ttu);
  }
  n[OC_INTT_ROW] = rbk * L1;
  n[OC_INTT_COL] = cb * L1;
  n[OC_UP_P] = cb * ndig * cdiv(K, ttu);
  n[OC_ROW_P] = rbq * K;
  n[OC_UP_Q] = cb * upq;
  n[OC_INTT_COL_DN] = cb * 2 * K;
  n[OC_DN] = cb * 2 * cdiv(L1, ttd);
  n[OC_ROW_Q] = rbq * L1;
}

// Effective targets per basis-conversion tile (1 or 2) for a column pass of
// length 2^loga.
uint32_t oc_effective_tt(uint32_t loga, uint32_t want, uint32_t l1);
// Tile counts of every phase (host).
void oc_tiles_host(const Plan &pl, uint32_t level, uint32_t tt, uint32_t *tiles);
// The same from the parameters alone (no plan, no device).
void oc_tiles_params(uint32_t log_n, uint32_t alpha, uint32_t K, uint32_t level, uint32_t tt, uint32_t *tiles);
// The work list of the persistent batch launch: one segment per (phase,
// job), phase-major then job-major, each starting where the previous ends.
// tiles: count x OC_NPHASE tile counts.  Returns the total item count.
uint32_t oc_segments(const uint32_t *tiles, uint32_t count, std::vector<OcSeg> &segs);
// One launch per phase; jobs == nullptr runs `one` alone.  rows: the
// row-stage kernels (plain, compressed keys, or extended); part: which
// phases run.
hipError_t launch_oc_phases(const Plan &pl, const OcJob &one, const OcJob *jobs, uint32_t count,
                            const uint32_t *max_tiles, uint32_t tt, OcRowVariant rows, OcPart part,
                            hipStream_t st);
// Persistent work-queue launch (tiles of one target per conversion tile).
hipError_t launch_oc_persistent(const Plan &pl, const OcJob *jobs, const OcSeg *segs, uint32_t nsegs,
                                uint32_t total, uint32_t count, uint32_t *ctl, uint32_t spin_limit, hipStream_t st);

// The fixed device scratch of ks_keyswitch_noalloc (noalloc.hip): looked up
// once per device with that device current (plan creation), then read.
hipError_t noalloc_scratch_init(int dev);
void *noalloc_scratch(int dev);  // nullptr until set up on `dev`

template <int A>
hipError_t oc_phases(const Plan &pl, const OcJob &one, const OcJob *jobs, uint32_t count, const uint32_t *max_tiles,
                     uint32_t tt, OcRowVariant rows, OcPart part, hipStream_t st);
template <int A>
hipError_t oc_persistent(const Plan &pl, const OcJob *jobs, const OcSeg *segs, uint32_t nsegs, uint32_t total,
                         uint32_t count, uint32_t *ctl, uint32_t spin_limit, hipStream_t st);

}  // namespace ks
