// oc_kernels.h -- Output-Centric key switching (Sec. IV-C) for gfx950.
//
// The paper's OC computes one output tower at a time: the basis-conversion
// expansion (ModUp P2) and the key products (P4) of a tower are produced and
// consumed on chip, P5 accumulates on chip, the INTT outputs are kept and
// reused by every tower, and ModDown converts one tower at a time from the
// K special towers.  With the two-pass NTT (column pass, row pass) a tower's
// transform is spread over many workgroups, so the unit of work here is an
// output tower (or a tile of towers) times a column block or a row block:
//
//   1. inverse row pass of the input towers            (ModUp P1, part 1)
//   2. inverse column pass + per-source constant        (ModUp P1, part 2)
//   3. per (digit, target tile, column block): basis conversion from the
//      digit's towers fused with the forward column pass (ModUp P2, P3)
//   4. per (P tower, row block): forward row pass of every digit, key
//      multiply-accumulate over digits in registers, then the inverse row
//      pass of both accumulators (ModUp P3-P5, ModDown P1 part 1)
//   5. inverse column pass of the 2K special towers + constant (ModDown P1)
//   6. per (poly, Q-target tile, column block): conversion P -> q_i fused
//      with the forward column pass (ModDown P2, P3)
//   7. per (Q tower, row block): forward row pass of the foreign digits,
//      bypass of the own digit, key multiply-accumulate, forward row pass of
//      the ModDown term and (acc - w) * P^-1 (ModUp P3-P5, ModDown P3-P4).
// The special towers go first (the paper's Section 2) so that every Q tower
// finishes ModUp and ModDown in one kernel and its accumulator never leaves
// registers.
#pragma once
#include "kernels.h"
#include "ntt_engine.h"

namespace ks {

__device__ __forceinline__ uint32_t oc_gidx(const DevPlan &P, uint32_t level, uint32_t t) {
  return t <= level ? t : P.num_q + (t - level - 1);
}

// ------------------------------------------------------------ step 2 / 5
// Inverse column pass of one limb, then x~ = [v * c]_m canonical with the
// per-source constant c (ModUp: N^-1 qhat^-1, ModDown: N^-1 2^32 phat^-1).
// mode 0: limb i of xt (ModUp sources); mode 1: limb s*K+k of zp.
template <int A, int W>
__global__ __launch_bounds__(W *SubNtt<A>::TPS) void k_oc_intt_col(DevPlan P, uint32_t *data, uint32_t level,
                                                                  int mode) {
  using S = SubNtt<A>;
  constexpr int R1 = S::R1, R2 = S::R2, TPS = S::TPS;
  __shared__ uint32_t lds[W << A];
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t rowlen = 1u << P.logb, c0 = blockIdx.x * W, li = blockIdx.y;
  uint32_t g;
  uint2 pre;
  if (mode == 0) {
    g = li;
    const uint32_t j = li / P.alpha, lo = j * P.alpha, s = min(lo + P.alpha, level + 1) - lo;
    pre = P.up_pre[((size_t)j * P.alpha + (s - 1)) * P.alpha + (li - lo)];
  } else {
    const uint32_t k = li % P.num_p;
    g = P.num_q + k;
    pre = P.dn_pre[k];
  }
  const uint32_t q = P.mods[g].q;
  const uint2 *tw = P.tw_inv + g * N;
  uint32_t *col = data + (size_t)li * N + c0;
  const int w = threadIdx.x % W, tig = threadIdx.x / W;
  if constexpr (R2 > 0) {
    using Ph = Phase<A, 1 + R1, R2>;
#pragma unroll
    for (int gi = 0; gi < Ph::GROUPS / TPS; gi++) {
      const int gg = tig + gi * TPS;
      uint32_t x[1 << R2];
#pragma unroll
      for (int u = 0; u < (1 << R2); u++) x[u] = col[(size_t)Ph::elem(gg, u) * rowlen + w];
      gs_group<A, 1 + R1, R2>(x, gg, 1u, tw, q);
#pragma unroll
      for (int u = 0; u < (1 << R2); u++) lds[Ph::elem(gg, u) * W + w] = x[u];
    }
    __syncthreads();
  }
  {
    using Ph = Phase<A, 1, R1>;
    uint32_t x[1 << R1];
#pragma unroll
    for (int u = 0; u < (1 << R1); u++)
      x[u] = R2 > 0 ? lds[Ph::elem(tig, u) * W + w] : col[(size_t)Ph::elem(tig, u) * rowlen + w];
    gs_group<A, 1, R1>(x, tig, 1u, tw, q);
#pragma unroll
    for (int u = 0; u < (1 << R1); u++)
      col[(size_t)Ph::elem(tig, u) * rowlen + w] = csub(mul_shoup(x[u], pre.x, pre.y, q), q);
  }
}

// ------------------------------------------------------------ step 3 / 6
// Basis conversion of one column block to TT target towers fused with the
// forward column pass.  Tile decode (blockIdx.y):
//   mode 0 (ModUp): digits in order, each split into ceil(beta_j / TT) tiles
//     over its targets D_l \ S_j (compressed index); sources xt[lo..hi),
//     constants up_conv (Montgomery form), output ycol[j][t];
//   mode 1 (ModDown): poly s = tile / ceil((l+1)/TT), targets q_i; sources
//     zp[s][0..K), constants dn_conv, output wcol[s][i].
template <int A, int W, int TT, int MAXS>
__global__ __launch_bounds__(W *SubNtt<A>::TPS) void k_oc_bconv_col(DevPlan P, OcArgs a, int mode) {
  using S = SubNtt<A>;
  constexpr int R1 = S::R1, R2 = S::R2, TPS = S::TPS, E = 1 << R1;
  __shared__ uint32_t lds[TT][W << A];
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t level = a.level, L1 = level + 1, T = L1 + P.num_p;
  const uint32_t rowlen = 1u << P.logb, c0 = blockIdx.x * W;
  const int w = threadIdx.x % W, tig = threadIdx.x / W;

  // ---- decode the tile
  uint32_t nsrc, cstride, ntgt = 0;
  const uint32_t *src;
  const uint32_t *cbase;
  uint32_t tg[TT], tcol[TT];
  uint32_t *tout[TT];
  if (mode == 0) {
    const uint32_t ndig = (level + P.alpha) / P.alpha;
    uint32_t tile = blockIdx.y, j = 0, lo = 0, hi = 0, nt = 0;
    for (; j < ndig; j++) {
      lo = j * P.alpha;
      hi = min(lo + P.alpha, L1);
      nt = (T - (hi - lo) + TT - 1) / TT;
      if (tile < nt) break;
      tile -= nt;
    }
    if (j == ndig) return;  // grid larger than the tile count: nothing to do
    const uint32_t s = hi - lo, beta = T - s;
    nsrc = s;
    src = a.xt + (size_t)lo * N;
    cstride = P.ntot;
    cbase = P.up_conv + (((size_t)j * P.alpha + (s - 1)) * P.alpha) * P.ntot;
#pragma unroll
    for (int e = 0; e < TT; e++) {
      const uint32_t ci = tile * TT + e;
      if (ci < beta) {
        const uint32_t t = ci < lo ? ci : ci + s;
        tg[e] = oc_gidx(P, level, t);
        tcol[e] = tg[e];
        tout[e] = a.ycol + ((size_t)j * T + t) * N;
        ntgt = e + 1;
      } else {
        tg[e] = tcol[e] = 0;
        tout[e] = nullptr;
      }
    }
  } else {
    const uint32_t per = (L1 + TT - 1) / TT, s = blockIdx.y / per, tile = blockIdx.y % per;
    nsrc = P.num_p;
    src = a.zp + (size_t)s * P.num_p * N;
    cstride = P.num_q;
    cbase = P.dn_conv;
#pragma unroll
    for (int e = 0; e < TT; e++) {
      const uint32_t i = tile * TT + e;
      if (i < L1) {
        tg[e] = i;
        tcol[e] = i;
        tout[e] = a.wcol + ((size_t)s * L1 + i) * N;
        ntgt = e + 1;
      } else {
        tg[e] = tcol[e] = 0;
        tout[e] = nullptr;
      }
    }
  }

  // ---- basis conversion of this thread's phase-1 group
  using Ph1 = Phase<A, 1, R1>;
  uint32_t y[TT][E];
  ModQ mq[TT];
#pragma unroll
  for (int e = 0; e < TT; e++) mq[e] = P.mods[tg[e]];
#pragma unroll
  for (int u = 0; u < E; u++) {
    const size_t off = (size_t)Ph1::elem(tig, u) * rowlen + c0 + w;
    uint32_t xs[MAXS];
#pragma unroll
    for (int i = 0; i < MAXS; i++)
      if ((uint32_t)i < nsrc) xs[i] = src[(size_t)i * N + off];
#pragma unroll
    for (int e = 0; e < TT; e++) {
      uint64_t acc = 0;
      uint32_t r = 0;
#pragma unroll
      for (int i = 0; i < MAXS; i++) {
        if ((uint32_t)i < nsrc) {
          acc = mad64(xs[i], cbase[(size_t)i * cstride + tcol[e]], acc);
          if ((i & 15) == 15) { r = csub(r + redc64(acc, mq[e]), mq[e].q); acc = 0; }
        }
      }
      y[e][u] = csub(r + redc64(acc, mq[e]), mq[e].q);
    }
  }

  // ---- forward column pass per target
#pragma unroll
  for (int e = 0; e < TT; e++) {
    if ((uint32_t)e < ntgt) {
      const uint2 *tw = P.tw_fwd + tg[e] * N;
      ct_group<A, 1, R1>(y[e], tig, 1u, tw, mq[e].q);
      if constexpr (R2 > 0) {
#pragma unroll
        for (int u = 0; u < E; u++) lds[e][Ph1::elem(tig, u) * W + w] = y[e][u];
      } else {
#pragma unroll
        for (int u = 0; u < E; u++) tout[e][(size_t)Ph1::elem(tig, u) * rowlen + c0 + w] = y[e][u];
      }
    }
  }
  if constexpr (R2 > 0) {
    __syncthreads();
    using Ph2 = Phase<A, 1 + R1, R2>;
#pragma unroll
    for (int e = 0; e < TT; e++) {
      if ((uint32_t)e < ntgt) {
        const uint2 *tw = P.tw_fwd + tg[e] * N;
#pragma unroll
        for (int gi = 0; gi < Ph2::GROUPS / TPS; gi++) {
          const int gg = tig + gi * TPS;
          uint32_t x[1 << R2];
#pragma unroll
          for (int u = 0; u < (1 << R2); u++) x[u] = lds[e][Ph2::elem(gg, u) * W + w];
          ct_group<A, 1 + R1, R2>(x, gg, 1u, tw, mq[e].q);
#pragma unroll
          for (int u = 0; u < (1 << R2); u++) tout[e][(size_t)Ph2::elem(gg, u) * rowlen + c0 + w] = x[u];
        }
      }
    }
  }
}

// ------------------------------------------------------------ step 4 / 7
// Row pass helpers.  A row of 256 words is handled by 16 threads; phase 1
// (stages 1-4 of the row) holds k = tig + 16u, phase 2 (stages 5-8) holds
// k = 16 tig + u.
constexpr int kPad = 272;
__device__ __forceinline__ int rl(int k) { return k + (k >> 4); }

// Forward row transform of a row read from global (phase-1 layout); leaves
// the result in x in phase-2 layout.  Uses lds row `lr` (kPad words).
__device__ __forceinline__ void row_fwd_from_global(uint32_t (&x)[16], const uint32_t *row, uint32_t *lr, int tig,
                                                    uint32_t M, const uint2 *tw, uint32_t q) {
#pragma unroll
  for (int u = 0; u < 16; u++) x[u] = row[tig + 16 * u];
  ct_group<8, 1, 4>(x, tig, M, tw, q);
#pragma unroll
  for (int u = 0; u < 16; u++) lr[rl(tig + 16 * u)] = x[u];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 16; u++) x[u] = lr[rl(16 * tig + u)];
  ct_group<8, 5, 4>(x, tig, M, tw, q);
  __syncthreads();
}

// Inverse row transform of x (phase-2 layout) written to global (phase-1
// layout, lazy [0, 2q)).
__device__ __forceinline__ void row_inv_to_global(uint32_t (&x)[16], uint32_t *row, uint32_t *lr, int tig, uint32_t M,
                                                  const uint2 *tw, uint32_t q) {
  gs_group<8, 5, 4>(x, tig, M, tw, q);
#pragma unroll
  for (int u = 0; u < 16; u++) lr[rl(16 * tig + u)] = x[u];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 16; u++) x[u] = lr[rl(tig + 16 * u)];
  gs_group<8, 1, 4>(x, tig, M, tw, q);
#pragma unroll
  for (int u = 0; u < 16; u++) row[tig + 16 * u] = x[u];
  __syncthreads();
}

__device__ __forceinline__ void load16(uint32_t (&x)[16], const uint32_t *p) {
  const uint4 *v = reinterpret_cast<const uint4 *>(p);
#pragma unroll
  for (int i = 0; i < 4; i++) {
    uint4 t = v[i];
    x[4 * i] = t.x; x[4 * i + 1] = t.y; x[4 * i + 2] = t.z; x[4 * i + 3] = t.w;
  }
}
__device__ __forceinline__ void store16(uint32_t *p, const uint32_t (&x)[16]) {
  uint4 *v = reinterpret_cast<uint4 *>(p);
#pragma unroll
  for (int i = 0; i < 4; i++) v[i] = make_uint4(x[4 * i], x[4 * i + 1], x[4 * i + 2], x[4 * i + 3]);
}

// IS_P: blockIdx.y = k, tower t = l+1+k; otherwise blockIdx.y = i, tower i.
template <int RB, bool IS_P>
__global__ __launch_bounds__(RB * 16) void k_oc_row(DevPlan P, OcArgs a) {
  __shared__ uint32_t lds[RB * kPad];
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t level = a.level, L1 = level + 1, T = L1 + P.num_p;
  const uint32_t t = IS_P ? L1 + blockIdx.y : blockIdx.y;
  const uint32_t g = oc_gidx(P, level, t);
  const ModQ m = P.mods[g];
  const uint32_t q = m.q;
  const uint2 *twf = P.tw_fwd + g * N, *twi = P.tw_inv + g * N;
  const int rr = threadIdx.x >> 4, tig = threadIdx.x & 15;
  const uint32_t row = blockIdx.x * RB + rr;
  const uint32_t M = (1u << P.loga) + row;
  const size_t roff = (size_t)row * 256;
  uint32_t *lr = lds + rr * kPad;
  const uint32_t ndig = (level + P.alpha) / P.alpha;

  uint64_t acc0[16], acc1[16];
  uint32_t part0[16], part1[16];
#pragma unroll
  for (int u = 0; u < 16; u++) { acc0[u] = acc1[u] = 0; part0[u] = part1[u] = 0; }
  for (uint32_t j = 0; j < ndig; j++) {
    const uint32_t lo = j * P.alpha, hi = min(lo + P.alpha, L1);
    uint32_t x[16];
    if (!IS_P && t >= lo && t < hi) {
      load16(x, a.d + (size_t)t * N + roff + 16 * tig);  // own digit: bypass
    } else {
      row_fwd_from_global(x, a.ycol + ((size_t)j * T + t) * N + roff, lr, tig, M, twf, q);
#pragma unroll
      for (int u = 0; u < 16; u++) x[u] = canon4(x[u], q);
    }
    uint32_t e0[16], e1[16];
    load16(e0, a.evk + (((size_t)j * 2 + 0) * P.ntot + g) * N + roff + 16 * tig);
    load16(e1, a.evk + (((size_t)j * 2 + 1) * P.ntot + g) * N + roff + 16 * tig);
#pragma unroll
    for (int u = 0; u < 16; u++) {
      acc0[u] = mad64(x[u], e0[u], acc0[u]);
      acc1[u] = mad64(x[u], e1[u], acc1[u]);
    }
    if ((j & 15) == 15) {
#pragma unroll
      for (int u = 0; u < 16; u++) {
        part0[u] = csub(part0[u] + redc64(acc0[u], m), q);
        part1[u] = csub(part1[u] + redc64(acc1[u], m), q);
        acc0[u] = acc1[u] = 0;
      }
    }
  }
  uint32_t r0[16], r1[16];
#pragma unroll
  for (int u = 0; u < 16; u++) {
    r0[u] = csub(part0[u] + redc64(acc0[u], m), q);
    r1[u] = csub(part1[u] + redc64(acc1[u], m), q);
  }
  if (IS_P) {
    const uint32_t k = blockIdx.y;
    row_inv_to_global(r0, a.zp + ((size_t)0 * P.num_p + k) * N + roff, lr, tig, M, twi, q);
    row_inv_to_global(r1, a.zp + ((size_t)1 * P.num_p + k) * N + roff, lr, tig, M, twi, q);
  } else {
    const uint2 f = P.dn_fin[t];
#pragma unroll
    for (int s = 0; s < 2; s++) {
      uint32_t wv[16];
      row_fwd_from_global(wv, a.wcol + ((size_t)s * L1 + t) * N + roff, lr, tig, M, twf, q);
      uint32_t o[16];
#pragma unroll
      for (int u = 0; u < 16; u++) {
        const uint32_t av = s ? r1[u] : r0[u];
        o[u] = csub(mul_shoup(av + q - canon4(wv[u], q), f.x, f.y, q), q);
      }
      store16(a.out + ((size_t)s * L1 + t) * N + roff + 16 * tig, o);
    }
  }
}

// ------------------------------------------------------------ launcher
// Unrolled basis-conversion variants are limited to TT * 2^R1 * MAXS <= 1024
// products per thread; larger requests fall back to fewer targets per tile.
template <int A, int TT, int MS>
constexpr bool bc_ok() { return TT * (1 << SubNtt<A>::R1) * MS <= 1024; }

template <int A, int TT, int MS>
static void launch_bc(const Plan &pl, const OcArgs &a, int mode, uint32_t tiles, hipStream_t st) {
  constexpr int NT = 16 * SubNtt<A>::TPS;
  const uint32_t cols = 1u << pl.dev.logb;
  KS_LAUNCH(pl, mode == 0 ? "oc.bconv_col.up" : "oc.bconv_col.down", (k_oc_bconv_col<A, 16, TT, MS>), dim3(cols / 16, tiles), dim3(NT), 0, st, pl.dev, a, mode);
}

// Largest allowed tile <= want for `nsrc` sources.
template <int A>
static uint32_t bc_tile(uint32_t want, uint32_t nsrc) {
  const uint32_t ms = nsrc <= 8 ? 8 : nsrc <= 16 ? 16 : 32;
  uint32_t tt = want >= 4 ? 4 : want >= 2 ? 2 : 1;
  while (tt > 1 && tt * (1u << SubNtt<A>::R1) * ms > 1024) tt >>= 1;
  return tt;
}

template <int A>
static bool dispatch_bc(const Plan &pl, const OcArgs &a, int mode, uint32_t tt, uint32_t nsrc, uint32_t tiles,
                        hipStream_t st) {
#define KS_TRY(TTv, MSv)                                                            \
  if constexpr (bc_ok<A, TTv, MSv>()) {                                             \
    if (tt == TTv && (MSv == 8 ? nsrc <= 8 : MSv == 16 ? (nsrc > 8 && nsrc <= 16) : nsrc > 16)) { \
      launch_bc<A, TTv, MSv>(pl, a, mode, tiles, st);                               \
      return true;                                                                  \
    }                                                                               \
  }
  KS_TRY(1, 8) KS_TRY(1, 16) KS_TRY(1, 32)
  KS_TRY(2, 8) KS_TRY(2, 16) KS_TRY(2, 32)
  KS_TRY(4, 8) KS_TRY(4, 16) KS_TRY(4, 32)
#undef KS_TRY
  return false;
}

template <int A>
hipError_t oc_cols(const Plan &pl, const OcArgs &a, hipStream_t st) {
  const uint32_t L1 = a.level + 1, T = L1 + pl.num_p, K = pl.num_p;
  const uint32_t cols = 1u << pl.dev.logb;
  constexpr int NT = 16 * SubNtt<A>::TPS;
  const uint32_t want = pl.cfg.tile_towers ? pl.cfg.tile_towers : 1;
  // step 2: inverse column pass of the inputs
  KS_LAUNCH(pl, "oc.intt_col.up", (k_oc_intt_col<A, 16>), dim3(cols / 16, L1), dim3(NT), 0, st, pl.dev, a.xt, a.level, 0);
  // step 3: ModUp conversion + forward column pass
  const uint32_t tt_up = bc_tile<A>(want, pl.alpha);
  uint32_t tiles = 0;
  const uint32_t D = num_digits(pl, a.level);
  for (uint32_t j = 0; j < D; j++) {
    uint32_t lo, hi;
    digit_range(pl, a.level, j, &lo, &hi);
    tiles += (T - (hi - lo) + tt_up - 1) / tt_up;
  }
  if (!dispatch_bc<A>(pl, a, 0, tt_up, pl.alpha, tiles, st)) return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // step 4: special towers, row pass
  const uint32_t rows = 1u << pl.dev.loga;
  const uint32_t RB = rows >= 8 ? 8 : rows;
  if (RB == 8) KS_LAUNCH(pl, "oc.row.p", (k_oc_row<8, true>), dim3(rows / 8, K), dim3(128), 0, st, pl.dev, a);
  else KS_LAUNCH(pl, "oc.row.p", (k_oc_row<4, true>), dim3(rows / 4, K), dim3(64), 0, st, pl.dev, a);
  // step 5: inverse column pass of the special towers
  KS_LAUNCH(pl, "oc.intt_col.down", (k_oc_intt_col<A, 16>), dim3(cols / 16, 2 * K), dim3(NT), 0, st, pl.dev, a.zp, a.level, 1);
  // step 6: ModDown conversion + forward column pass
  const uint32_t tt_dn = bc_tile<A>(want, K);
  if (!dispatch_bc<A>(pl, a, 1, tt_dn, K, 2 * ((L1 + tt_dn - 1) / tt_dn), st)) return hipErrorInvalidValue;
  // step 7: Q towers, row pass with ModDown
  if (RB == 8) KS_LAUNCH(pl, "oc.row.q", (k_oc_row<8, false>), dim3(rows / 8, L1), dim3(128), 0, st, pl.dev, a);
  else KS_LAUNCH(pl, "oc.row.q", (k_oc_row<4, false>), dim3(rows / 4, L1), dim3(64), 0, st, pl.dev, a);
  return hipGetLastError();
}

}  // namespace ks
