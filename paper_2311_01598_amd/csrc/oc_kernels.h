// oc_kernels.h -- Output-Centric key switching (Sec. IV-C) for gfx950.
//
// The paper's OC computes one output tower at a time: the basis-conversion
// expansion (ModUp P2) and the key products (P4) of a tower are produced and
// consumed on chip, P5 accumulates on chip, the INTT outputs are kept and
// reused by every tower, and ModDown converts one tower at a time from the
// K special towers.  A 2^16-point transform does not fit one CU, so a
// tower's transform is split into a column pass and a row pass (see
// ntt_engine.h) and the unit of work is a tile: an output tower (or a few)
// times a column block, or a tower times a block of rows.  Phases, in
// dependency order:
//
//   INTT_ROW    inverse row pass of the input towers              ModUp P1
//   INTT_COL    inverse column pass + per-source constant         ModUp P1
//   UP_P        per (digit, special target, column block): basis
//               conversion fused with the forward column pass     ModUp P2, P3
//   UP_Q        as UP_P for the Q targets outside each digit      ModUp P2, P3
//   ROW_P       per (special tower, row block): forward row pass of
//               every digit, key multiply-accumulate in registers,
//               inverse row pass of both accumulators             P3-P5, ModDown P1
//   INTT_COL_DN inverse column pass of the 2K special towers       ModDown P1
//   DN          per (poly, Q target, column block): conversion
//               P -> q_i fused with the forward column pass       ModDown P2, P3
//   ROW_Q       per (Q tower, row block): forward row pass of the
//               foreign digits, bypass of the own digit, key
//               multiply-accumulate, forward row pass of the
//               ModDown term, (acc - w) * P^-1                    P3-P5, ModDown P3-P4
//
// UP_P and UP_Q depend only on INTT_COL and are issued as one launch
// (OC_UP_PQ, special targets first).  The special towers go first (the
// paper's Section 2) so that every Q tower finishes ModUp and ModDown in one
// tile and its accumulator never leaves registers.  Every tile is one
// 256-thread workgroup; the same tile bodies serve one launch per phase
// (single key switch or a batch, job index in grid z) and the persistent
// work-queue kernel of oc_persist.h (switched off).
#pragma once
#include "kernels.h"
#include "ntt_engine.h"

namespace ks {

constexpr int kOcThreads = 256;
constexpr int kPad = 272;   // LDS words per row: 256 + one pad word per 16
constexpr int kRowLds = kRB * kPad;
__device__ __forceinline__ int rl(int k) { return k + (k >> 4); }

template <int A>
struct ColGeom {
  static constexpr int TPS = SubNtt<A>::TPS, R1 = SubNtt<A>::R1, R2 = SubNtt<A>::R2, E = 1 << R1;
  static constexpr int W = kOcThreads / TPS;  // columns per tile (TPS threads per column)
  static constexpr int CB = TPS;              // column blocks: 256 / W
  static constexpr int LDS = W << A;          // words per target tile
};

// ------------------------------------------------------------ twiddles
// Twiddles of one group in registers: entry (2^t - 1) + k is stage t's k-th.
template <int R>
struct GroupTw {
  uint2 w[(1 << R) - 1];
};
template <int A, int S0, int R>
__device__ __forceinline__ void load_group_tw(GroupTw<R> &gt, const uint2 *__restrict__ tw, int g, uint32_t M) {
  const uint32_t hi = (uint32_t)Phase<A, S0, R>::hi(g);
#pragma unroll
  for (int t = 0; t < R; t++) {
    const uint32_t node = (M << (S0 + t - 1)) + (hi << t);
#pragma unroll
    for (int k = 0; k < (1 << t); k++) gt.w[(1 << t) - 1 + k] = ldg2(tw + node + k);
  }
}
template <int R>
__device__ __forceinline__ void ct_regs(uint32_t (&x)[1 << R], const GroupTw<R> &gt, uint32_t q) {
#pragma unroll
  for (int t = 0; t < R; t++) {
    const int half = 1 << (R - 1 - t);
#pragma unroll
    for (int u = 0; u < (1 << R); u++) {
      if (u & half) continue;
      const uint2 w = gt.w[(1 << t) - 1 + (u >> (R - t))];
      bfly_ct(x[u], x[u + half], w.x, w.y, q);
    }
  }
}
template <int R>
__device__ __forceinline__ void gs_regs(uint32_t (&x)[1 << R], const GroupTw<R> &gt, uint32_t q) {
#pragma unroll
  for (int t = R - 1; t >= 0; t--) {
    const int half = 1 << (R - 1 - t);
#pragma unroll
    for (int u = 0; u < (1 << R); u++) {
      if (u & half) continue;
      const uint2 w = gt.w[(1 << t) - 1 + (u >> (R - t))];
      bfly_gs(x[u], x[u + half], w.x, w.y, q);
    }
  }
}

// A row (256 words) is transformed by 16 threads: phase 1 (row stages 1-4)
// holds k = tig + 16u, phase 2 (stages 5-8) holds k = 16 tig + u.
struct RowTw {
  GroupTw<4> p1, p2;
};
__device__ __forceinline__ void load_row_tw(RowTw &r, const uint2 *__restrict__ tw, int tig, uint32_t M) {
  load_group_tw<8, 1, 4>(r.p1, tw, tig, M);
  load_group_tw<8, 5, 4>(r.p2, tw, tig, M);
}

__device__ __forceinline__ void load16(uint32_t (&x)[16], const uint32_t *p) {
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const uint4 t = ldg4(p + 4 * i);
    x[4 * i] = t.x; x[4 * i + 1] = t.y; x[4 * i + 2] = t.z; x[4 * i + 3] = t.w;
  }
}
__device__ __forceinline__ void store16(uint32_t *p, const uint32_t (&x)[16]) {
#pragma unroll
  for (int i = 0; i < 4; i++) stg4(p + 4 * i, make_uint4(x[4 * i], x[4 * i + 1], x[4 * i + 2], x[4 * i + 3]));
}

// Forward transform of a row read from global in phase-1 layout; result in
// x (phase-2 layout, lazy [0, 4q)).  lr: this row's LDS slice.
__device__ __forceinline__ void row_fwd(uint32_t (&x)[16], const uint32_t *row, uint32_t *lr, int tig,
                                        const RowTw &tw, uint32_t q) {
#pragma unroll
  for (int u = 0; u < 16; u++) x[u] = gp(row)[tig + 16 * u];
  ct_regs<4>(x, tw.p1, q);
#pragma unroll
  for (int u = 0; u < 16; u++) lr[rl(tig + 16 * u)] = x[u];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 16; u++) x[u] = lr[rl(16 * tig + u)];
  ct_regs<4>(x, tw.p2, q);
  __syncthreads();
}

// Inverse transform of x (phase-2 layout, values < 2q) written to global in
// phase-1 layout (lazy [0, 2q)).
__device__ __forceinline__ void row_inv(uint32_t (&x)[16], uint32_t *row, uint32_t *lr, int tig, const RowTw &tw,
                                        uint32_t q) {
  gs_regs<4>(x, tw.p2, q);
#pragma unroll
  for (int u = 0; u < 16; u++) lr[rl(16 * tig + u)] = x[u];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 16; u++) x[u] = lr[rl(tig + 16 * u)];
  gs_regs<4>(x, tw.p1, q);
#pragma unroll
  for (int u = 0; u < 16; u++) gp(row)[tig + 16 * u] = x[u];
  __syncthreads();
}

// ------------------------------------------------------------ tile bodies
// INTT_ROW: inverse row pass of input tower `i`, row block `blk`, d -> xt.
__device__ __forceinline__ void tile_intt_row(const DevPlan &P, const OcJob &J, uint32_t tile, uint32_t *lds) {
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t rbk = (1u << P.loga) / kRB, i = tile / rbk, blk = tile % rbk;
  const int rr = threadIdx.x >> 4, tig = threadIdx.x & 15;
  const uint32_t row = blk * kRB + rr, M = (1u << P.loga) + row;
  const size_t roff = (size_t)i * N + (size_t)row * 256;
  RowTw tw;
  load_row_tw(tw, P.tw_inv + (size_t)i * N, tig, M);
  uint32_t x[16];
  load16(x, J.d + roff + 16 * tig);
  row_inv(x, J.xt + roff, lds + rr * kPad, tig, tw, ldmodc(P.mods + i).q);
}

// Column passes (node 1) use only the first 2^A entries of a modulus'
// twiddle table: a tile stages them in LDS once (one coalesced load per
// thread per 256 entries) instead of every thread loading its 2 x 15 pairs
// from global memory on the critical path.
template <int A>
struct ColTw {
  static constexpr int PER = (1 << A) > kOcThreads ? (1 << A) / kOcThreads : 1;  // entries per thread
  uint32_t v[PER];
  // tw32: the modulus' 4-byte table (psi^brv or psi^-brv)
  __device__ __forceinline__ void issue(const uint32_t *tw32) {
#pragma unroll
    for (int k = 0; k < PER; k++) {
      const uint32_t i = threadIdx.x + k * kOcThreads;
      v[k] = gp(tw32)[i < (1u << A) ? i : 0u];
    }
  }
  // forward tables hold -w mod 2^32 next to the companion of w (see bfly_ct)
  __device__ __forceinline__ void store(uint2 *twl, uint32_t q, double qr, bool fwd) const {
#pragma unroll
    for (int k = 0; k < PER; k++) {
      const uint32_t i = threadIdx.x + k * kOcThreads;
      if (i < (1u << A)) twl[i] = make_uint2(fwd ? 0u - v[k] : v[k], shoup_companion(v[k], q, qr));
    }
  }
};

// INTT_COL / INTT_COL_DN: inverse column pass of one limb, then
// x~ = [v * c]_m canonical with the per-source constant c.
template <int A>
__device__ __forceinline__ void tile_intt_col(const DevPlan &P, const OcJob &J, uint32_t tile, bool down,
                                              uint32_t *lds) {
  using G = ColGeom<A>;
  constexpr int R1 = G::R1, R2 = G::R2, TPS = G::TPS, W = G::W;
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t li = tile / G::CB, c0 = (tile % G::CB) * W, rowlen = 256;
  uint32_t g;
  uint2 pre;
  uint32_t *col;
  if (!down) {
    const uint32_t j = li / P.alpha, lo = j * P.alpha, s = min(lo + P.alpha, J.level + 1) - lo;
    g = li;
    pre = ldc2(P.up_pre + ((size_t)j * P.alpha + (s - 1)) * P.alpha + (li - lo));
    col = J.xt + (size_t)li * N + c0;
  } else {
    const uint32_t k = li % P.num_p;
    g = P.num_q + k;
    pre = ldc2(P.dn_pre + k);
    col = J.zp + (size_t)li * N + c0;
  }
  const uint32_t q = ldmodc(P.mods + g).q;
  const int w = threadIdx.x % W, tig = threadIdx.x / W;
  // twiddles first (staged in LDS after the data region), then the data
  ColTw<A> ct;
  ct.issue(P.tw_inv32 + (size_t)g * N);
  const double qr = ldcd(P.qrecip + g);
  uint2 *twl = reinterpret_cast<uint2 *>(lds + G::LDS);
  const LdsTw tw{twl};
  // the limb (col - c0) as a buffer: byte offset (row * 256 + c0 + w) * 4
  const __amdgpu_buffer_rsrc_t rc = buf_rsrc(col - c0, (uint32_t)(N * 4));
  using Ph = Phase<A, 1, R1>;
  const uint32_t vb = ((uint32_t)Ph::base(tig) * rowlen + c0 + w) * 4u;
  uint32_t x[1 << R1];
  if constexpr (R2 > 0) {
    using Ph2 = Phase<A, 1 + R1, R2>;
    constexpr int GPT = Ph2::GROUPS / TPS;
    uint32_t x2[GPT][1 << R2];
#pragma unroll
    for (int gi = 0; gi < GPT; gi++) {
      const int gg = tig + gi * TPS;
      const uint32_t vb2 = ((uint32_t)Ph2::base(gg) * rowlen + c0 + w) * 4u;
#pragma unroll
      for (int u = 0; u < (1 << R2); u++) x2[gi][u] = buf_ld(rc, vb2, ((uint32_t)u << Ph2::LOB) * rowlen * 4u);
    }
    ct.store(twl, q, qr, false);
    __syncthreads();
#pragma unroll
    for (int gi = 0; gi < GPT; gi++) {
      const int gg = tig + gi * TPS;
      gs_group<A, 1 + R1, R2>(x2[gi], gg, 1u, tw, q);
#pragma unroll
      for (int u = 0; u < (1 << R2); u++) lds[Ph2::elem(gg, u) * W + w] = x2[gi][u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < (1 << R1); u++) x[u] = lds[Ph::elem(tig, u) * W + w];
  } else {
#pragma unroll
    for (int u = 0; u < (1 << R1); u++) x[u] = buf_ld(rc, vb, ((uint32_t)u << Ph::LOB) * rowlen * 4u);
    ct.store(twl, q, qr, false);
    __syncthreads();
  }
  gs_group<A, 1, R1>(x, tig, 1u, tw, q);
#pragma unroll
  for (int u = 0; u < (1 << R1); u++)
    buf_st(rc, vb, ((uint32_t)u << Ph::LOB) * rowlen * 4u, csub(mul_shoup(x[u], pre.x, pre.y, q), q));
  __syncthreads();
}

// UP_P / UP_Q / DN: basis conversion of one column block to up to TT target
// towers, fused with the forward column pass.  Sources are canonical
// (prescaled) limbs src + i*N, i < nsrc; constant of source i for target e
// is cbase[i * cstride + tcol[e]] (REDC form).
// Targets of a tile share one LDS exchange region (transformed one after the
// other), so that two-target tiles are not held to 4 per CU by their LDS.
constexpr bool kConvSharedLds = true;
// Conversion tiles with at most 16 elements per thread keep the next
// source's loads in flight during the current source's products.
constexpr bool kConvPrefetch = true;
template <int TT>
constexpr int conv_lds_regions() { return kConvSharedLds ? 1 : TT; }

// ONEC: the launch guarantees nsrc <= 16 (one chunk of sums): compiled
// without the chunk loop, no partial result is live during the products.
template <int A, int TT, bool ONEC = false>
__device__ __forceinline__ void tile_bconv_col(const DevPlan &P, const uint32_t *src, uint32_t nsrc,
                                               const uint32_t *cbase, uint32_t cstride, const uint32_t (&tg)[TT],
                                               const uint32_t (&tcol)[TT], uint32_t *const (&tout)[TT],
                                               uint32_t ntgt, uint32_t c0, uint32_t *lds) {
  using G = ColGeom<A>;
  constexpr int R1 = G::R1, R2 = G::R2, TPS = G::TPS, W = G::W, E = G::E;
  const size_t N = (size_t)1 << P.log_n;
  const int w = threadIdx.x % W, tig = threadIdx.x / W;
  using Ph1 = Phase<A, 1, R1>;
  ModQ mq[TT];
#pragma unroll
  for (int e = 0; e < TT; e++) mq[e] = ldmodc(P.mods + tg[e]);
  // the targets' column twiddles, staged in LDS after the data regions once
  // the conversion is done
  ColTw<A> ct[TT];
  double qr[TT];
#pragma unroll
  for (int e = 0; e < TT; e++) {
    ct[e].issue(P.tw_fwd32 + (size_t)tg[e] * N);
    qr[e] = ldcd(P.qrecip + tg[e]);
  }
  uint2 *twl = reinterpret_cast<uint2 *>(lds + conv_lds_regions<TT>() * G::LDS);
  uint32_t y[TT][E];
#pragma unroll
  for (int e = 0; e < TT; e++)
#pragma unroll
    for (int u = 0; u < E; u++) y[e][u] = 0;
  // Element u of this thread sits at row (tig + u * 2^LOB) of the column
  // block: the per-thread part of its byte offset is one VGPR, the source
  // and row parts are uniform (no vector address arithmetic per load).
  constexpr int LOB = Ph1::LOB;
  const __amdgpu_buffer_rsrc_t rs = buf_rsrc(src, (uint32_t)(nsrc * N * 4));
  const uint32_t vsrc = ((uint32_t)tig * 256u + c0 + w) * 4u;
  auto load_src = [&](uint32_t (&xv)[E], uint32_t i) {
    const uint32_t sb = (uint32_t)(i * N) * 4u;
#pragma unroll
    for (int u = 0; u < E; u++) xv[u] = buf_ld(rs, vsrc, sb + ((uint32_t)u << (LOB + 10)));
  };
  for (uint32_t i0 = 0; i0 < (ONEC ? 1u : nsrc); i0 += 16) {
    const uint32_t i1 = min(nsrc, i0 + 16);
    uint64_t acc[TT][E];
#pragma unroll
    for (int e = 0; e < TT; e++)
#pragma unroll
      for (int u = 0; u < E; u++) acc[e][u] = 0;
    auto macc = [&](const uint32_t (&xv)[E], uint32_t i) {
      uint32_t c[TT];
#pragma unroll
      for (int e = 0; e < TT; e++) c[e] = ldc(cbase + (size_t)i * cstride + tcol[e]);
#pragma unroll
      for (int u = 0; u < E; u++)
#pragma unroll
        for (int e = 0; e < TT; e++) acc[e][u] = mad64(xv[u], c[e], acc[e][u]);
    };
    uint32_t xa[E];
    if constexpr (kConvPrefetch && E <= 16) {
      // two source buffers: the next source's loads are in flight while
      // this one's products run (loads past the last source read 0)
      uint32_t xb[E];
      load_src(xa, i0);
      for (uint32_t i = i0; i < i1; i += 2) {
        const bool two = i + 1 < i1;
        if (two) load_src(xb, i + 1);
        macc(xa, i);
        if (two) {
          if (i + 2 < i1) load_src(xa, i + 2);
          macc(xb, i + 1);
        }
      }
    } else {
      for (uint32_t i = i0; i < i1; i++) {
        load_src(xa, i);
        macc(xa, i);
      }
    }
#pragma unroll
    for (int e = 0; e < TT; e++)
#pragma unroll
      for (int u = 0; u < E; u++)  // one chunk: [0, 3q) feeds the forward column pass ([0, 4q) accepted)
        y[e][u] = ONEC ? redc64_lazy(acc[e][u], mq[e]) : csub(y[e][u] + redc64(acc[e][u], mq[e]), mq[e].q);
  }
#pragma unroll
  for (int e = 0; e < TT; e++) ct[e].store(twl + e * (1 << A), mq[e].q, qr[e], true);
  __syncthreads();
  // forward column pass of each target: phase 1 in registers, phase 2 after
  // an LDS exchange (region r = e, or 0 when the targets share one)
  auto phase2 = [&](int e, int r) {
    using Ph2 = Phase<A, 1 + R1, R2>;
    const LdsTw tw{twl + e * (1 << A)};
    const __amdgpu_buffer_rsrc_t rt = buf_rsrc(tout[e], (uint32_t)(N * 4));
#pragma unroll
    for (int gi = 0; gi < Ph2::GROUPS / TPS; gi++) {
      const int gg = tig + gi * TPS;
      uint32_t x[1 << R2];
#pragma unroll
      for (int u = 0; u < (1 << R2); u++) x[u] = lds[r * G::LDS + Ph2::elem(gg, u) * W + w];
      ct_group<A, 1 + R1, R2>(x, gg, 1u, tw, mq[e].q);
      const uint32_t vb = ((uint32_t)Ph2::base(gg) * 256u + c0 + w) * 4u;
#pragma unroll
      for (int u = 0; u < (1 << R2); u++) buf_st_nt(rt, vb, (uint32_t)u << (Ph2::LOB + 10), x[u]);
    }
  };
  constexpr bool SHARED = R2 > 0 && conv_lds_regions<TT>() == 1 && TT > 1;
#pragma unroll
  for (int e = 0; e < TT; e++) {
    if ((uint32_t)e < ntgt) {
      const LdsTw tw{twl + e * (1 << A)};
      ct_group<A, 1, R1>(y[e], tig, 1u, tw, mq[e].q);
      if constexpr (R2 > 0) {
        const int r = SHARED ? 0 : e;
#pragma unroll
        for (int u = 0; u < E; u++) lds[r * G::LDS + Ph1::elem(tig, u) * W + w] = y[e][u];
      } else {
        const __amdgpu_buffer_rsrc_t rt = buf_rsrc(tout[e], (uint32_t)(N * 4));
        const uint32_t vb = ((uint32_t)Ph1::base(tig) * 256u + c0 + w) * 4u;
#pragma unroll
        for (int u = 0; u < E; u++) buf_st_nt(rt, vb, (uint32_t)u << (LOB + 10), y[e][u]);
      }
    }
    if constexpr (SHARED) {  // this target's phase 2 before the next one's phase 1 overwrites the region
      __syncthreads();
      if ((uint32_t)e < ntgt) phase2(e, 0);
      if (e + 1 < TT) __syncthreads();
    }
  }
  if constexpr (R2 > 0 && !SHARED) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < TT; e++)
      if ((uint32_t)e < ntgt) phase2(e, e);
  }
  __syncthreads();
}

// UP_P and UP_Q tiles: decode (digit, target chunk, column block).
template <int A, int TT, bool ONEC = false>
__device__ __forceinline__ void tile_up(const DevPlan &P, const OcJob &J, uint32_t tile, bool special, uint32_t ttu,
                                        uint32_t *lds) {
  using G = ColGeom<A>;
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t L1 = J.level + 1, T = L1 + P.num_p, ndig = cdiv(L1, P.alpha);
  const uint32_t unit = tile / G::CB, c0 = (tile % G::CB) * G::W;
  uint32_t j, chunk, lo, s;
  if (special) {
    const uint32_t per = cdiv(P.num_p, ttu);
    j = unit / per;
    chunk = unit % per;
    lo = j * P.alpha;
    s = min(lo + P.alpha, L1) - lo;
  } else {
    uint32_t u = unit;
    for (j = 0; j < ndig; j++) {
      lo = j * P.alpha;
      s = min(lo + P.alpha, L1) - lo;
      const uint32_t nt = cdiv(L1 - s, ttu);
      if (u < nt) break;
      u -= nt;
    }
    if (j >= ndig) return;
    chunk = u;
  }
  uint32_t tg[TT], tcol[TT], ntgt = 0;
  uint32_t *tout[TT];
#pragma unroll
  for (int e = 0; e < TT; e++) {
    const uint32_t ci = chunk * ttu + e;
    uint32_t t = 0;
    bool ok;
    if (special) {
      ok = (uint32_t)e < ttu && ci < P.num_p;
      t = L1 + ci;
    } else {
      ok = (uint32_t)e < ttu && ci < L1 - s;
      t = ci < lo ? ci : ci + s;
    }
    tg[e] = ok ? oc_gidx(P.num_q, J.level, t) : 0;
    tcol[e] = tg[e];
    tout[e] = ok ? J.ycol + ((size_t)j * T + t) * N : nullptr;
    if (ok) ntgt = e + 1;
  }
  tile_bconv_col<A, TT, ONEC>(P, J.xt + (size_t)lo * N, s, P.up_conv + ((size_t)j * P.alpha + (s - 1)) * P.alpha * P.ntot,
                        P.ntot, tg, tcol, tout, ntgt, c0, lds);
}

// DN tiles: decode (poly, Q-target chunk, column block).
template <int A, int TT, bool ONEC = false>
__device__ __forceinline__ void tile_dn(const DevPlan &P, const OcJob &J, uint32_t tile, uint32_t ttd, uint32_t *lds) {
  using G = ColGeom<A>;
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t L1 = J.level + 1, per = cdiv(L1, ttd);
  const uint32_t unit = tile / G::CB, c0 = (tile % G::CB) * G::W, s = unit / per, chunk = unit % per;
  uint32_t tg[TT], tcol[TT], ntgt = 0;
  uint32_t *tout[TT];
#pragma unroll
  for (int e = 0; e < TT; e++) {
    const uint32_t i = chunk * ttd + e;
    const bool ok = (uint32_t)e < ttd && i < L1;
    tg[e] = tcol[e] = ok ? i : 0;
    tout[e] = ok ? J.wcol + ((size_t)s * L1 + i) * N : nullptr;
    if (ok) ntgt = e + 1;
  }
  tile_bconv_col<A, TT, ONEC>(P, J.zp + (size_t)s * P.num_p * N, P.num_p, P.dn_conv, P.num_q, tg, tcol, tout, ntgt, c0, lds);
}

// ROW_P / ROW_Q tiles: (tower, block of kRB4 = 4 rows).  A row's
// transforms are independent of each other (one per foreign digit, plus the
// two ModDown terms for a Q tower), so the 64 threads of a row form 4 slots
// of 16 threads, each slot running one row transform into its own LDS row;
// then all 64 threads finish element-wise, 4 consecutive words each: key
// multiply-accumulate over the digits, REDC, and either (Q) the ModDown
// subtraction and P^-1, or (P) the inverse row transforms of both
// accumulators (slots 0 and 1).
constexpr int kSlots = 4;
constexpr int kRB4 = kOcThreads / (16 * kSlots);  // rows per tile
static_assert(kRB4 == kRBQ, "tile shape matches the host tile count");
constexpr int kRowBufs = kSlots * kRB4;           // LDS rows used per round
// Buffer of slot b in row r: the 4 slots of a row (one wave) sit kPad = 272
// words apart, i.e. 16 banks apart, so the slots' accesses do not collide.
__device__ __forceinline__ uint32_t *row_buf(uint32_t *lds, int b, int r) { return lds + (r * kSlots + b) * kPad; }

// The row tiles keep the twiddles of their 4 rows in LDS, in heap order: a
// row's entry i in [1, 256) is stage s = floor(log2 i) + 1, index
// j = i - 2^(s-1) of that stage, i.e. table entry ((M - 1) << (s - 1)) + i of
// the row's node M.  One cooperative, coalesced fill per tile replaces 30
// register-resident twiddle pairs per thread.  Stages 5-8 (t = s - 5) are
// read by the 16 threads of a row at j = tig * 2^t + k; they are stored at
// 2^(s-1) + k * 16 + tig so that the 16 threads read 16 consecutive entries,
// and rows are 260 entries apart so that the 4 rows of a wave fall on
// different banks.
constexpr int kRowTw = 256;    // heap entries per row
constexpr int kRowTwS = 260;   // LDS stride between rows (uint2)
constexpr int kRowTileLds = kRowBufs * kPad + 2 * kRB4 * kRowTwS;
constexpr int kRowTileLdsExt = kRowTileLds + 2 * kRB4 * kRowTwS;  // + the permuted rows' twiddles
__device__ __forceinline__ uint2 *row_tw(uint32_t *lds) { return reinterpret_cast<uint2 *>(lds + kRowBufs * kPad); }
__device__ __forceinline__ int row_tw_slot(int i) {  // LDS position of heap entry i in its row
  const int lvl = 31 - __clz(i | 1);
  if (lvl < 4) return i;
  const int t = lvl - 4, j = i - (1 << lvl);
  return (1 << lvl) + ((j & ((1 << t) - 1)) << 4) + (j >> t);
}

// Issue the twiddle loads of the tile's rows (node of row 0: m0) from a
// 4-byte table; the LDS stores (with the Shoup companions derived there) are
// separate so that other loads can be issued in between.
__device__ __forceinline__ void row_tw_issue(uint32_t (&t)[kRB4 * kRowTw / kOcThreads], const uint32_t *tw32,
                                             uint32_t m0) {
#pragma unroll
  for (int k = 0; k < kRB4 * kRowTw / kOcThreads; k++) {
    const int e = (int)threadIdx.x + k * kOcThreads, r = e >> 8, i = e & 255;
    const int lvl = 31 - __clz(i | 1);
    t[k] = gp(tw32)[((size_t)(m0 + r - 1) << lvl) + (i | (i == 0))];  // entry 0 unused: read entry 1
  }
}
// fwd: entries (-w mod 2^32, companion of w) as bfly_ct wants them
__device__ __forceinline__ void row_tw_store(uint2 *twl, const uint32_t (&t)[kRB4 * kRowTw / kOcThreads], uint32_t q,
                                             double qr, bool fwd) {
#pragma unroll
  for (int k = 0; k < kRB4 * kRowTw / kOcThreads; k++) {
    const int e = (int)threadIdx.x + k * kOcThreads, r = e >> 8, i = e & 255;
    twl[r * kRowTwS + row_tw_slot(i)] = make_uint2(fwd ? 0u - t[k] : t[k], shoup_companion(t[k], q, qr));
  }
}

// Four forward / inverse stages on 16 registers with twiddles from a row's
// LDS heap: S0 = 1 for row stages 1-4 (every thread of the row reads the
// same entries), S0 = 5 for stages 5-8 (thread tig, transposed layout).
template <int S0>
__device__ __forceinline__ uint2 row_tw_at(const uint2 *twr, int tig, int t, int k) {
  if constexpr (S0 == 1) return twr[(1 << t) + k];
  else return twr[(1 << (4 + t)) + (k << 4) + tig];
}
template <int S0>
__device__ __forceinline__ void ct_lds(uint32_t (&x)[16], const uint2 *twr, int tig, uint32_t q) {
#pragma unroll
  for (int t = 0; t < 4; t++) {
    const int half = 1 << (3 - t);
#pragma unroll
    for (int u = 0; u < 16; u++) {
      if (u & half) continue;
      const uint2 w = row_tw_at<S0>(twr, tig, t, u >> (4 - t));
      bfly_ct(x[u], x[u + half], w.x, w.y, q);
    }
  }
}
template <int S0>
__device__ __forceinline__ void gs_lds(uint32_t (&x)[16], const uint2 *twr, int tig, uint32_t q) {
#pragma unroll
  for (int t = 3; t >= 0; t--) {
    const int half = 1 << (3 - t);
#pragma unroll
    for (int u = 0; u < 16; u++) {
      if (u & half) continue;
      const uint2 w = row_tw_at<S0>(twr, tig, t, u >> (4 - t));
      bfly_gs(x[u], x[u + half], w.x, w.y, q);
    }
  }
}

// Forward row transform of x (loaded from the source row in phase-1 order
// k = tig + 16u) into LDS row lrow (phase-2 order at rl(k)); `act` = this
// slot has a job.  Every thread executes the barriers.
__device__ __forceinline__ void row_round_fwd(uint32_t (&x)[16], bool act, uint32_t *lrow, int tig,
                                              const uint2 *twr, uint32_t q) {
  if (act) {
    ct_lds<1>(x, twr, tig, q);
#pragma unroll
    for (int u = 0; u < 16; u++) lrow[rl(tig + 16 * u)] = x[u];
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int u = 0; u < 16; u++) x[u] = lrow[rl(16 * tig + u)];
    ct_lds<5>(x, twr, tig, q);
#pragma unroll
    for (int u = 0; u < 16; u++) lrow[rl(16 * tig + u)] = x[u];  // same words: no other reader
  }
  __syncthreads();
}

__device__ __forceinline__ void lds4(uint32_t (&v)[4], const uint32_t *lrow, int k0) {
#pragma unroll
  for (int i = 0; i < 4; i++) v[i] = lrow[rl(k0 + i)];
}
__device__ __forceinline__ void ld4(uint32_t (&v)[4], const uint32_t *p) {
  const uint4 t = ldg4(p);
  v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
__device__ __forceinline__ void ld4_nt(uint32_t (&v)[4], const uint32_t *p) {
  const uint4 t = ldg4_nt(p);
  v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}

template <bool IS_P, bool SEEDED, bool EXT, bool ONE = false>
__device__ __forceinline__ void tile_row(const DevPlan &P, const OcJob &J, uint32_t tile, uint32_t *lds) {
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t level = J.level, L1 = level + 1, T = L1 + P.num_p;
  const uint32_t rbk = (1u << P.loga) / kRB4, unit = tile / rbk, blk = tile % rbk;
  const uint32_t t = IS_P ? L1 + unit : unit;
  const uint32_t g = oc_gidx(P.num_q, level, t);
  const ModQ m = ldmodc(P.mods + g);
  const uint32_t q = m.q;
  const int r = threadIdx.x >> 6, slot = (threadIdx.x >> 4) & 3, tig = threadIdx.x & 15;
  const int k0 = 4 * (threadIdx.x & 63);  // element-wise part: words k0..k0+3 of the row
  const uint32_t row0 = blk * kRB4, m0 = (1u << P.loga) + row0;
  const size_t roff = (size_t)(row0 + r) * 256;
  // EXT: digit word j of this row is read at pi(j) of the automorphism; pi
  // maps the whole row onto row roff_s / 256, word k0 + i onto pofs[i]
  // and the tile's 4 rows onto an aligned block of 4 rows from row rs0; a
  // permuted row is transformed with its own row twiddles (second table)
  size_t roff_s = roff;
  uint32_t pofs[4] = {(uint32_t)k0, (uint32_t)k0 + 1, (uint32_t)k0 + 2, (uint32_t)k0 + 3};
  uint32_t rs0 = 0;
  if (EXT) {
    roff_s = galois_perm((uint32_t)roff, J.galois, P.log_n) & ~255u;
#pragma unroll
    for (int i = 0; i < 4; i++) pofs[i] = galois_perm((uint32_t)roff + k0 + i, J.galois, P.log_n) & 255u;
    rs0 = (galois_perm(row0 * 256u, J.galois, P.log_n) >> 8) & ~(uint32_t)(kRB4 - 1);
  }
  const uint32_t ndig = cdiv(L1, P.alpha);
  const uint32_t own = IS_P ? 0xffffffffu : t / P.alpha;  // digit holding tower t (bypassed)
  uint2 *twl = row_tw(lds);
  const uint2 *twr = twl + r * kRowTwS;
  uint2 *twl_s = twl + kRB4 * kRowTwS;  // EXT: twiddles of the permuted rows
  const uint2 *twr_s = EXT ? twl_s + (uint32_t)((roff_s >> 8) - rs0) * kRowTwS : twr;
  // key row of digit j: full key, half h at (2 j + h) ntot N; compressed
  // key, b half at j ntot N (that offset is also the a half's counter)
  const uint32_t *evk_t = J.evk + (size_t)g * N + roff + k0;
  const size_t evk_step = (size_t)P.ntot * N;
  constexpr uint32_t kHalves = SEEDED ? 1 : 2;
  const uint32_t ctr0 = (uint32_t)((size_t)g * N + roff + k0);
  auto gen_a = [&](uint32_t (&a)[4], uint32_t j) { seeded_a4(a, J.a_seed, ctr0 + j * (uint32_t)evk_step, m); };

  // transform jobs: IS_P: every digit; Q: the two ModDown terms, then the
  // foreign digits.  Job jb of a round runs in slot jb % 4.  ONE: the launch
  // guarantees njobs <= 4, and the tile is compiled without the round loop,
  // whose back edge keeps about 70 more VGPRs live (71 instead of 153 for
  // ROW_Q: 6 instead of 3 waves per SIMD).
  const uint32_t njobs = IS_P ? ndig : ndig + 1;
  auto job_digit = [&](uint32_t jb) -> uint32_t {
    if (!IS_P && jb < 2) return 0xffffffffu;
    uint32_t j = IS_P ? jb : jb - 2;
    if (!IS_P && j >= own) j++;  // skip the own digit
    return j;
  };
  auto job_src = [&](uint32_t jb) -> const uint32_t * {
    const uint32_t j = job_digit(jb);
    if (j == 0xffffffffu) return J.wcol + ((size_t)jb * L1 + t) * N + roff;
    return J.ycol + ((size_t)j * T + t) * N + roff_s;
  };
  // Loads are unconditional (an idle slot re-reads the round's last row, a
  // job without a key reads a key row the tile reads anyway) so that the
  // number of loads in flight is the same on every path and each wait
  // covers exactly the loads it needs.  The one exception is decided at
  // compile time: the ModDown slots of a Q tile's first round load no key.
  auto load_src = [&](uint32_t (&x)[16], uint32_t base) {
    const uint32_t *src = job_src(min(base + slot, njobs - 1));
#pragma unroll
    for (int u = 0; u < 16; u++) x[u] = gp(src)[tig + 16 * u];
  };
  uint32_t ek[kSlots][2][4];
  const uint32_t dummy = IS_P ? 0 : own;
  auto load_keys = [&](uint32_t base) {
#pragma unroll
    for (int s2 = 0; s2 < kSlots; s2++) {
      const uint32_t jb2 = base + s2;
      // the ModDown terms of the first round have no key (known at compile
      // time: no registers and no loads for them)
      if (!IS_P && jb2 < 2) continue;
      uint32_t d2 = jb2 < njobs ? job_digit(jb2) : 0xffffffffu;
      d2 = d2 == 0xffffffffu ? dummy : d2;
      ld4_nt(ek[s2][0], evk_t + (kHalves * d2 + 0) * evk_step);
      if (!SEEDED) ld4_nt(ek[s2][1], evk_t + (kHalves * d2 + 1) * evk_step);
    }
  };

  // Loads in the order they are needed (the memory counter completes in
  // order): twiddles, the first round's source rows, the own digit (Q), the
  // first round's key words.
  uint32_t tw4[kRB4 * kRowTw / kOcThreads];
  row_tw_issue(tw4, P.tw_fwd32 + (size_t)g * N, m0);
  uint32_t tws4[EXT ? kRB4 * kRowTw / kOcThreads : 1];
  if constexpr (EXT) row_tw_issue(tws4, P.tw_fwd32 + (size_t)g * N, (1u << P.loga) + rs0);
  const double qr = ldcd(P.qrecip + g);
  uint32_t x[16];
  load_src(x, 0);
  uint32_t yo[4], eo0[4], eo1[4];
  auto load_own = [&]() {  // own digit: the input tower itself (Sec. IV-C bypass)
    if (EXT) {
#pragma unroll
      for (int i = 0; i < 4; i++) yo[i] = gp(J.d)[(size_t)t * N + roff_s + pofs[i]];
    } else {
      ld4(yo, J.d + (size_t)t * N + roff + k0);
    }
    ld4_nt(eo0, evk_t + (kHalves * own + 0) * evk_step);
    if (!SEEDED) ld4_nt(eo1, evk_t + (kHalves * own + 1) * evk_step);
  };
  // ONE: issued after the forward transform, so that they are not held
  // through it (their latency is covered by the slot products and the other
  // waves)
  if (!IS_P && !ONE) load_own();
  load_keys(0);
  // ROW_P: the inverse twiddles of its ModDown P1 pass are loaded now, so
  // that their latency overlaps the forward round instead of following it
  uint32_t twi4[kRB4 * kRowTw / kOcThreads];
  if (IS_P) row_tw_issue(twi4, P.tw_inv32 + (size_t)g * N, m0);
  row_tw_store(twl, tw4, q, qr, true);
  if constexpr (EXT) row_tw_store(twl_s, tws4, q, qr, true);
  __syncthreads();

  // at most 16 digits (checked at plan creation): one REDC per sum
  uint64_t acc0[4] = {0, 0, 0, 0}, acc1[4] = {0, 0, 0, 0};
  uint32_t w0[4] = {0, 0, 0, 0}, w1[4] = {0, 0, 0, 0};
  for (uint32_t base = 0; base < (ONE ? 1u : njobs); base += kSlots) {
    if (base) {
      load_src(x, base);
      load_keys(base);
    }
    // a ModDown term is a natural row; a digit row is permuted under EXT
    const bool perm_row = EXT && base + slot < njobs && job_digit(base + slot) != 0xffffffffu;
    row_round_fwd(x, base + slot < njobs, row_buf(lds, slot, r), tig, perm_row ? twr_s : twr, q);
    if (!IS_P && ONE) load_own();
#pragma unroll
    for (int s2 = 0; s2 < kSlots; s2++) {
      const uint32_t jb2 = base + s2;
      if (jb2 >= njobs) break;
      uint32_t y[4];
      if (EXT && job_digit(jb2) != 0xffffffffu) {
#pragma unroll
        for (int i = 0; i < 4; i++) y[i] = row_buf(lds, s2, r)[rl(pofs[i])];
      } else {
        lds4(y, row_buf(lds, s2, r), k0);
      }
#pragma unroll
      for (int i = 0; i < 4; i++) y[i] = canon4(y[i], q);
      if (job_digit(jb2) == 0xffffffffu) {
#pragma unroll
        for (int i = 0; i < 4; i++) (jb2 == 0 ? w0 : w1)[i] = y[i];
      } else {
        if (SEEDED) gen_a(ek[s2][1], job_digit(jb2));
#pragma unroll
        for (int i = 0; i < 4; i++) {
          acc0[i] = mad64(y[i], ek[s2][0][i], acc0[i]);
          acc1[i] = mad64(y[i], ek[s2][1][i], acc1[i]);
        }
      }
    }
    __syncthreads();  // LDS rows are rewritten by the next round
  }
  if (!IS_P) {
    if (SEEDED) gen_a(eo1, own);
#pragma unroll
    for (int i = 0; i < 4; i++) {
      acc0[i] = mad64(yo[i], eo0[i], acc0[i]);
      acc1[i] = mad64(yo[i], eo1[i], acc1[i]);
    }
  }
  // P: canonical for the inverse row pass; Q: [0, 3q) into (r + q - w) P^-1,
  // a Shoup product that takes any 32-bit word
  uint32_t r0[4], r1[4];
#pragma unroll
  for (int i = 0; i < 4; i++) {
    r0[i] = IS_P ? redc64(acc0[i], m) : redc64_lazy(acc0[i], m);
    r1[i] = IS_P ? redc64(acc1[i], m) : redc64_lazy(acc1[i], m);
  }
  if (IS_P) {
    // ModDown P1 for this special tower: inverse row transforms of both
    // accumulators by slots 0 and 1 (values canonical, < 2q as required)
#pragma unroll
    for (int i = 0; i < 4; i++) {
      row_buf(lds, 0, r)[rl(k0 + i)] = r0[i];
      row_buf(lds, 1, r)[rl(k0 + i)] = r1[i];
    }
    row_tw_store(twl, twi4, q, qr, false);
    __syncthreads();
    uint32_t *lrow = row_buf(lds, slot & 1, r);
    const bool act = slot < 2;
    if (act) {
#pragma unroll
      for (int u = 0; u < 16; u++) x[u] = lrow[rl(16 * tig + u)];
      gs_lds<5>(x, twr, tig, q);
#pragma unroll
      for (int u = 0; u < 16; u++) lrow[rl(16 * tig + u)] = x[u];
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int u = 0; u < 16; u++) x[u] = lrow[rl(tig + 16 * u)];
      gs_lds<1>(x, twr, tig, q);
      uint32_t *dst = J.zp + ((size_t)slot * P.num_p + unit) * N + roff;
#pragma unroll
      for (int u = 0; u < 16; u++) gp(dst)[tig + 16 * u] = x[u];
    }
  } else {
    const uint2 f = ldc2(P.dn_fin + t);
    uint32_t o0[4], o1[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      o0[i] = csub(mul_shoup(r0[i] + q - w0[i], f.x, f.y, q), q);
      o1[i] = csub(mul_shoup(r1[i] + q - w1[i], f.x, f.y, q), q);
    }
    if (EXT) {  // the caller's addends, read through the same automorphism
      if (J.add0) {
#pragma unroll
        for (int i = 0; i < 4; i++) o0[i] = csub(o0[i] + gp(J.add0)[(size_t)t * N + roff_s + pofs[i]], q);
      }
      if (J.add1) {
#pragma unroll
        for (int i = 0; i < 4; i++) o1[i] = csub(o1[i] + gp(J.add1)[(size_t)t * N + roff_s + pofs[i]], q);
      }
    }
    stg4_nt(J.out + ((size_t)0 * L1 + t) * N + roff + k0, make_uint4(o0[0], o0[1], o0[2], o0[3]));
    stg4_nt(J.out + ((size_t)1 * L1 + t) * N + roff + k0, make_uint4(o1[0], o1[1], o1[2], o1[3]));
  }
  __syncthreads();
}

// Double hoisting, fused (ROW_P_SUM / ROW_Q_SUM): the tile sums the job's
// rotation terms before its one ModDown.  ROW_Q first transforms the two
// ModDown terms (natural rows).  Then, per term: the twiddles of the term's
// permuted 4-row block are staged, the digit rows are read through the
// term's automorphism and multiplied by its key (the own digit of a Q tower
// gathered from the input), the sum is reduced, multiplied by the term's
// diagonal (exact: REDC then a Shoup product by 2^32) and added to the
// running total.  The total, carrying 2^-32 like a single key switch's
// accumulator, then takes the ModDown path of tile_row; ROW_Q adds
// sum_r diag_r * sigma_r(c0).
__device__ __forceinline__ uint32_t mulmod_exact32(uint32_t a, uint32_t b, const ModQ &m, uint32_t r32,
                                                   uint32_t r32p) {
  return csub(mul_shoup(redc64((uint64_t)a * b, m), r32, r32p, m.q), m.q);
}

template <bool IS_P, bool ONE = false, bool PAIR = false>
__device__ __forceinline__ void tile_row_sum(const DevPlan &P, const OcJob &J, uint32_t tile, uint32_t *lds) {
  static_assert(!PAIR || (!IS_P && ONE), "term pairs: summing ROW_Q tiles of one round");
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t level = J.level, L1 = level + 1, T = L1 + P.num_p;
  const uint32_t rbk = (1u << P.loga) / kRB4, unit = tile / rbk, blk = tile % rbk;
  const uint32_t t = IS_P ? L1 + unit : unit;
  const uint32_t g = oc_gidx(P.num_q, level, t);
  const ModQ m = ldmodc(P.mods + g);
  const uint32_t q = m.q;
  const int r = threadIdx.x >> 6, slot = (threadIdx.x >> 4) & 3, tig = threadIdx.x & 15;
  const int k0 = 4 * (threadIdx.x & 63);
  const uint32_t row0 = blk * kRB4, m0 = (1u << P.loga) + row0;
  const size_t roff = (size_t)(row0 + r) * 256;
  const uint32_t ndig = cdiv(L1, P.alpha);
  const uint32_t own = IS_P ? 0xffffffffu : t / P.alpha;
  const uint32_t nfd = IS_P ? ndig : ndig - 1;  // transformed digits per term (Q: own digit bypassed)
  auto digit = [&](uint32_t jb) -> uint32_t { return (!IS_P && jb >= own) ? jb + 1 : jb; };
  uint2 *twl = row_tw(lds);
  const uint2 *twr = twl + r * kRowTwS;
  uint2 *twl_s = twl + kRB4 * kRowTwS;
  const double qr = ldcd(P.qrecip + g);
  const uint32_t r32 = (0u - q) % q;
  const uint32_t r32p = shoup_companion(r32, q, qr);
  const size_t evk_step = (size_t)P.ntot * N;
  uint32_t x[16];
  uint32_t tot0[4] = {0, 0, 0, 0}, tot1[4] = {0, 0, 0, 0};
  // Q: the transformed ModDown terms wait in the natural-twiddle LDS table,
  // which nothing reads after their round (8 words per thread, conflict-free)
  uint32_t *wst = reinterpret_cast<uint32_t *>(twl);
  if (!IS_P) {  // the two ModDown terms: slots 0 and 1, natural rows and twiddles
    uint32_t tw4[kRB4 * kRowTw / kOcThreads];
    row_tw_issue(tw4, P.tw_fwd32 + (size_t)g * N, m0);
    const uint32_t *src = J.wcol + ((size_t)(slot & 1) * L1 + t) * N + roff;
#pragma unroll
    for (int u = 0; u < 16; u++) x[u] = gp(src)[tig + 16 * u];
    row_tw_store(twl, tw4, q, qr, true);
    __syncthreads();
    row_round_fwd(x, slot < 2, row_buf(lds, slot, r), tig, twr, q);
    uint32_t w0[4], w1[4];
    lds4(w0, row_buf(lds, 0, r), k0);
    lds4(w1, row_buf(lds, 1, r), k0);
    __syncthreads();  // every thread is done with the natural twiddles and the rows
#pragma unroll
    for (int i = 0; i < 4; i++) {
      wst[threadIdx.x + kOcThreads * i] = canon4(w0[i], q);
      wst[threadIdx.x + kOcThreads * (4 + i)] = canon4(w1[i], q);
    }
  }
  uint32_t twi4[kRB4 * kRowTw / kOcThreads];
  if (IS_P) row_tw_issue(twi4, P.tw_inv32 + (size_t)g * N, m0);
  if constexpr (!PAIR) {
    for (uint32_t ti = 0; ti < J.nterm; ti++) {
      const RotTerm rt = J.terms[ti];
      const size_t roff_s = galois_perm((uint32_t)roff, rt.galois, P.log_n) & ~255u;
      uint32_t pofs[4];
  #pragma unroll
      for (int i = 0; i < 4; i++) pofs[i] = galois_perm((uint32_t)roff + k0 + i, rt.galois, P.log_n) & 255u;
      const uint32_t rs0 = (galois_perm(row0 * 256u, rt.galois, P.log_n) >> 8) & ~(uint32_t)(kRB4 - 1);
      const uint2 *twr_s = twl_s + (uint32_t)((roff_s >> 8) - rs0) * kRowTwS;
      const uint32_t *evk_t = rt.evk + (size_t)g * N + roff + k0;
      uint32_t tws4[kRB4 * kRowTw / kOcThreads];
      row_tw_issue(tws4, P.tw_fwd32 + (size_t)g * N, (1u << P.loga) + rs0);
      auto load_src = [&](uint32_t base) {
        const uint32_t *src = J.ycol + ((size_t)digit(min(base + slot, nfd - 1)) * T + t) * N + roff_s;
  #pragma unroll
        for (int u = 0; u < 16; u++) x[u] = gp(src)[tig + 16 * u];
      };
      uint32_t ek[kSlots][2][4];
      auto load_keys = [&](uint32_t base) {
  #pragma unroll
        for (int s2 = 0; s2 < kSlots; s2++) {
          const uint32_t d2 = digit(min(base + s2, nfd - 1));  // idle slots re-read a row the tile reads
          ld4_nt(ek[s2][0], evk_t + (2 * d2 + 0) * evk_step);
          ld4_nt(ek[s2][1], evk_t + (2 * d2 + 1) * evk_step);
        }
      };
      if (nfd) {
        load_src(0);
        load_keys(0);
      }
      row_tw_store(twl_s, tws4, q, qr, true);  // the previous term's rounds ended with a barrier
      __syncthreads();
      uint64_t acc0[4] = {0, 0, 0, 0}, acc1[4] = {0, 0, 0, 0};
      // ONE: the launch guarantees nfd <= 4 (one round per term)
      for (uint32_t base = 0; base < (ONE ? 1u : nfd); base += kSlots) {
        if (base) {
          load_src(base);
          load_keys(base);
        }
        row_round_fwd(x, base + slot < nfd, row_buf(lds, slot, r), tig, twr_s, q);
  #pragma unroll
        for (int s2 = 0; s2 < kSlots; s2++) {
          if (base + s2 >= nfd) break;
          uint32_t y[4];
  #pragma unroll
          for (int i = 0; i < 4; i++) y[i] = canon4(row_buf(lds, s2, r)[rl(pofs[i])], q);
  #pragma unroll
          for (int i = 0; i < 4; i++) {
            acc0[i] = mad64(y[i], ek[s2][0][i], acc0[i]);
            acc1[i] = mad64(y[i], ek[s2][1][i], acc1[i]);
          }
        }
        __syncthreads();  // LDS rows are rewritten by the next round
      }
      if (!IS_P) {  // the own digit, loaded after the rounds: fewer registers held across them
        uint32_t yo[4], eo0[4], eo1[4];
  #pragma unroll
        for (int i = 0; i < 4; i++) yo[i] = gp(J.d)[(size_t)t * N + roff_s + pofs[i]];
        ld4_nt(eo0, evk_t + (2 * own + 0) * evk_step);
        ld4_nt(eo1, evk_t + (2 * own + 1) * evk_step);
  #pragma unroll
        for (int i = 0; i < 4; i++) {
          acc0[i] = mad64(yo[i], eo0[i], acc0[i]);
          acc1[i] = mad64(yo[i], eo1[i], acc1[i]);
        }
      }
  #pragma unroll
      for (int i = 0; i < 4; i++) {
        uint32_t v0 = redc64(acc0[i], m), v1 = redc64(acc1[i], m);
        if (rt.diag) {
          const uint32_t pv = gp(rt.diag)[(size_t)g * N + roff + k0 + i];
          v0 = mulmod_exact32(v0, pv, m, r32, r32p);
          v1 = mulmod_exact32(v1, pv, m, r32, r32p);
        }
        tot0[i] = csub(tot0[i] + v0, q);
        tot1[i] = csub(tot1[i] + v1, q);
      }
    }
  } else {
    // Terms a = ti and b = ti + 1 share a round: a's digits run in slots
    // [0, nfd), b's in [nfd, 2 nfd), each read through its own automorphism
    // with its own permuted twiddles (b's table after a's).
    uint2 *twl_b = twl_s + kRB4 * kRowTwS;
    struct View {
      const uint32_t *evk_t, *diag;
      uint32_t roff_s, rs0, pofs[4];
    };
    auto view = [&](const RotTerm &rt) {
      View v;
      v.roff_s = galois_perm((uint32_t)roff, rt.galois, P.log_n) & ~255u;
#pragma unroll
      for (int i = 0; i < 4; i++) v.pofs[i] = galois_perm((uint32_t)roff + k0 + i, rt.galois, P.log_n) & 255u;
      v.rs0 = (galois_perm(row0 * 256u, rt.galois, P.log_n) >> 8) & ~(uint32_t)(kRB4 - 1);
      v.evk_t = rt.evk + (size_t)g * N + roff + k0;
      v.diag = rt.diag;
      return v;
    };
    for (uint32_t ti = 0; ti < J.nterm; ti += 2) {
      const bool hb = ti + 1 < J.nterm;
      const View va = view(J.terms[ti]);
      const View vb = view(J.terms[hb ? ti + 1 : ti]);
      // this thread's slot: term b past nfd, idle past 2 nfd (or without b)
      const bool in_b = (uint32_t)slot >= nfd;
      const bool act = in_b ? (hb && (uint32_t)slot < 2 * nfd) : true;
      const uint32_t dj = in_b ? (uint32_t)slot - nfd : (uint32_t)slot;
      // Idle slots read the own digit's rows: always in range (its ycol
      // region is allocated, never written, and the values go unused; its
      // key rows are read by the tile anyway), also without foreign digits.
      {
        const uint32_t *src = act ? J.ycol + ((size_t)digit(dj) * T + t) * N + (in_b ? vb.roff_s : va.roff_s)
                                  : J.ycol + ((size_t)own * T + t) * N + va.roff_s;
#pragma unroll
        for (int u = 0; u < 16; u++) x[u] = gp(src)[tig + 16 * u];
      }
      uint32_t ek[kSlots][2][4];
#pragma unroll
      for (int s2 = 0; s2 < kSlots; s2++) {
        const bool b2 = hb && (uint32_t)s2 >= nfd && (uint32_t)s2 < 2 * nfd;
        const uint32_t d2 = (uint32_t)s2 < nfd ? digit(s2) : b2 ? digit(s2 - nfd) : own;
        const uint32_t *ev = b2 ? vb.evk_t : va.evk_t;
        ld4_nt(ek[s2][0], ev + (2 * d2 + 0) * evk_step);
        ld4_nt(ek[s2][1], ev + (2 * d2 + 1) * evk_step);
      }
      uint32_t twa[kRB4 * kRowTw / kOcThreads], twb[kRB4 * kRowTw / kOcThreads];
      row_tw_issue(twa, P.tw_fwd32 + (size_t)g * N, (1u << P.loga) + va.rs0);
      row_tw_issue(twb, P.tw_fwd32 + (size_t)g * N, (1u << P.loga) + vb.rs0);
      row_tw_store(twl_s, twa, q, qr, true);  // the previous pair's round ended with a barrier
      row_tw_store(twl_b, twb, q, qr, true);
      __syncthreads();
      const uint2 *twr_a = twl_s + (uint32_t)((va.roff_s >> 8) - va.rs0) * kRowTwS;
      const uint2 *twr_b = twl_b + (uint32_t)((vb.roff_s >> 8) - vb.rs0) * kRowTwS;
      row_round_fwd(x, act && nfd > 0, row_buf(lds, slot, r), tig, in_b ? twr_b : twr_a, q);
      uint64_t acc[2][2][4] = {};
#pragma unroll
      for (int s2 = 0; s2 < kSlots; s2++) {
        const bool b2 = (uint32_t)s2 >= nfd;
        if (b2 && !(hb && (uint32_t)s2 < 2 * nfd)) break;
        const View &v = b2 ? vb : va;
        uint32_t y[4];
#pragma unroll
        for (int i = 0; i < 4; i++) y[i] = canon4(row_buf(lds, s2, r)[rl(v.pofs[i])], q);
#pragma unroll
        for (int i = 0; i < 4; i++) {
          acc[b2][0][i] = mad64(y[i], ek[s2][0][i], acc[b2][0][i]);
          acc[b2][1][i] = mad64(y[i], ek[s2][1][i], acc[b2][1][i]);
        }
      }
      __syncthreads();  // LDS rows and tables are rewritten by the next pair
#pragma unroll
      for (int e = 0; e < 2; e++) {
        if (e && !hb) break;
        const View &v = e ? vb : va;
        uint32_t yo[4], eo0[4], eo1[4];  // the own digit, as above
#pragma unroll
        for (int i = 0; i < 4; i++) yo[i] = gp(J.d)[(size_t)t * N + v.roff_s + v.pofs[i]];
        ld4_nt(eo0, v.evk_t + (2 * own + 0) * evk_step);
        ld4_nt(eo1, v.evk_t + (2 * own + 1) * evk_step);
#pragma unroll
        for (int i = 0; i < 4; i++) {
          uint32_t v0 = redc64(mad64(yo[i], eo0[i], acc[e][0][i]), m);
          uint32_t v1 = redc64(mad64(yo[i], eo1[i], acc[e][1][i]), m);
          if (v.diag) {
            const uint32_t pv = gp(v.diag)[(size_t)g * N + roff + k0 + i];
            v0 = mulmod_exact32(v0, pv, m, r32, r32p);
            v1 = mulmod_exact32(v1, pv, m, r32, r32p);
          }
          tot0[i] = csub(tot0[i] + v0, q);
          tot1[i] = csub(tot1[i] + v1, q);
        }
      }
    }
  }
  if (IS_P) {
    // ModDown P1 for this special tower, as in tile_row
#pragma unroll
    for (int i = 0; i < 4; i++) {
      row_buf(lds, 0, r)[rl(k0 + i)] = tot0[i];
      row_buf(lds, 1, r)[rl(k0 + i)] = tot1[i];
    }
    row_tw_store(twl, twi4, q, qr, false);
    __syncthreads();
    uint32_t *lrow = row_buf(lds, slot & 1, r);
    const bool act = slot < 2;
    if (act) {
#pragma unroll
      for (int u = 0; u < 16; u++) x[u] = lrow[rl(16 * tig + u)];
      gs_lds<5>(x, twr, tig, q);
#pragma unroll
      for (int u = 0; u < 16; u++) lrow[rl(16 * tig + u)] = x[u];
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int u = 0; u < 16; u++) x[u] = lrow[rl(tig + 16 * u)];
      gs_lds<1>(x, twr, tig, q);
      uint32_t *dst = J.zp + ((size_t)slot * P.num_p + unit) * N + roff;
#pragma unroll
      for (int u = 0; u < 16; u++) gp(dst)[tig + 16 * u] = x[u];
    }
  } else {
    const uint2 f = ldc2(P.dn_fin + t);
    uint32_t o0[4], o1[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      o0[i] = csub(mul_shoup(tot0[i] + q - wst[threadIdx.x + kOcThreads * i], f.x, f.y, q), q);
      o1[i] = csub(mul_shoup(tot1[i] + q - wst[threadIdx.x + kOcThreads * (4 + i)], f.x, f.y, q), q);
    }
    for (uint32_t ti = 0; ti < J.nterm; ti++) {  // + sum_r diag_r sigma_r(c0)
      const RotTerm rt = J.terms[ti];
      const size_t roff_s = galois_perm((uint32_t)roff, rt.galois, P.log_n) & ~255u;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const uint32_t pi = galois_perm((uint32_t)roff + k0 + i, rt.galois, P.log_n) & 255u;
        uint32_t cv = gp(J.add0)[(size_t)t * N + roff_s + pi];
        if (rt.diag) cv = mulmod_exact32(cv, gp(rt.diag)[(size_t)g * N + roff + k0 + i], m, r32, r32p);
        o0[i] = csub(o0[i] + cv, q);
      }
    }
    stg4_nt(J.out + ((size_t)0 * L1 + t) * N + roff + k0, make_uint4(o0[0], o0[1], o0[2], o0[3]));
    stg4_nt(J.out + ((size_t)1 * L1 + t) * N + roff + k0, make_uint4(o1[0], o1[1], o1[2], o1[3]));
  }
  __syncthreads();
}

// One tile of one phase.
template <int A, int TTU, int TTD>
__device__ __forceinline__ void oc_tile(const DevPlan &P, const OcJob &J, uint32_t phase, uint32_t tile,
                                        uint32_t *lds) {
  switch (phase) {
    case OC_INTT_ROW: tile_intt_row(P, J, tile, lds); break;
    case OC_INTT_COL: tile_intt_col<A>(P, J, tile, false, lds); break;
    case OC_UP_P: tile_up<A, TTU>(P, J, tile, true, J.ttu, lds); break;
    case OC_ROW_P: tile_row<true, false, false>(P, J, tile, lds); break;
    case OC_UP_Q: tile_up<A, TTU>(P, J, tile, false, J.ttu, lds); break;
    case OC_INTT_COL_DN: tile_intt_col<A>(P, J, tile, true, lds); break;
    case OC_DN: tile_dn<A, TTD>(P, J, tile, J.ttd, lds); break;
    case OC_ROW_Q: tile_row<false, false, false>(P, J, tile, lds); break;
  }
}

template <int A, int TT>
constexpr int cmax(int a, int b) { return a > b ? a : b; }
// LDS words of one phase's tiles, and of any phase (persistent kernel)
template <int A, int PHASE, int TT>
constexpr int oc_phase_lds_words() {
  return (PHASE == OC_ROW_P_EXT || PHASE == OC_ROW_Q_EXT || PHASE == OC_ROW_P_SEEDED_EXT ||
          PHASE == OC_ROW_Q_SEEDED_EXT || PHASE == OC_ROW_P_SUM || PHASE == OC_ROW_Q_SUM)
             ? kRowTileLdsExt
         : (PHASE == OC_ROW_P || PHASE == OC_ROW_Q || PHASE == OC_ROW_P_SEEDED || PHASE == OC_ROW_Q_SEEDED)
             ? kRowTileLds
         : PHASE == OC_INTT_ROW                   ? kRowLds
         : (PHASE == OC_INTT_COL || PHASE == OC_INTT_COL_DN) ? ColGeom<A>::LDS + 2 * (1 << A)
                                                           : conv_lds_regions<TT>() * ColGeom<A>::LDS + TT * 2 * (1 << A);
}
template <int A, int TT>
constexpr int oc_lds_words() {
  return cmax<A, TT>(cmax<A, TT>(TT * (ColGeom<A>::LDS + 2 * (1 << A)), kRowLds), kRowTileLds);
}

// Blocks of a launch are dealt to the 8 XCDs in turn (block b runs on XCD
// b % 8, each XCD with its own L2).  A column-tile index is unit * CB +
// column block; the remap gives XCD x the column blocks [x CB/8, (x+1) CB/8)
// of every unit, so the two 64-byte halves of a 128-byte line, and a source
// column read by many conversion targets, stay in one L2.  A bijection on
// [0, T) for every T that is a multiple of CB (tile counts of column phases
// are), so the per-job range checks stay valid.
template <int CB>
__device__ __forceinline__ uint32_t xcd_col_tile(uint32_t b) {
  if constexpr (CB % 8 != 0) {
    return b;
  } else {
    constexpr uint32_t per = CB / 8;
    const uint32_t x = b & 7u, k = b >> 3;
    return (k / per) * CB + x * per + (k % per);
  }
}

// One launch per phase: grid x = tiles (max over jobs), grid z = job; the
// row phases of a batch interleave their jobs in x instead (see
// oc_row_phase).  The multi-round summing row phases are asked for 3
// workgroups per CU (3 waves per SIMD): their loops otherwise hold 174-184
// VGPRs.  The others need no bound (the one-round ROW_Q reaches 6 waves per
// SIMD, its LDS limit, at 71 VGPRs).
template <int PHASE_ID>
constexpr int oc_min_blocks() {
  constexpr int PHASE = PHASE_ID & OC_PHASE_BITS;
  return (PHASE == OC_ROW_P_SUM || PHASE == OC_ROW_Q_SUM) ? 3 : 1;
}

// The row phases read the key.  In a batch their jobs are interleaved per
// group of 8 tiles: block b runs on XCD b % 8, and with grid x =
// roundup8(tiles) * njobs it takes tile (k / njobs) * 8 + b % 8 of job
// k % njobs (k = b / 8).  Tile t of every job then runs on XCD t % 8 within
// one window of 8 njobs blocks, so jobs that share a key read each key row
// from that XCD's L2 after the first.  (With jobs along grid z, the same
// tile of the next job ran a full round of tiles later, after its key rows
// had left the L2.)
template <int PHASE>
constexpr bool oc_row_phase() {
  return PHASE == OC_ROW_P || PHASE == OC_ROW_Q || PHASE == OC_ROW_P_SEEDED || PHASE == OC_ROW_Q_SEEDED ||
         PHASE == OC_ROW_P_EXT || PHASE == OC_ROW_Q_EXT || PHASE == OC_ROW_P_SEEDED_EXT ||
         PHASE == OC_ROW_Q_SEEDED_EXT || PHASE == OC_ROW_P_SUM || PHASE == OC_ROW_Q_SUM;
}

template <int A, int PHASE_ID, int TT>
__global__ __launch_bounds__(kOcThreads, oc_min_blocks<PHASE_ID>()) void k_oc_phase(
    DevPlan P, OcJob one, const OcJob *jobs, uint32_t njobs) {
  constexpr int PHASE = PHASE_ID & OC_PHASE_BITS;
  constexpr bool ONE = (PHASE_ID & OC_ONE_ROUND) != 0;
  constexpr bool PAIR = (PHASE_ID & OC_PAIR_TERMS) != 0;
  __shared__ uint32_t lds[oc_phase_lds_words<A, PHASE, TT>() + (PAIR ? 2 * kRB4 * kRowTwS : 0)];
  uint32_t bx = blockIdx.x, jz = blockIdx.z;
  if (oc_row_phase<PHASE>() && jobs) {
    const uint32_t k = blockIdx.x >> 3;
    jz = k % njobs;
    bx = (k / njobs) * 8 + (blockIdx.x & 7);
  }
  // the job table is read-only while the kernel runs: scalar loads keep
  // every job field (pointers, level, tile counts) uniform in SGPRs
  OcJob J = one;
  if (jobs) {
    static_assert(sizeof(OcJob) % 4 == 0, "job entries are whole words");
    const __attribute__((address_space(4))) uint32_t *src =
        (const __attribute__((address_space(4))) uint32_t *)(jobs + jz);
    uint32_t *dst = reinterpret_cast<uint32_t *>(&J);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(OcJob) / 4); i++) dst[i] = src[i];
  }
  constexpr bool COL = PHASE != OC_INTT_ROW && PHASE != OC_ROW_P && PHASE != OC_ROW_Q;
  if constexpr (PHASE == OC_ROW_P || PHASE == OC_ROW_Q) {
    constexpr bool IS_P = PHASE == OC_ROW_P;
    if (bx >= J.tiles[PHASE]) return;
    tile_row<IS_P, false, false, ONE>(P, J, bx, lds);
  } else if constexpr (PHASE == OC_ROW_P_SEEDED || PHASE == OC_ROW_Q_SEEDED) {
    constexpr bool IS_P = PHASE == OC_ROW_P_SEEDED;
    if (bx >= J.tiles[IS_P ? OC_ROW_P : OC_ROW_Q]) return;
    tile_row<IS_P, true, false, ONE>(P, J, bx, lds);
  } else if constexpr (PHASE == OC_ROW_P_EXT || PHASE == OC_ROW_Q_EXT || PHASE == OC_ROW_P_SEEDED_EXT ||
                       PHASE == OC_ROW_Q_SEEDED_EXT) {
    constexpr bool IS_P = PHASE == OC_ROW_P_EXT || PHASE == OC_ROW_P_SEEDED_EXT;
    constexpr bool SEEDED = PHASE == OC_ROW_P_SEEDED_EXT || PHASE == OC_ROW_Q_SEEDED_EXT;
    if (bx >= J.tiles[IS_P ? OC_ROW_P : OC_ROW_Q]) return;
    tile_row<IS_P, SEEDED, true, ONE>(P, J, bx, lds);
  } else if constexpr (PHASE == OC_ROW_P_SUM || PHASE == OC_ROW_Q_SUM) {
    constexpr bool IS_P = PHASE == OC_ROW_P_SUM;
    if (bx >= J.tiles[IS_P ? OC_ROW_P : OC_ROW_Q]) return;
    if constexpr (PAIR) tile_row_sum<false, true, true>(P, J, bx, lds);
    else tile_row_sum<IS_P, ONE>(P, J, bx, lds);
  } else if constexpr (PHASE == OC_UP_PQ) {
    const uint32_t np = J.tiles[OC_UP_P];
    const bool special = blockIdx.x < np;
    const uint32_t b = special ? blockIdx.x : blockIdx.x - np;
    if (!special && b >= J.tiles[OC_UP_Q]) return;
    tile_up<A, TT, ONE>(P, J, xcd_col_tile<ColGeom<A>::CB>(b), special, J.ttu, lds);
  } else if constexpr (PHASE == OC_DN) {
    if (blockIdx.x >= J.tiles[OC_DN]) return;
    tile_dn<A, TT, ONE>(P, J, xcd_col_tile<ColGeom<A>::CB>(blockIdx.x), J.ttd, lds);
  } else {
    if (blockIdx.x >= J.tiles[PHASE]) return;
    const uint32_t tile = COL ? xcd_col_tile<ColGeom<A>::CB>(blockIdx.x) : blockIdx.x;
    oc_tile<A, TT, TT>(P, J, PHASE, tile, lds);
  }
}

static const char *const kOcPhaseName[OC_NPHASE + 9] = {
    "oc.intt_row",      "oc.intt_col.up",    "oc.bconv_col.up_p", "oc.row.p",        "oc.bconv_col.up_q",
    "oc.intt_col.down", "oc.bconv_col.down", "oc.row.q",          "oc.bconv_col.up", "oc.row.p.seeded",
    "oc.row.q.seeded",  "oc.row.p.ext",      "oc.row.q.ext",      "oc.row.p.seeded_ext", "oc.row.q.seeded_ext",
    "oc.row.p.sum",     "oc.row.q.sum"};

template <int A, int PHASE, int TT>
static void launch_phase(const Plan &pl, const OcJob &one, const OcJob *jobs, uint32_t count, uint32_t tiles,
                         hipStream_t st) {
  if (!tiles) return;  // e.g. no Q target outside the only digit at level 0
  const dim3 grid = (oc_row_phase<(PHASE & OC_PHASE_BITS)>() && jobs) ? dim3((tiles + 7) / 8 * 8 * count, 1, 1)
                                                                      : dim3(tiles, 1, count);
  KS_LAUNCH(pl, kOcPhaseName[PHASE & OC_PHASE_BITS], (k_oc_phase<A, PHASE, TT>), grid, dim3(kOcThreads), 0, st,
            pl.dev, one, jobs, count);
}

// The row stage of one tower kind (special: ROW_P, else ROW_Q) in the
// variant `rows`; ONE = OC_ONE_ROUND or 0.
template <int A, bool SPECIAL, uint32_t ONE>
static void launch_row(const Plan &pl, const OcJob &one, const OcJob *jobs, uint32_t count,
                       const uint32_t *max_tiles, OcRowVariant rows, hipStream_t st) {
  const uint32_t tiles = max_tiles[SPECIAL ? OC_ROW_P : OC_ROW_Q];
  switch (rows) {
    case OC_ROWS_SEEDED:
      launch_phase<A, (SPECIAL ? OC_ROW_P_SEEDED : OC_ROW_Q_SEEDED) | ONE, 1>(pl, one, jobs, count, tiles, st);
      break;
    case OC_ROWS_EXT:
      launch_phase<A, (SPECIAL ? OC_ROW_P_EXT : OC_ROW_Q_EXT) | ONE, 1>(pl, one, jobs, count, tiles, st);
      break;
    case OC_ROWS_SEEDED_EXT:
      launch_phase<A, (SPECIAL ? OC_ROW_P_SEEDED_EXT : OC_ROW_Q_SEEDED_EXT) | ONE, 1>(pl, one, jobs, count, tiles,
                                                                                        st);
      break;
    case OC_ROWS_SUM:
      launch_phase<A, (SPECIAL ? OC_ROW_P_SUM : OC_ROW_Q_SUM) | ONE, 1>(pl, one, jobs, count, tiles, st);
      break;
    default: launch_phase<A, (SPECIAL ? OC_ROW_P : OC_ROW_Q) | ONE, 1>(pl, one, jobs, count, tiles, st); break;
  }
}

template <int A, int TT>
static void launch_phases_tt(const Plan &pl, const OcJob &one, const OcJob *jobs, uint32_t count,
                             const uint32_t *max_tiles, OcRowVariant rows, OcPart part, hipStream_t st) {
  if (part != OC_PART_REST) {
    launch_phase<A, OC_INTT_ROW, 1>(pl, one, jobs, count, max_tiles[OC_INTT_ROW], st);
    launch_phase<A, OC_INTT_COL, 1>(pl, one, jobs, count, max_tiles[OC_INTT_COL], st);
    // a job's merged grid needs at most its own UP_P + UP_Q tiles; sums of
    // at most 16 products (alpha <= 16) take the one-chunk build
    if (pl.alpha <= 16)
      launch_phase<A, OC_UP_PQ | OC_ONE_ROUND, TT>(pl, one, jobs, count, max_tiles[OC_UP_P] + max_tiles[OC_UP_Q], st);
    else
      launch_phase<A, OC_UP_PQ, TT>(pl, one, jobs, count, max_tiles[OC_UP_P] + max_tiles[OC_UP_Q], st);
  }
  if (part == OC_PART_MODUP) return;
  // the largest l+1 of the launch (ROW_Q tiles: row blocks x towers) decides
  // whether the row tiles of every job fit one round of the slot loop
  // (a ROW_Q tile transforms the foreign digits and the two ModDown terms; a
  // summing ROW_Q tile transforms the ModDown terms once, then per term only
  // the foreign digits)
  const uint32_t ndig = cdiv(max_tiles[OC_ROW_Q] / ((1u << A) / kRBQ), pl.alpha);
  const uint32_t qjobs = rows == OC_ROWS_SUM ? ndig - 1 : ndig + 1;
  if (ndig <= (uint32_t)kSlots) launch_row<A, true, OC_ONE_ROUND>(pl, one, jobs, count, max_tiles, rows, st);
  else launch_row<A, true, 0>(pl, one, jobs, count, max_tiles, rows, st);
  launch_phase<A, OC_INTT_COL_DN, 1>(pl, one, jobs, count, max_tiles[OC_INTT_COL_DN], st);
  if (pl.num_p <= 16) launch_phase<A, OC_DN | OC_ONE_ROUND, TT>(pl, one, jobs, count, max_tiles[OC_DN], st);
  else launch_phase<A, OC_DN, TT>(pl, one, jobs, count, max_tiles[OC_DN], st);
  if (rows == OC_ROWS_SUM && qjobs <= 2)  // two terms per round
    launch_phase<A, OC_ROW_Q_SUM | OC_ONE_ROUND | OC_PAIR_TERMS, 1>(pl, one, jobs, count, max_tiles[OC_ROW_Q], st);
  else if (qjobs <= (uint32_t)kSlots) launch_row<A, false, OC_ONE_ROUND>(pl, one, jobs, count, max_tiles, rows, st);
  else launch_row<A, false, 0>(pl, one, jobs, count, max_tiles, rows, st);
}

template <int A>
hipError_t oc_phases(const Plan &pl, const OcJob &one, const OcJob *jobs, uint32_t count, const uint32_t *max_tiles,
                     uint32_t tt, OcRowVariant rows, OcPart part, hipStream_t st) {
  if (tt >= 2 && ColGeom<A>::E <= 32) launch_phases_tt<A, 2>(pl, one, jobs, count, max_tiles, rows, part, st);
  else launch_phases_tt<A, 1>(pl, one, jobs, count, max_tiles, rows, part, st);
  return hipGetLastError();
}

}  // namespace ks
