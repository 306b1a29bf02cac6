// kernels.hip -- stage kernels of hybrid key switching for gfx950.
//
// Generic NTT passes over limb lists and the element-wise stages of
// Sec. III: ModUp P2 (fast basis conversion), P4 (apply key), P5 (sum over
// digits), ModDown P2 and P4.  The Max-Parallel and Digit-Centric schedules
// are sequences of these launches; the Output-Centric fused kernels live in
// oc_kernels.hip.
//
// Value conventions between kernels:
//   * inverse passes produce N*x (the N^-1 factor is folded into the next
//     basis-conversion constant), lazy in [0, 2q);
//   * forward passes produce lazy values in [0, 4q);
//   * the key accumulators hold (sum_j yhat_j * evk_j) * 2^-32 mod m,
//     canonical -- the 2^-32 of REDC is undone by the ModDown constants.
#include "kernels.h"
#include "ntt_engine.h"

namespace ks {

__device__ __forceinline__ uint32_t gidx(const DevPlan &P, uint32_t level, uint32_t t) {
  return t <= level ? t : P.num_q + (t - level - 1);
}

// ------------------------------------------------------------ generic passes
struct ColAddr {
  int W, w;
  __device__ __forceinline__ int operator()(int k) const { return k * W + w; }
};
constexpr int kRowPad = 272;  // 256 words + one pad word per 16
struct RowAddr {
  int base;
  __device__ __forceinline__ int operator()(int k) const { return base + k + (k >> 4); }
};

template <bool INV, int A, int W>
__global__ __launch_bounds__(W *SubNtt<A>::TPS) void k_col(DevPlan P, const uint32_t *src,
                                                          uint32_t *dst, LimbList L) {
  __shared__ uint32_t lds[W << A];
  constexpr int NT = W * SubNtt<A>::TPS;
  const uint32_t li = blockIdx.y, g = L.g[li];
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t rowlen = 1u << P.logb, c0 = blockIdx.x * W;
  const uint32_t *s = src + (size_t)L.src_off[li] * N + c0;
  uint32_t *d = dst + (size_t)L.dst_off[li] * N + c0;
  for (int e = threadIdx.x; e < (W << A); e += NT) lds[e] = s[(size_t)(e / W) * rowlen + (e % W)];
  __syncthreads();
  const int w = threadIdx.x % W, tig = threadIdx.x / W;
  SubNtt<A>::template run<INV>(lds, ColAddr{W, w}, tig, 1u, (INV ? P.tw_inv : P.tw_fwd) + g * N, P.mods[g].q);
  __syncthreads();
  for (int e = threadIdx.x; e < (W << A); e += NT) d[(size_t)(e / W) * rowlen + (e % W)] = lds[e];
}

template <bool INV, int RB>
__global__ __launch_bounds__(RB * 16) void k_row(DevPlan P, const uint32_t *src,
                                                 uint32_t *dst, LimbList L) {
  __shared__ uint32_t lds[RB * kRowPad];
  constexpr int NT = RB * 16;
  const uint32_t li = blockIdx.y, g = L.g[li];
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t r0 = blockIdx.x * RB;
  const uint32_t *s = src + (size_t)L.src_off[li] * N + (size_t)r0 * 256;
  uint32_t *d = dst + (size_t)L.dst_off[li] * N + (size_t)r0 * 256;
  for (int e = threadIdx.x; e < RB * 256; e += NT) lds[(e >> 8) * kRowPad + (e & 255) + ((e & 255) >> 4)] = s[e];
  __syncthreads();
  const int r = threadIdx.x >> 4, tig = threadIdx.x & 15;
  const uint32_t M = (1u << P.loga) + r0 + r;
  SubNtt<8>::template run<INV>(lds, RowAddr{r * kRowPad}, tig, M, (INV ? P.tw_inv : P.tw_fwd) + g * N,
                               P.mods[g].q);
  __syncthreads();
  for (int e = threadIdx.x; e < RB * 256; e += NT) d[e] = lds[(e >> 8) * kRowPad + (e & 255) + ((e & 255) >> 4)];
}

__global__ __launch_bounds__(256) void k_finish(DevPlan P, bool inverse, uint32_t *data, LimbList L) {
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t li = blockIdx.y, g = L.g[li], q = P.mods[g].q;
  uint32_t *d = data + (size_t)L.dst_off[li] * N;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  uint32_t v = d[i];
  if (inverse) {
    const uint32_t ninv = q - (q - 1) / (uint32_t)N;  // N * (q-1)/N = -1 mod q
    const uint32_t ninv_sh = (uint32_t)(((uint64_t)ninv << 32) / q);
    v = csub(mul_shoup(v, ninv, ninv_sh, q), q);
  } else {
    v = canon4(v, q);
  }
  d[i] = v;
}

template <bool INV, int A>
static hipError_t col_dispatch(const Plan &pl, const uint32_t *src, uint32_t *dst, const LimbList &L, uint32_t W,
                               hipStream_t st) {
  const uint32_t cols = 1u << pl.dev.logb;
  if (W == 32 || (A <= 5 && W > 8)) {
    constexpr int Wc = 32;
    dim3 grid(cols / Wc, L.count);
    KS_LAUNCH(pl, INV ? "ntt.col.inv" : "ntt.col.fwd", (k_col<INV, A, Wc>), grid, dim3(Wc * SubNtt<A>::TPS), 0, st, pl.dev, src, dst, L);
  } else if (W == 16) {
    constexpr int Wc = 16;
    dim3 grid(cols / Wc, L.count);
    KS_LAUNCH(pl, INV ? "ntt.col.inv" : "ntt.col.fwd", (k_col<INV, A, Wc>), grid, dim3(Wc * SubNtt<A>::TPS), 0, st, pl.dev, src, dst, L);
  } else {
    constexpr int Wc = 8;
    dim3 grid(cols / Wc, L.count);
    KS_LAUNCH(pl, INV ? "ntt.col.inv" : "ntt.col.fwd", (k_col<INV, A, Wc>), grid, dim3(Wc * SubNtt<A>::TPS), 0, st, pl.dev, src, dst, L);
  }
  return hipGetLastError();
}

template <bool INV>
static hipError_t col_by_a(const Plan &pl, const uint32_t *src, uint32_t *dst, const LimbList &L, hipStream_t st) {
  const uint32_t W = run_cfg(pl).col_width ? run_cfg(pl).col_width : 16;
  switch (pl.dev.loga) {
    case 4: return col_dispatch<INV, 4>(pl, src, dst, L, W, st);
    case 5: return col_dispatch<INV, 5>(pl, src, dst, L, W, st);
    case 6: return col_dispatch<INV, 6>(pl, src, dst, L, W, st);
    case 7: return col_dispatch<INV, 7>(pl, src, dst, L, W, st);
    case 8: return col_dispatch<INV, 8>(pl, src, dst, L, W, st);
    case 9: return col_dispatch<INV, 9>(pl, src, dst, L, W, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_col(const Plan &pl, bool inverse, const uint32_t *src, uint32_t *dst, const LimbList &L,
                      hipStream_t st) {
  if (!L.count) return hipSuccess;
  return inverse ? col_by_a<true>(pl, src, dst, L, st) : col_by_a<false>(pl, src, dst, L, st);
}

template <bool INV>
static hipError_t row_launch(const Plan &pl, const uint32_t *src, uint32_t *dst, const LimbList &L, hipStream_t st) {
  const uint32_t rows = 1u << pl.dev.loga;
  uint32_t RB = run_cfg(pl).row_block ? run_cfg(pl).row_block : 8;
  if (RB > rows) RB = rows;
  if (RB >= 16) {
    KS_LAUNCH(pl, INV ? "ntt.row.inv" : "ntt.row.fwd", (k_row<INV, 16>), dim3(rows / 16, L.count), dim3(256), 0, st, pl.dev, src, dst, L);
  } else if (RB >= 8) {
    KS_LAUNCH(pl, INV ? "ntt.row.inv" : "ntt.row.fwd", (k_row<INV, 8>), dim3(rows / 8, L.count), dim3(128), 0, st, pl.dev, src, dst, L);
  } else {
    KS_LAUNCH(pl, INV ? "ntt.row.inv" : "ntt.row.fwd", (k_row<INV, 4>), dim3(rows / 4, L.count), dim3(64), 0, st, pl.dev, src, dst, L);
  }
  return hipGetLastError();
}

hipError_t launch_row(const Plan &pl, bool inverse, const uint32_t *src, uint32_t *dst, const LimbList &L,
                      hipStream_t st) {
  if (!L.count) return hipSuccess;
  return inverse ? row_launch<true>(pl, src, dst, L, st) : row_launch<false>(pl, src, dst, L, st);
}

hipError_t launch_finish_ntt(const Plan &pl, bool inverse, uint32_t *data, const LimbList &L, hipStream_t st) {
  if (!L.count) return hipSuccess;
  KS_LAUNCH(pl, "ntt.finish", k_finish, dim3((pl.n + 255) / 256, L.count), dim3(256), 0, st, pl.dev, inverse, data, L);
  return hipGetLastError();
}

hipError_t launch_ntt(const Plan &pl, bool inverse, const uint32_t *src, uint32_t *dst,
                      const std::vector<uint32_t> &src_off, const std::vector<uint32_t> &dst_off,
                      const std::vector<uint32_t> &g, hipStream_t st) {
  for (size_t b = 0; b < g.size(); b += kMaxList) {
    LimbList in{}, inplace{};
    const size_t e = std::min(g.size(), b + (size_t)kMaxList);
    in.count = inplace.count = (uint32_t)(e - b);
    for (size_t c = b; c < e; c++) {
      in.src_off[c - b] = src_off[c];
      in.dst_off[c - b] = dst_off[c];
      inplace.src_off[c - b] = inplace.dst_off[c - b] = dst_off[c];
      in.g[c - b] = inplace.g[c - b] = (uint16_t)g[c];
    }
    hipError_t err;
    if (!inverse) {  // stages 1..a, then a+1..log_n
      if ((err = launch_col(pl, false, src, dst, in, st)) != hipSuccess) return err;
      if ((err = launch_row(pl, false, dst, dst, inplace, st)) != hipSuccess) return err;
    } else {         // stages log_n..a+1, then a..1
      if ((err = launch_row(pl, true, src, dst, in, st)) != hipSuccess) return err;
      if ((err = launch_col(pl, true, dst, dst, inplace, st)) != hipSuccess) return err;
    }
  }
  return hipSuccess;
}

// ------------------------------------------------------------ ModUp P2
// One thread per coefficient.  Sources: x + (xbase + i) * N, i < s; targets
// written to y + (ybase + t) * N for every tower t of D_l outside the digit.
template <int MAXA>
__global__ __launch_bounds__(256) void k_bconv_up(DevPlan P, uint32_t level, uint32_t j0, bool digit_rel,
                                                  const uint32_t *__restrict__ x, uint32_t *__restrict__ y) {
  const size_t N = (size_t)1 << P.log_n;
  const size_t z = (size_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t j = j0 + blockIdx.y;
  const uint32_t lo = j * P.alpha, hi = min(lo + P.alpha, level + 1), s = hi - lo;
  const uint32_t T = level + 1 + P.num_p;
  const size_t row0 = ((size_t)j * P.alpha + (s - 1)) * P.alpha;
  const uint32_t xbase = digit_rel ? 0 : lo;
  const size_t ybase = digit_rel ? 0 : (size_t)blockIdx.y * T;
  uint32_t xs[MAXA];
#pragma unroll
  for (int i = 0; i < MAXA; i++) {
    if ((uint32_t)i < s) {
      const uint32_t q = P.mods[lo + i].q;
      const uint2 c = P.up_pre[row0 + i];
      xs[i] = csub(mul_shoup(x[(xbase + i) * N + z], c.x, c.y, q), q);
    }
  }
  for (uint32_t t = 0; t < T; t++) {
    if (t >= lo && t < hi) continue;
    const uint32_t g = gidx(P, level, t);
    const ModQ m = P.mods[g];
    const uint32_t *cv = P.up_conv + row0 * P.ntot + g;
    uint64_t acc = 0;
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < MAXA; i++) {
      if ((uint32_t)i < s) {
        acc = mad64(xs[i], cv[(size_t)i * P.ntot], acc);
        if ((i & 15) == 15) { r = csub(r + redc64(acc, m), m.q); acc = 0; }
      }
    }
    r = csub(r + redc64(acc, m), m.q);
    y[(ybase + t) * N + z] = r;
  }
}

hipError_t launch_bconv_up(const Plan &pl, uint32_t level, uint32_t j0, uint32_t nd, bool digit_rel,
                                const uint32_t *x, uint32_t *y, hipStream_t st) {
  dim3 grid((pl.n + 255) / 256, nd);
  if (pl.alpha <= 4)
    KS_LAUNCH(pl, "bconv.up", (k_bconv_up<4>), grid, dim3(256), 0, st, pl.dev, level, j0, digit_rel, x, y);
  else if (pl.alpha <= 8)
    KS_LAUNCH(pl, "bconv.up", (k_bconv_up<8>), grid, dim3(256), 0, st, pl.dev, level, j0, digit_rel, x, y);
  else if (pl.alpha <= 16)
    KS_LAUNCH(pl, "bconv.up", (k_bconv_up<16>), grid, dim3(256), 0, st, pl.dev, level, j0, digit_rel, x, y);
  else if (pl.alpha <= 32)
    KS_LAUNCH(pl, "bconv.up", (k_bconv_up<32>), grid, dim3(256), 0, st, pl.dev, level, j0, digit_rel, x, y);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ------------------------------------------------------------ ModUp P4 / P5
__device__ __forceinline__ uint32_t yhat_at(const DevPlan &P, uint32_t level, uint32_t j, uint32_t t,
                                            const uint32_t *d, const uint32_t *yj, size_t N, size_t c, uint32_t q) {
  const uint32_t lo = j * P.alpha, hi = min(lo + P.alpha, level + 1);
  if (t >= lo && t < hi) return d[(size_t)t * N + c];  // own digit: bypass (Sec. IV-C)
  return canon4(yj[(size_t)t * N + c], q);
}

// grid (N/256, T, ndig*2)
__global__ __launch_bounds__(256) void k_keymul(DevPlan P, uint32_t level, const uint32_t *__restrict__ d,
                                                const uint32_t *__restrict__ y, const uint32_t *__restrict__ evk,
                                                uint32_t *__restrict__ z) {
  const size_t N = (size_t)1 << P.log_n;
  const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t t = blockIdx.y, j = blockIdx.z >> 1, s = blockIdx.z & 1;
  const uint32_t T = level + 1 + P.num_p, g = gidx(P, level, t);
  const ModQ m = P.mods[g];
  const uint32_t yv = yhat_at(P, level, j, t, d, y + (size_t)j * T * N, N, c, m.q);
  const uint32_t e = evk[(((size_t)j * 2 + s) * P.ntot + g) * N + c];
  z[(((size_t)j * 2 + s) * T + t) * N + c] = redc64((uint64_t)yv * e, m);
}

hipError_t launch_keymul(const Plan &pl, uint32_t level, const uint32_t *d, const uint32_t *y, const uint32_t *evk,
                         uint32_t *z, hipStream_t st) {
  const uint32_t T = level + 1 + pl.num_p, D = num_digits(pl, level);
  KS_LAUNCH(pl, "keymul", k_keymul, dim3((pl.n + 255) / 256, T, D * 2), dim3(256), 0, st, pl.dev, level, d, y, evk, z);
  return hipGetLastError();
}

// grid (N/256, T, 2)
__global__ __launch_bounds__(256) void k_reduce_digits(DevPlan P, uint32_t level, uint32_t ndig,
                                                       const uint32_t *__restrict__ z, uint32_t *__restrict__ acc) {
  const size_t N = (size_t)1 << P.log_n;
  const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t t = blockIdx.y, s = blockIdx.z;
  const uint32_t T = level + 1 + P.num_p, q = P.mods[gidx(P, level, t)].q;
  uint32_t r = 0;
  for (uint32_t j = 0; j < ndig; j++) r = csub(r + z[(((size_t)j * 2 + s) * T + t) * N + c], q);
  acc[((size_t)s * T + t) * N + c] = r;
}

hipError_t launch_reduce_digits(const Plan &pl, uint32_t level, const uint32_t *z, uint32_t *acc, hipStream_t st) {
  const uint32_t T = level + 1 + pl.num_p, D = num_digits(pl, level);
  KS_LAUNCH(pl, "reduce_digits", k_reduce_digits, dim3((pl.n + 255) / 256, T, 2), dim3(256), 0, st, pl.dev, level, D, z, acc);
  return hipGetLastError();
}

// grid (N/256, T, 2); yj is digit j's [T][N] block.
__global__ __launch_bounds__(256) void k_keymac_digit(DevPlan P, uint32_t level, uint32_t j,
                                                      const uint32_t *__restrict__ d, const uint32_t *__restrict__ yj,
                                                      const uint32_t *__restrict__ evk, uint32_t *__restrict__ acc) {
  const size_t N = (size_t)1 << P.log_n;
  const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t t = blockIdx.y, s = blockIdx.z;
  const uint32_t T = level + 1 + P.num_p, g = gidx(P, level, t);
  const ModQ m = P.mods[g];
  const uint32_t yv = yhat_at(P, level, j, t, d, yj, N, c, m.q);
  const uint32_t e = evk[(((size_t)j * 2 + s) * P.ntot + g) * N + c];
  uint32_t r = redc64((uint64_t)yv * e, m);
  uint32_t *a = acc + ((size_t)s * T + t) * N + c;
  if (j) r = csub(r + *a, m.q);
  *a = r;
}

hipError_t launch_keymac_digit(const Plan &pl, uint32_t level, uint32_t j, const uint32_t *d, const uint32_t *yj,
                               const uint32_t *evk, uint32_t *acc, hipStream_t st) {
  const uint32_t T = level + 1 + pl.num_p;
  KS_LAUNCH(pl, "keymac_digit", k_keymac_digit, dim3((pl.n + 255) / 256, T, 2), dim3(256), 0, st, pl.dev, level, j, d, yj, evk,
                     acc);
  return hipGetLastError();
}

// ------------------------------------------------------------ ModDown P2 / P4
// grid (N/256, 2)
template <int MAXK>
__global__ __launch_bounds__(256) void k_bconv_down(DevPlan P, uint32_t level, const uint32_t *__restrict__ xp,
                                                    uint32_t *__restrict__ w) {
  const size_t N = (size_t)1 << P.log_n;
  const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t s = blockIdx.y, K = P.num_p, l1 = level + 1;
  uint32_t xs[MAXK];
#pragma unroll
  for (int k = 0; k < MAXK; k++) {
    if ((uint32_t)k < K) {
      const uint32_t p = P.mods[P.num_q + k].q;
      const uint2 cst = P.dn_pre[k];
      xs[k] = csub(mul_shoup(xp[((size_t)s * K + k) * N + c], cst.x, cst.y, p), p);
    }
  }
  for (uint32_t i = 0; i < l1; i++) {
    const ModQ m = P.mods[i];
    uint64_t acc = 0;
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < MAXK; k++) {
      if ((uint32_t)k < K) {
        acc = mad64(xs[k], P.dn_conv[(size_t)k * P.num_q + i], acc);
        if ((k & 15) == 15) { r = csub(r + redc64(acc, m), m.q); acc = 0; }
      }
    }
    w[((size_t)s * l1 + i) * N + c] = csub(r + redc64(acc, m), m.q);
  }
}

hipError_t launch_bconv_down(const Plan &pl, uint32_t level, const uint32_t *xp, uint32_t *w, hipStream_t st) {
  dim3 grid((pl.n + 255) / 256, 2);
  if (pl.num_p <= 4)
    KS_LAUNCH(pl, "bconv.down", (k_bconv_down<4>), grid, dim3(256), 0, st, pl.dev, level, xp, w);
  else if (pl.num_p <= 8)
    KS_LAUNCH(pl, "bconv.down", (k_bconv_down<8>), grid, dim3(256), 0, st, pl.dev, level, xp, w);
  else if (pl.num_p <= 16)
    KS_LAUNCH(pl, "bconv.down", (k_bconv_down<16>), grid, dim3(256), 0, st, pl.dev, level, xp, w);
  else if (pl.num_p <= 32)
    KS_LAUNCH(pl, "bconv.down", (k_bconv_down<32>), grid, dim3(256), 0, st, pl.dev, level, xp, w);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// grid (N/256, l+1, 2); acc is [2][T][N], what and out are [2][l+1][N].
__global__ __launch_bounds__(256) void k_moddown_final(DevPlan P, uint32_t level, const uint32_t *__restrict__ acc,
                                                       const uint32_t *__restrict__ what, uint32_t *__restrict__ out) {
  const size_t N = (size_t)1 << P.log_n;
  const size_t c = (size_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t i = blockIdx.y, s = blockIdx.z, l1 = level + 1, T = l1 + P.num_p;
  const uint32_t q = P.mods[i].q;
  const uint2 f = P.dn_fin[i];
  const uint32_t a = acc[((size_t)s * T + i) * N + c];
  const uint32_t wv = canon4(what[((size_t)s * l1 + i) * N + c], q);
  out[((size_t)s * l1 + i) * N + c] = csub(mul_shoup(a + q - wv, f.x, f.y, q), q);
}

hipError_t launch_moddown_final(const Plan &pl, uint32_t level, const uint32_t *acc, const uint32_t *what,
                                uint32_t *out, hipStream_t st) {
  KS_LAUNCH(pl, "moddown_final", k_moddown_final, dim3((pl.n + 255) / 256, level + 1, 2), dim3(256), 0, st, pl.dev, level, acc,
                     what, out);
  return hipGetLastError();
}

// ------------------------------------------------------------ compressed keys
// grid (N/1024, ntot, dnum): the a half of digit j, row g (evk order), four
// consecutive words per thread, written into a full-layout key.
__global__ __launch_bounds__(256) void k_expand_a(DevPlan P, uint64_t seed, uint32_t *__restrict__ evk) {
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t g = blockIdx.y, j = blockIdx.z;
  const uint32_t k = (blockIdx.x * 256 + threadIdx.x) * 4;
  const ModQ m = P.mods[g];
  uint32_t a[4];
  seeded_a4(a, seed, (uint32_t)(((size_t)j * P.ntot + g) * N + k), m);
  stg4(evk + (((size_t)2 * j + 1) * P.ntot + g) * N + k, make_uint4(a[0], a[1], a[2], a[3]));
}

hipError_t launch_expand_a(const Plan &pl, uint64_t seed, uint32_t *evk, hipStream_t st) {
  KS_LAUNCH(pl, "expand_a", k_expand_a, dim3(pl.n / 1024, pl.ntot, pl.dnum), dim3(256), 0, st, pl.dev, seed, evk);
  return hipGetLastError();
}

// ------------------------------------------------------------ automorphism, tensor
// grid (N/256, count)
__global__ __launch_bounds__(256) void k_automorphism(DevPlan P, uint32_t galois, const uint32_t *__restrict__ in,
                                                      uint32_t *__restrict__ out) {
  const size_t N = (size_t)1 << P.log_n, c = blockIdx.y;
  const uint32_t j = blockIdx.x * 256 + threadIdx.x;
  out[c * N + j] = in[c * N + galois_perm(j, galois, P.log_n)];
}

hipError_t launch_automorphism(const Plan &pl, uint32_t galois, uint32_t count, const uint32_t *in, uint32_t *out,
                               hipStream_t st) {
  if (!count) return hipSuccess;
  KS_LAUNCH(pl, "automorphism", k_automorphism, dim3(pl.n / 256, count), dim3(256), 0, st, pl.dev, galois, in, out);
  return hipGetLastError();
}

// grid (N/256, l+1); a b mod q as REDC(a b) = a b 2^-32, then times 2^32
// mod q with a Shoup product
__global__ __launch_bounds__(256) void k_tensor(DevPlan P, uint32_t level, const uint32_t *__restrict__ a0,
                                                const uint32_t *__restrict__ a1, const uint32_t *__restrict__ b0,
                                                const uint32_t *__restrict__ b1, uint32_t *__restrict__ d) {
  const size_t N = (size_t)1 << P.log_n, l1 = level + 1;
  const uint32_t i = blockIdx.y;
  const size_t w = i * N + blockIdx.x * 256 + threadIdx.x;
  const ModQ m = P.mods[i];
  const uint32_t r32 = (0u - m.q) % m.q;  // 2^32 mod q
  const uint32_t r32p = shoup_companion(r32, m.q, P.qrecip[i]);
  const uint32_t x0 = a0[w], x1 = a1[w], y0 = b0[w], y1 = b1[w];
  auto fin = [&](uint64_t t) { return csub(mul_shoup(redc64(t, m), r32, r32p, m.q), m.q); };
  d[w] = fin((uint64_t)x0 * y0);
  d[l1 * N + w] = fin((uint64_t)x0 * y1 + (uint64_t)x1 * y0);
  d[2 * l1 * N + w] = fin((uint64_t)x1 * y1);
}

hipError_t launch_tensor(const Plan &pl, uint32_t level, const uint32_t *a0, const uint32_t *a1, const uint32_t *b0,
                         const uint32_t *b1, uint32_t *d, hipStream_t st) {
  KS_LAUNCH(pl, "tensor", k_tensor, dim3(pl.n / 256, level + 1), dim3(256), 0, st, pl.dev, level, a0, a1, b0, b1, d);
  return hipGetLastError();
}

// ------------------------------------------------------------ double hoisting
// exact a b mod q: REDC(a b) = a b 2^-32, then a Shoup product by 2^32 mod q
__device__ __forceinline__ uint32_t mulmod_exact(uint32_t a, uint32_t b, const ModQ &m, uint32_t r32,
                                                 uint32_t r32p) {
  return csub(mul_shoup(redc64((uint64_t)a * b, m), r32, r32p, m.q), m.q);
}

// grid (N/256, T): both polynomials per thread, so each gathered digit word
// is read once for the two key halves
__global__ __launch_bounds__(256) void k_rotsum_keymul(DevPlan P, uint32_t level, const uint32_t *__restrict__ d,
                                                       const uint32_t *__restrict__ y,
                                                       const RotTerm *__restrict__ terms, uint32_t nterm,
                                                       uint32_t *__restrict__ acc) {
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t c = blockIdx.x * 256 + threadIdx.x, t = blockIdx.y;
  const uint32_t L1 = level + 1, T = L1 + P.num_p, g = gidx(P, level, t), ndig = (L1 + P.alpha - 1) / P.alpha;
  const ModQ m = P.mods[g];
  const uint32_t r32 = (0u - m.q) % m.q;
  const uint32_t r32p = shoup_companion(r32, m.q, P.qrecip[g]);
  const size_t half = (size_t)P.ntot * N;  // from a key row of half 0 to the same row of half 1
  uint32_t total0 = 0, total1 = 0;
  for (uint32_t r = 0; r < nterm; r++) {
    const RotTerm rt = terms[r];
    const size_t src = galois_perm(c, rt.galois, P.log_n);
    uint64_t a0 = 0, a1 = 0;  // at most 16 digits: no overflow
    for (uint32_t j = 0; j < ndig; j++) {
      const uint32_t yv = yhat_at(P, level, j, t, d, y + (size_t)j * T * N, N, src, m.q);
      const uint32_t *e = rt.evk + ((size_t)j * 2 * P.ntot + g) * N + c;
      a0 += (uint64_t)yv * e[0];
      a1 += (uint64_t)yv * e[half];
    }
    uint32_t v0 = redc64(a0, m), v1 = redc64(a1, m);
    if (rt.diag) {
      const uint32_t pv = rt.diag[(size_t)g * N + c];
      v0 = mulmod_exact(v0, pv, m, r32, r32p);
      v1 = mulmod_exact(v1, pv, m, r32, r32p);
    }
    total0 = csub(total0 + v0, m.q);
    total1 = csub(total1 + v1, m.q);
  }
  acc[(size_t)t * N + c] = total0;
  acc[((size_t)T + t) * N + c] = total1;
}

hipError_t launch_rotsum_keymul(const Plan &pl, uint32_t level, const uint32_t *d, const uint32_t *y,
                                const RotTerm *terms, uint32_t nterm, uint32_t *acc, hipStream_t st) {
  const uint32_t T = level + 1 + pl.num_p;
  KS_LAUNCH(pl, "rotsum_keymul", k_rotsum_keymul, dim3(pl.n / 256, T), dim3(256), 0, st, pl.dev, level, d, y, terms,
            nterm, acc);
  return hipGetLastError();
}

// grid (N/256, l+1); out[0][i] is canonical, so is the result
__global__ __launch_bounds__(256) void k_rotsum_c0(DevPlan P, const uint32_t *__restrict__ c0,
                                                   const RotTerm *__restrict__ terms, uint32_t nterm,
                                                   uint32_t *__restrict__ out) {
  const size_t N = (size_t)1 << P.log_n;
  const uint32_t c = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y;
  const ModQ m = P.mods[i];
  const uint32_t r32 = (0u - m.q) % m.q;
  const uint32_t r32p = shoup_companion(r32, m.q, P.qrecip[i]);
  uint32_t v = out[(size_t)i * N + c];
  for (uint32_t r = 0; r < nterm; r++) {
    const RotTerm rt = terms[r];
    uint32_t x = c0[(size_t)i * N + galois_perm(c, rt.galois, P.log_n)];
    if (rt.diag) x = mulmod_exact(x, rt.diag[(size_t)i * N + c], m, r32, r32p);
    v = csub(v + x, m.q);
  }
  out[(size_t)i * N + c] = v;
}

hipError_t launch_rotsum_c0(const Plan &pl, uint32_t level, const uint32_t *c0, const RotTerm *terms, uint32_t nterm,
                            uint32_t *out, hipStream_t st) {
  KS_LAUNCH(pl, "rotsum_c0", k_rotsum_c0, dim3(pl.n / 256, level + 1), dim3(256), 0, st, pl.dev, c0, terms, nterm, out);
  return hipGetLastError();
}

// ------------------------------------------------------------ OC entry
uint32_t oc_effective_tt(uint32_t loga, uint32_t want, uint32_t l1) {
  // Two targets per tile keep 2 x 16 accumulators per thread.  Columns of 32
  // elements per thread: at loga 9 two targets (169 VGPRs, 2 waves per SIMD)
  // halve the source re-reads, which pays from 17 towers up (l1 = the
  // largest l+1 of the launch); below, the lower occupancy costs more.  loga
  // 5 stays at one.
  if (want < 2 || loga == 5) return 1;
  return (loga != 9 || l1 >= 17) ? 2 : 1;
}

static uint32_t col_blocks(uint32_t loga) {
  switch (loga) {
    case 4: case 5: return 1;
    case 6: case 7: return 8;
    default: return 16;
  }
}

void oc_tiles_host(const Plan &pl, uint32_t level, uint32_t tt, uint32_t *tiles) {
  oc_phase_tiles(pl.dev.loga, col_blocks(pl.dev.loga), pl.alpha, pl.num_p, level, tt, tt, tiles);
}

void oc_tiles_params(uint32_t log_n, uint32_t alpha, uint32_t K, uint32_t level, uint32_t tt, uint32_t *tiles) {
  const uint32_t loga = log_n - kRowLog;
  oc_phase_tiles(loga, col_blocks(loga), alpha, K, level, tt, tt, tiles);
}

hipError_t launch_oc_phases(const Plan &pl, const OcJob &one, const OcJob *jobs, uint32_t count,
                            const uint32_t *max_tiles, uint32_t tt, OcRowVariant rows, OcPart part,
                            hipStream_t st) {
  switch (pl.dev.loga) {
    case 4: return oc_phases<4>(pl, one, jobs, count, max_tiles, tt, rows, part, st);
    case 5: return oc_phases<5>(pl, one, jobs, count, max_tiles, tt, rows, part, st);
    case 6: return oc_phases<6>(pl, one, jobs, count, max_tiles, tt, rows, part, st);
    case 7: return oc_phases<7>(pl, one, jobs, count, max_tiles, tt, rows, part, st);
    case 8: return oc_phases<8>(pl, one, jobs, count, max_tiles, tt, rows, part, st);
    case 9: return oc_phases<9>(pl, one, jobs, count, max_tiles, tt, rows, part, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_oc_persistent(const Plan &pl, const OcJob *jobs, const OcSeg *segs, uint32_t nsegs,
                                uint32_t total, uint32_t count, uint32_t *ctl, uint32_t spin_limit, hipStream_t st) {
  switch (pl.dev.loga) {
    case 4: return oc_persistent<4>(pl, jobs, segs, nsegs, total, count, ctl, spin_limit, st);
    case 5: return oc_persistent<5>(pl, jobs, segs, nsegs, total, count, ctl, spin_limit, st);
    case 6: return oc_persistent<6>(pl, jobs, segs, nsegs, total, count, ctl, spin_limit, st);
    case 7: return oc_persistent<7>(pl, jobs, segs, nsegs, total, count, ctl, spin_limit, st);
    case 8: return oc_persistent<8>(pl, jobs, segs, nsegs, total, count, ctl, spin_limit, st);
    case 9: return oc_persistent<9>(pl, jobs, segs, nsegs, total, count, ctl, spin_limit, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace ks
