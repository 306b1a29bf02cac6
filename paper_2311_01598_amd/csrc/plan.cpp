// plan.cpp -- moduli, roots of unity and precomputed tables of a plan.
//
// Derivations used here (all exact integer arithmetic on the host):
//  * moduli and psi: numtheory.cpp (deterministic Miller-Rabin; psi from a
//    generator of Z_q^*, the smallest of the primitive 2N-th roots);
//  * twiddles: psi^brv(i) and psi^-brv(i) for i < N with Shoup companions;
//  * basis-conversion constants of ModUp P2 and ModDown P2 (Sec. III-B/C),
//    with N^-1 of the preceding inverse NTT folded into the per-source
//    constant and the factors of 2^32 that REDC removes folded in where the
//    reduction happens (see DevPlan in plan.h).
#include "plan.h"

#include <algorithm>
#include <cstring>

namespace ks {

static inline uint64_t mulm(uint64_t a, uint64_t b, uint64_t m) {
  return (uint64_t)((unsigned __int128)a * b % m);
}

static uint32_t inv_mod(uint32_t a, uint32_t q) {  // extended Euclid
  int64_t t = 0, nt = 1, r = q, nr = a % q;
  while (nr) {
    int64_t k = r / nr;
    int64_t tmp = t - k * nt; t = nt; nt = tmp;
    tmp = r - k * nr; r = nr; nr = tmp;
  }
  if (t < 0) t += q;
  return (uint32_t)t;
}

static inline uint32_t shoup_of(uint32_t w, uint32_t q) { return (uint32_t)(((uint64_t)w << 32) / q); }
static inline uint2 shoup_pair(uint32_t w, uint32_t q) { return make_uint2(w, shoup_of(w, q)); }
static inline uint32_t mont_of(uint32_t w, uint32_t q) { return (uint32_t)(((uint64_t)w << 32) % q); }
static inline uint32_t bitrev(uint32_t x, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

template <class T>
static ks_status_t upload(Plan *pl, const std::vector<T> &h, const T **dst) {
  void *p = nullptr;
  size_t bytes = std::max<size_t>(h.size() * sizeof(T), 256);
  if (hipMalloc(&p, bytes) != hipSuccess) return KS_ERR_NOMEM;
  pl->allocs.push_back(p);
  if (!h.empty() && hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return KS_ERR_DEVICE;
  *dst = (const T *)p;
  return KS_OK;
}

ks_status_t plan_build(const ks_params_t *p, Plan *pl) {
  pl->log_n = p->log_n;
  pl->n = 1u << p->log_n;
  pl->num_q = p->num_q;
  pl->dnum = p->dnum;
  pl->alpha = (p->num_q + p->dnum - 1) / p->dnum;
  pl->num_p = p->num_p ? p->num_p : pl->alpha;
  pl->ntot = pl->num_q + pl->num_p;
  const uint32_t n = pl->n, ntot = pl->ntot, L1 = pl->num_q, K = pl->num_p, A = pl->alpha;

  pl->mod.resize(ntot);
  if (p->moduli) {
    std::copy(p->moduli, p->moduli + ntot, pl->mod.begin());
  } else {
    std::vector<uint32_t> pr(ntot);
    if (ntt_primes(p->log_n, ntot, pr.data()) != 0) return KS_ERR_UNSUPPORTED;
    for (uint32_t i = 0; i < L1; i++) pl->mod[i] = pr[K + i];
    for (uint32_t k = 0; k < K; k++) pl->mod[L1 + k] = pr[k];
  }
  pl->psi.resize(ntot);
  for (uint32_t g = 0; g < ntot; g++) {
    pl->psi[g] = min_root_2n(pl->mod[g], p->log_n);
    if (!pl->psi[g]) return KS_ERR_INVALID_ARG;
  }
  if (hipGetDevice(&pl->device) != hipSuccess) return KS_ERR_DEVICE;

  // --- twiddles
  std::vector<uint2> twf((size_t)ntot * n), twi((size_t)ntot * n);
  std::vector<uint32_t> twf32((size_t)ntot * n), twi32((size_t)ntot * n);
  std::vector<double> qrecip(ntot);
  std::vector<uint32_t> pw(n), pwi(n);
  for (uint32_t g = 0; g < ntot; g++) {
    const uint32_t q = pl->mod[g], s = pl->psi[g], si = inv_mod(s, q);
    pw[0] = pwi[0] = 1;
    for (uint32_t i = 1; i < n; i++) {
      pw[i] = (uint32_t)mulm(pw[i - 1], s, q);
      pwi[i] = (uint32_t)mulm(pwi[i - 1], si, q);
    }
    for (uint32_t i = 0; i < n; i++) {
      uint32_t r = bitrev(i, p->log_n);
      // forward entries carry -w mod 2^32 (see bfly_ct)
      twf[(size_t)g * n + i] = make_uint2(0u - pw[r], shoup_of(pw[r], q));
      twi[(size_t)g * n + i] = shoup_pair(pwi[r], q);
      twf32[(size_t)g * n + i] = pw[r];
      twi32[(size_t)g * n + i] = pwi[r];
    }
    qrecip[g] = 4294967296.0 / (double)q;
  }
  std::vector<ModQ> mq(ntot);
  for (uint32_t g = 0; g < ntot; g++) {
    const uint32_t q = pl->mod[g];
    uint32_t inv = 1;  // q^-1 mod 2^32 by Newton iteration
    for (int i = 0; i < 5; i++) inv *= 2u - q * inv;
    mq[g] = ModQ{q, (uint32_t)(0u - inv), (uint32_t)((1ull << 32) / q), 0};
  }

  // --- ModUp basis conversion (per digit j and digit size s)
  std::vector<uint2> up_pre((size_t)pl->dnum * A * A, make_uint2(0, 0));
  std::vector<uint32_t> up_conv((size_t)pl->dnum * A * A * ntot, 0);
  for (uint32_t j = 0; j < pl->dnum; j++) {
    const uint32_t lo = j * A;
    if (lo >= L1) break;
    const uint32_t smax = std::min(A, L1 - lo);
    for (uint32_t s = 1; s <= smax; s++) {
      for (uint32_t i = 0; i < s; i++) {
        const uint32_t qi = pl->mod[lo + i];
        uint64_t hat = 1;  // qhat_i mod q_i
        for (uint32_t i2 = 0; i2 < s; i2++)
          if (i2 != i) hat = mulm(hat, pl->mod[lo + i2] % qi, qi);
        uint32_t c = (uint32_t)mulm(inv_mod((uint32_t)hat, qi), inv_mod(n % qi, qi), qi);
        const size_t row = ((size_t)j * A + (s - 1)) * A + i;
        up_pre[row] = shoup_pair(c, qi);
        for (uint32_t g = 0; g < ntot; g++) {
          const uint32_t m = pl->mod[g];
          uint64_t h = 1;
          for (uint32_t i2 = 0; i2 < s; i2++)
            if (i2 != i) h = mulm(h, pl->mod[lo + i2] % m, m);
          up_conv[row * ntot + g] = mont_of((uint32_t)h, m);
        }
      }
    }
  }
  // --- ModDown
  std::vector<uint2> dn_pre(K), dn_fin(L1);
  std::vector<uint32_t> dn_conv((size_t)K * L1);
  for (uint32_t k = 0; k < K; k++) {
    const uint32_t pk = pl->mod[L1 + k];
    uint64_t hat = 1;
    for (uint32_t k2 = 0; k2 < K; k2++)
      if (k2 != k) hat = mulm(hat, pl->mod[L1 + k2] % pk, pk);
    uint32_t c = (uint32_t)mulm(inv_mod((uint32_t)hat, pk), inv_mod(n % pk, pk), pk);
    dn_pre[k] = shoup_pair(mont_of(c, pk), pk);
    for (uint32_t i = 0; i < L1; i++) {
      const uint32_t qi = pl->mod[i];
      uint64_t h = 1;
      for (uint32_t k2 = 0; k2 < K; k2++)
        if (k2 != k) h = mulm(h, pl->mod[L1 + k2] % qi, qi);
      dn_conv[(size_t)k * L1 + i] = (uint32_t)h;
    }
  }
  for (uint32_t i = 0; i < L1; i++) {
    const uint32_t qi = pl->mod[i];
    uint64_t P = 1;
    for (uint32_t k = 0; k < K; k++) P = mulm(P, pl->mod[L1 + k] % qi, qi);
    dn_fin[i] = shoup_pair(mont_of(inv_mod((uint32_t)P, qi), qi), qi);
  }

  DevPlan &d = pl->dev;
  ks_status_t st;
  if ((st = upload(pl, twf, &d.tw_fwd)) || (st = upload(pl, twi, &d.tw_inv)) || (st = upload(pl, mq, &d.mods)) ||
      (st = upload(pl, up_pre, &d.up_pre)) || (st = upload(pl, up_conv, &d.up_conv)) ||
      (st = upload(pl, dn_pre, &d.dn_pre)) || (st = upload(pl, dn_conv, &d.dn_conv)) ||
      (st = upload(pl, dn_fin, &d.dn_fin)) || (st = upload(pl, twf32, &d.tw_fwd32)) ||
      (st = upload(pl, twi32, &d.tw_inv32)) || (st = upload(pl, qrecip, &d.qrecip)))
    return st;
  d.log_n = p->log_n;
  d.logb = kRowLog;
  d.loga = p->log_n - kRowLog;
  d.num_q = L1;
  d.num_p = K;
  d.dnum = pl->dnum;
  d.alpha = A;
  d.ntot = ntot;
  return KS_OK;
}

void plan_free(Plan *pl) {
  for (void *p : pl->allocs) (void)hipFree(p);
  pl->allocs.clear();
  std::lock_guard<std::mutex> g(pl->trace.mu);
  for (auto &m : pl->trace.marks) {
    (void)hipEventDestroy(m.start);
    (void)hipEventDestroy(m.stop);
  }
  for (hipEvent_t e : pl->trace.pool) (void)hipEventDestroy(e);
  pl->trace.marks.clear();
  pl->trace.pool.clear();
  std::lock_guard<std::mutex> g2(pl->staging.mu);
  for (auto &s : pl->staging.slots) {
    (void)hipEventSynchronize(s.done);
    (void)hipEventDestroy(s.done);
    (void)hipHostFree(s.host);
  }
  pl->staging.slots.clear();
  std::lock_guard<std::mutex> g3(pl->fork.mu);
  if (pl->fork.side) {
    (void)hipStreamSynchronize(pl->fork.side);
    (void)hipStreamDestroy(pl->fork.side);
  }
  if (pl->fork.fork) (void)hipEventDestroy(pl->fork.fork);
  if (pl->fork.join) (void)hipEventDestroy(pl->fork.join);
  pl->fork.side = nullptr;
  pl->fork.fork = pl->fork.join = nullptr;
}

hipError_t fork_get(const Plan &pl, Fork **f) {
  Fork &k = pl.fork;
  if (!k.side) {
    const hipError_t e = hipStreamCreateWithFlags(&k.side, hipStreamNonBlocking);
    if (e != hipSuccess) {
      k.side = nullptr;
      return e;
    }
  }
  if (!k.fork && hipEventCreateWithFlags(&k.fork, hipEventDisableTiming) != hipSuccess) return hipErrorUnknown;
  if (!k.join && hipEventCreateWithFlags(&k.join, hipEventDisableTiming) != hipSuccess) return hipErrorUnknown;
  *f = &k;
  return hipSuccess;
}

hipError_t upload_async(const Plan &pl, void *dst, const void *src, size_t bytes, hipStream_t st) {
  Staging &sg = pl.staging;
  std::lock_guard<std::mutex> g(sg.mu);
  StagingSlot *slot = nullptr;
  for (auto &s : sg.slots)
    if (s.bytes >= bytes && hipEventQuery(s.done) == hipSuccess) {
      slot = &s;
      break;
    }
  if (!slot) {
    StagingSlot s;
    s.bytes = std::max<size_t>(bytes, 64 << 10);
    hipError_t e = hipHostMalloc(&s.host, s.bytes, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess) {
      (void)hipHostFree(s.host);
      return e;
    }
    sg.slots.push_back(s);
    slot = &sg.slots.back();
  }
  std::memcpy(slot->host, src, bytes);
  hipError_t e = hipMemcpyAsync(dst, slot->host, bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return hipEventRecord(slot->done, st);
}

namespace {
thread_local const ks_config_t *t_run_cfg = nullptr;
}

const ks_config_t &run_cfg(const Plan &pl) { return t_run_cfg ? *t_run_cfg : pl.cfg; }

RunCfgScope::RunCfgScope(const ks_config_t &c) : cfg_(c), prev_(t_run_cfg) { t_run_cfg = &cfg_; }
RunCfgScope::~RunCfgScope() { t_run_cfg = prev_; }

bool trace_pair(const Plan &pl, const char *stage, hipEvent_t *start, hipEvent_t *stop) {
  Trace &t = pl.trace;
  if (!t.on) return false;
  std::lock_guard<std::mutex> g(t.mu);
  if (!t.on) return false;
  hipEvent_t ev[2];
  for (int i = 0; i < 2; i++) {
    if (!t.pool.empty()) {
      ev[i] = t.pool.back();
      t.pool.pop_back();
    } else if (hipEventCreate(&ev[i]) != hipSuccess) {
      if (i) t.pool.push_back(ev[0]);
      return false;
    }
  }
  t.marks.push_back(TraceMark{stage, ev[0], ev[1]});
  *start = ev[0];
  *stop = ev[1];
  return true;
}

}  // namespace ks
