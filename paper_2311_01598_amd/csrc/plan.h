// plan.h -- host-side plan of a key-switching parameter set and the device
// view of its precomputed tables.
//
// Tower numbering.  Global index g in [0, num_q + num_p): g <= L is q_g,
// g = L+1+k is p_k -- the limb order of the evaluation key.  At level l the
// extended basis D_l has T = l+1+K towers; tower t < l+1 is q_t (g = t) and
// tower t >= l+1 is p_{t-l-1} (g = L+1+t-l-1).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "../../include/ks.h"
#include "modarith.h"
#include "numtheory.h"

namespace ks {

constexpr uint32_t kMaxTowers = 128;  // num_q + num_p
constexpr uint32_t kRowLog = 8;       // NTT row length 2^8 (second pass)

// Device view of a plan: plain pointers and scalars, passed by value.
struct DevPlan {
  const uint2 *tw_fwd;   // [ntot][N] (-psi^brv(i) mod 2^32, Shoup companion of psi^brv(i))
  const uint2 *tw_inv;   // [ntot][N] (psi^-brv(i), Shoup companion)
  const ModQ *mods;      // [ntot]
  // The same tables as plain residues (4 bytes per entry: psi^brv(i) and
  // psi^-brv(i)) for kernels that stage twiddles through LDS and derive the
  // Shoup companions there, with qrecip[g] = 2^32 / m_g in double precision.
  const uint32_t *tw_fwd32, *tw_inv32;
  const double *qrecip;
  // ModUp basis conversion, digit j holding s towers (the last digit of a
  // lower level may be partial):
  //   up_pre [(j*alpha + s-1)*alpha + i]          Shoup pair of N^-1 [qhat_i^-1]_{q_i}
  //   up_conv[((j*alpha + s-1)*alpha + i)*ntot + g] [qhat_i]_{m_g} * 2^32 mod m_g
  const uint2 *up_pre;
  const uint32_t *up_conv;
  // ModDown: dn_pre[k]  Shoup pair of N^-1 2^32 [phat_k^-1]_{p_k}
  //          dn_conv[k*num_q + i]  [phat_k]_{q_i}
  //          dn_fin[i]  Shoup pair of 2^32 [P^-1]_{q_i}
  const uint2 *dn_pre;
  const uint32_t *dn_conv;
  const uint2 *dn_fin;
  uint32_t log_n, loga, logb;  // N = 2^log_n = 2^loga columns-length x 2^logb row-length
  uint32_t num_q, num_p, dnum, alpha, ntot;
};

// Optional per-kernel event trace (tools and the benchmark): while `on`,
// every kernel the plan enqueues is launched with hipExtLaunchKernelGGL and
// a start/stop event pair attached to its own dispatch (no extra packets on
// the stream), tagged with the kernel's stage name.
struct TraceMark {
  const char *stage;
  hipEvent_t start, stop;
};
struct Trace {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<TraceMark> marks;
};

// Pinned host buffers for asynchronous uploads (batch job tables): a slot
// is reused only after the event recorded behind its copy has completed,
// so the source stays valid for as long as the copy may read it.
struct StagingSlot {
  void *host = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
};
struct Staging {
  std::mutex mu;
  std::vector<StagingSlot> slots;
};

// A second stream (default priority) for work that may overlap the caller's
// stream inside one call: `fork` is recorded on the caller's stream and
// waited for by the side stream, `join` the other way round.  Created on
// first use; `mu` is held while a call enqueues its fork ... join sequence,
// so calls from several threads or streams stay correctly ordered.
struct Fork {
  std::mutex mu;
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

// One autotuner result: the configuration for calls of `count` key
// switches whose largest level is `level` (used when the plan's schedule is
// KS_SCHED_AUTO).
struct TunedEntry {
  uint32_t level, count;
  ks_config_t cfg;
};

struct Plan {
  uint32_t log_n = 0, n = 0, num_q = 0, num_p = 0, dnum = 0, alpha = 0, ntot = 0;
  int device = -1;
  std::vector<uint32_t> mod;  // global order
  std::vector<uint32_t> psi;
  DevPlan dev{};
  std::vector<void *> allocs;
  ks_config_t cfg{};
  std::vector<TunedEntry> tuned;
  std::mutex lock;  // guards the graph cache, the configuration and the tuned entries
  void *graph_cache = nullptr;
  mutable Trace trace;
  mutable Staging staging;
  mutable Fork fork;
};

// The configuration the current call runs with: installed by the entry
// points for the duration of one call on the calling thread (the tuned
// entry when the plan's schedule is AUTO), the plan's own otherwise.
const ks_config_t &run_cfg(const Plan &pl);
class RunCfgScope {
 public:
  explicit RunCfgScope(const ks_config_t &c);
  ~RunCfgScope();
  RunCfgScope(const RunCfgScope &) = delete;
  RunCfgScope &operator=(const RunCfgScope &) = delete;

 private:
  ks_config_t cfg_;
  const ks_config_t *prev_;
};

// The plan's side stream and events, created on first use (caller holds
// pl.fork.mu).
hipError_t fork_get(const Plan &pl, Fork **f);

// Asynchronous host-to-device copy of `bytes` from `src` through a pinned
// staging slot (src may be freed as soon as this returns).
hipError_t upload_async(const Plan &pl, void *dst, const void *src, size_t bytes, hipStream_t st);

// True (with two events to attach to the launch) while tracing is on.
bool trace_pair(const Plan &pl, const char *stage, hipEvent_t *start, hipEvent_t *stop);

#define KS_LAUNCH(pl, stage, kernel, grid, block, shmem, st, ...)                            \
  do {                                                                                    \
    hipEvent_t ks_e0_, ks_e1_;                                                            \
    if (::ks::trace_pair((pl), (stage), &ks_e0_, &ks_e1_))                                \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, ks_e0_, ks_e1_, 0, __VA_ARGS__); \
    else                                                                                  \
      hipLaunchKernelGGL(kernel, grid, block, shmem, st, __VA_ARGS__);                    \
  } while (0)


ks_status_t plan_build(const ks_params_t *p, Plan *pl);
void plan_free(Plan *pl);

// Tower helpers.
inline uint32_t tower_g(const Plan &pl, uint32_t level, uint32_t t) {
  return t <= level ? t : pl.num_q + (t - level - 1);
}
inline uint32_t num_digits(const Plan &pl, uint32_t level) { return (level + pl.alpha) / pl.alpha; }
inline void digit_range(const Plan &pl, uint32_t level, uint32_t j, uint32_t *lo, uint32_t *hi) {
  *lo = j * pl.alpha;
  uint32_t h = (j + 1) * pl.alpha;
  *hi = h > level + 1 ? level + 1 : h;
}

}  // namespace ks
