// oc_persist.h -- one persistent launch for a batch of Output-Centric key
// switches at mixed levels (work queue with per-job phase counters).
//
// Work items are the tiles of every (phase, job), listed phase-major then
// job-major (the segment table, oc_segments).  Each workgroup takes the next
// item with an atomic increment, waits until the phases that item depends on
// are complete for its job, runs the tile, and bumps the (job, phase)
// completion counter.  Every dependency points to an earlier phase, so an
// item only ever waits on items dequeued before it, each held by a running
// workgroup: the wait always ends, whatever the number of resident
// workgroups (a host test replays this protocol on the real tables).  Each
// wait is nevertheless bounded (spin_limit polls); exceeding it sets the
// abort word, and every group stops at its next check.
//
// Switched off (the launch returns KS_ERR_UNSUPPORTED before reaching this
// code): a batch through it stopped making progress on the device and the
// cause is not established.
#pragma once
#include "oc_kernels.h"

namespace ks {

// Clears the control words with an ordinary kernel (a fill kernel rather
// than a memset node, so the launch captures cleanly into a graph).
template <int A>
__global__ __launch_bounds__(256) void k_zero_words(uint32_t *p, uint32_t n) {
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0;
}

// ctl: [0] queue head, [1] abort word (set when a dependency wait expires),
// [2..3] unused, [4 + job*8 + phase] done counters.  Every group reads the
// abort word before each dequeue and on every poll of a wait, so one expired
// wait ends the whole launch within a poll interval instead of every later
// item spinning to its own limit; ks_batch_status reports the word.
template <int A>
__global__ __launch_bounds__(kOcThreads) void k_oc_persistent(DevPlan P, const OcJob *jobs, const OcSeg *segs,
                                                              uint32_t nsegs, uint32_t total, uint32_t *ctl,
                                                              uint32_t spin_limit) {
  __shared__ uint32_t lds[oc_lds_words<A, 1>()];
  __shared__ uint32_t s_item, s_ok;
  uint32_t *done = ctl + 4;
  for (;;) {
    if (threadIdx.x == 0) {
      uint32_t item = 0xffffffffu;
      if (__hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) item = atomicAdd(&ctl[0], 1u);
      s_item = item;
    }
    __syncthreads();
    const uint32_t item = s_item;
    __syncthreads();
    if (item >= total) break;  // drained, or aborted
    uint32_t lo = 0, hi = nsegs;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (segs[mid].start <= item) lo = mid;
      else hi = mid;
    }
    const OcSeg sg = segs[lo];
    const OcJob J = jobs[sg.job];
    if (threadIdx.x == 0) {
      // relaxed agent-scope polls (coherent loads, no cache invalidation per
      // poll), one acquire fence once the counts are reached
      const uint32_t deps = oc_deps(sg.phase);
      uint32_t ok = 1;
      for (uint32_t q = 0; q < OC_NPHASE && ok; q++) {
        if (!((deps >> q) & 1u)) continue;
        const uint32_t need = J.tiles[q];
        uint32_t *cnt = &done[sg.job * OC_NPHASE + q];
        uint32_t spins = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (__hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || ++spins > spin_limit) {
            atomicOr(&ctl[1], 1u);
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(8);
        }
      }
      if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      s_ok = ok;
    }
    __syncthreads();
    if (!s_ok) break;  // aborted: this group leaves without running the item
    oc_tile<A, 1, 1>(P, J, sg.phase, item - sg.start, lds);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(&done[sg.job * OC_NPHASE + sg.phase], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int A>
hipError_t oc_persistent(const Plan &pl, const OcJob *jobs, const OcSeg *segs, uint32_t nsegs, uint32_t total,
                         uint32_t count, uint32_t *ctl, uint32_t spin_limit, hipStream_t st) {
  static int per_cu = 0, cus = 0;
  if (!per_cu) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return hipErrorUnknown;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_oc_persistent<A>, kOcThreads, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    cus = prop.multiProcessorCount;
  }
  const uint32_t nctl = 4 + count * OC_NPHASE;
  KS_LAUNCH(pl, "oc.zero_ctl", k_zero_words<A>, dim3((nctl + 255) / 256), dim3(256), 0, st, ctl, nctl);
  const uint32_t grid = std::min<uint32_t>((uint32_t)(per_cu * cus), total);
  KS_LAUNCH(pl, "oc.persistent", k_oc_persistent<A>, dim3(grid), dim3(kOcThreads), 0, st, pl.dev, jobs, segs, nsegs,
            total, ctl, spin_limit);
  return hipGetLastError();
}

}  // namespace ks
