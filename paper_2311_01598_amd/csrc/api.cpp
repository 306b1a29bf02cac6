// api.cpp -- the C ABI (include/ks.h): validation, workspace layout and the
// three execution orders of Sec. IV as launch sequences.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "kernels.h"

using namespace ks;

struct ks_plan {
  Plan p;
};

namespace {

inline size_t limb_bytes(const Plan &pl) { return (size_t)pl.n * sizeof(uint32_t); }

// The schedule the current call runs (run_cfg: the call's resolved
// configuration); AUTO with nothing tuned is OC.
ks_schedule_t effective(const Plan &pl) {
  const ks_config_t &c = run_cfg(pl);
  return c.schedule == KS_SCHED_AUTO ? KS_SCHED_OC : c.schedule;
}

// The configuration of a call of `count` key switches whose largest level is
// `level`: the plan's own, or, when its schedule is AUTO, the tuned entry for
// that shape -- the same level, else the nearest tuned level (the higher on a
// tie); among those, the largest tuned count not above `count`, else the
// smallest -- with its zero fields taken from the plan's configuration.
// With nothing tuned, AUTO runs OC with the plan's settings.  oc_only: calls
// that run the OC order only (compressed keys, rotations, the scratch-backed
// call) take OC with the plan's settings when the entry names another
// schedule.
ks_config_t resolve_cfg(Plan &pl, uint32_t level, uint32_t count, bool oc_only) {
  std::lock_guard<std::mutex> g(pl.lock);
  ks_config_t c = pl.cfg;
  if (c.schedule != KS_SCHED_AUTO) return c;
  const auto dist = [level](uint32_t l) { return l > level ? l - level : level - l; };
  const TunedEntry *best = nullptr;
  for (const TunedEntry &e : pl.tuned) {
    bool take = !best;
    if (!take) {
      if (dist(e.level) != dist(best->level)) take = dist(e.level) < dist(best->level);
      else if (e.level != best->level) take = e.level > best->level;
      else if ((e.count <= count) != (best->count <= count)) take = e.count <= count;
      else take = e.count <= count ? e.count > best->count : e.count < best->count;
    }
    if (take) best = &e;
  }
  const ks_config_t base = c;
  c.schedule = KS_SCHED_OC;
  if (best) {
    const ks_config_t &t = best->cfg;
    c.schedule = t.schedule;
    if (t.tile_towers) c.tile_towers = t.tile_towers;
    if (t.col_width) c.col_width = t.col_width;
    if (t.row_block) c.row_block = t.row_block;
    if (t.batch_mode) c.batch_mode = t.batch_mode;
    if (t.graph) c.graph = t.graph;
    if (t.batch_order) c.batch_order = t.batch_order;
  }
  if (oc_only && c.schedule != KS_SCHED_OC) {
    c = base;
    c.schedule = KS_SCHED_OC;
  }
  return c;
}

// Workspace of one key switch at `level`, in limbs, per schedule.
size_t ws_limbs(const Plan &pl, ks_schedule_t sch, uint32_t level) {
  const size_t L1 = level + 1, K = pl.num_p, T = L1 + K, D = num_digits(pl, level);
  switch (sch) {
    case KS_SCHED_MP: return L1 + D * T + D * 2 * T + 2 * T + 2 * K + 2 * L1;
    case KS_SCHED_DC: return pl.alpha + T + 2 * T + 2 * K + 2 * L1;
    default: return L1 + D * T + 2 * K + 2 * L1;
  }
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// OC batch workspace: control words, segment table, job table, then one
// OC region per job.
struct BatchLayout {
  size_t ctl, segs, jobs, regions, total;
  std::vector<size_t> region;  // byte offset of each job's region
};
BatchLayout batch_layout(const Plan &pl, uint32_t count, const uint32_t *levels) {
  BatchLayout b;
  b.ctl = 0;
  b.segs = align256((4 + (size_t)count * OC_NPHASE) * sizeof(uint32_t));
  b.jobs = b.segs + align256((size_t)count * OC_NPHASE * sizeof(OcSeg));
  b.regions = b.jobs + align256((size_t)count * sizeof(OcJob));
  size_t off = b.regions;
  b.region.resize(count);
  for (uint32_t i = 0; i < count; i++) {
    b.region[i] = off;
    off += align256(ws_limbs(pl, KS_SCHED_OC, levels[i]) * limb_bytes(pl));
  }
  b.total = off;
  return b;
}

// Hoisted rotations: job table, the shared ModUp output (xt, ycol), then
// the ModDown regions (zp, wcol) of every rotation.
struct RotLayout {
  size_t xt, ycol, rot0, per_rot, total;
};
RotLayout rot_layout(const Plan &pl, uint32_t level, uint32_t count) {
  const size_t L1 = level + 1, K = pl.num_p, T = L1 + K, D = num_digits(pl, level), lb = limb_bytes(pl);
  RotLayout r;
  r.xt = align256((size_t)count * sizeof(OcJob));
  r.ycol = r.xt + align256(L1 * lb);
  r.rot0 = r.ycol + align256(D * T * lb);
  r.per_rot = align256((2 * K + 2 * L1) * lb);
  r.total = count ? r.rot0 + (size_t)count * r.per_rot : 0;
  return r;
}

// Multiplication: the tensor product d [3][l+1][N], then one OC region.
size_t mult_tensor_bytes(const Plan &pl, uint32_t level) { return align256((size_t)3 * (level + 1) * limb_bytes(pl)); }
size_t mult_bytes(const Plan &pl, uint32_t level) {
  return mult_tensor_bytes(pl, level) + ws_limbs(pl, KS_SCHED_OC, level) * limb_bytes(pl);
}

bool galois_ok(const Plan &pl, uint32_t k) { return (k & 1u) && k < 2u * pl.n; }

// Double hoisting: term table, then the MP ModUp output X [l+1], Y [d'][T],
// the summed accumulator ACC [2][T] and the ModDown buffers XP [2][K],
// W [2][l+1].
struct SumLayout {
  size_t x, y, acc, xp, w, total;
};
SumLayout sum_layout(const Plan &pl, uint32_t level, uint32_t count) {
  const size_t L1 = level + 1, K = pl.num_p, T = L1 + K, D = num_digits(pl, level), lb = limb_bytes(pl);
  SumLayout r;
  r.x = align256((size_t)count * sizeof(RotTerm));
  r.y = r.x + align256(L1 * lb);
  r.acc = r.y + align256(D * T * lb);
  r.xp = r.acc + align256(2 * T * lb);
  r.w = r.xp + align256(2 * K * lb);
  r.total = count ? r.w + align256(2 * L1 * lb) : 0;
  return r;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + nb && y < x + na;
}

ks_status_t dev_err(hipError_t e) { return e == hipSuccess ? KS_OK : KS_ERR_DEVICE; }

#define TRY(expr)                                  \
  do {                                             \
    hipError_t _e = (expr);                        \
    if (_e != hipSuccess) return KS_ERR_DEVICE;    \
  } while (0)

#define TRYK(expr)                    \
  do {                                \
    const ks_status_t _s = (expr);    \
    if (_s != KS_OK) return _s;       \
  } while (0)

// ---------------------------------------------------------------- MP
// Sec. IV-A: every stage over all towers, every stage output in HBM.
// ModUp P1-P3 in the MP order: X [l+1] (INTT of d), Y [d'][T] (every digit
// extended, evaluation domain; a digit's own towers are left to d).
ks_status_t mp_modup(const Plan &pl, uint32_t level, const uint32_t *d, uint32_t *X, uint32_t *Y, hipStream_t st) {
  const uint32_t L1 = level + 1, K = pl.num_p, T = L1 + K, D = num_digits(pl, level);
  std::vector<uint32_t> so, dof, g;
  // ModUp P1: INTT of all towers
  for (uint32_t i = 0; i < L1; i++) { so.push_back(i); dof.push_back(i); g.push_back(i); }
  TRY(launch_ntt(pl, true, d, X, so, dof, g, st));
  // P2: basis conversion of every digit
  TRY(launch_bconv_up(pl, level, 0, D, false, X, Y, st));
  // P3: NTT of every extended tower
  so.clear(); dof.clear(); g.clear();
  for (uint32_t j = 0; j < D; j++) {
    uint32_t lo, hi;
    digit_range(pl, level, j, &lo, &hi);
    for (uint32_t t = 0; t < T; t++) {
      if (t >= lo && t < hi) continue;
      so.push_back(j * T + t); dof.push_back(j * T + t); g.push_back(tower_g(pl, level, t));
    }
  }
  TRY(launch_ntt(pl, false, Y, Y, so, dof, g, st));
  return KS_OK;
}

// ModDown P1-P4 in the MP order from ACC [2][T] (carrying 2^-32) to out.
ks_status_t mp_moddown(const Plan &pl, uint32_t level, const uint32_t *ACC, uint32_t *XP, uint32_t *W, uint32_t *out,
                       hipStream_t st) {
  const uint32_t L1 = level + 1, K = pl.num_p, T = L1 + K;
  std::vector<uint32_t> so, dof, g;
  // ModDown P1: INTT of the K special towers of both polynomials
  for (uint32_t s = 0; s < 2; s++)
    for (uint32_t k = 0; k < K; k++) { so.push_back(s * T + L1 + k); dof.push_back(s * K + k); g.push_back(pl.num_q + k); }
  TRY(launch_ntt(pl, true, ACC, XP, so, dof, g, st));
  // P2: basis conversion P -> Q_l; P3: NTT; P4: subtract, times P^-1
  TRY(launch_bconv_down(pl, level, XP, W, st));
  so.clear(); dof.clear(); g.clear();
  for (uint32_t s = 0; s < 2; s++)
    for (uint32_t i = 0; i < L1; i++) { so.push_back(s * L1 + i); dof.push_back(s * L1 + i); g.push_back(i); }
  TRY(launch_ntt(pl, false, W, W, so, dof, g, st));
  TRY(launch_moddown_final(pl, level, ACC, W, out, st));
  return KS_OK;
}

ks_status_t run_mp(const Plan &pl, const uint32_t *evk, uint32_t level, const uint32_t *d, uint32_t *out,
                   uint32_t *ws, hipStream_t st) {
  const uint32_t L1 = level + 1, K = pl.num_p, T = L1 + K, D = num_digits(pl, level), N = pl.n;
  uint32_t *X = ws, *Y = X + (size_t)L1 * N, *Z = Y + (size_t)D * T * N, *ACC = Z + (size_t)D * 2 * T * N;
  uint32_t *XP = ACC + (size_t)2 * T * N, *W = XP + (size_t)2 * K * N;
  TRYK(mp_modup(pl, level, d, X, Y, st));
  // P4: apply key, P5: sum over digits
  TRY(launch_keymul(pl, level, d, Y, evk, Z, st));
  TRY(launch_reduce_digits(pl, level, Z, ACC, st));
  return mp_moddown(pl, level, ACC, XP, W, out, st);
}

// ---------------------------------------------------------------- DC
// Sec. IV-B: one digit at a time through P1-P5, partial sums accumulated.
ks_status_t run_dc(const Plan &pl, const uint32_t *evk, uint32_t level, const uint32_t *d, uint32_t *out,
                   uint32_t *ws, hipStream_t st) {
  const uint32_t L1 = level + 1, K = pl.num_p, T = L1 + K, D = num_digits(pl, level), N = pl.n;
  uint32_t *X = ws, *Yj = X + (size_t)pl.alpha * N, *ACC = Yj + (size_t)T * N;
  uint32_t *XP = ACC + (size_t)2 * T * N, *W = XP + (size_t)2 * K * N;
  std::vector<uint32_t> so, dof, g;
  for (uint32_t j = 0; j < D; j++) {
    uint32_t lo, hi;
    digit_range(pl, level, j, &lo, &hi);
    so.clear(); dof.clear(); g.clear();
    for (uint32_t i = lo; i < hi; i++) { so.push_back(i); dof.push_back(i - lo); g.push_back(i); }
    TRY(launch_ntt(pl, true, d, X, so, dof, g, st));
    TRY(launch_bconv_up(pl, level, j, 1, true, X, Yj, st));
    so.clear(); dof.clear(); g.clear();
    for (uint32_t t = 0; t < T; t++) {
      if (t >= lo && t < hi) continue;
      so.push_back(t); dof.push_back(t); g.push_back(tower_g(pl, level, t));
    }
    TRY(launch_ntt(pl, false, Yj, Yj, so, dof, g, st));
    TRY(launch_keymac_digit(pl, level, j, d, Yj, evk, ACC, st));
  }
  so.clear(); dof.clear(); g.clear();
  for (uint32_t s = 0; s < 2; s++)
    for (uint32_t k = 0; k < K; k++) { so.push_back(s * T + L1 + k); dof.push_back(s * K + k); g.push_back(pl.num_q + k); }
  TRY(launch_ntt(pl, true, ACC, XP, so, dof, g, st));
  TRY(launch_bconv_down(pl, level, XP, W, st));
  so.clear(); dof.clear(); g.clear();
  for (uint32_t s = 0; s < 2; s++)
    for (uint32_t i = 0; i < L1; i++) { so.push_back(s * L1 + i); dof.push_back(s * L1 + i); g.push_back(i); }
  TRY(launch_ntt(pl, false, W, W, so, dof, g, st));
  TRY(launch_moddown_final(pl, level, ACC, W, out, st));
  return KS_OK;
}

// One key switch of a call: a full key, or a compressed one (b halves plus
// the seed of the a halves).
struct Job {
  const uint32_t *evk;
  uint64_t a_seed;
  uint32_t level;
  const uint32_t *in;
  uint32_t *out;
  uint32_t galois = 1;             // a rotation: the automorphism of its digits
  const uint32_t *add0 = nullptr;  // a rotation: c0, added (permuted) to output 0
};

// Row-stage kernels of a call, and the halves its keys hold.
bool rows_seeded(OcRowVariant rows) { return rows == OC_ROWS_SEEDED || rows == OC_ROWS_SEEDED_EXT; }

// ---------------------------------------------------------------- OC
OcJob make_oc_job(const Plan &pl, const Job &jb, uint32_t *ws, uint32_t tt) {
  const uint32_t *evk = jb.evk, *d = jb.in, level = jb.level;
  uint32_t *out = jb.out;
  const uint32_t L1 = level + 1, K = pl.num_p, T = L1 + K, D = num_digits(pl, level), N = pl.n;
  OcJob j{};
  j.d = d;
  j.evk = evk;
  j.out = out;
  j.level = level;
  j.xt = ws;
  j.ycol = j.xt + (size_t)L1 * N;
  j.zp = j.ycol + (size_t)D * T * N;
  j.wcol = j.zp + (size_t)2 * K * N;
  j.a_seed = jb.a_seed;
  j.galois = jb.galois;
  j.add0 = jb.add0;
  j.ttu = j.ttd = tt;
  oc_tiles_host(pl, level, tt, j.tiles);
  return j;
}

// l1: the largest l+1 of the launch
uint32_t oc_tt(const Plan &pl, uint32_t l1) {
  const ks_config_t &c = run_cfg(pl);
  return oc_effective_tt(pl.dev.loga, c.tile_towers ? c.tile_towers : 1, l1);
}

ks_status_t run_oc(const Plan &pl, const Job &jb, OcRowVariant rows, uint32_t *ws, hipStream_t st) {
  const uint32_t tt = oc_tt(pl, jb.level + 1);
  const OcJob j = make_oc_job(pl, jb, ws, tt);
  return dev_err(launch_oc_phases(pl, j, nullptr, 1, j.tiles, tt, rows, OC_PART_ALL, st));
}

// Compressed keys and rotations are supported by the OC schedule only
// (callers check).
ks_status_t run_one(const Plan &pl, ks_schedule_t sch, const Job &jb, OcRowVariant rows, uint32_t *ws,
                    hipStream_t st) {
  ks_status_t r;
  switch (sch) {
    case KS_SCHED_MP: r = run_mp(pl, jb.evk, jb.level, jb.in, jb.out, ws, st); break;
    case KS_SCHED_DC: r = run_dc(pl, jb.evk, jb.level, jb.in, jb.out, ws, st); break;
    default: r = run_oc(pl, jb, rows, ws, st); break;
  }
  return r;
}

// A captured batch: the graph replays the launches for one (count,
// workspace, configuration); the job table is re-uploaded before each replay.
struct GraphEntry {
  uint32_t count, mode, tt, spin, total;
  OcRowVariant rows;
  std::vector<uint32_t> max_tiles;
  const void *ws;
  hipGraphExec_t exec;
};
struct GraphCache {
  hipStream_t capture = nullptr;
  std::vector<GraphEntry> entries;
};

ks_status_t launch_oc_batch(const Plan &pl, uint32_t count, const std::vector<uint32_t> &max_tiles, uint32_t total,
                            char *ws, const BatchLayout &lay, uint32_t mode, uint32_t tt, uint32_t spin,
                            OcRowVariant rows, hipStream_t st) {
  const OcJob *djobs = (const OcJob *)(ws + lay.jobs);
  if (mode == 2 && rows != OC_ROWS_PLAIN) return KS_ERR_UNSUPPORTED;
  if (mode == 2)
    return dev_err(launch_oc_persistent(pl, djobs, (const OcSeg *)(ws + lay.segs), count * OC_NPHASE, total, count,
                                        (uint32_t *)(ws + lay.ctl), spin, st));
  const OcJob none{};
  if (mode != 3 || count < 2)
    return dev_err(launch_oc_phases(pl, none, djobs, count, max_tiles.data(), tt, rows, OC_PART_ALL, st));
  // Mode 3: the batch runs as two halves, the second on the plan's side stream:
  // the halves drift apart, so a bandwidth-bound phase of one overlaps a
  // compute-bound phase of the other.  (Each half launches with the batch's
  // largest tile counts; tiles past a job's own count return at once.)
  std::lock_guard<std::mutex> g(pl.fork.mu);
  Fork *f = nullptr;
  TRY(fork_get(pl, &f));
  TRY(hipEventRecord(f->fork, st));
  TRY(hipStreamWaitEvent(f->side, f->fork, 0));
  const uint32_t h = count / 2;
  TRY(launch_oc_phases(pl, none, djobs, h, max_tiles.data(), tt, rows, OC_PART_ALL, st));
  TRY(launch_oc_phases(pl, none, djobs + h, count - h, max_tiles.data(), tt, rows, OC_PART_ALL, f->side));
  TRY(hipEventRecord(f->join, f->side));
  TRY(hipStreamWaitEvent(st, f->join, 0));
  return KS_OK;
}

}  // namespace

uint32_t ks::oc_segments(const uint32_t *tiles, uint32_t count, std::vector<OcSeg> &segs) {
  segs.clear();
  segs.reserve((size_t)count * OC_NPHASE);
  uint32_t total = 0;
  for (uint32_t p = 0; p < OC_NPHASE; p++)
    for (uint32_t i = 0; i < count; i++) {
      segs.push_back(OcSeg{total, i, p, 0});
      total += tiles[(size_t)i * OC_NPHASE + p];
    }
  return total;
}

namespace {

ks_status_t run_oc_batch(Plan &pl, uint32_t count, const Job *jobs, OcRowVariant rows, const BatchLayout &lay,
                         char *ws, hipStream_t st) {
  const ks_config_t &cfg = run_cfg(pl);
  const uint32_t mode = cfg.batch_mode;
  uint32_t l1max = 0;
  for (uint32_t i = 0; i < count; i++) l1max = std::max(l1max, jobs[i].level + 1);
  const uint32_t tt = mode == 2 ? 1 : oc_tt(pl, l1max);
  const uint32_t spin = cfg.spin_limit ? cfg.spin_limit : (1u << 20);
  // host tables
  std::vector<OcJob> hj(count);
  std::vector<uint32_t> max_tiles(OC_NPHASE, 0);
  for (uint32_t i = 0; i < count; i++) {
    hj[i] = make_oc_job(pl, jobs[i], (uint32_t *)(ws + lay.region[i]), tt);
    for (uint32_t p = 0; p < OC_NPHASE; p++) max_tiles[p] = std::max(max_tiles[p], hj[i].tiles[p]);
  }
  std::vector<uint32_t> tiles((size_t)count * OC_NPHASE);
  for (uint32_t i = 0; i < count; i++) std::copy(hj[i].tiles, hj[i].tiles + OC_NPHASE, &tiles[(size_t)i * OC_NPHASE]);
  std::vector<OcSeg> segs;
  const uint32_t total = oc_segments(tiles.data(), count, segs);
  // the job and segment tables live in the workspace (the graph reads them there)
  // control words (zero), segment table and job table in one upload
  std::vector<char> blob(lay.regions, 0);
  std::memcpy(blob.data() + lay.segs, segs.data(), segs.size() * sizeof(OcSeg));
  std::memcpy(blob.data() + lay.jobs, hj.data(), hj.size() * sizeof(OcJob));
  TRY(upload_async(pl, ws, blob.data(), blob.size(), st));

  const bool use_graph = cfg.graph != 2 && !pl.trace.on;
  if (!use_graph) return launch_oc_batch(pl, count, max_tiles, total, ws, lay, mode, tt, spin, rows, st);

  // graph keyed by (count, workspace, mode, tile, spin); the persistent launch
  // reads `total` from its arguments, so it is part of the key as well
  std::lock_guard<std::mutex> g(pl.lock);
  GraphCache *gc = (GraphCache *)pl.graph_cache;
  if (!gc) {
    gc = new GraphCache();
    pl.graph_cache = gc;
  }
  hipGraphExec_t exec = nullptr;
  for (auto &e : gc->entries)
    if (e.count == count && e.ws == ws && e.mode == mode && e.tt == tt && e.spin == spin && e.total == total &&
        e.rows == rows && e.max_tiles == max_tiles)
      exec = e.exec;
  if (!exec) {
    if (!gc->capture && hipStreamCreateWithFlags(&gc->capture, hipStreamNonBlocking) != hipSuccess)
      return KS_ERR_DEVICE;
    TRY(hipStreamBeginCapture(gc->capture, hipStreamCaptureModeThreadLocal));
    ks_status_t r = launch_oc_batch(pl, count, max_tiles, total, ws, lay, mode, tt, spin, rows, gc->capture);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(gc->capture, &graph);
    if (r != KS_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return KS_ERR_DEVICE;
    }
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return KS_ERR_DEVICE;
    if (gc->entries.size() >= 64) {  // bounded cache: drop the oldest capture
      (void)hipGraphExecDestroy(gc->entries.front().exec);
      gc->entries.erase(gc->entries.begin());
    }
    gc->entries.push_back(GraphEntry{count, mode, tt, spin, total, rows, max_tiles, ws, exec});
  }
  TRY(hipGraphLaunch(exec, st));
  return KS_OK;
}

// evk_halves: 2 for a full key, 1 for a compressed key (b halves only).
ks_status_t check_job(const Plan &pl, const uint32_t *evk, uint32_t level, const uint32_t *in, const uint32_t *out,
                      const void *ws, size_t ws_bytes, size_t need, uint32_t evk_halves = 2) {
  if (!evk || !in || !out || !ws) return KS_ERR_INVALID_ARG;
  if (level >= pl.num_q) return KS_ERR_INVALID_ARG;
  if (((uintptr_t)evk | (uintptr_t)in | (uintptr_t)out) & 15) return KS_ERR_INVALID_ARG;
  if ((uintptr_t)ws & 255) return KS_ERR_INVALID_ARG;
  if (ws_bytes < need) return KS_ERR_BUDGET;
  const size_t lb = limb_bytes(pl);
  const size_t out_b = 2 * (size_t)(level + 1) * lb, in_b = (size_t)(level + 1) * lb;
  const size_t evk_b = (size_t)pl.dnum * evk_halves * pl.ntot * lb;
  if (overlaps(out, out_b, in, in_b) || overlaps(out, out_b, evk, evk_b) || overlaps(out, out_b, ws, ws_bytes))
    return KS_ERR_INVALID_ARG;
  if (overlaps(ws, ws_bytes, in, in_b) || overlaps(ws, ws_bytes, evk, evk_b)) return KS_ERR_INVALID_ARG;
  return KS_OK;
}

ks_status_t validate_params(const ks_params_t *p) {
  if (!p) return KS_ERR_INVALID_ARG;
  if (p->log_n < 12 || p->log_n > 17) return KS_ERR_UNSUPPORTED;
  if (p->num_q == 0 || p->dnum == 0 || p->dnum > p->num_q) return KS_ERR_INVALID_ARG;
  const uint32_t alpha = (p->num_q + p->dnum - 1) / p->dnum;
  const uint32_t K = p->num_p ? p->num_p : alpha;
  if (p->num_q + K > kMaxTowers) return KS_ERR_UNSUPPORTED;
  if (alpha > 32 || K > 32 || p->dnum > 16) return KS_ERR_UNSUPPORTED;
  if (p->moduli) {
    const uint64_t two_n = 2ull << p->log_n;
    for (uint32_t i = 0; i < p->num_q + K; i++) {
      const uint32_t m = p->moduli[i];
      if (m <= (1u << 29) || m >= (1u << 30) || m % two_n != 1 || !is_prime_u64(m)) return KS_ERR_INVALID_ARG;
      for (uint32_t j = 0; j < i; j++)
        if (p->moduli[j] == m) return KS_ERR_INVALID_ARG;
    }
  }
  return KS_OK;
}

}  // namespace

#ifdef KS_CHECK_RANGES
// The range-check build's registry: one reader per HIP compile unit, filled
// while the library loads.
namespace ks_range {
namespace {
struct Unit {
  reader_t read;
  strict_t strict;
};
std::mutex &registry_mu() {
  static std::mutex m;
  return m;
}
std::vector<Unit> &registry() {
  static std::vector<Unit> r;
  return r;
}
}  // namespace
void register_unit(reader_t read, strict_t strict) {
  std::lock_guard<std::mutex> g(registry_mu());
  registry().push_back({read, strict});
}
}  // namespace ks_range
#endif

extern "C" {

ks_status_t ks_range_violations(uint32_t *count, uint32_t *code, int reset) {
#ifdef KS_CHECK_RANGES
  if (!count || !code) return KS_ERR_INVALID_ARG;
  *count = 0;
  *code = 0;
  if (hipDeviceSynchronize() != hipSuccess) return KS_ERR_DEVICE;
  std::lock_guard<std::mutex> g(ks_range::registry_mu());
  for (const auto &u : ks_range::registry())
    if (u.read(count, code, reset) != 0) return KS_ERR_DEVICE;
  return KS_OK;
#else
  (void)count;
  (void)code;
  (void)reset;
  return KS_ERR_UNSUPPORTED;
#endif
}

ks_status_t ks_range_set_strict(int on) {
#ifdef KS_CHECK_RANGES
  if (hipDeviceSynchronize() != hipSuccess) return KS_ERR_DEVICE;
  std::lock_guard<std::mutex> g(ks_range::registry_mu());
  for (const auto &u : ks_range::registry())
    if (u.strict(on) != 0) return KS_ERR_DEVICE;
  return KS_OK;
#else
  (void)on;
  return KS_ERR_UNSUPPORTED;
#endif
}

const char *ks_status_string(ks_status_t s) {
  switch (s) {
    case KS_OK: return "ok";
    case KS_ERR_INVALID_ARG: return "invalid argument";
    case KS_ERR_UNSUPPORTED: return "unsupported parameters";
    case KS_ERR_NOMEM: return "out of memory";
    case KS_ERR_BUDGET: return "workspace too small";
    case KS_ERR_DEVICE: return "device error";
  }
  return "unknown status";
}

ks_status_t ks_params_moduli(const ks_params_t *p, uint32_t *host_out) {
  ks_status_t st = validate_params(p);
  if (st != KS_OK) return st;
  if (!host_out) return KS_ERR_INVALID_ARG;
  const uint32_t alpha = (p->num_q + p->dnum - 1) / p->dnum;
  const uint32_t K = p->num_p ? p->num_p : alpha, tot = p->num_q + K;
  if (p->moduli) {
    std::copy(p->moduli, p->moduli + tot, host_out);
    return KS_OK;
  }
  std::vector<uint32_t> pr(tot);
  if (ntt_primes(p->log_n, tot, pr.data()) != 0) return KS_ERR_UNSUPPORTED;
  for (uint32_t i = 0; i < p->num_q; i++) host_out[i] = pr[K + i];
  for (uint32_t k = 0; k < K; k++) host_out[p->num_q + k] = pr[k];
  return KS_OK;
}

uint32_t ks_root_of_unity(uint32_t q, uint32_t log_n) {
  if (log_n < 1 || log_n > 20) return 0;
  return min_root_2n(q, log_n);
}

ks_status_t ks_plan_create(const ks_params_t *p, ks_plan_t *out) {
  if (!out) return KS_ERR_INVALID_ARG;
  *out = nullptr;
  ks_status_t st = validate_params(p);
  if (st != KS_OK) return st;
  ks_plan *pl = new (std::nothrow) ks_plan();
  if (!pl) return KS_ERR_NOMEM;
  pl->p.cfg = ks_config_t{KS_SCHED_OC, 2, 16, 8, 1, 2, 0, 1};  // the starting configuration ks.h documents
  st = plan_build(p, &pl->p);
  if (st != KS_OK) {
    plan_free(&pl->p);
    delete pl;
    return st;
  }
  // set-up of ks_keyswitch_noalloc on this device (the plan's, current
  // here); a failure only makes that entry point return KS_ERR_DEVICE
  (void)noalloc_scratch_init(pl->p.device);
  *out = pl;
  return KS_OK;
}

ks_status_t ks_plan_destroy(ks_plan_t plan) {
  if (!plan) return KS_ERR_INVALID_ARG;
  (void)hipDeviceSynchronize();
  if (GraphCache *gc = (GraphCache *)plan->p.graph_cache) {
    for (auto &e : gc->entries) (void)hipGraphExecDestroy(e.exec);
    if (gc->capture) (void)hipStreamDestroy(gc->capture);
    delete gc;
    plan->p.graph_cache = nullptr;
  }
  plan_free(&plan->p);
  delete plan;
  return KS_OK;
}

ks_status_t ks_plan_moduli(ks_plan_t plan, uint32_t *host_out) {
  if (!plan || !host_out) return KS_ERR_INVALID_ARG;
  std::copy(plan->p.mod.begin(), plan->p.mod.end(), host_out);
  return KS_OK;
}

static ks_status_t check_cfg(const ks_config_t *cfg) {
  if ((int)cfg->schedule < 0 || (int)cfg->schedule > 3) return KS_ERR_INVALID_ARG;
  auto ok = [](uint32_t v, std::initializer_list<uint32_t> allowed) {
    if (!v) return true;
    for (uint32_t a : allowed) if (a == v) return true;
    return false;
  };
  if (!ok(cfg->tile_towers, {1, 2, 4}) || !ok(cfg->col_width, {8, 16, 32}) || !ok(cfg->row_block, {4, 8, 16}) ||
      !ok(cfg->batch_mode, {1, 2, 3}) || !ok(cfg->graph, {1, 2}) || !ok(cfg->batch_order, {1, 2}))
    return KS_ERR_INVALID_ARG;
  // The persistent work-queue launch is switched off: a batch run through it
  // stopped making progress on the device and the cause is not established.
  // (Graph capture of the per-phase launches, modes 1 and 3, is on.)
  if (cfg->batch_mode == 2) return KS_ERR_UNSUPPORTED;
  return KS_OK;
}

ks_status_t ks_plan_set_config(ks_plan_t plan, const ks_config_t *cfg) {
  if (!plan || !cfg) return KS_ERR_INVALID_ARG;
  const ks_status_t v = check_cfg(cfg);
  if (v != KS_OK) return v;
  std::lock_guard<std::mutex> g(plan->p.lock);
  ks_config_t &c = plan->p.cfg;
  c.schedule = cfg->schedule;
  if (cfg->tile_towers) c.tile_towers = cfg->tile_towers;
  if (cfg->col_width) c.col_width = cfg->col_width;
  if (cfg->row_block) c.row_block = cfg->row_block;
  if (cfg->batch_mode) c.batch_mode = cfg->batch_mode;
  if (cfg->graph) c.graph = cfg->graph;
  if (cfg->spin_limit) c.spin_limit = cfg->spin_limit;
  if (cfg->batch_order) c.batch_order = cfg->batch_order;
  return KS_OK;
}

ks_status_t ks_oc_work_list(const ks_params_t *p, uint32_t count, const uint32_t *levels, uint32_t *tiles,
                            uint32_t *seg_start, uint32_t *seg_job, uint32_t *seg_phase, uint32_t *deps,
                            uint32_t *total) {
  const ks_status_t v = validate_params(p);
  if (v != KS_OK) return v;
  if (!count || !levels || !tiles || !seg_start || !seg_job || !seg_phase || !deps || !total)
    return KS_ERR_INVALID_ARG;
  const uint32_t alpha = (p->num_q + p->dnum - 1) / p->dnum, K = p->num_p ? p->num_p : alpha;
  for (uint32_t i = 0; i < count; i++) {
    if (levels[i] >= p->num_q) return KS_ERR_INVALID_ARG;
    oc_tiles_params(p->log_n, alpha, K, levels[i], 1, tiles + (size_t)i * OC_NPHASE);
  }
  std::vector<OcSeg> segs;
  *total = oc_segments(tiles, count, segs);
  for (size_t k = 0; k < segs.size(); k++) {
    seg_start[k] = segs[k].start;
    seg_job[k] = segs[k].job;
    seg_phase[k] = segs[k].phase;
  }
  for (uint32_t q = 0; q < OC_NPHASE; q++) deps[q] = oc_deps(q);
  return KS_OK;
}

ks_status_t ks_plan_set_tuned(ks_plan_t plan, uint32_t level, uint32_t count, const ks_config_t *cfg) {
  if (!plan || !cfg || !count) return KS_ERR_INVALID_ARG;
  if (level >= plan->p.num_q || cfg->schedule == KS_SCHED_AUTO) return KS_ERR_INVALID_ARG;
  const ks_status_t v = check_cfg(cfg);
  if (v != KS_OK) return v;
  std::lock_guard<std::mutex> g(plan->p.lock);
  for (TunedEntry &e : plan->p.tuned)
    if (e.level == level && e.count == count) {
      e.cfg = *cfg;
      return KS_OK;
    }
  plan->p.tuned.push_back(TunedEntry{level, count, *cfg});
  return KS_OK;
}

ks_status_t ks_plan_clear_tuned(ks_plan_t plan) {
  if (!plan) return KS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(plan->p.lock);
  plan->p.tuned.clear();
  return KS_OK;
}

ks_status_t ks_plan_resolve_config(ks_plan_t plan, uint32_t level, uint32_t count, ks_config_t *out) {
  if (!plan || !out || !count || level >= plan->p.num_q) return KS_ERR_INVALID_ARG;
  *out = resolve_cfg(plan->p, level, count, false);
  if (out->schedule == KS_SCHED_AUTO) out->schedule = KS_SCHED_OC;
  return KS_OK;
}

ks_status_t ks_plan_get_config(ks_plan_t plan, ks_config_t *cfg) {
  if (!plan || !cfg) return KS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(plan->p.lock);
  *cfg = plan->p.cfg;
  return KS_OK;
}

ks_status_t ks_workspace_size(ks_plan_t plan, uint32_t count, const uint32_t *levels, size_t *bytes) {
  if (!plan || !bytes || (count && !levels)) return KS_ERR_INVALID_ARG;
  const Plan &pl = plan->p;
  uint32_t lmax = 0;
  for (uint32_t i = 0; i < count; i++) lmax = std::max(lmax, levels[i]);
  const RunCfgScope scope(resolve_cfg(plan->p, lmax, count, false));
  size_t mx = 0;
  for (uint32_t i = 0; i < count; i++) {
    if (levels[i] >= pl.num_q) return KS_ERR_INVALID_ARG;
    mx = std::max(mx, ws_limbs(pl, effective(pl), levels[i]));
  }
  *bytes = mx * limb_bytes(pl);
  if (count > 1 && effective(pl) == KS_SCHED_OC) *bytes = batch_layout(pl, count, levels).total;
  return KS_OK;
}

// Failure-handling tests: KS_FAULT_INJECT=<n> makes the n-th call (1-based)
// of ks_keyswitch_batch after the variable took its current value report
// KS_ERR_DEVICE without enqueuing anything.
static bool injected_fault() {
  static std::mutex mu;
  static std::string seen;
  static uint64_t calls = 0;
  const char *e = std::getenv("KS_FAULT_INJECT");
  const std::string now = e ? e : "";
  std::lock_guard<std::mutex> g(mu);
  if (now != seen) {
    seen = now;
    calls = 0;
  }
  if (now.empty()) return false;
  return ++calls == std::strtoull(now.c_str(), nullptr, 10);
}

}  // extern "C"

namespace {

ks_status_t keyswitch_one(ks_plan_t plan, const Job &jb, OcRowVariant rows, void *workspace, size_t workspace_bytes,
                          void *stream, bool oc_only = false) {
  if (!plan) return KS_ERR_INVALID_ARG;
  const Plan &pl = plan->p;
  const RunCfgScope scope(resolve_cfg(plan->p, jb.level, 1, oc_only || rows != OC_ROWS_PLAIN));
  const ks_schedule_t sch = effective(pl);
  if (rows != OC_ROWS_PLAIN && sch != KS_SCHED_OC) return KS_ERR_UNSUPPORTED;
  if (jb.level >= pl.num_q) return KS_ERR_INVALID_ARG;
  const size_t need = ws_limbs(pl, sch, jb.level) * limb_bytes(pl);
  ks_status_t st = check_job(pl, jb.evk, jb.level, jb.in, jb.out, workspace, workspace_bytes, need,
                             rows_seeded(rows) ? 1 : 2);
  if (st != KS_OK) return st;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl.device) return KS_ERR_INVALID_ARG;
  return run_one(pl, sch, jb, rows, (uint32_t *)workspace, (hipStream_t)stream);
}

ks_status_t keyswitch_batch(ks_plan_t plan, const std::vector<Job> &jobs_in, OcRowVariant rows, void *workspace,
                            size_t workspace_bytes, void *stream) {
  const uint32_t count = (uint32_t)jobs_in.size();
  Plan &pl = plan->p;
  uint32_t lmax = 0;
  for (const Job &j : jobs_in) lmax = std::max(lmax, j.level);
  const RunCfgScope scope(resolve_cfg(pl, lmax, count, rows != OC_ROWS_PLAIN));
  const ks_schedule_t sch = effective(pl);
  // batch order (a tuner choice): as given, or by decreasing level; every
  // job's result is the same either way
  std::vector<Job> jobs(jobs_in);
  if (run_cfg(pl).batch_order == 2)
    std::stable_sort(jobs.begin(), jobs.end(), [](const Job &a, const Job &b) { return a.level > b.level; });
  if (rows != OC_ROWS_PLAIN && sch != KS_SCHED_OC) return KS_ERR_UNSUPPORTED;
  if (!count) return KS_OK;
  std::vector<uint32_t> levels(count);
  for (uint32_t i = 0; i < count; i++) {
    if (jobs[i].level >= pl.num_q) return KS_ERR_INVALID_ARG;
    levels[i] = jobs[i].level;
  }
  const bool together = sch == KS_SCHED_OC && count > 1;
  size_t need = 0;
  for (uint32_t i = 0; i < count; i++) need = std::max(need, ws_limbs(pl, sch, levels[i]) * limb_bytes(pl));
  BatchLayout lay;
  if (together) {
    lay = batch_layout(pl, count, levels.data());
    need = lay.total;
  }
  for (uint32_t i = 0; i < count; i++) {
    ks_status_t st = check_job(pl, jobs[i].evk, jobs[i].level, jobs[i].in, jobs[i].out, workspace,
                               workspace_bytes, need, rows_seeded(rows) ? 1 : 2);
    if (st != KS_OK) return st;
    if (jobs[i].add0) {  // a rotation: its element, and c0 kept apart from every output and the workspace
      if (!galois_ok(pl, jobs[i].galois) || ((uintptr_t)jobs[i].add0 & 15) ||
          overlaps(workspace, workspace_bytes, jobs[i].add0, (size_t)(jobs[i].level + 1) * limb_bytes(pl)))
        return KS_ERR_INVALID_ARG;
      for (uint32_t k = 0; k < count; k++)
        if (overlaps(jobs[k].out, 2 * (size_t)(jobs[k].level + 1) * limb_bytes(pl), jobs[i].add0,
                     (size_t)(jobs[i].level + 1) * limb_bytes(pl)))
          return KS_ERR_INVALID_ARG;
    }
    // no job's output may overlap another job's output or input (either order)
    const size_t ob = 2 * (size_t)(jobs[i].level + 1) * limb_bytes(pl);
    const size_t ib = (size_t)(jobs[i].level + 1) * limb_bytes(pl);
    for (uint32_t k = 0; k < i; k++) {
      const size_t okb = 2 * (size_t)(jobs[k].level + 1) * limb_bytes(pl);
      const size_t ikb = (size_t)(jobs[k].level + 1) * limb_bytes(pl);
      if (overlaps(jobs[i].out, ob, jobs[k].out, okb) || overlaps(jobs[i].out, ob, jobs[k].in, ikb) ||
          overlaps(jobs[k].out, okb, jobs[i].in, ib))
        return KS_ERR_INVALID_ARG;
    }
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl.device) return KS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (!together) {
    for (uint32_t i = 0; i < count; i++) {
      ks_status_t r = run_one(pl, sch, jobs[i], rows, (uint32_t *)workspace, st);
      if (r != KS_OK) return r;
    }
    return KS_OK;
  }
  return run_oc_batch(pl, count, jobs.data(), rows, lay, (char *)workspace, st);
}

}  // namespace

extern "C" {

ks_status_t ks_keyswitch(ks_plan_t plan, const uint32_t *evk, uint32_t level, const uint32_t *in, uint32_t *out,
                         void *workspace, size_t workspace_bytes, void *stream) {
  return keyswitch_one(plan, Job{evk, 0, level, in, out}, OC_ROWS_PLAIN, workspace, workspace_bytes, stream);
}

ks_status_t ks_keyswitch_noalloc(ks_plan_t plan, const uint32_t *evk, uint32_t level, const uint32_t *in,
                                 uint32_t *out, void *stream) {
  if (!plan) return KS_ERR_INVALID_ARG;
  const Plan &pl = plan->p;
  if (pl.cfg.schedule != KS_SCHED_OC && pl.cfg.schedule != KS_SCHED_AUTO) return KS_ERR_UNSUPPORTED;
  if (pl.trace.on) return KS_ERR_UNSUPPORTED;
  if (level >= pl.num_q) return KS_ERR_INVALID_ARG;
  if (ws_limbs(pl, KS_SCHED_OC, level) * limb_bytes(pl) > KS_NOALLOC_SCRATCH_BYTES) return KS_ERR_BUDGET;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl.device) return KS_ERR_INVALID_ARG;
  void *ws = noalloc_scratch(dev);
  if (!ws) return KS_ERR_DEVICE;
  return keyswitch_one(plan, Job{evk, 0, level, in, out}, OC_ROWS_PLAIN, ws, KS_NOALLOC_SCRATCH_BYTES, stream, true);
}

ks_status_t ks_keyswitch_seeded(ks_plan_t plan, const uint32_t *evk_b, uint64_t a_seed, uint32_t level,
                                const uint32_t *in, uint32_t *out, void *workspace, size_t workspace_bytes,
                                void *stream) {
  return keyswitch_one(plan, Job{evk_b, a_seed, level, in, out}, OC_ROWS_SEEDED, workspace, workspace_bytes, stream);
}

ks_status_t ks_keyswitch_batch(ks_plan_t plan, uint32_t count, const ks_job_t *jobs, void *workspace,
                               size_t workspace_bytes, void *stream) {
  if (!plan || (count && !jobs)) return KS_ERR_INVALID_ARG;
  if (injected_fault()) return KS_ERR_DEVICE;
  std::vector<Job> jb(count);
  for (uint32_t i = 0; i < count; i++) jb[i] = Job{jobs[i].evk, 0, jobs[i].level, jobs[i].in, jobs[i].out};
  return keyswitch_batch(plan, jb, OC_ROWS_PLAIN, workspace, workspace_bytes, stream);
}

ks_status_t ks_keyswitch_batch_seeded(ks_plan_t plan, uint32_t count, const ks_seeded_job_t *jobs, void *workspace,
                                      size_t workspace_bytes, void *stream) {
  if (!plan || (count && !jobs)) return KS_ERR_INVALID_ARG;
  if (injected_fault()) return KS_ERR_DEVICE;
  std::vector<Job> jb(count);
  for (uint32_t i = 0; i < count; i++) jb[i] = Job{jobs[i].evk_b, jobs[i].a_seed, jobs[i].level, jobs[i].in, jobs[i].out};
  return keyswitch_batch(plan, jb, OC_ROWS_SEEDED, workspace, workspace_bytes, stream);
}

ks_status_t ks_rotate_batch(ks_plan_t plan, uint32_t count, const ks_rotate_job_t *jobs, void *workspace,
                            size_t workspace_bytes, void *stream) {
  if (!plan || (count && !jobs)) return KS_ERR_INVALID_ARG;
  if (injected_fault()) return KS_ERR_DEVICE;
  std::vector<Job> jb(count);
  for (uint32_t i = 0; i < count; i++) {
    if (!jobs[i].c0) return KS_ERR_INVALID_ARG;
    jb[i] = Job{jobs[i].evk, 0, jobs[i].level, jobs[i].c1, jobs[i].out, jobs[i].galois, jobs[i].c0};
  }
  return keyswitch_batch(plan, jb, OC_ROWS_EXT, workspace, workspace_bytes, stream);
}

ks_status_t ks_automorphism(ks_plan_t plan, uint32_t galois, uint32_t count, const uint32_t *in, uint32_t *out,
                            void *stream) {
  if (!plan) return KS_ERR_INVALID_ARG;
  const Plan &pl = plan->p;
  if (!galois_ok(pl, galois)) return KS_ERR_INVALID_ARG;
  if (!count) return KS_OK;
  if (!in || !out || (((uintptr_t)in | (uintptr_t)out) & 3)) return KS_ERR_INVALID_ARG;
  const size_t b = (size_t)count * limb_bytes(pl);
  if (overlaps(in, b, out, b)) return KS_ERR_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl.device) return KS_ERR_INVALID_ARG;
  return dev_err(launch_automorphism(pl, galois, count, in, out, (hipStream_t)stream));
}

ks_status_t ks_rotate_workspace_size(ks_plan_t plan, uint32_t level, uint32_t count, size_t *bytes) {
  if (!plan || !bytes || level >= plan->p.num_q) return KS_ERR_INVALID_ARG;
  *bytes = rot_layout(plan->p, level, count).total;
  return KS_OK;
}

}  // extern "C"

namespace {

// One rotation of a hoisted group: full key (a_seed unused) or compressed key.
struct Rot {
  const uint32_t *evk;
  uint64_t a_seed;
  uint32_t galois;
  uint32_t *out;
};

ks_status_t rotate_hoisted(ks_plan_t plan, uint32_t level, const uint32_t *c0, const uint32_t *c1,
                           const std::vector<Rot> &rots, bool seeded, void *workspace, size_t workspace_bytes,
                           void *stream) {
  if (!plan) return KS_ERR_INVALID_ARG;
  Plan &pl = plan->p;
  if (effective(pl) != KS_SCHED_OC) return KS_ERR_UNSUPPORTED;
  if (level >= pl.num_q) return KS_ERR_INVALID_ARG;
  const uint32_t count = (uint32_t)rots.size();
  if (!count) return KS_OK;
  if (!c0 || !c1 || !workspace) return KS_ERR_INVALID_ARG;
  if ((((uintptr_t)c0 | (uintptr_t)c1) & 15) || ((uintptr_t)workspace & 255)) return KS_ERR_INVALID_ARG;
  const RotLayout lay = rot_layout(pl, level, count);
  if (workspace_bytes < lay.total) return KS_ERR_BUDGET;
  const size_t lb = limb_bytes(pl), in_b = (size_t)(level + 1) * lb, out_b = 2 * in_b;
  const size_t evk_b = (size_t)pl.dnum * (seeded ? 1 : 2) * pl.ntot * lb;
  if (overlaps(workspace, workspace_bytes, c0, in_b) || overlaps(workspace, workspace_bytes, c1, in_b))
    return KS_ERR_INVALID_ARG;
  for (uint32_t r = 0; r < count; r++) {
    const Rot &x = rots[r];
    if (!x.evk || !x.out || (((uintptr_t)x.evk | (uintptr_t)x.out) & 15) || !galois_ok(pl, x.galois))
      return KS_ERR_INVALID_ARG;
    if (overlaps(x.out, out_b, c0, in_b) || overlaps(x.out, out_b, c1, in_b) ||
        overlaps(x.out, out_b, workspace, workspace_bytes) || overlaps(workspace, workspace_bytes, x.evk, evk_b))
      return KS_ERR_INVALID_ARG;
    for (uint32_t u = 0; u < count; u++)
      if (overlaps(x.out, out_b, rots[u].evk, evk_b) || (u != r && overlaps(x.out, out_b, rots[u].out, out_b)))
        return KS_ERR_INVALID_ARG;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl.device) return KS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  char *ws = (char *)workspace;
  const uint32_t tt = oc_tt(pl, level + 1);
  std::vector<OcJob> hj(count);
  for (uint32_t r = 0; r < count; r++) {
    OcJob &j = hj[r];
    j = make_oc_job(pl, Job{rots[r].evk, rots[r].a_seed, level, c1, rots[r].out}, (uint32_t *)(ws + lay.xt), tt);
    j.xt = (uint32_t *)(ws + lay.xt);  // shared: one ModUp for every rotation
    j.ycol = (uint32_t *)(ws + lay.ycol);
    j.zp = (uint32_t *)(ws + lay.rot0 + r * lay.per_rot);
    j.wcol = j.zp + (size_t)2 * pl.num_p * pl.n;
    j.galois = rots[r].galois;
    j.add0 = c0;
  }
  TRY(upload_async(pl, ws, hj.data(), hj.size() * sizeof(OcJob), st));
  const OcJob none{};
  const OcJob *djobs = (const OcJob *)ws;
  const OcRowVariant rows = seeded ? OC_ROWS_SEEDED_EXT : OC_ROWS_EXT;
  TRY(launch_oc_phases(pl, none, djobs, 1, hj[0].tiles, tt, rows, OC_PART_MODUP, st));
  return dev_err(launch_oc_phases(pl, none, djobs, count, hj[0].tiles, tt, rows, OC_PART_REST, st));
}

}  // namespace

extern "C" {

ks_status_t ks_rotate_hoisted(ks_plan_t plan, uint32_t level, const uint32_t *c0, const uint32_t *c1, uint32_t count,
                              const ks_rotation_t *rots, void *workspace, size_t workspace_bytes, void *stream) {
  if (count && !rots) return KS_ERR_INVALID_ARG;
  std::vector<Rot> r(count);
  for (uint32_t i = 0; i < count; i++) r[i] = Rot{rots[i].evk, 0, rots[i].galois, rots[i].out};
  return rotate_hoisted(plan, level, c0, c1, r, false, workspace, workspace_bytes, stream);
}

ks_status_t ks_rotate_hoisted_seeded(ks_plan_t plan, uint32_t level, const uint32_t *c0, const uint32_t *c1,
                                     uint32_t count, const ks_seeded_rotation_t *rots, void *workspace,
                                     size_t workspace_bytes, void *stream) {
  if (count && !rots) return KS_ERR_INVALID_ARG;
  std::vector<Rot> r(count);
  for (uint32_t i = 0; i < count; i++) r[i] = Rot{rots[i].evk_b, rots[i].a_seed, rots[i].galois, rots[i].out};
  return rotate_hoisted(plan, level, c0, c1, r, true, workspace, workspace_bytes, stream);
}

ks_status_t ks_rotate_sum_workspace_size(ks_plan_t plan, uint32_t level, uint32_t count, size_t *bytes) {
  if (!plan || !bytes || level >= plan->p.num_q) return KS_ERR_INVALID_ARG;
  *bytes = sum_layout(plan->p, level, count).total;
  return KS_OK;
}

ks_status_t ks_rotate_sum_hoisted(ks_plan_t plan, uint32_t level, const uint32_t *c0, const uint32_t *c1,
                                  uint32_t count, const ks_rotation_term_t *terms, uint32_t *out, void *workspace,
                                  size_t workspace_bytes, void *stream) {
  if (!plan) return KS_ERR_INVALID_ARG;
  const Plan &pl = plan->p;
  if (level >= pl.num_q) return KS_ERR_INVALID_ARG;
  if (!count) return KS_OK;
  if (!terms || !c0 || !c1 || !out || !workspace) return KS_ERR_INVALID_ARG;
  if ((((uintptr_t)c0 | (uintptr_t)c1 | (uintptr_t)out) & 15) || ((uintptr_t)workspace & 255))
    return KS_ERR_INVALID_ARG;
  const SumLayout lay = sum_layout(pl, level, count);
  if (workspace_bytes < lay.total) return KS_ERR_BUDGET;
  const size_t lb = limb_bytes(pl), in_b = (size_t)(level + 1) * lb, out_b = 2 * in_b;
  const size_t evk_b = (size_t)pl.dnum * 2 * pl.ntot * lb, diag_b = (size_t)pl.ntot * lb;
  if (overlaps(out, out_b, c0, in_b) || overlaps(out, out_b, c1, in_b) ||
      overlaps(out, out_b, workspace, workspace_bytes) || overlaps(workspace, workspace_bytes, c0, in_b) ||
      overlaps(workspace, workspace_bytes, c1, in_b))
    return KS_ERR_INVALID_ARG;
  std::vector<RotTerm> ht(count);
  for (uint32_t r = 0; r < count; r++) {
    const ks_rotation_term_t &x = terms[r];
    if (!x.evk || (((uintptr_t)x.evk | (uintptr_t)x.diag) & 15) || !galois_ok(pl, x.galois))
      return KS_ERR_INVALID_ARG;
    if (overlaps(out, out_b, x.evk, evk_b) || overlaps(workspace, workspace_bytes, x.evk, evk_b))
      return KS_ERR_INVALID_ARG;
    if (x.diag && (overlaps(out, out_b, x.diag, diag_b) || overlaps(workspace, workspace_bytes, x.diag, diag_b)))
      return KS_ERR_INVALID_ARG;
    ht[r] = RotTerm{x.evk, x.diag, x.galois, 0};
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl.device) return KS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  char *ws = (char *)workspace;
  uint32_t *X = (uint32_t *)(ws + lay.x), *Y = (uint32_t *)(ws + lay.y), *ACC = (uint32_t *)(ws + lay.acc);
  uint32_t *XP = (uint32_t *)(ws + lay.xp), *W = (uint32_t *)(ws + lay.w);
  const RotTerm *dterms = (const RotTerm *)ws;
  TRY(upload_async(pl, ws, ht.data(), ht.size() * sizeof(RotTerm), st));
  if (effective(pl) == KS_SCHED_OC) {
    // fused: the OC phases with summing row stages, one job whose regions
    // follow the term table (the OC regions are smaller than the MP ones)
    const uint32_t tt = oc_tt(pl, level + 1);
    OcJob j = make_oc_job(pl, Job{terms[0].evk, 0, level, c1, out}, X, tt);
    j.add0 = c0;
    j.terms = dterms;
    j.nterm = count;
    return dev_err(launch_oc_phases(pl, j, nullptr, 1, j.tiles, tt, OC_ROWS_SUM, OC_PART_ALL, st));
  }
  TRYK(mp_modup(pl, level, c1, X, Y, st));
  TRY(launch_rotsum_keymul(pl, level, c1, Y, dterms, count, ACC, st));
  TRYK(mp_moddown(pl, level, ACC, XP, W, out, st));
  return dev_err(launch_rotsum_c0(pl, level, c0, dterms, count, out, st));
}

ks_status_t ks_mult_workspace_size(ks_plan_t plan, uint32_t level, size_t *bytes) {
  if (!plan || !bytes || level >= plan->p.num_q) return KS_ERR_INVALID_ARG;
  *bytes = mult_bytes(plan->p, level);
  return KS_OK;
}

ks_status_t ks_mult_relin(ks_plan_t plan, const uint32_t *evk, uint32_t level, const uint32_t *a0, const uint32_t *a1,
                          const uint32_t *b0, const uint32_t *b1, uint32_t *out, void *workspace,
                          size_t workspace_bytes, void *stream) {
  if (!plan) return KS_ERR_INVALID_ARG;
  const Plan &pl = plan->p;
  if (effective(pl) != KS_SCHED_OC) return KS_ERR_UNSUPPORTED;
  if (level >= pl.num_q || !evk || !a0 || !a1 || !b0 || !b1 || !out || !workspace) return KS_ERR_INVALID_ARG;
  if ((((uintptr_t)evk | (uintptr_t)a0 | (uintptr_t)a1 | (uintptr_t)b0 | (uintptr_t)b1 | (uintptr_t)out) & 15) ||
      ((uintptr_t)workspace & 255))
    return KS_ERR_INVALID_ARG;
  if (workspace_bytes < mult_bytes(pl, level)) return KS_ERR_BUDGET;
  const size_t lb = limb_bytes(pl), in_b = (size_t)(level + 1) * lb, out_b = 2 * in_b;
  const size_t evk_b = (size_t)pl.dnum * 2 * pl.ntot * lb;
  const void *ins[4] = {a0, a1, b0, b1};
  for (const void *x : ins)
    if (overlaps(out, out_b, x, in_b) || overlaps(workspace, workspace_bytes, x, in_b)) return KS_ERR_INVALID_ARG;
  if (overlaps(out, out_b, evk, evk_b) || overlaps(out, out_b, workspace, workspace_bytes) ||
      overlaps(workspace, workspace_bytes, evk, evk_b))
    return KS_ERR_INVALID_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl.device) return KS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  uint32_t *d = (uint32_t *)workspace;
  const size_t limbs = (size_t)(level + 1) * pl.n;
  TRY(launch_tensor(pl, level, a0, a1, b0, b1, d, st));
  const uint32_t tt = oc_tt(pl, level + 1);
  OcJob j = make_oc_job(pl, Job{evk, 0, level, d + 2 * limbs, out},
                        (uint32_t *)((char *)workspace + mult_tensor_bytes(pl, level)), tt);
  j.add0 = d;
  j.add1 = d + limbs;
  return dev_err(launch_oc_phases(pl, j, nullptr, 1, j.tiles, tt, OC_ROWS_EXT, OC_PART_ALL, st));
}

ks_status_t ks_expand_seeded_a(ks_plan_t plan, uint64_t a_seed, uint32_t *evk, void *stream) {
  if (!plan || !evk || ((uintptr_t)evk & 15)) return KS_ERR_INVALID_ARG;
  const Plan &pl = plan->p;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl.device) return KS_ERR_INVALID_ARG;
  return dev_err(launch_expand_a(pl, a_seed, evk, (hipStream_t)stream));
}

ks_status_t ks_batch_status(ks_plan_t plan, const void *workspace, void *stream, uint32_t *error_flag) {
  if (!plan || !workspace || !error_flag) return KS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  uint32_t ctl[2] = {0, 0};
  if (hipStreamSynchronize(st) != hipSuccess) return KS_ERR_DEVICE;
  if (hipMemcpy(ctl, workspace, sizeof(ctl), hipMemcpyDeviceToHost) != hipSuccess) return KS_ERR_DEVICE;
  *error_flag = ctl[1] ? 1u : 0u;
  return KS_OK;
}

ks_status_t ks_ntt(ks_plan_t plan, uint32_t count, const uint32_t *g, int inverse, uint32_t *data, void *stream) {
  if (!plan || (count && (!g || !data))) return KS_ERR_INVALID_ARG;
  const Plan &pl = plan->p;
  std::vector<uint32_t> off(count), gv(count);
  for (uint32_t c = 0; c < count; c++) {
    if (g[c] >= pl.ntot) return KS_ERR_INVALID_ARG;
    off[c] = c;
    gv[c] = g[c];
  }
  hipStream_t st = (hipStream_t)stream;
  TRY(launch_ntt(pl, inverse != 0, data, data, off, off, gv, st));
  for (uint32_t b = 0; b < count; b += kMaxList) {
    LimbList L{};
    L.count = std::min(count - b, kMaxList);
    for (uint32_t c = 0; c < L.count; c++) { L.dst_off[c] = b + c; L.g[c] = (uint16_t)g[b + c]; }
    TRY(launch_finish_ntt(pl, inverse != 0, data, L, st));
  }
  return KS_OK;
}

ks_status_t ks_trace_enable(ks_plan_t plan, int on) {
  if (!plan) return KS_ERR_INVALID_ARG;
  Trace &t = plan->p.trace;
  std::lock_guard<std::mutex> g(t.mu);
  t.on = on != 0;
  return KS_OK;
}

ks_status_t ks_trace_read(ks_plan_t plan, uint32_t max, const char **names, uint32_t *launches, double *total_ms,
                          uint32_t *count) {
  if (!plan || !count || (max && (!names || !launches || !total_ms))) return KS_ERR_INVALID_ARG;
  Trace &t = plan->p.trace;
  std::lock_guard<std::mutex> g(t.mu);
  std::vector<const char *> nm;
  std::vector<uint32_t> ln;
  std::vector<double> ms;
  ks_status_t st = KS_OK;
  if (!t.marks.empty() && hipEventSynchronize(t.marks.back().stop) != hipSuccess) st = KS_ERR_DEVICE;
  for (size_t i = 0; st == KS_OK && i < t.marks.size(); i++) {
    const char *name = t.marks[i].stage;
    float e = 0;
    if (hipEventElapsedTime(&e, t.marks[i].start, t.marks[i].stop) != hipSuccess) { st = KS_ERR_DEVICE; break; }
    size_t k = 0;
    while (k < nm.size() && std::strcmp(nm[k], name) != 0) k++;
    if (k == nm.size()) { nm.push_back(name); ln.push_back(0); ms.push_back(0); }
    ln[k]++;
    ms[k] += e;
  }
  for (auto &m : t.marks) { t.pool.push_back(m.start); t.pool.push_back(m.stop); }
  t.marks.clear();
  *count = (uint32_t)nm.size();
  for (uint32_t k = 0; k < nm.size() && k < max; k++) {
    names[k] = nm[k];
    launches[k] = ln[k];
    total_ms[k] = ms[k];
  }
  return st;
}

}  // extern "C"
