/*
 * ks.h -- C ABI of the MI355X (gfx950) hybrid key-switching library.
 *
 * The operation (CiFlow, Sec. III): given a polynomial d in R_{Q_l} in the
 * evaluation domain that decrypts under a key s2, and an evaluation key evk
 * for s2 -> s, return (c0, c1) in R_{Q_l} with c0 + c1 s ~ d s2 (mod Q_l).
 * Steps: digit decomposition into dnum digits of alpha towers (Sec. III-A),
 * ModUp P1 INTT, P2 fast basis conversion to D_l = Q_l u P, P3 NTT, P4
 * multiply by evk, P5 sum over digits (Sec. III-B), then ModDown P1 INTT of
 * the K special towers, P2 conversion back to Q_l, P3 NTT, P4 subtract and
 * multiply by P^-1 mod q_i (Sec. III-C).  Three execution orders of the same
 * computation are available (Sec. IV): Max-Parallel, Digit-Centric and
 * Output-Centric; all return identical bits.
 *
 * Conventions shared by every entry point:
 *  - Residues are uint32, canonical in [0, m), moduli are primes with
 *    2^29 < m < 2^30 and m = 1 mod 2N.  Inputs outside [0, m) give
 *    unspecified (but memory-safe) outputs.
 *  - Polynomials are limb-major: [towers][N].  The evaluation domain is
 *    NTT(a)[j] = a(psi^(2 brv(j) + 1)) with psi the smallest primitive 2N-th
 *    root of unity mod m and brv the log2(N)-bit reversal.
 *  - Moduli order: q_0..q_L then p_0..p_{K-1}.  Unless given explicitly, the
 *    moduli are the primes 2^30 - t*2N + 1, t = 1, 2, ..., the first K
 *    becoming p_0..p_{K-1} and the next L+1 becoming q_0..q_L.
 *  - evk layout: [dnum][2][L+1+K][N] (Sec. III-B P4: dnum x 2 x N x (l+K)),
 *    pair index 0 = b_j, 1 = a_j, with b_j + a_j s = e_j + g_j s2 where g_j is
 *    [P]_m on digit j's own q-limbs and 0 on every other limb.
 *  - Device pointers are HIP device addresses on the plan's device; the
 *    caller owns every buffer (inputs, outputs, evk, workspace).  `stream` is
 *    a hipStream_t (NULL = default stream).  Calls are asynchronous on the
 *    stream; argument errors are reported synchronously before anything is
 *    enqueued; launch failures return KS_ERR_DEVICE.
 *  - No call aborts or throws across the ABI.
 */
#ifndef KS_H
#define KS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KS_OK = 0,
  KS_ERR_INVALID_ARG = 1,  /* bad pointer, size, level, alias, modulus */
  KS_ERR_UNSUPPORTED = 2,  /* valid, but not supported by this library */
  KS_ERR_NOMEM = 3,        /* device or host allocation failed */
  KS_ERR_BUDGET = 4,       /* workspace smaller than ks_workspace_size() */
  KS_ERR_DEVICE = 5        /* a HIP call or kernel launch failed */
} ks_status_t;

/* Execution orders of Sec. IV. */
typedef enum {
  KS_SCHED_AUTO = 0,  /* per call, the autotuner's entry for the call's shape
                         (ks_plan_set_tuned); OC when nothing is tuned */
  KS_SCHED_MP = 1,    /* Max-Parallel, Sec. IV-A: each stage over all towers */
  KS_SCHED_DC = 2,    /* Digit-Centric, Sec. IV-B: one digit at a time */
  KS_SCHED_OC = 3     /* Output-Centric, Sec. IV-C: one output tower tile at a time */
} ks_schedule_t;

/* Parameter set (Table I).  log_n in [12, 17]; num_q = L+1 >= 1;
 * 1 <= dnum <= min(num_q, 16) (alpha = ceil(num_q/dnum) <= 32); num_p = K
 * (0 => alpha, at most 32); num_q + num_p <= 128.  `moduli` is an optional host array of
 * num_q + num_p values (q_0..q_L, p_0..p_{K-1}); NULL selects the default
 * primes.  Explicit moduli are validated: prime, 2^29 < m < 2^30,
 * m = 1 mod 2N, pairwise distinct. */
typedef struct {
  uint32_t log_n;
  uint32_t num_q;
  uint32_t dnum;
  uint32_t num_p;
  const uint32_t *moduli;
} ks_params_t;

/* Launch configuration (what the autotuner chooses).  Zero fields keep the
 * plan's current value. */
typedef struct {
  ks_schedule_t schedule;
  uint32_t tile_towers;  /* OC: target towers per basis-conversion tile (1, 2;
                            4 is accepted and runs as 2).  Where a column
                            holds 32 elements per thread (N = 2^13, and
                            N = 2^17 when the launch's largest job has fewer
                            than 17 towers) the tiles take one target */
  uint32_t col_width;    /* MP/DC: columns per column-pass workgroup (8, 16, 32) */
  uint32_t row_block;    /* MP/DC: rows per row-pass workgroup (4, 8, 16) */
  uint32_t batch_mode;   /* OC batches: 1 = one launch per phase over all jobs,
                            2 = one persistent work-queue launch (currently
                            switched off: KS_ERR_UNSUPPORTED), 3 = as 1 but
                            the second half of the jobs on a second stream
                            owned by the plan (forked from and joined back
                            to `stream` with events) */
  uint32_t graph;        /* OC batches: 1 = capture the phase launches (modes 1
                            and 3) once per (count, workspace, configuration,
                            tile counts) in a hipGraph and replay it, 2 =
                            launch directly */
  uint32_t spin_limit;   /* persistent launch: polls before a dependency wait
                            gives up and flags an error (tests use tiny values) */
  uint32_t batch_order;  /* OC batches: 1 = jobs in the caller's order, 2 = by
                            decreasing level (results are the same) */
} ks_config_t;

typedef struct ks_plan *ks_plan_t;

/* One ciphertext component of a batch: `in` [level+1][N], `out`
 * [2][level+1][N], `evk` [dnum][2][L+1+K][N] (device pointers). */
typedef struct {
  const uint32_t *evk;
  uint32_t level;
  const uint32_t *in;
  uint32_t *out;
} ks_job_t;

/* Host only, needs no device: the moduli a plan with these parameters uses
 * (default primes, or the validated explicit list), written to host_out
 * [num_q + num_p].  Sec. II (RNS towers of word-size moduli). */
ks_status_t ks_params_moduli(const ks_params_t *p, uint32_t *host_out);

/* Host only, needs no device; for tests of the (switched-off) persistent
 * batch launch's work list, the tables it would run: for `count` jobs at
 * `levels`, tiles [count][8] = tile count of every Output-Centric phase
 * (one target per conversion tile), the segments in launch order (phase-major,
 * then job-major; count * 8 of them) as seg_start / seg_job / seg_phase,
 * deps [8] = bit mask of the phases each phase waits for (same job), and
 * *total = the number of work items. */
ks_status_t ks_oc_work_list(const ks_params_t *p, uint32_t count, const uint32_t *levels, uint32_t *tiles,
                            uint32_t *seg_start, uint32_t *seg_job, uint32_t *seg_phase, uint32_t *deps,
                            uint32_t *total);

/* Host only: psi for modulus q at ring degree 2^log_n (the smallest
 * primitive 2N-th root of unity), or 0 if q is not a prime = 1 mod 2N. */
uint32_t ks_root_of_unity(uint32_t q, uint32_t log_n);

/* Create a plan on the current HIP device: derive moduli and psi, build the
 * twiddle, basis-conversion and ModDown tables (Sec. III-B/C) and upload
 * them.  *out owns them until ks_plan_destroy.  The plan starts with the
 * configuration {OC, tile_towers 2, col_width 16, row_block 8, batch_mode 1,
 * graph 2, spin_limit 0, batch_order 1}: two targets per conversion tile
 * equal one target for a single key switch and are faster for batches.
 * Where a column holds 32 elements per thread the tiles take one target at
 * N = 2^13, and at N = 2^17 when the launch's largest job has fewer than
 * 17 towers (two from 17 towers up). */
ks_status_t ks_plan_create(const ks_params_t *p, ks_plan_t *out);
ks_status_t ks_plan_destroy(ks_plan_t plan);
/* Moduli of the plan, host_out [num_q + num_p]. */
ks_status_t ks_plan_moduli(ks_plan_t plan, uint32_t *host_out);
ks_status_t ks_plan_set_config(ks_plan_t plan, const ks_config_t *cfg);
ks_status_t ks_plan_get_config(ks_plan_t plan, ks_config_t *cfg);

/* Autotuner results (the tuning layer above the paper's method: every
 * configuration computes the same bits, Sec. IV, so tuning only measures
 * time).  ks_plan_set_tuned records the configuration (schedule MP, DC or
 * OC; zero fields mean "the plan's value at call time") for calls of `count`
 * key switches (count >= 1) whose largest level is `level`.  While the
 * plan's schedule is KS_SCHED_AUTO, ks_keyswitch (count 1),
 * ks_keyswitch_batch and ks_workspace_size take the entry for the call's
 * shape: the same level, else the nearest tuned level (the higher on a tie);
 * among those, the largest tuned count not above the call's count, else the
 * smallest.  Calls that run the OC order only (compressed keys, rotations,
 * ks_keyswitch_noalloc) take OC with the plan's settings when that entry
 * names another schedule.  ks_plan_resolve_config writes the configuration
 * a call of that shape runs with (never AUTO).  Workspaces must be sized
 * with ks_workspace_size under the same tuned entries. */
ks_status_t ks_plan_set_tuned(ks_plan_t plan, uint32_t level, uint32_t count, const ks_config_t *cfg);
ks_status_t ks_plan_clear_tuned(ks_plan_t plan);
ks_status_t ks_plan_resolve_config(ks_plan_t plan, uint32_t level, uint32_t count, ks_config_t *out);

/* Bytes of device workspace ks_keyswitch (count = 1) or ks_keyswitch_batch
 * needs for jobs at the given levels under the plan's current schedule.
 * `levels` is a host array of `count` levels (each <= L). */
ks_status_t ks_workspace_size(ks_plan_t plan, uint32_t count, const uint32_t *levels, size_t *bytes);

/* Hybrid key switch of one polynomial (Sec. III, order per the plan's
 * schedule, Sec. IV).  in [level+1][N] (device, evaluation domain), out
 * [2][level+1][N] (device; out must not overlap in, evk or workspace),
 * evk [dnum][2][L+1+K][N] (device), workspace >= ks_workspace_size bytes,
 * 256-byte aligned.  Output canonical, evaluation domain. */
ks_status_t ks_keyswitch(ks_plan_t plan, const uint32_t *evk, uint32_t level,
                         const uint32_t *in, uint32_t *out, void *workspace,
                         size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ks_keyswitch without a workspace argument.  The intermediates live in a
 * fixed device array of KS_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends (looked up when a plan is
 * created on that GPU).  Runs the Output-Centric order (the plan's schedule
 * must be OC or AUTO, else KS_ERR_UNSUPPORTED), and its output equals
 * ks_keyswitch's under OC.  A call whose OC workspace (ks_workspace_size of
 * the one level under OC) exceeds KS_NOALLOC_SCRATCH_BYTES returns
 * KS_ERR_BUDGET before enqueuing anything; with kernel tracing on it returns
 * KS_ERR_UNSUPPORTED (tracing creates events).  The call allocates nothing:
 * no hipMalloc, hipFree or other allocating routine.  Every call on one GPU
 * uses that GPU's one array, which keeps the last call's contents (every
 * word a call reads from it was written earlier by the same call): calls
 * that overlap on one GPU (other streams, other host threads) race and must
 * be serialised by the caller.  in/out/evk rules as for ks_keyswitch. */
#define KS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
ks_status_t ks_keyswitch_noalloc(ks_plan_t plan, const uint32_t *evk, uint32_t level,
                                 const uint32_t *in, uint32_t *out, void *stream);

/* Many key switches at mixed levels (jobs is a host array of `count`
 * entries; the key may differ per job).  Each job's output equals
 * ks_keyswitch of that job alone.  Outputs must not overlap each other, any
 * input or the workspace.  With the OC schedule the jobs run together: one
 * launch per phase over all jobs (batch_mode 1), or the same split over two
 * streams (3); with graph = 1 those launches are captured once per (count,
 * workspace, configuration, tile counts) in a hipGraph that later calls
 * replay.  The job table travels in the workspace (uploaded before every
 * launch or replay), so concurrent batches need distinct workspaces.  A count
 * of 0 returns KS_OK and enqueues nothing.  For tests of
 * failure handling, the environment variable KS_FAULT_INJECT=<n> makes the
 * n-th call after the variable took its current value return KS_ERR_DEVICE
 * without enqueuing work. */
ks_status_t ks_keyswitch_batch(ks_plan_t plan, uint32_t count, const ks_job_t *jobs,
                               void *workspace, size_t workspace_bytes, void *stream);

/* Key compression (Sec. IV-D, arithmetic-intensity comparison): the a half
 * of every key pair is pseudo-random, so it can be regenerated from a seed
 * where it is consumed instead of being read from memory, which halves the
 * key traffic of a key switch.  A compressed key is its b halves
 * evk_b [dnum][L+1+K][N] (device, the same order as the b halves of a full
 * key) plus a_seed.  Word k of row g (g in key order q_0..q_L, p_0..p_{K-1})
 * of digit j's a half is x * 2^-32 mod m_g, where x is output t =
 * (j (L+1+K) + g) N + k of SplitMix64 (Steele, Lea and Flood 2014) used as a
 * counter-based generator: x = mix(a_seed + (t + 1) * 0x9e3779b97f4a7c15),
 * mix(z) = z ^= z >> 30, z *= 0xbf58476d1ce4e5b9, z ^= z >> 27,
 * z *= 0x94d049bb133111eb, z ^= z >> 31 (64-bit arithmetic).  The a_seed
 * is public, like the a halves it stands for.
 *
 * ks_keyswitch_seeded: ks_keyswitch with a compressed key; the result equals
 * ks_keyswitch with the expanded key.  OC schedule only: another schedule
 * returns KS_ERR_UNSUPPORTED (expand the key with ks_expand_seeded_a and
 * call ks_keyswitch instead).  Same rules for alignment, overlap (evk_b
 * counts as dnum (L+1+K) N words) and workspace as ks_keyswitch. */
ks_status_t ks_keyswitch_seeded(ks_plan_t plan, const uint32_t *evk_b, uint64_t a_seed, uint32_t level,
                                const uint32_t *in, uint32_t *out, void *workspace,
                                size_t workspace_bytes, void *stream);

/* One job of a batch with a compressed key: evk_b [dnum][L+1+K][N] (device)
 * and its seed; in/out as in ks_job_t. */
typedef struct {
  const uint32_t *evk_b;
  uint64_t a_seed;
  uint32_t level;
  const uint32_t *in;
  uint32_t *out;
} ks_seeded_job_t;

/* ks_keyswitch_batch with compressed keys (every job's); same rules, OC
 * schedule only, KS_FAULT_INJECT counts these calls too. */
ks_status_t ks_keyswitch_batch_seeded(ks_plan_t plan, uint32_t count, const ks_seeded_job_t *jobs,
                                      void *workspace, size_t workspace_bytes, void *stream);

/* Writes the a half of every pair of a full-layout key evk [dnum][2][L+1+K]
 * [N] (device, 16-byte aligned) from a_seed as defined above, enqueued on
 * `stream`; the b halves are not touched.  For key generation (b is
 * computed from a) and for schedules that take full keys only. */
ks_status_t ks_expand_seeded_a(ks_plan_t plan, uint64_t a_seed, uint32_t *evk, void *stream);

/* ----------------------------------------------------------------------
 * Callers of the key switch (Sec. II: rotations and multiplications are
 * what need it).  Galois element k of the automorphism X -> X^k: odd and
 * below 2N (rotation by r slots: k = 5^r mod 2N; conjugation: 2N - 1).
 * In the evaluation domain (slot j holds the value at psi^(2 brv(j) + 1))
 * the automorphism is the permutation out[j] = in[pi(j)] with
 * 2 brv(pi(j)) + 1 = k (2 brv(j) + 1) mod 2N, the same for every modulus.
 * ---------------------------------------------------------------------- */

/* out[c] = automorphism of in[c] for `count` limbs [count][N] (device,
 * 4-byte aligned, out not overlapping in). */
ks_status_t ks_automorphism(ks_plan_t plan, uint32_t galois, uint32_t count, const uint32_t *in,
                            uint32_t *out, void *stream);

/* One rotation of a hoisted group: its key evk [dnum][2][L+1+K][N] switches
 * from s(X^galois) to s; out [2][level+1][N] receives the rotated ciphertext
 * (device pointers). */
typedef struct {
  const uint32_t *evk;
  uint32_t galois;
  uint32_t *out;
} ks_rotation_t;

/* One job of a rotation batch: the ciphertext (c0, c1) [level+1][N] each,
 * its rotation key evk [dnum][2][L+1+K][N] (from s(X^galois) to s) and the
 * output [2][level+1][N] (device pointers). */
typedef struct {
  const uint32_t *evk;
  uint32_t galois;
  uint32_t level;
  const uint32_t *c0;
  const uint32_t *c1;
  uint32_t *out;
} ks_rotate_job_t;

/* Many ciphertexts, each rotated by its own element at its own level, in one
 * launch per phase: the batch of ks_keyswitch_batch with every job a
 * hoisted group of one (its result equals ks_rotate_hoisted of that job
 * alone).  Workspace: ks_workspace_size with the jobs' levels.  Same rules
 * as ks_keyswitch_batch; c0 counts as an input.  OC schedule only. */
ks_status_t ks_rotate_batch(ks_plan_t plan, uint32_t count, const ks_rotate_job_t *jobs, void *workspace,
                            size_t workspace_bytes, void *stream);

/* Bytes of workspace ks_rotate_hoisted needs for `count` rotations at
 * `level` (0 for count 0). */
ks_status_t ks_rotate_workspace_size(ks_plan_t plan, uint32_t level, uint32_t count, size_t *bytes);

/* Hoisted rotations of the ciphertext (c0, c1) [level+1][N] each (device,
 * evaluation domain): ModUp of c1 (Sec. III-B P1-P3) runs once and every
 * rotation r reuses it (hoisting; double hoisting is named in Sec. VII):
 *   acc = sum_j sigma_r(ModUp_j(c1)) * evk_r[j]      (P4, P5)
 *   out_r = (ModDown(acc_0) + sigma_r(c0), ModDown(acc_1))
 * where sigma_r is the evaluation-domain automorphism.  The permutation is
 * applied inside the row stages of the Output-Centric order (a row of 256
 * slots maps onto one row), so nothing is permuted in memory.  OC schedule
 * only (KS_ERR_UNSUPPORTED otherwise).  Outputs must not overlap each
 * other, c0, c1, any key or the workspace; the workspace (>=
 * ks_rotate_workspace_size, 256-byte aligned) must not overlap c0, c1 or a
 * key. */
ks_status_t ks_rotate_hoisted(ks_plan_t plan, uint32_t level, const uint32_t *c0, const uint32_t *c1,
                              uint32_t count, const ks_rotation_t *rots, void *workspace,
                              size_t workspace_bytes, void *stream);

/* One rotation of a hoisted group with a compressed key: the b halves
 * evk_b [dnum][L+1+K][N] (device) and the seed of the a halves, as for
 * ks_keyswitch_seeded. */
typedef struct {
  const uint32_t *evk_b;
  uint64_t a_seed;
  uint32_t galois;
  uint32_t *out;
} ks_seeded_rotation_t;

/* ks_rotate_hoisted with compressed rotation keys (Sec. IV-D key
 * compression applied to the keys of a hoisted group): results equal
 * ks_rotate_hoisted with the expanded keys.  Same rules; a key counts as
 * dnum (L+1+K) N words for the overlap checks. */
ks_status_t ks_rotate_hoisted_seeded(ks_plan_t plan, uint32_t level, const uint32_t *c0, const uint32_t *c1,
                                     uint32_t count, const ks_seeded_rotation_t *rots, void *workspace,
                                     size_t workspace_bytes, void *stream);

/* One term of a double-hoisted rotation sum: the rotation's key evk
 * [dnum][2][L+1+K][N] (from s(X^galois) to s) and an optional plaintext
 * diagonal diag [L+1+K][N] (device, 16-byte aligned, key-row order
 * q_0..q_L, p_0..p_{K-1}, evaluation domain, canonical), or NULL for the
 * constant 1. */
typedef struct {
  const uint32_t *evk;
  uint32_t galois;
  const uint32_t *diag;
} ks_rotation_term_t;

/* Bytes of workspace ks_rotate_sum_hoisted needs (0 for count 0). */
ks_status_t ks_rotate_sum_workspace_size(ks_plan_t plan, uint32_t level, uint32_t count, size_t *bytes);

/* Double hoisting (named in Sec. VII): out = sum_r diag_r * sigma_r((c0, c1))
 * with one ModUp of c1 and one ModDown for the whole sum:
 *   ACC = sum_r diag_r * sum_j sigma_r(ModUp_j(c1)) * evk_r[j]  (extended basis)
 *   out = (ModDown(ACC_0) + sum_r diag_r * sigma_r(c0), ModDown(ACC_1)).
 * The building block of a linear transform's inner sum.  Under the OC
 * schedule the summing is fused into the row stages (each tile sums every
 * term for its rows before its one ModDown); under MP and DC it runs the
 * Max-Parallel stages with the sum in one extended-basis accumulator.  Both
 * give the same bits.  c0, c1 [level+1][N], out
 * [2][level+1][N] (device, 16-byte aligned); out must not overlap an input,
 * a key, a diagonal or the workspace (>= ks_rotate_sum_workspace_size,
 * 256-byte aligned). */
ks_status_t ks_rotate_sum_hoisted(ks_plan_t plan, uint32_t level, const uint32_t *c0, const uint32_t *c1,
                                  uint32_t count, const ks_rotation_term_t *terms, uint32_t *out,
                                  void *workspace, size_t workspace_bytes, void *stream);

/* Bytes of workspace ks_mult_relin needs at `level`. */
ks_status_t ks_mult_workspace_size(ks_plan_t plan, uint32_t level, size_t *bytes);

/* Multiplication with relinearisation (Sec. II): the tensor product of
 * (a0, a1) and (b0, b1) ([level+1][N] each, device, evaluation domain),
 * d = (a0 b0, a0 b1 + a1 b0, a1 b1), then out = (d0, d1) + KS(d2) with evk
 * [dnum][2][L+1+K][N] switching from s^2 to s; the additions are fused into
 * the key switch's last stage.  out [2][level+1][N] must not overlap an
 * input, the key or the workspace.  OC schedule only. */
ks_status_t ks_mult_relin(ks_plan_t plan, const uint32_t *evk, uint32_t level, const uint32_t *a0,
                          const uint32_t *a1, const uint32_t *b0, const uint32_t *b1, uint32_t *out,
                          void *workspace, size_t workspace_bytes, void *stream);

/* After a batch: waits for `stream`, then sets *error_flag to 1 if a
 * dependency wait of the persistent launch exceeded its spin limit (the
 * outputs of that batch are then invalid), else 0. */
ks_status_t ks_batch_status(ks_plan_t plan, const void *workspace, void *stream, uint32_t *error_flag);

/* Stage access for tests and tools: in-place forward (inverse = 0) or
 * inverse (inverse = 1, including the N^-1 factor) negacyclic NTT of
 * `count` limbs data[count][N] (device), limb c taken modulo the plan's
 * modulus number g[c] (host array, global index: q_0..q_L, p_0..p_{K-1}).
 * ModUp P1/P3 and ModDown P1/P3 use the same transform. */
ks_status_t ks_ntt(ks_plan_t plan, uint32_t count, const uint32_t *g, int inverse,
                   uint32_t *data, void *stream);

/* Tracing for tools (not part of the method): while enabled, the plan
 * records a HIP event on the launch stream before every kernel it enqueues
 * and one after each key switch, so event-to-event intervals time each
 * kernel on the stream it runs on.  Enabling clears nothing; reading
 * synchronises on the last event, returns per stage name the number of
 * launches and total milliseconds (up to `max` entries, `*count` = number of
 * distinct names) and clears the record.  names[i] are static strings. */
ks_status_t ks_trace_enable(ks_plan_t plan, int on);
ks_status_t ks_trace_read(ks_plan_t plan, uint32_t max, const char **names, uint32_t *launches,
                          double *total_ms, uint32_t *count);

/* Roofline probes for tools: on the current device, lane-operations per
 * second of long independent chains of single instructions v_add_u32,
 * v_mul_lo_u32, v_mul_hi_u32, v_mad_u64_u32, v_fma_f64 (out[0..4]), the
 * bytes per second of a 1 GiB device-to-device copy kernel (out[5], read +
 * write), and lazy modular butterflies per second (out[6]).  out must hold 7
 * doubles.  Allocates and frees 2 GiB of device memory; synchronous. */
ks_status_t ks_device_rates(double *out, void *stream);

/* Range checks for tools (not part of the method).  The library is also
 * built as libks_check.so with every lazy-range and accumulator bound the
 * exact arithmetic relies on tested where it is used: butterfly inputs
 * ([0, 4q) / [0, 2q) for 30-bit words, [0, 8q) / [0, 4q) for 64-bit ones),
 * Shoup products, multiply-accumulate operands below 2^30 and sums that do
 * not wrap, REDC inputs and outputs.  A violation is counted on the device
 * and the computation goes on.  ks_range_violations returns, for the
 * current device, the number of violations since the last reset and the
 * code of one of them (0 if none; the codes are listed in
 * csrc/range_check.h), clearing the counters when `reset` is nonzero; it
 * synchronises with the device's work.  ks_range_set_strict(1) makes the
 * REDC check demand results below q/2, which ordinary inputs violate, so a
 * caller can see that the counters are live.  libks.so compiles the checks
 * out and returns KS_ERR_UNSUPPORTED from both. */
ks_status_t ks_range_violations(uint32_t *count, uint32_t *code, int reset);
ks_status_t ks_range_set_strict(int on);

/* Arithmetic probes for tests (not part of the method): the kernels'
 * modular primitives applied element-wise, so that each can be compared
 * with a b mod q directly.  a, b: n device words each (any values); each
 * primitive gets them reduced into the range it is specified for; out:
 * device, n x 8 (30-bit) or n x 9 (64-bit) words, element-major.
 * Asynchronous on `stream`.  Errors: null pointers, n = 0, or q outside
 * the word size's modulus range (odd, 2^29 < q < 2^30, resp. 2^59 < q <
 * 2^60; and w < q for the 64-bit probe) give KS_ERR_INVALID_ARG.
 * 30-bit (w: n device words, reduced mod q; its Shoup companion derived on
 * the device as the transform tiles derive it):
 *   0: a w mod q (Shoup, any a < 2^32), canonical;
 *   1: (a mod q)(b mod q) 2^-32 mod q (one product, REDC), canonical;
 *   2: sum over k < 16 of (a_j mod q)(b_j mod q), j = (i + k) mod n, times
 *      2^-32 mod q (a full chunk of products, one REDC), canonical;
 *   3, 4: the forward butterfly of (x, y) = (a mod 4q, b mod 4q):
 *      x + w y and x - w y mod q, each in [0, 4q);
 *   5, 6: the inverse butterfly of (u, v) = (a mod 2q, b mod 2q):
 *      u + v and (u - v) w mod q, each in [0, 2q);
 *   7: (a mod 4q) mod q through the [0, 4q) -> [0, q) reduction.
 * 64-bit (one twiddle w < q for all elements; its companion computed on the
 * host as the plan computes it):
 *   0: a w mod q (Shoup), canonical;  1: a w mod q with the estimated
 *      quotient, in [0, 4q);
 *   2: (a mod q)(b mod q) 2^-64 mod q (30-bit-half products, REDC);
 *   3: the same for the 16 products from element i on (cyclically);
 *   4, 5: the forward butterfly of (a mod 8q, b mod 8q), each in [0, 8q);
 *   6, 7: the inverse butterfly of (a mod 4q, b mod 4q), each in [0, 4q);
 *   8: (a mod 8q) mod q through the forward transform's last reduction. */
ks_status_t ks_arith_probe(uint32_t q, uint32_t n, const uint32_t *a, const uint32_t *b, const uint32_t *w,
                           uint32_t *out, void *stream);
ks_status_t ks64_arith_probe(uint64_t q, uint64_t w, uint32_t n, const uint64_t *a, const uint64_t *b,
                             uint64_t *out, void *stream);

/* Cost model of the autotuner (not part of the key switch): an fp32 MLP
 * with F inputs, two hidden layers of H units with ReLU, and one linear
 * output.  Parameters are one device float array of ks_mlp_param_count(F,H)
 * values laid out W1[F][H], b1[H], W2[H][H], b2[H], W3[H], b3.  X is
 * [B][F], Y and T are [B].  `act` ([2][B][H]) receives the post-ReLU hidden
 * activations the backward pass needs; `scratch` is [2][B][H].  All
 * pointers are device pointers; calls are asynchronous on `stream`;
 * reductions are deterministic.  F <= 256, H <= 1024. */
uint32_t ks_mlp_param_count(uint32_t F, uint32_t H);
ks_status_t ks_mlp_forward(uint32_t F, uint32_t H, uint32_t B, const float *params, const float *X, float *Y,
                           float *act, void *stream);
/* dY = 2 (Y - T) / B and *loss = mean((Y - T)^2) (loss is a device float). */
ks_status_t ks_mlp_mse_grad(uint32_t B, const float *Y, const float *T, float *dY, float *loss, void *stream);
/* Gradients of the loss with respect to every parameter, given dY and the
 * activations of the matching forward call; grads has the params layout. */
ks_status_t ks_mlp_backward(uint32_t F, uint32_t H, uint32_t B, const float *params, const float *X,
                            const float *act, const float *dY, float *grads, float *scratch, void *stream);
/* One Adam step (Kingma & Ba) on n parameters; step counts from 1. */
ks_status_t ks_mlp_adam(uint32_t n, float *params, const float *grads, float *m, float *v, float lr, float beta1,
                        float beta2, float eps, uint32_t step, void *stream);

const char *ks_status_string(ks_status_t s);

/* ------------------------------------------------------------------------
 * 64-bit words.  The same key switch (Sec. III) on towers of ~60-bit primes
 * held in uint64 words: Sec. II's word-size moduli (36 to 64 bits), the word
 * size Table III's evk sizes count.  Moduli: primes 2^59 < m < 2^60 with
 * m = 1 mod 2N; by default 2^60 - t*2N + 1, t = 1, 2, ..., the first K
 * becoming p_0..p_{K-1} and the next L+1 q_0..q_L.  psi is the smallest x
 * with x^N = -1 (mod m); the evaluation domain, evk layout, digits and
 * output conventions are those above, with uint64 residues.  Runs the
 * Max-Parallel order (Sec. IV-A): every stage over all towers, each stage's
 * output in the workspace, with the row pass of a transform fused into the
 * key multiply-accumulate or the ModDown epilogue it feeds.  Parameter
 * limits as for ks_params_t.
 * ------------------------------------------------------------------------ */
typedef struct {
  uint32_t log_n;
  uint32_t num_q;
  uint32_t dnum;
  uint32_t num_p;
  const uint64_t *moduli; /* optional host array [num_q + num_p]; validated */
} ks64_params_t;

typedef struct ks64_plan *ks64_plan_t;

/* Host only: the moduli of these parameters, host_out [num_q + num_p]. */
ks_status_t ks64_params_moduli(const ks64_params_t *p, uint64_t *host_out);
/* Host only: psi for q at ring degree 2^log_n, or 0 if q is not a prime
 * = 1 mod 2N. */
uint64_t ks64_root_of_unity(uint64_t q, uint32_t log_n);
/* Plan on the current device (twiddles, conversion and ModDown tables). */
ks_status_t ks64_plan_create(const ks64_params_t *p, ks64_plan_t *out);
ks_status_t ks64_plan_destroy(ks64_plan_t plan);
ks_status_t ks64_plan_moduli(ks64_plan_t plan, uint64_t *host_out);
/* Workspace bytes of one key switch at `level`:
 * 8 N (l+1 + d'(l+1+K) + 2(l+1+K) + 2K + 2(l+1)). */
ks_status_t ks64_workspace_size(ks64_plan_t plan, uint32_t level, size_t *bytes);
/* Key switch: in [level+1][N], out [2][level+1][N], evk [dnum][2][L+1+K][N]
 * (device, uint64, 16-byte aligned; workspace 256-byte aligned, at least
 * ks64_workspace_size bytes; out overlaps none of in, evk, workspace).
 * Output canonical, evaluation domain. */
ks_status_t ks64_keyswitch(ks64_plan_t plan, const uint64_t *evk, uint32_t level, const uint64_t *in,
                           uint64_t *out, void *workspace, size_t workspace_bytes, void *stream);
/* Key switch with a compressed key (Sec. IV-D): evk_b holds the b halves
 * only, [dnum][L+1+K][N] (device, uint64, 16-byte aligned); the a half of
 * digit j's key row g is regenerated on the device, word k being X 2^-64
 * mod m_g for X = (x1 >> 5) 2^64 + x0, x0 and x1 the SplitMix64 outputs
 * (Steele, Lea and Flood 2014) of a_seed at counters 2t and 2t + 1,
 * t = (j (L+1+K) + g) N + k (123 bits: below 2^-65 from uniform mod a
 * 60-bit prime).  Everything else, including
 * the workspace and the errors, as ks64_keyswitch; out overlaps neither
 * evk_b nor the workspace. */
ks_status_t ks64_keyswitch_seeded(ks64_plan_t plan, const uint64_t *evk_b, uint64_t a_seed, uint32_t level,
                                  const uint64_t *in, uint64_t *out, void *workspace, size_t workspace_bytes,
                                  void *stream);
/* In-place forward (inverse = 0) or inverse NTT of `count` limbs of data
 * [count][N]; limb c uses modulus number g[c] (host array, order q_0..q_L,
 * p_0..p_{K-1}).  Words canonical on entry and on return. */
ks_status_t ks64_ntt(ks64_plan_t plan, uint32_t count, const uint32_t *g, int inverse, uint64_t *data,
                     void *stream);

#ifdef __cplusplus
}
#endif
#endif /* KS_H */
