#!/usr/bin/env python3
"""Benchmark: hybrid key switching on one MI355X.

Workload: N = 2^16, l+1 = 24 towers of 30-bit primes, dnum = 3 (alpha 8),
K = 8 special primes, uint32 residues; seeded uniform inputs and keys (key
switching is data-oblivious, so values do not change the timing).  A step is
one key switch of one polynomial through every stage (ModUp P1-P5, ModDown
P1-P4) with the plan's primary schedule (Output-Centric).  To make the key
stream from HBM instead of the 256 MB last-level cache, consecutive steps
rotate over `--evk-copies` distinct keys (48 MiB each).

Prints one JSON line (see the contract in the project documentation).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LOG_N, NUM_Q, DNUM, NUM_P, LEVEL = 16, 24, 3, 8, 23
HBM_PEAK_GBS = 8000.0
# 32-bit integer multiplies (v_mul_lo_u32, v_mul_hi_u32, v_mad_u64_u32) issue
# at the FP64 vector rate, 64 lanes per clock per CU: 256 CUs x 64 x 2.4 GHz.
MUL_PEAK_PER_S = 256 * 64 * 2.4e9
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_oc_n16_l24_dnum3.json")
SEED_MULS = 12  # multiplies per regenerated key word


def alg_bytes(n, l1, k, ndig):
    """Algorithmic HBM bytes of one key switch: input, key limbs read, output."""
    return 4 * n * (l1 + 2 * ndig * (l1 + k) + 2 * l1)


def batch_alg_bytes(n, l1, k, ndig, count):
    """Compulsory HBM bytes of one batch call of `count` key switches at one
    level sharing one key: every input and output once, the key once."""
    return 4 * n * (count * 3 * l1 + 2 * ndig * (l1 + k))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_CPU_CASE = None


def _cpu_prepare():
    """Worker set-up of the all-core CPU baseline: the bench workload's seeded
    inputs, generated once per process, outside the timed region."""
    global _CPU_CASE
    import oracle
    import synth
    op = oracle.Params(LOG_N, NUM_Q, DNUM, NUM_P)
    om = oracle.moduli(op)
    _CPU_CASE = (op, om, synth.uniform_evk(om, DNUM, op.n, synth.seed_for(2, 100)),
                 synth.uniform_limbs(om[:LEVEL + 1], op.n, synth.seed_for(2, 1)))


def _cpu_ready(_):
    time.sleep(0.3)
    return os.getpid()


def _cpu_run(count):
    import oracle
    if _CPU_CASE is None:
        _cpu_prepare()
    op, om, evk_h, d_h = _CPU_CASE
    for _ in range(count):
        oracle.keyswitch(op, om, LEVEL, evk_h, d_h)
    return count


def cpu_baseline(sample, per=2):
    """The oracle, untuned, on the host cores: one thread, then one process
    per core of the host's CPU share (at most 16), each running `per` key
    switches of the same workload."""
    import multiprocessing as mp
    _cpu_prepare()
    t0 = time.perf_counter()
    _cpu_run(sample)
    single = sample / (time.perf_counter() - t0)
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    with mp.get_context("spawn").Pool(cores, initializer=_cpu_prepare) as pool:
        pids = set(pool.map(_cpu_ready, range(cores), chunksize=1))  # every worker set up
        t0 = time.perf_counter()
        done = sum(pool.map(_cpu_run, [per] * cores, chunksize=1))
        wall = time.perf_counter() - t0
    return {"value": round(done / wall, 4), "unit": "key-switches/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} key switches of the bench workload (N=2^16, l+1=24, dnum=3, K=8): {per} in each "
                      f"of {cores} processes ({len(pids)} seen ready); single thread: {sample} key switches",
            "single_thread": {"value": round(single, 4), "cores": 1},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def stage_muls(log_n, l1, k, alpha):
    """Algorithmic 32-bit multiplies per launch of each Output-Centric stage.

    Counted per the method's arithmetic: a Shoup product (twiddle, constant)
    is 3 multiplies, a 32x32+64 multiply-accumulate 1, a REDC reduction of a
    64-bit sum 4; a length-2^s transform pass has s * N/2 butterflies."""
    n, a, b = 1 << log_n, log_n - 8, 8
    sizes = [min(alpha, l1 - lo) for lo in range(0, l1, alpha)]
    ndig = len(sizes)
    col_ntt, row_ntt = 3 * a * n // 2, 3 * b * n // 2
    up_p = sum(k * (n * (s + 4) + col_ntt) for s in sizes)
    up_q = sum((l1 - s) * (n * (s + 4) + col_ntt) for s in sizes)
    return {
        "oc.intt_row": l1 * row_ntt,
        "oc.intt_col.up": l1 * (col_ntt + 3 * n),
        "oc.bconv_col.up": up_p + up_q,
        "oc.row.p": k * (ndig * row_ntt + 2 * ndig * n + 2 * 4 * n + 2 * row_ntt),
        "oc.intt_col.down": 2 * k * (col_ntt + 3 * n),
        "oc.bconv_col.down": 2 * l1 * (n * (k + 4) + col_ntt),
        "oc.row.q": l1 * ((ndig - 1) * row_ntt + 2 * ndig * n + 2 * 4 * n + 2 * row_ntt + 2 * 3 * n),
        # compressed keys: each a-half word regenerated (two 64-bit products
        # of the generator, 4 multiplies each, and one REDC)
        "oc.row.p.seeded": k * (ndig * row_ntt + 2 * ndig * n + 2 * 4 * n + 2 * row_ntt) + SEED_MULS * ndig * k * n,
        "oc.row.q.seeded": l1 * ((ndig - 1) * row_ntt + 2 * ndig * n + 2 * 4 * n + 2 * row_ntt + 2 * 3 * n)
                           + SEED_MULS * ndig * l1 * n,
    }


def stage_bytes(log_n, l1, k, alpha):
    """Algorithmic HBM bytes per launch of each Output-Centric stage: every
    buffer the stage must read or write, once (inputs, key words, outputs and
    the intermediates handed between stages; constant tables excluded)."""
    limb = 4 << log_n
    sizes = [min(alpha, l1 - lo) for lo in range(0, l1, alpha)]
    ndig = len(sizes)
    up_targets = sum(k + (l1 - s) for s in sizes)
    return {
        "oc.intt_row": limb * 2 * l1,                                     # d in, xt out
        "oc.intt_col.up": limb * 2 * l1,                                  # xt in place
        "oc.bconv_col.up": limb * (l1 + up_targets),                      # xt in, ycol out
        "oc.row.p": limb * (ndig * k + 2 * ndig * k + 2 * k),             # ycol, key, zp out
        "oc.intt_col.down": limb * 2 * 2 * k,                             # zp in place
        "oc.bconv_col.down": limb * (2 * k + 2 * l1),                     # zp in, wcol out
        "oc.row.q": limb * ((ndig - 1) * l1 + 2 * l1 + l1 + 2 * ndig * l1 + 2 * l1),  # ycol, wcol, d, key, out
        "oc.row.p.seeded": limb * (ndig * k + ndig * k + 2 * k),          # b halves only
        "oc.row.q.seeded": limb * ((ndig - 1) * l1 + 2 * l1 + l1 + ndig * l1 + 2 * l1),
    }


# Compile units of the library that hold none of the 32-bit key switch's
# kernels or their launches: the 64-bit-word path, the cost-model MLP, the
# rate probes, the no-allocation scratch array and the arithmetic probe.
DIGEST_EXCLUDE = ("ks64.hip", "mlp.hip", "rates.hip", "noalloc.hip", "probe.hip")


def kernel_source_digest(csrc=None):
    """Digest of the library sources that build the 32-bit key switch, with
    comments and blank space removed: the traffic counters stay valid across
    comment edits and edits of the other compile units, not code edits of
    these."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = csrc or os.path.join(ROOT, "paper_2311_01598_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f in DIGEST_EXCLUDE:
            continue
        text = open(os.path.join(csrc, f), encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(f.encode() + b"\0" + " ".join(text.split()).encode())
    return h.hexdigest()[:16]


DEFAULT_CFG = {"schedule": "oc", "tile_towers": 2, "col_width": 16, "row_block": 8, "batch_mode": 1, "batch_order": 1}
# interleaved timing rounds of the sections that compare configurations
ROUNDS = 3


def timed_calls(fn, reps, torch, warmup=1):
    """Seconds per call of fn() over `reps` back-to-back calls (events on the
    current stream, `warmup` untimed calls first)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for r in range(reps):
        fn(r)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / 1e3 / reps


def batched_rate(ks, tune, tuner, plan, evks, mods, count, reps, np, torch, synth):
    """Key switches per second for `count` ciphertexts of the bench workload
    in one batch call (shared key per call, keys rotating across calls), with
    the configuration the autotuner picks for this shape (schedule AUTO),
    next to the plan's fixed starting configuration and each OC choice."""
    n, l1 = plan.n, LEVEL + 1
    ins = [torch.from_numpy(synth.uniform_limbs(mods[:l1], n, synth.seed_for(2, 200 + i)).view(np.int32)).cuda()
           for i in range(count)]
    outs = [torch.empty((2, l1, n), dtype=torch.int32, device="cuda") for _ in range(count)]
    jobs = lambda r: [(evks[r % len(evks)], LEVEL, x, o) for x, o in zip(ins, outs)]

    def rate(cfg):
        if cfg is None:
            plan.configure("auto")
        else:
            tune.apply_config(plan, cfg)
        ws = plan.workspace([LEVEL] * count)
        # the first configuration timed after tuning ran ~7 % slow with one
        # untimed call (clocks and caches settling): five untimed calls each
        s = timed_calls(lambda r=0: plan.keyswitch_batch(jobs(r), workspace=ws), reps, torch, warmup=5)
        del ws
        return count / s
    picked = tuner.tune(plan, LEVEL, count)
    # the tuned run, the fixed default and every OC configuration are timed in
    # ROUNDS interleaved rounds and each reports its median, so that a drift
    # of the device's speed over the section does not favour whichever runs
    # first (single rounds differed by up to 4 % for the same configuration)
    cands = [None, DEFAULT_CFG] + [c for c in tune.config_space() if c["schedule"] == "oc"
                                   and c.get("batch_order", 1) == 1]
    runs = [[] for _ in cands]
    for _ in range(ROUNDS):
        for i, c in enumerate(cands):
            runs[i].append(rate(c))
    med = [round(float(np.median(r)), 1) for r in runs]
    res = {"ciphertexts_per_call": count, "calls": reps, "rounds": ROUNDS, "ks_per_s": med[0],
           "schedule": "auto", "tuned_config": tune.config_key(picked)}
    res["ms_per_call"] = round(1e3 * count / res["ks_per_s"], 4)
    res["fixed_default"] = {"config": tune.config_key(DEFAULT_CFG), "ks_per_s": med[1]}
    res["configs"] = {tune.config_key(c): m for c, m in zip(cands[2:], med[2:])}
    plan.configure("auto")
    return res


def seeded_rate(ks, plan, evks, d, steps, warmup, count, np, torch, synth):
    """Key compression (Sec. IV-D): the bench workload with compressed keys
    (b halves, 24 MiB each, rotating like the full keys, plus a seed), one key
    switch per call and `count` per batch call; per-stage times of the two
    row stages that consume the key."""
    n, l1 = plan.n, LEVEL + 1
    keys = [e[:, 0].contiguous() for e in evks]
    out = torch.empty((2, l1, n), dtype=torch.int32, device="cuda")
    plan.configure("oc", tile_towers=1, batch_mode=1)
    ws = plan.workspace([LEVEL])

    def single(k):
        for i in range(k):
            plan.keyswitch_seeded(keys[i % len(keys)], 1000 + i % len(keys), LEVEL, d, out=out, workspace=ws)
    single(warmup)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    single(steps)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]  # latency pass
    for i in range(steps):
        ev[i].record()
        plan.keyswitch_seeded(keys[i % len(keys)], 1000 + i % len(keys), LEVEL, d, out=out, workspace=ws)
    ev[steps].record()
    torch.cuda.synchronize()
    lat = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    ks.ks_trace_enable(plan.handle, True)
    single(steps)
    ks.ks_trace_enable(plan.handle, False)
    trace = ks.ks_trace_read(plan.handle)
    sbytes = stage_bytes(LOG_N, l1, NUM_P, plan.alpha)
    stages = {}
    for k in ("oc.row.p.seeded", "oc.row.q.seeded"):
        if k in trace:
            t = 1e-3 * trace[k][1] / max(trace[k][0], 1)
            stages[k] = {"avg_us": round(t * 1e6, 3), "hbm_frac": round(sbytes[k] / t / (HBM_PEAK_GBS * 1e9), 4)}
    res = {"ks_per_s": round(steps / (ms / 1e3), 1), "p50_ms": round(lat[len(lat) // 2], 4),
           "p99_ms": round(lat[min(len(lat) - 1, int(len(lat) * 0.99))], 4),
           "key_bytes_per_ks": DNUM * (l1 + NUM_P) * n * 4, "stages": stages}
    ins = [torch.from_numpy(synth.uniform_limbs(plan.moduli[:l1], n, synth.seed_for(2, 200 + i)).view(np.int32)).cuda()
           for i in range(count)]
    outs = [torch.empty((2, l1, n), dtype=torch.int32, device="cuda") for _ in range(count)]
    reps = max(5, steps // 20)
    for tt, mode in ((1, 1), (2, 1), (2, 3)):
        plan.configure("oc", tile_towers=tt, batch_mode=mode)
        wsb = plan.workspace([LEVEL] * count)
        jobs = lambda r: [(keys[r % len(keys)], 1000 + r % len(keys), LEVEL, x, o) for x, o in zip(ins, outs)]
        plan.keyswitch_batch_seeded(jobs(0), workspace=wsb)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for r in range(reps):
            plan.keyswitch_batch_seeded(jobs(r), workspace=wsb)
        b.record()
        torch.cuda.synchronize()
        res.setdefault("batched", {})[f"t{tt}/m{mode}"] = round(count * reps / (a.elapsed_time(b) / 1e3), 1)
        del wsb
    plan.configure("oc", tile_towers=1, batch_mode=1)
    return res


def rotation_rate(ks, plan, evks, steps, np, torch, synth):
    """Hoisted rotations of one ciphertext of the bench workload: m rotations
    sharing one ModUp of c1 (keys rotating over the full-key copies) against
    the same m rotations one call each, and multiplication with
    relinearisation; rotations/s and multiplications/s."""
    n, l1 = plan.n, LEVEL + 1
    mods = plan.moduli
    c0 = torch.from_numpy(synth.uniform_limbs(mods[:l1], n, synth.seed_for(2, 400)).view(np.int32)).cuda()
    c1 = torch.from_numpy(synth.uniform_limbs(mods[:l1], n, synth.seed_for(2, 401)).view(np.int32)).cuda()
    plan.configure("oc", tile_towers=1, batch_mode=1)
    res = {"hoisted": {}, "one_at_a_time": {}}
    for m in (1, 4, 8):
        gal = [ks.galois_rotation(LOG_N, r + 1) for r in range(m)]
        rots = [(evks[i % len(evks)], g) for i, g in enumerate(gal)]
        ws = plan._ws(ks.ks_rotate_workspace_size(plan.handle, LEVEL, m), "cuda")
        wsm = plan._ws(ks.ks_rotate_workspace_size(plan.handle, LEVEL, 1), "cuda")
        outs = [torch.empty((2, l1, n), dtype=torch.int32, device="cuda") for _ in range(m)]
        reps = max(5, steps // (4 * m))
        for name, hoist in (("hoisted", True), ("one_at_a_time", False)):
            def once():
                if hoist:
                    ks.ks_rotate_hoisted(plan.handle, LEVEL, c0, c1, [(e, g, o) for (e, g), o in zip(rots, outs)], ws)
                else:
                    for (e, g), o in zip(rots, outs):
                        ks.ks_rotate_hoisted(plan.handle, LEVEL, c0, c1, [(e, g, o)], wsm)
            once()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                once()
            b.record()
            torch.cuda.synchronize()
            res[name][f"m{m}"] = round(m * reps / (a.elapsed_time(b) / 1e3), 1)
    res["hoisting_gain_m8"] = round(res["hoisted"]["m8"] / res["one_at_a_time"]["m8"], 3)
    # the same 8 rotations with compressed keys (b halves plus a seed)
    keys_b = [e[:, 0].contiguous() for e in evks]
    gal = [ks.galois_rotation(LOG_N, r + 1) for r in range(8)]
    ws = plan._ws(ks.ks_rotate_workspace_size(plan.handle, LEVEL, 8), "cuda")
    outs = [torch.empty((2, l1, n), dtype=torch.int32, device="cuda") for _ in range(8)]
    rots = [(keys_b[i % len(keys_b)], 1000 + i, g, o) for i, (g, o) in enumerate(zip(gal, outs))]
    ks.ks_rotate_hoisted_seeded(plan.handle, LEVEL, c0, c1, rots, ws)
    torch.cuda.synchronize()
    reps = max(5, steps // 32)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        ks.ks_rotate_hoisted_seeded(plan.handle, LEVEL, c0, c1, rots, ws)
    b.record()
    torch.cuda.synchronize()
    res["hoisted_compressed_keys"] = {"m8": round(8 * reps / (a.elapsed_time(b) / 1e3), 1)}
    del keys_b
    # 16 different ciphertexts, each with its own rotation, in one batch call
    cts = [(torch.from_numpy(synth.uniform_limbs(mods[:l1], n, synth.seed_for(2, 600 + 2 * i)).view(np.int32)).cuda(),
            torch.from_numpy(synth.uniform_limbs(mods[:l1], n, synth.seed_for(2, 601 + 2 * i)).view(np.int32)).cuda())
           for i in range(16)]
    rjobs = [(evks[i % len(evks)], ks.galois_rotation(LOG_N, i + 1), LEVEL, a0_, a1_) for i, (a0_, a1_) in enumerate(cts)]
    wsb = plan.workspace([LEVEL] * 16)
    plan.configure("oc", tile_towers=2, batch_mode=1)
    plan.rotate_batch(rjobs, workspace=wsb)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        plan.rotate_batch(rjobs, workspace=wsb)
    b.record()
    torch.cuda.synchronize()
    res["batch16_one_rotation_each"] = round(16 * reps / (a.elapsed_time(b) / 1e3), 1)
    plan.configure("oc", tile_towers=1, batch_mode=1)
    del cts, wsb
    # double hoisting: the sum of the same 8 rotations, each times a plaintext
    # diagonal, with one ModUp and one ModDown (Max-Parallel stages)
    diags = [torch.from_numpy(synth.uniform_limbs(mods, n, synth.seed_for(2, 500 + i)).view(np.int32)).cuda()
             for i in range(8)]
    terms = [(evks[i % len(evks)], g, diags[i]) for i, g in enumerate(gal)]
    ws = plan._ws(ks.ks_rotate_sum_workspace_size(plan.handle, LEVEL, 8), "cuda")
    out = torch.empty((2, l1, n), dtype=torch.int32, device="cuda")
    ks.ks_rotate_sum_hoisted(plan.handle, LEVEL, c0, c1, terms, out, ws)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        ks.ks_rotate_sum_hoisted(plan.handle, LEVEL, c0, c1, terms, out, ws)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    res["double_hoisted_sum_m8"] = {"sums_per_s": round(1e3 / ms, 1), "rotations_per_s": round(8e3 / ms, 1),
                                    "us_per_sum": round(ms * 1e3, 2)}
    del diags, ws
    a0, a1 = c0, c1
    b0 = torch.from_numpy(synth.uniform_limbs(mods[:l1], n, synth.seed_for(2, 402)).view(np.int32)).cuda()
    b1 = torch.from_numpy(synth.uniform_limbs(mods[:l1], n, synth.seed_for(2, 403)).view(np.int32)).cuda()
    out = torch.empty((2, l1, n), dtype=torch.int32, device="cuda")
    wsr = plan._ws(ks.ks_mult_workspace_size(plan.handle, LEVEL), "cuda")
    reps = max(10, steps // 2)
    for i in range(5):
        plan.mult_relin(evks[i % len(evks)], LEVEL, a0, a1, b0, b1, out=out, workspace=wsr)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(reps):
        plan.mult_relin(evks[i % len(evks)], LEVEL, a0, a1, b0, b1, out=out, workspace=wsr)
    b.record()
    torch.cuda.synchronize()
    res["mult_relin_per_s"] = round(reps / (a.elapsed_time(b) / 1e3), 1)
    return res


BTS_SETS = {"bts1": (17, 28, 1, 28), "bts2": (17, 40, 2, 20), "bts3": (17, 45, 3, 15),
            "ark": (16, 24, 4, 6), "dprive": (16, 26, 3, 7)}


def bts_rate(ks, steps, np, torch, synth):
    """Key switches per second at the parameter sets of Table III (BTS1/2/3
    at N = 2^17, ARK and DPRIVE at N = 2^16; tower counts as there), one
    ciphertext at the top level per call, keys rotating over 4 copies: OC,
    MP and DC with 30-bit towers, OC with compressed keys, and the 64-bit
    path with full and compressed keys."""
    res = {}
    for name, (log_n, num_q, dnum, num_p) in BTS_SETS.items():
        plan = ks.Plan(log_n, num_q, dnum, num_p)
        n, mods, level = plan.n, plan.moduli, num_q - 1
        evks = [torch.from_numpy(synth.uniform_evk(mods, dnum, n, synth.seed_for(31, c)).view(np.int32)).cuda()
                for c in range(4)]
        d = torch.from_numpy(synth.uniform_limbs(mods[:num_q], n, synth.seed_for(31, 9)).view(np.int32)).cuda()
        out = torch.empty((2, num_q, n), dtype=torch.int32, device="cuda")
        cur = {"evk_mib": round(evks[0].numel() * 4 / 2**20, 1)}
        for sched in ("oc", "mp", "dc"):
            plan.configure(sched)
            ws = plan.workspace([level])
            for i in range(5):
                plan.keyswitch(evks[i % 4], level, d, out=out, workspace=ws)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for i in range(steps):
                plan.keyswitch(evks[i % 4], level, d, out=out, workspace=ws)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / steps
            cur[sched] = {"ks_per_s": round(1e3 / ms, 1), "us_per_ks": round(ms * 1e3, 2)}
            del ws
        cur["oc_over_mp"] = round(cur["oc"]["ks_per_s"] / cur["mp"]["ks_per_s"], 3)
        cur["oc_over_dc"] = round(cur["oc"]["ks_per_s"] / cur["dc"]["ks_per_s"], 3)
        # compressed keys (b halves of the same keys plus a seed)
        keys_b = [e[:, 0].contiguous() for e in evks]
        plan.configure("oc")
        ws = plan.workspace([level])
        for i in range(5):
            plan.keyswitch_seeded(keys_b[i % 4], 77 + i % 4, level, d, out=out, workspace=ws)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for i in range(steps):
            plan.keyswitch_seeded(keys_b[i % 4], 77 + i % 4, level, d, out=out, workspace=ws)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        cur["oc_compressed_keys"] = {"ks_per_s": round(1e3 / ms, 1), "us_per_ks": round(ms * 1e3, 2)}
        del ws, keys_b
        del evks
        plan.close()
        # 64-bit words (~60-bit towers), Max-Parallel order
        p64 = ks.Plan64(log_n, num_q, dnum, num_p)
        evk64, d64 = (synth.uniform_words64_device(p64.moduli, p64.n, synth.seed_for(31, 64), torch, lead=(dnum, 2)),
                      synth.uniform_words64_device(p64.moduli[:num_q], p64.n, synth.seed_for(31, 65), torch))
        out64 = torch.empty((2, num_q, p64.n), dtype=torch.int64, device="cuda")
        ws64 = p64.workspace(level)
        s64 = timed_calls(lambda r=0: p64.keyswitch(evk64, level, d64, out=out64, workspace=ws64), max(5, steps // 4),
                          torch)
        cur["mp_64bit_words"] = {"ks_per_s": round(1 / s64, 1), "us_per_ks": round(s64 * 1e6, 2),
                                 "evk_mib": round(evk64.numel() * 8 / 2**20, 1)}
        # the same with compressed keys (b halves plus a seed)
        evk64_b = evk64[:, 0].contiguous()
        s64c = timed_calls(lambda r=0: p64.keyswitch_seeded(evk64_b, 78, level, d64, out=out64, workspace=ws64),
                           max(5, steps // 4), torch)
        cur["mp_64bit_words_compressed_keys"] = {"ks_per_s": round(1 / s64c, 1), "us_per_ks": round(s64c * 1e6, 2),
                                                 "evk_mib": round(evk64_b.numel() * 8 / 2**20, 1)}
        del evk64, evk64_b, d64, out64, ws64
        p64.close()
        res[name] = cur
    # the modulus of BTS3's 60-bit towers (45 + 15) in 30-bit towers: 90 + 30,
    # dnum 3 (alpha = K = 30), OC; BTS1/BTS2 would need alpha > 32
    log_n, num_q, dnum, num_p = 17, 90, 3, 30
    plan = ks.Plan(log_n, num_q, dnum, num_p)
    n, mods, level = plan.n, plan.moduli, num_q - 1
    evk = torch.from_numpy(synth.uniform_evk(mods, dnum, n, synth.seed_for(31, 90)).view(np.int32)).cuda()
    d = torch.from_numpy(synth.uniform_limbs(mods[:num_q], n, synth.seed_for(31, 91)).view(np.int32)).cuda()
    out = torch.empty((2, num_q, n), dtype=torch.int32, device="cuda")
    plan.configure("oc")
    ws = plan.workspace([level])
    s30 = timed_calls(lambda r=0: plan.keyswitch(evk, level, d, out=out, workspace=ws), max(5, steps // 4), torch)
    res["bts3"]["oc_30bit_towers_same_modulus"] = {"towers": "90 + 30, dnum 3", "ks_per_s": round(1 / s30, 1),
                                                   "us_per_ks": round(s30 * 1e6, 2),
                                                   "evk_mib": round(evk.numel() * 4 / 2**20, 1)}
    del evk, d, out, ws
    plan.close()
    return res


def mixed_rate(ks, tune, tuner, dnum, reps, np, torch, synth):
    """64 ciphertexts at levels with l+1 ~ U[8, 24], N=2^16, K = alpha, one
    shared key: OC batched with the autotuner's configuration for this batch
    (schedule AUTO), the plan's fixed starting configuration, and the same 64
    switched one at a time with MP."""
    alpha = -(-NUM_Q // dnum)
    plan = ks.Plan(LOG_N, NUM_Q, dnum, alpha)
    n, mods = plan.n, plan.moduli
    levels = synth.batch_levels(64, 8, 24, synth.seed_for(3, dnum))
    evk = torch.from_numpy(synth.uniform_evk(mods, dnum, n, synth.seed_for(3, 100 + dnum)).view(np.int32)).cuda()
    ins = [torch.from_numpy(synth.uniform_limbs(mods[:l + 1], n, synth.seed_for(3, 300 + i)).view(np.int32)).cuda()
           for i, l in enumerate(levels)]
    outs = [torch.empty((2, l + 1, n), dtype=torch.int32, device="cuda") for l in levels]
    jobs = [(evk, l, x, o) for l, x, o in zip(levels, ins, outs)]
    picked = tuner.tune(plan, None, levels=levels, seed=3000 + dnum)
    res = {"tuned_config": tune.config_key(picked), "rounds": ROUNDS}
    runs = {}
    for _ in range(ROUNDS):  # interleaved rounds, median per entry (see batched_rate)
        for name, cfg, batched in (("oc_batched_tuned", None, True),
                                   ("oc_batched_fixed_default", DEFAULT_CFG, True),
                                   ("mp_one_at_a_time", {**DEFAULT_CFG, "schedule": "mp"}, False)):
            if cfg is None:
                plan.configure("auto")
            else:
                tune.apply_config(plan, cfg)
            ws = plan.workspace(levels if batched else [max(levels)])

            def once(r=0):
                if batched:
                    plan.keyswitch_batch(jobs, workspace=ws)
                else:
                    for e, l, x, o in jobs:
                        plan.keyswitch(e, l, x, out=o, workspace=ws)
            runs.setdefault(name, []).append(64 / timed_calls(once, reps, torch, warmup=3))
            del ws
    for name, r in runs.items():
        res[name] = round(float(np.median(r)), 1)
    res["tuned_over_mp"] = round(res["oc_batched_tuned"] / res["mp_one_at_a_time"], 3)
    plan.close()
    return res


def serving_rate(ks, tune, tuner, count, np, torch, synth, seed=5, buffers=64):
    """Serving workload: Poisson arrivals of requests for the relinearisation
    key (a key switch of d2) or one of 16 rotation keys (a rotation of a
    ciphertext (c0, c1) by 5^k), 17 keys with distinct contents resident per
    ring degree, N in {2^16, 2^17}, l+1 ~ U[8, 48], dnum=3.  Request inputs
    cycle over `buffers` distinct ciphertexts per degree (1.5 and 3 GiB, far
    beyond the 256 MB last-level cache).  Reports saturation throughput (all
    requests queued at once), p50/p99 latency at 0.5, 0.8 and 0.95 of that
    rate, key switches with compressed keys, and the same requests one at a
    time with MP (a rotation as automorphisms then the MP key switch)."""
    from paper_2311_01598_amd.serve import Request, Server, poisson_arrivals
    plans, keys, pool, pool0 = {}, {}, {}, {}
    tuned = {}
    for log_n in (16, 17):
        p = ks.Plan(log_n, 48, 3)
        plans[log_n] = p
        # the autotuner's choice for batches of 16 (the server's largest) and
        # of 4 at four levels; every batch resolves to the nearest entry
        for level in (11, 23, 35, 47):
            for cnt in (4, 16):
                tuned[f"n{log_n}/l{level + 1}/c{cnt}"] = tune.config_key(tuner.tune(p, level, cnt, seed=level))
        keys[log_n] = [synth.uniform_limbs_device(p.moduli, p.n, synth.seed_for(4, 1000 * log_n + k), torch,
                                                  lead=(3, 2)) for k in range(17)]
        pool[log_n] = synth.uniform_limbs_device(p.moduli[:48], p.n, synth.seed_for(4, 100 * log_n), torch,
                                                 lead=(buffers,))
        pool0[log_n] = synth.uniform_limbs_device(p.moduli[:48], p.n, synth.seed_for(4, 100 * log_n + 50), torch,
                                                  lead=(buffers,))
    torch.cuda.synchronize()
    rng = np.random.default_rng(synth.seed_for(4, seed))

    def requests(rotations=True):
        out = []
        for i in range(count):
            log_n = int(rng.choice((16, 17)))
            level = int(rng.integers(7, 48))
            key = int(rng.integers(0, 17))
            d = pool[log_n][i % buffers][:level + 1]
            if rotations and key:
                out.append(Request(i, key, log_n, level, d, 0.0, c0=pool0[log_n][i % buffers][:level + 1],
                                   galois=ks.galois_rotation(log_n, key)))
            else:
                out.append(Request(i, key, log_n, level, d, 0.0))
        return out
    budget = 8 << 30
    res = {"requests": count, "keys_per_degree": 17, "budget_gib": budget >> 30, "streams": 2, "max_batch": 16,
           "input_buffers_per_degree": buffers, "tuned": tuned,
           "mix": "key 0 (relinearisation): key switch; keys 1-16: rotation of (c0, c1) by 5^k"}
    sat = Server(plans, keys, budget, streams=2, max_batch=16, keep_outputs=False)
    reqs = requests()
    sat.run([(0.0, r) for r in reqs[:256]])  # warm-up
    sat = Server(plans, keys, budget, streams=2, max_batch=16, keep_outputs=False)
    st = sat.run([(0.0, r) for r in reqs])
    res["saturation"] = {"requests_per_s": round(st["ks_per_s"], 1), "batches": st["batches"]}
    # warm-up at the lowest rate (small batches: the shapes the timed runs
    # meet first), not reported
    warm = Server(plans, keys, budget, streams=2, max_batch=16, keep_outputs=False)
    warm.run(list(zip(poisson_arrivals(0.5 * res["saturation"]["requests_per_s"], 1000, synth.seed_for(4, 99)),
                      requests()[:1000])))
    res["poisson"] = {}
    for frac in (0.5, 0.8, 0.95):
        rate = frac * res["saturation"]["requests_per_s"]
        srv = Server(plans, keys, budget, streams=2, max_batch=16, keep_outputs=False)
        st = srv.run(list(zip(poisson_arrivals(rate, count, synth.seed_for(4, seed + int(100 * frac))), requests())))
        res["poisson"][f"{frac:.2f}"] = {"offered_per_s": round(rate, 1), "requests_per_s": round(st["ks_per_s"], 1),
                                         "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                                         "batches": st["batches"],
                                         "high_water_gib": round(st["high_water_bytes"] / 2**30, 3)}
    # key-switch requests only, every key compressed (b halves plus a seed):
    # half the resident key bytes
    ckeys = {k: [(e[:, 0].contiguous(), 900 + i) for i, e in enumerate(v)] for k, v in keys.items()}
    srv = Server(plans, ckeys, budget, streams=2, max_batch=16, keep_outputs=False)
    st = srv.run([(0.0, r) for r in requests(rotations=False)])
    res["saturation_key_switches_compressed_keys"] = {"requests_per_s": round(st["ks_per_s"], 1),
                                                      "batches": st["batches"]}
    res["resident_key_gib"] = {"full": round(sum(e.numel() * 4 for v in keys.values() for e in v) / 2**30, 2),
                               "compressed": round(sum(b.numel() * 4 for v in ckeys.values() for b, _ in v) / 2**30,
                                                   2)}
    del ckeys
    # the same request mix, one request per call with MP on one stream
    for p in plans.values():
        p.configure("mp")
    ws = {k: p.workspace([47]) for k, p in plans.items()}
    outs = {k: torch.empty(2 * 48 * p.n, dtype=torch.int32, device="cuda") for k, p in plans.items()}
    tmp = {k: torch.empty(2 * 48 * p.n, dtype=torch.int32, device="cuda") for k, p in plans.items()}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        p = plans[r.log_n]
        limbs = (r.level + 1) * p.n
        d = r.d
        if r.galois is not None:  # rotation: permute c1 and c0, then the key switch
            d = tmp[r.log_n][:limbs]
            ks.ks_automorphism(p.handle, r.galois, r.level + 1, r.d, d)
            ks.ks_automorphism(p.handle, r.galois, r.level + 1, r.c0, tmp[r.log_n][limbs:2 * limbs])
        p.keyswitch(keys[r.log_n][r.key], r.level, d, out=outs[r.log_n][:2 * limbs], workspace=ws[r.log_n])
    torch.cuda.synchronize()
    res["mp_one_at_a_time_requests_per_s"] = round(count / (time.perf_counter() - t0), 1)
    del ws, outs, tmp, keys, pool, pool0, reqs
    for p in plans.values():
        p.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--evk-copies", type=int, default=8)
    ap.add_argument("--schedule", default="auto", choices=["auto", "oc", "mp", "dc"],
                    help="auto: the autotuner's choice for one key switch of the workload")
    ap.add_argument("--compare", type=int, default=1, help="also time MP and DC one key switch per call (0: skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=4, help="oracle key switches in the CPU sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy 3 times (counter calibration) and exit")
    ap.add_argument("--rates", action="store_true", help="also run the ALU / copy rate probes")
    ap.add_argument("--batch", type=int, default=16,
                    help="ciphertexts per call in the batched measurement of the same workload (0 = skip)")
    ap.add_argument("--seeded", type=int, default=1, help="also time compressed keys (0: skip)")
    ap.add_argument("--rotations", type=int, default=1, help="also time hoisted rotations and HMult (0: skip)")
    ap.add_argument("--bts", type=int, default=1, help="also time the N=2^17 bootstrapping-scale sets (0: skip)")
    ap.add_argument("--mixed", type=int, default=1,
                    help="also time 64-ciphertext batches at levels l+1 ~ U[8,24] for dnum 2, 3, 4 (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests per arrival rate in the serving measurement (0 = skip)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); "
              "the library runs on one GPU; multi-GPU key switching is described in the design notes only.", file=sys.stderr)
        return 2
    # the CPU baseline runs first, before this process touches the GPU (its
    # worker processes are started from a process without a GPU context)
    cpu = None if (args.no_cpu or args.copy_calibration) else cpu_baseline(args.cpu_sample)
    import numpy as np
    import torch

    import paper_2311_01598_amd as ks
    import synth

    torch.cuda.init()
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch_read": a.numel() * 4, "written": b.numel() * 4}))
        return 0
    from paper_2311_01598_amd import costmodel, tune
    model = costmodel.default_model()
    tuner = tune.Tuner(cache=None, model=model, top_m=3, reps=5)
    plan = ks.Plan(LOG_N, NUM_Q, DNUM, NUM_P)
    n, l1 = plan.n, LEVEL + 1
    ndig = -(-l1 // plan.alpha)
    mods = plan.moduli
    evks = [torch.from_numpy(synth.uniform_evk(mods, DNUM, n, synth.seed_for(2, 100 + c)).view(np.int32)).cuda()
            for c in range(args.evk_copies)]
    d = torch.from_numpy(synth.uniform_limbs(mods[:l1], n, synth.seed_for(2, 1)).view(np.int32)).cuda()
    out = torch.empty((2, l1, n), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def run(schedule, steps, warmup, lat=None):
        plan.configure(schedule)
        ws = plan.workspace([LEVEL])
        for i in range(warmup):
            plan.keyswitch(evks[i % len(evks)], LEVEL, d, out=out, workspace=ws)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)] if lat is not None else None
        t0 = time.perf_counter()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for i in range(steps):
            if ev:
                ev[i].record(stream)
            plan.keyswitch(evks[i % len(evks)], LEVEL, d, out=out, workspace=ws)
        if ev:
            ev[steps].record(stream)
        stop.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = start.elapsed_time(stop)
        if ev is not None:
            lat.extend(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
        return ms, wall

    single_cfg = None
    if args.schedule == "auto":
        single_cfg = tune.config_key(tuner.tune(plan, LEVEL, 1, seed=11))
    # throughput: K steps with nothing recorded between them; latency
    # percentiles from a second pass with an event before and after each step
    # (the events cost a few microseconds per step, kept out of `value`)
    ms, wall = run(args.schedule, args.steps, args.warmup)
    lat = []
    run(args.schedule, args.steps, 0, lat)
    # Per-kernel durations: the same K steps again with start/stop events
    # attached to every kernel dispatch (kept out of the timed region above,
    # because the traced launch path costs host time between kernels).
    ks.ks_trace_enable(plan.handle, True)
    run(args.schedule, args.steps, 0)
    ks.ks_trace_enable(plan.handle, False)
    trace = ks.ks_trace_read(plan.handle)
    ks_per_s = args.steps / (ms / 1e3)
    nbytes = alg_bytes(n, l1, NUM_P, ndig)
    lat.sort()
    res = {
        "metric": "key-switches/sec (N=2^16, l+1=24, dnum=3)",
        "value": round(ks_per_s, 1),
        "unit": "key-switches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded uniform residues and keys)",
        "config": {"workload": "hybrid key switch, N=2^16, l+1=24, dnum=3, alpha=8, K=8, 1 ciphertext per call",
                   "schedule": args.schedule, "tuned_config": single_cfg, "evk_copies": args.evk_copies},
        "hbm_gbs_algorithmic": round(nbytes * ks_per_s / 1e9, 1),
        "latency_ms": {"p50": round(lat[len(lat) // 2], 4), "p99": round(lat[min(len(lat) - 1, int(len(lat) * 0.99))], 4)},
    }
    muls = stage_muls(LOG_N, l1, NUM_P, plan.alpha)
    sbytes = stage_bytes(LOG_N, l1, NUM_P, plan.alpha)
    stages = {}
    for k, v in trace.items():
        st = {"launches": v[0], "avg_us": round(1e3 * v[1] / max(v[0], 1), 3)}
        if k in muls:
            t = 1e-3 * v[1] / max(v[0], 1)
            st.update({"mul_frac": round(muls[k] / t / MUL_PEAK_PER_S, 4),
                       "hbm_frac": round(sbytes[k] / t / (HBM_PEAK_GBS * 1e9), 4),
                       "bound": "hbm" if sbytes[k] / (HBM_PEAK_GBS * 1e9) >= muls[k] / MUL_PEAK_PER_S else "alu"})
        stages[k] = st
    # The roofline of the whole key switch (seven dependent launches, timed
    # together above): its compulsory HBM bytes (input, the key limbs it
    # reads, output) against the HBM peak, and its algorithmic 32-bit
    # multiplies against the integer multiply peak.  The roof that binds is
    # the one with the longer floor time; both fractions are reported.
    tot_muls = sum(v for k, v in muls.items() if not k.endswith(".seeded"))
    tot_bytes = sum(v for k, v in sbytes.items() if not k.endswith(".seeded"))
    step_s = ms / args.steps / 1e3
    t_hbm, t_mul = nbytes / (HBM_PEAK_GBS * 1e9), tot_muls / MUL_PEAK_PER_S
    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        prof = json.load(open(PROFILE_TRAFFIC))
        kern = prof.get("kernels", {})
        if prof.get("source_digest") == kernel_source_digest() and all(k in kern for k in muls
                                                                         if not k.endswith(".seeded")):
            traffic = sum(kern[k]["bytes_per_launch"] for k in muls if not k.endswith(".seeded"))
    hbm_part = {"achieved": round(nbytes / step_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(nbytes / step_s / (HBM_PEAK_GBS * 1e9), 4), "bytes_per_ks": nbytes,
                "floor_us": round(t_hbm * 1e6, 3)}
    mul_part = {"achieved": round(tot_muls / step_s / 1e12, 4), "peak": round(MUL_PEAK_PER_S / 1e12, 4),
                "unit": "T mul/s (32-bit integer multiplies)", "frac": round(tot_muls / step_s / MUL_PEAK_PER_S, 4),
                "muls_per_ks": tot_muls, "floor_us": round(t_mul * 1e6, 3)}
    bind = mul_part if t_mul >= t_hbm else hbm_part
    res["roofline"] = {"bound": "alu" if t_mul >= t_hbm else "hbm", "kernel": "one key switch (7 OC launches)",
                       "achieved": bind["achieved"], "peak": bind["peak"], "unit": bind["unit"],
                       "frac": bind["frac"], "traffic": traffic, "avg_us": round(step_s * 1e6, 3),
                       "hbm": hbm_part, "mul": mul_part}
    # diagnostics: the longest stage against its own stage bytes and multiplies
    oc_stages = [k for k in trace if k in muls]
    if oc_stages:
        dom = max(oc_stages, key=lambda k: trace[k][1] / max(trace[k][0], 1))
        res["roofline"]["longest_stage"] = {"kernel": dom, **{k: stages[dom][k] for k in ("avg_us", "hbm_frac",
                                                                                            "mul_frac", "bound")}}
    res["whole_keyswitch"] = {"muls": tot_muls, "mul_frac": round(tot_muls * ks_per_s / MUL_PEAK_PER_S, 4),
                              "hbm_frac": round(nbytes * ks_per_s / (HBM_PEAK_GBS * 1e9), 4),
                              "stage_bytes": tot_bytes,
                              "stage_bytes_frac": round(tot_bytes * ks_per_s / (HBM_PEAK_GBS * 1e9), 4)}
    res["stages"] = stages
    if args.batch:
        res["batched"] = batched_rate(ks, tune, tuner, plan, evks, mods, args.batch, max(20, args.steps // 10), np,
                                      torch, synth)
        bk = res["batched"]["ks_per_s"]
        # HBM rates of the batched run: compulsory bytes (every input and
        # output once, the call's shared key once) and the stages'
        # algorithmic bytes, per second, against the peak
        bb = batch_alg_bytes(n, l1, NUM_P, ndig, args.batch) / args.batch
        res["batched"]["compulsory_bytes_per_ks"] = round(bb)
        res["batched"]["hbm_gbs_algorithmic"] = round(bb * bk / 1e9, 1)
        res["batched"]["hbm_frac"] = round(bb * bk / (HBM_PEAK_GBS * 1e9), 4)
        res["batched"]["mul_frac"] = round(tot_muls * bk / MUL_PEAK_PER_S, 4)
        res["batched"]["stage_bytes_gbs"] = round(tot_bytes * bk / 1e9, 1)
        res["batched"]["stage_bytes_frac"] = round(tot_bytes * bk / (HBM_PEAK_GBS * 1e9), 4)
    if args.bts:
        res["bts_scale"] = bts_rate(ks, max(20, args.steps // 4), np, torch, synth)
    if args.rotations:
        res["rotations"] = rotation_rate(ks, plan, evks, args.steps, np, torch, synth)
    if args.seeded:
        res["key_compression"] = seeded_rate(ks, plan, evks, d, args.steps, args.warmup, args.batch or 16, np,
                                             torch, synth)
    if args.mixed:
        res["mixed_batches"] = {}
        for dn in (2, 3, 4):
            res["mixed_batches"][f"dnum{dn}"] = mixed_rate(ks, tune, tuner, dn, max(10, args.steps // 20), np, torch,
                                                           synth)
    if args.serve_requests:
        res["serving"] = serving_rate(ks, tune, tuner, args.serve_requests, np, torch, synth)
    if args.rates:
        res["device_rates"] = {k: round(v / 1e12, 4) for k, v in ks.ks_device_rates().items()}
    if args.compare:
        res["schedules"] = {}
        for sch in ("mp", "dc", "oc"):
            k2 = max(20, args.steps // 4)
            lat2 = []
            ms2, _ = run(sch, k2, 5)
            run(sch, k2, 0, lat2)
            lat2.sort()
            res["schedules"][sch] = {"ks_per_s": round(k2 / (ms2 / 1e3), 1),
                                     "p99_ms": round(lat2[min(len(lat2) - 1, int(len(lat2) * 0.99))], 4)}
        res["schedules"]["oc_over_mp"] = round(res["schedules"]["oc"]["ks_per_s"] / res["schedules"]["mp"]["ks_per_s"],
                                               3)
    plan.close()
    del evks, d, out
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    res["tuner"] = {"cost_model": "data/costmodel.npz" if model is not None else None, "top_m": tuner.top_m,
                    "shapes": [{k: e[k] for k in ("params", "level", "count", "source", "config")} for e in tuner.log]}
    if cpu is not None:
        res["cpu_baseline"] = cpu
    print(json.dumps(res), flush=True)
    return 0

if __name__ == "__main__":
    sys.exit(main())
