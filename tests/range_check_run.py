"""The key-switch paths on the range-check build, for tests/test_gpu_ranges.py.

Run in a process of its own with KS_LIBRARY=libks_check.so (a process loads
one of the two builds).  It first shows that the counters are live (the
strict REDC bound, which ordinary inputs violate, must be counted), then
runs every path the library has on inputs that reach the arithmetic's
limits -- every word at m - 1, alternating 0 and m - 1, conversion sources
scaled to q - 1, the longest key sums (dnum 16) and conversion sums
(alpha = K = 32) -- under every schedule and tile width, compressed keys,
hoisted rotations, double-hoisted sums, multiplication, mixed-level batches
in both modes, N = 2^17, and the 64-bit-word path up to BTS3 at full size.
Every result must still equal the oracle's (or the single call's, for a
batch).  It prints one JSON line: the strict count and code, the number of
checked calls, the mismatches, and the violations counted over all of them.
"""
import importlib.util
import json
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    assert os.environ.get("KS_LIBRARY") == "libks_check.so", "run with KS_LIBRARY=libks_check.so"
    import torch

    import oracle
    import synth
    from oracle import core
    from oracle import core64 as o64
    import paper_2311_01598_amd as ks

    spec = importlib.util.spec_from_file_location("edges", os.path.join(HERE, "test_gpu_edges.py"))
    edges = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(edges)

    def dev(a):
        a = np.ascontiguousarray(a)
        return torch.from_numpy(a.view(np.int64 if a.dtype == np.uint64 else np.int32)).cuda()

    def host(t):
        return t.cpu().numpy().view(np.uint64 if t.dtype == torch.int64 else np.uint32)

    res = {"library": os.path.basename(ks.LIB_PATH), "checked": 0, "mismatches": []}

    def check(name, got, want):
        res["checked"] += 1
        if not np.array_equal(got, want):
            res["mismatches"].append(name)
            say(f"[ranges] MISMATCH {name}")

    # the counters are live: the strict REDC bound fails on ordinary inputs
    p = oracle.Params(12, 4, 2, 2)
    mods = oracle.moduli(p)
    evk = synth.uniform_evk(mods, 2, p.n, synth.seed_for(40, 0))
    d = synth.uniform_limbs(mods[:4], p.n, synth.seed_for(40, 1))
    plan = ks.Plan(12, 4, 2, 2)
    ks.ks_range_violations(reset=True)
    ks.ks_range_set_strict(True)
    plan.keyswitch(dev(evk), 3, dev(d))
    res["strict_count"], res["strict_code"] = ks.ks_range_violations(reset=True)
    ks.ks_range_set_strict(False)
    ks.ks_range_violations(reset=True)
    say(f"[ranges] strict: {res['strict_count']} violations, code {res['strict_code']}")

    # the plain workload with real keys, every level and schedule
    s, s2, evk, h = oracle.keygen(p, mods, seed=41)
    for level in range(4):
        d = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(40, 10 + level))
        want = oracle.keyswitch(p, mods, level, evk, d)
        for sched, tt in (("oc", 1), ("oc", 2), ("mp", 1), ("dc", 1)):
            plan.configure(sched, tile_towers=tt)
            check(f"plain l={level} {sched}{tt}", host(plan.keyswitch(dev(evk), level, dev(d))), want)
    # compressed key, hoisted rotations, a double-hoisted sum, multiplication
    plan.configure("oc")
    ev2 = evk.copy()
    ev2[:, 1] = core.seeded_a(p, mods, 42)[:, 1]
    d = synth.uniform_limbs(mods[:4], p.n, synth.seed_for(40, 20))
    check("seeded", host(plan.keyswitch_seeded(dev(np.ascontiguousarray(ev2[:, 0])), 42, 3, dev(d))),
          oracle.keyswitch(p, mods, 3, ev2, d))
    c0 = synth.uniform_limbs(mods[:4], p.n, synth.seed_for(40, 21))
    gal = [core.galois_rotation(12, 1), core.galois_rotation(12, 3), (2 << 12) - 1]
    keys = [synth.uniform_evk(mods, 2, p.n, synth.seed_for(40, 30 + i)) for i in range(3)]
    outs = plan.rotate_hoisted(3, dev(c0), dev(d), [(dev(k), g) for k, g in zip(keys, gal)])
    for o, w in zip(outs, core.rotate_hoisted(p, mods, 3, c0, d, gal, keys)):
        check("rotate_hoisted", host(o), w)
    diags = [synth.uniform_limbs(mods, p.n, synth.seed_for(40, 40 + i)) for i in range(3)]  # every key row
    check("rotate_sum", host(plan.rotate_sum_hoisted(3, dev(c0), dev(d),
                                                     [(dev(k), g, dev(dg)) for k, g, dg in zip(keys, gal, diags)])),
          core.rotate_sum_hoisted(p, mods, 3, c0, d, gal, keys, diags))
    a0, a1, b0, b1 = [synth.uniform_limbs(mods[:4], p.n, synth.seed_for(40, 50 + i)) for i in range(4)]
    check("mult_relin", host(plan.mult_relin(dev(keys[0]), 3, dev(a0), dev(a1), dev(b0), dev(b1))),
          core.mult_relin(p, mods, 3, a0, a1, b0, b1, keys[0]))
    plan.close()

    # mixed-level batches in both modes against single calls
    p = oracle.Params(14, 12, 3, 0)
    mods = oracle.moduli(p)
    plan = ks.Plan(14, 12, 3, 0)
    evk_d = dev(synth.uniform_evk(mods, 3, p.n, synth.seed_for(40, 60)))
    levels = [11, 3, 7, 0, 10, 5, 11, 8]
    ins = [dev(synth.uniform_limbs(mods[:lv + 1], p.n, synth.seed_for(40, 61 + i))) for i, lv in enumerate(levels)]
    singles = [host(plan.keyswitch(evk_d, lv, x)) for lv, x in zip(levels, ins)]
    for mode in (1, 3):
        plan.configure("oc", tile_towers=2, batch_mode=mode)
        outs = [torch.empty((2, lv + 1, p.n), dtype=torch.int32, device="cuda") for lv in levels]
        plan.keyswitch_batch([(evk_d, lv, x, o) for lv, x, o in zip(levels, ins, outs)])
        for i, o in enumerate(outs):
            check(f"batch mode {mode} job {i}", host(o), singles[i])
    plan.close()

    # the arithmetic's edges (the edge test's inputs), N = 2^16 and 2^17
    cases = []
    for s_ in [(16, 32, 16, 2), (16, 64, 2, 32), (17, 32, 1, 32)]:
        p = oracle.Params(*s_)
        mods = oracle.moduli(p)
        for pat in (edges.PATTERNS if s_[0] == 16 else ["eval_max"]):
            edges.warm(p, mods)
            d, ev = edges.edge_input(pat, p, mods, s_[1], p.n)
            cases.append((s_, pat, p, mods, d, ev))
    say(f"[ranges] {len(cases)} edge cases: oracle")
    with ThreadPoolExecutor(max_workers=len(cases)) as ex:
        wants = list(ex.map(lambda c: oracle.keyswitch(c[2], c[3], c[0][1] - 1, c[5], c[4]), cases))
    for (s_, pat, p, mods, d, ev), want in zip(cases, wants):
        plan = ks.Plan(*s_)
        ev_d, d_d = dev(ev), dev(d)
        runs = (("oc", 1), ("oc", 2), ("mp", 1), ("dc", 1)) if s_[0] == 16 else (("oc", 2),)
        for sched, tt in runs:
            say(f"[ranges] edge {s_} {pat} {sched}{tt}")
            plan.configure(sched, tile_towers=tt)
            check(f"edge {s_} {pat} {sched}{tt}", host(plan.keyswitch(ev_d, s_[1] - 1, d_d)), want)
        plan.close()

    # the bench workload and the serving workload's largest plan
    for s_, tts in (((16, 24, 3, 8), (1, 2)), ((17, 48, 3, 16), (2,))):
        p = oracle.Params(*s_)
        mods = oracle.moduli(p)
        ev = synth.uniform_evk(mods, s_[2], p.n, synth.seed_for(40, 70 + s_[0]))
        d = synth.uniform_limbs(mods[:s_[1]], p.n, synth.seed_for(40, 72 + s_[0]))
        say(f"[ranges] {s_}: oracle")
        want = oracle.keyswitch(p, mods, s_[1] - 1, ev, d)
        plan = ks.Plan(*s_)
        for sched, tt in [("oc", t) for t in tts] + ([("mp", 1), ("dc", 1)] if s_[0] == 16 else []):
            plan.configure(sched, tile_towers=tt)
            check(f"{s_} {sched}{tt}", host(plan.keyswitch(dev(ev), s_[1] - 1, dev(d))), want)
        plan.close()

    # 64-bit words: real seeded keys, every word at m - 1 at the longest sums,
    # and BTS3 at full size
    p = oracle.Params(12, 4, 2, 2)
    mods = o64.moduli(p)
    s, s2, evk, h = o64.keygen_seeded(p, mods, seed=43, a_seed=44)
    d = np.stack([np.random.default_rng(45 + i).integers(0, int(m), p.n, dtype=np.uint64)
                  for i, m in enumerate(mods[:4])])
    want = o64.keyswitch(p, mods, 3, evk, d)
    plan = ks.Plan64(12, 4, 2, 2)
    check("64 plain", host(plan.keyswitch(dev(evk), 3, dev(d))), want)
    check("64 seeded", host(plan.keyswitch_seeded(dev(np.ascontiguousarray(evk[:, 0])), 44, 3, dev(d))), want)
    plan.close()
    for s_ in [(13, 32, 16, 2), (13, 64, 2, 32)]:
        p = oracle.Params(*s_)
        mods = o64.moduli(p)
        ev = np.empty((p.dnum, 2, len(mods), p.n), np.uint64)
        for r, m in enumerate(mods):
            ev[:, :, r, :] = int(m) - 1
        d = np.stack([np.full(p.n, int(m) - 1, np.uint64) for m in mods[:s_[1]]])
        say(f"[ranges] 64 edge {s_}")
        plan = ks.Plan64(*s_)
        check(f"64 edge {s_}", host(plan.keyswitch(dev(ev), s_[1] - 1, dev(d))),
              o64.keyswitch(p, mods, s_[1] - 1, ev, d))
        plan.close()
    p = oracle.Params(17, 45, 3, 15)
    mods = o64.moduli(p)
    rng = np.random.default_rng(46)
    ev = np.stack([np.stack([np.stack([rng.integers(0, int(m), p.n, dtype=np.uint64) for m in mods])
                             for _ in range(2)]) for _ in range(3)])
    d = np.stack([rng.integers(0, int(m), p.n, dtype=np.uint64) for m in mods[:45]])
    say("[ranges] 64 BTS3: oracle")
    want = o64.keyswitch(p, mods, 44, ev, d)
    plan = ks.Plan64(17, 45, 3, 15)
    check("64 BTS3", host(plan.keyswitch(dev(ev), 44, dev(d))), want)
    plan.close()

    torch.cuda.synchronize()
    res["violations"], res["code"] = ks.ks_range_violations()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
