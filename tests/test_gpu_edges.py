"""GPU parity at the edges of the arithmetic, and the batch shapes of the
mixed-level workloads.

Edge values: the 64-bit sums of the kernels are longest in the key
multiply-accumulate (one product per live digit, up to dnum = 16) and in the
basis conversions (one product per source tower, up to alpha = K = 32).
Uniform residues stay well below those sums' limits on average, so these
cases drive every input word and every key word to its largest residue
(m - 1), or alternate 0 and m - 1, in the evaluation domain, in the
coefficient domain, and at the conversion's scaled sources ([x q^_i^-1]_q_i
= q_i - 1, Sec. III-B P2).  Every output word must equal the oracle's.

Batches: 64 ciphertexts at N = 2^16 with l+1 ~ U[8, 24] for dnum 2, 3 and
4 with K = alpha (one shared key each), and an N = 2^17 batch whose levels
sit on both sides of the tower count where the conversion tiles switch to
two targets, plus hoisted rotations at N = 2^17 on both sides of it.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth
from oracle import core

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_01598_amd as m
    return m


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint32)


# (log N, l+1, dnum, K): the longest key sum (16 digits) and the longest
# conversion sums (32 sources, 32 special towers), at N = 2^16 and 2^17
EDGE_SETS = [(16, 32, 16, 2), (16, 64, 2, 32), (17, 16, 16, 1), (17, 32, 1, 32)]
PATTERNS = ["eval_max", "scaled_max", "alternating"]


def warm(p, mods):
    """Fill the oracle's per-modulus root cache from this thread before the
    oracle runs in several threads: those then only read it."""
    for m in mods:
        oracle.min_psi(int(m), p.log_n)


def _digits(l1, alpha):
    return [list(range(lo, min(lo + alpha, l1))) for lo in range(0, l1, alpha)]


def edge_input(pattern, p, mods, l1, n):
    """Input d [l+1][N] and key [dnum][2][L+1+K][N] of one edge pattern.

    eval_max:    d = q_i - 1 and key = m - 1 at every word;
    scaled_max:  d = NTT(x) with x constant per tower, chosen so that the
                 conversion's scaled source [x q^_{j,i}^-1]_{q_i} is q_i - 1
                 (x = -q^_{j,i} mod q_i, q^_{j,i} = Q_j / q_i), key = m - 1;
    alternating: d and key alternate 0 and m - 1 word by word (the key with
                 the opposite phase)."""
    alpha = -(-p.num_q // p.dnum)
    ev = np.empty((p.dnum, 2, len(mods), n), np.uint32)
    d = np.empty((l1, n), np.uint32)
    if pattern == "eval_max":
        for r, m in enumerate(mods):
            ev[:, :, r, :] = int(m) - 1
        for i in range(l1):
            d[i] = int(mods[i]) - 1
    elif pattern == "scaled_max":
        for r, m in enumerate(mods):
            ev[:, :, r, :] = int(m) - 1
        for dig in _digits(l1, alpha):
            for i in dig:
                qi = int(mods[i])
                qhat = 1
                for t in dig:
                    if t != i:
                        qhat = qhat * int(mods[t]) % qi
                x = np.full(n, (-qhat) % qi, np.uint32)
                d[i] = oracle.ntt(x, mods[i])
    else:
        mask = (np.arange(n) & 1).astype(np.uint32)
        for r, m in enumerate(mods):
            ev[:, :, r, :] = (1 - mask) * (int(m) - 1)
        for i in range(l1):
            d[i] = mask * (int(mods[i]) - 1)
    return d, ev


@pytest.fixture(scope="module")
def edge_cases():
    """Every (set, pattern) with its oracle output; the oracle runs are
    independent, so they run in threads (the C oracle releases the GIL)."""
    cases = []
    for s in EDGE_SETS:
        p = oracle.Params(*s)
        mods = oracle.moduli(p)
        for pat in PATTERNS:
            warm(p, mods)
            d, ev = edge_input(pat, p, mods, s[1], p.n)
            cases.append((s, pat, p, mods, d, ev))
    say(f"[edges] computing {len(cases)} oracle key switches")
    with ThreadPoolExecutor(max_workers=min(12, len(cases))) as ex:
        wants = list(ex.map(lambda c: oracle.keyswitch(c[2], c[3], c[0][1] - 1, c[5], c[4]), cases))
    return {(c[0], c[1]): (c[2], c[3], c[4], c[5], w) for c, w in zip(cases, wants)}


@pytest.mark.parametrize("pattern", PATTERNS)
@pytest.mark.parametrize("params", EDGE_SETS, ids=lambda s: "n%d_l%d_dnum%d_k%d" % s)
def test_edge_values_every_schedule(ks, edge_cases, params, pattern):
    p, mods, d, ev, want = edge_cases[(params, pattern)]
    log_n, num_q, dnum, num_p = params
    plan = ks.Plan(log_n, num_q, dnum, num_p)
    assert plan.moduli == [int(m) for m in mods]
    ev_d, d_d = dev(ev), dev(d)
    for sched, tt in (("oc", 1), ("oc", 2), ("mp", 1), ("dc", 1)):
        say(f"[edges] {params} {pattern} {sched} tile={tt}")
        plan.configure(sched, tile_towers=tt)
        got = host(plan.keyswitch(ev_d, num_q - 1, d_d))
        torch.cuda.synchronize()
        bad = np.argwhere(got != want)
        assert bad.size == 0, (sched, tt, bad[:5], len(bad))
    plan.close()


@pytest.mark.parametrize("dnum", [2, 3, 4])
def test_batch_64_mixed_levels_every_dnum(ks, dnum):
    """64 ciphertexts at N = 2^16, l+1 ~ U[8, 24], K = alpha, one shared key,
    for dnum 2, 3 and 4: every job of one batch call equals the same job
    switched alone (two targets per conversion tile and one), and sampled
    jobs equal the oracle."""
    alpha = -(-24 // dnum)
    p = oracle.Params(16, 24, dnum, alpha)
    mods = oracle.moduli(p)
    evk = synth.uniform_evk(mods, dnum, p.n, synth.seed_for(3, 100 + dnum))
    levels = synth.batch_levels(64, 8, 24, synth.seed_for(3, dnum))
    ins = [synth.uniform_limbs(mods[:l + 1], p.n, synth.seed_for(3, 300 + i)) for i, l in enumerate(levels)]
    sample = (0, 31, 63)
    warm(p, mods)
    with ThreadPoolExecutor(max_workers=3) as ex:
        want = dict(zip(sample, ex.map(lambda i: oracle.keyswitch(p, mods, levels[i], evk, ins[i]), sample)))
    plan = ks.Plan(16, 24, dnum, alpha, schedule="oc")
    evk_d = dev(evk)
    ins_d = [dev(x) for x in ins]
    ws1 = plan.workspace([max(levels)])
    alone = []
    for l, x in zip(levels, ins_d):
        alone.append(plan.keyswitch(evk_d, l, x, workspace=ws1))
    torch.cuda.synchronize()
    for i in sample:
        assert np.array_equal(host(alone[i]), want[i]), (dnum, i)
    for tt, mode in ((2, 1), (1, 3)):
        say(f"[batch64] dnum={dnum} tile={tt} mode={mode}")
        plan.configure("oc", tile_towers=tt, batch_mode=mode)
        outs = [torch.full((2, l + 1, p.n), -1, dtype=torch.int32, device="cuda") for l in levels]
        plan.keyswitch_batch([(evk_d, l, x, o) for l, x, o in zip(levels, ins_d, outs)])
        torch.cuda.synchronize()
        for i, (a, o) in enumerate(zip(alone, outs)):
            assert torch.equal(a, o), (dnum, tt, mode, i)
    plan.close()


def test_n17_batch_levels_across_the_two_target_switch(ks):
    """At N = 2^17 a launch takes two targets per conversion tile when its
    largest job has at least 17 towers, so smaller jobs of the same batch run
    through the two-target build.  Levels on both sides of 17 towers: every
    job of the batch equals its single call, and sampled jobs the oracle."""
    p = oracle.Params(17, 24, 3, 8)
    mods = oracle.moduli(p)
    evks = [synth.uniform_evk(mods, 3, p.n, synth.seed_for(17, k)) for k in range(2)]
    levels = [5, 12, 15, 16, 17, 20, 23, 2]
    ins = [synth.uniform_limbs(mods[:l + 1], p.n, synth.seed_for(17, 10 + i)) for i, l in enumerate(levels)]
    sample = (0, 2, 3, 6)
    warm(p, mods)
    with ThreadPoolExecutor(max_workers=4) as ex:
        want = dict(zip(sample, ex.map(lambda i: oracle.keyswitch(p, mods, levels[i], evks[i % 2], ins[i]),
                                       sample)))
    plan = ks.Plan(17, 24, 3, 8, schedule="oc")
    evk_d = [dev(e) for e in evks]
    ins_d = [dev(x) for x in ins]
    ws1 = plan.workspace([max(levels)])
    for tt in (1, 2):
        plan.configure("oc", tile_towers=tt)
        say(f"[n17 batch] tile={tt}")
        alone = [plan.keyswitch(evk_d[i % 2], l, x, workspace=ws1) for i, (l, x) in enumerate(zip(levels, ins_d))]
        outs = [torch.full((2, l + 1, p.n), -1, dtype=torch.int32, device="cuda") for l in levels]
        plan.keyswitch_batch([(evk_d[i % 2], l, x, o) for i, (l, x, o) in enumerate(zip(levels, ins_d, outs))])
        torch.cuda.synchronize()
        for i in sample:
            assert np.array_equal(host(alone[i]), want[i]), (tt, i)
        for i, (a, o) in enumerate(zip(alone, outs)):
            assert torch.equal(a, o), (tt, i)
    plan.close()


@pytest.mark.parametrize("level", [9, 20])
def test_n17_hoisted_rotations_across_the_two_target_switch(ks, level):
    """Two hoisted rotations of one ciphertext at N = 2^17, at l+1 = 10 (one
    target per conversion tile) and 21 (two), against the oracle."""
    p = oracle.Params(17, 24, 3, 8)
    mods = oracle.moduli(p)
    evks = [synth.uniform_evk(mods, 3, p.n, synth.seed_for(18, k)) for k in range(2)]
    c0 = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(18, 20))
    c1 = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(18, 21))
    gal = [core.galois_rotation(17, 3), (2 << 17) - 1]
    want = core.rotate_hoisted(p, mods, level, c0, c1, gal, evks)
    plan = ks.Plan(17, 24, 3, 8, schedule="oc", tile_towers=2)
    say(f"[n17 rotations] level={level}")
    outs = plan.rotate_hoisted(level, dev(c0), dev(c1), [(dev(e), g) for e, g in zip(evks, gal)])
    torch.cuda.synchronize()
    for o, w in zip(outs, want):
        assert np.array_equal(host(o), w), level
    plan.close()


def test_calls_with_nothing_to_do(ks):
    """Degenerate sizes: a batch of no jobs (full and compressed keys), a
    rotation batch of no jobs, hoisted rotations with no rotation, a
    double-hoisted sum of no terms and an automorphism of no limbs return
    KS_OK and write nothing."""
    plan = ks.Plan(12, 4, 2, 2)
    n = plan.n
    ws = plan.workspace([3])
    c = torch.zeros((4, n), dtype=torch.int32, device="cuda")
    out = torch.full((2, 4, n), -1, dtype=torch.int32, device="cuda")
    ks.ks_keyswitch_batch(plan.handle, [], ws)
    ks.ks_keyswitch_batch_seeded(plan.handle, [], ws)
    ks.ks_rotate_batch(plan.handle, [], ws)
    ks.ks_rotate_hoisted(plan.handle, 3, c, c, [], ws)
    ks.ks_rotate_sum_hoisted(plan.handle, 3, c, c, [], out, ws)
    ks.ks_automorphism(plan.handle, 5, 0, c, out)
    torch.cuda.synchronize()
    assert bool((out == -1).all())
    plan.close()


def test_largest_plan(ks):
    """The largest plan the library accepts in towers: 96 + 32 = 128 towers,
    alpha = K = 32 (two chunks of 16 products in every conversion), at
    N = 2^16, at the top level under every schedule and at l+1 = 51 (a
    partial last digit of 19 towers), every word against the oracle."""
    p = oracle.Params(16, 96, 3, 32)
    mods = oracle.moduli(p)
    evk = synth.uniform_evk(mods, 3, p.n, synth.seed_for(44, 0))
    plan = ks.Plan(16, 96, 3, 32)
    assert plan.moduli == [int(m) for m in mods] and len(mods) == 128
    evk_d = dev(evk)
    for level, runs in ((95, (("oc", 1), ("oc", 2), ("mp", 1), ("dc", 1))), (50, (("oc", 2), ("mp", 1)))):
        d = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(44, 1 + level))
        say(f"[largest] level={level}: oracle")
        want = oracle.keyswitch(p, mods, level, evk, d)
        d_d = dev(d)
        for sched, tt in runs:
            say(f"[largest] level={level} {sched} tile={tt}")
            plan.configure(sched, tile_towers=tt)
            got = host(plan.keyswitch(evk_d, level, d_d))
            torch.cuda.synchronize()
            bad = np.argwhere(got != want)
            assert bad.size == 0, (level, sched, tt, bad[:5], len(bad))
    plan.close()
