"""Seeded random sweep of the parameter space against the oracle.

Twenty-four parameter sets drawn (seeded) from everything a plan accepts:
log N 12..14, 1..40 q towers, dnum 1..min(16, towers) (so alpha up to 32,
where conversion sums are accumulated in chunks of 16 products), K = 0
(alpha) or 1..32, at a random level.  Each runs MP, DC and OC with one and
two targets per conversion tile, every output word compared with the
oracle; every third set also runs a compressed key and a hoisted pair of
rotations.  Eight random batches of random parameter sets check the batch
launches against single calls.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import core
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_01598_amd as m
    return m


def _cases(count=24, seed=2311):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        log_n = int(rng.integers(12, 15))
        num_q = int(rng.integers(1, 41))
        dnum = int(rng.integers(1, min(16, num_q) + 1))
        alpha = -(-num_q // dnum)
        num_p = 0 if rng.random() < 0.4 else int(rng.integers(1, 33))
        K = num_p or alpha
        if alpha > 32 or K > 32 or num_q + K > 128:
            continue
        level = int(rng.integers(0, num_q))
        out.append((log_n, num_q, dnum, num_p, level))
    return out


CASES = _cases()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("i", range(len(CASES)))
def test_random_parameter_set(ks, i):
    log_n, num_q, dnum, num_p, level = CASES[i]
    print(f"[sweep {i}] log_n={log_n} num_q={num_q} dnum={dnum} num_p={num_p} level={level}", flush=True)
    sys.stdout.flush()
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = oracle.moduli(p)
    evk = synth.uniform_evk(mods, dnum, p.n, synth.seed_for(40, i))
    d = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(40, 100 + i))
    want = oracle.keyswitch(p, mods, level, evk, d)
    plan = ks.Plan(log_n, num_q, dnum, num_p)
    assert plan.moduli == [int(m) for m in mods]
    evk_d, d_d = dev(evk), dev(d)
    for sched, tt in (("mp", 1), ("dc", 1), ("oc", 1), ("oc", 2)):
        plan.configure(sched, tile_towers=tt)
        got = host(plan.keyswitch(evk_d, level, d_d))
        assert np.array_equal(got, want), (sched, tt, np.argwhere(got != want)[:3])
    if i % 3 == 0:
        plan.configure("oc", tile_towers=1)
        a_seed = synth.seed_for(40, 200 + i)
        ev2 = evk.copy()
        ev2[:, 1] = core.seeded_a(p, mods, a_seed)[:, 1]
        got = host(plan.keyswitch_seeded(dev(np.ascontiguousarray(ev2[:, 0])), a_seed, level, d_d))
        assert np.array_equal(got, oracle.keyswitch(p, mods, level, ev2, d)), "compressed key"
        gal = [core.galois_rotation(log_n, 1 + i), (2 << log_n) - 1]
        c0 = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(40, 300 + i))
        outs = plan.rotate_hoisted(level, dev(c0), d_d, [(evk_d, g) for g in gal])
        want_r = core.rotate_hoisted(p, mods, level, c0, d, gal, [evk, evk])
        for o, w in zip(outs, want_r):
            assert np.array_equal(host(o), w), "hoisted rotation"
    plan.close()


def _batch_cases(count=8, seed=4242):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        log_n = int(rng.integers(12, 15))
        num_q = int(rng.integers(2, 41))
        dnum = int(rng.integers(1, min(16, num_q) + 1))
        alpha = -(-num_q // dnum)
        num_p = 0 if rng.random() < 0.4 else int(rng.integers(1, 33))
        K = num_p or alpha
        if alpha > 32 or K > 32 or num_q + K > 128:
            continue
        njobs = int(rng.integers(2, 41))
        out.append((log_n, num_q, dnum, num_p, [int(x) for x in rng.integers(0, num_q, njobs)],
                    [int(x) for x in rng.integers(0, 3, njobs)]))
    return out


BATCH_CASES = _batch_cases()


@pytest.mark.parametrize("i", range(len(BATCH_CASES)))
def test_random_batch(ks, i):
    """A random batch (2-40 jobs at random levels, three keys) of a random
    parameter set: the row phases pick one-round or multi-round builds from
    the largest job, the conversions one-chunk builds from alpha and K, and
    the jobs are interleaved per group of 8 row tiles.  Every job equals its
    own single call, at both conversion tile widths, and one sampled job
    equals the oracle."""
    log_n, num_q, dnum, num_p, levels, kid = BATCH_CASES[i]
    print(f"[batch {i}] log_n={log_n} num_q={num_q} dnum={dnum} num_p={num_p} jobs={len(levels)}", flush=True)
    sys.stdout.flush()
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = oracle.moduli(p)
    keys = [synth.uniform_evk(mods, dnum, p.n, synth.seed_for(41, 10 * i + k)) for k in range(3)]
    ins = [synth.uniform_limbs(mods[:l + 1], p.n, synth.seed_for(42, 1000 * i + j)) for j, l in enumerate(levels)]
    plan = ks.Plan(log_n, num_q, dnum, num_p)
    kd = [dev(k) for k in keys]
    xd = [dev(x) for x in ins]
    j0 = len(levels) // 2
    want = oracle.keyswitch(p, mods, levels[j0], keys[kid[j0]], ins[j0])
    for tt in (1, 2):
        plan.configure("oc", tile_towers=tt)
        singles = [host(plan.keyswitch(kd[kid[j]], l, xd[j])) for j, l in enumerate(levels)]
        assert np.array_equal(singles[j0], want), ("oracle", tt)
        outs = [torch.empty((2, l + 1, p.n), dtype=torch.int32, device="cuda") for l in levels]
        plan.keyswitch_batch([(kd[kid[j]], l, xd[j], outs[j]) for j, l in enumerate(levels)])
        for j, o in enumerate(outs):
            assert np.array_equal(host(o), singles[j]), (tt, j, levels[j])
    plan.close()
