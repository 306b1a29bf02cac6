"""GPU parity of key compression (Sec. IV-D): compressed keys (b halves plus
the seed of the a halves) against the oracle, bit for bit.

* ks_expand_seeded_a writes exactly the oracle's a halves (every word), at
  small sizes and at the N=2^16 / 24-tower / dnum 3 workload.
* ks_keyswitch_seeded equals the oracle's key switch with the expanded key:
  a real RLWE key at every level (and its output decrypts), the full-size
  workload with every element compared, partial last digits, dnum = 1,
  K != alpha, alpha = 1, both conversion tile widths.
* ks_keyswitch_batch_seeded at mixed levels and distinct keys equals the
  oracle per job, for both batch launch modes.
* Rejections: a schedule other than OC, an output overlapping the key.
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint32)


def compressed(p, mods, seed, a_seed):
    """(b halves [dnum][L+1+K][N], full key with the oracle's a halves)."""
    full = synth.uniform_evk(mods, p.dnum, p.n, seed)
    full[:, 1] = core.seeded_a(p, mods, a_seed)[:, 1]
    return np.ascontiguousarray(full[:, 0]), full


@pytest.mark.parametrize("shape", [(12, 4, 2, 2), (13, 5, 2, 0), (16, 24, 3, 8)])
def test_expand_matches_oracle(ks, shape):
    log_n, num_q, dnum, num_p = shape
    say(f"[expand] {shape}")
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = oracle.moduli(p)
    plan = ks.Plan(log_n, num_q, dnum, num_p)
    a_seed = 0xfeedface12345678
    want = core.seeded_a(p, mods, a_seed)
    evk = torch.zeros(want.shape, dtype=torch.int32, device="cuda")
    plan.expand_seeded_a(a_seed, evk)
    torch.cuda.synchronize()
    got = host(evk)
    assert np.array_equal(got[:, 1], want[:, 1])
    assert not got[:, 0].any()  # b halves untouched
    plan.close()


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_seeded_keygen_all_levels_and_decrypts(ks, level):
    p = oracle.Params(12, 4, 2, 2)
    mods = oracle.moduli(p)
    s, s2, evk, h = core.keygen_seeded(p, mods, seed=99, a_seed=0x1234)
    plan = ks.Plan(12, 4, 2, 2)
    d = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(9, level))
    want = oracle.keyswitch(p, mods, level, evk, d)
    for tt in (1, 2):
        say(f"[seeded plain] level={level} tile={tt}")
        plan.configure("oc", tile_towers=tt)
        out = plan.keyswitch_seeded(dev(np.ascontiguousarray(evk[:, 0])), 0x1234, level, dev(d))
        torch.cuda.synchronize()
        got = host(out)
        assert np.array_equal(got, want), (level, tt, np.argwhere(got != want)[:5])
    r = oracle.decrypt_residual(p, mods, level, d, got, s, s2)
    assert max(abs(v) for v in r) <= oracle.noise_bound(p, mods, level, h)
    plan.close()


def test_seeded_full_size_n16_l24_dnum3(ks):
    p = oracle.Params(16, 24, 3, 8)
    mods = oracle.moduli(p)
    a_seed = synth.seed_for(10, 7)
    b, full = compressed(p, mods, synth.seed_for(10, 0), a_seed)
    d = synth.uniform_limbs(mods[:24], p.n, synth.seed_for(10, 1))
    want = oracle.keyswitch(p, mods, 23, full, d)
    plan = ks.Plan(16, 24, 3, 8)
    for tt in (1, 2):
        say(f"[seeded n16] tile={tt}")
        plan.configure("oc", tile_towers=tt)
        out = plan.keyswitch_seeded(dev(b), a_seed, 23, dev(d))
        torch.cuda.synchronize()
        bad = np.argwhere(host(out) != want)
        assert bad.size == 0, (tt, bad[:5], len(bad))
    # the same key expanded on the GPU and used as a full key gives the same bits
    ev = torch.zeros(full.shape, dtype=torch.int32, device="cuda")
    ev[:, 0] = dev(b)
    plan.expand_seeded_a(a_seed, ev)
    out = plan.keyswitch(ev, 23, dev(d))
    torch.cuda.synchronize()
    assert np.array_equal(host(out), want)
    plan.close()


SHAPES = [
    # (log_n, num_q, dnum, num_p, levels)
    (12, 5, 2, 0, [4, 2]),     # partial last digit
    (12, 4, 1, 0, [3, 1]),     # dnum = 1
    (13, 9, 3, 2, [8, 4, 0]),  # K != alpha
    (12, 7, 7, 1, [6, 3]),     # alpha = 1
    (14, 12, 4, 3, [11, 5]),
]


@pytest.mark.parametrize("log_n,num_q,dnum,num_p,levels", SHAPES)
def test_seeded_shapes(ks, log_n, num_q, dnum, num_p, levels):
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = oracle.moduli(p)
    a_seed = synth.seed_for(11, log_n * 100 + num_q)
    b, full = compressed(p, mods, synth.seed_for(11, num_q), a_seed)
    plan = ks.Plan(log_n, num_q, dnum, num_p)
    b_d = dev(b)
    for level in levels:
        say(f"[seeded shape] {log_n},{num_q},{dnum},{num_p} level={level}")
        d = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(11, 50 + level))
        want = oracle.keyswitch(p, mods, level, full, d)
        out = plan.keyswitch_seeded(b_d, a_seed, level, dev(d))
        torch.cuda.synchronize()
        assert np.array_equal(host(out), want), (level, np.argwhere(host(out) != want)[:5])
    plan.close()


@pytest.mark.parametrize("tt,mode", [(1, 1), (2, 3)])
def test_seeded_batch_mixed_levels_and_keys(ks, tt, mode):
    p = oracle.Params(13, 8, 3, 0)
    mods = oracle.moduli(p)
    plan = ks.Plan(13, 8, 3)
    plan.configure("oc", tile_towers=tt, batch_mode=mode)
    keys = [compressed(p, mods, synth.seed_for(12, k), 1000 + k) for k in range(3)]
    keys_d = [dev(b) for b, _ in keys]
    levels = synth.batch_levels(9, 1, 8, synth.seed_for(12, 99))
    jobs, wants = [], []
    for i, level in enumerate(levels):
        k = i % 3
        d = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(12, 200 + i))
        wants.append(oracle.keyswitch(p, mods, level, keys[k][1], d))
        out = torch.empty((2, level + 1, p.n), dtype=torch.int32, device="cuda")
        jobs.append((keys_d[k], 1000 + k, level, dev(d), out))
    say(f"[seeded batch] tt={tt} mode={mode} levels={levels}")
    plan.keyswitch_batch_seeded(jobs)
    torch.cuda.synchronize()
    for i, (job, want) in enumerate(zip(jobs, wants)):
        assert np.array_equal(host(job[4]), want), (i, levels[i])
    plan.close()


def test_seeded_rejections(ks):
    plan = ks.Plan(12, 4, 2, 2)
    p = oracle.Params(12, 4, 2, 2)
    mods = oracle.moduli(p)
    b, _ = compressed(p, mods, 5, 6)
    b_d = dev(b)
    d = dev(synth.uniform_limbs(mods[:4], p.n, 7))
    ws = plan.workspace([3])
    out = torch.empty((2, 4, p.n), dtype=torch.int32, device="cuda")
    full_d = dev(synth.uniform_evk(mods, p.dnum, p.n, 8))  # full-size buffer: in bounds either way
    for sched in ("mp", "dc"):
        plan.configure(sched)
        with pytest.raises(ks.KsError) as e:
            ks.ks_keyswitch_seeded(plan.handle, full_d, 6, 3, d, out, ws)
        assert e.value.status == 2  # KS_ERR_UNSUPPORTED
        with pytest.raises(ks.KsError) as e:
            ks.ks_keyswitch_batch_seeded(plan.handle, [(full_d, 6, 3, d, out)], ws)
        assert e.value.status == 2
    plan.configure("oc")
    # the output may not overlap the compressed key (dnum (L+1+K) N words);
    # this output lies inside the key buffer
    inside = b_d.view(-1)[:2 * 4 * p.n].view(2, 4, p.n)
    with pytest.raises(ks.KsError) as e:
        ks.ks_keyswitch_seeded(plan.handle, b_d, 6, 3, d, inside, ws)
    assert e.value.status == 1  # KS_ERR_INVALID_ARG
    plan.close()
