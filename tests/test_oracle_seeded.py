"""Pins of the oracle's key compression (Sec. IV-D: the a half of every key
pair is regenerated from a seed, so only the b halves travel).

* The counter-based generator equals SplitMix64's published first outputs
  (tests/golden/splitmix64_kat.json) and, at any counter, the sequential
  generator stepped that many times (written here from its definition).
* Word (j, g, k) of the a halves is the generator's output at counter
  (j (L+1+K) + g) N + k, mapped into [0, m_g) as x 2^-32 mod m_g: checked
  through the defining property a 2^32 = x (mod m_g), on every word of a
  small key, and against a sequential walk of the counter.
* The expanded a halves are uniform: per-tower chi-square over 16 bins.
* A key generated with seeded a halves decrypts within the bound of the
  key switch, and its a halves equal the stand-alone expansion.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import core

M64 = 2**64 - 1
GAMMA = 0x9e3779b97f4a7c15


class _Sequential:
    """SplitMix64 as a stateful generator: add gamma, then mix."""

    def __init__(self, seed):
        self.x = seed & M64

    def next(self):
        self.x = (self.x + GAMMA) & M64
        z = self.x
        z = ((z ^ (z >> 30)) * 0xbf58476d1ce4e5b9) & M64
        z = ((z ^ (z >> 27)) * 0x94d049bb133111eb) & M64
        return z ^ (z >> 31)


def test_splitmix_known_answers():
    kat = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64_kat.json")))
    got = [core.splitmix_at(kat["seed"], t) for t in range(len(kat["outputs_hex"]))]
    assert got == [int(h, 16) for h in kat["outputs_hex"]]


@pytest.mark.parametrize("seed", [0, 1, 0x0123456789abcdef, M64])
def test_counter_form_equals_sequential_generator(seed):
    g = _Sequential(seed)
    seq = [g.next() for _ in range(300)]
    assert [core.splitmix_at(seed, t) for t in range(300)] == seq


def _params():
    return oracle.Params(9, 5, 2, 3)


def test_seeded_a_words_follow_the_counter_layout():
    p = _params()
    mods = oracle.moduli(p)
    a_seed = 0x5eed
    ev = core.seeded_a(p, mods, a_seed)
    EL = p.num_q + p.num_p
    assert not ev[:, 0].any()  # b halves untouched
    g = _Sequential(a_seed)  # counter order: j, then g, then k
    for j in range(p.dnum):
        for gi in range(EL):
            m = int(mods[gi])  # key rows and moduli share one order: q_0..q_L, p_0..p_{K-1}
            a = ev[j, 1, gi].astype(np.int64)
            assert int(a.max()) < m
            for k in range(p.n):
                x = g.next()
                assert (int(a[k]) << 32) % m == x % m, (j, gi, k)


def test_seeded_a_is_uniform():
    p = oracle.Params(12, 4, 2, 2)
    mods = oracle.moduli(p)
    ev = core.seeded_a(p, mods, 77)
    EL = p.num_q + p.num_p
    for gi in range(EL):
        m = int(mods[gi])
        for j in range(p.dnum):
            a = ev[j, 1, gi].astype(np.float64)
            counts = np.bincount((a * 16 / m).astype(np.int64), minlength=16)
            exp = p.n / 16
            chi2 = float(((counts - exp) ** 2 / exp).sum())
            assert chi2 < 45.0, (gi, j, chi2)  # 15 dof: p < 1e-4 under uniformity
    # different seeds give unrelated words
    ev2 = core.seeded_a(p, mods, 78)
    assert np.mean(ev[:, 1] == ev2[:, 1]) < 1e-3


@pytest.mark.parametrize("log_n,num_q,dnum,num_p,levels", [(11, 4, 2, 2, [3, 1]), (10, 6, 3, 3, [5, 0])])
def test_seeded_key_decrypts_within_bound(log_n, num_q, dnum, num_p, levels):
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = oracle.moduli(p)
    s, s2, evk, h = core.keygen_seeded(p, mods, seed=21, a_seed=0xabc)
    assert np.array_equal(evk[:, 1], core.seeded_a(p, mods, 0xabc)[:, 1])
    for gi, m in enumerate(mods):  # every half canonical for its own row's modulus
        assert int(evk[:, :, gi].max()) < int(m)
    _, _, evk_plain, _ = oracle.keygen(p, mods, seed=21)
    assert not np.array_equal(evk[:, 1], evk_plain[:, 1])
    rng = np.random.default_rng(3)
    for level in levels:
        d = np.stack([rng.integers(0, int(q), p.n, dtype=np.uint64) for q in mods[:level + 1]]).astype(np.uint32)
        out = oracle.keyswitch(p, mods, level, evk, d)
        r = oracle.decrypt_residual(p, mods, level, d, out, s, s2)
        B = oracle.noise_bound(p, mods, level, h)
        assert max(abs(v) for v in r) <= B
