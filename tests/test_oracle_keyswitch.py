"""End-to-end pins of the oracle's hybrid key switch (Sec. III).

The key switch has no shorter closed form: many outputs decrypt correctly.
What fixes it is (a) the decryption bound: c0 + c1*s - d*s2 is small modulo
Q_l, with the bound derived below; (b) exact special cases; (c) the
ModDown identity checked with big integers; (d) planted mistakes in the
oracle that these checks must catch.

Derivation of the bound.  ModUp turns digit j (towers S_j, modulus Q_j) into
D_j + u_j Q_j with 0 <= u_j < |S_j|, so every coefficient lies in
[0, |S_j| Q_j).  The key for digit j satisfies b_j + a_j s = e_j + g_j s2
with g_j = P on the digit's towers and 0 elsewhere, so
    c0' + c1' s = P d s2 + sum_j (D_j + u_j Q_j) e_j      (mod P Q_l),
because u_j Q_j g_j = 0 mod P Q_l.  With |e| <= B_e the error term is at
most E = sum_j N |S_j| Q_j B_e.  ModDown returns (c' - [c']_P)/P - v with
0 <= v < K, so the residual is at most E/P + (1 + h) + (K - 1)(1 + h),
bounded by B = floor(E/P) + (1 + h)(1 + K), h = ||s||_1.
"""
import numpy as np
import pytest

import oracle


def _uniform(mods, n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, int(q), n, dtype=np.uint64) for q in mods]).astype(np.uint32)


CASES = [
    # (log_n, num_q, dnum, num_p, levels)
    (12, 4, 2, 2, [0, 1, 2, 3]),      # the plain single-ciphertext workload
    (10, 5, 2, 0, [4, 2]),            # partial last digit (alpha 3: digits 3+2)
    (10, 4, 1, 0, [3, 1]),            # dnum = 1: one conversion Q -> P
    (10, 6, 3, 3, [5, 3, 0]),
    (9, 9, 3, 2, [8, 4]),             # K != alpha (alpha 3, K 2)
    (9, 7, 7, 1, [6, 3]),             # alpha = 1
]


@pytest.mark.parametrize("log_n,num_q,dnum,num_p,levels", CASES)
def test_decrypts_within_bound(log_n, num_q, dnum, num_p, levels):
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = oracle.moduli(p)
    s, s2, evk, h = oracle.keygen(p, mods, seed=11 + log_n + num_q)
    for level in levels:
        d = _uniform(mods[:level + 1], p.n, seed=level)
        out = oracle.keyswitch(p, mods, level, evk, d)
        assert out.dtype == np.uint32 and out.shape == (2, level + 1, p.n)
        for i in range(level + 1):
            assert int(out[:, i].max()) < int(mods[i])
        r = oracle.decrypt_residual(p, mods, level, d, out, s, s2)
        B = oracle.noise_bound(p, mods, level, h)
        Q = oracle.prod(mods[:level + 1])
        worst = max(abs(v) for v in r)
        assert worst <= B, (level, worst, B)
        assert B < Q // 4  # the check is decisive: a wrong result is ~Q/2


@pytest.mark.parametrize("log_n,num_q,dnum,num_p,levels", CASES[:4])
def test_output_centric_order_matches(log_n, num_q, dnum, num_p, levels):
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = oracle.moduli(p)
    rng = np.random.default_rng(5)
    evk = np.stack([rng.integers(0, int(q), (p.dnum, 2, p.n), dtype=np.uint64) for q in mods], axis=2)
    evk = evk.astype(np.uint32)
    for level in levels:
        d = _uniform(mods[:level + 1], p.n, seed=20 + level)
        assert np.array_equal(oracle.keyswitch(p, mods, level, evk, d),
                              oracle.keyswitch(p, mods, level, evk, d, order="oc"))


def test_zero_input_gives_zero():
    p = oracle.Params(10, 4, 2, 2)
    mods = oracle.moduli(p)
    _, _, evk, _ = oracle.keygen(p, mods, seed=1)
    out = oracle.keyswitch(p, mods, 3, evk, np.zeros((4, p.n), np.uint32))
    assert not out.any()


def test_moddown_identity_bigint():
    """With an all-one key at dnum = 1 the ModUp output is known exactly, and
    ModDown must return (C - [C]_P)/P - v mod Q_l with C the CRT value over
    D_l and one integer v in [0, K) per coefficient."""
    p = oracle.Params(6, 3, 1, 3)
    mods = [int(x) for x in oracle.moduli(p)]
    level = 2
    n = p.n
    ones = np.ones((1, 2, 6, n), np.uint32)
    d = _uniform(mods[:3], n, seed=9)
    out = oracle.keyswitch(p, mods, level, ones, d)
    # ModUp with a unit key: the accumulator is the digit extended to D_l
    x = np.stack([oracle.intt(d[i], mods[i]) for i in range(3)])
    ext = oracle.bconv(x, mods[:3], mods[3:])
    acc_p = np.stack([oracle.ntt(ext[k], mods[3 + k]) for k in range(3)])
    acc = np.concatenate([d, acc_p])
    coef = np.stack([oracle.intt(acc[t], (mods[:3] + mods[3:])[t]) for t in range(6)])
    C = oracle.crt(coef, mods[:3] + mods[3:])
    P = oracle.prod(mods[3:])
    want = [(c - c % P) // P for c in C]
    got_coef = np.stack([oracle.intt(out[0, i], mods[i]) for i in range(3)])
    G = oracle.crt(got_coef, mods[:3])
    Q = oracle.prod(mods[:3])
    for z in range(n):
        v = (want[z] - G[z]) % Q
        assert 0 <= v < 3, (z, v)


@pytest.mark.parametrize("fault", [1, 2, 3, 4])
def test_planted_mistakes_break_the_bound(fault):
    """Each planted mistake (dropped digit, wrong ModDown sign, wrong BConv
    constant, wrong bypass tower) makes the decryption residual ~Q_l."""
    p = oracle.Params(10, 4, 2, 2)
    mods = oracle.moduli(p)
    s, s2, evk, h = oracle.keygen(p, mods, seed=4)
    d = _uniform(mods[:4], p.n, seed=8)
    oracle.set_fault(fault)
    try:
        out = oracle.keyswitch(p, mods, 3, evk, d)
    finally:
        oracle.set_fault(0)
    r = oracle.decrypt_residual(p, mods, 3, d, out, s, s2)
    assert max(abs(v) for v in r) > oracle.noise_bound(p, mods, 3, h)


def test_wrong_secret_fails_the_bound():
    p = oracle.Params(10, 4, 2, 2)
    mods = oracle.moduli(p)
    s, s2, evk, h = oracle.keygen(p, mods, seed=4)
    d = _uniform(mods[:4], p.n, seed=8)
    out = oracle.keyswitch(p, mods, 3, evk, d)
    r = oracle.decrypt_residual(p, mods, 3, d, out, -s, s2)
    assert max(abs(v) for v in r) > oracle.noise_bound(p, mods, 3, h)
