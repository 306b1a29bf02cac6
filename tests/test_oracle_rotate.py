"""Pins of the oracle's callers of the key switch (Sec. II: rotations and
multiplications are what need it): automorphisms, hoisted rotations and
multiplication with relinearisation.

* The coefficient automorphism equals a(X^k) reduced modulo X^N + 1,
  written out here with Python integers; the evaluation-domain one equals
  NTT(a(X^k)) (the NTT itself is pinned to evaluation at the roots of
  X^N + 1); both compose (k1 then k2 is k1 k2 mod 2N) and k = 1 is the
  identity; the rotation element 5 has order N/2.
* Rotations decrypt: with a key from s(X^k) to s, c0' + c1' s equals
  sigma(c0 + c1 s) up to the key switch's error bound, for several Galois
  elements sharing one ModUp, hoisted or not; k = 1 (identity) gives exactly
  the key switch of c1 plus (c0, 0).
* Multiplication decrypts: c0' + c1' s = (a0 + a1 s)(b0 + b1 s) up to the
  bound, with a key from s^2 to s.
* The planted key-switch mistakes break the rotation's bound too.
"""
import numpy as np
import pytest

import oracle
from oracle import core


def _poly_subst(a, k, q):
    """a(X^k) mod (X^N + 1, q) with Python integers, term by term."""
    n = len(a)
    out = [0] * n
    for i, c in enumerate(int(x) for x in a):
        e = i * k
        sign = -1 if (e // n) % 2 else 1  # X^N = -1
        out[e % n] = (out[e % n] + sign * c) % q
    return np.array(out, np.uint32)


@pytest.mark.parametrize("log_n,k", [(4, 3), (5, 5), (6, 127), (8, 5 ** 3 % 512), (10, 2047)])
def test_coefficient_automorphism_is_substitution(log_n, k):
    q = int(oracle.gen_primes(max(log_n, 12), 1)[0])
    rng = np.random.default_rng(log_n)
    a = rng.integers(0, q, 1 << log_n, dtype=np.uint64).astype(np.uint32)
    assert np.array_equal(core.automorphism_coeff(a, log_n, k, q), _poly_subst(a, k, q))


@pytest.mark.parametrize("log_n", [12, 13])
def test_eval_automorphism_is_ntt_of_substitution(log_n):
    q = int(oracle.gen_primes(log_n, 2)[1])
    rng = np.random.default_rng(7)
    a = rng.integers(0, q, 1 << log_n, dtype=np.uint64).astype(np.uint32)
    ah = oracle.ntt(a, q)
    for k in (5, core.galois_rotation(log_n, 3), core.galois_rotation(log_n, -1), (2 << log_n) - 1, 1):
        want = oracle.ntt(core.automorphism_coeff(a, log_n, k, q), q)
        assert np.array_equal(core.automorphism_eval(ah, log_n, k), want), k


def test_automorphisms_compose_and_identity():
    log_n = 10
    two_n = 2 << log_n
    a = np.arange(1 << log_n, dtype=np.uint32)
    assert np.array_equal(core.automorphism_eval(a, log_n, 1), a)
    for k1, k2 in ((5, 25), (3, 2 * two_n // 2 - 1), (125, 7)):
        both = core.automorphism_eval(core.automorphism_eval(a, log_n, k1), log_n, k2)
        assert np.array_equal(both, core.automorphism_eval(a, log_n, k1 * k2 % two_n))
        assert sorted(core.automorphism_eval(a, log_n, k1).tolist()) == a.tolist()  # a permutation
    # 5 generates a cyclic group of order N/2 (the slot rotations)
    assert core.galois_rotation(log_n, (1 << log_n) // 2) == 1
    assert core.galois_rotation(log_n, 1) == 5
    with pytest.raises(ValueError):
        core.automorphism_eval(a, log_n, 4)  # even: not an automorphism


def _cipher(p, mods, level, seed):
    rng = np.random.default_rng(seed)
    return [np.stack([rng.integers(0, int(q), p.n, dtype=np.uint64) for q in mods[:level + 1]]).astype(np.uint32)
            for _ in range(2)]


def _sub(a, b, mods):
    return np.stack([((a[i].astype(np.int64) - b[i]) % int(mods[i])) for i in range(len(a))]).astype(np.uint32)


CASES = [(12, 4, 2, 2, 3), (10, 6, 3, 3, 4), (10, 5, 2, 0, 2)]


@pytest.mark.parametrize("log_n,num_q,dnum,num_p,level", CASES)
def test_hoisted_rotations_decrypt(log_n, num_q, dnum, num_p, level):
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = oracle.moduli(p)
    c0, c1 = _cipher(p, mods, level, 3)
    gal = [core.galois_rotation(log_n, r) for r in (1, 2, -1)] + [(2 << log_n) - 1]
    keys = [core.keygen_rotation(p, mods, 40 + i, k) for i, k in enumerate(gal)]
    # one secret s for every key would be needed by a real scheme; the
    # check below is per key, so each key may carry its own s
    outs = core.rotate_hoisted(p, mods, level, c0, c1, gal, [k[2] for k in keys])
    for k, (s, sk, _, h), out in zip(gal, keys, outs):
        sc0 = core.automorphism_eval(c0, log_n, k)
        sc1 = core.automorphism_eval(c1, log_n, k)
        r = oracle.decrypt_residual(p, mods, level, sc1, np.stack([_sub(out[0], sc0, mods), out[1]]), s, sk)
        assert max(abs(v) for v in r) <= oracle.noise_bound(p, mods, level, h), k
        # not hoisted: a different result, the same guarantee
        plain = core.rotate(p, mods, level, c0, c1, k, keys[gal.index(k)][2])
        r2 = oracle.decrypt_residual(p, mods, level, sc1, np.stack([_sub(plain[0], sc0, mods), plain[1]]), s, sk)
        assert max(abs(v) for v in r2) <= oracle.noise_bound(p, mods, level, h)
    # each output is the single-rotation output (rotations are independent)
    one = core.rotate_hoisted(p, mods, level, c0, c1, gal[1:2], [keys[1][2]])
    assert np.array_equal(one[0], outs[1])


def test_identity_rotation_is_the_key_switch():
    p = oracle.Params(12, 4, 2, 2)
    mods = oracle.moduli(p)
    c0, c1 = _cipher(p, mods, 3, 5)
    s, sk, evk, h = core.keygen_rotation(p, mods, 9, 1)
    assert np.array_equal(s, sk)
    out = core.rotate_hoisted(p, mods, 3, c0, c1, [1], [evk])[0]
    ks = oracle.keyswitch(p, mods, 3, evk, c1)
    assert np.array_equal(out[1], ks[1])
    assert np.array_equal(out[0], np.stack([(ks[0][i].astype(np.uint64) + c0[i]) % int(mods[i])
                                            for i in range(4)]).astype(np.uint32))


def _negacyclic_square(s):
    n = len(s)
    full = np.convolve(s.astype(np.int64), s.astype(np.int64))
    out = full[:n].copy()
    out[:len(full) - n] -= full[n:]
    return out


@pytest.mark.parametrize("log_n,num_q,dnum,num_p,level", CASES[:2])
def test_mult_relin_decrypts(log_n, num_q, dnum, num_p, level):
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = oracle.moduli(p)
    s, evk, h = core.keygen_relin(p, mods, 77)
    a0, a1 = _cipher(p, mods, level, 11)
    b0, b1 = _cipher(p, mods, level, 12)
    out = core.mult_relin(p, mods, level, a0, a1, b0, b1, evk)
    l1 = level + 1
    d = [np.stack([(x[i].astype(np.uint64) * y[i] % int(mods[i])) for i in range(l1)]).astype(np.uint32)
         for x, y in ((a0, b0), (a0, b1), (a1, b0), (a1, b1))]
    d0, d1 = d[0], np.stack([(d[1][i].astype(np.uint64) + d[2][i]) % int(mods[i]) for i in range(l1)]).astype(np.uint32)
    s2 = _negacyclic_square(s)
    r = oracle.decrypt_residual(p, mods, level, d[3], np.stack([_sub(out[0], d0, mods), _sub(out[1], d1, mods)]), s, s2)
    assert max(abs(v) for v in r) <= oracle.noise_bound(p, mods, level, h)


@pytest.mark.parametrize("fault", [1, 2, 4, 5])  # 5: the inverse permutation of the digits
def test_planted_mistakes_break_the_rotation_bound(fault):
    p = oracle.Params(12, 4, 2, 2)
    mods = oracle.moduli(p)
    c0, c1 = _cipher(p, mods, 3, 21)
    k = core.galois_rotation(12, 1)
    s, sk, evk, h = core.keygen_rotation(p, mods, 22, k)
    oracle.set_fault(fault)
    try:
        out = core.rotate_hoisted(p, mods, 3, c0, c1, [k], [evk])[0]
    finally:
        oracle.set_fault(0)
    sc0 = core.automorphism_eval(c0, 12, k)
    sc1 = core.automorphism_eval(c1, 12, k)
    r = oracle.decrypt_residual(p, mods, 3, sc1, np.stack([_sub(out[0], sc0, mods), out[1]]), s, sk)
    assert max(abs(v) for v in r) > oracle.noise_bound(p, mods, 3, h)


# ---------------------------------------------------------------- double hoisting

def _small_diag(p, mods, seed, bound=2):
    """A plaintext diagonal with coefficients in [-bound, bound], in the
    evaluation domain of every key row (q_0..q_L, p_0..p_{K-1})."""
    rng = np.random.default_rng(seed)
    coef = rng.integers(-bound, bound + 1, p.n)
    return np.stack([oracle.ntt(np.array([int(v) % int(m) for v in coef], np.uint32), int(m)) for m in mods]), coef


def _sum_residual(p, mods, level, c0, c1, out, s, sks, gal, coefs):
    """c0' + c1' s - sum_r p_r (sigma_r(c0) + sigma_r(c1) sigma_r(s)), centred."""
    l1 = level + 1
    r = np.zeros((l1, p.n), np.uint32)
    for i in range(l1):
        q = int(mods[i])
        f = lambda v: oracle.ntt(np.array([int(x) % q for x in v], np.uint32), q).astype(object)
        v = out[0, i].astype(object) + out[1, i].astype(object) * f(s)
        for k, sk, cf in zip(gal, sks, coefs):
            pr = f(cf) if cf is not None else 1
            sc0 = core.automorphism_eval(c0[i], p.log_n, k).astype(object)
            sc1 = core.automorphism_eval(c1[i], p.log_n, k).astype(object)
            v = v - pr * (sc0 + sc1 * f(sk))
        r[i] = oracle.intt(np.array([int(x) % q for x in v], np.uint32), q)
    Q = oracle.prod(mods[:l1])
    return [core.centre(v, Q) for v in core.crt(r, mods[:l1])]


def test_sum_of_one_rotation_is_the_hoisted_rotation():
    p = oracle.Params(12, 4, 2, 2)
    mods = oracle.moduli(p)
    c0, c1 = _cipher(p, mods, 3, 31)
    k = core.galois_rotation(12, 3)
    _, _, evk, _ = core.keygen_rotation(p, mods, 32, k)
    one = core.rotate_sum_hoisted(p, mods, 3, c0, c1, [k], [evk])
    assert np.array_equal(one, core.rotate_hoisted(p, mods, 3, c0, c1, [k], [evk])[0])
    ones = np.ones((1, p.num_q + p.num_p, p.n), np.uint32)
    assert np.array_equal(core.rotate_sum_hoisted(p, mods, 3, c0, c1, [k], [evk], ones), one)


@pytest.mark.parametrize("with_diag", [False, True])
def test_rotation_sum_decrypts(with_diag):
    p = oracle.Params(11, 5, 2, 3)
    mods = oracle.moduli(p)
    level = 4
    c0, c1 = _cipher(p, mods, level, 41)
    gal = [core.galois_rotation(11, r) for r in (0, 1, 2, 5)] + [(2 << 11) - 1]
    keys = [core.keygen_rotation(p, mods, 42, k) for k in gal]  # one seed: one secret s for every key
    s, h = keys[0][0], keys[0][3]
    assert all(np.array_equal(kk[0], s) for kk in keys)
    diags, coefs = None, [None] * len(gal)
    if with_diag:
        dd = [_small_diag(p, mods, 50 + i) for i in range(len(gal))]
        diags, coefs = [d[0] for d in dd], [d[1] for d in dd]
    out = core.rotate_sum_hoisted(p, mods, level, c0, c1, gal, [k[2] for k in keys], diags)
    r = _sum_residual(p, mods, level, c0, c1, out, s, [k[1] for k in keys], gal, coefs)
    # one ModDown for the sum: the key-switch error of every term, scaled by
    # the diagonal (at most N * 2 per coefficient), then one rounding
    E = oracle.noise_bound(p, mods, level, h) - (1 + h) * (1 + p.num_p)
    scale = p.n * 2 if with_diag else 1
    B = len(gal) * scale * (E + 1) + (1 + h) * (1 + p.num_p)
    assert max(abs(v) for v in r) <= B
    assert B < oracle.prod(mods[:level + 1]) // 4


@pytest.mark.parametrize("fault", [1, 2, 5])
def test_planted_mistakes_break_the_sum_bound(fault):
    p = oracle.Params(11, 5, 2, 3)
    mods = oracle.moduli(p)
    c0, c1 = _cipher(p, mods, 4, 61)
    gal = [core.galois_rotation(11, r) for r in (1, 3)]
    keys = [core.keygen_rotation(p, mods, 62, k) for k in gal]
    s, h = keys[0][0], keys[0][3]
    oracle.set_fault(fault)
    try:
        out = core.rotate_sum_hoisted(p, mods, 4, c0, c1, gal, [k[2] for k in keys])
    finally:
        oracle.set_fault(0)
    r = _sum_residual(p, mods, 4, c0, c1, out, s, [k[1] for k in keys], gal, [None, None])
    E = oracle.noise_bound(p, mods, 4, h) - (1 + h) * (1 + p.num_p)
    assert max(abs(v) for v in r) > len(gal) * (E + 1) + (1 + h) * (1 + p.num_p)
