"""Pins of the 64-bit-word oracle (oracle/ks_oracle64.c): towers of ~60-bit
primes in uint64 words (Sec. II word-size moduli).

Every function is pinned by a fact that does not come from the oracle
itself:
- moduli: a Lucas certificate for every accepted prime (the factors of
  q - 1 found by a sieve, a witness of order q - 1), a Fermat witness or a
  factor for every skipped candidate, and the range and residue class;
- psi: x^N = -1 by Python's pow, and minimality over all N solutions,
  listed from a primitive root found through the certificate (not from a
  quadratic non-residue, as the oracle does);
- NTT: Horner evaluation at the N roots of X^N + 1 with Python integers,
  the convolution theorem against a Python schoolbook negacyclic product,
  monomials, and the round trip;
- basis conversion: the big-integer identity y = X + u Q (one integer u in
  [0, |S|) per coefficient, shared by every target);
- ModDown: the big-integer identity out = (C - [C]_P)/P - v, v in [0, K);
- the key switch: decryption within the bound derived in
  test_oracle_keyswitch.py (it holds for any word size), d = 0 gives 0, and
  planted mistakes break the bound;
- compressed keys (Sec. IV-D): every a-half word satisfies a 2^64 = x
  (mod m) for the generator's output x at its counter, the words are
  uniform, and a key built on them decrypts within the bound.
"""
import numpy as np
import pytest

import oracle
from oracle import core, core64 as o64


def _sieve(limit):
    s = np.ones(limit + 1, bool)
    s[:2] = False
    for i in range(2, int(limit ** 0.5) + 1):
        if s[i]:
            s[i * i::i] = False
    return np.nonzero(s)[0].astype(np.int64)


SMALL_PRIMES = _sieve(1 << 24)


def factor(n):
    """Distinct prime factors of n < 2^63: every factor below 2^24 from the
    sieve; what remains is 1 or, when below 2^48, a prime (a composite
    without factors below 2^24 is at least 2^48)."""
    assert n < (1 << 63)
    fs = []
    for p in SMALL_PRIMES[(n % SMALL_PRIMES) == 0].tolist():
        fs.append(p)
        while n % p == 0:
            n //= p
    if n > 1:
        assert n < (1 << 48), "cofactor too large for the sieve argument"
        fs.append(n)
    return fs


def lucas_prime(q):
    """q is prime iff some a has order q - 1 (Lucas): a^(q-1) = 1 and
    a^((q-1)/p) != 1 for every prime p | q - 1.  Returns (is_prime, a, fs)."""
    fs = factor(q - 1)
    for a in range(2, 200):
        if pow(a, q - 1, q) != 1:
            return False, None, fs
        if all(pow(a, (q - 1) // p, q) != 1 for p in fs):
            return True, a, fs
    return False, None, fs


@pytest.mark.parametrize("log_n", [12, 14, 16, 17])
def test_moduli_are_the_first_primes_of_the_sequence(log_n):
    count = 12
    got = [int(v) for v in o64.gen_primes(log_n, count)]
    two_n = 2 << log_n
    t, k = 1, 0
    while k < count:
        c = (1 << 60) - t * two_n + 1
        if c == got[k]:
            ok, a, fs = lucas_prime(c)
            assert ok, (c, fs)
            assert (1 << 59) < c < (1 << 60) and c % two_n == 1
            k += 1
        else:  # a skipped candidate must be composite
            assert c > got[k]
            fermat = any(pow(b, c - 1, c) != 1 for b in (2, 3, 5, 7, 11, 13))
            assert fermat or any(c % p == 0 for p in SMALL_PRIMES[:100000].tolist()), c
        t += 1
    assert len(set(got)) == count


def test_moduli_of_a_parameter_set():
    p = oracle.Params(13, 5, 2, 3)
    mods = [int(v) for v in o64.moduli(p)]
    pr = [int(v) for v in o64.gen_primes(13, 8)]
    assert mods == pr[3:] + pr[:3]  # q_0..q_L are primes K.., p_k the first K


@pytest.mark.parametrize("log_n", [12, 16, 17])
def test_psi_is_the_smallest_root_of_x_n_plus_1(log_n):
    n = 1 << log_n
    for q in [int(v) for v in o64.gen_primes(log_n, 2)]:
        psi = o64.min_psi(q, log_n)
        assert pow(psi, n, q) == q - 1
        ok, g, _ = lucas_prime(q)  # g has order q - 1: a primitive root
        assert ok
        root = pow(g, (q - 1) // (2 * n), q)
        sq, x, best = root * root % q, root, root
        for _ in range(n - 1):
            x = x * sq % q
            best = min(best, x)
        assert psi == best


def _uniform64(mods, n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, int(q), n, dtype=np.uint64) for q in mods])


@pytest.mark.parametrize("log_n", [3, 5, 6])
def test_ntt_is_evaluation_at_the_roots(log_n):
    n = 1 << log_n
    q = int(o64.gen_primes(log_n, 1)[0])
    psi = o64.min_psi(q, log_n)
    a = _uniform64([q], n, log_n)[0]
    got = o64.ntt(a, q, psi)
    brv = lambda j: int(format(j, f"0{log_n}b")[::-1], 2)
    for j in range(n):
        x = pow(psi, 2 * brv(j) + 1, q)
        acc = 0
        for c in reversed(a.tolist()):
            acc = (acc * x + c) % q
        assert int(got[j]) == acc
    assert np.array_equal(o64.ntt_direct(a, q, psi), got)


@pytest.mark.parametrize("log_n", [8, 10])
def test_convolution_theorem_against_python_schoolbook(log_n):
    n = 1 << log_n
    q = int(o64.gen_primes(log_n, 2)[1])
    a, b = _uniform64([q, q], n, 3 + log_n)
    c = [0] * n
    al, bl = a.tolist(), b.tolist()
    for i in range(n):
        for j in range(n):
            if i + j < n:
                c[i + j] += al[i] * bl[j]
            else:
                c[i + j - n] -= al[i] * bl[j]
    want = np.array([v % q for v in c], np.uint64)
    ha, hb = o64.ntt(a, q), o64.ntt(b, q)
    prod_eval = np.array([int(x) * int(y) % q for x, y in zip(ha, hb)], np.uint64)
    assert np.array_equal(o64.intt(prod_eval, q), want)
    if log_n == 8:
        assert np.array_equal(o64.negacyclic_mul(a, b, q), want)


def test_monomials_and_round_trip():
    log_n, n = 12, 1 << 12
    q = int(o64.gen_primes(log_n, 1)[0])
    psi = o64.min_psi(q, log_n)
    brv = lambda j: int(format(j, f"0{log_n}b")[::-1], 2)
    for k in (0, 1, 7, n - 1):
        e = np.zeros(n, np.uint64)
        e[k] = 1
        got = o64.ntt(e, q, psi)
        for j in (0, 1, 2, n // 2, n - 1):
            assert int(got[j]) == pow(psi, (2 * brv(j) + 1) * k, q)
    a = _uniform64([q], n, 77)[0]
    assert np.array_equal(o64.intt(o64.ntt(a, q, psi), q, psi), a)


@pytest.mark.parametrize("ns,nt", [(1, 3), (3, 4), (5, 2)])
def test_bconv_bigint_identity(ns, nt):
    log_n, n = 4, 16
    pr = [int(v) for v in o64.gen_primes(log_n, ns + nt)]
    src, dst = pr[:ns], pr[ns:]
    x = _uniform64(src, n, ns * 10 + nt)
    y = o64.bconv(x, src, dst)
    Q = oracle.prod(src)
    X = oracle.crt(x, src)
    for z in range(n):
        us = set()
        for t, m in enumerate(dst):
            # y = X + u Q (mod m) for some integer u in [0, ns)
            cands = [u for u in range(ns) if (X[z] + u * Q - int(y[t, z])) % m == 0]
            assert len(cands) == 1, (z, t, cands)
            us.add(cands[0])
        assert len(us) == 1  # one u shared by every target


def test_moddown_identity_bigint():
    """All-one key at dnum = 1: ModDown returns (C - [C]_P)/P - v mod Q_l
    with C the CRT value of the accumulator over D_l and v in [0, K)."""
    p = oracle.Params(6, 3, 1, 3)
    mods = [int(x) for x in o64.moduli(p)]
    n = p.n
    ones = np.ones((1, 2, 6, n), np.uint64)
    d = _uniform64(mods[:3], n, 9)
    out = o64.keyswitch(p, mods, 2, ones, d)
    x = np.stack([o64.intt(d[i], mods[i]) for i in range(3)])
    ext = o64.bconv(x, mods[:3], mods[3:])
    acc = np.concatenate([d, np.stack([o64.ntt(ext[k], mods[3 + k]) for k in range(3)])])
    coef = np.stack([o64.intt(acc[t], (mods[:3] + mods[3:])[t]) for t in range(6)])
    C = oracle.crt(coef, mods[:3] + mods[3:])
    P = oracle.prod(mods[3:])
    G = oracle.crt(np.stack([o64.intt(out[0, i], mods[i]) for i in range(3)]), mods[:3])
    Q = oracle.prod(mods[:3])
    for z in range(n):
        v = ((C[z] - C[z] % P) // P - G[z]) % Q
        assert 0 <= v < 3, (z, v)


CASES = [
    (12, 4, 2, 2, [0, 1, 3]),   # the plain workload's shape
    (10, 5, 2, 0, [4, 2]),      # partial last digit
    (10, 4, 1, 0, [3]),         # dnum = 1
    (9, 9, 3, 2, [8, 4]),       # K != alpha
    (9, 7, 7, 1, [6]),          # alpha = 1
]


@pytest.mark.parametrize("log_n,num_q,dnum,num_p,levels", CASES)
def test_decrypts_within_bound(log_n, num_q, dnum, num_p, levels):
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = o64.moduli(p)
    s, s2, evk, h = o64.keygen(p, mods, seed=31 + log_n + num_q)
    for level in levels:
        d = _uniform64(mods[:level + 1], p.n, level)
        out = o64.keyswitch(p, mods, level, evk, d)
        assert out.dtype == np.uint64 and out.shape == (2, level + 1, p.n)
        for i in range(level + 1):
            assert int(out[:, i].max()) < int(mods[i])
        r = o64.decrypt_residual(p, mods, level, d, out, s, s2)
        B = oracle.noise_bound(p, mods, level, h)
        assert max(abs(v) for v in r) <= B
        assert B < oracle.prod(mods[:level + 1]) // 4


def test_zero_input_gives_zero():
    p = oracle.Params(10, 4, 2, 2)
    mods = o64.moduli(p)
    _, _, evk, _ = o64.keygen(p, mods, seed=1)
    assert not o64.keyswitch(p, mods, 3, evk, np.zeros((4, p.n), np.uint64)).any()


@pytest.mark.parametrize("fault", [1, 2, 3, 4])
def test_planted_mistakes_break_the_bound(fault):
    p = oracle.Params(10, 4, 2, 2)
    mods = o64.moduli(p)
    s, s2, evk, h = o64.keygen(p, mods, seed=4)
    d = _uniform64(mods[:4], p.n, 8)
    o64.set_fault(fault)
    try:
        out = o64.keyswitch(p, mods, 3, evk, d)
    finally:
        o64.set_fault(0)
    r = o64.decrypt_residual(p, mods, 3, d, out, s, s2)
    assert max(abs(v) for v in r) > oracle.noise_bound(p, mods, 3, h)


# ---- key compression with 64-bit words (Sec. IV-D) -------------------------
# Word (j, g, k) of the a halves is X 2^-64 mod m_g, X = (x1 >> 5) 2^64 + x0
# for the SplitMix64 outputs x0, x1 at counters 2t, 2t + 1 of the word's
# counter t = (j (L+1+K) + g) N + k (123 bits, so the words sit below 2^-65
# from uniform, where one 64-bit output mod a 60-bit prime would sit up to
# 2^-6 away): pinned by the defining property a 2^64 = X (mod m_g) on every
# word (the generator itself is pinned against its published outputs in
# test_oracle_seeded.py), uniformity, and decryption of a key switch with a
# key built on them.

def test_seeded_a64_words_satisfy_the_defining_property():
    p = oracle.Params(6, 3, 2, 2)
    mods = [int(v) for v in o64.moduli(p)]
    ev = o64.seeded_a(p, mods, 0x5eed)
    EL = p.num_q + p.num_p
    for j in range(p.dnum):
        for g in range(EL):
            m = mods[g]
            for k in range(p.n):
                t = (j * EL + g) * p.n + k
                x = ((core.splitmix_at(0x5eed, 2 * t + 1) >> 5) << 64) + core.splitmix_at(0x5eed, 2 * t)
                a = int(ev[j, 1, g, k])
                assert a < m and (a * (1 << 64) - x) % m == 0, (j, g, k)
    assert not ev[:, 0].any()


def test_seeded_a64_is_uniform():
    p = oracle.Params(12, 4, 2, 2)
    mods = [int(v) for v in o64.moduli(p)]
    ev = o64.seeded_a(p, mods, 91)
    for g in range(p.num_q + p.num_p):
        m = mods[g]
        for j in range(p.dnum):
            a = ev[j, 1, g].astype(np.float64)
            counts = np.bincount((a * 16 / m).astype(np.int64), minlength=16)
            exp = p.n / 16
            chi2 = float(((counts - exp) ** 2 / exp).sum())
            assert chi2 < 45.0, (g, j, chi2)  # 15 dof: p < 1e-4 under uniformity
    assert np.mean(ev[:, 1] == o64.seeded_a(p, mods, 92)[:, 1]) < 1e-3


@pytest.mark.parametrize("log_n,num_q,dnum,num_p,level", [(10, 4, 2, 2, 3), (9, 9, 3, 2, 5)])
def test_seeded_key64_decrypts_within_bound(log_n, num_q, dnum, num_p, level):
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = o64.moduli(p)
    s, s2, evk, h = o64.keygen_seeded(p, mods, 17, 4242)
    assert np.array_equal(evk[:, 1], o64.seeded_a(p, mods, 4242)[:, 1])
    d = _uniform64(mods[:level + 1], p.n, 5)
    out = o64.keyswitch(p, mods, level, evk, d)
    r = o64.decrypt_residual(p, mods, level, d, out, s, s2)
    assert max(abs(v) for v in r) <= oracle.noise_bound(p, mods, level, h)
