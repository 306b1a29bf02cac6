"""Pins of the CPU oracle against facts outside the oracle itself.

Each check ties an oracle function to a textbook definition evaluated a
different way, an exact big-integer identity, a closed-form bound, or a value
the paper prints (Table III).  None of these tests needs a GPU.
"""
import json
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ moduli
@pytest.mark.parametrize("log_n", [4, 6, 12, 16, 17])
def test_primes_are_the_ordered_ntt_friendly_primes(log_n):
    """Candidates 2^30 - t*2N + 1 in t order: every returned value is prime
    (Fermat witnesses 2,3,5,7 plus a distinct factor search) and every skipped
    candidate has an explicit factor."""
    two_n = 2 << log_n
    pr = [int(x) for x in oracle.gen_primes(log_n, 20)]
    assert len(set(pr)) == 20
    t, got = 1, []
    while len(got) < 20:
        c = (1 << 30) - t * two_n + 1
        small = next((f for f in range(3, 40000, 2) if c % f == 0 and f < c), None)
        if small is None:
            assert all(pow(a, c - 1, c) == 1 for a in (2, 3, 5, 7))
            got.append(c)
        t += 1
    assert got == pr
    for q in pr:
        assert q % two_n == 1 and (1 << 29) < q < (1 << 30)


def test_moduli_order_p_first_then_q():
    p = oracle.Params(12, 4, 2, 2)
    m = [int(x) for x in oracle.moduli(p)]
    pr = [int(x) for x in oracle.gen_primes(12, 6)]
    assert m[4:] == pr[:2] and m[:4] == pr[2:]
    # P (the two largest) exceeds every digit modulus Q_j
    P = m[4] * m[5]
    assert P > m[0] * m[1] and P > m[2] * m[3]


@pytest.mark.parametrize("log_n", [12, 14, 16])
def test_psi_is_smallest_primitive_2n_root(log_n):
    n = 1 << log_n
    for q in oracle.gen_primes(log_n, 2):
        q = int(q)
        psi = oracle.min_psi(q, log_n)
        assert pow(psi, n, q) == q - 1 and pow(psi, 2 * n, q) == 1
        # brute force: no x in [2, psi) is a root of X^N + 1
        assert all(pow(x, n, q) != q - 1 for x in range(2, psi))


# ------------------------------------------------------------------ NTT
def _horner_eval(a, x, q):
    acc = 0
    for c in reversed([int(v) for v in a]):
        acc = (acc * x + c) % q
    return acc


@pytest.mark.parametrize("log_n", [5, 6, 7])
def test_ntt_is_evaluation_at_roots_of_xn_plus_1(log_n):
    """The evaluation points psi^(2 brv(j)+1) are exactly the N distinct roots
    of X^N+1, and NTT(a)[j] is a evaluated there (Horner, Python ints)."""
    n = 1 << log_n
    rng = np.random.default_rng(log_n)
    for q in oracle.gen_primes(log_n, 2):
        q = int(q)
        psi = oracle.min_psi(q, log_n)
        pts = [pow(psi, 2 * oracle.bitrev(j, log_n) + 1, q) for j in range(n)]
        assert len(set(pts)) == n and all(pow(x, n, q) == q - 1 for x in pts)
        a = rng.integers(0, q, n, dtype=np.uint64).astype(np.uint32)
        want = [_horner_eval(a, x, q) for x in pts]
        assert oracle.ntt(a, q, psi).tolist() == want
        assert oracle.ntt_direct(a, q, psi).tolist() == want


def _schoolbook_py(a, b, q):
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                c[k] += int(a[i]) * int(b[j])
            else:
                c[k - n] -= int(a[i]) * int(b[j])
    return [v % q for v in c]


def test_schoolbook_matches_python_definition():
    q = int(oracle.gen_primes(6, 1)[0])
    rng = np.random.default_rng(7)
    a = rng.integers(0, q, 64, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, q, 64, dtype=np.uint64).astype(np.uint32)
    assert oracle.negacyclic_mul(a, b, q).tolist() == _schoolbook_py(a, b, q)


@pytest.mark.parametrize("log_n", [7, 10, 12])
def test_convolution_theorem_against_schoolbook(log_n):
    """NTT(a) * NTT(b) = NTT(a*b mod X^N+1): the transform is the ring
    isomorphism the key switch relies on (Sec. II)."""
    n = 1 << log_n
    rng = np.random.default_rng(100 + log_n)
    q = int(oracle.gen_primes(log_n, 1)[0])
    a = rng.integers(0, q, n, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, q, n, dtype=np.uint64).astype(np.uint32)
    c = oracle.negacyclic_mul(a, b, q)
    prod_hat = (oracle.ntt(a, q).astype(np.uint64) * oracle.ntt(b, q).astype(np.uint64)) % q
    assert np.array_equal(prod_hat.astype(np.uint32), oracle.ntt(c, q))
    assert np.array_equal(oracle.intt(oracle.ntt(a, q), q), a)


def test_ntt_of_monomials():
    """NTT(X^k)[j] = psi^((2 brv(j)+1) k): a closed form per coefficient."""
    log_n, n = 6, 64
    q = int(oracle.gen_primes(log_n, 1)[0])
    psi = oracle.min_psi(q, log_n)
    for k in (0, 1, 7, 31):
        a = np.zeros(n, np.uint32)
        a[k] = 1
        want = [pow(psi, (2 * oracle.bitrev(j, log_n) + 1) * k, q) for j in range(n)]
        assert oracle.ntt(a, q).tolist() == want


# ------------------------------------------------------------------ basis conversion
def test_bconv_is_crt_value_plus_small_multiple():
    """Fast basis conversion returns X + u*Q_src for one integer u in
    [0, |src|) shared by every target modulus (exact big-integer check)."""
    rng = np.random.default_rng(3)
    pr = [int(x) for x in oracle.gen_primes(4, 9)]
    src, dst = pr[:4], pr[4:]
    n = 16
    x = np.stack([rng.integers(0, q, n, dtype=np.uint64) for q in src]).astype(np.uint32)
    y = oracle.bconv(x, src, dst)
    X = oracle.crt(x, src)
    Q = oracle.prod(src)
    for z in range(n):
        us = set()
        for t, m in enumerate(dst):
            u = ((int(y[t, z]) - X[z]) * pow(Q % m, -1, m)) % m
            us.add(u)
        assert len(us) == 1 and 0 <= us.pop() < len(src)


def test_bconv_single_source_is_plain_reduction():
    """With one source modulus the conversion is exact: y = x mod m."""
    pr = [int(x) for x in oracle.gen_primes(4, 3)]
    x = np.arange(16, dtype=np.uint32) * 1234567 % pr[0]
    y = oracle.bconv(x[None, :], pr[:1], pr[1:])
    for t, m in enumerate(pr[1:]):
        assert y[t].tolist() == [int(v) % m for v in x]


# ------------------------------------------------------------------ Table III
def test_table3_evk_sizes_pin_the_evk_shape():
    """evk shape dnum x 2 x N x (L+1+K) (Sec. III-B, P4) reproduces every evk
    size printed in Table III with the paper's 8-byte words."""
    g = json.load(open(os.path.join(HERE, "golden", "table3_params.json")))
    for r in g["rows"]:
        words = oracle.evk_words(r["log_n"], r["k_l"], r["k_p"], r["dnum"])
        assert words * g["word_bytes"] == r["evk_mb"] * 2**20, r["name"]
        assert r["alpha"] == -(-r["k_l"] // r["dnum"]), r["name"]
