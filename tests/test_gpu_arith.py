"""Unit test of the kernels' modular arithmetic on the GPU, primitive by
primitive, against a b mod q computed directly (numpy integers for 30-bit
moduli, Python integers for 64-bit ones).

ks_arith_probe / ks64_arith_probe apply the device functions the kernels use
-- Shoup products (with the companion derived on the device as the transform
tiles derive it), Montgomery reduction of one product and of a full chunk of
16 products, both Harvey butterflies, the final reductions, and for 64-bit
words the estimated-quotient Shoup product and the 30-bit-half accumulator --
to every pair of edge operands (0, 1, q - 1, q, 2q - 1, 4q - 1, 2^32 - 1,
...) and to about a million random pairs per 30-bit modulus.  Every result
must be the right residue and lie in the range the primitive promises.
"""
import random

import numpy as np
import pytest

import oracle
from oracle import core64 as o64

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_01598_amd as m
    return m


def _mods30():
    big = [int(m) for m in oracle.moduli(oracle.Params(17, 48, 3, 16))]
    small = [int(m) for m in oracle.moduli(oracle.Params(12, 4, 2, 2))]
    return sorted(set([big[0], big[-1], max(big), min(big), small[0], small[-1]]))


@pytest.mark.parametrize("q", _mods30())
def test_arith30_every_primitive(ks, q):
    E = [0, 1, 2, q - 2, q - 1, q, q + 1, 2 * q - 1, 2 * q, 2 * q + 1, 3 * q, 4 * q - 1, 4 * q, 2**30 - 1, 2**31,
         2**32 - 1]
    W = [0, 1, 2, q - 1, q - 2, (q - 1) // 2, q, 2**32 - 1]
    rng = np.random.default_rng(q)
    nr = 1 << 20
    a = np.concatenate([np.repeat(np.array(E, np.uint64), len(E)), rng.integers(0, 2**32, nr, dtype=np.uint64)])
    b = np.concatenate([np.tile(np.array(E, np.uint64), len(E)), rng.integers(0, 2**32, nr, dtype=np.uint64)])
    w = np.concatenate([np.array([W[i % len(W)] for i in range(len(E) ** 2)], np.uint64),
                        rng.integers(0, 2**32, nr, dtype=np.uint64)])
    n = a.size
    dev = lambda x: torch.from_numpy(x.astype(np.uint32).view(np.int32)).cuda()
    out = ks.ks_arith_probe(q, dev(a), dev(b), dev(w)).cpu().numpy().view(np.uint32).astype(np.uint64)
    Q = np.uint64(q)
    inv32 = np.uint64(pow(2**32, -1, q))
    ar, br, wc = a % Q, b % Q, w % Q
    prod = ar * br % Q
    assert np.array_equal(out[:, 0], ar * wc % Q), "Shoup product"
    assert np.array_equal(out[:, 1], prod * inv32 % Q), "REDC of one product"
    idx = np.arange(n)
    s = np.zeros(n, np.uint64)
    for k in range(16):
        s += prod[(idx + k) % n]
    assert np.array_equal(out[:, 2], (s % Q) * inv32 % Q), "REDC of 16 products"
    x, y = a % (4 * Q), b % (4 * Q)
    wy = wc * (y % Q) % Q
    assert (out[:, 3] < 4 * Q).all() and (out[:, 4] < 4 * Q).all(), "forward butterfly range"
    assert np.array_equal(out[:, 3] % Q, (x % Q + wy) % Q), "forward butterfly, sum"
    assert np.array_equal(out[:, 4] % Q, (x % Q + Q - wy) % Q), "forward butterfly, difference"
    u, v = a % (2 * Q), b % (2 * Q)
    assert (out[:, 5] < 2 * Q).all() and (out[:, 6] < 2 * Q).all(), "inverse butterfly range"
    assert np.array_equal(out[:, 5] % Q, (u + v) % Q), "inverse butterfly, sum"
    assert np.array_equal(out[:, 6] % Q, (u % Q + Q - v % Q) % Q * wc % Q), "inverse butterfly, product"
    assert np.array_equal(out[:, 7], x % Q), "[0, 4q) -> [0, q)"


def _mods64():
    m = [int(x) for x in o64.moduli(oracle.Params(17, 45, 3, 15))]
    return [m[0], m[-1], max(m), min(m)]


@pytest.mark.parametrize("q", _mods64())
def test_arith64_every_primitive(ks, q):
    E = [0, 1, 2, q - 1, q, q + 1, 2 * q - 1, 4 * q - 1, 8 * q - 1, 8 * q, 2**60 - 1, 2**63, 2**64 - 1]
    rnd = random.Random(q)
    inv64 = pow(2**64, -1, q)
    for w in (0, 1, q - 1, q // 3, rnd.randrange(q)):
        a = [x for x in E for _ in E] + [rnd.randrange(2**64) for _ in range(4096)]
        b = [y for _ in E for y in E] + [rnd.randrange(2**64) for _ in range(4096)]
        n = len(a)
        dev = lambda xs: torch.from_numpy(np.array(xs, np.uint64).view(np.int64)).cuda()
        out = ks.ks64_arith_probe(q, w, dev(a), dev(b)).cpu().numpy().view(np.uint64)
        prods = [(x % q) * (y % q) for x, y in zip(a, b)]
        for i in range(n):
            o = [int(v) for v in out[i]]
            ai, bi = a[i], b[i]
            assert o[0] == ai * w % q, (i, "Shoup product")
            assert o[1] < 4 * q and o[1] % q == ai * w % q, (i, "estimated-quotient product")
            assert o[2] == prods[i] * inv64 % q, (i, "REDC of one product")
            assert o[3] == sum(prods[(i + k) % n] for k in range(16)) * inv64 % q, (i, "REDC of 16 products")
            x, y = ai % (8 * q), bi % (8 * q)
            assert o[4] < 8 * q and o[5] < 8 * q, (i, "forward butterfly range")
            assert o[4] % q == (x + w * y) % q and o[5] % q == (x - w * y) % q, (i, "forward butterfly")
            u, v = ai % (4 * q), bi % (4 * q)
            assert o[6] < 4 * q and o[7] < 4 * q, (i, "inverse butterfly range")
            assert o[6] % q == (u + v) % q and o[7] % q == (u - v) * w % q, (i, "inverse butterfly")
            assert o[8] == x % q, (i, "[0, 8q) -> [0, q)")


def test_arith_probe_rejections(ks):
    a = torch.zeros(4, dtype=torch.int32, device="cuda")
    q = _mods30()[0]
    for qq in (q + 1, 3, (1 << 30) + 1):  # even, too small, too large
        with pytest.raises(ks.KsError) as e:
            ks.ks_arith_probe(qq, a, a, a)
        assert e.value.status == ks.KS_ERR_INVALID_ARG
    a64 = torch.zeros(4, dtype=torch.int64, device="cuda")
    q64 = _mods64()[0]
    for qq, w in ((q64 + 1, 0), (3, 0), (q64, q64)):  # even, too small, w >= q
        with pytest.raises(ks.KsError) as e:
            ks.ks64_arith_probe(qq, w, a64, a64)
        assert e.value.status == ks.KS_ERR_INVALID_ARG
