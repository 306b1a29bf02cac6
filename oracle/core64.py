"""ctypes wrappers of the 64-bit-word oracle (ks_oracle64.c).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Residues are uint64
arrays; the big-integer helpers of core.py (crt, noise_bound, centre) work
on Python integers and serve both word sizes.
"""
import ctypes

import numpy as np

from . import core
from .core import Params, centre, crt, prod

_U64P = ctypes.POINTER(ctypes.c_uint64)
_I8P = ctypes.POINTER(ctypes.c_int8)
_ready = False


def lib():
    global _ready
    L = core.lib()
    if not _ready:
        P = ctypes.POINTER(core._Params)
        sig = {
            "oracle64_is_prime": (ctypes.c_int, [ctypes.c_uint64]),
            "oracle64_gen_primes": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, _U64P]),
            "oracle64_moduli": (ctypes.c_int, [P, _U64P]),
            "oracle64_min_psi": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_uint32]),
            "oracle64_powmod": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]),
            "oracle64_ntt_direct": (None, [_U64P, _U64P, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64]),
            "oracle64_ntt": (None, [_U64P, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64]),
            "oracle64_intt": (None, [_U64P, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64]),
            "oracle64_negacyclic_mul": (None, [_U64P, _U64P, _U64P, ctypes.c_uint32, ctypes.c_uint64]),
            "oracle64_bconv": (None, [_U64P, _U64P, ctypes.c_uint32, _U64P, _U64P, ctypes.c_uint32,
                                      ctypes.c_uint32]),
            "oracle64_keyswitch": (ctypes.c_int, [P, _U64P, ctypes.c_uint32, _U64P, _U64P, _U64P]),
            "oracle64_keygen": (ctypes.c_int, [P, _U64P, ctypes.c_uint64, _I8P, _I8P, _U64P]),
            "oracle64_seeded_a": (ctypes.c_int, [P, _U64P, ctypes.c_uint64, _U64P]),
            "oracle64_keygen_seeded": (ctypes.c_int, [P, _U64P, ctypes.c_uint64, ctypes.c_uint64, _I8P, _I8P,
                                                      _U64P]),
            "oracle64_set_fault": (None, [ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _ready = True
    return L


def _u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(_U64P)


def is_prime(n):
    return bool(lib().oracle64_is_prime(int(n)))


def gen_primes(log_n, count):
    out = np.zeros(count, np.uint64)
    if lib().oracle64_gen_primes(log_n, count, out.ctypes.data_as(_U64P)) != 0:
        raise ValueError("not enough primes")
    return out


def moduli(p):
    out = np.zeros(p.num_q + p.num_p, np.uint64)
    if lib().oracle64_moduli(ctypes.byref(p.c()), out.ctypes.data_as(_U64P)) != 0:
        raise ValueError("not enough primes")
    return out


def min_psi(q, log_n):
    return int(lib().oracle64_min_psi(int(q), log_n))


def _log(n):
    log_n = int(n).bit_length() - 1
    assert 1 << log_n == n
    return log_n


def ntt(a, q, psi=None):
    a, pa = _u64(np.array(a, dtype=np.uint64, copy=True))
    log_n = _log(a.size)
    lib().oracle64_ntt(pa, log_n, int(q), int(psi if psi is not None else min_psi(q, log_n)))
    return a


def intt(a, q, psi=None):
    a, pa = _u64(np.array(a, dtype=np.uint64, copy=True))
    log_n = _log(a.size)
    lib().oracle64_intt(pa, log_n, int(q), int(psi if psi is not None else min_psi(q, log_n)))
    return a


def ntt_direct(a, q, psi=None):
    a, pa = _u64(a)
    log_n = _log(a.size)
    out = np.zeros_like(a)
    lib().oracle64_ntt_direct(pa, out.ctypes.data_as(_U64P), log_n, int(q),
                              int(psi if psi is not None else min_psi(q, log_n)))
    return out


def negacyclic_mul(a, b, q):
    a, pa = _u64(a)
    b, pb = _u64(b)
    c = np.zeros_like(a)
    lib().oracle64_negacyclic_mul(pa, pb, c.ctypes.data_as(_U64P), _log(a.size), int(q))
    return c


def bconv(x, src, dst):
    """x [len(src)][n] -> y [len(dst)][n] (fast basis conversion)."""
    x, px = _u64(x)
    s, ps = _u64(np.array(src, dtype=np.uint64))
    d, pd = _u64(np.array(dst, dtype=np.uint64))
    n = x.shape[-1]
    y = np.zeros((len(d), n), np.uint64)
    lib().oracle64_bconv(px, ps, len(s), y.ctypes.data_as(_U64P), pd, len(d), n)
    return y


def keyswitch(p, mods, level, evk, d):
    mods_a, pm = _u64(np.array(mods, dtype=np.uint64))
    evk, pe = _u64(evk)
    d, pd = _u64(d)
    out = np.zeros((2, level + 1, p.n), np.uint64)
    if lib().oracle64_keyswitch(ctypes.byref(p.c()), pm, level, pe, pd, out.ctypes.data_as(_U64P)) != 0:
        raise ValueError("bad parameters")
    return out


def keygen(p, mods, seed):
    """(s, s2, evk [dnum][2][L+1+K][N] uint64, h = ||s||_1)."""
    mods_a, pm = _u64(np.array(mods, dtype=np.uint64))
    s = np.zeros(p.n, np.int8)
    s2 = np.zeros(p.n, np.int8)
    evk = np.zeros((p.dnum, 2, p.num_q + p.num_p, p.n), np.uint64)
    h = lib().oracle64_keygen(ctypes.byref(p.c()), pm, int(seed), s.ctypes.data_as(_I8P),
                              s2.ctypes.data_as(_I8P), evk.ctypes.data_as(_U64P))
    if h < 0:
        raise ValueError("bad parameters")
    return s, s2, evk, h


def seeded_a(p, mods, a_seed):
    """Key compression (Sec. IV-D): evk-shaped array whose a halves ([:, 1])
    are regenerated from a_seed (X 2^-64 mod m for the 123-bit X formed by
    the SplitMix64 outputs at counters 2t and 2t + 1 of the word's counter
    t); the b halves are zero."""
    mods_a, pm = _u64(np.array(mods, dtype=np.uint64))
    evk = np.zeros((p.dnum, 2, p.num_q + p.num_p, p.n), np.uint64)
    if lib().oracle64_seeded_a(ctypes.byref(p.c()), pm, int(a_seed), evk.ctypes.data_as(_U64P)) != 0:
        raise ValueError("bad parameters")
    return evk


def keygen_seeded(p, mods, seed, a_seed):
    """keygen with the a halves of seeded_a(a_seed): (s, s2, evk, h)."""
    mods_a, pm = _u64(np.array(mods, dtype=np.uint64))
    s = np.zeros(p.n, np.int8)
    s2 = np.zeros(p.n, np.int8)
    evk = np.zeros((p.dnum, 2, p.num_q + p.num_p, p.n), np.uint64)
    h = lib().oracle64_keygen_seeded(ctypes.byref(p.c()), pm, int(seed), int(a_seed), s.ctypes.data_as(_I8P),
                                     s2.ctypes.data_as(_I8P), evk.ctypes.data_as(_U64P))
    if h < 0:
        raise ValueError("bad parameters")
    return s, s2, evk, h


def set_fault(k):
    lib().oracle64_set_fault(int(k))


def decrypt_residual(p, mods, level, d, out, s, s2):
    """r = c0 + c1*s - d*s2 mod Q_level, as centred integers (list of N)."""
    l1 = level + 1
    r = []
    for i in range(l1):
        q = int(mods[i])
        psi = min_psi(q, p.log_n)
        sh = ntt(np.array([int(v) % q for v in s], np.uint64), q, psi)
        s2h = ntt(np.array([int(v) % q for v in s2], np.uint64), q, psi)
        v = [(int(a) + int(b) * int(x) - int(e) * int(y)) % q
             for a, b, x, e, y in zip(out[0, i], out[1, i], sh, d[i], s2h)]
        r.append(intt(np.array(v, np.uint64), q, psi))
    Q = prod(mods[:l1])
    return [centre(v, Q) for v in crt(np.array(r, dtype=np.uint64), mods[:l1])]


__all__ = ["Params", "is_prime", "gen_primes", "moduli", "min_psi", "ntt", "intt", "ntt_direct",
           "negacyclic_mul", "bconv", "keyswitch", "keygen", "set_fault", "decrypt_residual"]
