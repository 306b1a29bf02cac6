"""ctypes wrappers of the plain-C oracle plus exact big-integer checks.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The big-integer
functions use Python integers, which are exact at any size, so the checks
below hold without any rounding argument.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

_lib = None
_U32P = ctypes.POINTER(ctypes.c_uint32)
_I8P = ctypes.POINTER(ctypes.c_int8)


class _Params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("num_q", ctypes.c_uint32),
                ("dnum", ctypes.c_uint32), ("num_p", ctypes.c_uint32)]


def lib():
    """Load (building once if absent) the oracle shared library."""
    global _lib
    if _lib is None:
        srcs = [os.path.join(os.path.dirname(LIB), f) for f in ("ks_oracle.c", "ks_oracle64.c", "ks_oracle.h")]
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(f) for f in srcs):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER(_Params)
        sig = {
            "oracle_is_prime": (ctypes.c_int, [ctypes.c_uint64]),
            "oracle_gen_primes": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, _U32P]),
            "oracle_moduli": (ctypes.c_int, [P, _U32P]),
            "oracle_min_psi": (ctypes.c_uint32, [ctypes.c_uint32, ctypes.c_uint32]),
            "oracle_powmod": (ctypes.c_uint32, [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32]),
            "oracle_invmod": (ctypes.c_uint32, [ctypes.c_uint32, ctypes.c_uint32]),
            "oracle_bitrev": (ctypes.c_uint32, [ctypes.c_uint32, ctypes.c_uint32]),
            "oracle_ntt_direct": (None, [_U32P, _U32P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]),
            "oracle_ntt": (None, [_U32P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]),
            "oracle_intt": (None, [_U32P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]),
            "oracle_negacyclic_mul": (None, [_U32P, _U32P, _U32P, ctypes.c_uint32, ctypes.c_uint32]),
            "oracle_bconv": (None, [_U32P, _U32P, ctypes.c_uint32, _U32P, _U32P, ctypes.c_uint32,
                                    ctypes.c_uint32]),
            "oracle_keyswitch": (ctypes.c_int, [P, _U32P, ctypes.c_uint32, _U32P, _U32P, _U32P]),
            "oracle_keyswitch_oc": (ctypes.c_int, [P, _U32P, ctypes.c_uint32, _U32P, _U32P, _U32P]),
            "oracle_keygen": (ctypes.c_int, [P, _U32P, ctypes.c_uint64, _I8P, _I8P, _U32P]),
            "oracle_keygen_seeded": (ctypes.c_int, [P, _U32P, ctypes.c_uint64, ctypes.c_uint64, _I8P, _I8P, _U32P]),
            "oracle_splitmix_at": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_uint64]),
            "oracle_seeded_a": (ctypes.c_int, [P, _U32P, ctypes.c_uint64, _U32P]),
            "oracle_automorphism_coeff": (ctypes.c_int, [_U32P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                                         _U32P]),
            "oracle_automorphism_eval": (ctypes.c_int, [_U32P, ctypes.c_uint32, ctypes.c_uint32, _U32P]),
            "oracle_keygen_rotation": (ctypes.c_int, [P, _U32P, ctypes.c_uint64, ctypes.c_uint32, _I8P, _I8P, _U32P]),
            "oracle_keygen_relin": (ctypes.c_int, [P, _U32P, ctypes.c_uint64, _I8P, _U32P]),
            "oracle_rotate_hoisted": (ctypes.c_int, [P, _U32P, ctypes.c_uint32, _U32P, _U32P, ctypes.c_uint32, _U32P,
                                                     _U32P, _U32P]),
            "oracle_rotate": (ctypes.c_int, [P, _U32P, ctypes.c_uint32, _U32P, _U32P, ctypes.c_uint32, _U32P, _U32P]),
            "oracle_rotate_sum_hoisted": (ctypes.c_int, [P, _U32P, ctypes.c_uint32, _U32P, _U32P, ctypes.c_uint32,
                                                         _U32P, _U32P, _U32P, _U32P]),
            "oracle_mult_relin": (ctypes.c_int, [P, _U32P, ctypes.c_uint32, _U32P, _U32P, _U32P, _U32P, _U32P, _U32P]),
            "oracle_set_fault": (None, [ctypes.c_int]),
            "oracle_evk_words": (ctypes.c_uint64, [ctypes.c_uint32] * 4),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(_U32P)


class Params:
    """CKKS key-switching parameters (Table I): N = 2^log_n, num_q = L+1,
    dnum digits, num_p = K special moduli."""

    def __init__(self, log_n, num_q, dnum, num_p=0):
        self.log_n, self.num_q, self.dnum = int(log_n), int(num_q), int(dnum)
        self.alpha = -(-self.num_q // self.dnum)
        self.num_p = int(num_p) if num_p else self.alpha
        self.n = 1 << self.log_n

    def c(self):
        return _Params(self.log_n, self.num_q, self.dnum, self.num_p)

    def digits(self, level):
        """Digit ranges [lo, hi) of the towers q_0..q_level (Sec. III-A)."""
        out, lo = [], 0
        while lo <= level:
            out.append((lo, min(lo + self.alpha, level + 1)))
            lo += self.alpha
        return out

    def __repr__(self):
        return (f"Params(log_n={self.log_n}, num_q={self.num_q}, dnum={self.dnum}, "
                f"alpha={self.alpha}, num_p={self.num_p})")


# ---------------------------------------------------------------- number theory
def is_prime(n):
    return bool(lib().oracle_is_prime(int(n)))


def gen_primes(log_n, count):
    out = np.zeros(count, np.uint32)
    if lib().oracle_gen_primes(log_n, count, out.ctypes.data_as(_U32P)) != 0:
        raise ValueError("not enough primes")
    return out


def moduli(p):
    out = np.zeros(p.num_q + p.num_p, np.uint32)
    if lib().oracle_moduli(ctypes.byref(p.c()), out.ctypes.data_as(_U32P)) != 0:
        raise ValueError("not enough primes")
    return out


def min_psi(q, log_n):
    return int(lib().oracle_min_psi(int(q), int(log_n)))


def bitrev(x, bits):
    return int(lib().oracle_bitrev(int(x), int(bits)))


# ---------------------------------------------------------------- NTT
def ntt(a, q, psi=None):
    a = np.array(a, dtype=np.uint32, copy=True)
    log_n = int(a.shape[-1]).bit_length() - 1
    psi = min_psi(q, log_n) if psi is None else psi
    lib().oracle_ntt(a.ctypes.data_as(_U32P), log_n, int(q), int(psi))
    return a


def intt(a, q, psi=None):
    a = np.array(a, dtype=np.uint32, copy=True)
    log_n = int(a.shape[-1]).bit_length() - 1
    psi = min_psi(q, log_n) if psi is None else psi
    lib().oracle_intt(a.ctypes.data_as(_U32P), log_n, int(q), int(psi))
    return a


def ntt_direct(a, q, psi=None):
    a, ap = _u32(a)
    log_n = int(a.shape[-1]).bit_length() - 1
    psi = min_psi(q, log_n) if psi is None else psi
    out = np.zeros_like(a)
    lib().oracle_ntt_direct(ap, out.ctypes.data_as(_U32P), log_n, int(q), int(psi))
    return out


def negacyclic_mul(a, b, q):
    a, ap = _u32(a)
    b, bp = _u32(b)
    out = np.zeros_like(a)
    lib().oracle_negacyclic_mul(ap, bp, out.ctypes.data_as(_U32P), int(a.shape[-1]).bit_length() - 1, int(q))
    return out


def bconv(x, src, dst):
    """Fast basis conversion of x [len(src)][N] to [len(dst)][N]."""
    x, xp = _u32(x)
    src, sp = _u32(src)
    dst, dp = _u32(dst)
    y = np.zeros((len(dst), x.shape[-1]), np.uint32)
    lib().oracle_bconv(xp, sp, len(src), y.ctypes.data_as(_U32P), dp, len(dst), x.shape[-1])
    return y


# ---------------------------------------------------------------- key switching
def keyswitch(p, mods, level, evk, d, order="mp"):
    """Hybrid key switching of d [level+1][N] with evk [dnum][2][L+1+K][N]."""
    mods, mp_ = _u32(mods)
    evk, ep = _u32(evk)
    d, dp = _u32(d)
    assert d.shape == (level + 1, p.n), d.shape
    assert evk.size == p.dnum * 2 * (p.num_q + p.num_p) * p.n
    out = np.zeros((2, level + 1, p.n), np.uint32)
    f = lib().oracle_keyswitch if order == "mp" else lib().oracle_keyswitch_oc
    if f(ctypes.byref(p.c()), mp_, int(level), ep, dp, out.ctypes.data_as(_U32P)) != 0:
        raise ValueError("oracle_keyswitch rejected its arguments")
    return out


def keygen(p, mods, seed):
    """Returns (s, s2, evk, h): ternary secrets as int8 [N] and the evaluation
    key [dnum][2][L+1+K][N] switching from s2 to s."""
    mods, mp_ = _u32(mods)
    s = np.zeros(p.n, np.int8)
    s2 = np.zeros(p.n, np.int8)
    evk = np.zeros((p.dnum, 2, p.num_q + p.num_p, p.n), np.uint32)
    h = lib().oracle_keygen(ctypes.byref(p.c()), mp_, int(seed), s.ctypes.data_as(_I8P),
                            s2.ctypes.data_as(_I8P), evk.ctypes.data_as(_U32P))
    if h < 0:
        raise ValueError("oracle_keygen rejected its arguments")
    return s, s2, evk, h


def splitmix_at(seed, t):
    """Output t of the counter-based SplitMix64 generator for `seed`."""
    return int(lib().oracle_splitmix_at(int(seed) & (2**64 - 1), int(t)))


def seeded_a(p, mods, a_seed):
    """The a halves of a key compressed to `a_seed` (Sec. IV-D), returned as a
    full-layout evk [dnum][2][L+1+K][N] whose b halves are zero."""
    mods, mp_ = _u32(mods)
    evk = np.zeros((p.dnum, 2, p.num_q + p.num_p, p.n), np.uint32)
    if lib().oracle_seeded_a(ctypes.byref(p.c()), mp_, int(a_seed) & (2**64 - 1), evk.ctypes.data_as(_U32P)) != 0:
        raise ValueError("oracle_seeded_a rejected its arguments")
    return evk


def keygen_seeded(p, mods, seed, a_seed):
    """keygen whose a halves are regenerated from `a_seed`: the b halves
    evk[:, 0] plus a_seed are the whole key."""
    mods, mp_ = _u32(mods)
    s = np.zeros(p.n, np.int8)
    s2 = np.zeros(p.n, np.int8)
    evk = np.zeros((p.dnum, 2, p.num_q + p.num_p, p.n), np.uint32)
    h = lib().oracle_keygen_seeded(ctypes.byref(p.c()), mp_, int(seed), int(a_seed) & (2**64 - 1),
                                   s.ctypes.data_as(_I8P), s2.ctypes.data_as(_I8P), evk.ctypes.data_as(_U32P))
    if h < 0:
        raise ValueError("oracle_keygen_seeded rejected its arguments")
    return s, s2, evk, h


def _arr(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(_U32P)


def automorphism_coeff(a, log_n, galois, q):
    """a(X^k) of a coefficient-domain limb."""
    a, ap = _arr(a)
    out = np.zeros(1 << log_n, np.uint32)
    if lib().oracle_automorphism_coeff(ap, log_n, int(galois), int(q), out.ctypes.data_as(_U32P)) != 0:
        raise ValueError("bad Galois element")
    return out


def automorphism_eval(a, log_n, galois):
    """a(X^k) of an evaluation-domain limb (a permutation of the slots);
    a may be [..., N], each limb permuted."""
    a = np.ascontiguousarray(a, dtype=np.uint32)
    flat = a.reshape(-1, 1 << log_n)
    out = np.zeros_like(flat)
    for i in range(flat.shape[0]):
        if lib().oracle_automorphism_eval(flat[i].ctypes.data_as(_U32P), log_n, int(galois),
                                          out[i].ctypes.data_as(_U32P)) != 0:
            raise ValueError("bad Galois element")
    return out.reshape(a.shape)


def galois_rotation(log_n, r):
    """Galois element of a rotation by r slots: 5^r mod 2N (r may be negative)."""
    two_n = 2 << log_n
    return pow(5, r % (two_n // 4), two_n)


def keygen_rotation(p, mods, seed, galois):
    """(s, s_k, evk, h): evk switches from s_k = s(X^k) to s."""
    mods, mp_ = _u32(mods)
    s = np.zeros(p.n, np.int8)
    s2 = np.zeros(p.n, np.int8)
    evk = np.zeros((p.dnum, 2, p.num_q + p.num_p, p.n), np.uint32)
    h = lib().oracle_keygen_rotation(ctypes.byref(p.c()), mp_, int(seed), int(galois), s.ctypes.data_as(_I8P),
                                     s2.ctypes.data_as(_I8P), evk.ctypes.data_as(_U32P))
    if h < 0:
        raise ValueError("oracle_keygen_rotation rejected its arguments")
    return s, s2, evk, h


def keygen_relin(p, mods, seed):
    """(s, evk, h): evk switches from s^2 to s."""
    mods, mp_ = _u32(mods)
    s = np.zeros(p.n, np.int8)
    evk = np.zeros((p.dnum, 2, p.num_q + p.num_p, p.n), np.uint32)
    h = lib().oracle_keygen_relin(ctypes.byref(p.c()), mp_, int(seed), s.ctypes.data_as(_I8P),
                                  evk.ctypes.data_as(_U32P))
    if h < 0:
        raise ValueError("oracle_keygen_relin rejected its arguments")
    return s, evk, h


def rotate_hoisted(p, mods, level, c0, c1, galois, evks):
    """Rotations of (c0, c1) by each Galois element, one shared ModUp;
    returns [count][2][level+1][N]."""
    mods, mp_ = _u32(mods)
    c0, c0p = _arr(c0)
    c1, c1p = _arr(c1)
    g, gp_ = _arr(list(galois))
    ev, evp = _arr(np.stack(list(evks)))
    outs = np.zeros((len(g), 2, level + 1, p.n), np.uint32)
    if lib().oracle_rotate_hoisted(ctypes.byref(p.c()), mp_, int(level), c0p, c1p, len(g), gp_, evp,
                                   outs.ctypes.data_as(_U32P)) != 0:
        raise ValueError("oracle_rotate_hoisted rejected its arguments")
    return outs


def rotate_sum_hoisted(p, mods, level, c0, c1, galois, evks, diags=None):
    """sum_r p_r sigma_r((c0, c1)) with one ModUp and one ModDown (double
    hoisting); diags None or [count][L+1+K][N]; returns [2][level+1][N]."""
    mods, mp_ = _u32(mods)
    c0, c0p = _arr(c0)
    c1, c1p = _arr(c1)
    g, gp_ = _arr(list(galois))
    ev, evp = _arr(np.stack(list(evks)))
    dg = None
    if diags is not None:
        dg, dgp = _arr(np.stack(list(diags)))
    out = np.zeros((2, level + 1, p.n), np.uint32)
    if lib().oracle_rotate_sum_hoisted(ctypes.byref(p.c()), mp_, int(level), c0p, c1p, len(g), gp_, evp,
                                       dgp if dg is not None else None, out.ctypes.data_as(_U32P)) != 0:
        raise ValueError("oracle_rotate_sum_hoisted rejected its arguments")
    return out


def rotate(p, mods, level, c0, c1, galois, evk):
    mods, mp_ = _u32(mods)
    c0, c0p = _arr(c0)
    c1, c1p = _arr(c1)
    ev, evp = _arr(evk)
    out = np.zeros((2, level + 1, p.n), np.uint32)
    if lib().oracle_rotate(ctypes.byref(p.c()), mp_, int(level), c0p, c1p, int(galois), evp,
                           out.ctypes.data_as(_U32P)) != 0:
        raise ValueError("oracle_rotate rejected its arguments")
    return out


def mult_relin(p, mods, level, a0, a1, b0, b1, evk):
    mods, mp_ = _u32(mods)
    bufs = [_arr(x) for x in (a0, a1, b0, b1)]
    ev, evp = _arr(evk)
    out = np.zeros((2, level + 1, p.n), np.uint32)
    if lib().oracle_mult_relin(ctypes.byref(p.c()), mp_, int(level), *[b[1] for b in bufs], evp,
                               out.ctypes.data_as(_U32P)) != 0:
        raise ValueError("oracle_mult_relin rejected its arguments")
    return out


def set_fault(k):
    lib().oracle_set_fault(int(k))


def evk_words(log_n, num_q, num_p, dnum):
    return int(lib().oracle_evk_words(log_n, num_q, num_p, dnum))


# ---------------------------------------------------------------- big integers
def prod(xs):
    r = 1
    for x in xs:
        r *= int(x)
    return r


def crt(residues, mods):
    """Exact CRT: residues [len(mods)][N] -> list of N integers in [0, prod)."""
    M = prod(mods)
    coef = []
    for m in mods:
        m = int(m)
        Mi = M // m
        coef.append(Mi * pow(Mi % m, -1, m))
    res = np.asarray(residues, dtype=np.uint64)
    n = res.shape[-1]
    out = [0] * n
    for i in range(len(mods)):
        ci = coef[i]
        row = res[i].tolist()
        for z in range(n):
            out[z] += row[z] * ci
    return [v % M for v in out]


def centre(v, M):
    return v - M if v > M // 2 else v


def signed_residues(s, mods, n):
    return np.array([[int(v) % int(m) for v in s] for m in mods], dtype=np.uint32).reshape(len(mods), n)


def noise_bound(p, mods, level, h, b_e=19):
    """B = floor(sum_j N |S_j| Q_j B_e / P) + (1+h)(1+K)  (decryption bound of
    the key-switched output; the derivation is in the oracle tests)."""
    P = prod(mods[p.num_q:p.num_q + p.num_p])
    tot = 0
    for lo, hi in p.digits(level):
        tot += p.n * (hi - lo) * prod(mods[lo:hi]) * b_e
    return tot // P + (1 + h) * (1 + p.num_p)


def decrypt_residual(p, mods, level, d, out, s, s2):
    """r = c0 + c1*s - d*s2 mod Q_level, as centred integers (list of N)."""
    l1 = level + 1
    r = np.zeros((l1, p.n), np.uint32)
    for i in range(l1):
        q = int(mods[i])
        psi = min_psi(q, p.log_n)
        sh = ntt(signed_residues(s, [q], p.n)[0], q, psi).astype(np.uint64)
        s2h = ntt(signed_residues(s2, [q], p.n)[0], q, psi).astype(np.uint64)
        v = (out[0, i].astype(np.uint64) + out[1, i].astype(np.uint64) * sh % q) % q
        v = (v + q - d[i].astype(np.uint64) * s2h % q) % q
        r[i] = intt(v.astype(np.uint32), q, psi)
    Q = prod(mods[:l1])
    return [centre(v, Q) for v in crt(r, mods[:l1])]
