"""Seeded synthetic inputs shared by the tests, the bench and the oracle runs.

This module draws uniform random residues and picks workload shapes; it holds
none of the key-switching arithmetic.  Key switching is data-oblivious (the
same instructions and addresses for every input value), so timing inputs are
uniform residues in [0, m) for every limb of the input polynomial and of the
evaluation key; parity inputs use the same generator.
"""
import numpy as np


def seed_for(config, i=0):
    """Seed of input i of workload `config`."""
    return 0x5EED0000 + 1000 * int(config) + int(i)


def uniform_limbs(moduli, n, seed):
    """[len(moduli)][n] uint32, limb r uniform in [0, moduli[r])."""
    rng = np.random.default_rng(seed)
    out = np.empty((len(moduli), n), np.uint32)
    for r, m in enumerate(moduli):
        out[r] = rng.integers(0, int(m), n, dtype=np.uint64).astype(np.uint32)
    return out


def uniform_evk(moduli, dnum, n, seed):
    """[dnum][2][len(moduli)][n] uint32 uniform residues (timing-only key)."""
    rng = np.random.default_rng(seed)
    out = np.empty((dnum, 2, len(moduli), n), np.uint32)
    for r, m in enumerate(moduli):
        out[:, :, r, :] = rng.integers(0, int(m), (dnum, 2, n), dtype=np.uint64).astype(np.uint32)
    return out


def batch_levels(count, towers_lo, towers_hi, seed):
    """Levels l with l+1 uniform in [towers_lo, towers_hi]."""
    rng = np.random.default_rng(seed)
    return [int(t) - 1 for t in rng.integers(towers_lo, towers_hi + 1, count)]


def uniform_limbs_device(moduli, n, seed, torch, lead=()):
    """[*lead][len(moduli)][n] int32 tensor on the current GPU: limb r uniform
    in [0, moduli[r]) (the same uint32 bits), drawn with torch's seeded device
    generator as the residue of a uniform 62-bit integer (bias below 2^-32).
    For large timing inputs (resident serving keys and request buffers)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(int(seed))
    m = torch.tensor([int(x) for x in moduli], dtype=torch.int64, device="cuda").view(*([1] * len(lead)), -1, 1)
    x = torch.randint(0, 1 << 62, (*lead, len(moduli), n), dtype=torch.int64, device="cuda", generator=g)
    return (x % m).to(torch.int32)


def uniform_words64_device(moduli, n, seed, torch, lead=()):
    """[*lead][len(moduli)][n] int64 tensor on the current GPU: limb r in
    [0, moduli[r]) (moduli below 2^62; the same uint64 bits), the residue of
    a uniform 63-bit integer.  Close to uniform, not exactly (for m near 2^60
    the low residues are up to m / 2^63 more frequent): timing inputs for
    64-bit-word plans, whose key switch is data-oblivious."""
    g = torch.Generator(device="cuda")
    g.manual_seed(int(seed))
    m = torch.tensor([int(x) for x in moduli], dtype=torch.int64, device="cuda").view(*([1] * len(lead)), -1, 1)
    x = torch.randint(0, (1 << 63) - 1, (*lead, len(moduli), n), dtype=torch.int64, device="cuda", generator=g)
    return x % m
