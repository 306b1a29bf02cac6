"""GPU parity of the callers of the key switch (Sec. II): the automorphism,
hoisted rotations (one ModUp of c1 shared by every rotation key) and
multiplication with relinearisation, bit for bit against the oracle.

Cases: the N=2^12 / 4-tower / dnum 2 workload with real rotation and
relinearisation keys (outputs also decrypt), the N=2^16 / 24-tower / dnum 3
workload at full size (every element), partial last digits, dnum = 1,
K != alpha, alpha = 1, level 0, both conversion tile widths, conjugation
and the identity element; rejections of bad arguments.
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


@pytest.mark.parametrize("log_n", [12, 16])
def test_automorphism_matches_oracle(ks, log_n):
    plan = ks.Plan(log_n, 3, 1, 1)
    a = synth.uniform_limbs(plan.moduli[:3], plan.n, synth.seed_for(20, log_n))
    for k in (5, core.galois_rotation(log_n, -7), (2 << log_n) - 1, 1):
        say(f"[auto] log_n={log_n} k={k}")
        got = host(plan.automorphism(dev(a), k))
        assert np.array_equal(got, core.automorphism_eval(a, log_n, k)), k
    plan.close()


def _sub(a, b, mods):
    return np.stack([((a[i].astype(np.int64) - b[i]) % int(mods[i])) for i in range(len(a))]).astype(np.uint32)


@pytest.mark.parametrize("tt", [1, 2])
def test_hoisted_plain_workload_decrypts(ks, tt):
    p = oracle.Params(12, 4, 2, 2)
    mods = oracle.moduli(p)
    level = 3
    c0 = synth.uniform_limbs(mods[:4], p.n, synth.seed_for(21, 0))
    c1 = synth.uniform_limbs(mods[:4], p.n, synth.seed_for(21, 1))
    gal = [core.galois_rotation(12, r) for r in (1, 5, -3)] + [(2 << 12) - 1, 1]
    keys = [core.keygen_rotation(p, mods, 60 + i, k) for i, k in enumerate(gal)]
    want = core.rotate_hoisted(p, mods, level, c0, c1, gal, [k[2] for k in keys])
    plan = ks.Plan(12, 4, 2, 2)
    plan.configure("oc", tile_towers=tt)
    say(f"[rot plain] tt={tt}")
    outs = plan.rotate_hoisted(level, dev(c0), dev(c1), [(dev(k[2]), g) for k, g in zip(keys, gal)])
    torch.cuda.synchronize()
    for i, (o, w) in enumerate(zip(outs, want)):
        assert np.array_equal(host(o), w), (i, gal[i], np.argwhere(host(o) != w)[:5])
    s, sk, _, h = keys[0]
    got = host(outs[0])
    sc0 = core.automorphism_eval(c0, 12, gal[0])
    sc1 = core.automorphism_eval(c1, 12, gal[0])
    r = oracle.decrypt_residual(p, mods, level, sc1, np.stack([_sub(got[0], sc0, mods), got[1]]), s, sk)
    assert max(abs(v) for v in r) <= oracle.noise_bound(p, mods, level, h)
    # identity element: the key switch of c1 plus (c0, 0), from the plain entry point
    ks1 = host(plan.keyswitch(dev(keys[-1][2]), level, dev(c1)))
    ident = host(outs[-1])
    assert np.array_equal(ident[1], ks1[1])
    assert np.array_equal(ident[0], np.stack([(ks1[0][i].astype(np.uint64) + c0[i]) % int(mods[i])
                                              for i in range(4)]).astype(np.uint32))
    plan.close()


def test_hoisted_full_size_n16_l24_dnum3(ks):
    p = oracle.Params(16, 24, 3, 8)
    mods = oracle.moduli(p)
    c0 = synth.uniform_limbs(mods[:24], p.n, synth.seed_for(22, 0))
    c1 = synth.uniform_limbs(mods[:24], p.n, synth.seed_for(22, 1))
    gal = [core.galois_rotation(16, r) for r in (1, 2, -1)]
    keys = [synth.uniform_evk(mods, 3, p.n, synth.seed_for(22, 10 + i)) for i in range(3)]
    want = core.rotate_hoisted(p, mods, 23, c0, c1, gal, keys)
    plan = ks.Plan(16, 24, 3, 8)
    for tt in (1, 2):
        say(f"[rot n16] tt={tt}")
        plan.configure("oc", tile_towers=tt)
        outs = plan.rotate_hoisted(23, dev(c0), dev(c1), [(dev(k), g) for k, g in zip(keys, gal)])
        torch.cuda.synchronize()
        for i, (o, w) in enumerate(zip(outs, want)):
            bad = np.argwhere(host(o) != w)
            assert bad.size == 0, (tt, i, bad[:5], len(bad))
    plan.close()


@pytest.mark.parametrize("shape", [(12, 4, 2, 2, 3), (16, 24, 3, 8, 23), (13, 9, 3, 2, 4)])
def test_hoisted_compressed_keys(ks, shape):
    """Rotation keys stored as b halves plus a seed give the bits of the
    expanded keys."""
    log_n, num_q, dnum, num_p, level = shape
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = oracle.moduli(p)
    c0 = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(26, 0))
    c1 = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(26, 1))
    gal = [core.galois_rotation(log_n, r) for r in (1, 4)] + [(2 << log_n) - 1]
    seeds = [synth.seed_for(26, 50 + i) for i in range(3)]
    keys = []
    for i, a_seed in enumerate(seeds):
        full = synth.uniform_evk(mods, dnum, p.n, synth.seed_for(26, 10 + i))
        full[:, 1] = core.seeded_a(p, mods, a_seed)[:, 1]
        keys.append(full)
    want = core.rotate_hoisted(p, mods, level, c0, c1, gal, keys)
    plan = ks.Plan(log_n, num_q, dnum, num_p)
    print(f"[rot seeded] {shape}", flush=True)
    outs = plan.rotate_hoisted_seeded(level, dev(c0), dev(c1), [(dev(np.ascontiguousarray(k[:, 0])), a, g)
                                                                 for k, a, g in zip(keys, seeds, gal)])
    torch.cuda.synchronize()
    for i, (o, w) in enumerate(zip(outs, want)):
        bad = np.argwhere(host(o) != w)
        assert bad.size == 0, (i, bad[:5], len(bad))
    plan.close()


def _diag(mods, n, seed):
    """A plaintext diagonal in every key row: uniform residues (any value is
    a valid operand of the exact product)."""
    return synth.uniform_limbs(mods, n, seed)


@pytest.mark.parametrize("shape,with_diag,nterm", [((12, 4, 2, 2, 3), False, 4), ((12, 4, 2, 2, 2), True, 4),
                                                   ((16, 24, 3, 8, 23), True, 4), ((13, 9, 3, 2, 5), True, 4),
                                                   ((12, 7, 7, 1, 6), False, 4), ((13, 9, 3, 3, 8), True, 3),
                                                   ((13, 9, 3, 3, 8), False, 1), ((12, 6, 3, 2, 1), True, 3),
                                                   ((12, 8, 4, 2, 7), True, 3), ((12, 10, 5, 2, 9), False, 4)])
def test_double_hoisted_sum(ks, shape, with_diag, nterm):
    """Every build of the OC summing row stage: terms with at most 2 foreign
    digits run two per round (odd term counts leave the last one alone),
    terms with 3 or 4 one per round, terms with more over several rounds."""
    log_n, num_q, dnum, num_p, level = shape
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = oracle.moduli(p)
    c0 = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(27, 0))
    c1 = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(27, 1))
    gal = ([core.galois_rotation(log_n, r) for r in (0, 1, 3)] + [(2 << log_n) - 1])[:nterm]
    keys = [synth.uniform_evk(mods, dnum, p.n, synth.seed_for(27, 10 + i)) for i in range(len(gal))]
    diags = [_diag(mods, p.n, synth.seed_for(27, 30 + i)) for i in range(len(gal))] if with_diag else None
    want = core.rotate_sum_hoisted(p, mods, level, c0, c1, gal, keys, diags)
    plan = ks.Plan(log_n, num_q, dnum, num_p)
    print(f"[rot sum] {shape} diag={with_diag} terms={nterm}", flush=True)
    terms = [(dev(k), g, dev(diags[i]) if with_diag else None) for i, (k, g) in enumerate(zip(keys, gal))]
    for sched in ("oc", "mp"):  # the sum runs the same stages under any schedule
        plan.configure(sched)
        got = host(plan.rotate_sum_hoisted(level, dev(c0), dev(c1), terms))
        bad = np.argwhere(got != want)
        assert bad.size == 0, (sched, bad[:5], len(bad))
    plan.close()


def test_double_hoisted_sum_decrypts(ks):
    p = oracle.Params(12, 4, 2, 2)
    mods = oracle.moduli(p)
    level = 3
    c0 = synth.uniform_limbs(mods[:4], p.n, synth.seed_for(28, 0))
    c1 = synth.uniform_limbs(mods[:4], p.n, synth.seed_for(28, 1))
    gal = [core.galois_rotation(12, r) for r in (1, 2, 7)]
    keys = [core.keygen_rotation(p, mods, 71, k) for k in gal]  # one seed: one secret
    plan = ks.Plan(12, 4, 2, 2)
    got = host(plan.rotate_sum_hoisted(level, dev(c0), dev(c1), [(dev(k[2]), g, None) for k, g in zip(keys, gal)]))
    torch.cuda.synchronize()
    assert np.array_equal(got, core.rotate_sum_hoisted(p, mods, level, c0, c1, gal, [k[2] for k in keys]))
    # r = c0' + c1' s - sum_r sigma_r(c0 + c1 s), assembled from the oracle's
    # residual helper (linear modulo Q before centring), is within the summed
    # key-switch error plus one ModDown rounding
    s, h = keys[0][0], keys[0][3]
    Q = oracle.prod(mods[:4])
    sc0 = sum(core.automorphism_eval(c0, 12, k).astype(np.int64) for k in gal)
    out0 = np.stack([(got[0][i].astype(np.int64) - sc0[i]) % int(mods[i]) for i in range(4)]).astype(np.uint32)
    zero = np.zeros((4, p.n), np.uint32)
    r = oracle.decrypt_residual(p, mods, level, zero, np.stack([out0, got[1]]), s, s)  # c0'' + c1' s
    for k, (_, sk, _, _) in zip(gal, keys):  # - sigma_r(c1) sigma_r(s)
        sc1 = core.automorphism_eval(c1, 12, k)
        r = [a + b for a, b in zip(r, oracle.decrypt_residual(p, mods, level, sc1, np.stack([zero, zero]), s, sk))]
    worst = max(abs(core.centre(v % Q, Q)) for v in r)
    E = oracle.noise_bound(p, mods, level, h) - (1 + h) * (1 + p.num_p)
    assert worst <= len(gal) * (E + 1) + (1 + h) * (1 + p.num_p)
    plan.close()


@pytest.mark.parametrize("tt,mode", [(1, 1), (2, 3)])
def test_rotation_batch_mixed_levels(ks, tt, mode):
    """Nine ciphertexts at mixed levels, each rotated by its own element with
    its own key, in one batch: each equals the oracle's rotation of that
    ciphertext alone (a hoisted group of one)."""
    p = oracle.Params(13, 8, 3, 0)
    mods = oracle.moduli(p)
    plan = ks.Plan(13, 8, 3)
    plan.configure("oc", tile_towers=tt, batch_mode=mode)
    keys = [synth.uniform_evk(mods, 3, p.n, synth.seed_for(29, k)) for k in range(3)]
    keys_d = [dev(k) for k in keys]
    levels = synth.batch_levels(9, 1, 8, synth.seed_for(29, 50))
    jobs, wants = [], []
    for i, level in enumerate(levels):
        c0 = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(29, 100 + i))
        c1 = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(29, 200 + i))
        k = core.galois_rotation(13, i + 1) if i % 4 else (2 << 13) - 1
        wants.append(core.rotate_hoisted(p, mods, level, c0, c1, [k], [keys[i % 3]])[0])
        jobs.append((keys_d[i % 3], k, level, dev(c0), dev(c1)))
    print(f"[rot batch] tt={tt} mode={mode} levels={levels}", flush=True)
    outs = plan.rotate_batch(jobs)
    torch.cuda.synchronize()
    for i, (o, w) in enumerate(zip(outs, wants)):
        assert np.array_equal(host(o), w), (i, levels[i])
    plan.close()


SHAPES = [
    (12, 5, 2, 0, [4, 0]),     # partial last digit; level 0
    (12, 4, 1, 0, [3]),        # dnum = 1
    (13, 9, 3, 2, [8, 4]),     # K != alpha
    (12, 7, 7, 1, [6, 2]),     # alpha = 1
]


@pytest.mark.parametrize("log_n,num_q,dnum,num_p,levels", SHAPES)
def test_hoisted_shapes(ks, log_n, num_q, dnum, num_p, levels):
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = oracle.moduli(p)
    gal = [core.galois_rotation(log_n, 3), (2 << log_n) - 1]
    keys = [synth.uniform_evk(mods, dnum, p.n, synth.seed_for(23, 10 * num_q + i)) for i in range(2)]
    plan = ks.Plan(log_n, num_q, dnum, num_p)
    for level in levels:
        say(f"[rot shape] {log_n},{num_q},{dnum},{num_p} level={level}")
        c0 = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(23, 100 + level))
        c1 = synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(23, 200 + level))
        want = core.rotate_hoisted(p, mods, level, c0, c1, gal, keys)
        outs = plan.rotate_hoisted(level, dev(c0), dev(c1), [(dev(k), g) for k, g in zip(keys, gal)])
        torch.cuda.synchronize()
        for o, w in zip(outs, want):
            assert np.array_equal(host(o), w), (level, np.argwhere(host(o) != w)[:5])
    plan.close()


def test_mult_relin_plain_workload_decrypts(ks):
    p = oracle.Params(12, 4, 2, 2)
    mods = oracle.moduli(p)
    s, evk, h = core.keygen_relin(p, mods, 31)
    plan = ks.Plan(12, 4, 2, 2)
    for level in (3, 1, 0):
        a0, a1, b0, b1 = [synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(24, 10 * level + i))
                          for i in range(4)]
        want = core.mult_relin(p, mods, level, a0, a1, b0, b1, evk)
        for tt in (1, 2):
            say(f"[relin plain] level={level} tt={tt}")
            plan.configure("oc", tile_towers=tt)
            got = host(plan.mult_relin(dev(evk), level, dev(a0), dev(a1), dev(b0), dev(b1)))
            assert np.array_equal(got, want), (level, tt, np.argwhere(got != want)[:5])
    plan.close()


@pytest.mark.parametrize("log_n,num_q,dnum,num_p,level", [(16, 24, 3, 8, 23), (13, 9, 3, 2, 6), (12, 7, 7, 1, 6)])
def test_mult_relin_shapes(ks, log_n, num_q, dnum, num_p, level):
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = oracle.moduli(p)
    evk = synth.uniform_evk(mods, dnum, p.n, synth.seed_for(25, num_q))
    a0, a1, b0, b1 = [synth.uniform_limbs(mods[:level + 1], p.n, synth.seed_for(25, 100 + i)) for i in range(4)]
    want = core.mult_relin(p, mods, level, a0, a1, b0, b1, evk)
    plan = ks.Plan(log_n, num_q, dnum, num_p)
    say(f"[relin] {log_n},{num_q},{dnum},{num_p} level={level}")
    got = host(plan.mult_relin(dev(evk), level, dev(a0), dev(a1), dev(b0), dev(b1)))
    bad = np.argwhere(got != want)
    assert bad.size == 0, (bad[:5], len(bad))
    plan.close()


def test_rotation_rejections(ks):
    plan = ks.Plan(12, 4, 2, 2)
    mods = plan.moduli
    c0 = dev(synth.uniform_limbs(mods[:4], plan.n, 1))
    c1 = dev(synth.uniform_limbs(mods[:4], plan.n, 2))
    evk = dev(synth.uniform_evk(mods, 2, plan.n, 3))
    out = torch.empty((2, 4, plan.n), dtype=torch.int32, device="cuda")
    ws = plan._ws(ks.ks_rotate_workspace_size(plan.handle, 3, 1), "cuda")

    def call(**kw):
        args = dict(c0=c0, c1=c1, rots=[(evk, 5, out)], ws=ws)
        args.update(kw)
        with pytest.raises(ks.KsError) as e:
            ks.ks_rotate_hoisted(plan.handle, 3, args["c0"], args["c1"], args["rots"], args["ws"])
        return e.value.status
    assert call(rots=[(evk, 4, out)]) == ks.KS_ERR_INVALID_ARG           # even element
    assert call(rots=[(evk, 2 * plan.n + 1, out)]) == ks.KS_ERR_INVALID_ARG
    big = torch.empty((4, 4, plan.n), dtype=torch.int32, device="cuda")
    # an output over c0 (both inside one buffer, so in bounds either way)
    assert call(c0=big[0], rots=[(evk, 5, big[0:2])]) == ks.KS_ERR_INVALID_ARG
    assert call(ws=ws[: ws.numel() // 2]) == ks.KS_ERR_BUDGET
    plan.configure("mp")
    assert call() == ks.KS_ERR_UNSUPPORTED
    with pytest.raises(ks.KsError) as e:
        plan.mult_relin(evk, 3, c0, c1, c0, c1)
    assert e.value.status == ks.KS_ERR_UNSUPPORTED
    plan.configure("oc")
    with pytest.raises(ks.KsError) as e:
        plan.automorphism(c0, 6)
    assert e.value.status == ks.KS_ERR_INVALID_ARG
    plan.close()


def test_argument_errors_of_the_callers(ks):
    """Argument errors of the rotation, sum, multiplication, automorphism and
    compressed-key entry points are rejected on the host before any launch
    (every buffer here is in bounds either way); empty calls succeed."""
    plan = ks.Plan(12, 4, 2, 2)
    mods, n = plan.moduli, plan.n
    c0 = dev(synth.uniform_limbs(mods[:4], n, 1))
    c1 = dev(synth.uniform_limbs(mods[:4], n, 2))
    evk = dev(synth.uniform_evk(mods, 2, n, 3))
    big = torch.zeros((8, 4, n), dtype=torch.int32, device="cuda")
    out = big[0:2]
    E = ks.KsError
    # empty calls
    ks.ks_rotate_hoisted(plan.handle, 3, c0, c1, [], plan._ws(256, "cuda"))
    ks.ks_rotate_sum_hoisted(plan.handle, 3, c0, c1, [], out, plan._ws(256, "cuda"))
    ks.ks_automorphism(plan.handle, 5, 0, c0, out)
    ks.ks_keyswitch_batch_seeded(plan.handle, [], plan._ws(256, "cuda"))
    assert ks.ks_rotate_workspace_size(plan.handle, 3, 0) == 0
    assert ks.ks_rotate_sum_workspace_size(plan.handle, 3, 0) == 0
    # rotation sum
    ws = plan._ws(ks.ks_rotate_sum_workspace_size(plan.handle, 3, 1), "cuda")
    diag = big[4:8].reshape(-1)[: 6 * n]  # one diagonal of L+1+K = 6 rows
    cases = [
        (dict(terms=[(evk, 6, None)]), ks.KS_ERR_INVALID_ARG),              # even element
        (dict(terms=[(evk, 5, diag[1:])]), ks.KS_ERR_INVALID_ARG),          # misaligned diagonal
        (dict(terms=[(evk, 5, big[2:].reshape(-1))], out=big[2:4]), ks.KS_ERR_INVALID_ARG),  # out inside a diagonal
        (dict(ws=ws[: ws.numel() // 2]), ks.KS_ERR_BUDGET),
        (dict(out=big[0:2], c0=big[1]), ks.KS_ERR_INVALID_ARG),             # out over c0
    ]
    for kw, status in cases:
        a = dict(terms=[(evk, 5, diag)], out=out, ws=ws, c0=c0)
        a.update(kw)
        with pytest.raises(E) as e:
            ks.ks_rotate_sum_hoisted(plan.handle, 3, a["c0"], c1, a["terms"], a["out"], a["ws"])
        assert e.value.status == status, kw
    # multiplication
    wsm = plan._ws(ks.ks_mult_workspace_size(plan.handle, 3), "cuda")
    with pytest.raises(E) as e:
        ks.ks_mult_relin(plan.handle, evk, 3, c0, c1, c0, c1, out, wsm[: wsm.numel() // 2])
    assert e.value.status == ks.KS_ERR_BUDGET
    with pytest.raises(E) as e:
        ks.ks_mult_relin(plan.handle, evk, 3, big[0], c1, c0, c1, big[0:2], wsm)  # out over a0
    assert e.value.status == ks.KS_ERR_INVALID_ARG
    with pytest.raises(E) as e:
        ks.ks_mult_relin(plan.handle, evk, 4, c0, c1, c0, c1, out, wsm)  # level beyond L
    assert e.value.status == ks.KS_ERR_INVALID_ARG
    # automorphism: output over the input, bad element
    with pytest.raises(E) as e:
        ks.ks_automorphism(plan.handle, 5, 2, big[0], big[0])
    assert e.value.status == ks.KS_ERR_INVALID_ARG
    with pytest.raises(E) as e:
        ks.ks_automorphism(plan.handle, 2 * n + 1, 1, c0, out)
    assert e.value.status == ks.KS_ERR_INVALID_ARG
    # expansion of compressed keys: misaligned destination
    with pytest.raises(E) as e:
        ks.ks_expand_seeded_a(plan.handle, 1, evk.view(-1)[1:])
    assert e.value.status == ks.KS_ERR_INVALID_ARG
    # hoisted rotations with compressed keys: an output inside a key
    b = evk.view(2, 2, -1)[:, 0].contiguous()
    wsr = plan._ws(ks.ks_rotate_workspace_size(plan.handle, 3, 1), "cuda")
    with pytest.raises(E) as e:
        ks.ks_rotate_hoisted_seeded(plan.handle, 3, c0, c1, [(b, 1, 5, b.view(-1)[: 8 * n].view(2, 4, n))], wsr)
    assert e.value.status == ks.KS_ERR_INVALID_ARG
    plan.close()
