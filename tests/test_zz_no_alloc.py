"""ks_keyswitch_noalloc: the key switch for callers that cannot allocate.

Its intermediates live in the library's fixed per-GPU device array instead of
a caller workspace.  Two calls in a row through the C ABI, the second with a
smaller input, each equal to ks_keyswitch (OC) with a workspace of its own,
word for word; the array keeps the first call's contents, so the second call
shows that nothing stale is read.  The call allocates no device memory
(free device memory is unchanged across it), and it refuses oversized
levels, other schedules and traced plans before enqueuing anything.
"""
import sys

import numpy as np
import pytest

import oracle
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


def test_noalloc_equals_keyswitch_twice_smaller_second(ks):
    plan = ks.Plan(16, 24, 3, 8, schedule="oc")
    mods = plan.moduli
    n = plan.n
    evk = dev(synth.uniform_evk(mods, 3, n, synth.seed_for(9, 0)))
    big = dev(synth.uniform_limbs(mods[:24], n, synth.seed_for(9, 1)))
    small = dev(synth.uniform_limbs(mods[:10], n, synth.seed_for(9, 2)))
    assert plan.workspace_bytes([23]) <= ks.KS_NOALLOC_SCRATCH_BYTES
    # references through the existing entry point, each with its own workspace
    want_big = plan.keyswitch(evk, 23, big)
    want_small = plan.keyswitch(evk, 9, small)
    out_big = torch.full((2, 24, n), -1, dtype=torch.int32, device="cuda")
    out_small = torch.full((2, 10, n), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    say("[noalloc] call 1: N=2^16 l+1=24 dnum=3 K=8")
    ks.ks_keyswitch_noalloc(plan.handle, evk, 23, big, out_big)
    say("[noalloc] call 2: N=2^16 l+1=10")
    ks.ks_keyswitch_noalloc(plan.handle, evk, 9, small, out_small)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert torch.equal(out_big, want_big)
    assert torch.equal(out_small, want_small)
    plan.close()


def test_noalloc_small_plan_equals_oracle_after_a_large_call(ks):
    """Another plan on the same GPU shares the array: after the large call
    above (or on its own), a small key switch still equals the oracle and
    ks_keyswitch."""
    p = oracle.Params(12, 4, 2, 2)
    mods = oracle.moduli(p)
    s, s2, evk, h = oracle.keygen(p, mods, seed=31)
    d = synth.uniform_limbs(mods[:4], p.n, synth.seed_for(9, 3))
    plan = ks.Plan(12, 4, 2, 2, schedule="oc")
    evk_d, d_d = dev(evk), dev(d)
    for level in (3, 1):
        say(f"[noalloc] N=2^12 level={level}")
        out = torch.full((2, level + 1, p.n), -1, dtype=torch.int32, device="cuda")
        ks.ks_keyswitch_noalloc(plan.handle, evk_d, level, d_d[:level + 1], out)
        ref = plan.keyswitch(evk_d, level, d_d[:level + 1])
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        assert np.array_equal(host(out), oracle.keyswitch(p, mods, level, evk, d[:level + 1]))
    plan.close()


def test_noalloc_refusals(ks):
    """Refused on the host, before anything is enqueued: a level whose OC
    workspace exceeds the array, another schedule, a traced plan, a bad
    level."""
    plan = ks.Plan(17, 45, 3, 15, schedule="oc")  # Table III BTS3: 172 MiB of OC workspace at the top level
    n = plan.n
    assert plan.workspace_bytes([44]) > ks.KS_NOALLOC_SCRATCH_BYTES
    evk = torch.zeros((3, 2, 60, n), dtype=torch.int32, device="cuda")
    d = torch.zeros((45, n), dtype=torch.int32, device="cuda")
    out = torch.empty((2, 45, n), dtype=torch.int32, device="cuda")
    with pytest.raises(ks.KsError) as e:
        ks.ks_keyswitch_noalloc(plan.handle, evk, 44, d, out)
    assert e.value.status == ks.KS_ERR_BUDGET
    with pytest.raises(ks.KsError) as e:
        ks.ks_keyswitch_noalloc(plan.handle, evk, 45, d, out)
    assert e.value.status == ks.KS_ERR_INVALID_ARG
    d4 = torch.zeros((4, n), dtype=torch.int32, device="cuda")
    out4 = torch.empty((2, 4, n), dtype=torch.int32, device="cuda")
    plan.configure("mp")
    with pytest.raises(ks.KsError) as e:
        ks.ks_keyswitch_noalloc(plan.handle, evk, 3, d4, out4)
    assert e.value.status == ks.KS_ERR_UNSUPPORTED
    plan.configure("oc")
    ks.ks_trace_enable(plan.handle, True)
    with pytest.raises(ks.KsError) as e:
        ks.ks_keyswitch_noalloc(plan.handle, evk, 3, d4, out4)
    assert e.value.status == ks.KS_ERR_UNSUPPORTED
    ks.ks_trace_enable(plan.handle, False)
    torch.cuda.synchronize()
    plan.close()
