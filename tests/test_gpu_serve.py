"""Serving loop tests.

* Under Poisson arrivals with several streams and batches that mix levels and
  keys, each result equals the same request run alone (tolerance 0, the
  arithmetic is exact), and two of them equal the oracle.
* Admission by memory: a budget below one request rejects it and a budget of
  about one request serialises the work; bytes in flight never exceed it.
* Failure handling forced from the host: KS_FAULT_INJECT makes one batch
  launch report a device error; only that batch's requests fail, the server
  goes on and the rest complete correctly.
* Invalid requests (unknown key, level beyond the plan) are rejected.
"""
import os

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")


def test_pool_first_fit_and_merge():
    from paper_2311_01598_amd.serve import HbmPool
    p = HbmPool(4096, device="cpu")
    a = p.alloc(1000)
    b = p.alloc(256)
    c = p.alloc(300)
    assert a == (0, 1024) and b == (1024, 256) and c == (1280, 512)
    assert p.alloc(4096) is None
    p.release(*b)
    assert p.alloc(200) == (1024, 256)  # first fit reuses the hole
    p.release(1024, 256)
    p.release(*a)
    p.release(*c)
    assert p.free == [(0, 4096)]  # neighbours merge back into one block


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_01598_amd as m
    return m


LOG_N, NUM_Q, DNUM, NKEYS = 13, 8, 3, 3


@pytest.fixture(scope="module")
def setup(ks):
    plan = ks.Plan(LOG_N, NUM_Q, DNUM)
    keys = [torch.from_numpy(synth.uniform_evk(plan.moduli, DNUM, plan.n, 900 + k).view(np.int32)).cuda()
            for k in range(NKEYS)]
    yield plan, keys
    plan.close()


def _requests(plan, count, seed):
    from paper_2311_01598_amd.serve import Request
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        level = int(rng.integers(0, NUM_Q))
        d = torch.from_numpy(synth.uniform_limbs(plan.moduli[:level + 1], plan.n, seed * 1000 + i).view(np.int32)).cuda()
        reqs.append(Request(i, int(rng.integers(0, NKEYS)), LOG_N, level, d, 0.0))
    return reqs


def _alone(plan, keys, r):
    plan.configure("mp")  # a different schedule: identical bits are required
    out = plan.keyswitch(keys[r.key], r.level, r.d)
    plan.configure("oc", batch_mode=1, tile_towers=2)
    return out


@pytest.mark.gpu
def test_served_results_equal_alone(ks, setup):
    from paper_2311_01598_amd.serve import Server, poisson_arrivals
    plan, keys = setup
    reqs = _requests(plan, 48, seed=5)
    server = Server({LOG_N: plan}, {LOG_N: keys}, budget_bytes=64 << 20, streams=3, max_batch=8)
    t = poisson_arrivals(20000.0, len(reqs), seed=6)
    st = server.run(list(zip(t, reqs)), max_seconds=60)
    print(st, flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["rejected"] == 0
    assert st["batches"] < len(reqs)  # requests were batched together
    assert st["high_water_bytes"] <= st["budget_bytes"]
    assert st["p99_ms"] >= st["p50_ms"] > 0
    for r in reqs:
        want = _alone(plan, keys, r)
        assert torch.equal(r.out, want), f"request {r.rid} level {r.level} key {r.key}"
    # two of them against the oracle
    from oracle import core
    for r in reqs[:2]:
        evk = keys[r.key].cpu().numpy().view(np.uint32)
        d = r.d.cpu().numpy().view(np.uint32)
        want = core.keyswitch(core.Params(LOG_N, NUM_Q, DNUM, plan.num_p), plan.moduli, r.level, evk, d)
        assert np.array_equal(r.out.cpu().numpy().view(np.uint32), want)


@pytest.mark.gpu
def test_budget_admission(ks, setup):
    from paper_2311_01598_amd.serve import Server
    plan, keys = setup
    reqs = _requests(plan, 6, seed=7)
    one = max(plan.workspace_bytes([r.level]) + 2 * (r.level + 1) * plan.n * 4 for r in reqs)
    # below the largest single request: that request is rejected, never run
    small = Server({LOG_N: plan}, {LOG_N: keys}, budget_bytes=one - 4096, streams=2)
    small.run([(0.0, r) for r in reqs], max_seconds=60)
    big = max(reqs, key=lambda r: r.level)
    assert big.status.startswith("rejected") and big.out is None
    assert small.high_water <= small.budget
    # about one request's worth: everything completes, one batch at a time
    reqs = _requests(plan, 6, seed=7)
    tight = Server({LOG_N: plan}, {LOG_N: keys}, budget_bytes=one + 4096, streams=2)
    st = tight.run([(0.0, r) for r in reqs], max_seconds=60)
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    assert tight.high_water <= tight.budget
    for r in reqs:
        assert torch.equal(r.out, _alone(plan, keys, r))


@pytest.mark.gpu
def test_injected_device_error_fails_only_that_batch(ks, setup):
    from paper_2311_01598_amd.serve import Server
    plan, keys = setup
    reqs = _requests(plan, 12, seed=9)
    server = Server({LOG_N: plan}, {LOG_N: keys}, budget_bytes=64 << 20, streams=2, max_batch=4)
    os.environ["KS_FAULT_INJECT"] = "2"  # the second batch launch reports a device error
    try:
        st = server.run([(0.0, r) for r in reqs], max_seconds=60)
    finally:
        del os.environ["KS_FAULT_INJECT"]
    assert st["failed"] == 4 and st["completed"] == 8, st
    for r in reqs:
        if r.status == "done":
            assert torch.equal(r.out, _alone(plan, keys, r))
        else:
            assert r.status.startswith("failed")


@pytest.mark.gpu
def test_invalid_requests_rejected(ks, setup):
    from paper_2311_01598_amd.serve import Request, Server
    plan, keys = setup
    d = _requests(plan, 1, seed=11)[0].d
    server = Server({LOG_N: plan}, {LOG_N: keys}, budget_bytes=64 << 20)
    bad = [Request(0, NKEYS, LOG_N, 0, d, 0.0), Request(1, 0, LOG_N, NUM_Q, d, 0.0), Request(2, 0, 16, 0, d, 0.0)]
    st = server.run([(0.0, r) for r in bad], max_seconds=10)
    assert st["rejected"] == 3 and st["completed"] == 0


@pytest.mark.gpu
def test_compressed_keys_served_equal_alone(ks, setup):
    """Keys resident half full, half compressed (b halves plus a seed): batches
    never mix the two kinds, and every served result equals the request run
    alone with MP on the expanded key (tolerance 0); one also equals the
    oracle."""
    from paper_2311_01598_amd.serve import Server, poisson_arrivals
    plan, full_keys = setup
    keys, expanded = [], []
    for k, e in enumerate(full_keys):
        if k % 2:
            b = e.view(DNUM, 2, -1)[:, 0].contiguous()
            ex = torch.zeros_like(e)
            ex.view(DNUM, 2, -1)[:, 0] = b
            plan.expand_seeded_a(4242 + k, ex)
            keys.append((b, 4242 + k))
            expanded.append(ex)
        else:
            keys.append(e)
            expanded.append(e)
    reqs = _requests(plan, 40, seed=13)
    server = Server({LOG_N: plan}, {LOG_N: keys}, budget_bytes=64 << 20, streams=3, max_batch=8)
    st = server.run(list(zip(poisson_arrivals(20000.0, len(reqs), seed=14), reqs)), max_seconds=60)
    print(st, flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert any(k % 2 for k in (r.key for r in reqs)) and any(k % 2 == 0 for k in (r.key for r in reqs))
    for r in reqs:
        assert torch.equal(r.out, _alone(plan, expanded, r)), f"request {r.rid} key {r.key}"
    from oracle import core
    r = next(x for x in reqs if x.key % 2)
    evk = expanded[r.key].cpu().numpy().view(np.uint32)
    want = core.keyswitch(core.Params(LOG_N, NUM_Q, DNUM, plan.num_p), plan.moduli, r.level, evk,
                          r.d.cpu().numpy().view(np.uint32))
    assert np.array_equal(r.out.cpu().numpy().view(np.uint32), want)


@pytest.mark.gpu
def test_rotation_requests_served_equal_alone(ks, setup):
    """A mix of key-switch requests and rotation requests (c0, c1, Galois
    element, full rotation key): batches hold one kind, and every served
    rotation equals the same rotation run alone (a hoisted group of one),
    every key switch the MP key switch alone; one rotation also equals the
    oracle."""
    from paper_2311_01598_amd.serve import Request, Server, poisson_arrivals
    from oracle import core
    plan, keys = setup
    rng = np.random.default_rng(17)
    reqs = []
    for i in range(40):
        level = int(rng.integers(0, NUM_Q))
        d = torch.from_numpy(synth.uniform_limbs(plan.moduli[:level + 1], plan.n, 17000 + i).view(np.int32)).cuda()
        key = int(rng.integers(0, NKEYS))
        if i % 2:
            c0 = torch.from_numpy(synth.uniform_limbs(plan.moduli[:level + 1], plan.n, 18000 + i).view(np.int32)).cuda()
            reqs.append(Request(i, key, LOG_N, level, d, 0.0, c0=c0, galois=core.galois_rotation(LOG_N, key + 1)))
        else:
            reqs.append(Request(i, key, LOG_N, level, d, 0.0))
    server = Server({LOG_N: plan}, {LOG_N: keys}, budget_bytes=64 << 20, streams=3, max_batch=8)
    st = server.run(list(zip(poisson_arrivals(20000.0, len(reqs), seed=18), reqs)), max_seconds=60)
    print(st, flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["rejected"] == 0
    for r in reqs:
        if r.galois is None:
            want = _alone(plan, keys, r)
        else:
            want = plan.rotate(keys[r.key], r.galois, r.level, r.c0, r.d)
        assert torch.equal(r.out, want), f"request {r.rid}"
    r = next(x for x in reqs if x.galois is not None)
    ev = keys[r.key].cpu().numpy().view(np.uint32)
    want = core.rotate_hoisted(core.Params(LOG_N, NUM_Q, DNUM, plan.num_p), plan.moduli, r.level,
                               r.c0.cpu().numpy().view(np.uint32), r.d.cpu().numpy().view(np.uint32), [r.galois],
                               [ev])[0]
    assert np.array_equal(r.out.cpu().numpy().view(np.uint32), want)
    # a rotation request with a compressed key is rejected (rotation batches take full keys)
    bad = Request(99, 0, LOG_N, 0, reqs[0].d[:1], 0.0, c0=reqs[0].d[:1], galois=5)
    srv = Server({LOG_N: plan}, {LOG_N: [(keys[0].view(DNUM, 2, -1)[:, 0].contiguous(), 1)]}, budget_bytes=64 << 20)
    assert srv.run([(0.0, bad)], max_seconds=10)["rejected"] == 1
