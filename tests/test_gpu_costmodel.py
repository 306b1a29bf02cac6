"""GPU tests of the autotuner and its learned cost model.

* The MLP kernels (forward, loss gradient, backward, Adam) match the float64
  oracle (oracle/mlp.py, itself pinned by finite differences) within fp32
  tolerances: relative 1e-4 of the largest magnitude.
* Exhaustive tuning picks the fastest measured configuration and the tune
  cache returns it.
* On real timings of small workloads, the trained network's top-3 pruned
  search (3 of 24 timings per workload) has no more regret than the fixed
  default configuration (the method without the network) and less than
  timing 3 random configurations.
* The tuner's choice is the live path: with the schedule AUTO, a call runs
  the configuration tuned for its shape (resolution rules, the kernels that
  actually launch, and identical outputs).
"""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_01598_amd as m
    return m


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def _t32(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def _close(got, want, rel=1e-4):
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    scale = max(1.0, np.abs(want).max())
    assert np.abs(got - want).max() <= rel * scale, (np.abs(got - want).max(), scale)


@pytest.mark.parametrize("F,H,B", [(13, 64, 257), (5, 16, 33), (13, 64, 1)])
def test_mlp_kernels_match_oracle(ks, F, H, B):
    rng = np.random.default_rng(F * 100 + B)
    p = rng.normal(0, 0.3, omlp.param_count(F, H)).astype(np.float32)
    X = rng.normal(0, 1, (B, F)).astype(np.float32)
    T = rng.normal(0, 1, B).astype(np.float32)
    P = ks.ks_mlp_param_count(F, H)
    assert P == omlp.param_count(F, H)
    pd, Xd, Td = _t(p), _t(X), _t(T)
    Y = torch.empty(B, device="cuda")
    act = torch.empty(2 * B * H, device="cuda")
    ks.ks_mlp_forward(F, H, B, pd, Xd, Y, act)
    y_want, h1, h2 = omlp.forward(p.astype(np.float64), X.astype(np.float64), F, H)
    _close(Y.cpu().numpy(), y_want)
    _close(act.cpu().numpy(), np.concatenate([h1.ravel(), h2.ravel()]))
    dY = torch.empty(B, device="cuda")
    loss = torch.empty(1, device="cuda")
    ks.ks_mlp_mse_grad(B, Y, Td, dY, loss)
    _close(loss.cpu().numpy()[0], omlp.loss(p.astype(np.float64), X.astype(np.float64), T, F, H))
    grads = torch.empty(P, device="cuda")
    scratch = torch.empty(2 * B * H, device="cuda")
    ks.ks_mlp_backward(F, H, B, pd, Xd, act, dY, grads, scratch)
    _close(grads.cpu().numpy(), omlp.grad(p.astype(np.float64), X.astype(np.float64), T, F, H))
    # one Adam step
    g = grads.cpu().numpy().astype(np.float64)
    m0 = rng.normal(0, 0.01, P)
    v0 = np.abs(rng.normal(0, 0.01, P))
    md, vd = _t(m0), _t(v0)
    ks.ks_mlp_adam(P, pd, grads, md, vd, 1e-2, 0.9, 0.999, 1e-8, 3)
    p_want, m_want, v_want = omlp.adam_step(p.astype(np.float64), g, m0, v0, 1e-2, 0.9, 0.999, 1e-8, 3)
    _close(pd.cpu().numpy(), p_want)
    _close(md.cpu().numpy(), m_want)


def test_training_fits_a_smooth_function(ks):
    from paper_2311_01598_amd import costmodel
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, (512, len(costmodel.FEATURES)))
    y = np.sin(2 * X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] + 0.3 * X[:, 7]
    m = costmodel.CostModel(seed=1)
    hist = m.fit(X, y, steps=1500, lr=3e-3, log_every=500)
    assert hist[-1][1] < 0.05 * np.var(y) / np.var(y), hist  # standardised loss below 5 %
    assert np.mean((m.predict(X) - y) ** 2) < 0.05 * np.var(y)


def test_exhaustive_tuning_and_cache(ks, tmp_path):
    from paper_2311_01598_amd import tune
    plan = ks.Plan(12, 6, 2)
    work = tune.Workload(plan, 5, 1, seed=7)
    best, times = tune.exhaustive(work, reps=3)
    assert len(times) == len(tune.config_space())
    assert times[tune.config_key(best)] == min(times.values())
    cache = tune.TuneCache(str(tmp_path / "cache.json"))
    cfg = tune.tune(plan, 5, 1, cache=cache, reps=3)
    again = tune.TuneCache(str(tmp_path / "cache.json")).get("gpu0", (12, 6, 2, plan.num_p), 5, 1)
    assert again == cfg
    plan.close()


def test_pruned_search_against_fixed_default_and_random(ks, tmp_path):
    """Collect real timings for small parameter points, train on 70 %, and
    compare on the held-out 30 %, against exhaustive search: the network's
    top-3 pruned search versus the fixed default configuration (no network,
    no timing) and versus timing 3 random configurations."""
    from paper_2311_01598_amd import costmodel, tune
    rows = []
    for log_n in (12, 13):
        for nq in (4, 8, 12):
            for dn in (1, 2, 3):
                if -(-nq // dn) > 32:
                    continue
                plan = ks.Plan(log_n, nq, dn)
                for level in sorted({nq - 1, nq // 2}):
                    work = tune.Workload(plan, level, 1, seed=level)
                    for c in tune.config_space():
                        rows.append(tune.record((log_n, nq, dn, plan.num_p), level, 1, c, tune.time_config(work, c, 3)))
                    print(f"[collect] N=2^{log_n} towers={nq} dnum={dn} level={level}", flush=True)
                plan.close()
    res = costmodel.experiment(rows, top_m=3, seed=0, steps=1500, holdout=0.3)
    s = res["summary"]
    print(s, flush=True)
    assert s["test_workloads"] >= 3
    assert s["regret_pruned_top_m"]["mean"] <= s["regret_fixed_default"]["mean"] + 0.02
    assert s["regret_pruned_top_m"]["mean"] < s["regret_random_top_m"]["mean"]
    assert s["timings_per_workload"]["pruned"] * 5 < s["timings_per_workload"]["exhaustive"]


def test_auto_resolves_tuned_entries(ks):
    """ks_plan_resolve_config: the same level, else the nearest (the higher on
    a tie); the largest tuned count not above the call's, else the smallest;
    zero fields from the plan; OC with the plan's settings when nothing is
    tuned."""
    plan = ks.Plan(12, 8, 2, schedule="auto")
    r = plan.resolve(7, 1)
    assert r["schedule"] == ks.KS_SCHED_OC and r["tile_towers"] == 2 and r["batch_order"] == 1
    plan.set_tuned(7, 1, "mp", col_width=8, row_block=4)
    plan.set_tuned(7, 4, "oc", tile_towers=1, batch_mode=3, batch_order=2)
    plan.set_tuned(3, 1, "dc", col_width=32, row_block=16)
    mp = {"schedule": ks.KS_SCHED_MP, "col_width": 8, "row_block": 4}
    dc = {"schedule": ks.KS_SCHED_DC, "col_width": 32, "row_block": 16}
    oc = {"schedule": ks.KS_SCHED_OC, "tile_towers": 1, "batch_mode": 3, "batch_order": 2}
    for (level, count), want in {(7, 1): mp, (7, 2): mp, (7, 4): oc, (7, 64): oc, (5, 1): mp, (5, 9): oc,
                                 (4, 1): dc, (3, 16): dc, (0, 1): dc}.items():
        got = plan.resolve(level, count)
        assert {k: got[k] for k in want} == want, (level, count, got)
    # a plan whose schedule is not AUTO runs its own configuration
    plan.configure("mp", col_width=16)
    assert plan.resolve(7, 4)["schedule"] == ks.KS_SCHED_MP and plan.resolve(7, 4)["col_width"] == 16
    plan.configure("auto")
    plan.clear_tuned()
    assert plan.resolve(7, 1)["schedule"] == ks.KS_SCHED_OC
    with pytest.raises(ks.KsError):
        plan.set_tuned(8, 1, "oc")       # level beyond the plan
    with pytest.raises(ks.KsError):
        plan.set_tuned(7, 1, "auto")     # an entry names a schedule
    plan.close()


def test_auto_runs_the_tuned_pick(ks, tmp_path):
    """The tuner (exhaustive here, as the arbiter) records its pick in the plan;
    with the schedule AUTO a call of that shape resolves to the pick, launches
    that schedule's kernels, and returns the same words as the pick run
    explicitly and as the oracle.  Calls that run the OC order only
    (compressed keys) still run OC when the tuned entry names MP."""
    import oracle
    import synth
    from paper_2311_01598_amd import tune
    p = oracle.Params(12, 6, 2, 3)
    mods = oracle.moduli(p)
    evk = synth.uniform_evk(mods, 2, p.n, synth.seed_for(40, 0))
    d = synth.uniform_limbs(mods[:6], p.n, synth.seed_for(40, 1))
    want = oracle.keyswitch(p, mods, 5, evk, d)
    plan = ks.Plan(12, 6, 2, 3)
    tuner = tune.Tuner(cache=tune.TuneCache(str(tmp_path / "cache.json")), reps=3)
    cfg = tuner.tune(plan, 5, 1)
    assert plan.config["schedule"] == ks.KS_SCHED_AUTO
    r = plan.resolve(5, 1)
    assert r["schedule"] == ks.SCHEDULES[cfg["schedule"]]
    assert {k: r[k] for k in tune.config_fields(cfg)} == tune.config_fields(cfg)
    ev, dd = _t32(evk), _t32(d)
    ks.ks_trace_enable(plan.handle, True)
    got = plan.keyswitch(ev, 5, dd)
    torch.cuda.synchronize()
    ks.ks_trace_enable(plan.handle, False)
    names = set(ks.ks_trace_read(plan.handle))
    assert any(n.startswith("oc.") for n in names) == (cfg["schedule"] == "oc"), (cfg, names)
    assert np.array_equal(got.cpu().numpy().view(np.uint32), want)
    # a tuned MP entry: AUTO runs MP (its kernels), compressed keys still OC
    plan.set_tuned(5, 1, "mp", col_width=8, row_block=4)
    ks.ks_trace_enable(plan.handle, True)
    got = plan.keyswitch(ev, 5, dd)
    torch.cuda.synchronize()
    ks.ks_trace_enable(plan.handle, False)
    names = set(ks.ks_trace_read(plan.handle))
    assert names and not any(n.startswith("oc.") for n in names), names
    assert np.array_equal(got.cpu().numpy().view(np.uint32), want)
    ev_b = evk.copy()
    from oracle import core
    ev_b[:, 1] = core.seeded_a(p, mods, 5)[:, 1]
    got = plan.keyswitch_seeded(_t32(np.ascontiguousarray(ev_b[:, 0])), 5, 5, dd)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().view(np.uint32), oracle.keyswitch(p, mods, 5, ev_b, d))
    # the cache answers the same shape without timing again
    again = tune.Tuner(cache=tune.TuneCache(str(tmp_path / "cache.json"))).tune(plan, 5, 1)
    assert tune.config_key(again) == tune.config_key(cfg)
    plan.close()
