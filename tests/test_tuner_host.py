"""Host-side logic of the autotuner and cost model (no GPU): the search
space, configuration keys, workload grouping, feature vectors, the tune
cache round trip, the regret report and the mixed-level workload draw."""
import json

import numpy as np

from paper_2311_01598_amd import costmodel, tune


def test_config_space_is_unique_and_complete():
    cs = tune.config_space()
    keys = [tune.config_key(c) for c in cs]
    assert len(cs) == 24 and len(set(keys)) == len(keys)
    assert sum(c["schedule"] == "mp" for c in cs) == 9
    assert sum(c["schedule"] == "dc" for c in cs) == 9
    assert {tune.config_key(c) for c in cs if c["schedule"] == "oc"} == {
        "oc/t1/c16/r8", "oc/t2/c16/r8", "oc/t2/c16/r8/m3", "oc/t1/c16/r8/o2", "oc/t2/c16/r8/o2",
        "oc/t2/c16/r8/m3/o2"}
    # every configuration maps onto ks_config_t fields the binding accepts
    import paper_2311_01598_amd as ks
    for c in cs:
        assert set(tune.config_fields(c)) <= set(ks.CONFIG_FIELDS)


def test_features_match_the_feature_list():
    for c in tune.config_space():
        f = costmodel.features(16, 24, 3, 8, 23, 4, c)
        assert len(f) == len(costmodel.FEATURES)
        assert sum(f[8:11]) == 1  # exactly one schedule flag
    oc3 = [c for c in tune.config_space() if c.get("batch_mode") == 3][0]
    assert costmodel.features(16, 24, 3, 8, 23, 4, oc3)[-2] == 1
    assert costmodel.features(16, 24, 3, 8, 23, 4, oc3)[-1] == 0
    o2 = [c for c in tune.config_space() if c.get("batch_order") == 2][0]
    assert costmodel.features(16, 24, 3, 8, 23, 4, o2)[-1] == 1
    assert costmodel.features(16, 24, 3, 8, 23, 4, o2, spread=0.5)[7] == 0.5
    # live digits at a lower level: 12 towers of alpha 8 -> 2 digits
    assert costmodel.features(16, 24, 3, 8, 11, 1, tune.config_space()[0])[5] == 2


def test_group_workloads_and_report(tmp_path):
    rows = []
    rng = np.random.default_rng(0)
    for nq in (8, 16):
        for c in tune.config_space():
            ms = (1.0 if c["schedule"] == "oc" else 3.0) * nq * (1 + 0.01 * rng.random())
            rows.append(tune.record((14, nq, 2, nq // 2), nq - 1, 1, c, ms))
    g = tune.group_workloads(rows)
    assert len(g) == 2 and all(len(t) == 24 for t in g.values())
    exp = {"summary": {"train_records": 24, "test_workloads": 1, "configs": 24, "top_m": 3,
                       "regret_model_pick": {"mean": 0.0, "p90": 0.0, "max": 0.0},
                       "regret_pruned_top_m": {"mean": 0.0, "p90": 0.0, "max": 0.0},
                       "regret_random_top_m": {"mean": 1.0, "p90": 2.0, "max": 2.0},
                       "regret_fixed_default": {"mean": 0.0, "p90": 0.0, "max": 0.0},
                       "final_train_loss": 0.01}}
    text = tune.report(rows, exp, ("cmd",))
    assert "24 configurations" in text and "median 3.00x" in text


def test_tune_cache_round_trip(tmp_path):
    path = str(tmp_path / "cache.json")
    c = tune.TuneCache(path)
    cfg = tune.config_space()[-1]
    c.put("gpu0", (16, 24, 3, 8), 23, 16, cfg)
    again = tune.TuneCache(path).get("gpu0", (16, 24, 3, 8), 23, 16)
    assert again == cfg
    assert json.load(open(path))


def test_mixed_levels_cover_the_stated_range():
    lv = tune.mixed_levels(48, 4000, seed=1)
    towers = [l + 1 for l in lv]
    assert min(towers) == 16 and max(towers) == 48
    assert lv == tune.mixed_levels(48, 4000, seed=1)
