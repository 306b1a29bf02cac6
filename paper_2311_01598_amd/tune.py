"""Autotuner: exhaustive search over launch configurations, a timing
database, and a tune cache.

A configuration is (schedule, tile_towers, col_width, row_block,
batch_mode, batch_order): the execution order of Sec. IV (MP, DC or OC), its
tile shapes, and for batches the two-stream split and the job order.  All
configurations compute identical bits, so the tuner only measures time.
Exhaustive search times every configuration (median of `reps` runs after a
warm-up) and is the fallback, and the reference that the cost-model-pruned
search (costmodel.py), which times only the predicted best few, is scored
against.  `Tuner` puts the result in the live path: it records the choice in
the plan (ks_plan_set_tuned) and sets the plan's schedule to AUTO, so every
later call of that shape runs with it.

Command line (on a machine with the GPU):
    python -m paper_2311_01598_amd.tune collect --out timings.jsonl [--quick]
    python -m paper_2311_01598_amd.tune experiment --db timings.jsonl --out result.json
    python -m paper_2311_01598_amd.tune train --db timings.jsonl   # weights of the live tuner
    python -m paper_2311_01598_amd.tune report --db timings.jsonl --exp result.json --out summary.md
"""
import argparse
import itertools
import json
import os
import random
import sys
import time

import numpy as np

SCHEDULES = ("mp", "dc", "oc")


def config_space():
    """Every configuration the tuner considers (24): MP and DC with 3 x 3
    tile shapes; OC with 1 or 2 targets per conversion tile, for batches the
    two-stream split (batch mode 3), and the batch order (jobs as given, or
    by decreasing level: it changes how a mixed-level batch's tiles spread
    over the XCDs, not its results)."""
    out = []
    for cw, rb in itertools.product((8, 16, 32), (4, 8, 16)):
        out.append({"schedule": "mp", "tile_towers": 1, "col_width": cw, "row_block": rb})
    for cw, rb in itertools.product((8, 16, 32), (4, 8, 16)):
        out.append({"schedule": "dc", "tile_towers": 1, "col_width": cw, "row_block": rb})
    for tt, mode, order in ((1, 1, 1), (2, 1, 1), (2, 3, 1), (1, 1, 2), (2, 1, 2), (2, 3, 2)):
        out.append({"schedule": "oc", "tile_towers": tt, "col_width": 16, "row_block": 8, "batch_mode": mode,
                    "batch_order": order})
    return out


def config_key(c):
    k = f"{c['schedule']}/t{c['tile_towers']}/c{c['col_width']}/r{c['row_block']}"
    k += "/m3" if c.get("batch_mode", 1) == 3 else ""
    return k + "/o2" if c.get("batch_order", 1) == 2 else k


def config_fields(c):
    """ks_config_t fields of a configuration (schedule aside)."""
    return {"tile_towers": c["tile_towers"], "col_width": c["col_width"], "row_block": c["row_block"],
            "batch_mode": c.get("batch_mode", 1), "batch_order": c.get("batch_order", 1)}


def apply_config(plan, c):
    plan.configure(c["schedule"], **config_fields(c))


class Workload:
    """Synthetic inputs for timing one (plan, level, count): `count` key
    switches at `level`, or, with `levels`, one batch at those levels (level
    = the largest, count = how many)."""

    def __init__(self, plan, level, count, seed=0, levels=None):
        import torch

        import synth
        self.levels = list(levels) if levels is not None else [level] * count
        self.plan, self.level, self.count = plan, max(self.levels), len(self.levels)
        self.spread = float(np.mean(self.levels) + 1) / (self.level + 1)
        mods = plan.moduli
        self.evk = synth.uniform_limbs_device(mods, plan.n, seed, torch, lead=(plan.dnum, 2))
        self.ins = [synth.uniform_limbs_device(mods[:l + 1], plan.n, seed + 1 + i, torch)
                    for i, l in enumerate(self.levels)]
        self.outs = [torch.empty((2, l + 1, plan.n), dtype=torch.int32, device="cuda") for l in self.levels]

    def run(self, ws):
        if self.count == 1:
            self.plan.keyswitch(self.evk, self.level, self.ins[0], out=self.outs[0], workspace=ws)
        else:
            self.plan.keyswitch_batch([(self.evk, l, x, o) for l, x, o in zip(self.levels, self.ins, self.outs)],
                                      workspace=ws)


def time_config(work, cfg, reps=5, span_ms=1.0):
    """Median milliseconds per key switch of `work` under configuration `cfg`.

    Each of the `reps` timings covers enough back-to-back calls to span about
    `span_ms` (at most 32 calls), so that a single key switch of ~0.1 ms is
    not timed against the resolution and jitter of one event pair."""
    import torch
    plan = work.plan
    apply_config(plan, cfg)
    ws = plan.workspace(work.levels)
    work.run(ws)
    torch.cuda.synchronize()

    def timed(calls):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(calls):
            work.run(ws)
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / calls

    inner = int(min(32, max(1, np.ceil(span_ms / max(timed(1), 1e-3)))))
    ts = [timed(inner) / work.count for _ in range(reps)]
    del ws
    return float(np.median(ts))


def exhaustive(work, reps=5, configs=None):
    """Time every configuration; returns (best config, {key: ms})."""
    configs = configs or config_space()
    times = {config_key(c): time_config(work, c, reps) for c in configs}
    best = min(configs, key=lambda c: times[config_key(c)])
    return best, times


def record(params, level, count, cfg, ms, spread=1.0):
    log_n, num_q, dnum, num_p = params
    return {"log_n": log_n, "num_q": num_q, "dnum": dnum, "num_p": num_p, "level": level, "count": count,
            "spread": spread, **cfg, "ms": ms}


class TuneCache:
    """Best configuration per (device, parameters, level, count), as JSON."""

    def __init__(self, path):
        self.path = path
        self.data = json.load(open(path)) if path and os.path.exists(path) else {}

    @staticmethod
    def key(device, params, level, count):
        return f"{device}|{'/'.join(map(str, params))}|l{level}|c{count}"

    def get(self, device, params, level, count):
        return self.data.get(self.key(device, params, level, count))

    def put(self, device, params, level, count, cfg):
        self.data[self.key(device, params, level, count)] = cfg
        if self.path:
            tmp = self.path + ".tmp"
            json.dump(self.data, open(tmp, "w"), indent=1)
            os.replace(tmp, self.path)


def plan_params(plan):
    return (plan.log_n, plan.num_q, plan.dnum, plan.num_p)


def install(plan, level, count, cfg):
    """Put a tuned configuration in the live path: record it in the plan for
    calls of that shape and switch the plan's schedule to AUTO."""
    plan.set_tuned(level, count, cfg["schedule"], **config_fields(cfg))
    plan.configure("auto")


class Tuner:
    """The autotuner in the live path.  tune(plan, level, count) returns the
    configuration for that call shape: the cached choice; else, with a cost
    model, the fastest of the model's top-M configurations timed on the GPU;
    else (no model, or verify=True as the arbiter) every configuration timed.
    The choice is recorded in the plan (install) and in the cache."""

    def __init__(self, cache=None, model=None, top_m=3, reps=5, device="gpu0", verify=False):
        self.cache, self.model, self.top_m, self.reps = cache, model, top_m, reps
        self.device, self.verify = device, verify
        self.log = []  # per tuned shape: how it was decided and what was timed

    def tune(self, plan, level, count=1, levels=None, seed=0):
        params = plan_params(plan)
        if levels is not None:
            level, count = max(levels), len(levels)
        cfg = self.cache.get(self.device, params, level, count) if self.cache else None
        entry = {"params": list(params), "level": level, "count": count}
        if cfg is not None:
            entry["source"] = "cache"
        else:
            work = Workload(plan, level, count, seed=seed, levels=levels)
            if self.model is not None and not self.verify:
                from . import costmodel
                cfg, times = costmodel.pruned_search(self.model, work, self.top_m, self.reps)
                entry["source"] = f"model top-{self.top_m}, timed"
            else:
                cfg, times = exhaustive(work, self.reps)
                entry["source"] = "exhaustive"
            entry["timed_ms"] = times
            del work
            if self.cache:
                self.cache.put(self.device, params, level, count, cfg)
        entry["config"] = config_key(cfg)
        self.log.append(entry)
        install(plan, level, count, cfg)
        return cfg


def tune(plan, level, count=1, cache=None, device="gpu0", reps=5, model=None, top_m=3):
    """Tune `plan` for (level, count) and put the choice in its live path:
    the cached choice, else the model's top-M timed, else exhaustive."""
    return Tuner(cache, model, top_m, reps, device).tune(plan, level, count)


# ------------------------------------------------------------------ collection
def collect_grid(quick=False):
    """(log_n, num_q, dnum, levels, counts) points of the timing database:
    N in 2^14..2^17, up to 48 towers, dnum 1..6 (alpha <= 32)."""
    pts = []
    logs = (14, 15) if quick else (14, 15, 16, 17)
    towers = (8, 16) if quick else (8, 16, 24, 32, 40, 48)
    dnums = (1, 2, 3) if quick else (1, 2, 3, 4, 6)
    for log_n, nq, dn in itertools.product(logs, towers, dnums):
        alpha = -(-nq // dn)
        if alpha > 32 or dn > nq:
            continue
        levels = sorted({nq - 1, max(0, nq // 2 - 1)})
        counts = (1,) if quick else (1, 4)
        pts.append((log_n, nq, dn, levels, counts))
    return pts


def mixed_levels(nq, count, seed):
    """Levels of a mixed-level batch: l+1 uniform in [ceil(nq/3), nq]."""
    rng = np.random.default_rng(seed)
    return [int(t) - 1 for t in rng.integers(-(-nq // 3), nq + 1, count)]


def collect(out, quick=False, reps=5, log=print, mixed=16):
    """Time every configuration on every workload of the grid: single-level
    calls of 1 and 4 key switches per level, and (mixed > 0) one batch of
    `mixed` key switches at mixed levels per point."""
    import paper_2311_01598_amd as ks
    t0 = time.time()
    pts = collect_grid(quick)
    n = 0
    with open(out, "a") as f:
        for pi, (log_n, nq, dn, levels, counts) in enumerate(pts):
            plan = ks.Plan(log_n, nq, dn)
            params = (log_n, nq, dn, plan.num_p)
            works = [(level, count, None) for level in levels for count in counts]
            if mixed and not quick:
                works.append((None, None, mixed_levels(nq, mixed, 7000 + pi)))
            for level, count, lv in works:
                work = Workload(plan, level, count, seed=1000 * pi + (level or 0), levels=lv)
                for cfg in config_space():
                    ms = time_config(work, cfg, reps)
                    f.write(json.dumps(record(params, work.level, work.count, cfg, ms, round(work.spread, 4)))
                            + "\n")
                    n += 1
                del work
            f.flush()
            plan.close()
            log(f"[collect] {pi + 1}/{len(pts)} N=2^{log_n} towers={nq} dnum={dn}: {n} timings, "
                f"{time.time() - t0:.0f} s", flush=True)
    return n


def load_db(path):
    return [json.loads(l) for l in open(path) if l.strip()]


def group_workloads(rows):
    """{(log_n, num_q, dnum, num_p, level, count, spread): {config key: ms}}."""
    out = {}
    for r in rows:
        k = (r["log_n"], r["num_q"], r["dnum"], r["num_p"], r["level"], r["count"], r.get("spread", 1.0))
        out.setdefault(k, {})[config_key(r)] = r["ms"]
    return out


def report(rows, exp, commands=()):
    """Markdown summary of a timing database and a cost-model experiment."""
    import collections
    s = exp["summary"]
    g = group_workloads(rows)
    best = collections.Counter(min(t, key=t.get) for t in g.values())
    sp = []
    for t in g.values():
        mp = [v for k, v in t.items() if k.startswith("mp")]
        oc = [v for k, v in t.items() if k.startswith("oc")]
        if mp and oc:
            sp.append(min(mp) / min(oc))
    sp = np.array(sp)
    f = lambda d: f"mean {100 * d['mean']:.2f} %, p90 {100 * d['p90']:.2f} %, max {100 * d['max']:.2f} %"
    lines = ["# Autotuner timing database and cost-model regret (N = 2^14..2^17, up to 48 towers)", "",
             "Commands (one GPU, MI355X):", ""] + ["    " + c for c in commands] + [
        "", f"Database: {len(rows)} timings = {len(g)} workloads x {s['configs']} configurations; log N in 14..17,",
        "towers in {8,16,24,32,40,48}, dnum in {1,2,3,4,6} (alpha <= 32), two levels per point, 1 or 4",
        "ciphertexts per call, and one batch of 16 at mixed levels (l+1 uniform in [towers/3, towers]) per point;",
        "median of 3 timed runs after one warm-up.", "",
        f"Cost model: fp32 MLP {len(exp.get('features', [])) or 14} -> 64 -> 64 -> 1 (ReLU), target log(ms), trained on the",
        "GPU by ks_mlp_forward / ks_mlp_mse_grad / ks_mlp_backward / ks_mlp_adam (full batch, Adam).",
        f"Split by parameter point: {s['train_records']} training timings, {s['test_workloads']} held-out workloads;",
        f"final standardised training loss {s['final_train_loss']:.2e}.", "",
        "Top-1 regret on the held-out workloads (time of the chosen configuration / exhaustive best - 1):", "",
        "| method | timings per workload | regret |", "|---|---|---|",
        f"| exhaustive search (arbiter) | {s['configs']} | 0 |",
        f"| model pick (no timing) | 0 | {f(s['regret_model_pick'])} |",
        f"| model top-{s['top_m']}, timed | {s['top_m']} | {f(s['regret_pruned_top_m'])} |",
        f"| {s['top_m']} random configurations, timed | {s['top_m']} | {f(s['regret_random_top_m'])} |",
        f"| fixed default (oc/t2, the plan's starting configuration) | 0 | {f(s['regret_fixed_default'])} |", "",
        f"Best configuration per workload over the whole database: {dict(best)}.",
        f"Best OC over best MP configuration, per workload: median {np.median(sp):.2f}x, "
        f"min {sp.min():.2f}x, max {sp.max():.2f}x."]
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--out", required=True)
    c.add_argument("--quick", action="store_true")
    c.add_argument("--reps", type=int, default=5)
    e = sub.add_parser("experiment")
    e.add_argument("--db", required=True)
    e.add_argument("--out", required=True)
    e.add_argument("--top", type=int, default=3)
    e.add_argument("--seed", type=int, default=0)
    t = sub.add_parser("train")
    t.add_argument("--db", required=True)
    t.add_argument("--out", default=None, help="weights file (default: the package's data/costmodel.npz)")
    t.add_argument("--steps", type=int, default=3000)
    r = sub.add_parser("report")
    r.add_argument("--db", required=True)
    r.add_argument("--exp", required=True)
    r.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "collect":
        collect(a.out, a.quick, a.reps)
    elif a.cmd == "report":
        # the commands that produced the report's inputs, with this call's paths
        cmds = (f"python3 -u -m paper_2311_01598_amd.tune collect --out {a.db} --reps 3",
                f"python3 -u -m paper_2311_01598_amd.tune experiment --db {a.db} --out {a.exp}",
                f"python3 -m paper_2311_01598_amd.tune report --db {a.db} --exp {a.exp} --out {a.out}")
        open(a.out, "w").write(report(load_db(a.db), json.load(open(a.exp)), cmds))
    elif a.cmd == "train":
        from . import costmodel
        model, hist = costmodel.train(load_db(a.db), steps=a.steps)
        out = a.out or costmodel.WEIGHTS
        os.makedirs(os.path.dirname(out), exist_ok=True)
        model.save(out)
        print(json.dumps({"weights": out, "final_train_loss": hist[-1][1] if hist else None}), flush=True)
    else:
        from . import costmodel
        res = costmodel.experiment(load_db(a.db), top_m=a.top, seed=a.seed)
        res.pop("model")
        json.dump(res, open(a.out, "w"), indent=1)
        print(json.dumps(res["summary"]), flush=True)


if __name__ == "__main__":
    sys.exit(main())
