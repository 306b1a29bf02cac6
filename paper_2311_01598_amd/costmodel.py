"""Learned cost model of the autotuner: an fp32 MLP (16 features -> 64 -> 64
-> 1, ReLU) that predicts log(milliseconds per key switch) of a
configuration, trained on the GPU by the library's own kernels
(ks_mlp_forward / ks_mlp_mse_grad / ks_mlp_backward / ks_mlp_adam).

Pruned search: rank every configuration by predicted time and time only the
top M; exhaustive search (tune.exhaustive) stays as fallback and arbiter.
`default_model()` loads the weights trained on the timing database of this
GPU (data/costmodel.npz, written by `tune train`), which the live tuner
uses to prune.
"""
import json
import math
import os

import numpy as np

from . import tune

FEATURES = ("log_n", "towers", "dnum", "alpha", "num_p", "ndig", "log2_count", "spread", "is_mp", "is_dc",
            "is_oc", "tile_towers", "log2_col", "log2_row", "split", "order_desc")
HIDDEN = 64
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "costmodel.npz")


def features(log_n, num_q, dnum, num_p, level, count, cfg, spread=1.0):
    """spread: mean over the call's jobs of l+1, divided by the largest l+1
    (1 for a single level)."""
    alpha = -(-num_q // dnum)
    towers = level + 1
    ndig = -(-towers // alpha)
    s = cfg["schedule"]
    return [log_n, towers, dnum, alpha, num_p, ndig, math.log2(count), spread, s == "mp", s == "dc", s == "oc",
            cfg["tile_towers"], math.log2(cfg["col_width"]), math.log2(cfg["row_block"]),
            cfg.get("batch_mode", 1) == 3, cfg.get("batch_order", 1) == 2]


def record_features(r):
    return features(r["log_n"], r["num_q"], r["dnum"], r["num_p"], r["level"], r["count"], r, r.get("spread", 1.0))


class CostModel:
    """MLP parameters live on the GPU; inputs are standardised features."""

    def __init__(self, n_features=len(FEATURES), hidden=HIDDEN, seed=0):
        import torch

        import paper_2311_01598_amd as ks
        self.ks, self.torch = ks, torch
        self.F, self.H = n_features, hidden
        self.P = ks.ks_mlp_param_count(self.F, self.H)
        rng = np.random.default_rng(seed)
        F, H = self.F, self.H
        p = np.concatenate([rng.normal(0, math.sqrt(2 / F), F * H), np.zeros(H),
                            rng.normal(0, math.sqrt(2 / H), H * H), np.zeros(H),
                            rng.normal(0, math.sqrt(1 / H), H), [0.0]]).astype(np.float32)
        self.params = torch.from_numpy(p).cuda()
        self.mu = np.zeros(F)
        self.sd = np.ones(F)
        self.y_mu, self.y_sd = 0.0, 1.0

    def _x(self, X):
        X = (np.asarray(X, np.float64) - self.mu) / self.sd
        return self.torch.from_numpy(X.astype(np.float32)).cuda().contiguous()

    def fit(self, X, y, steps=3000, lr=3e-3, log_every=0):
        torch, ks = self.torch, self.ks
        X = np.asarray(X, np.float64)
        y = np.asarray(y, np.float64)
        self.mu = X.mean(0)
        self.sd = np.where(X.std(0) > 0, X.std(0), 1.0)
        self.y_mu, self.y_sd = float(y.mean()), float(y.std() or 1.0)
        B, F, H, P = X.shape[0], self.F, self.H, self.P
        Xd = self._x(X)
        T = torch.from_numpy(((y - self.y_mu) / self.y_sd).astype(np.float32)).cuda()
        Y = torch.empty(B, device="cuda")
        dY = torch.empty(B, device="cuda")
        loss = torch.empty(1, device="cuda")
        act = torch.empty(2 * B * H, device="cuda")
        scratch = torch.empty(2 * B * H, device="cuda")
        grads = torch.empty(P, device="cuda")
        m = torch.zeros(P, device="cuda")
        v = torch.zeros(P, device="cuda")
        hist = []
        for step in range(1, steps + 1):
            ks.ks_mlp_forward(F, H, B, self.params, Xd, Y, act)
            ks.ks_mlp_mse_grad(B, Y, T, dY, loss)
            ks.ks_mlp_backward(F, H, B, self.params, Xd, act, dY, grads, scratch)
            ks.ks_mlp_adam(P, self.params, grads, m, v, lr, 0.9, 0.999, 1e-8, step)
            if log_every and step % log_every == 0:
                hist.append((step, float(loss.item())))
        torch.cuda.synchronize()
        return hist

    def predict(self, X):
        torch, ks = self.torch, self.ks
        X = np.asarray(X, np.float64)
        B = X.shape[0]
        Y = torch.empty(B, device="cuda")
        act = torch.empty(2 * B * self.H, device="cuda")
        ks.ks_mlp_forward(self.F, self.H, B, self.params, self._x(X), Y, act)
        return Y.cpu().numpy().astype(np.float64) * self.y_sd + self.y_mu

    def rank(self, params, level, count, configs=None, spread=1.0):
        """Configurations sorted by predicted time (best first)."""
        configs = configs or tune.config_space()
        log_n, num_q, dnum, num_p = params
        pred = self.predict([features(log_n, num_q, dnum, num_p, level, count, c, spread) for c in configs])
        return [configs[i] for i in np.argsort(pred)]

    def save(self, path):
        np.savez(path, params=self.params.cpu().numpy(), mu=self.mu, sd=self.sd, y=[self.y_mu, self.y_sd],
                 shape=[self.F, self.H])

    @classmethod
    def load(cls, path):
        z = np.load(path, allow_pickle=False)
        m = cls(int(z["shape"][0]), int(z["shape"][1]))
        m.params = m.torch.from_numpy(z["params"].astype(np.float32)).cuda()
        m.mu, m.sd = z["mu"], z["sd"]
        m.y_mu, m.y_sd = float(z["y"][0]), float(z["y"][1])
        return m


def default_model():
    """The cost model trained on this GPU's timing database, or None when no
    weights are present (the tuner then times every configuration)."""
    return CostModel.load(WEIGHTS) if os.path.exists(WEIGHTS) else None


def pruned_search(model, work, top_m=3, reps=5):
    """Time only the model's top-M configurations; returns (best, timed)."""
    params = (work.plan.log_n, work.plan.num_q, work.plan.dnum, work.plan.num_p)
    cands = model.rank(params, work.level, work.count, spread=work.spread)[:top_m]
    times = {tune.config_key(c): tune.time_config(work, c, reps) for c in cands}
    best = min(cands, key=lambda c: times[tune.config_key(c)])
    return best, times


def train(rows, steps=3000, seed=0):
    """The model trained on every timing of a database (for the live tuner)."""
    model = CostModel(seed=seed)
    hist = model.fit([record_features(r) for r in rows], [math.log(r["ms"]) for r in rows], steps=steps,
                     log_every=max(1, steps // 10))
    return model, hist


def experiment(rows, top_m=3, seed=0, steps=3000, holdout=0.2):
    """Train on 80% of the parameter points of a timing database and score
    the held-out workloads: top-1 regret of the model's pick and of the
    pruned search (top-M timed) against exhaustive search, next to a random
    choice of M configurations and a fixed default configuration."""
    groups = tune.group_workloads(rows)
    points = sorted({k[:4] for k in groups})
    rng = np.random.default_rng(seed)
    rng.shuffle(points)
    n_test = max(1, int(round(holdout * len(points))))
    test_pts = set(points[:n_test])
    cfgs = tune.config_space()
    keys = [tune.config_key(c) for c in cfgs]
    Xtr, ytr = [], []
    for r in rows:
        if (r["log_n"], r["num_q"], r["dnum"], r["num_p"]) not in test_pts:
            Xtr.append(record_features(r))
            ytr.append(math.log(r["ms"]))
    model = CostModel(seed=seed)
    hist = model.fit(Xtr, ytr, steps=steps, log_every=max(1, steps // 10))
    reg_pick, reg_pruned, reg_rand, reg_default = [], [], [], []
    per = []
    # the plan's starting configuration (ks_plan_create)
    default = tune.config_key({"schedule": "oc", "tile_towers": 2, "col_width": 16, "row_block": 8, "batch_mode": 1})
    for k, times in groups.items():
        if k[:4] not in test_pts or len(times) < len(cfgs):
            continue
        best = min(times.values())
        pred = model.predict([features(*k[:4], k[4], k[5], c, k[6]) for c in cfgs])
        order = [keys[i] for i in np.argsort(pred)]
        pick = times[order[0]]
        pruned = min(times[x] for x in order[:top_m])
        rand = np.mean([min(times[x] for x in rng.choice(keys, top_m, replace=False)) for _ in range(20)])
        reg_pick.append(pick / best - 1)
        reg_pruned.append(pruned / best - 1)
        reg_rand.append(rand / best - 1)
        reg_default.append(times[default] / best - 1)
        per.append({"workload": list(k), "best_ms": best, "pick": order[0], "pick_ms": pick, "pruned_ms": pruned})

    def stats(v):
        v = np.asarray(v)
        return {"mean": float(v.mean()), "p90": float(np.quantile(v, 0.9)), "max": float(v.max())}
    summary = {
        "train_records": len(Xtr), "test_workloads": len(reg_pick), "configs": len(cfgs), "top_m": top_m,
        "regret_model_pick": stats(reg_pick), "regret_pruned_top_m": stats(reg_pruned),
        "regret_random_top_m": stats(reg_rand), "regret_fixed_default": stats(reg_default),
        "timings_per_workload": {"exhaustive": len(cfgs), "pruned": top_m},
        "final_train_loss": hist[-1][1] if hist else None,
    }
    return {"summary": summary, "features": list(FEATURES), "loss_history": hist, "per_workload": per,
            "model": model}
