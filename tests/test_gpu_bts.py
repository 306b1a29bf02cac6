"""GPU parity at the parameter sets of Table III: BTS1 / BTS2 / BTS3
(N = 2^17; 28+28 towers with dnum 1, 40+20 with dnum 2, 45+15 with dnum 3)
and ARK / DPRIVE (N = 2^16; 24+6 towers with dnum 4, 26+7 with dnum 3:
alpha 9, a partial last digit and K != alpha), 30-bit towers, and the
serving workload's largest plan (N = 2^17, 48 towers, dnum 3, K = 16, two
targets per conversion tile), at full size with every output element
compared against the oracle.  These stress the 2^17 two-pass transform
(512 x 256), conversions with more than 16 source towers (alpha 28 and 20,
and K = 28 / 20 for ModDown, accumulated in chunks of 16 products), and
the single-digit case where ModUp has no Q target.  BTS3 also runs with a
compressed key; BTS2, ARK and DPRIVE also with the Max-Parallel and
Digit-Centric schedules.  BTS3's modulus in 30-bit towers (90 + 30, 120
towers, alpha = K = 30) runs the OC order.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import core
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BTS = {"bts1": (17, 28, 1, 28), "bts2": (17, 40, 2, 20), "bts3": (17, 45, 3, 15),
       # the serving workload's largest plan: N = 2^17, 48 towers, dnum 3, K = alpha = 16
       "serve17": (17, 48, 3, 0),
       # BTS3's modulus (45 + 15 towers of 60 bits) in 30-bit towers: 90 + 30,
       # alpha = K = 30, 120 towers (the bench times it beside the 64-bit path)
       "bts3_30bit": (17, 90, 3, 30),
       "ark": (16, 24, 4, 6), "dprive": (16, 26, 3, 7)}


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_01598_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def host(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("name", ["bts1", "bts2", "bts3", "serve17", "bts3_30bit", "ark", "dprive"])
def test_bts_full_size(ks, name):
    log_n, num_q, dnum, num_p = BTS[name]
    p = oracle.Params(log_n, num_q, dnum, num_p)
    mods = oracle.moduli(p)
    level = num_q - 1
    evk = synth.uniform_evk(mods, dnum, p.n, synth.seed_for(30, num_q))
    a_seed = synth.seed_for(30, 500 + num_q)
    if name == "bts3":  # the a halves regenerated from a seed
        evk[:, 1] = core.seeded_a(p, mods, a_seed)[:, 1]
    d = synth.uniform_limbs(mods[:num_q], p.n, synth.seed_for(30, 100 + num_q))
    print(f"[{name}] oracle", flush=True)
    want = oracle.keyswitch(p, mods, level, evk, d)
    plan = ks.Plan(log_n, num_q, dnum, num_p)
    runs = ([("oc", None)] + ([("mp", None), ("dc", None)] if name == "bts2" else [])
            + ([("oc", "seeded")] if name == "bts3" else []))
    if name == "serve17":  # the serving loop's configuration: two targets per conversion tile
        runs = [("oc2", None)]
    if name in ("ark", "dprive"):
        runs = [("oc", None), ("mp", None), ("dc", None)]
    for sched, kind in runs:
        print(f"[{name}] {sched} {kind or ''}", flush=True)
        sys.stdout.flush()
        if sched == "oc2":
            plan.configure("oc", tile_towers=2)
        else:
            plan.configure(sched)
        if kind == "seeded":
            out = plan.keyswitch_seeded(dev(np.ascontiguousarray(evk[:, 0])), a_seed, level, dev(d))
        else:
            out = plan.keyswitch(dev(evk), level, dev(d))
        torch.cuda.synchronize()
        bad = np.argwhere(host(out) != want)
        assert bad.size == 0, (name, sched, kind, bad[:5], len(bad))
    plan.close()
