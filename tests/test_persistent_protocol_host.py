"""Host-only replay of the persistent batch launch's work-queue protocol on the
exact tables the library builds (ks_oc_work_list, no GPU).

The launch is switched off on the device.  These tests establish on the CPU
what its liveness argument needs from the tables alone:
- the segment table is phase-major then job-major, every segment starts where
  the previous one ends, and it covers every tile of every (phase, job);
- every dependency of a phase names an earlier phase, so the items an item
  waits for all have smaller indices (they were dequeued before it);
- a simulation with fewer resident groups than items, under adversarial
  (random, and oldest-last) completion orders, never reaches a state where
  no group can move while items remain: every wait is satisfiable.
"""
import ctypes

import numpy as np
import pytest

import paper_2311_01598_amd as ks

NPHASE = 8


def work_list(log_n, num_q, dnum, num_p, levels):
    lib = ks.lib()
    count = len(levels)
    U = ctypes.c_uint32
    tiles = (U * (count * NPHASE))()
    start, job, phase = (U * (count * NPHASE))(), (U * (count * NPHASE))(), (U * (count * NPHASE))()
    deps = (U * NPHASE)()
    total = U()
    params, _ = ks._params(log_n, num_q, dnum, num_p)
    st = lib.ks_oc_work_list(ctypes.byref(params), count, (U * count)(*levels), tiles, start, job, phase, deps,
                             ctypes.byref(total))
    assert st == ks.KS_OK, st
    return (np.array(tiles).reshape(count, NPHASE), np.array(start), np.array(job), np.array(phase),
            [int(d) for d in deps], int(total.value))


CASES = [
    (12, 4, 2, 2, [3, 0, 1, 2, 3]),
    (13, 8, 3, 3, [7, 3, 0, 5, 7, 1, 6, 2, 4, 7]),
    (16, 24, 3, 8, [23, 7, 15, 0, 11]),
    (14, 40, 16, 5, [39, 2, 17]),
    (17, 45, 3, 15, [44, 20]),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "n%d_l%d_d%d_k%d" % c[:4])
def test_tables_are_ordered_and_complete(case):
    tiles, start, job, phase, deps, total = work_list(*case)
    count = len(case[4])
    # phase-major, then job-major, contiguous
    assert list(phase) == [p for p in range(NPHASE) for _ in range(count)]
    assert list(job) == [j for _ in range(NPHASE) for j in range(count)]
    ends = start + np.array([tiles[j, p] for j, p in zip(job, phase)])
    assert start[0] == 0 and list(start[1:]) == list(ends[:-1]) and ends[-1] == total
    assert total == tiles.sum()
    # dependencies point to earlier phases only, and the first phase has none
    assert deps[0] == 0
    for p in range(NPHASE):
        assert deps[p] >> p == 0, (p, deps[p])
    # the phases the Output-Centric order needs (Sec. IV-C): ROW_Q after both
    # conversions, the ModDown column pass after the special-tower rows
    assert deps[7] == (1 << 6) | (1 << 4) and deps[5] == 1 << 3 and deps[2] == 1 << 1 and deps[4] == 1 << 1


def simulate(tiles, start, job, phase, deps, total, groups, rng, policy):
    """Work-queue protocol with `groups` resident workgroups.  A group with
    no item dequeues the next one; a group holding an item may finish it once
    every phase its phase depends on is complete for its job.  `policy`
    picks which movable group moves next.  Returns the number of moves."""
    seg_of = np.repeat(np.arange(len(start)), [tiles[j, p] for j, p in zip(job, phase)])
    done = np.zeros_like(tiles)
    head, finished, moves = 0, 0, 0
    held = [None] * groups
    while finished < total:
        movable = []
        for g in range(groups):
            if held[g] is None:
                if head < total:
                    movable.append(g)
            else:
                s = seg_of[held[g]]
                j, p = job[s], phase[s]
                if all(done[j, q] >= tiles[j, q] for q in range(NPHASE) if (deps[p] >> q) & 1):
                    movable.append(g)
        assert movable, f"no group can move: head={head} finished={finished}/{total} held={held}"
        if policy == "random":
            g = movable[rng.integers(len(movable))]
        else:  # finish the newest held item first, dequeue only when forced
            holding = [g for g in movable if held[g] is not None]
            g = max(holding, key=lambda g: held[g]) if holding else movable[0]
        if held[g] is None:
            held[g] = head
            head += 1
        else:
            s = seg_of[held[g]]
            done[job[s], phase[s]] += 1
            finished += 1
            held[g] = None
        moves += 1
    assert (done == tiles).all()
    return moves


@pytest.mark.parametrize("case", CASES[:3] + [(13, 10, 5, 3, [1, 3, 5, 7, 9, 0])], ids=lambda c: "n%d_l%d" % c[:2])
@pytest.mark.parametrize("groups", [1, 3, 17, 256])
@pytest.mark.parametrize("policy", ["random", "newest_first"])
def test_every_wait_is_satisfiable(case, groups, policy):
    tiles, start, job, phase, deps, total = work_list(*case)
    rng = np.random.default_rng(groups * 7 + len(case[4]))
    groups = min(groups, total - 1)  # fewer resident groups than items
    assert simulate(tiles, start, job, phase, deps, total, groups, rng, policy) == 2 * total
