"""Progress of the persistent batch kernel's hand-out protocol (host model, no GPU).

`batch_persistent_kernel` (csrc/batched.hip) takes tiles in chunks from one
counter, in the schedule's order, runs a chunk's tiles in order, waits on the
groups a stage reads only when the stage changes, and publishes the
completions it holds for a group when the group changes, before any wait and
at the end of a chunk.  This model runs that loop for W workgroups on
generated schedules with the schedule builder's invariants:

  * tiles are numbered stage after stage;
  * a stage reads only groups whose tiles all belong to earlier stages;
  * tiles of one stage never read each other, and a group may span stages;

and interleaves the workgroups' steps at random (any workgroup may stall for
any time; a waiting workgroup only re-polls).  Every run must finish, with
every group's count equal to its tile count.  The same model with the
publish-before-wait rule removed must deadlock on some schedule, so the
check can tell the two apart.
"""
import numpy as np
import pytest


def make_schedule(rng, depths=6, max_stages=4, max_tiles=40):
    stages, groups = [], []  # stage: (tile0, ntiles, signal, [(group, need)]); groups: tile counts
    tile = 0
    done_before = []  # groups complete by the end of the previous depth
    for _ in range(depths):
        depth_groups = []
        for _ in range(int(rng.integers(1, max_stages + 1))):
            nt = int(rng.integers(1, max_tiles + 1))
            if depth_groups and rng.random() < 0.3:
                sig = depth_groups[int(rng.integers(0, len(depth_groups)))]  # a group spanning stages
            else:
                sig = len(groups)
                groups.append(0)
                depth_groups.append(sig)
            groups[sig] += nt
            waits = []
            if done_before:
                for g in rng.choice(done_before, size=min(len(done_before), int(rng.integers(0, 3))), replace=False):
                    waits.append(int(g))
            stages.append([tile, nt, sig, waits])
            tile += nt
        done_before = done_before + depth_groups
    for st in stages:
        st[3] = [(g, groups[g]) for g in st[3]]
    return stages, groups, tile


def stage_of(stages, g):
    lo, hi = 0, len(stages) - 1
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if stages[mid][0] <= g:
            lo = mid
        else:
            hi = mid - 1
    return lo


def run(stages, groups, total, W, chunk, rng, publish_before_wait=True, max_steps=200000):
    done = [0] * len(groups)
    nxt = 0
    wg = [dict(base=None, g=0, end=0, ready=-1, sig=-1, pend=0, fin=False) for _ in range(W)]

    def publish(s):
        if s["pend"]:
            done[s["sig"]] += s["pend"]
            s["pend"] = 0

    for _ in range(max_steps):
        live = [i for i in range(W) if not wg[i]["fin"]]
        if not live:
            return done
        progressed = False
        for i in rng.permutation(live):
            s = wg[i]
            if s["base"] is None:  # take a chunk
                if nxt >= total:
                    s["fin"] = True
                    progressed = True
                    break
                s["base"], s["g"], s["end"] = nxt, nxt, min(nxt + chunk, total)
                nxt += chunk
                progressed = True
                break
            st = stages[stage_of(stages, s["g"])]
            si = stage_of(stages, s["g"])
            if si != s["ready"]:
                if publish_before_wait:
                    publish(s)
                if not all(done[g] >= need for g, need in st[3]):
                    continue  # waiting: try another workgroup
                s["ready"] = si
            # run the tile, then count it for its group
            if s["sig"] != st[2]:
                publish(s)
            s["sig"] = st[2]
            s["pend"] += 1
            s["g"] += 1
            if s["g"] >= s["end"]:
                publish(s)
                s["base"] = None
            progressed = True
            break
        if not progressed:
            return None  # every live workgroup waits: deadlock
    raise AssertionError("model did not finish")


@pytest.mark.parametrize("seed", range(40))
def test_chunked_protocol_always_finishes(seed):
    rng = np.random.default_rng(seed)
    stages, groups, total = make_schedule(rng)
    for W, chunk in ((1, 1), (1, 32), (3, 8), (4, 32), (16, 32), (64, 32)):
        done = run(stages, groups, total, W, chunk, rng)
        assert done is not None, (seed, W, chunk)
        assert done == groups


def test_waiting_while_holding_completions_deadlocks():
    """Without publishing before a wait, a workgroup can hold the last completions of a group it (or
    another workgroup) then waits for."""
    found = False
    for seed in range(200):
        rng = np.random.default_rng(1000 + seed)
        stages, groups, total = make_schedule(rng)
        if run(stages, groups, total, 4, 32, rng, publish_before_wait=False) is None:
            found = True
            break
    assert found
