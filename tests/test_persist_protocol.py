"""A model of the persistent kernel's task-queue protocol (k_persist in
paper_1303_4538_amd/csrc/sip_kernels.hip), run on the CPU under random
interleavings of its workgroups: every workgroup takes the next ticket,
waits until the ticket's task is published (or leaves when no job is left
and the ticket lies beyond every reserved one), works the tile, and the
workgroup that finishes a job's sweep publishes the job's next sweep --
either whole, in the job's topological tile order, or (dataflow) as its
first tile, each later tile being published by the workgroup that takes its
last upstream tile.  A tile finishes only after the tiles it depends on (W
and S in a forward sweep, E and N backward) have finished, as the sweeps'
face-record waits enforce.

Checked for both publications, with fewer workgroups than tiles: no
deadlock (some workgroup can always move until all have left), every tile
of every sweep taken exactly once, every job runs all its sweeps, the queue
never holds more unconsumed tasks than its capacity (the tiles of all jobs),
and under dataflow publication a tile's task is published only after all of
its upstream tiles were taken.
"""
import random

import pytest


def upstream(nti, ntj, tile, kind):
    ti, tj = tile % nti, tile // nti
    d = -1 if kind == 0 else 1
    out = []
    for di, dj in ((d, 0), (0, d)):
        i, j = ti + di, tj + dj
        if 0 <= i < nti and 0 <= j < ntj:
            out.append(j * nti + i)
    return out


def downstream(nti, ntj, tile, kind):
    return upstream(nti, ntj, tile, 1 - kind)


def topo(nti, ntj, kind):
    order = sorted(range(nti * ntj), key=lambda t: (t % nti + t // nti, t))
    return order if kind == 0 else order[::-1]


def run(jobs, workers, dataflow, seed):
    """jobs: list of (nti, ntj, sweeps).  Returns the event log; raises on a
    broken property."""
    rng = random.Random(seed)
    cap = sum(a * b for a, b, _ in jobs) + 8
    slots = {}                      # ticket -> (job, kind, tile)
    head = alloc = 0
    active = len(jobs)
    sweep = [0] * len(jobs)         # sweeps published so far, per job
    done_in_sweep = [0] * len(jobs)
    finished = [set() for _ in jobs]   # tiles finished in the current sweep
    taken = {}                      # (job, sweep, tile) -> times taken
    dep = {}                        # (job, kind, tile) -> upstream tiles taken
    taken_now = [set() for _ in jobs]

    def publish(job, kind, tile):
        nonlocal alloc
        assert len(slots) < cap, "queue capacity exceeded"
        if dataflow:   # its upstream tiles in this sweep were all taken
            nti, ntj, _ = jobs[job]
            assert all(u in taken_now[job] for u in upstream(nti, ntj, tile, kind))
        slots[alloc] = (job, kind, tile)
        alloc += 1

    def publish_sweep(job):
        nti, ntj, _ = jobs[job]
        kind = sweep[job] % 2
        sweep[job] += 1
        finished[job].clear()
        taken_now[job].clear()
        done_in_sweep[job] = 0
        if dataflow:
            publish(job, kind, topo(nti, ntj, kind)[0])
        else:
            for t in topo(nti, ntj, kind):
                publish(job, kind, t)

    for j in range(len(jobs)):
        publish_sweep(j)
    # worker state: ('take', ticket or None) | ('work', job, kind, tile) | ('gone',)
    state = [("take", None)] * workers
    moves = 0
    while True:
        movable = []
        for w, st in enumerate(state):
            if st[0] == "take":
                t = st[1]
                if t is None or t in slots or (active == 0 and t >= alloc):
                    movable.append(w)
            elif st[0] == "work":
                _, job, kind, tile = st
                nti, ntj, _ = jobs[job]
                if all(u in finished[job] for u in upstream(nti, ntj, tile, kind)):
                    movable.append(w)
        if not movable:
            assert all(st[0] == "gone" for st in state), f"deadlock: {state}"
            break
        w = rng.choice(movable)
        moves += 1
        st = state[w]
        if st[0] == "take":
            if st[1] is None:
                state[w] = ("take", head)
                head += 1
                continue
            t = st[1]
            if t in slots:
                job, kind, tile = slots.pop(t)
                key = (job, sweep[job] - 1, tile)
                taken[key] = taken.get(key, 0) + 1
                taken_now[job].add(tile)
                if dataflow:   # count this tile for its downstream neighbours
                    nti, ntj, _ = jobs[job]
                    dep[(job, kind, tile)] = 0
                    for d in downstream(nti, ntj, tile, kind):
                        dep[(job, kind, d)] = dep.get((job, kind, d), 0) + 1
                        if dep[(job, kind, d)] == len(upstream(nti, ntj, d, kind)):
                            publish(job, kind, d)
                state[w] = ("work", job, kind, tile)
            else:
                state[w] = ("gone",)
        else:
            _, job, kind, tile = st
            nti, ntj, sweeps = jobs[job]
            finished[job].add(tile)
            done_in_sweep[job] += 1
            if done_in_sweep[job] == nti * ntj:   # this workgroup runs the finaliser
                if sweep[job] < sweeps:
                    publish_sweep(job)
                else:
                    active -= 1
            state[w] = ("take", None)
    for j, (nti, ntj, sweeps) in enumerate(jobs):
        assert sweep[j] == sweeps
        for s in range(sweeps):
            for t in range(nti * ntj):
                assert taken.get((j, s, t)) == 1, (j, s, t)
    assert not slots
    return moves


JOBS = [[(3, 2, 4)], [(4, 4, 3), (1, 1, 5), (2, 5, 2)], [(5, 3, 2), (3, 5, 3), (2, 2, 4), (1, 3, 1)]]


@pytest.mark.parametrize("dataflow", [True, False])
@pytest.mark.parametrize("jobs", JOBS)
@pytest.mark.parametrize("workers", [1, 2, 5, 16])
def test_queue_protocol_under_random_interleavings(dataflow, jobs, workers):
    for seed in range(30):
        run(jobs, workers, dataflow, seed)


def test_the_model_detects_a_lost_publication():
    """The same model with the last upstream tile never counted (a dataflow
    publication lost) deadlocks, so the checks above are not vacuous."""
    orig = downstream

    def lossy(nti, ntj, tile, kind):
        out = orig(nti, ntj, tile, kind)
        return out[:-1] if tile == 0 and kind == 0 else out

    globals()["downstream"] = lossy
    try:
        with pytest.raises(AssertionError, match="deadlock"):
            run([(3, 3, 2)], 4, True, 0)
    finally:
        globals()["downstream"] = orig
