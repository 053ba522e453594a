"""The grouped kernel's work-queue protocol, modelled on the CPU.

A step-by-step model of what thread 0 of every work-group does in
grouped_kernel (csrc/grouped.hip): draw a ticket from its XCD's queue
(atomic add), resolve it against the queue's length, move on to the next
queue when one is exhausted, draw the next tile's ticket when a tile starts
and resolve it when the tile ends, and count itself out; the last work-group
out zeroes the counters.  Every atomic is one step, and the steps of the
work-groups are interleaved in random orders.  Whatever the order, every
tile must be taken exactly once, every work-group must stop after at most
(its tiles + queues) draws, and the counters must be zero afterwards, so
that the next launch starts clean.
"""
import random

import numpy as np
import pytest

NO_TILE = None


def run_launch(qlens, grid, rng, counters):
    """One launch over queues of the given lengths (tiles numbered by queue
    offset), `grid` work-groups; returns the tiles each work-group took."""
    nq = len(qlens)
    qstart = np.concatenate([[0], np.cumsum(qlens)]).astype(int)

    def wg(w):
        """Generator: yields before every atomic; returns its tiles."""
        q, left = w % nq, nq
        taken, draws = [], 0

        def resolve(ticket):
            nonlocal q, left, draws
            while True:
                if ticket < qlens[q]:
                    return qstart[q] + ticket
                q = 0 if q + 1 == nq else q + 1
                left -= 1
                if left == 0:
                    return NO_TILE
                yield
                ticket = counters[q]
                counters[q] += 1
                draws += 1

        yield
        ticket = counters[q]
        counters[q] += 1
        draws += 1
        t = yield from resolve(ticket)
        while t is not NO_TILE:
            yield
            ticket = counters[q]          # drawn when the tile starts
            counters[q] += 1
            draws += 1
            taken.append(t)               # the tile runs
            t = yield from resolve(ticket)
        assert draws <= len(taken) + nq
        yield
        done = counters[nq]
        counters[nq] += 1
        if done == grid - 1:
            for i in range(nq + 1):
                counters[i] = 0
        return taken

    gens = {w: wg(w) for w in range(grid)}
    results = {}
    while gens:
        w = rng.choice(list(gens))
        try:
            next(gens[w])
        except StopIteration as stop:
            results[w] = stop.value
            del gens[w]
    return results


@pytest.mark.parametrize("seed", range(40))
def test_every_tile_once_and_counters_reset(seed):
    rng = random.Random(seed)
    nq = rng.randint(1, 8)
    qlens = [rng.choice([0, 1, 2, 5, 17, 60]) for _ in range(nq)]
    grid = rng.randint(max(1, nq), 70) if sum(qlens) else rng.randint(nq, 9)
    counters = [0] * (nq + 1)
    for launch in range(3):               # back-to-back launches share the counters
        res = run_launch(qlens, grid, rng, counters)
        tiles = sorted(t for v in res.values() for t in v)
        assert tiles == list(range(sum(qlens))), (seed, launch)
        assert counters == [0] * (nq + 1), (seed, launch)


def test_a_work_group_helps_other_queues():
    """One work-group per queue of eight, all tiles in queue 3: the others
    find their own queues empty and take queue 3's tiles."""
    rng = random.Random(1)
    counters = [0] * 9
    res = run_launch([0, 0, 0, 40, 0, 0, 0, 0], 8, rng, counters)
    assert sorted(t for v in res.values() for t in v) == list(range(40))
    assert sum(1 for v in res.values() if v) > 1
