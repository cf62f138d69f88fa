"""Host-side models of the compressor's tile protocols, run under adversarial
interleavings on the CPU.

1. Plain launches: a persistent grid of workgroups claims tiles from one counter,
   publishes each tile's output size (an aggregate) at once, may park a finished tile
   and place it only after claiming and finishing the next one, and finds a tile's
   output offset by a look-back over the status words of its predecessors (the
   single-pass scan with decoupled look-back of Merrill and Garland): one wave reads
   the W nearest unvisited words per round; the nearest word holding an inclusive
   prefix ends the walk; a round in which a nearer word is still empty is read again.
   Each workgroup here is a generator that yields at every shared-memory access, so a
   random scheduler interleaves them at that granularity; a status word goes only
   from empty to aggregate to inclusive prefix.

2. Binned launches: the bin plan (tiles per bin from the bin sizes and lines per
   tile, first tile of every bin) and the ticket -> (bin, first line, line count)
   mapping of a launch covering a run of bins: every line is taken exactly once.

These models restate the protocols as the kernels implement them; they check the
protocols' logic (offsets equal the exclusive scan of the tile sizes; every
schedule ends), not the device code itself.
"""
import random

import pytest

EMPTY, AGG, INC = 0, 1, 2


class Shared:
    def __init__(self, ntiles):
        self.ticket = 0
        self.status = [(EMPTY, 0)] * ntiles
        self.base = [None] * ntiles


def lookback(sh, t, agg, window):
    """Generator: the walk of tile t (whose aggregate is published); returns the
    exclusive prefix and publishes t's inclusive prefix."""
    if t == 0:
        return 0
    excl = 0
    top = t - 1
    while True:
        words = []
        for lane in range(window):
            j = top - lane
            words.append(sh.status[j] if j >= 0 else (INC, 0))
            yield
        first = next((i for i, (f, _) in enumerate(words) if f == INC), window)
        if any(f == EMPTY for f, _ in words[:first + 1]):
            continue  # a nearer predecessor has not published yet: read the round again
        excl += sum(v for f, v in words[:first + 1])
        if first < window:
            break
        top -= window
    sh.status[t] = (INC, excl + agg)
    yield
    return excl


def workgroup(sh, sizes, parks, window):
    """Generator: one workgroup of a plain launch."""
    pend = None
    while True:
        t = sh.ticket
        sh.ticket += 1  # one atomic add
        yield
        have = t < len(sizes)
        if have:
            sh.status[t] = ((INC if t == 0 else AGG), sizes[t])
            yield
        if pend is not None:
            pt = pend
            sh.base[pt] = yield from lookback(sh, pt, sizes[pt], window)
            pend = None
        if not have:
            return
        if parks[t]:
            pend = t  # placed after the next claim
        else:
            sh.base[t] = yield from lookback(sh, t, sizes[t], window)


def run_schedule(sizes, parks, nwg, window, rng, max_steps=200000):
    sh = Shared(len(sizes))
    live = [workgroup(sh, sizes, parks, window) for _ in range(nwg)]
    steps = 0
    while live:
        g = rng.choice(live)
        try:
            next(g)
        except StopIteration:
            live.remove(g)
        steps += 1
        assert steps < max_steps, "the schedule did not end (a walk waits on a word never published)"
    return sh


@pytest.mark.parametrize("seed", range(300))
def test_lookback_with_parking_gives_exclusive_scan(seed):
    rng = random.Random(seed)
    ntiles = rng.randint(1, 40)
    sizes = [rng.randint(0, 1000) for _ in range(ntiles)]
    parks = [rng.random() < 0.6 for _ in range(ntiles)]
    nwg = rng.randint(1, 8)
    window = rng.choice([1, 2, 3, 64])
    sh = run_schedule(sizes, parks, nwg, window, rng)
    run = 0
    for t in range(ntiles):
        assert sh.base[t] == run, (t, sh.base[t], run)
        run += sizes[t]
        assert sh.status[t] == (INC, run)
    assert sh.ticket == ntiles + nwg  # every workgroup claimed once past the last tile


def test_every_tile_parked_and_one_workgroup():
    # a single workgroup parks every tile: tile t is placed after tile t + 1 is claimed
    rng = random.Random(1)
    sizes = [5, 0, 7, 1, 9]
    sh = run_schedule(sizes, [True] * 5, 1, 2, rng)
    assert sh.base == [0, 5, 5, 12, 13]


def test_model_catches_a_walk_that_skips_empty_words():
    # the check above is not vacuous: a walk that treats an empty word as a zero
    # aggregate gives wrong offsets under some schedule
    def bad_lookback(sh, t, agg, window):
        if t == 0:
            return 0
        excl = 0
        for j in range(t - 1, -1, -1):
            f, v = sh.status[j]
            yield
            excl += v
            if f == INC:
                break
        sh.status[t] = (INC, excl + agg)
        yield
        return excl

    global lookback
    good = lookback
    lookback = bad_lookback
    try:
        wrong = 0
        for seed in range(40):
            rng = random.Random(seed)
            sizes = [rng.randint(1, 100) for _ in range(12)]
            sh = run_schedule(sizes, [False] * 12, 4, 1, rng)
            run = 0
            for t in range(12):
                wrong += sh.base[t] != run
                run += sizes[t]
        assert wrong > 0
    finally:
        lookback = good


# ---- binned launches: plan and ticket mapping

def bin_plan(counts, lpt):
    """Bin starts in the id order and the first tile of every bin (processing order)."""
    start, first, s, tiles = [], [], 0, 0
    for c, p in zip(counts, lpt):
        start.append(s)
        first.append(tiles)
        s += c
        tiles += (c + p - 1) // p
    first.append(tiles)
    return start, first


def launch_tiles(counts, lpt, lo, hi):
    """The (first line, line count) of every ticket of a launch over bins [lo, hi)."""
    start, first = bin_plan(counts, lpt)
    out = []
    ticket = 0
    while True:
        t = first[lo] + ticket
        ticket += 1
        if t >= first[hi]:
            return out
        b = lo
        while t >= first[b + 1]:
            b += 1
        k0 = start[b] + (t - first[b]) * lpt[b]
        nl = min(lpt[b], start[b] + counts[b] - k0)
        assert nl >= 1
        out.append((b, k0, nl))


@pytest.mark.parametrize("seed", range(40))
def test_binned_launches_take_every_line_once(seed):
    rng = random.Random(seed)
    nb = rng.randint(1, 8)
    counts = [rng.choice([0, 1, rng.randint(0, 5000)]) for _ in range(nb)]
    lpt = [rng.choice([32, 64, 100, 128, 256]) for _ in range(nb)]
    # launches: runs of bins sharing a layout
    layout = [rng.randint(0, 2) for _ in range(nb)]
    seen = [0] * sum(counts)
    b = 0
    while b < nb:
        e = b + 1
        while e < nb and layout[e] == layout[b]:
            e += 1
        for bb, k0, nl in launch_tiles(counts, lpt, b, e):
            assert b <= bb < e
            start = bin_plan(counts, lpt)[0][bb]
            assert start <= k0 and k0 + nl <= start + counts[bb]  # inside its own bin
            for k in range(k0, k0 + nl):
                seen[k] += 1
        b = e
    assert all(s == 1 for s in seen)
