"""A model of the walk's hand-off protocol (the drain phase of the tail
build), run under many random interleavings on the CPU.

Each wave is a generator that yields at every access to the shared words, in
the order the kernel makes them: the live-wave count, the records reserved and
taken (compare-and-swap on both), and each record's ready flag, which its
writer sets after the record and before it leaves.  The scheduler picks a
random wave at every yield, so waves stall at any point.  Whatever the
interleaving, every photon must end exactly once, every wave must exit, and
no record may be left untaken.  The model checks the protocol's logic; the
GPU tests check the kernel against the plain walk bit for bit."""
import random

import pytest


class Shared:
    def __init__(self):
        self.alive = 0
        self.reserved = 0
        self.claimed = 0
        self.records = {}          # index -> photon (remaining steps)
        self.flags = set()
        self.ended = 0             # photons that finished
        self.stays = 0             # last waves that found records left and stayed


def wave(sh, photons, regroup, refill_min, floor, lane_count=64, steps_per_round=3):
    """One wave: starts with `photons` (remaining step counts) in flight."""
    live = list(photons)
    sh.alive += 1
    yield
    handed = False
    wait = 0
    while True:
        dead = lane_count - len(live)
        # take over listed photons
        if regroup and dead > 0 and (dead == lane_count or dead >= refill_min):
            if wait > 0 and dead != lane_count:
                wait -= 1
            else:
                take, base = 0, 0
                h = sh.claimed
                yield
                for _ in range(4):
                    r = sh.reserved
                    yield
                    if r <= h:
                        break
                    n = min(r - h, dead)
                    if sh.claimed == h:            # compare-and-swap
                        sh.claimed = h + n
                        take, base = n, h
                        yield
                        break
                    h = sh.claimed
                    yield
                if take == 0:
                    wait = 4
                else:
                    for j in range(base, base + take):
                        while j not in sh.flags:   # the writer is between reserving and flagging
                            yield
                        live.append(sh.records[j])
                        yield
        if not live:
            # leave: the wave that takes the count to zero looks at the list once more
            old = sh.alive
            sh.alive -= 1
            yield
            if old == 1:
                c, r = sh.claimed, sh.reserved
                yield
                if c < r:
                    sh.alive += 1
                    sh.stays += 1
                    yield
                    continue
            return
        # hand the few photons in flight to other waves and leave
        if regroup and not handed and len(live) <= regroup:
            aw = sh.alive
            yield
            if aw <= floor:
                handed = True          # the count only falls: never try again
            else:
                r, h = sh.reserved, sh.claimed
                yield
                if r - h < 64 and sh.reserved == r:     # compare-and-swap
                    sh.reserved = r + len(live)
                    yield
                    for i, p in enumerate(live):
                        sh.records[r + i] = p
                        yield
                        sh.flags.add(r + i)
                        yield
                    live = []
                    handed = True
                    old = sh.alive
                    sh.alive -= 1
                    yield
                    if old == 1:
                        c, rr = sh.claimed, sh.reserved
                        yield
                        if c < rr:
                            sh.alive += 1
                            sh.stays += 1
                            yield
                            continue
                    return
        # walk: every photon in flight takes a few steps; finished ones end here
        still = []
        for p in live:
            p -= steps_per_round
            if p <= 0:
                sh.ended += 1
            else:
                still.append(p)
        live = still
        yield


def run(seed, regroup=8, refill_min=4, floor=2):
    rnd = random.Random(seed)
    n_waves = rnd.randint(3, 12)
    sh = Shared()
    total = 0
    gens = []
    for _ in range(n_waves):
        k = rnd.randint(0, 20)
        photons = [rnd.choice([1, 2, 5, 40, 400]) for _ in range(k)]
        total += len(photons)
        gens.append(wave(sh, photons, regroup, refill_min, floor, lane_count=24))
    ticks = 0
    running = list(range(n_waves))
    while running:
        i = rnd.choice(running)
        try:
            next(gens[i])
        except StopIteration:
            running.remove(i)
        ticks += 1
        assert ticks < 2_000_000, "no progress"
    return sh, total


@pytest.mark.parametrize("block", range(20))
def test_every_photon_ends_once_and_every_wave_exits(block):
    for seed in range(100 * block, 100 * block + 100):
        sh, total = run(seed)
        assert sh.ended == total, seed
        assert sh.claimed == sh.reserved, seed
        assert sh.alive == 0, seed


def test_the_interleavings_reach_hand_offs_and_the_last_wave_staying():
    """The runs above are not vacuous: photons are handed off in most of
    them, and in some the wave that empties the live count finds records
    left and takes them."""
    handed = stays = 0
    for seed in range(2000):
        sh, _ = run(seed)
        handed += sh.reserved > 0
        stays += sh.stays > 0
    assert handed > 1000 and stays > 10
