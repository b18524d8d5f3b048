"""CPU model of the grid-wide barrier of the persistent schedule (k_persist in
device.hip), run by host threads standing for the blocks of one
cooperative launch: the first thread of a block reads the generation, then
arrives on the counter (fetch-add); the block that arrives last resets the
counter and moves the generation on; the others poll the generation and
pass when it moves, or give up after a time limit or when the abort flag
is set (and set it themselves).

Checked over 96 and over 200 steps of three phases each (the number of
barriers a run of that length makes), with random delays: no block passes
a barrier before every block has arrived at it, every block makes the same
number of barriers, the generation ends at the number of barriers (the
counter at zero), and a block that stalls past the limit makes every other
block leave its wait (no wait outlives the limit by much)."""
import random
import threading
import time

import pytest


class Atomic:
    """A word with the device-scope operations the barrier uses."""

    def __init__(self, v=0):
        self.v = v
        self.lock = threading.Lock()

    def load(self):
        with self.lock:
            return self.v

    def store(self, v):
        with self.lock:
            self.v = v

    def fetch_add(self, d):
        with self.lock:
            old = self.v
            self.v += d
            return old


class GridBarrier:
    def __init__(self, nblocks, limit_s):
        self.nblocks = nblocks
        self.count, self.gen, self.abort = Atomic(0), Atomic(0), Atomic(0)
        self.limit = limit_s

    def sync(self):
        """The block's side of one barrier; False if it gave up."""
        g = self.gen.load()
        if self.count.fetch_add(1) == self.nblocks - 1:
            self.count.store(0)
            self.gen.store(g + 1)
            return True
        t0 = time.monotonic()
        while self.gen.load() == g:
            if self.abort.load() or time.monotonic() - t0 > self.limit:
                self.abort.store(1)
                return False
            time.sleep(0)
        return True


def run_model(nblocks, steps, phases=3, limit_s=5.0, stall=None, seed=0):
    bar = GridBarrier(nblocks, limit_s)
    arrived = [[0] * nblocks for _ in range(steps * phases)]   # arrival marks per barrier
    passed_early = []
    made = [0] * nblocks
    rng = random.Random(seed)
    delays = [[rng.random() * 2e-4 for _ in range(steps * phases)] for _ in range(nblocks)]

    def block(b):
        for k in range(steps * phases):
            if stall is not None and stall == (b, k):
                time.sleep(limit_s * 1.5)       # a block stuck in its phase
            time.sleep(delays[b][k])             # the phase's work
            arrived[k][b] = 1
            ok = bar.sync()
            if not ok:
                return
            if sum(arrived[k]) != nblocks:
                passed_early.append((b, k))
            made[b] += 1

    threads = [threading.Thread(target=block, args=(b,)) for b in range(nblocks)]
    t0 = time.monotonic()
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=60)
    assert not any(t.is_alive() for t in threads), "a modelled block never left its wait"
    return bar, made, passed_early, time.monotonic() - t0


@pytest.mark.parametrize("steps", [96, 200])
def test_barrier_generations_over_a_run(steps):
    nb = 24
    bar, made, early, _ = run_model(nb, steps, seed=steps)
    assert early == []
    assert made == [3 * steps] * nb
    assert bar.gen.load() == 3 * steps and bar.count.load() == 0 and bar.abort.load() == 0


def test_barrier_abandons_a_stalled_run():
    nb, limit = 12, 0.2
    bar, made, early, wall = run_model(nb, 20, limit_s=limit, stall=(5, 17))
    assert early == []
    assert bar.abort.load() == 1
    # the others pass barriers 0 .. 16 and give up at 17; the stalled block,
    # arriving last there, passes it and leaves at the next one on the flag
    assert made[5] <= 18 and all(m == 17 for b, m in enumerate(made) if b != 5)
    assert wall < 20 * 3 * 2e-4 * 20 + limit * 1.5 + 5.0
