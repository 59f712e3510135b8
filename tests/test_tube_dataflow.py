"""The schedule of the tube kernel (k_tubes), modelled on the CPU.

Inside a workgroup a tube is cut into chunks of one wavefront (32 cells in
float64, 64 in float32); the work is the sequence of (step s, chunk c) items
in the order k = s * nch + c, which eight wavefronts take from a counter.
An item waits until every chunk its gathers reach (chunk_reach, the same
arithmetic as the kernel's) has finished step s - 1, as seen through one
byte per chunk holding the step count modulo 256; then it reads the
previous step's populations of the cells within 6 of its own and writes its
own cells in the other buffer.

The model runs that protocol with random item durations and checks what the
kernel relies on: every read sees exactly the previous step's value of its
source cell (no read of a slot written too early or not yet written), no
write lands on a slot while an older reader of it is still running, every
item is taken and finished (no deadlock), and the byte counters stay correct
past 255 steps.  A schedule that waits only for chunks c - 1 .. c + 1 --
the interior rule -- fails it: with a last chunk shorter than 6 cells the
periodic wrap reaches one chunk further."""
import heapq
import random

import pytest

MAXD = 6        # largest displacement along z
WAVES = 8       # wavefronts of a tube workgroup


def chunk_reach(c, nch, n, ch):
    """Cyclic run (first, count) of the chunks the gathers of chunk c reach."""
    start = c * ch
    end = min(start + ch, n)
    if end - start + 2 * MAXD >= n:
        return 0, nch
    lo = start - MAXD
    if lo < 0:
        lo += n
    hi = end - 1 + MAXD
    if hi >= n:
        hi -= n
    first = lo // ch
    count = hi // ch - first + 1 if hi >= lo else nch - first + hi // ch + 1
    return first, min(count, nch)


def interior_reach(c, nch, n, ch):
    return ((c - 1) % nch, 3) if nch >= 3 else (0, nch)


def simulate(n, ch, steps, seed, reach=chunk_reach):
    rnd = random.Random(seed)
    nch = (n + ch - 1) // ch
    total = steps * nch
    done = [0] * nch                      # the kernel's byte per chunk
    version = [[0] * n, [-1] * n]         # which step's input each slot holds
    readers = [[0] * n, [0] * n]          # items still reading each slot
    taken = 0
    waiting, running, t = {}, [], 0.0

    def take(w):
        nonlocal taken
        if taken < total:
            waiting[w] = taken
            taken += 1

    def reached(c, s):
        return ((done[c] - s) & 255) < 128

    def sources(c):
        for x in range(c * ch, min(c * ch + ch, n)):
            for s in range(-MAXD, MAXD + 1):
                yield (x - s) % n

    for w in range(WAVES):
        take(w)
    while waiting or running:
        for w, k in list(waiting.items()):
            s, c = divmod(k, nch)
            first, count = reach(c, nch, n, ch)
            if all(reached((first + q) % nch, s & 255) for q in range(count)):
                del waiting[w]
                b = s % 2
                for src in sources(c):
                    assert version[b][src] == s, ("read of a stale or early slot", n, ch, s, c, src)
                    readers[b][src] += 1
                heapq.heappush(running, (t + rnd.uniform(1.0, 3.0), w, k))
        assert running, ("deadlock", n, ch, waiting)
        t, w, k = heapq.heappop(running)
        s, c = divmod(k, nch)
        b = s % 2
        for src in sources(c):
            readers[b][src] -= 1
        for x in range(c * ch, min(c * ch + ch, n)):
            assert readers[1 - b][x] == 0, ("write under a running reader", n, ch, s, c, x)
            version[1 - b][x] = s + 1
        done[c] = (s + 1) & 255
        take(w)
    assert taken == total
    assert all(v == steps for v in version[steps % 2])


@pytest.mark.parametrize("ch", [32, 64])
def test_reach_covers_every_gather(ch):
    for n in range(1, 700):
        nch = (n + ch - 1) // ch
        for c in range(nch):
            first, count = chunk_reach(c, nch, n, ch)
            run = {(first + q) % nch for q in range(count)}
            need = {src // ch for src in ((x - s) % n for x in range(c * ch, min(c * ch + ch, n))
                                          for s in range(-MAXD, MAXD + 1))}
            assert need <= run, (n, c, need - run)


@pytest.mark.parametrize("ch", [32, 64])
def test_schedule_is_race_free_and_finishes(ch):
    for n in list(range(1, 70, 3)) + [70, 71, 200, 257, 333, 1999]:
        simulate(n, ch, 9 if n > 300 else 13, seed=n)


def test_step_counters_wrap():
    simulate(257, 32, 600, seed=1)


def test_interior_rule_alone_is_not_enough():
    with pytest.raises(AssertionError):
        simulate(257, 32, 13, seed=1, reach=interior_reach)
