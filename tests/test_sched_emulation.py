"""Host emulation of the persistent form's work distribution (the claim loop
of chem_persistent): cells' global positions are dealt to nq queues
(position q, q + nq, ...), a wave claims as many positions as it has idle
lanes from its queue with one atomic add, moves to the next queue when its
queue cannot fill the request, and stops after finding every queue short;
lanes refill when at least `refill` are idle.  Waves are threads here, the
atomic add a locked fetch-add, and random yields and per-cell durations
shuffle the interleavings.  Every position must be processed exactly once
and every wave must stop.  No GPU."""
import random
import threading
import time

import pytest

LANES = 64


class Heads:
    def __init__(self, nq):
        self.v = [0] * nq
        self.lock = threading.Lock()

    def fetch_add(self, q, n):
        with self.lock:
            old = self.v[q]
            self.v[q] += n
            return old


def wave(wid, total, nq, refill, perm, heads, done, done_lock, rng):
    q = wid % nq                          # home queue (the workgroup's XCD)
    tried, exhausted = 0, False
    have = [False] * LANES
    work = [0] * LANES
    cell = [-1] * LANES
    while True:
        idle = [not h for h in have]
        nidle = sum(idle)
        if not exhausted and (nidle >= refill or nidle == LANES):
            need, assigned = nidle, 0
            ranks = {}
            r = 0
            for lane in range(LANES):          # rank of each idle lane among the idle ones
                if idle[lane]:
                    ranks[lane] = r
                    r += 1
            claimed = {}
            while need > 0 and not exhausted:
                old = heads.fetch_add(q, need)
                if rng.random() < 0.3:
                    time.sleep(0)
                qsize = (total - q + nq - 1) // nq
                avail = qsize - old
                got = 0 if avail <= 0 else min(avail, need)
                for lane, rk in ranks.items():
                    if lane not in claimed and assigned <= rk < assigned + got:
                        pos = (old + (rk - assigned)) * nq + q
                        claimed[lane] = perm[pos] if perm is not None else pos
                assigned += got
                if got < need:
                    q = 0 if q + 1 == nq else q + 1
                    tried += 1
                    if tried >= nq:
                        exhausted = True
                need -= got
            for lane, g in claimed.items():
                have[lane], cell[lane], work[lane] = True, g, rng.randint(1, 6)
        if not any(have):
            if exhausted:
                return
            continue
        for lane in range(LANES):               # one substep attempt per busy lane
            if have[lane]:
                work[lane] -= 1
                if work[lane] == 0:
                    with done_lock:
                        done.append(cell[lane])
                    have[lane] = False
        if rng.random() < 0.2:
            time.sleep(0)


@pytest.mark.parametrize("total,nwaves,refill,ordered", [(1, 3, 1, False), (63, 5, 16, False),
                                                          (5000, 24, 1, True), (5000, 24, 16, False),
                                                          (4097, 40, 64, True), (777, 2, 8, True)])
def test_every_cell_exactly_once(total, nwaves, refill, ordered):
    nq = 8
    rng = random.Random(total * 31 + nwaves)
    perm = list(range(total))
    if ordered:
        rng.shuffle(perm)
    heads = Heads(nq)
    done, done_lock = [], threading.Lock()
    threads = [threading.Thread(target=wave, args=(w, total, nq, refill, perm if ordered else None, heads, done,
                                                   done_lock, random.Random(1000 + w)))
               for w in range(nwaves)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
        assert not t.is_alive(), "a wave did not stop"
    assert sorted(done) == list(range(total))
    # every queue was drained past its size (heads only grow)
    assert all(heads.v[q] >= (total - q + nq - 1) // nq for q in range(nq))
