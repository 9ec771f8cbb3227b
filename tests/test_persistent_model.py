"""A CPU model of the persistent batch launch's schedule (ZPM_BATCH_PERSISTENT), run
before the kernel is trusted on the device.

The model has what a one-launch schedule on MI355X depends on:
* co-residency: a few workgroup slots per compute unit (the LDS and register limits),
  a workgroup holding its slot until it exits;
* dispatch order: block b goes to XCD b mod 8 (here b mod n_xcd); either each XCD
  dispatches its own blocks in increasing order as its slots free up, or one dispatcher
  issues all blocks in increasing order and stalls while the next block's XCD is full
  (head-of-line blocking, the stricter case);
* visibility: one L2 cache per XCD, not coherent with the others.  Plain loads and
  stores go through the XCD's L2 (a line, once cached, is reused until an acquire fence
  invalidates that L2; stores stay in it until a release fence writes them back).
  Agent-scope atomics (increments, polling loads) act on memory itself.

Workgroups are interleaved by a seeded random scheduler, one step at a time.  A task is
one tile of one stage of one product; it needs every tile of the previous stage of its
product, which it reads after its wait.  Checked:

* the library's protocol (tasks taken from a ticket counter in stage order, counters
  polled with agent-scope atomic loads, release fence before each count, acquire fence
  after each wait) finishes every batch, never exceeds its wait bound and never reads a
  stale tile, for 1 to 4 slots per CU, 1, 2 and 8 XCDs and many interleavings;
* the two failures seen with the earlier single launch are reproduced by mechanisms
  absent from the library's protocol: tasks fixed to block numbers through an XCD-aware
  remap (a waiting consumer holds the slot its producer needs: no progress, so the
  waits run into their bound), and counters polled with plain loads (a consumer on
  another XCD keeps reading its own stale cached line: the waits run into their bound).
  Without the fences a consumer reads stale tiles.
"""
import random

import pytest


class Batch:
    """Products with a chain of stages each; tasks in stage order (all products' stage 0
    tiles, then stage 1, ...), as the library's grouped launches order them."""

    def __init__(self, rng, n_jobs):
        self.levels = [rng.choice([3, 5, 7]) for _ in range(n_jobs)]
        self.tiles = {}
        for j, nl in enumerate(self.levels):
            for lv in range(nl):
                self.tiles[(j, lv)] = rng.randint(1, 6)
        self.tasks = []
        for lv in range(max(self.levels)):
            for j in range(n_jobs):
                if lv < self.levels[j]:
                    for t in range(self.tiles[(j, lv)]):
                        self.tasks.append((j, lv, t))


class Device:
    def __init__(self, n_xcd, cus, slots):
        self.n_xcd, self.cus, self.slots = n_xcd, cus, slots
        self.mem = {}
        self.l2 = [dict() for _ in range(n_xcd)]      # addr -> value
        self.dirty = [set() for _ in range(n_xcd)]

    # plain accesses through the XCD's L2
    def load(self, x, addr):
        c = self.l2[x]
        if addr not in c:
            c[addr] = self.mem.get(addr, 0)
        return c[addr]

    def store(self, x, addr, v):
        self.l2[x][addr] = v
        self.dirty[x].add(addr)

    # agent-scope atomics act on memory
    def atomic_load(self, addr):
        return self.mem.get(addr, 0)

    def atomic_add(self, addr, v=1):
        old = self.mem.get(addr, 0)
        self.mem[addr] = old + v
        return old

    def release(self, x):
        for a in self.dirty[x]:
            self.mem[a] = self.l2[x][a]
        self.dirty[x].clear()

    def acquire(self, x):
        keep = {a: self.l2[x][a] for a in self.dirty[x]}
        self.l2[x] = keep


def run(batch, n_xcd=8, cus=2, slots=2, seed=0, protocol="library", spin_limit=400,
        n_blocks=None, dispatch_mode="per_xcd"):
    """Simulates one launch; returns (finished, aborted, stale_reads)."""
    rng = random.Random(seed)
    dev = Device(n_xcd, cus, slots)
    ntasks = len(batch.tasks)
    static = protocol == "static_remap"
    G = n_blocks or (ntasks if static else n_xcd * cus * slots)
    if static:
        G = 8 * ((ntasks + 7) // 8)
        chunk = G // 8

        def task_of(b):       # the column passes' XCD-aware block remap
            return (b % 8) * chunk + b // 8
    queues = [[b for b in range(G) if b % n_xcd == x] for x in range(n_xcd)]
    free = [cus * slots for _ in range(n_xcd)]
    resident = []
    wg = {}
    TICKET, ABORT = ("ticket",), ("abort",)
    done_tasks = 0
    stale = 0
    aborted = False

    order = list(range(G))

    def place(b, x):
        free[x] -= 1
        resident.append(b)
        wg[b] = {"x": x, "state": "take", "spins": 0}

    def dispatch():
        if dispatch_mode == "per_xcd":
            for x in range(n_xcd):
                while free[x] and queues[x]:
                    place(queues[x].pop(0), x)
        else:
            while order and free[order[0] % n_xcd]:
                b = order.pop(0)
                place(b, b % n_xcd)

    dispatch()
    steps = 0
    while resident and steps < 2_000_000:
        steps += 1
        b = rng.choice(resident)
        w = wg[b]
        x = w["x"]
        if w["state"] == "take":
            if dev.atomic_load(ABORT):
                w["state"] = "exit"
            elif static:
                if w.get("took"):
                    w["state"] = "exit"
                else:
                    w["took"] = True
                    t = task_of(b)
                    w["task"] = batch.tasks[t] if t < ntasks else None
                    w["state"] = "wait" if w["task"] else "exit"
            else:
                t = dev.atomic_add(TICKET)
                w["task"] = batch.tasks[t] if t < ntasks else None
                w["state"] = "wait" if w["task"] else "exit"
        elif w["state"] == "wait":
            j, lv, _ = w["task"]
            if lv == 0:
                ready = True
            else:
                ctr = ("done", j, lv - 1)
                v = dev.load(x, ctr) if protocol == "plain_poll" else dev.atomic_load(ctr)
                ready = v >= batch.tiles[(j, lv - 1)]
            if ready:
                if protocol != "no_fences":
                    dev.acquire(x)
                w["state"] = "run"
                w["left"] = rng.randint(1, 4)
            elif dev.atomic_load(ABORT):
                w["state"] = "exit"
            else:
                w["spins"] += 1
                if w["spins"] > spin_limit:
                    dev.atomic_add(ABORT)
                    aborted = True
                    w["state"] = "exit"
        elif w["state"] == "run":
            j, lv, t = w["task"]
            w["left"] -= 1
            if w["left"] <= 0:
                if lv > 0:
                    for u in range(batch.tiles[(j, lv - 1)]):
                        if dev.load(x, ("data", j, lv - 1, u)) != 1:
                            stale += 1
                dev.store(x, ("data", j, lv, t), 1)
                if protocol != "no_fences":
                    dev.release(x)
                dev.atomic_add(("done", j, lv))
                done_tasks += 1
                w["spins"] = 0
                w["state"] = "take"
        if w["state"] == "exit":
            resident.remove(b)
            free[x] += 1
            dispatch()
    return done_tasks == ntasks, aborted, stale


@pytest.mark.parametrize("n_xcd", [1, 2, 8])
@pytest.mark.parametrize("slots", [1, 2, 4])
@pytest.mark.parametrize("mode", ["per_xcd", "in_order"])
def test_library_protocol_always_finishes(n_xcd, slots, mode):
    for seed in range(6):
        rng = random.Random(1000 * seed + 10 * n_xcd + slots)
        b = Batch(rng, rng.randint(3, 12))
        # as many blocks as slots, fewer, and more (blocks wait to be dispatched)
        for grid in (None, 1, 3, 4 * n_xcd * 2 * slots):
            fin, ab, stale = run(b, n_xcd=n_xcd, cus=2, slots=slots, seed=seed,
                                 n_blocks=grid, dispatch_mode=mode)
            assert fin and not ab and stale == 0, (n_xcd, slots, seed, grid, mode)


def test_static_remapped_blocks_stall():
    """Tasks fixed to block numbers through the XCD-aware remap, under in-order dispatch:
    consumers dispatched first hold every slot of an XCD while the producers they wait
    for queue behind a block of that XCD."""
    stalls = 0
    for seed in range(12):
        rng = random.Random(seed)
        b = Batch(rng, 8)
        fin, ab, _ = run(b, n_xcd=8, cus=1, slots=1, seed=seed, protocol="static_remap",
                         dispatch_mode="in_order")
        stalls += (not fin) and ab
    assert stalls >= 6


def test_plain_polling_never_sees_other_xcds():
    """Counters polled through the XCD's L2: a consumer whose producer ran on another XCD
    keeps reading its stale cached line until its wait bound."""
    stalls = 0
    for seed in range(12):
        rng = random.Random(50 + seed)
        b = Batch(rng, 8)
        fin, ab, _ = run(b, n_xcd=8, cus=2, slots=2, seed=seed, protocol="plain_poll")
        stalls += (not fin) and ab
    assert stalls >= 10


def test_missing_fences_read_stale_tiles():
    stale_runs = 0
    for seed in range(8):
        rng = random.Random(90 + seed)
        b = Batch(rng, 8)
        fin, ab, stale = run(b, n_xcd=8, cus=2, slots=2, seed=seed, protocol="no_fences")
        stale_runs += stale > 0
    assert stale_runs >= 6
