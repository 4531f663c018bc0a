"""Pins for the pool oracle: invariants on random sequences and
hand-worked eviction sequences."""
import numpy as np
import pytest

from oracle import dedup as D
from oracle.pool import PoolSim


def _check(sim: PoolSim):
    assert len(sim.resident) <= sim.budget
    for c, r in sim.rc.items():
        assert r >= 0
        if r > 0:
            assert c in sim.resident
    assert set(sim.lru) == {c for c in sim.resident if sim.rc[c] == 0}
    assert len(sim.lru) == len(set(sim.lru))


def test_no_eviction_matches_dedup_partition():
    rng = np.random.default_rng(0)
    B = 64
    pool = [rng.integers(0, 256, B, dtype=np.uint8) for _ in range(5)]
    blobs = []
    for f in range(4):
        buf = rng.integers(0, 256, 9 * B, dtype=np.uint8)
        for k in range(9):
            if rng.random() < 0.4:
                buf[k * B:(k + 1) * B] = pool[int(rng.integers(0, 5))]
        blobs.append(buf)
    sim = PoolSim(budget_slots=1000)
    for f, b in enumerate(blobs):
        keys = [b[o:o + L].tobytes() for o, L in D.block_spans(b.size, B)]
        assert sim.register(f, keys, [len(k) for k in keys])
    canon = D.partition_bruteforce(blobs, B)
    sim_canon = [[(c,) for c in sim.fn_classes[f]] for f in range(4)]
    assert D.same_partition(canon, sim_canon)
    assert sim.h2d_bytes == sum(b.size for b in blobs)


def test_hand_worked_eviction():
    sim = PoolSim(budget_slots=4)
    assert sim.register("a", ["x", "y"], [1, 1])       # classes 0,1
    assert sim.register("b", ["y", "z"], [1, 1])       # joins 1, new 2
    assert sim.lru == [0, 1, 2]
    h = sim.setup("a")
    assert sim.rc == {0: 1, 1: 1, 2: 0} and sim.lru == [2]
    # c needs 2 new slots: 1 free, then evicts front unreferenced (class 2)
    assert sim.register("c", ["u", "v"], [1, 1])
    assert 2 not in sim.resident
    # b's setup needs class 2 back: budget full, nothing unreferenced outside b?
    # lru = [3, 4] (c's classes) -> evicts 3 to reload 2
    assert sim.lru == [3, 4]
    hb = sim.setup("b")
    assert hb is not None and 2 in sim.resident and 3 not in sim.resident
    assert sim.h2d_bytes == 2 + 2 + 2 + 1
    sim.release(h)
    sim.release(hb)
    assert all(v == 0 for v in sim.rc.values())
    assert sim.lru == [4, 0, 1, 2]


def test_admission_all_or_nothing():
    sim = PoolSim(budget_slots=3)
    assert sim.register("a", ["p", "q"], [1, 1])
    ha = sim.setup("a")
    assert sim.register("b", ["r"], [1])
    hb = sim.setup("b")
    before = (set(sim.resident), dict(sim.rc), list(sim.lru))
    # everything referenced: a new function cannot even register
    assert sim.register("d", ["t"], [1]) is False
    assert (set(sim.resident), dict(sim.rc), list(sim.lru)) == before
    sim.release(ha)
    sim.release(hb)


@pytest.mark.parametrize("seed", range(8))
def test_random_sequences_invariants(seed):
    rng = np.random.default_rng(seed)
    sim = PoolSim(budget_slots=int(rng.integers(3, 12)))
    contents = [f"k{i}" for i in range(10)]
    registered, live = [], []
    for step in range(300):
        op = rng.random()
        if op < 0.15 and len(registered) < 6:
            fn = f"f{step}"
            nb = int(rng.integers(1, 5))
            keys = [contents[int(rng.integers(0, 10))] for _ in range(nb)]
            if sim.register(fn, keys, [1] * nb):
                registered.append(fn)
        elif op < 0.6 and registered:
            fn = registered[int(rng.integers(0, len(registered)))]
            h = sim.setup(fn)
            if h is not None:
                live.append(h)
                for c in sim.fn_classes[fn]:
                    assert c in sim.resident
        elif op < 0.9 and live:
            sim.release(live.pop(int(rng.integers(0, len(live)))))
        elif registered:
            fn = registered[int(rng.integers(0, len(registered)))]
            if fn not in sim.live.values():
                sim.unregister(fn)
                registered.remove(fn)
        _check(sim)
    for h in live:
        sim.release(h)
    _check(sim)
    assert all(v == 0 for v in sim.rc.values())
