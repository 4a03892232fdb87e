"""Pins of the oracle's serial LRU simulator (Sec. 4.2, Alg. 1): a
hand-worked scenario (values worked out on paper from the algorithm's text)
and invariants over random isovalue sequences."""
import numpy as np
import pytest

HIGH = 2 ** 31


def _mask(n, ids):
    m = np.zeros(n, np.uint8)
    m[list(ids)] = 1
    return m


def test_hand_worked_sequence(orc):
    c = orc.LRU(6, 2, 8)
    # call 1: blocks 0,1 new; two empty slots of equal age -> slot order
    rc, I_new, ev = c.update(_mask(6, [0, 1]))
    assert rc == 0 and I_new.tolist() == [0, 1] and ev == 0
    I_slot, S_block, S_age = c.state()
    assert I_slot.tolist() == [0, 1, -1, -1, -1, -1]
    assert S_block.tolist() == [0, 1] and S_age.tolist() == [0, 0]
    # call 2: block 1 hit, block 2 new; block 0 inactive -> its slot is reused
    rc, I_new, ev = c.update(_mask(6, [1, 2]))
    assert I_new.tolist() == [2] and ev == 1
    I_slot, S_block, S_age = c.state()
    assert I_slot.tolist() == [-1, 1, 0, -1, -1, -1]
    assert S_block.tolist() == [2, 1] and S_age.tolist() == [0, 0]
    # call 3: two new blocks, nothing available -> grow by max(2, ceil(2/2)) = 2
    rc, I_new, ev = c.update(_mask(6, [0, 1, 2, 3]))
    assert I_new.tolist() == [0, 3] and ev == 0 and c.n_slots == 4
    I_slot, S_block, S_age = c.state()
    assert I_slot.tolist() == [2, 1, 0, 3, -1, -1]
    assert S_block.tolist() == [2, 1, 0, 3] and S_age.tolist() == [0, 0, 0, 0]
    # call 4: nothing active -> ages only
    rc, I_new, ev = c.update(_mask(6, []))
    assert len(I_new) == 0 and c.state()[2].tolist() == [1, 1, 1, 1]
    # call 5: block 1 active and cached -> its age resets
    c.update(_mask(6, [1]))
    assert c.state()[2].tolist() == [2, 0, 2, 2]
    # call 6: block 4 new; oldest available slots are 0, 2, 3 (age 3): slot 0
    rc, I_new, ev = c.update(_mask(6, [4]))
    assert I_new.tolist() == [4] and ev == 1
    I_slot, S_block, S_age = c.state()
    assert I_slot.tolist() == [2, 1, -1, 3, 0, -1]
    assert S_block.tolist() == [4, 1, 0, 3] and S_age.tolist() == [0, 1, 3, 3]


def test_empty_slots_have_high_age(orc):
    c = orc.LRU(10, 4, 4)
    c.update(_mask(10, [7]))
    _, S_block, S_age = c.state()
    assert S_block.tolist() == [7, -1, -1, -1]
    assert S_age.tolist() == [0, HIGH + 1, HIGH + 1, HIGH + 1]


def test_cap_error_resets(orc):
    c = orc.LRU(10, 2, 3)
    rc, _, _ = c.update(_mask(10, [0, 1, 2, 3]))
    assert rc == -3
    I_slot, S_block, S_age = c.state()
    assert (I_slot == -1).all() and c.n_slots == 2 and (S_block == -1).all()


def test_growth_rule(orc):
    c = orc.LRU(100, 10, 1000)
    c.update(_mask(100, range(12)))          # need 12, have 10 -> +max(2, 5)
    assert c.n_slots == 15
    # 48 new; available: 12 released + 3 empty = 15 -> +max(33, ceil(15/2))
    c.update(_mask(100, range(12, 60)))
    assert c.n_slots == 48
    c.update(_mask(100, range(0, 80)))       # 32 new, 0 available -> +max(32, 24)
    assert c.n_slots == 80
    c0 = orc.LRU(100, 0, 50)
    c0.update(_mask(100, range(5)))          # empty cache grows to exactly 5
    assert c0.n_slots == 5


@pytest.mark.parametrize("seed", [0, 1])
def test_invariants_random_sequences(orc, seed):
    rng = np.random.default_rng(seed)
    nb = 500
    c = orc.LRU(nb, 40, 10_000)
    prev = None
    for it in range(40):
        if prev is not None and rng.random() < 0.2:
            act = prev.copy()
        else:
            lo = rng.integers(0, nb - 50)
            act = np.zeros(nb, np.uint8)
            act[lo:lo + rng.integers(1, 120)] = 1
            act[rng.integers(0, nb, 5)] = 1
        rc, I_new, ev = c.update(act)
        assert rc == 0
        I_slot, S_block, S_age = c.state()
        # mutual inverses
        for b in np.nonzero(I_slot >= 0)[0]:
            assert S_block[I_slot[b]] == b
        for s in np.nonzero(S_block >= 0)[0]:
            assert I_slot[S_block[s]] == s
        # every active block is cached, with age 0
        assert (I_slot[act == 1] >= 0).all()
        assert (S_age[I_slot[act == 1]] == 0).all()
        assert c.n_slots >= int(act.sum())
        # new blocks: exactly the active ones that were not cached before
        assert np.all(np.diff(I_new.astype(np.int64)) > 0)
        if prev is not None and np.array_equal(prev, act):
            assert len(I_new) == 0
        prev = act


def test_idle_equals_repeated_empty_updates(orc):
    """k idle calls at once == k updates with nothing active, from a cache
    with mixed ages, empty slots and a grown slot range; then both caches
    evolve identically (the availability marks agree too)."""
    rng = np.random.default_rng(5)
    n = 40
    a, b = orc.LRU(n, 6, 30), orc.LRU(n, 6, 30)
    for _ in range(12):
        m = (rng.random(n) < 0.2).astype(np.uint8)
        assert a.update(m)[0] == b.update(m)[0]
    for k in (1, 7, 1000):
        a.idle(k)
        for _ in range(k):
            b.update(np.zeros(n, np.uint8))
        for x, y in zip(a.state(), b.state()):
            assert np.array_equal(x, y)
        m = (rng.random(n) < 0.3).astype(np.uint8)
        ra, rb = a.update(m), b.update(m)
        assert ra[0] == rb[0] and np.array_equal(ra[1], rb[1]) and ra[2] == rb[2]
        for x, y in zip(a.state(), b.state()):
            assert np.array_equal(x, y)
    # ages saturate at 2^32 - 1
    a.idle(2 ** 33)
    assert np.all(a.state()[2] == 2 ** 32 - 1)
