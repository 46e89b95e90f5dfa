"""Host logic of the XCD-grouped row order (ofm_grouped_order, the order that
ofm_build_laplacian_grouped lays out), through the C ABI without a device:
a permutation of the rows in eight contiguous slots; each group in one slot
and contiguous there; the rows of 64 or more entries first in their slot,
then the groups, then the rows without a group; entry counts descending
inside each run; slot loads balanced; argument errors."""
import numpy as np
import pytest

from paper_2305_10356_amd import ofm

HEAVY = 64


def random_csr_degrees(n, rng):
    deg = np.where(rng.random(n) < 0.1, rng.integers(40, 300, n), rng.integers(1, 30, n))
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum(deg)
    return rp.astype(np.int32), deg


def check_order(rp, groups, order, slots):
    n = rp.shape[0] - 1
    deg = np.diff(rp).astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(n))
    assert slots[0] == 0 and slots[8] == n and np.all(np.diff(slots) >= 0)
    slot_of = np.empty(n, dtype=np.int64)
    for x in range(8):
        rows = order[slots[x]:slots[x + 1]]
        slot_of[rows] = x
        d = deg[rows]
        g = groups[rows]
        phase = np.where(d >= HEAVY, 0, np.where(g >= 0, 1, 2))
        assert np.all(np.diff(phase) >= 0), "heavy rows, then groups, then no group"
        key = np.where(phase == 1, g, -1 - phase)
        # runs of one key: contiguous (a key never reappears) and entry counts descending
        change = np.flatnonzero(np.diff(key) != 0) + 1
        starts = np.concatenate([[0], change])
        ends = np.concatenate([change, [len(rows)]])
        seen = set()
        for a, b in zip(starts, ends):
            k = int(key[a])
            assert k not in seen, "a group split inside its slot"
            seen.add(k)
            assert np.all(np.diff(d[a:b]) <= 0), "entry counts descending in a run"
    # every (non-heavy) row of a group sits in one slot
    light = deg < HEAVY
    for gid in np.unique(groups[(groups >= 0) & light]):
        assert len(np.unique(slot_of[(groups == gid) & light])) == 1
    return slot_of


@pytest.mark.parametrize("seed", range(6))
def test_grouped_order_invariants(lib, seed):
    rng = np.random.default_rng([9, seed])
    n = int(rng.integers(1, 6000))
    rp, deg = random_csr_degrees(n, rng)
    ng = int(rng.integers(1, 80))
    groups = rng.integers(0, ng, n).astype(np.int32)
    neg = rng.random(n) < 0.15
    groups[neg] = -1 - rng.integers(0, 3, int(neg.sum()))
    order, slots = ofm.grouped_order(rp, groups)
    check_order(rp, groups, order, slots)


def test_grouped_order_balances_equal_groups(lib):
    # 32 equal groups of equal degree: four groups per slot, equal loads
    n = 32 * 500
    rp = (np.arange(n + 1) * 10).astype(np.int32)
    groups = np.repeat(np.arange(32), 500).astype(np.int32)
    order, slots = ofm.grouped_order(rp, groups)
    slot_of = check_order(rp, groups, order, slots)
    assert np.all(np.diff(slots) == 4 * 500)
    assert all(len(np.unique(groups[slot_of == x])) == 4 for x in range(8))


def test_grouped_order_without_groups_deals_rows_evenly(lib):
    rng = np.random.default_rng(5)
    rp, deg = random_csr_degrees(4000, rng)
    groups = np.full(4000, -1, dtype=np.int32)
    order, slots = ofm.grouped_order(rp, groups)
    slot_of = check_order(rp, groups, order, slots)
    load = np.array([(deg[slot_of == x] + 1).sum() for x in range(8)])
    assert load.max() - load.min() <= (deg + 1).max()


def test_grouped_order_errors(lib):
    rp = np.array([0, 2, 4, 6], dtype=np.int32)
    with pytest.raises(ofm.OfmError):
        ofm.grouped_order(rp, np.array([0, 1, 3], dtype=np.int32))  # id >= n
    with pytest.raises(ofm.OfmError):
        ofm.grouped_order(np.array([0, 2, 1, 6], dtype=np.int32), np.zeros(3, np.int32))
    with pytest.raises(ValueError):
        ofm.grouped_order(rp, np.zeros(2, np.int32))
