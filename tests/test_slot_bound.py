"""Host-side arithmetic of the hub-row hash tables (bin G of the evaluation
kernels): every row of d entries takes the smallest power of two that is at
least max(2, 2d) slots, and the buffer is sized 4 * (total entries) +
2 * (rows) + 16 slots.  The sum of the row capacities must never exceed that
size, for any degree list (the kernel also checks it before writing)."""
import numpy as np


def row_capacity(d):
    c = 2
    while c < 2 * d:
        c <<= 1
    return c


def buffer_slots(degrees):
    return 4 * int(np.sum(degrees)) + 2 * len(degrees) + 16


def test_capacity_sum_fits_buffer_random_degree_lists():
    rng = np.random.default_rng(7)
    for trial in range(300):
        n = int(rng.integers(1, 200))
        # hub rows (> 4096 entries) and, for the bound itself, any positive degree
        lo = 4097 if trial % 2 == 0 else 1
        d = rng.integers(lo, lo + int(rng.integers(1, 1 << 17)), n)
        caps = [row_capacity(int(x)) for x in d]
        assert sum(caps) <= buffer_slots(d)


def test_capacity_worst_case_just_above_powers_of_two():
    # d = 2^k + 1 needs 4d - 4 slots, the largest ratio the rounding allows
    d = np.array([(1 << k) + 1 for k in range(12, 24)])
    caps = [row_capacity(int(x)) for x in d]
    assert all(c == 4 * x - 4 for c, x in zip(caps, d))
    assert sum(caps) <= buffer_slots(d)
