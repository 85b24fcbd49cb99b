"""The server's admission rule (host logic, no GPU): requests leave the
queue in arrival order while their I/O fits the budget beside what is in
flight, one graph and at most max_batch queries per launch."""
from collections import deque

import numpy as np

from paper_2212_00977_amd.serve import BYTES_PER_QUERY_IO, Request, take_batch


def reqs(sizes, graphs=None):
    graphs = graphs or [0] * len(sizes)
    return deque(Request(i, np.zeros(n, np.uint32), np.zeros(n, np.uint32), 0.0, g)
                 for i, (n, g) in enumerate(zip(sizes, graphs)))


def test_coalesces_within_budget_and_batch_limit():
    q = reqs([10, 20, 30, 40])
    assert take_batch(q, 0, 1 << 30, False, True, 1 << 18) == 4
    assert take_batch(q, 0, 1 << 30, False, True, 60) == 3   # 10+20+30 = 60 fits, +40 does not
    assert take_batch(q, 0, 1 << 30, False, False, 1 << 18) == 1


def test_budget_defers_and_oversize_runs_alone():
    q = reqs([100, 100])
    b = 150 * BYTES_PER_QUERY_IO
    assert take_batch(q, 0, b, False, True, 1 << 18) == 1
    assert take_batch(q, 60 * BYTES_PER_QUERY_IO, b, True, True, 1 << 18) == 0  # waits for memory
    big = reqs([1000])
    assert take_batch(big, 0, b, False, True, 1 << 18) == 1   # nothing in flight: runs alone
    assert take_batch(big, 0, b, True, True, 1 << 18) == 0


def test_one_graph_per_launch():
    q = reqs([5, 5, 5, 5], graphs=[1, 1, 2, 1])
    assert take_batch(q, 0, 1 << 30, False, True, 1 << 18) == 2
    assert take_batch(deque(), 0, 1 << 30, False, True, 1 << 18) == 0
