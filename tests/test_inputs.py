"""The seeded input generators (the workloads' recipe): the same seed gives
the same graph, outputs are simple symmetric CSRs, and the sizes the recipe
states hold (exact edge counts for G(n, m) and Chung-Lu, all 2^scale
vertices for R-MAT, the largest component of a grid, request batch sizes)."""
import numpy as np
import pytest

from paper_2212_00977_amd import inputs


def simple_symmetric(g):
    n = g.n
    rows = np.repeat(np.arange(n), np.diff(g.off).astype(np.int64))
    cols = g.adj.astype(np.int64)
    assert (cols < n).all() and not (rows == cols).any()
    fwd = set(zip(rows.tolist(), cols.tolist()))
    assert len(fwd) == cols.shape[0]                      # no duplicates
    assert all((b, a) in fwd for a, b in fwd)             # symmetric


@pytest.mark.parametrize("make", [
    lambda s: inputs.erdos_renyi(500, 1200, seed=s),
    lambda s: inputs.chung_lu(1 << 11, seed=s),
    lambda s: inputs.rmat(10, 8, seed=s),
    lambda s: inputs.grid_lcc(40, 0.05, seed=s),
])
def test_seeded_and_well_formed(make):
    a, b, c = make(3), make(3), make(4)
    assert np.array_equal(a.off, b.off) and np.array_equal(a.adj, b.adj)
    assert not (a.off.shape == c.off.shape and np.array_equal(a.adj, c.adj) and np.array_equal(a.off, c.off))
    simple_symmetric(a)


def test_stated_sizes():
    assert inputs.erdos_renyi(500, 1200, seed=1).m == 1200
    g = inputs.chung_lu(1 << 12, seed=2)
    assert g.n == 4096 and g.m == 4096 * 10 // 2           # mean degree exactly 10
    assert inputs.rmat(9, 4, seed=3).n == 512
    grid = inputs.grid_lcc(30, 0.05, seed=3)
    assert grid.n <= 900 and grid.tie_key is not None and grid.tie_key.shape[0] == grid.n
    s, t = inputs.queries(1000, 5000, seed=7)
    assert s.shape == t.shape == (5000,) and s.max() < 1000 and t.max() < 1000
    reqs = inputs.poisson_requests(1000, 1e4, 200, seed=8, max_batch=512)
    arr = [r[3] for r in reqs]
    assert all(1 <= r[1].shape[0] <= 512 and r[1].shape == r[2].shape for r in reqs)
    assert arr[0] == 0.0 and all(x <= y for x, y in zip(arr, arr[1:]))


def test_batch_is_reproducible_per_graph():
    a = inputs.rmat_batch(6, seed=4, scale_lo=6, scale_hi=9)
    b = inputs.rmat_batch(6, seed=4, scale_lo=6, scale_hi=9)
    assert [g.n for g in a] == [g.n for g in b]
    assert all(np.array_equal(x.adj, y.adj) for x, y in zip(a, b))
