"""Served queries: every request's answers in the mix (continuous batching,
several streams, memory-limited admission) equal the same request run
alone, and the oracle's answers."""
import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests.gpu_util import dist_as_u32

pytestmark = pytest.mark.gpu


def test_served_equals_alone_and_oracle():
    import torch

    from paper_2212_00977_amd import serve, spc

    g = inputs.chung_lu(1 << 12, seed=2)
    print(f"[case] serve on {g.name}", flush=True)
    ix = spc.build_graph(g)
    ref = oracle.build_graph(g)
    reqs = serve.requests_from(inputs.poisson_requests(g.n, 20000.0, 60, seed=3, max_batch=4096))
    srv = serve.Server(ix, io_budget_bytes=2 * 4096 * serve.BYTES_PER_QUERY_IO, streams=3,
                       max_batch=8192)

    def check(out):
        assert len(out.results) == len(reqs)
        for r in reqs:
            got = out.results[r.rid]
            d, c, f = ix.query(r.s, r.t)
            torch.cuda.synchronize()
            assert np.array_equal(got.dist, spc.as_dist(d)), r.rid
            assert np.array_equal(got.count, spc.as_u64(c)), r.rid
            assert np.array_equal(got.flags, f.cpu().numpy()), r.rid
            rd, rc = ref.query(r.s, r.t)
            assert np.array_equal(dist_as_u32(got.dist, 8), rd) and np.array_equal(got.count, rc)

    # open-loop Poisson arrivals: answers only (the overlap depends on timing)
    check(srv.run(reqs))
    # a burst (every request due at once): the budget holds about two
    # requests' I/O, so admission must defer some and coalesce others
    burst = serve.requests_from(inputs.poisson_requests(g.n, 20000.0, 60, seed=3, max_batch=4096))
    for r in burst:
        r.arrival = 0.0
    out = srv.run(burst)
    check(out)
    assert out.launches < len(reqs)          # some requests were coalesced
    assert out.deferred > 0                  # the small budget made some wait
    base = serve.fifo_baseline(ix, reqs[:10])
    for r in reqs[:10]:
        assert np.array_equal(base.results[r.rid].count, out.results[r.rid].count)
