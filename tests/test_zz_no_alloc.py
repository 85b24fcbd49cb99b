"""spc_query_batch_multi_noalloc (the entry point for callers that cannot
allocate) against spc_query_batch_multi, called through the C ABI: two calls
in a row on the same scratch array, the second with fewer queries, on a
batch of graphs with every bucket in use; answers, counts and flags equal
bit for bit.  Sizes beyond the limit are refused before any launch."""
import ctypes as C

import numpy as np
import pytest

from paper_2212_00977_amd import inputs

pytestmark = pytest.mark.gpu


def _call(fn, ix, gid, s, t, dist, cnt, flg, stream):
    return fn(ix.handle, gid.data_ptr(), s.data_ptr(), t.data_ptr(), int(s.shape[0]), dist.data_ptr(),
              cnt.data_ptr(), flg.data_ptr(), C.c_void_p(stream.cuda_stream))


def test_noalloc_equals_multi_two_calls():
    import torch
    from paper_2212_00977_amd import native, spc

    L = native.load()
    graphs = inputs.rmat_batch(24, seed=11, scale_lo=6, scale_hi=12)
    print(f"[case] no-alloc multi query, {len(graphs)} graphs", flush=True)
    ix = spc.build_index_batch(graphs)
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(5)
    dt = torch.uint8 if ix.dist_bits == 8 else torch.int16
    for nq in (300_000, 70_001):  # second call smaller: stale scratch must not leak in
        gid = rng.integers(0, len(graphs) + 1, size=nq).astype(np.uint32)  # some invalid ids
        n = np.array([g.n for g in graphs] + [1], dtype=np.int64)[gid]
        s = (rng.random(nq) * n).astype(np.uint32)
        t = (rng.random(nq) * n).astype(np.uint32)
        g_d, s_d, t_d = (torch.from_numpy(x.view(np.int32)).to(dev) for x in (gid, s, t))
        outs = []
        for fn in (L.spc_query_batch_multi, L.spc_query_batch_multi_noalloc):
            dist = torch.full((nq,), 7, dtype=dt, device=dev)
            cnt = torch.full((nq,), 7, dtype=torch.int64, device=dev)
            flg = torch.full((nq,), 7, dtype=torch.uint8, device=dev)
            assert _call(fn, ix, g_d, s_d, t_d, dist, cnt, flg, stream) == 0
            torch.cuda.synchronize()
            outs.append((dist.cpu().numpy(), cnt.cpu().numpy(), flg.cpu().numpy()))
        for a, b in zip(*outs):
            assert np.array_equal(a, b), nq
        assert np.any(outs[0][2] == spc.FLAG_INVALID)
    # beyond the limit: refused, nothing launched
    big = 1 << 22
    assert L.spc_query_batch_multi_noalloc(ix.handle, None, 1, 1, big + 1, 1, 1, None, None) == 5
    assert L.spc_query_batch_multi_noalloc(ix.handle, None, None, None, 0, None, None, None, None) == 0
    assert L.spc_query_batch_multi_noalloc(None, None, None, None, 1, None, None, None, None) == 1
    ix.free()
