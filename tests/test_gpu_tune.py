"""Query launch configurations and their autotuner: every configuration
gives the oracle's answers (8- and 16-bit labels), and tuning keeps a valid
configuration without changing any answer."""
import numpy as np
import pytest

import oracle
from paper_2212_00977_amd import inputs
from tests.gpu_util import gpu_query

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["chunglu14", "path300"])
def test_every_config_matches_oracle(name):
    from paper_2212_00977_amd import spc

    g = inputs.chung_lu(1 << 14, seed=2) if name == "chunglu14" else inputs.from_edges(
        300, np.stack([np.arange(299), np.arange(1, 300)], axis=1), name="path300")
    print(f"[case] {g.name}", flush=True)
    ix = spc.build_graph(g)
    assert ix.dist_bits == (8 if name == "chunglu14" else 16)
    ref = oracle.build_graph(g)
    s, t = inputs.queries(g.n, 20000, seed=31)
    rd, rc = ref.query(s, t)
    cfgs = spc.query_configs()
    for k in range(len(cfgs)):
        ix.set_query_config(k)
        assert ix.query_config == k
        d, c, f = gpu_query(ix, s, t)
        assert np.array_equal(d, rd) and np.array_equal(c, rc), cfgs[k]


def test_tuner_keeps_answers():
    from paper_2212_00977_amd import spc

    g = inputs.rmat(12, 8, seed=4)
    print(f"[case] tune on {g.name}", flush=True)
    ix = spc.build_graph(g)
    ref = oracle.build_graph(g)
    ss, tt = inputs.queries(g.n, 50000, seed=32)
    k = ix.tune_queries(ss, tt)
    assert 0 <= k < len(spc.query_configs()) and ix.query_config == k
    s, t = inputs.queries(g.n, 20000, seed=33)
    d, c, f = gpu_query(ix, s, t)
    rd, rc = ref.query(s, t)
    assert np.array_equal(d, rd) and np.array_equal(c, rc)
    with pytest.raises(spc.SpcError):
        ix.set_query_config(len(spc.query_configs()))


def test_tune_cache_round_trip(tmp_path):
    """The on-disk tuning cache: the tuners write the index's configuration
    and bucket threshold; a later build of the same graph takes both (and
    answers as the oracle does); another graph finds nothing and adds its
    own line."""
    from paper_2212_00977_amd import spc

    path = str(tmp_path / "spc_tune.txt")
    opts = spc.BuildOptions(tune_cache=path)
    g = inputs.rmat(12, 8, seed=4)
    print(f"[case] tune cache on {g.name}", flush=True)
    ix = spc.build_graph(g, opts=opts)
    assert ix.stats()["tune_cached"] == 0
    ss, tt = inputs.queries(g.n, 50000, seed=32)
    k = ix.tune_queries(ss, tt)
    small = ix.tune_query_buckets(None, ss, tt)
    with open(path) as f:
        lines = f.read().splitlines()
    assert len(lines) == 1
    key, cfg, thr = lines[0].split()
    assert len(key) == 16 and int(cfg) == k and int(thr) == small
    ix.free()

    ix2 = spc.build_graph(g, opts=opts)
    st = ix2.stats()
    assert st["tune_cached"] == 1 and st["query_config"] == k and st["query_small"] == small
    ref = oracle.build_graph(g)
    s, t = inputs.queries(g.n, 20000, seed=33)
    d, c, f = gpu_query(ix2, s, t)
    rd, rc = ref.query(s, t)
    assert np.array_equal(d, rd) and np.array_equal(c, rc)
    ix2.free()

    g3 = inputs.rmat(11, 8, seed=4)
    print(f"[case] tune cache on {g3.name}", flush=True)
    ix3 = spc.build_graph(g3, opts=opts)
    assert ix3.stats()["tune_cached"] == 0
    ix3.tune_queries(*inputs.queries(g3.n, 20000, seed=34))
    with open(path) as f:
        lines = f.read().splitlines()
    assert len(lines) == 2 and lines[0].split()[0] == key
    ix3.free()

    ix4 = spc.build_graph(g)  # no cache path: defaults, nothing read
    assert ix4.stats()["tune_cached"] == 0
    ix4.free()
