"""The oracle-side byte model (oracle/byte_model.py) against quantities
recomputed here from full oracle indexes: label sizes and the number of
common hubs at the minimum for sampled queries, and the per-round byte
terms from the PULL build's counters."""
import numpy as np

import oracle
from oracle import byte_model
from paper_2212_00977_amd import inputs


def test_build_bytes_terms_worked_example():
    g = inputs.worked_example()
    L = oracle.build_graph(g, method="pull")
    st = oracle.pull_stats(g.off, g.adj, order=g.order)
    for k in ("raw", "merged", "kept", "scanned"):
        assert np.array_equal(st[k], L.stats[k])
    b = byte_model.build_bytes(st, delta=1)
    r1 = b["rounds"][1]
    # round 1: each of the example's 13 edges gives its lower-ranked end one
    # candidate, which is kept
    assert g.m == 13
    assert r1["expand"] == 12 * 13
    assert r1["write"] == 2 * 13 * 13
    assert b["finalize"] == 2 * 13 * L.entries
    assert b["rounds"][0]["write"] == 2 * 13 * g.n
    assert b["total"] == b["finalize"] + sum(r["total"] for r in b["rounds"])
    for r in b["rounds"]:
        d = r["round"]
        assert r["csr"] == 8 * int(L.stats["active"][d]) + 4 * int(L.stats["active_adj"][d])
        assert r["stage"] == 5 * int(L.stats["staged"][d])
        assert r["probe"] == 5 * int(L.stats["scanned"][d])


def test_query_bytes_from_full_labels():
    for g in (inputs.rmat(10, 8, seed=3), inputs.erdos_renyi(500, 2000, seed=8)):
        L = oracle.build_graph(g, method="definition")
        s, t = inputs.queries(g.n, 300, seed=4)
        got = byte_model.query_bytes_sample(g.off, g.adj, L.order, s, t, delta=1, threads=3)
        rk = L.rank_of()
        per = []
        for a, b in zip(rk[s].tolist(), rk[t].tolist()):
            la = {int(L.hub[i]): int(L.dist[i]) for i in range(int(L.off[a]), int(L.off[a + 1]))}
            lb = {int(L.hub[i]): int(L.dist[i]) for i in range(int(L.off[b]), int(L.off[b + 1]))}
            common = [la[h] + lb[h] for h in la if h in lb]
            k = common.count(min(common)) if common else 0
            per.append((len(la) + len(lb)) * 5 + 16 * k + 8 + 10)
        assert got["queries"] == 300
        assert abs(got["mean_bytes"] - float(np.mean(per))) < 1e-9
