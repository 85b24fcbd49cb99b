"""Parity of the small-table test build (libspc_smalltab.so: a 128-slot hash
for the puller's label, 256 distinct candidates per chunk) against the
oracle.  Run as a separate process (python -m tests.smalltab_check) so that
the library it loads is the only one in the process; exits non-zero on the
first mismatch.  Small graphs here take the paths that only large labels
take in the default build: unstaged label parts searched in HBM or in the
chunk's LDS window, chunk overflow and narrowing, many chunks per puller."""
import sys
import time

import numpy as np


def main():
    from paper_2212_00977_amd import native
    native.load(native.SMALL_TABLES_PATH)
    import oracle
    from paper_2212_00977_amd import inputs, spc
    from tests.gpu_util import assert_labels_equal, gpu_query

    graphs = [inputs.worked_example(), inputs.erdos_renyi(2000, 8000, seed=1),
              inputs.chung_lu(1 << 13, seed=2), inputs.chung_lu(1 << 14, seed=7),
              inputs.rmat(12, 16, seed=5), inputs.rmat(13, 16, seed=6),
              inputs.rmat(11, 8, seed=4), inputs.grid_lcc(40, 0.05, seed=3),
              inputs.from_edges(300, np.stack([np.arange(299), np.arange(1, 300)], axis=1),
                                name="path300")]
    for g in graphs:
        print(f"[case] small tables: {g.name} n={g.n} m={g.m}", flush=True)
        t0 = time.perf_counter()
        ix = spc.build_graph(g)
        st = ix.stats()
        print(f"[case]   build {1e3 * (time.perf_counter() - t0):.0f} ms, "
              f"{st['round_kernel_launches']} round-kernel launches", flush=True)
        ref = oracle.build_graph(g, method="pull")
        assert_labels_equal(ix.export(), ref, g.name)
        rs = ix.round_stats()
        k = len(ref.stats["kept"])
        for key in ("raw", "merged", "kept"):
            assert np.array_equal(rs[key][:k], ref.stats[key]), (g.name, key)
        s, t = inputs.queries(g.n, 20000, seed=9)
        d, c, f = gpu_query(ix, s, t)
        rd, rc = ref.query(s, t)
        assert np.array_equal(d, rd) and np.array_equal(c, rc), g.name
        ix.free()
    batch = inputs.rmat_batch(12, seed=4, scale_lo=6, scale_hi=11)
    print(f"[case] small tables: batch of {len(batch)}", flush=True)
    ix = spc.build_index_batch(batch)
    for gi, g in enumerate(batch):
        assert_labels_equal(ix.export(gi), oracle.build_graph(g), g.name)
    # the reductions: the weighted pull (equivalence) and the core builds
    # (1-shell) through the same overflow paths
    import dataclasses
    for g in (inputs.rmat(12, 16, seed=5), inputs.rmat(11, 8, seed=4), inputs.chung_lu(1 << 12, seed=2)):
        for kind in ("equivalence", "one_shell"):
            print(f"[case] small tables {kind}: {g.name} n={g.n}", flush=True)
            ix = spc.build_graph(g, opts=spc.BuildOptions(**{kind: True}))
            if kind == "equivalence":
                red = oracle.build_twin_reduced(g.off, g.adj, order=g.order, tie_key=g.tie_key)
                ids = red.ids
            else:
                red = oracle.build_reduced(g.off, g.adj, order=g.order, tie_key=g.tie_key)
                ids = red.core_ids
            ref = dataclasses.replace(red.labels, order=ids[red.labels.order])
            assert_labels_equal(ix.export(), ref, f"{g.name} {kind}")
            s, t = inputs.queries(g.n, 20000, seed=9)
            d, c, f = gpu_query(ix, s, t)
            rd, rc = red.query(s, t)
            assert np.array_equal(d, rd) and np.array_equal(c, rc), (g.name, kind)
            ix.free()
    # PUSH rounds: the merged pushes through one virtual neighbour, same paths
    for g in (inputs.rmat(12, 16, seed=5), inputs.chung_lu(1 << 13, seed=2)):
        print(f"[case] small tables push: {g.name} n={g.n}", flush=True)
        ix = spc.build_graph(g, opts=spc.BuildOptions(propagation="push"))
        ref = oracle.build_graph(g, method="pull")
        assert_labels_equal(ix.export(), ref, f"{g.name} push")
        rs = ix.round_stats()
        k = len(ref.stats["kept"])
        for key in ("raw", "merged", "kept"):
            assert np.array_equal(rs[key][:k], ref.stats[key]), (g.name, key, "push")
        ix.free()
    print("small tables ok", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
