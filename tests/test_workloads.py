"""The seeded synthetic inputs: determinism and graph well-formedness."""
import numpy as np

from paper_2410_21634_amd import workloads as W


def test_chung_lu_deterministic_and_simple():
    a = W.chung_lu(5000, 25000, 2.5, seed=42)
    b = W.chung_lu(5000, 25000, 2.5, seed=42)
    c = W.chung_lu(5000, 25000, 2.5, seed=43)
    assert a.sha256() == b.sha256() != c.sha256()
    assert a.nnz == 50000
    rp, ci = a.row_ptr, a.col_idx
    rows = np.repeat(np.arange(a.n), np.diff(rp))
    assert (ci != rows).all()                                   # no self-loops
    for u in range(0, a.n, 97):                                 # ascending, no duplicates
        row = ci[rp[u]:rp[u + 1]]
        assert (np.diff(row) > 0).all()
    key = rows.astype(np.int64) * a.n + ci
    rkey = ci.astype(np.int64) * a.n + rows
    assert np.array_equal(np.sort(key), np.sort(rkey))          # symmetric


def test_power_law_shape():
    g = W.chung_lu(20000, 100000, 2.5, seed=1)
    d = g.degrees
    assert d.max() > 10 * d.mean()
    assert abs(d.mean() - 10.0) < 1e-9


def test_seed_samplers():
    g = W.chung_lu(5000, 25000, 2.5, seed=42)
    s = W.uniform_seeds(g, 64)
    assert len(np.unique(s)) == 64 and (g.degrees[s] > 0).all()
    st = W.stratified_seeds(g, 64, bins=8)
    assert len(np.unique(st)) == 64
    eps = W.log_uniform_eps(1000)
    assert eps.min() >= 1e-7 and eps.max() <= 1e-4
    idx, val = W.seed_set(g, int(s[0]), 8)
    assert len(idx) == 8 and (np.diff(idx) > 0).all() and abs(val.sum() - 1) < 1e-15
    t = W.poisson_arrivals(1000.0, 1.0)
    assert 850 < len(t) < 1150 and (np.diff(t) > 0).all()
    rng = np.random.default_rng(0)
    u, v = W.insert_batch(g, 100, rng)
    assert (u < v).all() and len(set(zip(u.tolist(), v.tolist()))) == 100


def test_grid_2d_matches_edge_list():
    from paper_2410_21634_amd import workloads as W
    rows, cols = 5, 7
    edges = [(i * cols + j, i * cols + j + 1) for i in range(rows) for j in range(cols - 1)]
    edges += [(i * cols + j, (i + 1) * cols + j) for i in range(rows - 1) for j in range(cols)]
    G, H = W.grid_2d(rows, cols), W.from_edges(rows * cols, edges)
    assert np.array_equal(G.row_ptr, H.row_ptr) and np.array_equal(G.col_idx, H.col_idx)
    big = W.grid_2d(1000, 1000)
    assert big.n == 10**6 and big.nnz == 2 * 1_998_000


def test_snapshots_insert_then_delete_sequence():
    from paper_2410_21634_amd import workloads as W
    G = W.chung_lu(3000, 15000, 2.5, seed=5)
    u, v = W.edge_arrays(G)
    H = W.from_edge_arrays(G.n, u, v)
    assert np.array_equal(G.row_ptr, H.row_ptr) and np.array_equal(G.col_idx, H.col_idx)
    protect = [int(s) for s in W.uniform_seeds(G, 4, seed=1)]
    g0, batches = W.snapshots(G, 8, 0.179, 0.1, seed=7, protect=protect)
    g0b, _ = W.snapshots(G, 8, 0.179, 0.0, seed=7)
    assert np.array_equal(g0.col_idx, g0b.col_idx)  # graph 0 does not depend on the deletions
    E = set(zip(*W.edge_arrays(g0)))
    assert len(E) == round(0.179 * len(u))
    for iu, iv, du, dv in batches:
        for a, b in zip(du.tolist(), dv.tolist()):
            assert (a, b) in E and a not in protect and b not in protect
            E.discard((a, b))
        for a, b in zip(iu.tolist(), iv.tolist()):
            assert (a, b) not in E
            E.add((a, b))
    assert len(E) == len(u) - sum(len(b[2]) for b in batches)
