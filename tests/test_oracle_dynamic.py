"""Pins of the oracle's dynamic-graph functions and of the global PPR reference.

* ``exact.global_ppr`` (the "exact f" used where a dense solve is too large)
  against the dense solve of Eq. (2).
* ``solvers.edge_events`` (the Insert / Delete procedures of LocalGS(Dynamic)
  and LocalSOR(Dynamic), Sec. 4, in the generic form; Katz derived): after any
  batch of events the state must satisfy r = b - Q_new x, recomputed here from
  the new graph's dense matrices -- exact up to rounding.  A missing, mis-signed
  or misdirected correction breaks that identity, which the sensitivity checks
  below confirm.
* ``solvers.localgd_warm`` (the re-solve that follows the corrections): its
  result meets the stop rule and the Theorem 3.2 bound on the new graph.
"""
import numpy as np
import pytest

from oracle import exact as X
from oracle import solvers as O
from paper_2410_21634_amd import workloads as W

PPR, KATZ = O.PPR, O.KATZ


def edge_set(G):
    s = set()
    for a in range(G.n):
        for b in G.col_idx[G.row_ptr[a]:G.row_ptr[a + 1]]:
            if a < b:
                s.add((a, int(b)))
    return s


def residual_of(G, kind, param, svec, x):
    """r = b - Q x from the dense matrices of G (the definition, Eqs. (2)-(4))."""
    A = X.dense_adjacency(G.row_ptr, G.col_idx)
    if kind == PPR:
        return param * svec - (x - (1.0 - param) * (X.walk_matrix(A) @ x))
    return svec - (x - param * (A @ x))


@pytest.fixture(scope="module")
def g300():
    return W.chung_lu(300, 1200, 2.5, seed=7)


@pytest.mark.parametrize("seed", [3, 41])
def test_global_ppr_matches_dense_solve(seed):
    G = W.chung_lu(2000, 10000, 2.5, seed=seed)
    A = X.dense_adjacency(G.row_ptr, G.col_idx)
    for s in W.uniform_seeds(G, 3, seed=seed):
        svec = X.seed_vector(G.n, [s])
        f = X.ppr_exact(A, 0.1, svec)
        g = X.global_ppr(G.row_ptr, G.col_idx, 0.1, svec, tol=1e-14)
        assert np.abs(f - g).sum() <= 1e-12
        # a seed set with unequal weights, and a looser tolerance that must still
        # leave at most tol * ||s||_1 of mass unaccounted for
        sv = X.seed_vector(G.n, [s, (s + 1) % G.n], [0.25, 0.75])
        f2 = X.ppr_exact(A, 0.1, sv)
        g2 = X.global_ppr(G.row_ptr, G.col_idx, 0.1, sv, tol=1e-6)
        assert np.abs(f2 - g2).sum() <= 1e-6 * sv.sum() / 0.1


def _events(G, rng, k_ins, k_del):
    """k_ins new edges and k_del existing ones (one chosen to isolate a leaf)."""
    E = edge_set(G)
    d = np.diff(G.row_ptr)
    ins = []
    while len(ins) < k_ins:
        a, b = sorted(int(v) for v in rng.integers(0, G.n, 2))
        if a != b and (a, b) not in E and (a, b) not in ins:
            ins.append((a, b))
    leaf = int(np.flatnonzero(d == 1)[0])
    nb = int(G.col_idx[G.row_ptr[leaf]])
    dels = [tuple(sorted((leaf, nb)))]
    pool = sorted(E - set(dels))
    for j in rng.choice(len(pool), k_del - 1, replace=False):
        dels.append(pool[j])
    return ins, dels, leaf


@pytest.mark.parametrize("kind", [PPR, KATZ])
def test_edge_events_keep_r_exact(g300, kind):
    G = g300
    rng = np.random.default_rng(5)
    A0 = X.dense_adjacency(G.row_ptr, G.col_idx)
    lam = float(np.max(np.abs(np.linalg.eigvalsh(A0))))
    param = 0.1 if kind == PPR else 0.25 / lam
    s = int(W.uniform_seeds(G, 1, seed=5)[0])
    svec = X.seed_vector(G.n, [s])
    res = O.localgd(G.row_ptr, G.col_idx, kind, param, 1e-5, [s])
    x, r = res["x"], res["r"]
    np.testing.assert_allclose(residual_of(G, kind, param, svec, x), r, atol=1e-15)
    ins, dels, leaf = _events(G, rng, 40, 30)
    E = edge_set(G)
    deg = np.diff(G.row_ptr).astype(np.int64)
    # inserts, then deletes (some of them of edges just inserted)
    x1, r1, deg1 = O.edge_events(kind, param, x, r, deg, [e[0] for e in ins], [e[1] for e in ins], +1)
    G1 = W.from_edges(G.n, sorted(E | set(ins)))
    assert np.array_equal(deg1, np.diff(G1.row_ptr))
    np.testing.assert_allclose(residual_of(G1, kind, param, svec, x1), r1, atol=1e-14)
    dels = dels + ins[:5]
    x2, r2, deg2 = O.edge_events(kind, param, x1, r1, deg1, [e[0] for e in dels], [e[1] for e in dels], -1)
    G2 = W.from_edges(G.n, sorted((E | set(ins)) - set(dels)))
    assert np.array_equal(deg2, np.diff(G2.row_ptr)) and deg2[leaf] == 0
    np.testing.assert_allclose(residual_of(G2, kind, param, svec, x2), r2, atol=1e-14)
    if kind == PPR:
        assert x2[leaf] == 0.0  # an isolated node's x is returned to its residual
    # sensitivity: no correction, or the opposite procedure, breaks r = b - Q_new x by far more than rounding
    assert np.abs(residual_of(G1, kind, param, svec, x) - r).max() > 1e-8
    xw, rw, _ = O.edge_events(kind, param, x, r, deg, [e[0] for e in ins], [e[1] for e in ins], -1)
    assert np.abs(residual_of(G1, kind, param, svec, xw) - rw).max() > 1e-8


def test_edge_event_on_an_isolated_node():
    # 0-1 plus isolated 2; x_2 = 0 and r_2 = 0; inserting (1, 2) then (0, 2)
    G = W.from_edges(3, [(0, 1)])
    svec = X.seed_vector(3, [0])
    res = O.localgd(G.row_ptr, G.col_idx, PPR, 0.1, 1e-8, [0])
    x, r = res["x"], res["r"]
    deg = np.diff(G.row_ptr).astype(np.int64)
    x1, r1, deg1 = O.edge_events(PPR, 0.1, x, r, deg, [1, 0], [2, 2], +1)
    G1 = W.from_edges(3, [(0, 1), (1, 2), (0, 2)])
    np.testing.assert_allclose(residual_of(G1, PPR, 0.1, svec, x1), r1, atol=1e-15)
    # node 1 had degree 1: its x is scaled by 2/1 and gives back x_1 / 1 to r_1
    assert x1[1] == pytest.approx(2 * x[1]) and x1[2] == 0.0
    with pytest.raises(ValueError):  # deleting a missing edge at a degree-0 node
        O.edge_events(PPR, 0.1, x, r, deg, [2], [1], -1)


@pytest.mark.parametrize("kind", [PPR, KATZ])
def test_warm_resolve_meets_the_new_graph_bounds(g300, kind):
    G = g300
    rng = np.random.default_rng(9)
    A0 = X.dense_adjacency(G.row_ptr, G.col_idx)
    lam = float(np.max(np.abs(np.linalg.eigvalsh(A0))))
    param = 0.1 if kind == PPR else 0.25 / lam
    eps = 1e-5
    for s in W.uniform_seeds(G, 3, seed=9):
        svec = X.seed_vector(G.n, [s])
        res = O.localgd(G.row_ptr, G.col_idx, kind, param, eps, [s])
        # no events: the state already meets the stop rule, nothing runs
        same = O.localgd_warm(G.row_ptr, G.col_idx, kind, param, eps, res["x"], res["r"])
        assert same["iters"] == 0 and np.array_equal(same["x"], res["x"])
        ins, dels, _ = _events(G, rng, 25, 25)
        E = edge_set(G)
        deg = np.diff(G.row_ptr).astype(np.int64)
        x, r, deg = O.edge_events(kind, param, res["x"], res["r"], deg, [e[0] for e in ins], [e[1] for e in ins], +1)
        x, r, deg = O.edge_events(kind, param, x, r, deg, [e[0] for e in dels], [e[1] for e in dels], -1)
        G2 = W.from_edges(G.n, sorted((E | set(ins)) - set(dels)))
        d2 = np.diff(G2.row_ptr).astype(float)
        w = O.localgd_warm(G2.row_ptr, G2.col_idx, kind, param, eps, x, r)
        assert w["status"] == O.OK
        np.testing.assert_allclose(residual_of(G2, kind, param, svec, w["x"]), w["r"], atol=1e-14)
        sc = 1.0 / param if kind == PPR else 1.0
        act = np.abs(w["r"]) * sc >= eps * d2
        assert not (act & (w["r"] != 0)).any()                        # stop rule on the new graph
        A2 = X.dense_adjacency(G2.row_ptr, G2.col_idx)
        if kind == PPR:
            f = X.ppr_exact(A2, param, svec)
            # Theorem 3.2 with signed residuals: |f - x| = |Pi r~| <= eps d (Prop. B.1 symmetry)
            assert (np.abs(f - w["x"]) <= eps * d2 + 1e-14).all()
        else:
            f = X.katz_exact(A2, param, svec)
            np.testing.assert_allclose(f - w["x"], np.linalg.solve(np.eye(G.n) - param * A2, w["r"]), atol=1e-12)
