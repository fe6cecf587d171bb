"""Pins of the oracle's general truncated-series level push (oracle.series):
f_K = sum_{k<=K} c_k (A D^-1)^k s with positive coefficients (Eq. (1), Table 1).

* eps -> 0 (every nonzero residual active): x equals the truncated series
  computed densely term by term, for random positive coefficients;
* heat-kernel coefficients: x equals the truncated Taylor series of e^{-tau L}
  at eps -> 0, and at finite eps the level-push guarantee holds:
  0 <= f_K - x, ||D^-1 (f_K - x)||_inf <= eps, ||f_K - x||_1 equals the
  psi-weighted leftover (residual_l1);
* truncated PPR coefficients alpha (1-alpha)^k approach the PPR vector (Eq. (2))
  within the truncation tail plus the stop-rule error;
* invalid coefficients (zero, negative, non-finite) are rejected.
"""
import math

import numpy as np
import pytest

from oracle import exact as X
from oracle import solvers as O
from paper_2410_21634_amd import workloads as W

TINY = 1e-300


@pytest.fixture(scope="module")
def g300():
    return W.chung_lu(300, 1200, 2.5, seed=7)


def dense_series(A, c, s):
    M = X.walk_matrix(A)
    v = np.asarray(s, dtype=np.float64).copy()
    f = np.zeros_like(v)
    for ck in c:
        f += ck * v
        v = M @ v
    return f


def test_series_eps_to_zero_is_truncated_series(g300):
    G = g300
    A = X.dense_adjacency(G.row_ptr, G.col_idx)
    rng = np.random.default_rng(3)
    c = rng.uniform(0.05, 1.0, size=13)
    seeds = [int(v) for v in W.uniform_seeds(G, 3, seed=4)]
    s = np.zeros(G.n)
    s[seeds] = [0.5, 0.3, 0.2]
    res = O.series(G.row_ptr, G.col_idx, c, TINY, seeds, [0.5, 0.3, 0.2])
    np.testing.assert_allclose(res["x"], dense_series(A, c, s), rtol=1e-12, atol=1e-16)
    assert res["residual_l1"] == 0.0
    np.testing.assert_allclose(res["psi"], [c[k:].sum() / c[k] for k in range(len(c))], rtol=1e-14)


def test_series_heat_kernel_coefficients(g300):
    G = g300
    A = X.dense_adjacency(G.row_ptr, G.col_idx)
    tau, K = 5.0, 30
    c = np.array([math.exp(-tau) * tau**k / math.factorial(k) for k in range(K + 1)])
    seed = int(W.uniform_seeds(G, 1, seed=5)[0])
    s = np.zeros(G.n)
    s[seed] = 1.0
    fK = X.hk_taylor(A, tau, K, s)
    np.testing.assert_allclose(O.series(G.row_ptr, G.col_idx, c, TINY, [seed])["x"], fK, rtol=1e-12, atol=1e-16)
    d = A.sum(axis=1)
    for eps in (1e-3, 1e-5):
        res = O.series(G.row_ptr, G.col_idx, c, eps, [seed])
        gap = fK - res["x"]
        assert (gap >= -1e-15).all()
        assert (gap[d > 0] / d[d > 0] <= eps * (1 + 1e-12)).all()
        assert gap.sum() == pytest.approx(res["residual_l1"], rel=1e-10)
        assert res["residual_dinf"] < eps


def test_series_truncated_ppr_approaches_ppr(g300):
    G = g300
    A = X.dense_adjacency(G.row_ptr, G.col_idx)
    alpha, K, eps = 0.2, 120, 1e-6
    c = alpha * (1.0 - alpha) ** np.arange(K + 1)
    seed = int(W.uniform_seeds(G, 1, seed=6)[0])
    s = np.zeros(G.n)
    s[seed] = 1.0
    f = X.ppr_exact(A, alpha, s)
    res = O.series(G.row_ptr, G.col_idx, c, eps, [seed])
    # ||f - f_K||_1 = (1-alpha)^{K+1}; ||f_K - x||_1 = residual_l1
    assert np.abs(f - res["x"]).sum() <= (1 - alpha) ** (K + 1) + res["residual_l1"] + 1e-12


@pytest.mark.parametrize("bad", [[1.0, 0.0, 0.5], [1.0, -0.1], [1.0, float("nan")], [float("inf")]])
def test_series_rejects_bad_coefficients(g300, bad):
    with pytest.raises(ValueError):
        O.series(g300.row_ptr, g300.col_idx, np.array(bad), 1e-4, [0])


def sym_matrix(A):
    d = A.sum(axis=0)
    inv = np.where(d > 0, 1.0 / np.sqrt(np.where(d > 0, d, 1.0)), 0.0)
    return inv[:, None] * A * inv[None, :]


def test_symmetric_series_is_the_appnp_series(g300):
    # M = D^-1/2 A D^-1/2 (Table 1, APPNP): at eps -> 0 the transformed level push
    # equals sum_k c_k M^k s computed densely from M itself; at finite eps the
    # A D^-1 guarantee, scaled by D^-1/2, gives 0 <= f - x <= eps sqrt(d)
    G = g300
    A = X.dense_adjacency(G.row_ptr, G.col_idx)
    Ms = sym_matrix(A)
    d = np.diff(G.row_ptr).astype(float)
    c = 0.1 * 0.9 ** np.arange(21)
    seeds = [int(v) for v in W.uniform_seeds(G, 3, seed=8)]
    vals = [0.2, 0.7, 0.1]
    s = np.zeros(G.n)
    s[seeds] = vals
    f = np.zeros(G.n)
    v = s.copy()
    for ck in c:
        f += ck * v
        v = Ms @ v
    res = O.symmetric(O.series, G.row_ptr, G.col_idx, c, TINY, seed_idx=seeds, seed_val=vals)
    np.testing.assert_allclose(res["x"], f, rtol=1e-12, atol=1e-16)
    for eps in (1e-3, 1e-5):
        res = O.symmetric(O.series, G.row_ptr, G.col_idx, c, eps, seed_idx=seeds, seed_val=vals)
        gap = f - res["x"]
        assert (gap >= -1e-15).all() and (gap <= eps * np.sqrt(d) + 1e-15).all()
        if eps == 1e-3:
            assert (gap > eps * np.sqrt(d) * 1e-2).any()  # the stop rule left something behind


def test_symmetric_ppr_localgd(g300):
    # PPR with M = D^-1/2 A D^-1/2: f = alpha (I - (1 - alpha) M)^-1 s; LocalGD
    # through the transform stops with |f - x| <= eps sqrt(d) componentwise
    G = g300
    A = X.dense_adjacency(G.row_ptr, G.col_idx)
    Ms = sym_matrix(A)
    d = np.diff(G.row_ptr).astype(float)
    a = 0.15
    for s_node in W.uniform_seeds(G, 3, seed=9):
        s = np.zeros(G.n)
        s[int(s_node)] = 1.0
        f = a * np.linalg.solve(np.eye(G.n) - (1 - a) * Ms, s)
        for eps in (1e-4, 1e-7):
            res = O.symmetric(O.localgd, G.row_ptr, G.col_idx, O.PPR, a, eps, seed_idx=[int(s_node)])
            gap = f - res["x"]
            assert (gap >= -1e-14).all() and (gap <= eps * np.sqrt(d) + 1e-14).all()
        res = O.symmetric(O.localgd, G.row_ptr, G.col_idx, O.PPR, a, 1e-15, seed_idx=[int(s_node)])
        np.testing.assert_allclose(res["x"], f, rtol=1e-9, atol=1e-13)
