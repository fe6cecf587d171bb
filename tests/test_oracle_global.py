"""Pins of the oracle's global solvers (the standard GD / Chebyshev counterparts
of Table 2 and of the eps sweep of Sec. 5) against facts fixed by the
mathematics, on small graphs with dense matrices:

* global GD after T iterations is the truncated Neumann series
  x_T = sum_{k<T} (I - Q)^k b with residual (I - Q)^T b, and T is the first
  iteration count after which no node satisfies |r_u| >= theta_u;
* global CH after T iterations has the residual of the Chebyshev residual
  polynomial T_T((L+mu-2Q)/(L-mu)) b / T_T((L+mu)/(L-mu)) (Sec. 3.3), and
  x_T = Q^-1 (b - r_T);
* ops = T * nnz and pushes = T * n; for PPR, 0 <= f - x = Q^-1 r (the error
  bound the stop rule gives, Theorem 3.2 with S_t = V).
"""
import numpy as np
import pytest

from oracle import exact as X
from oracle import solvers as O
from paper_2410_21634_amd import workloads as W

PPR, KATZ = O.PPR, O.KATZ


@pytest.fixture(scope="module")
def g300():
    return W.chung_lu(300, 1200, 2.5, seed=7)


def _dense(G):
    A = X.dense_adjacency(G.row_ptr, G.col_idx)
    d = A.sum(axis=1)
    return A, d


def _Qb(A, d, kind, param, s):
    n = len(d)
    if kind == PPR:
        P = A / np.where(d > 0, d, 1.0)[None, :]
        return np.eye(n) - (1.0 - param) * P, param * s
    return np.eye(n) - param * A, s.copy()


def _largest_component_seed(G):
    return int(W.uniform_seeds(G, 1, seed=3)[0])


@pytest.mark.parametrize("kind,param,eps", [(PPR, 0.1, 1e-5), (PPR, 0.25, 1e-3), (KATZ, None, 1e-6)])
def test_global_gd_is_truncated_neumann(g300, kind, param, eps):
    G = g300
    A, d = _dense(G)
    if kind == KATZ:
        param = 0.5 / np.linalg.eigvalsh(A)[-1]
    s = np.zeros(G.n)
    seed = _largest_component_seed(G)
    s[seed] = 1.0
    res = O.global_gd_ch(G.row_ptr, G.col_idx, 0, kind, param, eps, [seed])
    T = res["iters"]
    assert res["status"] == O.OK and T >= 1
    Q, b = _Qb(A, d, kind, param, s)
    M = np.eye(G.n) - Q
    xs = X.neumann_ppr(A, param, s, T) if kind == PPR else X.neumann_katz(A, param, s, T)
    np.testing.assert_allclose(res["x"], xs, rtol=1e-12, atol=1e-15)
    # T is the first count after which no node is active: r_k = M^k b
    eff = param * eps if kind == PPR else eps
    r = b.copy()
    for k in range(1, T + 1):
        r = M @ r
        active = (r != 0) & (np.abs(r) >= eff * d)
        assert active.any() == (k < T), (k, T)
    np.testing.assert_allclose(res["r"], r, rtol=1e-10, atol=1e-16)
    assert res["ops"] == T * len(G.col_idx) and res["pushes"] == T * G.n
    if kind == PPR:
        f = np.linalg.solve(Q, b)
        assert (f - res["x"] >= -1e-15).all()
        np.testing.assert_allclose(f - res["x"], np.linalg.solve(Q, res["r"]), atol=1e-13)


@pytest.mark.parametrize("kind,eps", [(PPR, 1e-7), (KATZ, 1e-7)])
def test_global_ch_is_chebyshev_residual_polynomial(g300, kind, eps):
    G = g300
    A, d = _dense(G)
    s = np.zeros(G.n)
    seed = _largest_component_seed(G)
    s[seed] = 1.0
    if kind == PPR:
        param, lam = 0.1, 0.0
        mu, L = 0.1, 1.9
    else:
        ev = np.linalg.eigvalsh(A)
        lam = max(ev[-1], -ev[0]) * 1.0001
        param = 0.5 / ev[-1]
        mu, L = 1.0 - param * lam, 1.0 + param * lam
    res = O.global_gd_ch(G.row_ptr, G.col_idx, 1, kind, param, eps, [seed], lam=lam)
    T = res["iters"]
    assert res["status"] == O.OK and T >= 2
    Q, b = _Qb(A, d, kind, param, s)
    r_T = X.chebyshev_residual(Q, b, mu, L, T)
    np.testing.assert_allclose(res["r"], r_T, atol=1e-12 * np.abs(b).sum())
    np.testing.assert_allclose(res["x"], np.linalg.solve(Q, b - res["r"]), atol=1e-11)
    # Chebyshev needs fewer iterations than GD for the same stop rule
    gd = O.global_gd_ch(G.row_ptr, G.col_idx, 0, kind, param, eps, [seed])
    assert T < gd["iters"]


def test_global_stop_rule_and_norms(g300):
    G = g300
    seed = _largest_component_seed(G)
    for method in (0, 1):
        res = O.global_gd_ch(G.row_ptr, G.col_idx, method, PPR, 0.1, 1e-6, [seed])
        d = np.diff(G.row_ptr).astype(float)
        rt = res["r"] / 0.1
        assert (np.abs(rt[d > 0]) / d[d > 0] < 1e-6).all()
        assert res["residual_l1"] == pytest.approx(np.abs(rt).sum(), rel=1e-12)
        assert res["residual_dinf"] == pytest.approx((np.abs(rt[d > 0]) / d[d > 0]).max(), rel=1e-12)
    # the iteration cap
    capped = O.global_gd_ch(G.row_ptr, G.col_idx, 0, PPR, 0.1, 1e-9, [seed], max_iters=3)
    assert capped["status"] == O.NOT_CONVERGED and capped["iters"] == 3
