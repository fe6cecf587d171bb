"""GPU parity of the plain solver (through the C ABI) against the FP64 oracle.

Graphs span several push tiles (1024 edges) and ragged tails; seeds include
single nodes, hubs, leaves and 8-node seed sets.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import exact as X  # noqa: E402
from paper_2410_21634_amd import workloads as W  # noqa: E402

from _parity import check  # noqa: E402


@pytest.fixture(scope="module")
def gde():
    from paper_2410_21634_amd import gde as mod
    return mod


@pytest.fixture(scope="module")
def ctx(gde):
    c = gde.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c1(gde, ctx):
    """n = 10,000, gamma = 2.5, average degree 10, seed 42 (the small PPR workload)."""
    G = W.chung_lu(10000, 50000, 2.5, seed=42)
    return G, gde.Graph(ctx, G.row_ptr, G.col_idx)


@pytest.fixture(scope="module")
def g2k(gde, ctx):
    G = W.chung_lu(2000, 10000, 2.3, seed=5)
    return G, gde.Graph(ctx, G.row_ptr, G.col_idx)


def seeds_of(G, k=4, seed=1):
    s = list(W.uniform_seeds(G, k, seed=seed))
    d = G.degrees
    s.append(int(np.argmax(d)))  # the hub
    return sorted(set(int(v) for v in s))


@pytest.mark.parametrize("vt", [1, 0])  # F64 then F32
@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_ppr_localgd(gde, ctx, c1, vt, eps):
    G, g = c1
    for s in seeds_of(G):
        rep = check(ctx, g, G, gde.PPR, gde.LOCAL_GD, vt, dict(alpha=0.1, eps=eps), [s])
        print("ppr-gd", vt, eps, s, rep, flush=True)


@pytest.mark.parametrize("vt", [1, 0])
def test_ppr_seed_set(gde, ctx, c1, vt):
    G, g = c1
    rng = np.random.default_rng(3)
    for a in W.uniform_seeds(G, 3, seed=7):
        idx, val = W.seed_set(G, int(a), 8, rng)
        rep = check(ctx, g, G, gde.PPR, gde.LOCAL_GD, vt, dict(alpha=0.1, eps=1e-6), idx, val)
        print("ppr-set", vt, rep, flush=True)


@pytest.mark.parametrize("vt", [1, 0])
def test_katz_localgd(gde, ctx, g2k, vt):
    G, g = g2k
    A = X.dense_adjacency(G.row_ptr, G.col_idx)
    lo, hi = X.adjacency_eig_bounds(A)
    lam = max(hi, -lo)
    beta = 0.5 / lam
    for s in seeds_of(G, 3, seed=2):
        for eps in (1e-4, 1e-6):
            rep = check(ctx, g, G, gde.KATZ, gde.LOCAL_GD, vt, dict(beta=beta, eps=eps, lambda_bound=lam * 1.001), [s])
            print("katz-gd", vt, eps, s, rep, flush=True)


@pytest.mark.parametrize("vt", [1, 0])
def test_hk_level_push(gde, ctx, c1, vt):
    G, g = c1
    for s in seeds_of(G, 3, seed=4):
        for eps in (1e-4, 1e-6):
            rep = check(ctx, g, G, gde.HK, gde.LOCAL_GD, vt, dict(tau=5.0, K=30, eps=eps), [s])
            print("hk", vt, eps, s, rep, flush=True)


@pytest.mark.parametrize("vt", [1, 0])
def test_localch(gde, ctx, g2k, vt):
    G, g = g2k
    A = X.dense_adjacency(G.row_ptr, G.col_idx)
    lo, hi = X.adjacency_eig_bounds(A)
    lam = max(hi, -lo) * 1.001
    for s in seeds_of(G, 3, seed=6):
        rep = check(ctx, g, G, gde.PPR, gde.LOCAL_CH, vt, dict(alpha=0.1, eps=1e-6), [s])
        print("ppr-ch", vt, s, rep, flush=True)
        rep = check(ctx, g, G, gde.KATZ, gde.LOCAL_CH, vt, dict(beta=0.5 / lam, eps=1e-6, lambda_bound=lam), [s])
        print("katz-ch", vt, s, rep, flush=True)


def test_tiny_graphs_exact(gde, ctx):
    # 2-node graph: the closed-form trace (T = 132) must come out of the GPU too
    G = W.from_edges(2, [(0, 1)])
    g = gde.Graph(ctx, G.row_ptr, G.col_idx)
    res = gde.solve(ctx, g, gde.make_params("ppr", alpha=0.1, eps=1e-6, value_type=gde.F64), [0])
    assert res.iters == 132 and res.ops == 132
    np.testing.assert_allclose(res.dense(2), [0.52631531, 0.47368378], atol=1e-8)
    star = W.from_edges(5, [(0, j) for j in range(1, 5)])
    gs = gde.Graph(ctx, star.row_ptr, star.col_idx)
    for vt in (gde.F64, gde.F32):
        rep = check(ctx, gs, star, gde.PPR, gde.LOCAL_GD, vt, dict(alpha=0.1, eps=1e-8), [1])
        assert rep["l1_err_vs_oracle"] < (1e-12 if vt == gde.F64 else 1e-6)


def test_status_paths(gde, ctx, c1):
    G, g = c1
    s = int(W.uniform_seeds(G, 1, seed=9)[0])
    # max_iters = 1 -> NOT_CONVERGED with a valid result
    p = gde.make_params("ppr", alpha=0.1, eps=1e-6, max_iters=1, value_type=gde.F64)
    res = gde.solve(ctx, g, p, [s])
    assert res.status == gde.NOT_CONVERGED and res.iters == 1 and len(res.idx) == 1
    # capacity too small -> CAPACITY, nnz needed reported, workspace left clean
    p = gde.make_params("ppr", alpha=0.1, eps=1e-6, value_type=gde.F64)
    r1 = gde.solve(ctx, g, p, [s], capacity=2, raise_on_error=False)
    assert r1.status == gde.CAPACITY and r1.extra["nnz_needed"] > 2
    r2 = gde.solve(ctx, g, p, [s])
    assert r2.status == gde.OK and len(r2.idx) == r1.extra["nnz_needed"]
    r3 = gde.solve(ctx, g, p, [s])
    np.testing.assert_array_equal(r2.idx, r3.idx)
    # isolated seed
    iso = int(np.flatnonzero(G.degrees == 0)[0])
    with pytest.raises(gde.GDEError):
        gde.solve(ctx, g, p, [iso])
    # Katz centrality option subtracts the seed
    A_lam = 1.0 / 0.01
    pk = gde.make_params("katz", beta=0.004, eps=1e-6, lambda_bound=A_lam, value_type=gde.F64)
    a = gde.solve(ctx, g, pk, [s]).dense(G.n)
    pk.flags = gde.KATZ_SUBTRACT_SEED
    b = gde.solve(ctx, g, pk, [s]).dense(G.n)
    assert abs(a[s] - b[s] - 1.0) < 1e-12


def test_device_output_and_torch_graph(gde, ctx, c1):
    import torch
    G, _ = c1
    rp = torch.from_numpy(G.row_ptr).cuda()
    ci = torch.from_numpy(G.col_idx).cuda()
    g = gde.Graph(ctx, rp, ci)
    s = int(W.uniform_seeds(G, 1, seed=11)[0])
    p = gde.make_params("ppr", alpha=0.1, eps=1e-6, value_type=gde.F32)
    oi = torch.zeros(G.n, dtype=torch.int32, device="cuda")
    ov = torch.zeros(G.n, dtype=torch.float32, device="cuda")
    res = gde.solve(ctx, g, p, [s], out=(oi, ov))
    host = gde.solve(ctx, g, p, [s])
    assert len(res.idx) == len(host.idx)
    np.testing.assert_array_equal(res.idx.cpu().numpy(), host.idx)
    np.testing.assert_allclose(res.val.cpu().numpy(), host.val, rtol=1e-5, atol=1e-9)
    # device buffers too small: CAPACITY with the size needed, and nothing written
    need = len(host.idx)
    oi.fill_(-7)
    ov.fill_(-7.0)
    small = gde.solve(ctx, g, p, [s], out=(oi, ov), capacity=need - 1, raise_on_error=False)
    assert small.status == gde.CAPACITY and small.extra["nnz_needed"] == need
    assert int((oi != -7).sum()) == 0 and int((ov != -7.0).sum()) == 0
    # and the workspace is clean afterwards: the same solve again gives the same answer
    again = gde.solve(ctx, g, p, [s], out=(oi, ov))
    np.testing.assert_array_equal(again.idx.cpu().numpy(), host.idx)


def test_lambda_bounds(gde, ctx, g2k):
    G, g = g2k
    lo, hi = g.lambda_max(max_iters=2000, rtol=1e-6)
    A = X.dense_adjacency(G.row_ptr, G.col_idx)
    ev = np.linalg.eigvalsh(A)
    lam = max(ev[-1], -ev[0])
    assert lo <= ev[-1] * (1 + 1e-12) and hi >= lam * (1 - 1e-12)
    assert (hi - lo) / hi < 0.05


@pytest.mark.parametrize("vt", [1, 0])
@pytest.mark.parametrize("strategy", ["binned", "atomic"])
def test_scatter_strategies(gde, ctx, c1, g2k, vt, strategy):
    """Every iteration binned (destination-range bins summed in LDS) or every
    iteration atomic: the same iteration either way, for all kinds and methods."""
    G, g = c1
    f = gde.SCATTER_BINNED if strategy == "binned" else gde.SCATTER_ATOMIC
    for s in seeds_of(G, k=2, seed=3):
        for method in (gde.LOCAL_GD, gde.LOCAL_CH):
            rep = check(ctx, g, G, gde.PPR, method, vt, dict(alpha=0.1, eps=1e-6), [s], extra_flags=f)
            print("scatter", strategy, vt, method, s, rep, flush=True)
        rep = check(ctx, g, G, gde.HK, gde.LOCAL_GD, vt, dict(tau=5.0, K=30, eps=1e-6), [s], extra_flags=f)
        print("scatter hk", strategy, vt, s, rep, flush=True)
    G2, g2 = g2k
    A = X.dense_adjacency(G2.row_ptr, G2.col_idx)
    ev = np.linalg.eigvalsh(A)
    lam = max(ev[-1], -ev[0])
    for s in seeds_of(G2, k=2, seed=4):
        for method in (gde.LOCAL_GD, gde.LOCAL_CH):
            rep = check(ctx, g2, G2, gde.KATZ, method, vt, dict(beta=0.5 / lam, eps=1e-6, lambda_bound=lam * 1.001),
                        [s], extra_flags=f)
            print("scatter katz", strategy, vt, method, s, rep, flush=True)
