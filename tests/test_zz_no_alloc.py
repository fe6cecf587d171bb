"""gde_solve_noalloc (the plain solver on the library's fixed device array)
against gde_solve on the same queries, two calls in a row with the second on a
smaller graph, through the C ABI.

The no-allocation entry point always uses the atomic scatter, so it is compared
with gde_solve under GDE_SCATTER_ATOMIC: in FP64 the integer traces (T, sum
vol(S_t), sum |S_t|) must be equal and x must agree within 1e-12 of the
diffusion's mass; in FP32 x must agree within 1e-6 of it when the traces agree
(an FP32 value within rounding of its threshold may flip between two runs of
the atomic scatter; then the result must meet the FP32 stop certificate).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import exact as X  # noqa: E402
from paper_2410_21634_amd import workloads as W  # noqa: E402

from _parity import TOL, fp32_residual_bound, mass  # noqa: E402


@pytest.fixture(scope="module")
def gde():
    from paper_2410_21634_amd import gde as mod
    return mod


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def ctx(gde):
    c = gde.Context(0)
    yield c
    c.close()


def _queries(gde, G, beta, lam):
    seeds = [int(s) for s in W.uniform_seeds(G, 2, seed=7)]
    set8 = sorted(set(int(v) for v in W.uniform_seeds(G, 12, seed=8)))[:8]
    out = []
    for vt in (gde.F64, gde.F32):
        for s in seeds:
            out.append((gde.PPR, "ppr", "gd", dict(alpha=0.1, eps=1e-6), [s], vt))
            out.append((gde.PPR, "ppr", "ch", dict(alpha=0.1, eps=1e-6), [s], vt))
            out.append((gde.KATZ, "katz", "gd", dict(beta=beta, eps=1e-6, lambda_bound=lam), [s], vt))
            out.append((gde.KATZ, "katz", "ch", dict(beta=beta, eps=1e-6, lambda_bound=lam), [s], vt))
            out.append((gde.HK, "hk", "gd", dict(tau=5.0, K=30, eps=1e-6), [s], vt))
        out.append((gde.PPR, "ppr", "gd", dict(alpha=0.1, eps=1e-7), set8, vt))
    return out


def _compare(gde, torch, ctx, g, G, beta, lam):
    dev = torch.device("cuda:0")
    for kind, kname, method, prm, seeds, vt in _queries(gde, G, beta, lam):
        tdt = torch.float64 if vt == gde.F64 else torch.float32
        flags = gde.SCATTER_ATOMIC
        p = gde.make_params(kname, method, value_type=vt, flags=flags, **prm)
        oi = torch.empty(G.n, dtype=torch.int32, device=dev)
        ov = torch.empty(G.n, dtype=tdt, device=dev)
        ref = gde.solve(ctx, g, p, seeds, out=(oi, ov))
        ni = torch.full((G.n,), -1, dtype=torch.int32, device=dev)
        nv = torch.full((G.n,), -1.0, dtype=tdt, device=dev)
        q = gde.make_params(kname, method, value_type=vt, **prm)
        got = gde.solve_noalloc(g, q, seeds, out=(ni, nv))
        torch.cuda.synchronize()
        xr, xg = ref.dense(G.n), got.dense(G.n)
        m = mass(kind, np.ones(len(seeds)), xr)
        err = float(np.abs(xg - xr).sum()) / m
        same = (got.iters, got.ops, got.pushes) == (ref.iters, ref.ops, ref.pushes)
        print("noalloc", G.n, kname, method, vt, seeds[:2], "iters", got.iters, ref.iters, "ops", got.ops, ref.ops,
              "l1", err, flush=True)
        assert got.status == ref.status == gde.OK
        assert np.all(np.diff(got.idx.cpu().numpy()) > 0)
        if vt == gde.F64:
            assert same, (kname, method, seeds)
            assert err <= TOL[vt], (kname, method, err)
            np.testing.assert_allclose(got.residual_l1, ref.residual_l1, rtol=1e-10, atol=1e-300)
        elif same:
            assert err <= TOL[vt], (kname, method, err)
        else:
            assert kind != gde.HK, "heat-kernel FP32 trace flip"
            sv = np.ones(len(seeds))
            param = prm["alpha"] if kind == gde.PPR else prm["beta"]
            bound = fp32_residual_bound(G.row_ptr, G.col_idx, kind, param, prm["eps"], xg, got.iters)
            r = X.residual(G.row_ptr, G.col_idx, kind, param, np.array(seeds), sv, xg)
            assert (np.abs(r) <= bound).all(), (kname, method)


def _graph(gde, ctx, torch, G):
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(G.row_ptr).to(dev)
    ci = torch.from_numpy(G.col_idx).to(dev)
    return gde.Graph(ctx, rp, ci), (rp, ci)


def test_noalloc_matches_gde_solve_twice(gde, torch, ctx):
    """First call on the 10,000-node graph, second on a 2,000-node graph."""
    for n, e, gam, seed in ((10000, 50000, 2.5, 42), (2000, 10000, 2.3, 5)):
        G = W.chung_lu(n, e, gam, seed=seed)
        g, keep = _graph(gde, ctx, torch, G)
        lo, hi = X.lambda_bounds_power(G.row_ptr, G.col_idx, iters=200)
        _compare(gde, torch, ctx, g, G, 0.5 / lo, hi * 1.0001)
        g.close()


def test_noalloc_limits(gde, torch, ctx):
    """A graph whose workspace exceeds the fixed array is refused before any
    device work; host results and traces are refused; a small solve still
    works after the refusals."""
    G = W.from_edges(2_000_000, [(i, i + 1) for i in range(0, 2_000_000 - 1, 2)])
    g, keep = _graph(gde, ctx, torch, G)
    p = gde.make_params("ppr", alpha=0.1, eps=1e-4, value_type=gde.F64)
    assert gde.noalloc_bytes(g, p, [0]) > gde.NOALLOC_SCRATCH_BYTES
    dev = torch.device("cuda:0")
    oi = torch.empty(16, dtype=torch.int32, device=dev)
    ov = torch.empty(16, dtype=torch.float64, device=dev)
    r = gde.solve_noalloc(g, p, [0], out=(oi, ov), raise_on_error=False)
    assert r.status == gde.OOM and "fixed array" in gde.last_error()
    g.close()
    G2 = W.chung_lu(2000, 10000, 2.3, seed=5)
    g2, keep2 = _graph(gde, ctx, torch, G2)
    pt = gde.make_params("ppr", alpha=0.1, eps=1e-4, value_type=gde.F64, flags=gde.TRACE)
    oi = torch.empty(G2.n, dtype=torch.int32, device=dev)
    ov = torch.empty(G2.n, dtype=torch.float64, device=dev)
    assert gde.solve_noalloc(g2, pt, [1], out=(oi, ov), raise_on_error=False).status == gde.UNSUPPORTED
    p2 = gde.make_params("ppr", alpha=0.1, eps=1e-4, value_type=gde.F64)
    s = int(np.argmax(G2.degrees))
    got = gde.solve_noalloc(g2, p2, [s], out=(oi, ov))
    ref = gde.solve(ctx, g2, gde.make_params("ppr", alpha=0.1, eps=1e-4, value_type=gde.F64,
                                              flags=gde.SCATTER_ATOMIC), [s])
    assert (got.iters, got.ops) == (ref.iters, ref.ops)
    assert np.abs(got.dense(G2.n) - ref.dense(G2.n)).sum() <= 1e-12
    g2.close()
