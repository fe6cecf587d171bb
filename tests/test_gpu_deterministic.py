"""Deterministic mode (GDE_DETERMINISTIC): every floating-point operation of an
iteration in a fixed order -- at each node the updates arrive in ascending order
of the pushed node, its own change at its place -- which is the sequential
order of the FP64 oracle.  So:

* FP64: x equals the oracle's x bit for bit (dense comparison with ==), the
  integer traces are equal, and the residual norms agree to rounding (they are
  summed in a different order);
* FP32: two runs are bit-identical (x, support, traces, norms), and the result
  passes the ordinary parity protocol against the FP64 oracle;
* gde_solve_batch with the flag gives what gde_solve gives, bit for bit; the
  server refuses the flag.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import exact as X  # noqa: E402
from paper_2410_21634_amd import workloads as W  # noqa: E402

from _parity import check, oracle_run  # noqa: E402


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
    G = W.chung_lu(10000, 50000, 2.5, seed=42)
    return G, gde.Graph(ctx, G.row_ptr, G.col_idx)


@pytest.fixture(scope="module")
def katz_beta(c1):
    G, _ = c1
    lo, hi = X.lambda_bounds_power(G.row_ptr, G.col_idx, iters=200)
    return 0.5 / lo, hi * 1.0001


def queries(G, beta, lam):
    seeds = [int(s) for s in W.uniform_seeds(G, 3, seed=4)] + [int(np.argmax(G.degrees))]
    out = []
    for s in seeds:
        out.append(("ppr", "gd", dict(alpha=0.1, eps=1e-6), s))
        out.append(("ppr", "ch", dict(alpha=0.1, eps=1e-6), s))
        out.append(("katz", "gd", dict(beta=beta, eps=1e-5, lambda_bound=lam), s))
        out.append(("katz", "ch", dict(beta=beta, eps=1e-5, lambda_bound=lam), s))
        out.append(("hk", "gd", dict(tau=5.0, K=30, eps=1e-5), s))
    return out


def run(gde, ctx, g, kind, method, prm, s, vt):
    p = gde.make_params(kind, method, value_type=vt, flags=gde.DETERMINISTIC | gde.TRACE, **prm)
    return gde.solve(ctx, g, p, [s], trace_cap=100000, nodes_cap=4_000_000)


def test_fp64_bit_exact_vs_oracle(gde, ctx, c1, katz_beta):
    G, g = c1
    beta, lam = katz_beta
    kinds = {"ppr": gde.PPR, "katz": gde.KATZ, "hk": gde.HK}
    for kind, method, prm, s in queries(G, beta, lam):
        res = run(gde, ctx, g, kind, method, prm, s, gde.F64)
        m = gde.LOCAL_GD if method == "gd" else gde.LOCAL_CH
        ref = oracle_run(G, kinds[kind], m, prm, np.array([s], np.int32), np.ones(1))
        x = res.dense(G.n)
        assert res.status == ref["status"]
        assert (res.iters, res.ops, res.pushes) == (ref["iters"], ref["ops"], ref["pushes"]), (kind, method, s)
        assert np.array_equal(res.trace_size, ref["trace_size"]) and np.array_equal(res.trace_vol, ref["trace_vol"])
        diff = int(np.count_nonzero(x != ref["x"]))
        print("det fp64", kind, method, s, "iters", res.iters, "ops", res.ops, "nodes differing", diff, flush=True)
        assert diff == 0, (kind, method, s, float(np.abs(x - ref["x"]).max()))
        np.testing.assert_allclose(res.residual_l1, ref["residual_l1"], rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(res.residual_dinf, ref["residual_dinf"], rtol=1e-12, atol=1e-300)


def _same(a, b):
    return (a.iters == b.iters and a.ops == b.ops and a.pushes == b.pushes and np.array_equal(a.idx, b.idx)
            and np.array_equal(np.asarray(a.val).view(np.uint32), np.asarray(b.val).view(np.uint32))
            and a.residual_l1 == b.residual_l1 and a.residual_dinf == b.residual_dinf
            and np.array_equal(a.trace_size, b.trace_size) and np.array_equal(a.trace_nodes, b.trace_nodes))


def test_fp32_runs_bit_identical_and_parity(gde, ctx, c1, katz_beta):
    G, g = c1
    beta, lam = katz_beta
    kinds = {"ppr": gde.PPR, "katz": gde.KATZ, "hk": gde.HK}
    for kind, method, prm, s in queries(G, beta, lam):
        a = run(gde, ctx, g, kind, method, prm, s, gde.F32)
        b = run(gde, ctx, g, kind, method, prm, s, gde.F32)
        assert _same(a, b), (kind, method, s)
        m = gde.LOCAL_GD if method == "gd" else gde.LOCAL_CH
        rep = check(ctx, g, G, kinds[kind], m, gde.F32, prm, [s], extra_flags=gde.DETERMINISTIC)
        print("det fp32", kind, method, s, rep, flush=True)


def test_fp32_large_graph_bit_identical(gde, ctx):
    """n = 10^6 (the plain benchmark graph) at eps 1e-6: frontiers of 10^4-10^5
    nodes, several workgroups per pull; two runs bit-identical, parity green."""
    G = W.chung_lu(1_000_000, 10_000_000, 2.5, seed=42)
    g = gde.Graph(ctx, G.row_ptr, G.col_idx)
    for s in W.uniform_seeds(G, 64, seed=42)[:2]:
        for method in ("gd", "ch"):
            a = run(gde, ctx, g, "ppr", method, dict(alpha=0.1, eps=1e-6), int(s), gde.F32)
            b = run(gde, ctx, g, "ppr", method, dict(alpha=0.1, eps=1e-6), int(s), gde.F32)
            assert _same(a, b), (method, int(s))
            m = gde.LOCAL_GD if method == "gd" else gde.LOCAL_CH
            rep = check(ctx, g, G, gde.PPR, m, gde.F32, dict(alpha=0.1, eps=1e-6), [int(s)],
                        extra_flags=gde.DETERMINISTIC)
            print("det n1M", method, int(s), rep, flush=True)
    g.close()


def test_batch_and_server(gde, ctx, c1):
    G, g = c1
    seeds = [int(s) for s in W.uniform_seeds(G, 8, seed=9)]
    ps = [gde.make_params("ppr", alpha=0.1, eps=10.0 ** -(4 + i % 3), flags=gde.DETERMINISTIC) for i in range(8)]
    br = gde.solve_batch(ctx, g, ps, [([s], None) for s in seeds])
    for i, s in enumerate(seeds):
        one = gde.solve(ctx, g, ps[i], [s])
        assert np.array_equal(br[i].idx, one.idx)
        assert np.array_equal(np.asarray(br[i].val).view(np.uint32), np.asarray(one.val).view(np.uint32))
        assert br[i].residual_l1 == one.residual_l1
    srv = gde.Server(ctx, g, lanes_per_group=8, max_groups=1, iters_per_step=2)
    with pytest.raises(gde.GDEError) as e:
        srv.submit(ps[0], [seeds[0]])
    assert e.value.status == gde.UNSUPPORTED
    srv.close()
