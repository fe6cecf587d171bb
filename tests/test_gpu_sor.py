"""LocalSOR / APPR / AKatz on the GPU (method GDE_LOCAL_SOR: the FIFO push of
Algorithm 1 with the relaxation of Eq. (7), one query per wavefront) against the
oracle's FIFO push (oracle.push_fifo).

The GPU executes the same sequential steps in the same order, so in FP64 x and r
equal the oracle's bit for bit, with the same pops, work (sum of popped degrees)
and queue generations.  FP32: when the pops and work equal the oracle's, x must
match within 1e-6 of the mass; a threshold decision within FP32 rounding changes
the queue from there on, and the result must then meet the stop rule of the
FP64-recomputed residual within the FP32 bound.  A batch gives each query what
it gives alone; queries beyond the memory budget run in rounds.  (The device
state is FP64 for either value type, which only sets the type of x returned, so
FP32 results are the FP64 ones rounded.)
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import exact as X  # noqa: E402
from oracle import solvers as O  # noqa: E402
from paper_2410_21634_amd import workloads as W  # noqa: E402

from _parity import RTOL, TOL, fp32_residual_bound, mass  # noqa: E402

OMEGA_STAR = 2.0 / (1.0 + math.sqrt(1.0 - 0.9 ** 2))  # Sec. 3.2, alpha = 0.1


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


def queries(G, beta):
    seeds = [int(s) for s in W.uniform_seeds(G, 3, seed=31)] + [int(np.argmax(G.degrees))]
    out = []
    for s in seeds:
        for om in (1.0, OMEGA_STAR, 0.7):
            out.append((O.PPR, "ppr", 0.1, 1e-6, om, [s]))
        out.append((O.KATZ, "katz", beta, 1e-6, 1.0, [s]))
        out.append((O.KATZ, "katz", beta, 1e-6, 1.2, [s]))
    set8 = sorted(set(int(v) for v in W.uniform_seeds(G, 12, seed=32)))[:8]
    out.append((O.PPR, "ppr", 0.15, 1e-7, OMEGA_STAR, set8))
    return out


def params(gde, kname, param, eps, om, vt, lam):
    prm = dict(alpha=param) if kname == "ppr" else dict(beta=param, lambda_bound=lam)
    return gde.make_params(kname, "sor", eps=eps, omega=om, value_type=vt, **prm)


def grade(gde, G, res, kind, param, eps, om, sd, vt):
    ref = O.push_fifo(G.row_ptr, G.col_idx, kind, param, eps, sd, omega=om)
    x = res.dense(G.n)
    same = (res.pushes, res.ops, res.iters) == (ref["pops"], ref["ops"], ref["epochs"])
    if vt == gde.F64:
        assert same, (res.pushes, ref["pops"], res.ops, ref["ops"], res.iters, ref["epochs"])
        assert np.array_equal(x, ref["x"]), float(np.abs(x - ref["x"]).max())
        np.testing.assert_allclose(res.residual_l1, ref["residual_l1"], rtol=RTOL[vt], atol=1e-300)
        np.testing.assert_allclose(res.residual_dinf, ref["residual_dinf"], rtol=RTOL[vt], atol=1e-300)
        return 0.0, "exact"
    err = float(np.abs(x - ref["x"]).sum()) / mass(kind, np.ones(len(sd)), ref["x"])
    if same:
        assert err <= TOL[vt], err
        return err, "same-queue"
    # another valid queue: the FP64 residual of this x meets the stop rule within the FP32 bound
    n = G.n
    s = np.zeros(n)
    s[np.asarray(sd)] = 1.0
    A = X.sparse_adjacency(G.row_ptr, G.col_idx)
    d = np.diff(G.row_ptr).astype(float)
    if kind == O.PPR:
        inv = np.where(d > 0, 1.0 / np.maximum(d, 1), 0.0)
        r = (param * s - (x - (1 - param) * (A @ (inv * x)))) / param
    else:
        r = s - (x - param * (A @ x))
    bound = fp32_residual_bound(G.row_ptr, G.col_idx, kind, param, eps, x, int(res.pushes))
    assert (np.abs(r) <= bound).all()
    return err, "certificate"


@pytest.mark.parametrize("vt", [1, 0])
def test_sor_matches_oracle_fifo(gde, ctx, c1, vt):
    G, g = c1
    lo, hi = X.lambda_bounds_power(G.row_ptr, G.col_idx, iters=300)
    beta = 0.3 / hi
    for kind, kname, param, eps, om, sd in queries(G, beta):
        res = gde.solve(ctx, g, params(gde, kname, param, eps, om, vt, hi * 2.0), sd)
        err, how = grade(gde, G, res, kind, param, eps, om, sd, vt)
        print("sor", kname, round(om, 3), sd[:2], vt, "pops", res.pushes, "gens", res.iters, how, err, flush=True)


def test_sor_batch_equals_alone(gde, ctx, c1):
    G, g = c1
    seeds = [int(s) for s in W.uniform_seeds(G, 24, seed=33)]
    ps = [params(gde, "ppr", 0.1, 10.0 ** -(4 + i % 4), (1.0, OMEGA_STAR, 0.8)[i % 3], gde.F64, 0.0)
          for i in range(24)]
    out = gde.solve_batch(ctx, g, ps, [([s], None) for s in seeds])
    for i, s in enumerate(seeds):
        one = gde.solve(ctx, g, ps[i], [s])
        assert np.array_equal(out[i].idx, one.idx) and np.array_equal(out[i].val, one.val)
        assert (out[i].pushes, out[i].ops, out[i].iters) == (one.pushes, one.ops, one.iters)


def test_sor_rounds_and_full_size(gde, ctx):
    """1,100 queries on the n = 10^6 graph need two rounds of slots (the 24 GiB
    budget holds 1,030 slots of 25 MB); sampled queries of both rounds, and
    a query at eps 1e-6 with device outputs, against the oracle in FP64."""
    import torch
    G = W.chung_lu(1_000_000, 10_000_000, 2.5, seed=42)
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(G.row_ptr).to(dev)
    ci = torch.from_numpy(G.col_idx).to(dev)
    g = gde.Graph(ctx, rp, ci)
    seeds = [int(s) for s in W.uniform_seeds(G, 1100, seed=34)]
    ps = [params(gde, "ppr", 0.1, 1e-4, OMEGA_STAR if i % 2 else 1.0, gde.F64, 0.0) for i in range(1100)]
    out = gde.solve_batch(ctx, g, ps, [([s], None) for s in seeds])
    for i in (0, 1, 549, 1029, 1030, 1099):
        grade(gde, G, out[i], O.PPR, 0.1, 1e-4, OMEGA_STAR if i % 2 else 1.0, [seeds[i]], gde.F64)
    oi = torch.empty(G.n, dtype=torch.int32, device=dev)
    ov = torch.empty(G.n, dtype=torch.float64, device=dev)
    res = gde.solve(ctx, g, params(gde, "ppr", 0.1, 1e-6, OMEGA_STAR, gde.F64, 0.0), [seeds[5]], out=(oi, ov))
    torch.cuda.synchronize()
    grade(gde, G, res, O.PPR, 0.1, 1e-6, OMEGA_STAR, [seeds[5]], gde.F64)
    print("sor n1M eps 1e-6 pops", res.pushes, "ops", res.ops, flush=True)
    g.close()
