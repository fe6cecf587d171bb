"""The continuous-batching server: mixed PPR / Katz / HK queries arriving while
others run, and edge insertions applied to in-flight queries.

A static-graph result must be the same alone and inside the mix (within the
FP32 tolerance 1e-6 ||s||_1, or, if an FP32 threshold decision flipped --
atomic adds land in a different order from run to run -- both must satisfy the
stop certificate of their kind), and must agree with the FP64 oracle.  A
result that lived through edge insertions is checked against the *new* graph:
r = b - Q_new x recomputed in FP64 on the host satisfies the stop rule within
the FP32 rounding bound of _parity.fp32_residual_bound, and (PPR)
|f_new - x| <= eps d_new componentwise (the Theorem 3.2 bound, which holds for
signed residuals as well).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import exact as X  # noqa: E402
from oracle import solvers as O  # noqa: E402
from paper_2410_21634_amd import workloads as W  # noqa: E402

from _parity import TOL, fp32_residual_bound, mass  # noqa: E402


@pytest.fixture(scope="module")
def gde():
    from paper_2410_21634_amd import gde as mod
    return mod


@pytest.fixture(scope="module")
def ctx(gde):
    c = gde.Context(0)
    yield c
    c.close()


def ppr_residual(row_ptr, col_idx, alpha, seed_idx, seed_val, x):
    """FP64 residual r~ = (alpha s - (I - (1-alpha) A D^-1) x) / alpha of x on the given graph."""
    n = len(row_ptr) - 1
    d = np.diff(row_ptr).astype(float)
    A = X.sparse_adjacency(row_ptr, col_idx)
    s = np.zeros(n)
    s[np.asarray(seed_idx)] = seed_val
    inv = np.where(d > 0, 1.0 / np.maximum(d, 1), 0.0)
    r = alpha * s - (x - (1 - alpha) * (A @ (inv * x)))
    return r / alpha


def katz_residual(row_ptr, col_idx, beta, seed_idx, seed_val, x):
    """FP64 residual r = s - (I - beta A) x of x on the given graph."""
    n = len(row_ptr) - 1
    A = X.sparse_adjacency(row_ptr, col_idx)
    s = np.zeros(n)
    s[np.asarray(seed_idx)] = seed_val
    return s - (x - beta * (A @ x))


def assert_certificate(row_ptr, col_idx, kind, param, eps, seed_idx, seed_val, x, T, events=0, signed=False):
    """The stop rule on the FP64 residual of x, within the derived FP32 rounding
    bound; for nonnegative residuals (static LocalGD) also r >= -(rounding)."""
    d = np.diff(row_ptr).astype(float)
    if kind == "ppr":
        r = ppr_residual(row_ptr, col_idx, param, seed_idx, seed_val, x)
        bound = fp32_residual_bound(row_ptr, col_idx, 0, param, eps, x, T, events)
    else:
        r = katz_residual(row_ptr, col_idx, param, seed_idx, seed_val, x)
        bound = fp32_residual_bound(row_ptr, col_idx, 1, param, eps, x, T, events)
    live = d > 0
    worst = float((np.abs(r[live]) / bound[live]).max())
    assert worst < 1.0, (kind, worst)
    if not signed:
        assert (r[live] >= -(bound[live] - eps * d[live])).all(), (kind, float(r.min()))
    return worst


def hk_truncated(row_ptr, col_idx, tau, K, seed_idx, seed_val):
    """f_K = sum_{k<=K} e^-tau tau^k/k! (A D^-1)^k s, by sparse products."""
    n = len(row_ptr) - 1
    d = np.diff(row_ptr).astype(float)
    A = X.sparse_adjacency(row_ptr, col_idx)
    inv = np.where(d > 0, 1.0 / np.maximum(d, 1), 0.0)
    v = np.zeros(n)
    v[np.asarray(seed_idx)] = seed_val
    v *= np.exp(-tau)
    f = v.copy()
    for k in range(1, K + 1):
        v = (tau / k) * (A @ (inv * v))
        f += v
    return f


def drain(srv, want, limit=20000):
    got = {}
    for _ in range(limit):
        for c in srv.poll():
            got[c["ticket"]] = c
        if len(got) >= want:
            break
    return got


def test_server_static_mix(gde, ctx):
    G = W.chung_lu(10000, 50000, 2.5, seed=42)
    g = gde.Graph(ctx, G.row_ptr, G.col_idx)
    lo, hi = g.lambda_max(max_iters=500, rtol=1e-4)
    beta = 0.5 / lo
    rng = np.random.default_rng(5)
    seeds = W.uniform_seeds(G, 48, seed=5)
    qs = []
    for i, s in enumerate(seeds):
        eps = float(10 ** rng.uniform(-6, -4))
        kind = ("ppr", "katz", "hk")[i % 3]
        if i % 4 == 1:
            idx, val = W.seed_set(G, int(s), 8, rng)
        else:
            idx, val = np.array([s], np.int32), np.ones(1)
        if kind == "ppr":
            p = gde.make_params("ppr", alpha=0.1, eps=eps)
        elif kind == "katz":
            p = gde.make_params("katz", beta=beta, eps=eps, lambda_bound=hi)
        else:
            p = gde.make_params("hk", tau=5.0, K=30, eps=eps)
        qs.append((kind, p, idx, val, eps))
    srv = gde.Server(ctx, g, lanes_per_group=8, max_groups=3, iters_per_step=3)
    tickets = {}
    # staggered arrivals: a third now, the rest while the first groups run
    for j, q in enumerate(qs[:16]):
        tickets[srv.submit(q[1], q[2], q[3])] = j
    got = {}
    for c in srv.poll():
        got[c["ticket"]] = c
    for j, q in enumerate(qs[16:], start=16):
        tickets[srv.submit(q[1], q[2], q[3])] = j
    got.update(drain(srv, len(qs)))
    assert len(got) == len(qs)
    mix = {tickets[t]: c for t, c in got.items()}
    srv.close()
    # each query alone on a fresh server, and against the FP64 oracle
    srv1 = gde.Server(ctx, g, lanes_per_group=8, max_groups=1, iters_per_step=3)
    for j, (kind, p, idx, val, eps) in enumerate(qs):
        t = srv1.submit(p, idx, val)
        alone = drain(srv1, 1)[t]
        m = mix[j]
        assert m["status"] == gde.OK and alone["status"] == gde.OK
        xm = np.zeros(G.n)
        xm[m["idx"]] = m["val"]
        xa = np.zeros(G.n)
        xa[alone["idx"]] = alone["val"]
        if kind == "ppr":
            ref = O.localgd(G.row_ptr, G.col_idx, O.PPR, 0.1, eps, idx, val)["x"]
        elif kind == "katz":
            ref = O.localgd(G.row_ptr, G.col_idx, O.KATZ, beta, eps, idx, val)["x"]
        else:
            ref = O.hk(G.row_ptr, G.col_idx, 5.0, 30, eps, idx, val)["x"]
        s1 = mass({"ppr": gde.PPR, "katz": gde.KATZ, "hk": gde.HK}[kind], val, ref)
        d_mix_alone = np.abs(xm - xa).sum() / s1
        d_oracle = np.abs(xm - ref).sum() / s1
        if kind == "ppr" and (d_mix_alone > 1e-6 or d_oracle > 1e-6):
            # an FP32 threshold flip: both answers must still meet the Theorem 3.2
            # bound |f - x| <= eps d (x holds FP32 rounding, hence the small slack)
            svec = np.zeros(G.n)
            svec[idx] = val
            f = X.global_ppr(G.row_ptr, G.col_idx, 0.1, svec, tol=1e-13)
            dd = np.diff(G.row_ptr).astype(float)
            for x, T in ((xm, m["iters"]), (xa, alone["iters"])):
                assert (np.abs(f - x) <= eps * dd * (1 + 1e-3) + 1e-6 * np.abs(f) + 1e-9).all(), j
                assert_certificate(G.row_ptr, G.col_idx, "ppr", 0.1, eps, idx, val, x, T)
        elif kind == "hk" and (d_mix_alone > 1e-6 or d_oracle > 1e-6):
            # an FP32 threshold flip at some level: both answers must meet the
            # level-push guarantee 0 <= f_K - x and ||D^-1 (f_K - x)||_inf <= eps
            fK = hk_truncated(G.row_ptr, G.col_idx, 5.0, 30, idx, val)
            dd = np.diff(G.row_ptr).astype(float)
            for x in (xm, xa):
                gap = fK - x
                assert (gap >= -1e-6 * fK - 1e-9).all(), j
                assert (gap[dd > 0] <= eps * dd[dd > 0] * (1 + 1e-3) + 1e-6 * fK[dd > 0] + 1e-9).all(), j
        elif kind == "katz" and (d_mix_alone > TOL[gde.F32] or d_oracle > TOL[gde.F32]):
            for x, T in ((xm, m["iters"]), (xa, alone["iters"])):
                assert_certificate(G.row_ptr, G.col_idx, "katz", beta, eps, idx, val, x, T)
        else:
            assert d_mix_alone <= TOL[gde.F32], (j, kind, d_mix_alone)
            assert d_oracle <= TOL[gde.F32], (j, kind, d_oracle)
    srv1.close()
    g.close()


def test_server_dynamic_inserts(gde, ctx):
    """PPR and Katz queries in flight while three 500-edge insert batches land: the
    server applies the warm-start corrections (Algorithm 3's Insert per directed
    event for PPR; r_c += beta x_a for Katz) to every in-flight query.  Each final
    x is graded on the new graph by its FP64 residual (stop rule within the
    derived FP32 bound) and, for PPR, by |f_new - x| <= eps d_new."""
    G = W.chung_lu(10000, 50000, 2.5, seed=7)
    g = gde.Graph(ctx, G.row_ptr, G.col_idx)
    lo, hi = g.lambda_max(max_iters=500, rtol=1e-4)
    beta = 0.5 / lo
    rng = np.random.default_rng(11)
    seeds = W.uniform_seeds(G, 32, seed=11)
    eps = 1e-6
    srv = gde.Server(ctx, g, lanes_per_group=8, max_groups=3, iters_per_step=2)
    tickets = {}
    for i, s in enumerate(seeds):
        if i % 2 == 0:
            p = gde.make_params("ppr", alpha=0.1, eps=eps)
        else:
            # the bound is checked against the pre-insert graph; the inserts grow
            # lambda_max by a few percent, far from beta * lambda = 1
            p = gde.make_params("katz", beta=beta, eps=eps, lambda_bound=hi)
        tickets[srv.submit(p, [int(s)])] = ("ppr" if i % 2 == 0 else "katz", int(s))
    got = {}
    for c in srv.poll():  # the first groups are in flight now
        got[c["ticket"]] = c
    existing = set()
    all_u, all_v = [], []
    batches = 3
    for _ in range(batches):
        u, v = W.insert_batch(G, 500, rng, existing)
        all_u.append(u)
        all_v.append(v)
        srv.insert_edges(u, v)
        for c in srv.poll():
            got[c["ticket"]] = c
    got.update(drain(srv, len(seeds)))
    assert len(got) == len(seeds)
    # the final graph
    u = np.concatenate(all_u)
    v = np.concatenate(all_v)
    edges = set()
    for a in range(G.n):
        for b in G.col_idx[G.row_ptr[a]:G.row_ptr[a + 1]]:
            if a < b:
                edges.add((a, int(b)))
    edges.update(zip(u.tolist(), v.tolist()))
    Gn = W.from_edges(G.n, sorted(edges))
    d = np.diff(Gn.row_ptr).astype(float)
    new_deg = np.bincount(np.concatenate([u, v]), minlength=G.n)
    # roundings per node and batch: x rescale, own residual, one addition per new neighbour
    events = batches * (2 + int(new_deg.max()))
    kinds_seen = set()
    for t, c in got.items():
        kind, s = tickets[t]
        kinds_seen.add(kind)
        assert c["status"] == gde.OK
        x = np.zeros(G.n)
        x[c["idx"]] = c["val"]
        param = 0.1 if kind == "ppr" else beta
        # the corrections make PPR residuals signed; Katz corrections only add
        assert_certificate(Gn.row_ptr, Gn.col_idx, kind, param, eps, [s], [1.0], x, c["iters"], events,
                           signed=(kind == "ppr"))
        if kind == "ppr":
            svec = np.zeros(G.n)
            svec[s] = 1.0
            f = X.global_ppr(Gn.row_ptr, Gn.col_idx, 0.1, svec, tol=1e-13)
            assert (np.abs(f - x) <= eps * d * (1 + 1e-3) + 1e-6 * np.abs(f) + 1e-9).all()
    assert kinds_seen == {"ppr", "katz"}
    srv.close()
    g.close()


def _hk_ok(row_ptr, col_idx, eps, idx, val, x):
    """x is the level-push answer on this graph: it agrees with the FP64 oracle,
    or (an FP32 threshold flip at some level) it meets the level-push guarantee
    0 <= f_K - x and ||D^-1 (f_K - x)||_inf <= eps."""
    s1 = float(np.sum(val))
    ref = O.hk(row_ptr, col_idx, 5.0, 30, eps, idx, val)["x"]
    if np.abs(x - ref).sum() / s1 <= 1e-6:
        return True
    fK = hk_truncated(row_ptr, col_idx, 5.0, 30, idx, val)
    dd = np.diff(row_ptr).astype(float)
    gap = fK - x
    return bool((gap >= -1e-6 * fK - 1e-9).all()
                and (gap[dd > 0] <= eps * dd[dd > 0] * (1 + 1e-3) + 1e-6 * fK[dd > 0] + 1e-9).all())


def test_server_hk_with_inserts(gde, ctx):
    """Heat-kernel queries run on worker threads while an insert batch is applied:
    each is solved on one graph version, the old or the new one for queries that
    were queued before the batch, the new one for queries submitted after the
    poll that applied it."""
    G = W.chung_lu(10000, 50000, 2.5, seed=9)
    g = gde.Graph(ctx, G.row_ptr, G.col_idx)
    rng = np.random.default_rng(9)
    seeds = W.uniform_seeds(G, 16, seed=9)
    eps = 1e-5
    srv = gde.Server(ctx, g, lanes_per_group=8, max_groups=2, iters_per_step=2)
    p = gde.make_params("hk", tau=5.0, K=30, eps=eps)
    early = {srv.submit(p, [int(s)]): int(s) for s in seeds[:8]}
    u, v = W.insert_batch(G, 500, rng, set())
    srv.insert_edges(u, v)
    got = {c["ticket"]: c for c in srv.poll()}  # applies the batch
    late = {srv.submit(p, [int(s)]): int(s) for s in seeds[8:]}
    got.update(drain(srv, len(seeds) - len(got)))
    assert len(got) == len(seeds)
    edges = set()
    for a in range(G.n):
        for b in G.col_idx[G.row_ptr[a]:G.row_ptr[a + 1]]:
            if a < b:
                edges.add((a, int(b)))
    edges.update(zip(u.tolist(), v.tolist()))
    Gn = W.from_edges(G.n, sorted(edges))
    one = np.ones(1)
    for t, c in got.items():
        assert c["status"] == gde.OK, c["status"]
        x = np.zeros(G.n)
        x[c["idx"]] = c["val"]
        if t in late:
            assert _hk_ok(Gn.row_ptr, Gn.col_idx, eps, [late[t]], one, x), late[t]
        else:
            s = early[t]
            assert (_hk_ok(Gn.row_ptr, Gn.col_idx, eps, [s], one, x)
                    or _hk_ok(G.row_ptr, G.col_idx, eps, [s], one, x)), s
    srv.close()
    g.close()


def test_server_admission_errors(gde, ctx):
    """Submit-time errors: a full queue is BUSY (and accepts again once polled
    empty), LocalCH is UNSUPPORTED, a seed of degree 0 is ISOLATED_SEED."""
    G = W.chung_lu(2000, 10000, 2.5, seed=3)
    g = gde.Graph(ctx, G.row_ptr, G.col_idx)
    srv = gde.Server(ctx, g, lanes_per_group=8, max_groups=1, iters_per_step=2, queue_capacity=4)
    deg = np.diff(G.row_ptr)
    seeds = [int(u) for u in np.flatnonzero(deg > 0)[:5]]
    p = gde.make_params("ppr", alpha=0.1, eps=1e-4)
    tickets = [srv.submit(p, [s]) for s in seeds[:4]]
    with pytest.raises(gde.GDEError) as e:
        srv.submit(p, [seeds[4]])
    assert e.value.status == gde.BUSY
    with pytest.raises(gde.GDEError) as e:
        srv.submit(gde.make_params("ppr", alpha=0.1, eps=1e-4, method="ch"), [seeds[0]])
    assert e.value.status == gde.UNSUPPORTED
    iso = np.flatnonzero(deg == 0)
    if len(iso):
        with pytest.raises(gde.GDEError) as e:
            srv.submit(p, [int(iso[0])])
        assert e.value.status == gde.ISOLATED_SEED
    got = drain(srv, 4)
    assert sorted(got) == sorted(tickets) and all(c["status"] == gde.OK for c in got.values())
    t = srv.submit(p, [seeds[4]])
    assert drain(srv, 1)[t]["status"] == gde.OK
    srv.close()
    g.close()
