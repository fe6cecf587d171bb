"""The C ABI library loads, exports every symbol of include/gde.h and validates
arguments on the host (no GPU needed: validation runs before any device work)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "gde.h")) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^(?:int|size_t|const char \*|const gde_graph \*)\s*(gde_[a-z_]+)\s*\(", text,
                                 re.M)))


def test_header_symbols_exported():
    from paper_2410_21634_amd import gde
    lib = C.CDLL(gde.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(gde.EXPORTED)
    assert gde.abi_version() == 2


@pytest.fixture(scope="module")
def small():
    from paper_2410_21634_amd import workloads as W
    return W.from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 4), (0, 4)])  # node 5 isolated


def test_validation_errors(small):
    from paper_2410_21634_amd import gde
    rp, ci = small.row_ptr, small.col_idx

    def v(seed=(0,), val=None, **kw):
        base = dict(kind="ppr", method="gd", alpha=0.1, eps=1e-4)
        base.update(kw)
        return gde.validate(rp, ci, gde.make_params(**base), list(seed), val)

    assert v() == gde.OK
    assert v(eps=0.0) == gde.INVALID_ARG
    assert v(eps=float("nan")) == gde.INVALID_ARG
    assert v(alpha=1.0) == gde.INVALID_ARG
    assert v(alpha=0.0) == gde.INVALID_ARG
    assert v(kind="katz", beta=0.1, lambda_bound=2.0) == gde.OK
    assert v(kind="katz", beta=0.6, lambda_bound=2.0) == gde.INVALID_ARG   # beta * lambda >= 1
    assert v(kind="katz", beta=0.1, lambda_bound=0.0) == gde.INVALID_ARG
    assert v(kind="hk", tau=5.0, K=30) == gde.OK
    assert v(kind="hk", tau=-1.0) == gde.INVALID_ARG
    assert v(kind="hk", K=300) == gde.INVALID_ARG
    assert v(kind="hk", method="ch") == gde.UNSUPPORTED
    assert v(kind="series", c=[0.5, 0.3, 0.2]) == gde.OK
    assert v(kind="series", c=[0.5, 0.0, 0.2]) == gde.INVALID_ARG         # a zero coefficient
    assert v(kind="series", c=[0.5, float("inf")]) == gde.INVALID_ARG
    assert v(kind="series", c=[0.5, 0.3], method="ch") == gde.UNSUPPORTED
    assert v(kind="series") == gde.INVALID_ARG                            # no coefficients
    assert v(kind="ppr", c=[0.5]) == gde.INVALID_ARG                      # c is for SERIES only
    assert v(kind="series", c=[1.0] * 258) == gde.INVALID_ARG             # K > 256
    assert v(method="sor") == gde.OK and v(method="sor", omega=1.4) == gde.OK
    assert v(method="sor", omega=2.0) == gde.INVALID_ARG
    assert v(method="sor", omega=-0.5) == gde.INVALID_ARG
    assert v(kind="hk", method="sor") == gde.UNSUPPORTED
    assert v(method=3) == gde.INVALID_ARG
    assert v(max_iters=0) == gde.INVALID_ARG
    assert v(seed=(1, 0)) == gde.INVALID_ARG            # unsorted
    assert v(seed=(1, 1)) == gde.INVALID_ARG            # duplicate
    assert v(seed=(9,)) == gde.INVALID_ARG              # out of range
    assert v(seed=(0,), val=[-1.0]) == gde.INVALID_ARG  # nonpositive value
    assert v(seed=(5,)) == gde.ISOLATED_SEED
    p = gde.make_params(value_type=7)
    assert gde.validate(rp, ci, p, [0]) == gde.INVALID_ARG
    p = gde.make_params(flags=0x100)
    assert gde.validate(rp, ci, p, [0]) == gde.INVALID_ARG
    p = gde.make_params(flags=gde.SCATTER_BINNED | gde.SCATTER_ATOMIC)  # exclusive strategies
    assert gde.validate(rp, ci, p, [0]) == gde.INVALID_ARG
    for f in (gde.SCATTER_BINNED, gde.SCATTER_ATOMIC, gde.DETERMINISTIC, gde.DETERMINISTIC | gde.TRACE):
        assert gde.validate(rp, ci, gde.make_params(flags=f), [0]) == gde.OK
    p = gde.make_params(flags=gde.SYM_NORM << 1)  # the first undefined flag bit
    assert gde.validate(rp, ci, p, [0]) == gde.INVALID_ARG
    # D^-1/2 A D^-1/2: PPR, HK and series with LocalGD / LocalCH / the level push
    for kw in (dict(), dict(method="ch"), dict(kind="hk", tau=5.0, K=30), dict(kind="series", c=[0.5, 0.25])):
        assert gde.validate(rp, ci, gde.make_params(flags=gde.SYM_NORM, **kw), [0]) == gde.OK
    assert gde.validate(rp, ci, gde.make_params(kind="katz", beta=0.1, lambda_bound=2.0, flags=gde.SYM_NORM),
                        [0]) == gde.INVALID_ARG
    for kw in (dict(method="sor", flags=gde.SYM_NORM), dict(flags=gde.SYM_NORM | gde.DETERMINISTIC)):
        assert gde.validate(rp, ci, gde.make_params(**kw), [0]) == gde.UNSUPPORTED
    # malformed CSR
    bad = rp.copy()
    bad[-1] += 1
    assert gde.validate(bad, ci, gde.make_params(), [0]) == gde.INVALID_ARG
    ci2 = ci.copy()
    ci2[0] = 0  # self-loop at node 0
    assert gde.validate(rp, ci2, gde.make_params(), [0]) == gde.INVALID_ARG
    ci3 = ci.copy()
    ci3[0] = 17
    assert gde.validate(rp, ci3, gde.make_params(), [0]) == gde.INVALID_ARG
    assert "self-loop" in gde.last_error() or "range" in gde.last_error()
