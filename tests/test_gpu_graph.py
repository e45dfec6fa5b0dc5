"""Chunks of CG iterations replayed as HIP graphs give the same bits as eager
launches: several blocks per call (so every graph is replayed many times,
with the host's own polling and synchronisation between replays), in FP64,
mixed precision, the even-odd and the plain solver.  With profiling on the
library launches eagerly (per-kernel events), which must agree as well."""

import os

import numpy as np
import pytest

from conftest import gpu_binding, to_dev
from paper_1302_4018_amd import inputs

pytestmark = pytest.mark.gpu


def _run(tip, gop, n, env, **kw):
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return tip.trace_inv_probe(gop, n, 1e-11, 4018, **kw)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


@pytest.mark.parametrize("dims,kind,n,prec,eo", [
    ([8, 8, 8, 8], 1, 48, "fp64", True),      # 144 solves in blocks of 64
    ([8, 8, 8, 8], 1, 48, "mixed", True),
    ([16, 16, 16], 0, 200, "fp64", False),    # plain CG, marching stencil
    ([6, 10, 12], 0, 150, "fp64", False),     # odd sides: generic stencil
])
def test_graph_replays_match_eager(dims, kind, n, prec, eo):
    tip = gpu_binding()
    w = inputs.couplings(dims, seed=700)
    U = inputs.haar_links(dims, seed=701) if kind == 1 else None
    mf = inputs.mass_field(dims, seed=702)
    gop = tip.Operator(dims, kind, mass_field=to_dev(mf), coupling=to_dev(w), links=to_dev(U))
    precision = tip.PREC_MIXED if prec == "mixed" else tip.PREC_FP64
    env_eo = {} if eo else {"TIP_EO": "0"}
    ref = _run(tip, gop, n, {"TIP_GRAPH": "0", **env_eo}, precision=precision)
    for profiling in (False, True, False):
        tip.tip_set_profiling(profiling)
        try:
            got = _run(tip, gop, n, env_eo, precision=precision)
        finally:
            tip.tip_set_profiling(False)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        assert got[2]["total_iters"] == ref[2]["total_iters"]
        assert got[2]["even_odd"] == (1 if eo else 0)
        if profiling:
            assert got[2]["stencil_seconds"] > 0.0
