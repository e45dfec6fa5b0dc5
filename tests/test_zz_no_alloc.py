"""The operator application that allocates nothing (tip_apply_operator_noalloc)
against tip_apply_operator: the same kernels on the same inputs, so the
outputs must agree bit for bit; and against the oracle's operator.  Two calls
in a row share the library's scratch, the second on a smaller lattice."""

import ctypes

import numpy as np
import pytest
import torch

from conftest import gpu_binding, to_dev
from oracle.operators import Operator as OracleOp
from paper_1302_4018_amd import inputs

pytestmark = pytest.mark.gpu


def _case(tip, dims, kind, seed):
    w = inputs.couplings(dims, seed=seed + 1)
    mf = inputs.mass_field(dims, seed=seed + 2)
    U = inputs.haar_links(dims, seed=seed + 3) if kind == 1 else None
    orc = OracleOp(dims, kind, mass=0.1, mass_field=mf, coupling=w, links=U)
    gop = tip.Operator(dims, kind, mass=0.1, mass_field=to_dev(mf), coupling=to_dev(w), links=to_dev(U))
    rng = np.random.default_rng(seed)
    V = orc.V
    if kind == 1:
        x = rng.standard_normal((3, V, 3)) + 1j * rng.standard_normal((3, V, 3))
    else:
        x = rng.standard_normal((3, V))
    return orc, gop, x


@pytest.mark.parametrize("kind", [1, 0])
def test_noalloc_matches_apply_operator_on_two_calls(kind):
    tip = gpu_binding()
    # the second lattice is smaller than the first: its call reuses the scratch
    for dims, seed in (([8, 8, 8, 8], 11), ([6, 4, 5], 23)):
        orc, gop, x = _case(tip, dims, kind, seed)
        xd = to_dev(x)
        print(f"noalloc: kind {kind}, dims {dims}", flush=True)
        ref = tip.tip_apply_operator(gop, xd)
        got = tip.tip_apply_operator_noalloc(gop, xd)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), f"{dims}: no-allocation result differs from tip_apply_operator"
        y = got.cpu().numpy()
        for j in range(x.shape[0]):
            want = orc.apply(x[j])
            assert np.abs(y[j] - want).max() <= 16e-14 * np.abs(want).max()


def test_noalloc_rejects_lattices_beyond_the_scratch():
    tip = gpu_binding()
    # 2^23 scalar sites need two 64 MiB vectors: refused before any device work
    op = tip.tip_operator()
    op.ndim = 3
    op.dims[0], op.dims[1], op.dims[2] = 256, 256, 128
    op.kind = tip.KIND_SCALAR
    op.mass = 0.1
    sentinel = torch.full((4,), 7.0, dtype=torch.float64, device="cuda")
    st = tip.lib.tip_apply_operator_noalloc(ctypes.byref(op), 1, ctypes.c_void_p(sentinel.data_ptr()),
                                            ctypes.c_void_p(sentinel.data_ptr()), None)
    assert st == tip.TIP_EINVAL
    assert "scratch" in tip.tip_last_error()
    assert torch.equal(sentinel.cpu(), torch.full((4,), 7.0, dtype=torch.float64))
