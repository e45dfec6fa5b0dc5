"""GPU parity of the stencil operators against the oracle (FP64)."""

import numpy as np
import pytest
import torch

from conftest import gpu_binding, to_dev
from oracle.operators import Operator as OracleOp
from paper_1302_4018_amd import inputs

pytestmark = pytest.mark.gpu

SHAPES = [[16, 16], [4, 2, 2], [8, 8, 2], [32, 32, 32], [16, 16, 16, 16], [2, 4, 8, 2], [1, 8], [64], [2, 2],
          [8, 4, 4, 8]]


def _pair(tip, dims, kind, coupled, field, seed=0):
    V = int(np.prod(dims))
    w = inputs.couplings(dims, seed=seed + 1) if coupled else None
    mf = inputs.mass_field(dims, seed=seed + 2) if field else None
    U = inputs.haar_links(dims, seed=seed + 3) if kind == 1 else None
    orc = OracleOp(dims, kind, mass=0.1, mass_field=mf, coupling=w, links=U)
    gop = tip.Operator(dims, kind, mass=0.1, mass_field=to_dev(mf), coupling=to_dev(w), links=to_dev(U))
    return orc, gop


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("coupled,field", [(False, False), (True, True)])
def test_apply_operator_parity(dims, kind, coupled, field):
    tip = gpu_binding()
    orc, gop = _pair(tip, dims, kind, coupled, field)
    V = orc.V
    rng = np.random.default_rng(7)
    nrhs = 3
    if kind == 1:
        x = rng.standard_normal((nrhs, V, 3)) + 1j * rng.standard_normal((nrhs, V, 3))
    else:
        x = rng.standard_normal((nrhs, V))
    y = tip.tip_apply_operator(gop, to_dev(x)).cpu().numpy()
    for j in range(nrhs):
        want = orc.apply(x[j])
        scale = np.abs(want).max()
        assert np.abs(y[j] - want).max() <= 1e-14 * scale * 16


def test_apply_operator_rejects_missing_links():
    tip = gpu_binding()
    op = tip.Operator([4, 4], 1, mass=0.1)
    with pytest.raises(tip.TipError):
        tip.tip_apply_operator(op, torch.zeros((1, 16, 3), dtype=torch.complex128, device="cuda"))
