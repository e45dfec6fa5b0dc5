"""The comparison probes of Sec. 5 on the GPU path: natural-order Hadamard
and plain Monte-Carlo (random Z2 / Z4) probes, bit for bit against the oracle
and through the whole solve, plus the study workload (a 32^3 torus with a
closed-form trace) checked for parity against the oracle on its first probes."""

import numpy as np
import pytest

from conftest import gpu_binding, to_dev
from oracle import exact, general
from oracle.mask import MASK_Z2, MASK_Z4
from oracle.operators import Operator as OracleOp
from paper_1302_4018_amd import inputs

pytestmark = pytest.mark.gpu
REL = 1e-10


@pytest.mark.parametrize("dims,ncomp,mask,probe", [
    ([16, 16], 1, MASK_Z2, general.PROBE_NATURAL), ([4, 8, 2], 3, MASK_Z4, general.PROBE_NATURAL),
    ([16, 16], 1, MASK_Z2, general.PROBE_RANDOM), ([6, 5, 3], 3, MASK_Z4, general.PROBE_RANDOM),
    ([32, 32, 32, 32], 3, MASK_Z4, general.PROBE_RANDOM),
])
def test_probe_kinds_bit_exact(dims, ncomp, mask, probe):
    tip = gpu_binding()
    V = int(np.prod(dims))
    for comp in range(ncomp):
        for m in sorted({0, 1, 7, V // 3, V - 1}):
            got = tip.tip_probe_vectors(dims, ncomp, mask, 55, m, 1, comp, probe=probe)[0].cpu().numpy()
            want = general.rhs_kind(dims, ncomp, m, comp, 55, mask, probe)[:, comp]
            assert np.array_equal(got, want), (m, comp)


@pytest.mark.parametrize("dims,kind,n,mask,probe,prec", [
    ([16, 16], 0, 64, MASK_Z2, general.PROBE_NATURAL, "fp64"),
    ([16, 16], 0, 64, MASK_Z2, general.PROBE_RANDOM, "fp64"),
    ([8, 4, 8], 1, 12, MASK_Z4, general.PROBE_RANDOM, "mixed"),
    ([6, 10], 0, 40, MASK_Z4, general.PROBE_RANDOM, "fp64"),
    ([4, 4, 4, 8], 1, 8, MASK_Z4, general.PROBE_NATURAL, "fp64"),
])
def test_probe_kinds_through_the_solver(dims, kind, n, mask, probe, prec):
    tip = gpu_binding()
    w = inputs.couplings(dims, seed=600)
    U = inputs.haar_links(dims, seed=601) if kind == 1 else None
    orc = OracleOp(dims, kind, mass=0.2, coupling=w, links=U)
    gop = tip.Operator(dims, kind, mass=0.2, coupling=to_dev(w), links=to_dev(U))
    precision = tip.PREC_MIXED if prec == "mixed" else tip.PREC_FP64
    est, q, st = tip.trace_inv_probe(gop, n, 1e-12, 4018, mask=mask, probe=probe, precision=precision)
    est_o, q_o, _ = general.trace_inv_probe(orc, n, 1e-12, 4018, mask, probe=probe)
    assert np.max(np.abs(est - est_o) / np.abs(est_o)) <= REL
    assert np.max(np.abs(q - q_o) / np.abs(q_o)) <= REL


def test_study_workload_first_probes_against_oracle():
    """32^3 free torus, m = 0.05: the three probe kinds; estimates at s = 1, 2, 4
    against the oracle, and the last estimate's error against the closed form."""
    tip = gpu_binding()
    import torch
    dims, m = [32, 32, 32], 0.05
    gop = tip.Operator(dims, tip.KIND_SCALAR, mass=m)
    orc = OracleOp(dims, 0, mass=m)
    tr = exact.free_trace_inverse(dims, m)
    for probe in (general.PROBE_HIERARCHICAL, general.PROBE_NATURAL, general.PROBE_RANDOM):
        est, q, st = tip.trace_inv_probe(gop, 4, 1e-10, 7, mask=MASK_Z2, probe=probe)
        est_o, _, _ = general.trace_inv_probe(orc, 4, 1e-10, 7, MASK_Z2, probe=probe)
        assert np.max(np.abs(est - est_o) / np.abs(est_o)) <= REL, probe
        assert abs(est[-1] - tr) / tr < 0.5
