"""The probe variants of Sec. 5 on the GPU path: the hierarchy stopped after
k bit-levels (Sec. 5.1) and the Fourier-grouped columns, bit for bit against
the oracle's generators and through the solver; the Fourier-grouped estimate
equals the hierarchical one at level boundaries; argument errors."""

import numpy as np
import pytest

from conftest import gpu_binding, to_dev
from oracle import general
from oracle.mask import MASK_NONE, MASK_Z2, MASK_Z4
from oracle.operators import Operator as OracleOp
from paper_1302_4018_amd import inputs

pytestmark = pytest.mark.gpu
REL = 1e-10


@pytest.mark.parametrize("dims,ncomp,mask,probe,levels", [
    ([16, 16], 1, MASK_Z2, general.PROBE_STOPPED, 0),
    ([16, 16], 1, MASK_Z2, general.PROBE_STOPPED, 2),
    ([4, 8, 2], 3, MASK_Z4, general.PROBE_STOPPED, 1),
    ([2, 4, 8, 4], 1, MASK_NONE, general.PROBE_STOPPED, 2),
    ([8, 8, 8], 1, MASK_Z2, general.PROBE_STOPPED, 7),
    ([16, 16], 1, MASK_Z2, general.PROBE_FOURIER, 0),
    ([4, 8, 2], 3, MASK_Z4, general.PROBE_FOURIER, 0),
    ([2, 4, 8, 4], 1, MASK_NONE, general.PROBE_FOURIER, 0),
    ([32, 32, 32, 32], 3, MASK_Z4, general.PROBE_FOURIER, 0),
    ([32, 32, 32, 32], 3, MASK_Z4, general.PROBE_STOPPED, 3),
])
def test_variant_probes_bit_exact(dims, ncomp, mask, probe, levels):
    tip = gpu_binding()
    V = int(np.prod(dims))
    print(f"variant generator: dims {dims} probe {probe} levels {levels} mask {mask}", flush=True)
    ms = sorted({0, 1, 3, 5, 16, V // 3, V - 1})
    for comp in range(ncomp):
        for m in ms:
            got = tip.tip_probe_vectors(dims, ncomp, mask, 77, m, 1, comp, probe=probe,
                                        stop_levels=levels)[0].cpu().numpy()
            want = general.rhs_kind(dims, ncomp, m, comp, 77, mask, probe, levels=levels)[:, comp]
            assert np.array_equal(got, want), (m, comp)


@pytest.mark.parametrize("dims,kind,n,mask,probe,levels,prec", [
    ([16, 16], 0, 64, MASK_Z2, general.PROBE_STOPPED, 1, "fp64"),
    ([16, 16], 0, 64, MASK_Z2, general.PROBE_FOURIER, 0, "fp64"),     # complex solves of a real operator
    ([8, 4, 8], 1, 12, MASK_Z4, general.PROBE_FOURIER, 0, "mixed"),
    ([4, 4, 4, 8], 1, 8, MASK_Z4, general.PROBE_STOPPED, 2, "fp64"),
    ([8, 8, 8], 0, 40, MASK_NONE, general.PROBE_STOPPED, 1, "fp64"),
])
def test_variants_through_the_solver(dims, kind, n, mask, probe, levels, prec):
    tip = gpu_binding()
    w = inputs.couplings(dims, seed=630)
    U = inputs.haar_links(dims, seed=631) if kind == 1 else None
    orc = OracleOp(dims, kind, mass=0.2, coupling=w, links=U)
    gop = tip.Operator(dims, kind, mass=0.2, coupling=to_dev(w), links=to_dev(U))
    precision = tip.PREC_MIXED if prec == "mixed" else tip.PREC_FP64
    print(f"variant solve: dims {dims} kind {kind} probe {probe} levels {levels} {prec}", flush=True)
    est, q, st = tip.trace_inv_probe(gop, n, 1e-12, 4018, mask=mask, probe=probe, stop_levels=levels,
                                     precision=precision)
    est_o, q_o, _ = general.trace_inv_probe(orc, n, 1e-12, 4018, mask, probe=probe, levels=levels)
    assert st["max_true_relres"] <= 1e-12
    assert np.max(np.abs(est - est_o) / np.abs(est_o)) <= REL
    assert np.max(np.abs(q - q_o) / np.abs(q_o)) <= REL


def test_fourier_equals_hierarchy_at_level_boundaries():
    """8^3 scalar torus, Z2 mask: at s = 1, 8, 64 (every level boundary of three
    active dimensions) the Fourier-grouped and hierarchical estimates agree to
    the solve tolerance; between them they differ."""
    tip = gpu_binding()
    dims = [8, 8, 8]
    w = inputs.couplings(dims, seed=640)
    gop = tip.Operator(dims, tip.KIND_SCALAR, mass=0.3, coupling=to_dev(w))
    eh, _, _ = tip.trace_inv_probe(gop, 64, 1e-13, 11, mask=MASK_Z2)
    ef, _, _ = tip.trace_inv_probe(gop, 64, 1e-13, 11, mask=MASK_Z2, probe=tip.PROBE_FOURIER)
    for k in (0, 3, 6):
        assert abs(ef[k] - eh[k]) <= 1e-11 * abs(eh[k]), k
    assert abs(ef[1] - eh[1]) > 1e-6 * abs(eh[1])


def test_variant_argument_errors():
    tip = gpu_binding()
    gop = tip.Operator([6, 4], tip.KIND_SCALAR, mass=0.5)
    for probe in (tip.PROBE_STOPPED, tip.PROBE_FOURIER):
        est, q, st = tip.trace_inv_probe(gop, 4, 1e-10, 1, probe=probe, raise_on_error=False)
        assert st["status"] == tip.TIP_EINVAL and "power-of-two" in tip.tip_last_error()
    gop = tip.Operator([4, 4], tip.KIND_SCALAR, mass=0.5)
    est, q, st = tip.trace_inv_probe(gop, 4, 1e-10, 1, probe=tip.PROBE_STOPPED, stop_levels=-2,
                                     raise_on_error=False)
    assert st["status"] == tip.TIP_EINVAL and "stop_levels" in tip.tip_last_error()
