"""Tori whose sides are not all powers of two (Sec. 3.4): the generator
(binary levels, three-colouring level with F_3 columns, mask sweeps) bit for
bit against the oracle, and the whole probing run against the oracle's CG."""

import numpy as np
import pytest

from conftest import assert_gradient_entries, gpu_binding, to_dev
from oracle import general
from oracle.gradient import trace_inv_probe_grad as oracle_grad
from oracle.mask import MASK_NONE, MASK_Z2, MASK_Z4
from oracle.operators import Operator as OracleOp
from paper_1302_4018_amd import inputs

pytestmark = pytest.mark.gpu
REL = 1e-10

SHAPES = [[6, 4], [12, 5, 8], [24, 6, 10], [3, 3, 3], [5], [48, 8], [7, 1, 2], [6, 4, 4, 6], [12, 12]]


@pytest.mark.parametrize("dims", SHAPES)
def test_binary_colour_bit_exact(dims):
    tip = gpu_binding()
    got = tip.tip_hier_perm(dims).cpu().numpy().astype(np.int64)
    assert np.array_equal(got, general.binary_colour(dims).astype(np.int64))


@pytest.mark.parametrize("dims,ncomp,mask", [([6, 4], 1, MASK_Z2), ([12, 5, 8], 3, MASK_Z4), ([3, 3, 3], 1, MASK_NONE),
                                            ([24, 6, 10], 1, MASK_Z4), ([48, 8], 3, MASK_Z2), ([5], 1, MASK_Z2)])
def test_probe_vectors_bit_exact_with_f3_columns_and_sweeps(dims, ncomp, mask):
    tip = gpu_binding()
    lv = general.Levels(dims)
    V = int(np.prod(dims))
    PB, C = general.binary_colour(dims, lv), general.last_level_colour(dims, lv)
    edge = 1 << lv.LB
    ms = sorted({0, 1, edge - 1, edge, edge + 1, lv.gamma - 1, lv.gamma, lv.gamma + edge, V - 1} & set(range(V)))
    for comp in range(ncomp):
        for m in ms:
            got = tip.tip_probe_vectors(dims, ncomp, mask, 77, m, 1, comp)[0].cpu().numpy()
            want = general.rhs(dims, ncomp, m, comp, 77, mask, lv, PB, C)[:, comp]
            assert np.array_equal(got, want), (m, comp)


@pytest.mark.parametrize("dims,kind,n,mask,coupled", [
    ([6, 10], 0, 60, MASK_Z2, True),         # gamma = 12: binary, F_3 columns, then 4 more sweeps
    ([12, 5, 8], 0, 9, MASK_Z2, False),      # no binary level: gamma = 3, F_3 from m = 1
    ([3, 3, 3], 0, 27, MASK_Z4, True),
    ([24, 6, 10], 0, 40, MASK_Z2, True),
    ([6, 4, 4, 6], 1, 20, MASK_Z4, False),   # covariant, generic stencil
    ([7, 1, 2], 1, 14, MASK_NONE, True),
])
def test_estimates_match_oracle(dims, kind, n, mask, coupled):
    tip = gpu_binding()
    w = inputs.couplings(dims, seed=500) if coupled else None
    mf = inputs.mass_field(dims, m0=0.2, seed=501)
    U = inputs.haar_links(dims, seed=502) if kind == 1 else None
    orc = OracleOp(dims, kind, mass_field=mf, coupling=w, links=U)
    gop = tip.Operator(dims, kind, mass_field=to_dev(mf), coupling=to_dev(w), links=to_dev(U))
    print(f"general parity: dims {dims} kind {kind} n {n} mask {mask}", flush=True)
    est, q, st = tip.trace_inv_probe(gop, n, 1e-12, 4018, mask=mask)
    est_o, q_o, _ = general.trace_inv_probe(orc, n, 1e-12, 4018, mask)
    assert st["even_odd"] == 0
    assert np.max(np.abs(est - est_o) / np.abs(est_o)) <= REL
    assert np.max(np.abs(q - q_o) / np.abs(q_o)) <= REL


def test_gradient_on_an_odd_torus():
    tip = gpu_binding()
    dims = [6, 5, 4]
    w = inputs.couplings(dims, seed=510)
    mf = inputs.mass_field(dims, m0=0.3, seed=511)
    orc = OracleOp(dims, 0, mass_field=mf, coupling=w)
    gop = tip.Operator(dims, 0, mass_field=to_dev(mf), coupling=to_dev(w))
    with tip.OpHandle(gop) as h:
        est, q, gm, gw, st = h.trace_inv_probe_grad(30, 1e-12, 4018)
    T, gm_o, gw_o, _ = oracle_grad(orc, 30, 1e-12, 4018, MASK_Z2)
    assert abs(est[-1] - T) <= REL * abs(T)
    assert_gradient_entries(gm.cpu().numpy(), gw.cpu().numpy(), gm_o, gw_o, 1e-12, orc.V, float(np.min(mf)))


def _no_split(tip, fn):
    import os
    os.environ["TIP_CONJ_SPLIT"] = "0"
    try:
        return fn()
    finally:
        del os.environ["TIP_CONJ_SPLIT"]


@pytest.mark.parametrize("dims,n,prec,reused", [
    ([12, 5, 8], 9, "fp64", 3),      # gamma = 3: probes 2, 5, 8 are conjugates of 1, 4, 7
    ([6, 10], 60, "fp64", 20),       # gamma = 12: columns 8..11 of each of 5 sweeps
    ([6, 10], 60, "mixed", 20),
])
def test_conjugate_f3_columns_reuse_their_partner(dims, n, prec, reused):
    """Real operator, Z2 mask: column j3 = 2 is the conjugate of column j3 = 1,
    so its quadrature is conj(q) of probe m - 2^LB and is not solved; j3 = 0
    probes run in real arithmetic.  Same estimates as solving every probe."""
    tip = gpu_binding()
    w = inputs.couplings(dims, seed=520)
    mf = inputs.mass_field(dims, m0=0.2, seed=521)
    orc = OracleOp(dims, 0, mass_field=mf, coupling=w)
    gop = tip.Operator(dims, 0, mass_field=to_dev(mf), coupling=to_dev(w))
    precision = tip.PREC_MIXED if prec == "mixed" else tip.PREC_FP64
    print(f"conjugate split: dims {dims} n {n} {prec}", flush=True)
    est, q, st = tip.trace_inv_probe(gop, n, 1e-12, 4018, mask=MASK_Z2, precision=precision)
    est_a, q_a, st_a = _no_split(tip, lambda: tip.trace_inv_probe(gop, n, 1e-12, 4018, mask=MASK_Z2,
                                                                   precision=precision))
    assert st["reused"] == reused and st["solves"] == n - reused
    assert st_a["reused"] == 0 and st_a["solves"] == n
    assert np.max(np.abs(q - q_a) / np.abs(q_a)) <= 1e-10
    assert np.max(np.abs(est - est_a) / np.abs(est_a)) <= 1e-12
    est_o, q_o, _ = general.trace_inv_probe(orc, n, 1e-12, 4018, MASK_Z2)
    assert np.max(np.abs(est - est_o) / np.abs(est_o)) <= REL
    assert np.max(np.abs(q - q_o) / np.abs(q_o)) <= REL


def test_conjugate_reuse_across_a_resumed_run():
    """m_begin = 30 on [6, 10] (gamma = 12): probes 32..35 take the conjugates of
    28..31, two of which come from the earlier call's quadratures."""
    tip = gpu_binding()
    dims = [6, 10]
    w = inputs.couplings(dims, seed=530)
    gop = tip.Operator(dims, 0, mass=0.3, coupling=to_dev(w))
    est, q, st = tip.trace_inv_probe(gop, 60, 1e-12, 7, mask=MASK_Z2)
    est1, q1, _ = tip.trace_inv_probe(gop, 30, 1e-12, 7, mask=MASK_Z2)
    est2, q2, st2 = tip.trace_inv_probe(gop, 60, 1e-12, 7, mask=MASK_Z2, m_begin=30, quadratures=q1)
    assert np.array_equal(q2[:30], q1)
    assert np.max(np.abs(q2 - q) / np.abs(q)) <= 1e-10
    assert np.max(np.abs(est2 - est) / np.abs(est)) <= 1e-12
    assert st2["reused"] == 12
