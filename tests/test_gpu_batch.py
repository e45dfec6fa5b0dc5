"""Batches of independent problems solved together (trace_inv_probe_batch:
one launch per CG phase for every problem of a group): every problem against
its own trace_inv_probe call and against the oracle, batches that mix
operator kinds, element types, probe classes and precisions, the batch
autotuner, and the 64 uneven 3-D tori (sides 8..48) against the stored
oracle quadratures."""

import numpy as np
import pytest

from conftest import gpu_binding, read_quadratures, to_dev
from oracle import general
from oracle.estimator import estimates_from_quadratures
from oracle.mask import MASK_Z2, MASK_Z4
from oracle.operators import Operator as OracleOp
from paper_1302_4018_amd import inputs

pytestmark = pytest.mark.gpu
REL = 1e-10

SMALL = [([6, 10, 3], 0.1, 24), ([8, 8, 8], 0.05, 16), ([5, 9, 7], 0.2, 40), ([12, 4, 6], 0.02, 8),
         ([3, 3, 3], 0.3, 27), ([16, 6, 2], 0.15, 32)]


def _ops(tip, cases):
    orcs, gops = [], []
    for i, (dims, m, _) in enumerate(cases):
        w = inputs.uneven_torus_couplings(dims, i)
        orcs.append(OracleOp(dims, 0, mass=m, coupling=w))
        gops.append(tip.Operator(dims, tip.KIND_SCALAR, mass=m, coupling=to_dev(w)))
    return orcs, gops


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_single_calls_and_oracle(precision):
    tip = gpu_binding()
    prec = tip.PREC_MIXED if precision == "mixed" else tip.PREC_FP64
    orcs, gops = _ops(tip, SMALL)
    ns = [n for _, _, n in SMALL]
    print(f"batch of {len(ns)} small tori, {precision}", flush=True)
    out = tip.trace_inv_probe_batch(gops, ns, 1e-12, 4018, precision=prec)
    for i, (est, st) in enumerate(out):
        assert st["status"] == 0 and st["max_true_relres"] <= 1e-12
        single, q1, st1 = tip.trace_inv_probe(gops[i], ns[i], 1e-12, 4018, precision=prec)
        assert st["reused"] == st1["reused"] and st["solves"] == st1["solves"], i
        assert np.max(np.abs(est - single) / np.abs(single)) <= REL, i
        assert np.max(np.abs(st["quadratures"] - q1) / np.abs(q1)) <= REL, i
        est_o, _, _ = general.trace_inv_probe(orcs[i], ns[i], 1e-12, 4018, MASK_Z2)
        assert np.max(np.abs(est - est_o) / np.abs(est_o)) <= REL, i


def test_batch_mixing_kinds_masks_and_precisions():
    """Covariant and scalar problems, Z4 and Z2 masks, real and complex
    solves, FP64 and mixed precision in one call: one group per (kind,
    element type, precision), each against the oracle."""
    tip = gpu_binding()
    cases = [  # dims, kind, mass, n, mask, coupled
        ([4, 4, 4, 4], 1, 0.1, 6, MASK_Z4, False),
        ([6, 4, 3, 2], 1, 0.2, 5, MASK_Z4, True),
        ([8, 8], 0, 0.05, 10, MASK_Z4, True),
        ([5, 9, 7], 0, 0.2, 12, MASK_Z2, True),
        ([16, 16], 0, 0.1, 33, MASK_Z2, False),
    ]
    for prec in (tip.PREC_FP64, tip.PREC_MIXED):
        gops, orcs, ns = [], [], []
        for k, (dims, kind, m, n, mask, coupled) in enumerate(cases):
            w = inputs.couplings(dims, seed=700 + k) if coupled else None
            U = inputs.haar_links(dims, seed=710 + k) if kind == 1 else None
            orcs.append(OracleOp(dims, kind, mass=m, coupling=w, links=U))
            gops.append(tip.Operator(dims, kind, mass=m, coupling=to_dev(w), links=to_dev(U)))
            ns.append(n)
        masks = [c[4] for c in cases]
        print(f"mixed batch, precision {prec}", flush=True)
        out = tip.trace_inv_probe_batch(gops, ns, 1e-12, 99, mask=masks, precision=prec)
        for i, (est, st) in enumerate(out):
            assert st["status"] == 0, i
            est_o, q_o, _ = general.trace_inv_probe(orcs[i], ns[i], 1e-12, 99, masks[i])
            assert np.max(np.abs(est - est_o) / np.abs(est_o)) <= REL, (prec, i)
            assert np.max(np.abs(st["quadratures"] - q_o) / np.abs(q_o)) <= REL, (prec, i)


def test_batch_autotuner_picks_a_candidate():
    tip = gpu_binding()
    orcs, gops = _ops(tip, SMALL)
    ns = [n for _, _, n in SMALL]
    best, tried = tip.tip_autotune_batch(gops, ns, 1e-10, 4018, sample_vectors=8)
    assert len(tried) == 12
    assert best["rhs_block"] in (16, 32, 64) and best["item_sites"] in (256, 512, 1024, 2048)
    assert best["seconds_per_solve"] == min(t["seconds_per_solve"] for t in tried)
    out = tip.trace_inv_probe_batch(gops, ns, 1e-12, 4018, rhs_block=best["rhs_block"],
                                    item_sites=best["item_sites"])
    for i, (est, st) in enumerate(out):
        est_o, _, _ = general.trace_inv_probe(orcs[i], ns[i], 1e-12, 4018, MASK_Z2)
        assert np.max(np.abs(est - est_o) / np.abs(est_o)) <= REL, i


def test_batch_validates_every_problem_first():
    tip = gpu_binding()
    _, gops = _ops(tip, SMALL[:3])
    with pytest.raises(tip.TipError) as e:
        tip.trace_inv_probe_batch(gops, [4, 10 ** 6, 4], 1e-10, 1)
    assert "torus 1" in str(e.value) or "torus 1" in tip.tip_last_error()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_uneven_tori_batch_first_probes_against_oracle(precision):
    """The 64 uneven 3-D tori in one batch call: every problem converges, and
    on every torus the estimates at s = 1, 2, 4 (which use probes 0..3 only,
    F_3 columns included on tori with odd sides) match the stored oracle
    quadratures."""
    tip = gpu_binding()
    tori = inputs.uneven_tori()
    gops = []
    for i, t in enumerate(tori):
        w = inputs.uneven_torus_couplings(t["dims"], i)
        gops.append(tip.Operator(t["dims"], tip.KIND_SCALAR, mass=t["mass"], coupling=to_dev(w)))
    ns = [t["n_vectors"] for t in tori]
    prec = tip.PREC_MIXED if precision == "mixed" else tip.PREC_FP64
    out = tip.trace_inv_probe_batch(gops, ns, 1e-10, 4018, mask=MASK_Z2, precision=prec)
    assert all(st["status"] == 0 and st["max_true_relres"] <= 1e-10 for _, st in out)
    golden = read_quadratures("quadratures_c4_uneven_tori.txt")
    for i, t in enumerate(tori):
        est_o = estimates_from_quadratures(golden[f"torus{i}"])
        assert np.max(np.abs(out[i][0][:3] - est_o) / np.abs(est_o)) <= REL, (i, t["dims"])


@pytest.mark.parametrize("probe,precision", [(general.PROBE_NATURAL, "fp64"), (general.PROBE_RANDOM, "fp64"),
                                             (general.PROBE_RANDOM, "mixed")])
def test_batch_comparison_probe_kinds_against_oracle(probe, precision):
    """The batch with the comparison probes of Sec. 5 (natural-order Hadamard,
    plain Monte Carlo), whose right-hand sides the batch kernels regenerate
    per lane rather than from per-site probe codes: every torus against the
    oracle, scalar and covariant; odd sides with the random probes (natural
    order takes power-of-two sides)."""
    tip = gpu_binding()
    if probe == general.PROBE_NATURAL:
        cases = [([16, 16], 0, 0.2, 24), ([8, 4, 8], 1, 0.15, 6), ([8, 8, 8], 0, 0.1, 32), ([4, 4, 4, 8], 1, 0.2, 5)]
    else:
        cases = [([6, 10], 0, 0.2, 24), ([8, 4, 8], 1, 0.15, 6), ([16, 16], 0, 0.1, 32), ([5, 9, 7], 0, 0.2, 12)]
    gops, orcs, ns = [], [], []
    for k, (dims, kind, m, n) in enumerate(cases):
        w = inputs.couplings(dims, seed=720 + k)
        U = inputs.haar_links(dims, seed=730 + k) if kind == 1 else None
        orcs.append(OracleOp(dims, kind, mass=m, coupling=w, links=U))
        gops.append(tip.Operator(dims, kind, mass=m, coupling=to_dev(w), links=to_dev(U)))
        ns.append(n)
    prec = tip.PREC_MIXED if precision == "mixed" else tip.PREC_FP64
    print(f"batch with probe kind {probe}, {precision}", flush=True)
    out = tip.trace_inv_probe_batch(gops, ns, 1e-12, 31, mask=MASK_Z4, precision=prec, probe=probe)
    for i, (est, st) in enumerate(out):
        assert st["status"] == 0, i
        est_o, q_o, _ = general.trace_inv_probe(orcs[i], ns[i], 1e-12, 31, MASK_Z4, probe=probe)
        assert np.max(np.abs(est - est_o) / np.abs(est_o)) <= REL, (probe, i)
        assert np.max(np.abs(st["quadratures"] - q_o) / np.abs(q_o)) <= REL, (probe, i)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("ndim", [1, 2, 4])
def test_batch_stencil_per_dimension(ndim, precision):
    """Batches whose scalar problems all have the same dimension run the
    stencil compiled for that dimension (lane k of a site reads the site's
    coupling or mass k for the site's lanes): odd and even sides, a mass
    field, no couplings, and blocks of fewer lanes than a site has values
    (B = 1, 2, 4 against 2 ndim + 1), each against its own single call and
    the oracle."""
    tip = gpu_binding()
    cases = {  # dims, mass, mass field, coupled, probes
        1: [([30], 0.1, False, True, 1), ([17], 0.05, True, True, 2), ([64], 0.2, False, False, 5)],
        2: [([6, 10], 0.1, True, True, 2), ([9, 7], 0.05, False, True, 4), ([16, 16], 0.2, False, False, 24)],
        4: [([4, 6, 3, 5], 0.1, False, True, 3), ([6, 4, 4, 4], 0.2, True, True, 1), ([3, 5, 4, 2], 0.15, False, False, 20)],
    }[ndim]
    orcs, gops, ns = [], [], []
    for k, (dims, m, field, coupled, n) in enumerate(cases):
        w = inputs.couplings(dims, seed=740 + k) if coupled else None
        mf = inputs.mass_field(dims, m0=m, seed=750 + k) if field else None
        orcs.append(OracleOp(dims, 0, mass=m, mass_field=mf, coupling=w))
        gops.append(tip.Operator(dims, tip.KIND_SCALAR, mass=m, mass_field=to_dev(mf), coupling=to_dev(w)))
        ns.append(n)
    prec = tip.PREC_MIXED if precision == "mixed" else tip.PREC_FP64
    print(f"batch of {ndim}-D scalar problems, {precision}", flush=True)
    out = tip.trace_inv_probe_batch(gops, ns, 1e-12, 57, mask=MASK_Z2, precision=prec)
    for i, (est, st) in enumerate(out):
        assert st["status"] == 0 and st["max_true_relres"] <= 1e-12, i
        single, q1, _ = tip.trace_inv_probe(gops[i], ns[i], 1e-12, 57, mask=MASK_Z2, precision=prec)
        assert np.max(np.abs(st["quadratures"] - q1) / np.abs(q1)) <= REL, (ndim, i)
        est_o, q_o, _ = general.trace_inv_probe(orcs[i], ns[i], 1e-12, 57, MASK_Z2)
        assert np.max(np.abs(est - est_o) / np.abs(est_o)) <= REL, (ndim, i)
        assert np.max(np.abs(st["quadratures"] - q_o) / np.abs(q_o)) <= REL, (ndim, i)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_forked_chains_equal_one_chain(precision, monkeypatch):
    """Inside the chunk graphs each group's chain of launches runs on a side
    stream of its own; the groups share no data, so the quadratures are the
    same bit for bit as with one chain (TIP_BATCH_FORK=0), in both
    precisions (the mixed solver's reliable updates included)."""
    tip = gpu_binding()
    prec = tip.PREC_MIXED if precision == "mixed" else tip.PREC_FP64
    _, gops = _ops(tip, SMALL)
    ns = [n for _, _, n in SMALL]
    print(f"forked against one chain, {precision}", flush=True)
    a = tip.trace_inv_probe_batch(gops, ns, 1e-12, 4018, precision=prec)
    monkeypatch.setenv("TIP_BATCH_FORK", "0")
    b = tip.trace_inv_probe_batch(gops, ns, 1e-12, 4018, precision=prec)
    for i, ((ea, sa), (eb, sb)) in enumerate(zip(a, b)):
        assert np.array_equal(sa["quadratures"], sb["quadratures"]), i
        assert np.array_equal(ea, eb), i
        assert sa["total_iters"] == sb["total_iters"], i
