"""The stored oracle quadratures (tests/golden/quadratures_*.txt, written by
tests/golden/make_quadratures.py) against the oracle as it stands, on a
sample small enough for the CPU suite: a stale or hand-edited file fails."""

import numpy as np

from conftest import read_quadratures
from oracle import general
from oracle.estimator import trace_inv_probe
from oracle.mask import MASK_Z2, MASK_Z4
from oracle.operators import Operator
from paper_1302_4018_amd import inputs


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b))))


def test_c2_first_probes():
    dims = [32, 32, 32]
    op = Operator(dims, 0, mass=0.05, coupling=inputs.couplings(dims, seed=1))
    _, q, _ = trace_inv_probe(op, 2, 1e-10, 4018, MASK_Z2)
    stored = read_quadratures("quadratures_c2_32x32x32.txt")["c2"]
    assert len(stored) == 512
    assert _rel(q, stored[:2]) <= 1e-13


def test_c3_first_probe():
    dims = [16, 16, 16, 16]
    op = Operator(dims, 1, mass=0.1, links=inputs.haar_links(dims, seed=3))
    _, q, _ = trace_inv_probe(op, 1, 1e-10, 4018, MASK_Z4)
    stored = read_quadratures("quadratures_c3_16x16x16x16.txt")["c3"]
    assert len(stored) == 64
    assert _rel(q, stored[:1]) <= 1e-13


def test_c4_smallest_tori():
    tori = inputs.uneven_tori()
    stored = read_quadratures("quadratures_c4_uneven_tori.txt")
    assert len(stored) == 64 and all(len(v) == 4 for v in stored.values())
    vol = [int(np.prod(t["dims"])) for t in tori]
    for i in sorted(range(len(tori)), key=lambda k: vol[k])[:3]:
        t = tori[i]
        op = Operator(t["dims"], 0, mass=t["mass"], coupling=inputs.uneven_torus_couplings(t["dims"], i))
        _, q, _ = general.trace_inv_probe(op, 4, 1e-10, 4018, MASK_Z2)
        assert _rel(q, stored[f"torus{i}"]) <= 1e-13, i
