"""The comparison probes of Sec. 5 (plain Z2 Monte Carlo and Hadamard vectors
in natural order) against hierarchical probing, with exact quadratures from a
dense inverse on a 32 x 32 torus whose trace is known in closed form
(m = 0.05).  Pins the generators (natural order = columns of the Sylvester
matrix H_N, random = the sweep masks) and the qualitative result of Sec. 5:
at the colouring completion points hierarchical probing has a much smaller
error than both, and it (like natural order) is exact at s = N."""

import numpy as np
import pytest

from oracle import exact, general, mask
from oracle.hadamard import hadamard_kron
from oracle.lattice import volume
from oracle.operators import Operator

DIMS = [32, 32]
M = 0.05
SEEDS = range(6)


def test_natural_probes_are_sylvester_columns():
    dims = [4, 8]
    V = volume(dims)
    H = hadamard_kron(V)
    z0 = general.mask_sweep(3, V, 1, 0, mask.MASK_Z2, 0)
    for m in [0, 1, 5, V - 1]:
        b = general.rhs_kind(dims, 1, m, 0, 3, mask.MASK_Z2, general.PROBE_NATURAL)[:, 0]
        assert np.array_equal(b, z0 * H[:, m])


def test_random_probes_are_independent_sweep_masks():
    dims = [6, 5]
    V = volume(dims)
    for m in [0, 1, 7]:
        b = general.rhs_kind(dims, 3, m, 2, 9, mask.MASK_Z4, general.PROBE_RANDOM)
        assert np.array_equal(b[:, 2], general.mask_sweep(9, V, 3, 2, mask.MASK_Z4, m))
        assert not np.any(b[:, :2])
    with pytest.raises(ValueError):
        general.rhs_kind(dims, 1, 0, 0, 9, mask.MASK_NONE, general.PROBE_RANDOM)


@pytest.fixture(scope="module")
def errors():
    op = Operator(DIMS, 0, mass=M)
    Ainv = np.linalg.inv(op.dense().real)
    tr = exact.free_trace_inverse(DIMS, M)
    out = {}
    for probe in (general.PROBE_HIERARCHICAL, general.PROBE_NATURAL, general.PROBE_RANDOM):
        e = [np.abs(general.estimates_dense(Ainv, DIMS, 1, op.V, s, mask.MASK_Z2, probe).real - tr) / tr
             for s in SEEDS]
        out[probe] = np.sqrt(np.mean(np.array(e) ** 2, axis=0))      # RMS over masks, per s = 2^k
    return out


def test_hierarchical_beats_monte_carlo_and_natural_order(errors):
    hier, nat, rnd = errors[0], errors[1], errors[2]
    # completion points of the distance-2 and distance-4 colourings in 2-D: s = 2^{2m+1}
    for k in (5, 7):                   # s = 32, 128
        assert hier[k] < rnd[k] / 2 and hier[k] < nat[k] / 2, k
    assert hier[9] < rnd[9] / 10       # s = 512
    assert hier[-1] < 1e-12 and nat[-1] < 1e-12 and rnd[-1] > 1e-4   # s = N: exact for the bases
