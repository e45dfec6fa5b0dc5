"""Pins for the oracle's trace estimator: exact recovery at s = N (eq. removebias),
closed-form traces (Sec. 5), the partial-sum identity, probing of A^p
(Proposition 1.2) and the red-black example of Sec. 2."""

import math

import numpy as np
import pytest

from oracle import exact, mask
from oracle.estimator import (checkpoint_sizes, estimates_from_quadratures,
                              neumaier_prefix_sums, trace_inv_probe)
from oracle.hadamard import hadamard_kron
from oracle.hierperm import hier_perm
from oracle.lattice import total_levels, volume
from oracle.operators import Operator
from oracle.probing import rhs
from paper_1302_4018_amd import inputs


def test_closed_form_trace_agrees_with_dense_lu():
    for dims, m in [([16, 16], 0.1), ([4, 8, 4], 0.05)]:
        op = Operator(dims, 0, mass=m)
        assert abs(exact.free_trace_inverse(dims, m) - exact.dense_trace_inverse(op.dense()).real) \
            <= 1e-12 * exact.free_trace_inverse(dims, m)


def test_c1_exact_recovery_at_s_equals_N():
    """2-D 16x16, m = 0.1, Z2 mask, tol 1e-12: T_256 = Tr(A^-1) = 116.9497434033..."""
    op = Operator([16, 16], 0, mass=0.1)
    est, q, st = trace_inv_probe(op, 256, 1e-12, 4018, mask.MASK_Z2)
    exact_tr = exact.free_trace_inverse([16, 16], 0.1)
    assert abs(exact_tr - 116.949743403339) < 1e-11
    assert abs(est[-1] - exact_tr) <= 1e-12 * exact_tr
    assert len(est) == 9


@pytest.mark.parametrize("kind_mask", [(1, mask.MASK_Z4), (1, mask.MASK_NONE), (0, mask.MASK_Z4)])
def test_covariant_and_complex_exact_recovery(kind_mask):
    kind, mk = kind_mask
    dims = [2, 2, 4, 2]
    mf = inputs.mass_field(dims, seed=40)
    w = inputs.couplings(dims, seed=41)
    U = inputs.haar_links(dims, seed=42) if kind == 1 else None
    op = Operator(dims, kind, mass_field=mf, coupling=w, links=U)
    est, q, st = trace_inv_probe(op, op.V, 1e-12, 9, mk)
    tr = exact.dense_trace_inverse(op.dense())
    assert abs(est[-1] - tr) <= 1e-10 * abs(tr)


CASES = [([8, 8], 0, mask.MASK_Z2), ([4, 4, 2], 0, mask.MASK_Z2), ([4, 2, 2, 2], 1, mask.MASK_Z4),
         ([2, 8, 4], 0, mask.MASK_NONE)]


@pytest.mark.parametrize("dims,kind,mk", CASES)
def test_partial_sum_identity(dims, kind, mk):
    """T_{2^t} equals the sum of masked A^-1 entries over same-colour pairs."""
    V = volume(dims)
    w = inputs.couplings(dims, seed=50)
    U = inputs.haar_links(dims, seed=51) if kind == 1 else None
    op = Operator(dims, kind, mass=0.3, coupling=w, links=U)
    est, q, st = trace_inv_probe(op, V, 1e-13, 77, mk)
    Ainv = np.linalg.inv(op.dense())
    P = hier_perm(dims)
    L = total_levels(dims)
    z0 = np.stack([mask.mask_values(77, V, op.ncomp, c, mk) for c in range(op.ncomp)])
    for t, s in enumerate(checkpoint_sizes(V)):
        ref = exact.partial_sum_estimate(Ainv, P, L, t, op.ncomp, z0)
        assert abs(est[t] - ref) <= 1e-10 * abs(ref)


def _probe_trace_of_power(op, p, s, mk):
    """(1/s) sum_{m<s} sum_c b^H A^p b, using only matvecs."""
    P = hier_perm(op.dims)
    tot = 0.0
    for m in range(s):
        for c in range(op.ncomp):
            b = rhs(op.dims, op.ncomp, m, c, 5, mk, P)
            y = b
            for _ in range(p):
                y = op.apply(y)
            tot += np.vdot(b, y)
    return tot / s


def test_probing_powers_proposition_1_2():
    """Tr(A^p) is exact once same-colour sites are more than p apart:
    8^3 torus -> distance 2 at s = 2, distance 4 at s = 16, distance 8 at s = 128."""
    dims = [8, 8, 8]
    op = Operator(dims, 0, mass=0.25, coupling=inputs.couplings(dims, seed=60))
    A = op.dense().real
    trp = {p: np.trace(np.linalg.matrix_power(A, p)) for p in (1, 2, 3, 4)}
    close = lambda a, b: abs(a - b) <= 1e-13 * abs(b)
    assert close(_probe_trace_of_power(op, 1, 2, mask.MASK_Z2), trp[1])
    assert not close(_probe_trace_of_power(op, 2, 2, mask.MASK_Z2), trp[2])
    assert close(_probe_trace_of_power(op, 2, 16, mask.MASK_Z2), trp[2])
    assert close(_probe_trace_of_power(op, 3, 16, mask.MASK_Z2), trp[3])
    assert not close(_probe_trace_of_power(op, 4, 16, mask.MASK_Z2), trp[4])
    assert close(_probe_trace_of_power(op, 4, 128, mask.MASK_Z2), trp[4])
    # constant coefficients: closed form Tr(A^p) = sum lambda^p
    free = Operator(dims, 0, mass=0.25)
    assert close(_probe_trace_of_power(free, 3, 16, mask.MASK_NONE),
                 exact.free_trace_power(dims, 0.25, 3))


def test_red_black_example_of_section_2():
    """2^n x 2^n torus in lexicographic order: natural-order Hadamard vectors
    need s = 2^{n+1} for the exact Tr(A); in red-black (hierarchical) order
    the first and the middle vector (s = 2) suffice."""
    n = 3
    dims = [2 ** n, 2 ** n]
    op = Operator(dims, 0, mass=0.5)
    A = op.dense().real
    H = hadamard_kron(op.V)
    tr = np.trace(A)

    def natural(s):
        Z = H[:, :s]
        return np.trace(Z.T @ A @ Z) / s

    for s in (2, 4, 2 ** n):
        assert abs(natural(s) - tr) > 1e-6
    assert abs(natural(2 ** (n + 1)) - tr) < 1e-12
    assert abs(_probe_trace_of_power(op, 1, 2, mask.MASK_NONE) - tr) < 1e-12


def test_checkpoints_and_compensated_sums():
    assert checkpoint_sizes(256) == [1, 2, 4, 8, 16, 32, 64, 128, 256]
    assert checkpoint_sizes(100) == [1, 2, 4, 8, 16, 32, 64, 100]
    assert checkpoint_sizes(1) == [1]
    rng = np.random.default_rng(9)
    v = rng.standard_normal(1000) * 10.0 ** rng.integers(-8, 8, 1000)
    S = neumaier_prefix_sums(v)
    for k in (1, 10, 999, 1000):
        assert S[k - 1] == math.fsum(v[:k]) or abs(S[k - 1] - math.fsum(v[:k])) <= 1e-15 * abs(math.fsum(v[:k]))
    q = np.array([1.0, 3.0, 2.0 + 1j, 6.0, 5.0])
    est = estimates_from_quadratures(q)
    assert np.allclose(est, [1.0, 2.0, 3.0 + 0.25j, 17.0 / 5 + 0.2j])
