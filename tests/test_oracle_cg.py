"""Pins for the oracle's CG solves (Sec. 1.1.2): dense LU, FFT and pure-gauge exact solves."""

import numpy as np
import pytest

from oracle import exact
from oracle.cg import CGError, cg_solve
from oracle.lattice import volume
from oracle.operators import Operator
from paper_1302_4018_amd import inputs


def test_cg_matches_dense_solve():
    dims = [4, 2, 4]
    w = inputs.couplings(dims, seed=1)
    mf = inputs.mass_field(dims, seed=2)
    U = inputs.haar_links(dims, seed=3)
    rng = np.random.default_rng(0)
    for op in [Operator(dims, 0, mass_field=mf, coupling=w),
               Operator(dims, 1, mass_field=mf, coupling=w, links=U)]:
        n = op.V * op.ncomp
        b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        b = b.reshape(op.V, op.ncomp)
        x, it, rr = cg_solve(op.apply, b, 1e-12, 1000)
        xd = np.linalg.solve(op.dense(), b.reshape(-1)).reshape(b.shape)
        assert rr <= 1e-12
        assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_cg_matches_fft_solve():
    dims = [16, 16, 8]
    op = Operator(dims, 0, mass=0.05)
    rng = np.random.default_rng(1)
    b = rng.choice([-1.0, 1.0], size=op.V)
    x, it, rr = cg_solve(op.apply, b, 1e-10, 10000)
    xe = exact.fft_solve(dims, 0.05, b[:, None])[:, 0]
    assert np.abs(xe.imag).max() < 1e-12
    assert np.linalg.norm(x - xe.real) <= 1e-8 * np.linalg.norm(xe)
    # quadrature error of CG from x0 = 0 is nonnegative and O(||r||^2)
    qe = np.vdot(b, xe).real
    q = np.vdot(b, x).real
    assert -1e-12 * qe <= qe - q <= (1e-10 * np.linalg.norm(b)) ** 2 / 0.05 + 1e-12 * qe


def test_cg_matches_pure_gauge_solve():
    dims = [8, 8, 4, 4]
    V = volume(dims)
    g = inputs.random_site_unitaries(V, seed=31)
    op = Operator(dims, 1, mass=0.1, links=exact.pure_gauge_links(g, dims))
    rng = np.random.default_rng(2)
    b = rng.standard_normal((V, 3)) + 1j * rng.standard_normal((V, 3))
    x, it, rr = cg_solve(op.apply, b, 1e-10, 10000)
    xe = exact.pure_gauge_solve(dims, 0.1, g, b)
    assert np.linalg.norm(x - xe) <= 1e-8 * np.linalg.norm(xe)


def test_cg_failure_modes():
    op = Operator([4, 4], 0, mass=0.1)
    b = np.ones(16)
    b[3] = -1.0
    with pytest.raises(CGError) as e:
        cg_solve(op.apply, b, 1e-12, 1)
    assert e.value.kind == "noconv"
    neg = Operator([4, 4], 0, mass=-10.0)        # negative definite
    with pytest.raises(CGError) as e:
        cg_solve(neg.apply, b, 1e-12, 100)
    assert e.value.kind == "breakdown"
    x, it, rr = cg_solve(op.apply, np.zeros(16), 1e-12, 10)
    assert it == 0 and not np.any(x)
