"""Pins for the oracle's lattice operators (Sec. 5 control problem and the
3-component covariant variant)."""

import numpy as np
import pytest

from oracle import exact
from oracle.lattice import coordinates, volume
from oracle.operators import Operator
from paper_1302_4018_amd import inputs


def _plane_wave(dims, kvec):
    X = coordinates(dims)
    phase = sum(2 * np.pi * kvec[j] * X[:, j] / dims[j] for j in range(len(dims)))
    return np.exp(1j * phase)


@pytest.mark.parametrize("dims", [[16, 16], [8, 4, 2], [4, 4, 4, 4], [2, 8]])
def test_fourier_modes_are_eigenvectors(dims):
    """Constant coefficients: A e_k = (m + sum 4 sin^2(pi k_mu / n_mu)) e_k."""
    mass = 0.37
    rng = np.random.default_rng(0)
    lam = exact.free_eigenvalues(dims, mass)
    op = Operator(dims, 0, mass=mass)
    U1 = np.broadcast_to(np.eye(3, dtype=np.complex128), (len(dims), volume(dims), 3, 3)).copy()
    opc = Operator(dims, 1, mass=mass, links=U1)
    for _ in range(4):
        kvec = [int(rng.integers(0, n)) for n in dims]
        e = _plane_wave(dims, kvec)
        want = lam[tuple(reversed(kvec))]
        assert np.allclose(op.apply(e), want * e, rtol=0, atol=1e-12)
        E = np.stack([e, 2 * e, -e], axis=1)
        assert np.allclose(opc.apply(E), want * E, rtol=0, atol=1e-12)


def test_weighted_laplacian_kills_constants():
    """Graph-Laplacian diagonal: A 1 = m 1 for any edge weights."""
    dims = [8, 4, 4]
    w = inputs.couplings(dims, seed=3)
    op = Operator(dims, 0, mass=0.05, coupling=w)
    one = np.ones(volume(dims))
    assert np.allclose(op.apply(one), 0.05 * one, atol=1e-13)


def _ops(dims, seed=5):
    V = volume(dims)
    w = inputs.couplings(dims, seed=seed)
    mf = inputs.mass_field(dims, seed=seed + 1)
    U = inputs.haar_links(dims, seed=seed + 2)
    return [Operator(dims, 0, mass=0.1),
            Operator(dims, 0, mass_field=mf, coupling=w),
            Operator(dims, 1, mass=0.1, links=U),
            Operator(dims, 1, mass_field=mf, coupling=w, links=U)]


@pytest.mark.parametrize("dims", [[4, 4], [2, 4, 2], [2, 2, 2, 4], [1, 4], [2, 2]])
def test_dense_assembly_equals_apply_and_is_hpd(dims):
    rng = np.random.default_rng(1)
    for op in _ops(dims):
        A = op.dense()
        n = A.shape[0]
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        assert np.allclose(A @ x, op.apply(x.reshape(op.V, op.ncomp)).reshape(-1), atol=1e-12)
        assert np.allclose(A, A.conj().T, atol=0)
        lam = np.linalg.eigvalsh(A)
        assert lam.min() >= op.mass_at_sites().min() - 1e-12


def test_hermitian_on_larger_lattice():
    dims = [8, 8, 4, 4]
    rng = np.random.default_rng(2)
    for op in _ops(dims):
        x = rng.standard_normal((op.V, op.ncomp)) + 1j * rng.standard_normal((op.V, op.ncomp))
        y = rng.standard_normal((op.V, op.ncomp)) + 1j * rng.standard_normal((op.V, op.ncomp))
        lhs = np.vdot(x, op.apply(y))
        rhs = np.vdot(op.apply(x), y)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_gauge_covariance():
    """U^g_mu(x) = g(x) U_mu(x) g(x+mu)^H  =>  A[U^g] G = G A[U]."""
    dims = [4, 4, 4, 2]
    V = volume(dims)
    U = inputs.haar_links(dims, seed=11)
    g = inputs.random_site_unitaries(V, seed=12)
    Ug = np.einsum("sab,msbc->msac", g, U)
    Ug = np.einsum("msac,mscd->msad", Ug, _fwd_dag(g, dims))
    mf = inputs.mass_field(dims, seed=13)
    w = inputs.couplings(dims, seed=14)
    A = Operator(dims, 1, mass_field=mf, coupling=w, links=U)
    Ag = Operator(dims, 1, mass_field=mf, coupling=w, links=Ug)
    rng = np.random.default_rng(3)
    y = rng.standard_normal((V, 3)) + 1j * rng.standard_normal((V, 3))
    Gy = np.einsum("sab,sb->sa", g, y)
    assert np.allclose(Ag.apply(Gy), np.einsum("sab,sb->sa", g, A.apply(y)), atol=1e-12)


def _fwd_dag(g, dims):
    """g(x+mu)^H for every mu, as [d, V, 3, 3]."""
    nd = len(dims)
    grid = g.reshape(tuple(reversed(dims)) + (3, 3))
    return np.stack([np.roll(grid, -1, axis=nd - 1 - mu).reshape(g.shape).conj().swapaxes(-1, -2)
                     for mu in range(nd)])


def test_pure_gauge_is_free_laplacian_in_disguise():
    dims = [4, 4, 2, 4]
    V = volume(dims)
    g = inputs.random_site_unitaries(V, seed=21)
    U = exact.pure_gauge_links(g, dims)
    op = Operator(dims, 1, mass=0.2, links=U)
    lam = np.linalg.eigvalsh(op.dense())
    free = np.sort(np.repeat(exact.free_eigenvalues(dims, 0.2).reshape(-1), 3))
    assert np.allclose(lam, free, atol=1e-12)


def test_haar_links_are_unitary():
    U = inputs.haar_links([4, 4], seed=1)
    I = np.einsum("msba,msbc->msac", U.conj(), U)
    assert np.allclose(I, np.eye(3), atol=1e-14)
