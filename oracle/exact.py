"""Exact values that pin the oracle (test infrastructure only).

* Closed-form traces for constant-coefficient tori (Sec. 5: the trace of the
  inverse of the shifted lattice Laplacian is known analytically): the
  Fourier modes exp(2 pi i k.x / n) diagonalise the periodic Laplacian with
  eigenvalues lambda(k) = m + sum_mu 4 sin^2(pi k_mu / n_mu), so
  Tr(A^-1) = ncomp * sum_k 1 / lambda(k).
* FFT solves for the same operators; pure-gauge links U_mu(x) = g(x) g(x+mu)^H
  give A = G (A_free (x) I_3) G^H with G = diag(g(x)), so their solves are
  exact too, at any size.
* Dense LU (numpy.linalg) on tiny lattices (Sec. 1: small problems can be
  done by LU).
* The partial-sum identity of the probing estimator: for s = 2^t the first s
  columns of the reordered Hadamard matrix satisfy
  sum_{m<s} z_m(x) z_m(y) = s when the leading t bits of P(x) and P(y) agree
  and 0 otherwise (eq. HadamardElements with eq. HpermSequence), so
  T_s = sum_c sum_{x ~ y} conj(z0(x,c)) A^-1[(x,c),(y,c)] z0(y,c)
  over pairs in the same colour class -- a formula that uses the colouring
  and A^-1 but no probing vector and no solve.
"""

import numpy as np

from .lattice import volume


def free_eigenvalues(dims, mass):
    """lambda(k) for every Fourier mode, as an array shaped [n_d, ..., n_1]."""
    lam = np.full(tuple(reversed([int(n) for n in dims])), float(mass))
    nd = len(dims)
    for mu, n in enumerate(dims):
        k = np.arange(int(n))
        shape = [1] * nd
        shape[nd - 1 - mu] = int(n)
        lam = lam + (4.0 * np.sin(np.pi * k / n) ** 2).reshape(shape)
    return lam


def free_trace_inverse(dims, mass, ncomp=1):
    return ncomp * float(np.sum(1.0 / free_eigenvalues(dims, mass)))


def free_trace_power(dims, mass, p, ncomp=1):
    """Tr(A^p) of the constant-coefficient operator."""
    return ncomp * float(np.sum(free_eigenvalues(dims, mass) ** p))


def fft_solve(dims, mass, b):
    """x = A_free^-1 b for b [V, ncomp] (each component separately)."""
    V = volume(dims)
    lam = free_eigenvalues(dims, mass)
    b = np.asarray(b).reshape(V, -1)
    out = np.empty(b.shape, dtype=np.complex128)
    for c in range(b.shape[1]):
        g = b[:, c].reshape(lam.shape)
        out[:, c] = np.fft.ifftn(np.fft.fftn(g) / lam).reshape(V)
    return out


def pure_gauge_links(g, dims):
    """U_mu(x) = g(x) g(x+mu)^H for site matrices g [V, 3, 3]."""
    nd = len(dims)
    grid = g.reshape(tuple(reversed([int(n) for n in dims])) + (3, 3))
    links = np.empty((nd, g.shape[0], 3, 3), dtype=np.complex128)
    for mu in range(nd):
        g_fwd = np.roll(grid, -1, axis=nd - 1 - mu).reshape(g.shape)
        links[mu] = np.einsum("sab,scb->sac", g, g_fwd.conj())
    return links


def pure_gauge_solve(dims, mass, g, b):
    """x = A^-1 b for pure-gauge links: x = G A_free^-1 G^H b."""
    y = np.einsum("sba,sb->sa", g.conj(), b)          # G^H b
    y = fft_solve(dims, mass, y)
    return np.einsum("sab,sb->sa", g, y)


def dense_trace_inverse(A):
    return complex(np.trace(np.linalg.inv(A)))


def partial_sum_estimate(Ainv, P, L, t, ncomp, z0):
    """T_{2^t} from the partial-sum identity; z0 is complex [ncomp, V]."""
    V = len(P)
    cls = (np.asarray(P, dtype=np.uint64) >> np.uint64(L - t)).astype(np.int64)
    same = cls[:, None] == cls[None, :]
    total = 0.0 + 0.0j
    for c in range(ncomp):
        idx = np.arange(V) * ncomp + c
        block = Ainv[np.ix_(idx, idx)]
        w = np.conj(z0[c])[:, None] * block * z0[c][None, :]
        total += np.sum(w[same])
    return total
