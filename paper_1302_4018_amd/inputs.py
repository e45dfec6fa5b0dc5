"""Seeded synthetic inputs for the lattice operators.

This module only draws random coefficient arrays (numpy PCG64,
``numpy.random.default_rng(seed)``); it holds none of the method's arithmetic.
The same arrays are handed to the HIP library and, in tests, to the CPU
checker, so neither side needs the other's random-number code.

Workloads (the paper's control problems are shifted periodic Laplacians,
Sec. 5; the 3-component covariant operator stands in for the internal
dimension of the LQCD matrix, Sec. 1.1.1):

* ``haar_links``   U_mu(x) = Q of the QR factorisation of a 3x3 complex
  Gaussian matrix, with the phases of diag(R) moved into Q so that U is Haar
  distributed on U(3) (Mezzadri, Notices AMS 54 (2007) 592).
* ``mass_field``   m(x) = m0 + sigma * clip(xi, -3, 3), xi ~ N(0, 1).
* ``couplings``    w_mu(x) ~ U[lo, hi] independently per forward edge.
* ``uneven_tori``  the batch of 3-D tori with sides drawn from [8, 48].

Array layouts match ``include/tip.h``:  links [ndim][V][3][3] complex128
(row-major 3x3), coupling [ndim][V] float64, mass_field [V] float64, with
sites numbered s = x1 + n1 (x2 + n2 (x3 + n3 x4)).
"""

import numpy as np

OPERATOR_SEED = 1302
MASK_SEED = 4018


def volume(dims):
    v = 1
    for n in dims:
        v *= int(n)
    return v


def haar_links(dims, seed=OPERATOR_SEED, chunk=1 << 20):
    """complex128 [ndim, V, 3, 3] of Haar-random U(3) matrices."""
    nd, V = len(dims), volume(dims)
    rng = np.random.default_rng(seed)
    out = np.empty((nd, V, 3, 3), dtype=np.complex128)
    flat = out.reshape(nd * V, 3, 3)
    for start in range(0, nd * V, chunk):
        n = min(chunk, nd * V - start)
        z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2.0)
        q, r = np.linalg.qr(z)
        d = np.diagonal(r, axis1=1, axis2=2)
        ph = d / np.abs(d)
        flat[start:start + n] = q * ph[:, None, :]
    return out


def mass_field(dims, m0=0.1, sigma=0.02, seed=OPERATOR_SEED + 1):
    rng = np.random.default_rng(seed)
    xi = np.clip(rng.standard_normal(volume(dims)), -3.0, 3.0)
    return m0 + sigma * xi


def couplings(dims, lo=0.5, hi=1.5, seed=OPERATOR_SEED + 2):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(len(dims), volume(dims)))


def random_site_unitaries(V, seed):
    """Haar U(3) per site, e.g. for gauge transformations g(x) in tests."""
    return haar_links([V], seed=seed)[0]


def uneven_tori(count=64, lo=8, hi=48, seed=OPERATOR_SEED + 3):
    """Sides, masses and probe counts of the batch of independent 3-D tori."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(lo, hi + 1, size=(count, 3))
    masses = rng.uniform(0.02, 0.2, size=count)
    nvec = 2 ** rng.integers(4, 9, size=count)            # 16 .. 256
    return [dict(dims=[int(v) for v in s], mass=float(m), n_vectors=int(k))
            for s, m, k in zip(sides, masses, nvec)]


def uneven_torus_couplings(dims, index, lo=0.5, hi=1.5):
    """w_mu(x) ~ U[lo, hi] iid per forward edge of torus `index` of the batch."""
    return couplings(dims, lo, hi, seed=OPERATOR_SEED + 100 + int(index))
