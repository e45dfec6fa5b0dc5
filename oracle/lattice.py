"""Lattice geometry for the oracle (test infrastructure only).

A d-dimensional torus with sides n_1..n_d, each n_j = 2^{k_j} (Sec. 3 and
Sec. 3.3).  Sites are numbered lexicographically with the first coordinate
fastest:  s(x) = x_1 + n_1 (x_2 + n_2 (x_3 + n_3 x_4)).  The paper does not fix
a memory order; this numbering is a convention shared with the GPU path only
through its statement here and in the C header.
"""

import numpy as np


def volume(dims):
    v = 1
    for n in dims:
        v *= int(n)
    return v


def log2_exact(n):
    """k with n == 2^k, or ValueError (Sec. 3 assumes power-of-two sides)."""
    n = int(n)
    if n < 1 or (n & (n - 1)) != 0:
        raise ValueError(f"side {n} is not a power of two")
    return n.bit_length() - 1


def coordinates(dims):
    """Array [V, d] of the coordinates (x_1..x_d) of every site, in site order."""
    dims = [int(n) for n in dims]
    V = volume(dims)
    s = np.arange(V, dtype=np.int64)
    out = np.empty((V, len(dims)), dtype=np.int64)
    for j, n in enumerate(dims):
        out[:, j] = s % n
        s = s // n
    return out


def site_index(coords, dims):
    """Inverse of ``coordinates``: s(x) = x_1 + n_1 (x_2 + n_2 (...))."""
    coords = np.asarray(coords, dtype=np.int64)
    s = np.zeros(coords.shape[:-1], dtype=np.int64)
    for j in reversed(range(len(dims))):
        s = s * int(dims[j]) + coords[..., j]
    return s


def active_dims(dims):
    """Per bit-level m = 1..max k_j, the dimensions j (0-based, increasing)
    with m <= k_j, i.e. those that can still be subdivided at that level
    (Sec. 3.3, Alg. 5)."""
    k = [log2_exact(n) for n in dims]
    kmax = max(k) if k else 0
    return [[j for j in range(len(dims)) if m <= k[j]] for m in range(1, kmax + 1)]


def total_levels(dims):
    """L = sum_j k_j = log2 V, the number of bits of a permuted location."""
    return sum(log2_exact(n) for n in dims)


def torus_distance(a, b, dims):
    """Graph (L1) distance on the torus between coordinate arrays a and b."""
    a = np.asarray(a)
    b = np.asarray(b)
    d = 0
    for j, n in enumerate(dims):
        diff = np.abs(a[..., j] - b[..., j])
        d = d + np.minimum(diff, n - diff)
    return d
