"""The random vector z0 that removes the deterministic bias (test infrastructure only).

Sec. 4 (eq. removebias) multiplies every probing vector elementwise by one
random vector z0.  The paper does not say how z0 is drawn.  Reading used by
this project: z0 entry number n = s(x) * ncomp + c (site s, internal component
c) takes the n-th output (0-based) of SplitMix64 seeded with ``seed``
(Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014; the public-domain C reference by S. Vigna).  Its state is the Weyl
sequence seed + (n+1) * GOLDEN_GAMMA and each output is a fixed 64-bit mixing
of the state, so any entry can be computed on its own.

* Z2 mask (real operators): +1 if the top output bit is 0, else -1.
* Z4 mask (complex operators): i^t with t = the top two output bits.
* none: every entry is 1 (the deterministic sequence of Sec. 5.1).
"""

import numpy as np

MASK_NONE, MASK_Z2, MASK_Z4 = 0, 1, 2

GOLDEN_GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def _mix(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


class SplitMix64:
    """The sequential generator exactly as published: advance, then mix."""

    def __init__(self, seed):
        self.state = int(seed) & _M64

    def next(self):
        self.state = (self.state + GOLDEN_GAMMA) & _M64
        return _mix(self.state)


def splitmix64_at(seed, n):
    """n-th output (0-based) of SplitMix64(seed), for an integer array n.

    The state after n+1 steps is seed + (n+1) * GOLDEN_GAMMA mod 2^64;
    numpy uint64 arithmetic wraps modulo 2^64.
    """
    n = np.asarray(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(int(seed) & _M64) + (n + np.uint64(1)) * np.uint64(GOLDEN_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def mask_values(seed, V, ncomp, c, kind):
    """z0(x, c) for all sites x (site order), component c: complex128 [V]."""
    if kind == MASK_NONE:
        return np.ones(V, dtype=np.complex128)
    n = np.arange(V, dtype=np.uint64) * np.uint64(ncomp) + np.uint64(c)
    z = splitmix64_at(seed, n)
    if kind == MASK_Z2:
        top = (z >> np.uint64(63)).astype(np.int64)
        return (1 - 2 * top).astype(np.complex128)
    if kind == MASK_Z4:
        t = (z >> np.uint64(62)).astype(np.int64)
        return np.array([1, 1j, -1, -1j], dtype=np.complex128)[t]
    raise ValueError(f"unknown mask kind {kind}")
