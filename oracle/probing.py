"""Hierarchical probing vectors, masked and colour-diluted (test infrastructure only).

* eq. row-col-permutation: z_m(i) = H_N(iperm(i), Hperm(m)), where iperm is
  the 0-based location P(x) of site x in the hierarchical permutation (Sec. 3)
  and Hperm is the column order of eq. HpermSequence; H entries by
  eq. HadamardElements.  m is 0-based, so vector 0 is column 0 = all ones.
* eq. removebias: every vector is multiplied elementwise by the same random
  vector z0 (``mask``).
* Dilution of the internal ("colour") components (Sec. 1.1.3, and the full
  internal dilution used in Sec. 5.3): spatial probe m is split into ncomp
  right-hand sides b_{m,c}(y, c') = delta_{c c'} z0(y, c) z_m(y).
"""

import numpy as np

from .hadamard import hadamard_element, hperm
from .hierperm import hier_perm
from .lattice import total_levels, volume
from .mask import mask_values


def probe_sign(P, m, L):
    """z_m(x) = H(P(x), Hperm(m)) for all sites: int64 [V] of +-1."""
    return hadamard_element(P, np.uint64(hperm(m, L)))


def rhs(dims, ncomp, m, c, seed, mask_kind, P=None):
    """Right-hand side b_{m,c} as complex128 [V, ncomp] (zero outside comp c)."""
    V = volume(dims)
    if P is None:
        P = hier_perm(dims)
    z = probe_sign(P, m, total_levels(dims)).astype(np.complex128)
    b = np.zeros((V, ncomp), dtype=np.complex128)
    b[:, c] = mask_values(seed, V, ncomp, c, mask_kind) * z
    return b
