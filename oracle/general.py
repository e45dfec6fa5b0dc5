"""Hierarchical probing on tori whose sides are not all powers of two
(test infrastructure only).

Sec. 3.4 of the paper: with n_j = 2^{k_j} p_j (p_j odd), the hierarchical
red-black colouring runs while the factors of two last, then a torus with an
odd side is three-coloured by the theorem of Sec. 3.4, and no further level
follows.  The probe columns of mixed-radix levels come from the general
recursion eq. Hperm-general-recursive (Fourier columns for a level with three
colours).  Readings taken here (the paper gives the ingredients, not this
exact schedule):

* Binary levels m = 1..B colour red-black the conformal sub-torus exactly as
  Alg. 5 does (dimension j is active at level m when k_j >= m).  They continue
  while every side whose remaining size n_j / 2^{m-1} exceeds 1 is even:
  B = min{k_j : p_j > 1}, or max k_j when every p_j = 1 (the power-of-two case,
  where this is Alg. 5 unchanged).  Their colour P_B(x) has L_B bits.
* If some p_j > 1, one more level colours each block with C(y) of the theorem
  of Sec. 3.4, applied to the sub-torus coordinates y_j = x_j >> B (sides
  n_j / 2^B) of the dimensions whose remaining side exceeds 1.
* eq. Hperm-general-recursive puts the newest level's Fourier column index
  above the earlier ones: with gamma = 2^{L_B} c colours (c = 3 with the extra
  level, else 1), column j < gamma has binary part j mod 2^{L_B}, read through
  eq. HpermSequence (bit reversal), and F_3 part j3 = j >> L_B, contributing
  w^{j3 C(x)}, w = exp(2 pi i / 3).  F_3 is taken as the conjugate-free
  exp(+2 pi i j k / 3), as eq. FourierElements writes F_n.
* The colouring is exhausted after gamma columns.  The end of Sec. 3 suggests
  replacing the remaining constant factor by a random vector; probe
  m = r gamma + j is read as column j under the r-th mask, which takes the
  next V ncomp outputs of the same SplitMix64 stream (sweep r = 0 is the
  ordinary mask).

The complex unit w uses the double nearest to sqrt(3)/2 so that its value is
a fixed constant, not the result of a library exp.
"""

import numpy as np

from .hadamard import hperm
from .hierperm import rb_table_fast
from .lattice import coordinates, volume
from .mask import MASK_NONE, MASK_Z2, MASK_Z4, splitmix64_at

SQRT3_2 = 0.8660254037844386          # nearest double to sqrt(3)/2
OMEGA3 = np.array([1.0 + 0.0j, complex(-0.5, SQRT3_2), complex(-0.5, -SQRT3_2)])


def two_adic(n):
    """(k, p) with n = 2^k p and p odd."""
    n = int(n)
    if n < 1:
        raise ValueError(f"side {n} must be >= 1")
    k = 0
    while n % 2 == 0:
        n //= 2
        k += 1
    return k, n


class Levels:
    """The level schedule of a torus: binary levels, then an optional
    three-colouring level."""

    def __init__(self, dims):
        self.dims = [int(n) for n in dims]
        kp = [two_adic(n) for n in self.dims]
        self.k = [k for k, _ in kp]
        self.p = [p for _, p in kp]
        odd = [self.k[j] for j in range(len(dims)) if self.p[j] > 1]
        self.B = min(odd) if odd else (max(self.k) if self.k else 0)
        self.active = [[j for j in range(len(dims)) if self.k[j] >= m] for m in range(1, self.B + 1)]
        self.LB = sum(len(a) for a in self.active)
        self.has3 = bool(odd)
        self.sub = [n >> self.B for n in self.dims]
        self.gamma = (1 << self.LB) * (3 if self.has3 else 1)


def binary_colour(dims, lv=None):
    """P_B(x) for every site: the location over the binary levels (Alg. 5 run
    for levels 1..B), uint64 [V] in [0, 2^{L_B})."""
    lv = lv or Levels(dims)
    d = len(lv.dims)
    rb = np.array(rb_table_fast(d), dtype=np.int64)
    X = coordinates(lv.dims)
    V = volume(lv.dims)
    loc = np.zeros(V, dtype=np.int64)
    for m in range(1, lv.B + 1):
        bits = np.zeros(V, dtype=np.int64)
        active = 0
        for j in range(d):
            if m <= lv.k[j]:
                bits = (bits << 1) | ((X[:, j] >> (m - 1)) & 1)
                active += 1
        s = rb[bits * 2 ** (d - active)] // 2 ** (d - active)
        loc = (loc << active) | s
    return loc.astype(np.uint64)


def three_colouring(Y, sides):
    """C(y) of the theorem of Sec. 3.4 for coordinates Y [V, d] on a torus with
    the given sides: (sum_j y_j + sum_j delta_j(y_j)) mod 3, delta_j = 1 iff
    y_j = n_j - 1 and (n_j - 1) mod 3 = 0.  Sides equal to 1 take no part."""
    Y = np.asarray(Y, dtype=np.int64)
    total = np.zeros(Y.shape[0], dtype=np.int64)
    for j, n in enumerate(sides):
        if n <= 1:
            continue
        total += Y[:, j]
        if (n - 1) % 3 == 0:
            total += (Y[:, j] == n - 1).astype(np.int64)
    return total % 3


def last_level_colour(dims, lv=None):
    """C(x >> B) for every site (zeros without a three-colouring level)."""
    lv = lv or Levels(dims)
    if not lv.has3:
        return np.zeros(volume(lv.dims), dtype=np.int64)
    X = coordinates(lv.dims)
    return three_colouring(X >> lv.B, lv.sub)


def _parity(v):
    """Parity of the one-bits of each uint64 (eq. HadamardElements' sign)."""
    v = np.asarray(v, dtype=np.uint64).copy()
    for sh in (32, 16, 8, 4, 2, 1):
        v ^= v >> np.uint64(sh)
    return (v & np.uint64(1)).astype(np.int64)


def probe(dims, m, lv=None, PB=None, C=None):
    """z_m(x) without the mask: complex128 [V], and the sweep index r."""
    lv = lv or Levels(dims)
    PB = binary_colour(dims, lv) if PB is None else PB
    C = last_level_colour(dims, lv) if C is None else C
    r, j = divmod(int(m), lv.gamma)
    jb, j3 = j % (1 << lv.LB), j >> lv.LB
    col = np.uint64(hperm(jb, lv.LB)) if lv.LB > 0 else np.uint64(0)
    z = (1 - 2 * _parity(PB & col)).astype(np.complex128)
    if j3:
        z = z * OMEGA3[(C * j3) % 3]
    return z, r


def mask_sweep(seed, V, ncomp, c, kind, r):
    """Sweep r's mask z0_r(x, c): outputs n = (r V + s) ncomp + c of SplitMix64(seed)."""
    if kind == MASK_NONE:
        return np.ones(V, dtype=np.complex128)
    n = (np.uint64(r) * np.uint64(V) + np.arange(V, dtype=np.uint64)) * np.uint64(ncomp) + np.uint64(c)
    z = splitmix64_at(seed, n)
    if kind == MASK_Z2:
        return (1 - 2 * (z >> np.uint64(63)).astype(np.int64)).astype(np.complex128)
    if kind == MASK_Z4:
        return np.array([1, 1j, -1, -1j], dtype=np.complex128)[(z >> np.uint64(62)).astype(np.int64)]
    raise ValueError(f"unknown mask kind {kind}")


def rhs(dims, ncomp, m, c, seed, mask_kind, lv=None, PB=None, C=None):
    """Right-hand side b_{m,c} as complex128 [V, ncomp] (zero outside comp c)."""
    lv = lv or Levels(dims)
    V = volume(dims)
    z, r = probe(dims, m, lv, PB, C)
    b = np.zeros((V, ncomp), dtype=np.complex128)
    b[:, c] = mask_sweep(seed, V, ncomp, c, mask_kind, r) * z
    return b


def trace_inv_probe(op, n_vectors, tol, seed, mask_kind, max_iter=None, probe=0, levels=0):
    """Estimates (1/s) sum_{m<s} q_m at the checkpoints, with these probes (or the
    comparison probe kind given); q_m = sum_c b_{m,c}^H x_{m,c} by the oracle's
    CG.  Returns (est, q, stats)."""
    from .cg import cg_solve
    from .estimator import estimates_from_quadratures
    if max_iter is None:
        max_iter = 10 * op.V * op.ncomp
    lv = Levels(op.dims)
    PB = binary_colour(op.dims, lv)
    C = last_level_colour(op.dims, lv)
    q, iters = [], []
    for m in range(n_vectors):
        qm = 0.0 + 0.0j
        for c in range(op.ncomp):
            b = rhs_kind(op.dims, op.ncomp, m, c, seed, mask_kind, probe, lv, PB, C, levels)
            if op.kind == 0 and np.all(b.imag == 0):
                b = b.real
            x, it, _ = cg_solve(op.apply, b, tol, max_iter)
            qm += complex(np.vdot(b, x))
            iters.append(it)
        q.append(qm)
    return estimates_from_quadratures(q), np.array(q), {"iters": iters}


# ---------------------------------------------------------------------------
# The comparison probes of Sec. 5 (test infrastructure only).  Sec. 5 sets
# hierarchical probing against random Z2 vectors (plain Monte Carlo) and
# against Hadamard vectors taken in natural order; both run through the same
# estimator and solver here.
#   PROBE_HIERARCHICAL: the probes above.
#   PROBE_NATURAL: z_m(x) = H(s(x), m), the Hadamard columns in natural order
#     on the natural site numbering (power-of-two sides), times the mask.
#   PROBE_RANDOM: z_m = the mask of sweep m alone, i.e. independent Z2 / Z4
#     noise vectors (Hutchinson's estimator of Sec. 1).
# ---------------------------------------------------------------------------

PROBE_HIERARCHICAL, PROBE_NATURAL, PROBE_RANDOM = 0, 1, 2
# the variants of oracle/variants.py: the hierarchy stopped after `levels`
# bit-levels (Sec. 5.1) and the Fourier-grouped columns; power-of-two sides,
# one mask for all probes
PROBE_STOPPED, PROBE_FOURIER = 3, 4


def rhs_kind(dims, ncomp, m, c, seed, mask_kind, probe, lv=None, PB=None, C=None, levels=0):
    """b_{m,c} for the given probe kind: complex128 [V, ncomp]."""
    V = volume(dims)
    if probe == PROBE_HIERARCHICAL:
        return rhs(dims, ncomp, m, c, seed, mask_kind, lv, PB, C)
    b = np.zeros((V, ncomp), dtype=np.complex128)
    if probe in (PROBE_STOPPED, PROBE_FOURIER):
        from . import variants
        if not 0 <= int(m) < V:
            raise ValueError(f"probe {m} outside [0, V)")
        z = variants.stopped_probe(dims, m, levels) if probe == PROBE_STOPPED else variants.fourier_probe(dims, m)
        b[:, c] = mask_sweep(seed, V, ncomp, c, mask_kind, 0) * z
    elif probe == PROBE_NATURAL:
        if V & (V - 1):
            raise ValueError("natural-order Hadamard probes need a power-of-two volume")
        z = (1 - 2 * _parity(np.arange(V, dtype=np.uint64) & np.uint64(m))).astype(np.complex128)
        b[:, c] = mask_sweep(seed, V, ncomp, c, mask_kind, 0) * z
    elif probe == PROBE_RANDOM:
        if mask_kind == MASK_NONE:
            raise ValueError("random probes need a Z2 or Z4 mask")
        b[:, c] = mask_sweep(seed, V, ncomp, c, mask_kind, m)
    else:
        raise ValueError(f"unknown probe kind {probe}")
    return b


def estimates_dense(Ainv, dims, ncomp, n, seed, mask_kind, probe, levels=0):
    """T_s at the checkpoints from exact quadratures b^H A^-1 b (dense A^-1, tiny lattices)."""
    from .estimator import estimates_from_quadratures
    lv = Levels(dims)
    PB, C = binary_colour(dims, lv), last_level_colour(dims, lv)
    q = np.zeros(n, dtype=np.complex128)
    for c in range(ncomp):
        Z = np.stack([rhs_kind(dims, ncomp, m, c, seed, mask_kind, probe, lv, PB, C, levels).reshape(-1)
                      for m in range(n)], axis=1)
        q += np.sum(np.conj(Z) * (Ainv @ Z), axis=0)       # b_m^H A^-1 b_m for every m at once
    return estimates_from_quadratures(q)
