"""Probe variants of Sec. 5 and the variance of the probing estimator over
the random mask (test infrastructure only).

Stopped hierarchy (Sec. 5.1).  The recursive colouring of Sec. 3 is run for
`levels` bit-levels only.  The sites of each colour class then keep their
natural relative order.  On a power-of-two torus the class of x after k levels
is fixed by the low k bits of every coordinate, and its members differ in
y_j = x_j >> min(k, k_j).  So the stopped permutation is the Alg. 5 location
over levels 1..k (t_k = sum_{l <= k} a_l bits), followed by the natural index
of y on the sub-torus with sides n_j >> min(k, k_j):

    P_k(x) = loc_k(x) * 2^{L - t_k} + sum_j y_j prod_{i < j} (n_i >> min(k, k_i)).

The probes are the same Hadamard columns as for the full hierarchy,
z_m(x) = H(P_k(x), bitrev_L(m)) (eq. HpermSequence, eq. HadamardElements),
times the mask.  k = 0 is the natural site order; k >= max k_j is Alg. 5.

Fourier-grouped columns.  eq. Hperm-general-recursive builds the probes level
by level with the Fourier matrix of each level's colour count, with the newest
level's column index most significant.  Taking the a_l bits of one Alg. 5
level as one level with c_l = 2^{a_l} colours gives

    z_m(x) = prod_l F_{c_l}(s_l(x), j_l) = prod_l w_{c_l}^{s_l(x) j_l},   m = sum_l j_l prod_{l' < l} c_{l'},

with s_l(x) the Red-Black index of level l (Lemma 3.3) and F_n(i, j) =
exp(2 pi i i j / n) (eq. FourierElements).  With c_l <= 16 every entry is a
16th root of unity w16^e, e = sum_l (s_l j_l mod c_l) (16 / c_l) mod 16.  The
table below holds the doubles nearest to cos and sin of 2 pi e / 16, so that
the entries are fixed constants, not the output of a library exp.  At every
level boundary s = 2^{t_k} the columns span the functions of (s_1..s_k), as
the Hadamard columns do, so the two estimates agree there exactly.

Variance over the mask (Sec. 1, Lemma 1.1; Sec. 5.2).  With one mask zeta
shared by all probes (eq. removebias) and internal dilution,
T_s = sum_c sum_{x,y} conj(zeta_x) zeta_y G_c(x, y) M(x, y) / s, with
G_c = A^-1 restricted to component c and M(x, y) = sum_{m<s} conj z_m(x) z_m(y).
The mean is Tr(A^-1) because |z_m(x)| = 1.  Distinct pairs (x, y) are
uncorrelated, so with W = G M / s:
    Z2 masks:  Var T_s = 2 sum_c sum_{x != y} (Re W_c(x, y))^2,
    Z4 masks:  Var T_s =   sum_c sum_{x != y} |W_c(x, y)|^2
(the second because E zeta^2 = 0 for Z4).  For independent masks per probe
(plain Monte Carlo, Sec. 1) the quadratures are independent and
Var T_s = Var q / s, with Var q the same sums at M = 1.
"""

import numpy as np

from .general import _parity
from .hadamard import hperm
from .hierperm import rb_table_fast
from .lattice import coordinates, log2_exact, volume
from .mask import MASK_NONE, MASK_Z2, MASK_Z4

COS_PI_8 = 0.9238795325112867        # nearest double to cos(pi/8)
SIN_PI_8 = 0.3826834323650898        # nearest double to sin(pi/8)
SQRT1_2 = 0.7071067811865476         # nearest double to sqrt(2)/2

# w16^e = exp(2 pi i e / 16), e = 0..15, as (re, im) built from the three constants
_C = [(1.0, 0.0), (COS_PI_8, SIN_PI_8), (SQRT1_2, SQRT1_2), (SIN_PI_8, COS_PI_8)]
OMEGA16 = np.array([complex(r, i) for r, i in _C]
                   + [complex(-i, r) for r, i in _C]
                   + [complex(-r, -i) for r, i in _C]
                   + [complex(i, -r) for r, i in _C])


def level_indices(dims):
    """Per Alg. 5 level l = 1..max k_j: (s_l [V] int64, a_l), the Red-Black
    index of the level's bits and the number of active dimensions."""
    dims = [int(n) for n in dims]
    d = len(dims)
    k = [log2_exact(n) for n in dims]
    rb = np.array(rb_table_fast(d), dtype=np.int64)
    X = coordinates(dims)
    out = []
    for m in range(1, (max(k) if k else 0) + 1):
        bits = np.zeros(len(X), dtype=np.int64)
        a = 0
        for j in range(d):
            if m <= k[j]:
                bits = (bits << 1) | ((X[:, j] >> (m - 1)) & 1)
                a += 1
        out.append((rb[bits * 2 ** (d - a)] // 2 ** (d - a), a))
    return out


def stopped_perm(dims, levels):
    """P_k(x) for every site, uint64 [V] (k = levels)."""
    dims = [int(n) for n in dims]
    k = [log2_exact(n) for n in dims]
    L = sum(k)
    lv = level_indices(dims)[:max(0, int(levels))]
    loc = np.zeros(volume(dims), dtype=np.int64)
    t = 0
    for s, a in lv:
        loc = (loc << a) | s
        t += a
    X = coordinates(dims)
    kk = len(lv)
    nat = np.zeros(len(X), dtype=np.int64)
    stride = 1
    for j, n in enumerate(dims):
        cut = min(kk, k[j])
        nat += (X[:, j] >> cut) * stride
        stride *= n >> cut
    return ((loc << (L - t)) | nat).astype(np.uint64)


def stopped_probe(dims, m, levels, P=None):
    """z_m(x) = H(P_k(x), bitrev_L(m)) as float64 +-1 [V]."""
    L = sum(log2_exact(n) for n in dims)
    P = stopped_perm(dims, levels) if P is None else P
    col = np.uint64(hperm(int(m), L)) if L > 0 else np.uint64(0)
    return (1 - 2 * _parity(P & col)).astype(np.float64)


def fourier_exponents(dims, m, lv=None):
    """e(x) in [0, 16) with z_m(x) = w16^e(x) for the Fourier-grouped columns."""
    lv = level_indices(dims) if lv is None else lv
    e = np.zeros(volume(dims), dtype=np.int64)
    rest = int(m)
    for s, a in lv:
        c = 1 << a
        j = rest % c
        rest //= c
        e += ((s * j) % c) * (16 // c)
    if rest:
        raise ValueError(f"column {m} exceeds the {volume(dims)} Fourier-grouped columns")
    return e % 16


def fourier_probe(dims, m, lv=None):
    """z_m(x) for the Fourier-grouped columns, complex128 [V]."""
    return OMEGA16[fourier_exponents(dims, m, lv)]


def probe_matrix(dims, s, kind, levels=0):
    """Unmasked probes z_0..z_{s-1} as columns of a complex [V, s] array, for the
    hierarchical (levels >= max k_j), stopped or Fourier-grouped sequences."""
    if kind == "fourier":
        lv = level_indices(dims)
        return np.stack([fourier_probe(dims, m, lv) for m in range(s)], axis=1)
    P = stopped_perm(dims, levels)
    return np.stack([stopped_probe(dims, m, levels, P) for m in range(s)], axis=1).astype(np.complex128)


def variance_shared_mask(Ainv, Z, ncomp, mask_kind):
    """Var T_s over the mask for probes Z [V, s] that share one mask."""
    V, s = Z.shape
    if mask_kind == MASK_NONE:
        return 0.0
    M = np.conj(Z) @ Z.T                        # M(x, y) = sum_m conj z_m(x) z_m(y)
    off = ~np.eye(V, dtype=bool)
    total = 0.0
    for c in range(ncomp):
        idx = np.arange(V) * ncomp + c
        W = Ainv[np.ix_(idx, idx)] * M / s
        if mask_kind == MASK_Z2:
            total += 2.0 * float(np.sum(W.real[off] ** 2))
        elif mask_kind == MASK_Z4:
            total += float(np.sum(np.abs(W[off]) ** 2))
        else:
            raise ValueError(f"unknown mask kind {mask_kind}")
    return total


def variance_monte_carlo(Ainv, V, ncomp, s, mask_kind):
    """Var T_s for s independent masked probes (z_m = the mask of sweep m)."""
    Z1 = np.ones((V, 1), dtype=np.complex128)
    return variance_shared_mask(Ainv, Z1, ncomp, mask_kind) / s
