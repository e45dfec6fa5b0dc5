"""The probing estimator of Tr(A^-1) reported at s = 2^k (test infrastructure only).

* Hutchinson's estimator (Sec. 1, Lemma 1.1): (1/s) sum_{m<s} z_m^H A^-1 z_m.
* eq. Hperm-recursive and the remark after it: Z(k-1) is the first 2^{k-1}
  columns of Z(k), so the quadratures of earlier levels are reused and the
  estimate is reported after every power of two s = 2^k (Sec. 1.1.4: only
  those s annihilate a whole sparsity structure).  When n_vectors is not a
  power of two a last estimate at s = n_vectors is added.
* With internal dilution each spatial probe m contributes
  q_m = sum_c b_{m,c}^H x_{m,c}, and s counts spatial probes.

Quadratures are summed in m order with Neumaier's compensated summation
(Neumaier 1974), real and imaginary parts separately.
"""

import numpy as np

from .cg import cg_solve
from .hierperm import hier_perm
from .probing import rhs


def neumaier_prefix_sums(values):
    """Compensated running sums S_1..S_n of a real sequence."""
    out = []
    s = 0.0
    comp = 0.0
    for v in values:
        v = float(v)
        t = s + v
        if abs(s) >= abs(v):
            comp += (s - t) + v
        else:
            comp += (v - t) + s
        s = t
        out.append(s + comp)
    return out


def checkpoint_sizes(n_vectors):
    """s = 1, 2, 4, ..., 2^floor(log2 n), and n itself if it is not a power of two."""
    sizes = []
    s = 1
    while s <= n_vectors:
        sizes.append(s)
        s *= 2
    if sizes and sizes[-1] != n_vectors:
        sizes.append(n_vectors)
    return sizes


def estimates_from_quadratures(q):
    """T_s = S_s / s at every checkpoint size; q is complex [n]."""
    q = np.asarray(q, dtype=np.complex128)
    re = neumaier_prefix_sums(q.real)
    im = neumaier_prefix_sums(q.imag)
    return np.array([complex(re[s - 1], im[s - 1]) / s for s in checkpoint_sizes(len(q))])


def quadrature(op, m, c, tol, seed, mask_kind, max_iter, P=None):
    """b_{m,c}^H A^-1 b_{m,c} by one CG solve; returns (q, iterations, relres)."""
    b = rhs(op.dims, op.ncomp, m, c, seed, mask_kind, P)
    real = op.kind == 0 and np.all(b.imag == 0)
    if real:
        b = b.real
    x, it, relres = cg_solve(op.apply, b, tol, max_iter)
    return complex(np.vdot(b, x)), it, relres


def trace_inv_probe(op, n_vectors, tol, seed, mask_kind, max_iter=None, m_begin=0):
    """Returns (estimates [n_ckpt] complex, q [n_vectors - m_begin] complex, stats dict)."""
    if max_iter is None:
        max_iter = 10 * op.V * op.ncomp
    P = hier_perm(op.dims)
    q = []
    iters = []
    relres = []
    for m in range(m_begin, n_vectors):
        qm = 0.0 + 0.0j
        for c in range(op.ncomp):
            v, it, rr = quadrature(op, m, c, tol, seed, mask_kind, max_iter, P)
            qm += v
            iters.append(it)
            relres.append(rr)
        q.append(qm)
    est = estimates_from_quadratures(q) if m_begin == 0 else None
    return est, np.array(q), {"iters": iters, "relres": relres}
