"""Gradient of the probing estimate with respect to the operator's parameters
(test infrastructure only).

The estimate T_s = (1/s) sum_{m<s} sum_c b_{m,c}^H A^-1 b_{m,c} (Sec. 1,
Hutchinson's estimator with the hierarchical probes and internal dilution)
depends on the mass field m(y) and the edge weights w_mu(y) of
A = sum_e w_e L_e + diag(m) (x) I only through A^-1.  Holding the probes
fixed and using d(A^-1) = -A^-1 (dA) A^-1:

    dT/dtheta = -(1/s) sum_{m,c} x_{m,c}^H (dA/dtheta) x_{m,c},  x_{m,c} = A^-1 b_{m,c},

where A^-H b = A^-1 b because A is Hermitian.  dA/dm(y) is the identity on the
components of site y, so its quadratic form is ||x(y)||^2; dA/dw_mu(y) is the
edge matrix L_e of e = (y, y+mu), whose quadratic form is
||x(y) - U_mu(y) x(y+mu)||^2 (U = 1 for the scalar operator).

The solves are the oracle's CG solves (textbook CG with a true-residual
acceptance test) of the probes of oracle/general.py, which are Alg. 5's on
power-of-two sides; nothing here is blocked or fused.
"""

import numpy as np

from .cg import cg_solve
from .general import Levels, binary_colour, last_level_colour, rhs


def edge_forms(op, x):
    """||x(y) - U_mu(y) x(y+mu)||^2 for every edge: [ndim, V] float64."""
    xv = np.asarray(x).reshape(op.V, op.ncomp)
    out = np.empty((op.ndim, op.V))
    for mu in range(op.ndim):
        x_fwd = op._shift(xv, mu, +1)                          # x(y+mu)
        if op.kind == 0:
            hop = x_fwd
        else:
            hop = np.einsum("sab,sb->sa", op.links[mu], x_fwd)  # U_mu(y) x(y+mu)
        d = xv - hop
        out[mu] = np.sum(np.abs(d) ** 2, axis=1)
    return out


def site_forms(op, x):
    """||x(y)||^2 per site: [V] float64."""
    xv = np.asarray(x).reshape(op.V, op.ncomp)
    return np.sum(np.abs(xv) ** 2, axis=1)


def trace_inv_probe_grad(op, n_vectors, tol, seed, mask_kind, max_iter=None):
    """T_s at s = n_vectors with dT/dm [V] and dT/dw [ndim, V].

    Returns (T complex, grad_mass, grad_coupling, stats).  Each solve's
    contribution is added in probe order m, then component c.
    """
    if max_iter is None:
        max_iter = 10 * op.V * op.ncomp
    lv = Levels(op.dims)
    PB, C = binary_colour(op.dims, lv), last_level_colour(op.dims, lv)
    gm = np.zeros(op.V)
    gw = np.zeros((op.ndim, op.V))
    total = 0.0 + 0.0j
    iters = []
    for m in range(n_vectors):
        for c in range(op.ncomp):
            b = rhs(op.dims, op.ncomp, m, c, seed, mask_kind, lv, PB, C)
            if op.kind == 0 and np.all(b.imag == 0):
                b = b.real
            x, it, _ = cg_solve(op.apply, b, tol, max_iter)
            iters.append(it)
            total += complex(np.vdot(b, x))
            gm += site_forms(op, x)
            gw += edge_forms(op, x)
    s = float(n_vectors)
    return total / s, -gm / s, -gw / s, {"iters": iters}


def dense_edge_matrix(op, mu, y):
    """dA/dw_mu(y): the matrix L_e of edge e = (y, y+mu) embedded in the full space."""
    V, nc = op.V, op.ncomp
    t = int(op._shift(np.arange(V), mu, +1)[y])
    Ue = np.eye(1) if op.kind == 0 else op.links[mu, y]
    E = np.zeros((V * nc, V * nc), dtype=np.complex128)
    bs, bt = slice(y * nc, (y + 1) * nc), slice(t * nc, (t + 1) * nc)
    E[bs, bs] += np.eye(nc)
    E[bt, bt] += np.eye(nc)
    E[bs, bt] -= Ue
    E[bt, bs] -= Ue.conj().T
    return E


def dense_trace_inverse_grad(op):
    """Exact d Tr(A^-1) / dtheta = -Tr(A^-1 (dA/dtheta) A^-1) = -Tr(A^-2 dA/dtheta)
    from a dense inverse (tiny lattices only): (grad_mass [V], grad_coupling [ndim, V])."""
    A = op.dense()
    Ainv = np.linalg.inv(A)
    A2 = Ainv @ Ainv
    nc = op.ncomp
    gm = np.array([-np.trace(A2[y * nc:(y + 1) * nc, y * nc:(y + 1) * nc]).real for y in range(op.V)])
    gw = np.empty((op.ndim, op.V))
    for mu in range(op.ndim):
        for y in range(op.V):
            gw[mu, y] = -np.trace(A2 @ dense_edge_matrix(op, mu, y)).real
    return gm, gw
