"""Shifted lattice Laplacians on a periodic d-dimensional torus (test infrastructure only).

The paper's control problem (Sec. 5) is the Laplacian of a uniform periodic
lattice with a diagonal shift that sets the condition number.  Both operators
here are that Laplacian written as a sum over the edges e = (x, x+mu) of the
torus plus a diagonal mass:

    A = sum_e w_e L_e + diag(m(x)) (x) I_ncomp,

where edge e joins x and x+mu, carries the weight w_mu(x) (1 when no coupling
array is given) and, for the covariant operator, the unitary 3x3 parallel
transporter U_mu(x):

    scalar   (ncomp = 1):  L_e = [[1, -1], [-1, 1]]
    covariant (ncomp = 3): L_e = [[I, -U_mu(x)], [-U_mu(x)^H, I]].

The covariant form stands in for the internal dimension 3 of the LQCD matrix
(Sec. 1.1.1); it is Hermitian positive definite with lambda_min >= min m(x).
At w = 1 and constant m the diagonal is m + 2d, e.g. (4+m) I - sum of the
neighbours on a 2-D lattice.

Array conventions (shared with the C header by statement only):
  x        [V, ncomp] complex128 (or [V] real for ncomp = 1), site order s(x)
  mass     scalar, or mass_field [V]
  coupling [d, V]  w_mu(x) for the edge x -> x+mu, or None (all ones)
  links    [d, V, 3, 3] complex128, U_mu(x)[a, b] acting as (U x)_a = sum_b U_ab x_b
"""

import numpy as np

from .lattice import volume


class Operator:
    def __init__(self, dims, kind, mass=0.0, mass_field=None, coupling=None, links=None):
        self.dims = [int(n) for n in dims]
        self.ndim = len(self.dims)
        self.V = volume(self.dims)
        self.kind = kind                      # 0 scalar, 1 covariant
        self.ncomp = 1 if kind == 0 else 3
        self.mass = float(mass)
        self.mass_field = None if mass_field is None else np.asarray(mass_field, dtype=np.float64)
        self.coupling = None if coupling is None else np.asarray(coupling, dtype=np.float64)
        self.links = None if links is None else np.asarray(links, dtype=np.complex128)
        if kind == 1 and self.links is None:
            raise ValueError("covariant operator needs links")

    # -- lattice helpers -------------------------------------------------
    def _grid(self, a):
        """View a per-site array [V, ...] as [n_d, ..., n_1, ...]."""
        return a.reshape(tuple(reversed(self.dims)) + a.shape[1:])

    def _shift(self, a, mu, sign):
        """Array whose value at site s is a(s + sign * mu_hat) (periodic)."""
        g = self._grid(a)
        axis = self.ndim - 1 - mu
        return np.roll(g, -sign, axis=axis).reshape(a.shape)

    def mass_at_sites(self):
        if self.mass_field is not None:
            return self.mass_field
        return np.full(self.V, self.mass)

    def weight(self, mu):
        if self.coupling is None:
            return np.ones(self.V)
        return self.coupling[mu]

    # -- y = A x -----------------------------------------------------------
    def apply(self, x):
        x = np.asarray(x)
        xv = x.reshape(self.V, self.ncomp)
        diag = self.mass_at_sites().copy()
        y = np.zeros(xv.shape, dtype=np.result_type(xv.dtype, np.float64,
                                                     np.complex128 if self.kind == 1 else np.float64))
        for mu in range(self.ndim):
            w_fwd = self.weight(mu)                       # w_mu(s): edge s -> s+mu
            w_bwd = self._shift(w_fwd, mu, -1)            # w_mu(s-mu): edge s-mu -> s
            diag = diag + w_fwd + w_bwd
            x_fwd = self._shift(xv, mu, +1)               # x(s+mu)
            x_bwd = self._shift(xv, mu, -1)               # x(s-mu)
            if self.kind == 0:
                y -= w_fwd[:, None] * x_fwd + w_bwd[:, None] * x_bwd
            else:
                U = self.links[mu]                        # U_mu(s)
                U_bwd = self._shift(U, mu, -1)            # U_mu(s-mu)
                hop_fwd = np.einsum("sab,sb->sa", U, x_fwd)
                hop_bwd = np.einsum("sba,sb->sa", U_bwd.conj(), x_bwd)   # U^H x
                y -= w_fwd[:, None] * hop_fwd + w_bwd[:, None] * hop_bwd
        y += diag[:, None] * xv
        return y.reshape(x.shape)

    # -- dense matrix, assembled edge by edge (tiny lattices only) ----------
    def dense(self):
        V, nc = self.V, self.ncomp
        A = np.zeros((V * nc, V * nc), dtype=np.complex128)
        m = self.mass_at_sites()
        for s in range(V):
            A[s * nc:(s + 1) * nc, s * nc:(s + 1) * nc] += m[s] * np.eye(nc)
        idx = np.arange(V)
        for mu in range(self.ndim):
            nbr = self._shift(idx, mu, +1)                # s + mu
            w = self.weight(mu)
            for s in range(V):
                t = int(nbr[s])
                Ue = np.eye(1) if self.kind == 0 else self.links[mu, s]
                bs, bt = slice(s * nc, (s + 1) * nc), slice(t * nc, (t + 1) * nc)
                A[bs, bs] += w[s] * np.eye(nc)
                A[bt, bt] += w[s] * np.eye(nc)
                A[bs, bt] -= w[s] * Ue
                A[bt, bs] -= w[s] * Ue.conj().T
        return A
