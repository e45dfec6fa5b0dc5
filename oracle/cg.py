"""Conjugate gradients for the quadratures z^H A^-1 z (test infrastructure only).

Sec. 1.1.2: instead of Lanczos quadrature one may solve A x = z and form
z^H x; for Hermitian A the quadrature error falls as the square of the
residual norm, so the residual only has to reach the square root of the
wanted quadrature accuracy.  The paper does not name a solver or a stopping
rule.  Reading used by this project: textbook Hestenes-Stiefel CG from x0 = 0
with the recursive residual, and a solve is accepted only when the TRUE
residual b - A x (recomputed in FP64) satisfies ||b - A x||_2 <= tol ||b||_2;
if the recursive residual passes but the true one does not, CG restarts from
the current x with r = p = b - A x.
"""

import numpy as np


class CGError(RuntimeError):
    def __init__(self, kind, msg):
        super().__init__(msg)
        self.kind = kind                  # "noconv" or "breakdown"


def _dot(a, b):
    return np.vdot(a, b)                  # a^H b


def cg_solve(apply, b, tol, max_iter):
    """Returns (x, iterations, true relative residual)."""
    b = np.asarray(b)
    bnorm = np.sqrt(_dot(b, b).real)
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    r = b.copy()
    p = r.copy()
    rho = _dot(r, r).real
    it = 0
    while True:
        if np.sqrt(rho) <= tol * bnorm:
            rt = b - apply(x)
            rt_norm = np.sqrt(_dot(rt, rt).real)
            if rt_norm <= tol * bnorm:
                return x, it, rt_norm / bnorm
            r = rt
            p = r.copy()
            rho = rt_norm ** 2
        if it >= max_iter:
            raise CGError("noconv", f"CG did not converge in {max_iter} iterations")
        Ap = apply(p)
        pAp = _dot(p, Ap).real
        if not np.isfinite(pAp) or pAp <= 0.0:
            raise CGError("breakdown", f"p^H A p = {pAp} at iteration {it}")
        alpha = rho / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        rho_new = _dot(r, r).real
        beta = rho_new / rho
        p = r + beta * p
        rho = rho_new
        it += 1
