"""The probing estimate of Tr(A^-1) as a differentiable function of the
operator's mass field m(x) and edge couplings w_mu(x).

forward:  one probing run through the HIP library (trace_inv_probe_grad) that
          returns Re T_s at s = n_vectors.
backward: the gradient of that estimate with the probes held fixed,
          dT/dtheta = -(1/s) sum_{m,c} x_{m,c}^H (dA/dtheta) x_{m,c}
          (Sec. 1's estimator differentiated; A is Hermitian, so the adjoint
          solves are the forward ones).  The library adds each block's
          contribution while its solutions are still in the CG workspace, so
          the forward pass stores two O(V) arrays instead of all
          n_vectors x ncomp solutions; backward only scales them.

The imaginary part of T_s vanishes up to rounding (b^H A^-1 b is real for
Hermitian A) and is dropped.
"""

import torch

from . import binding as tip


class TraceInv(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mass_field, coupling, links, dims, kind, n_vectors, tol, seed, mask, precision,
                reliable_delta, rhs_block):
        want_m = ctx.needs_input_grad[0]
        want_w = coupling is not None and ctx.needs_input_grad[1]
        op = tip.Operator(dims, kind, mass_field=mass_field.detach().contiguous(),
                          coupling=None if coupling is None else coupling.detach().contiguous(),
                          links=None if links is None else links.detach().contiguous())
        with tip.OpHandle(op) as h:
            kw = dict(mask=mask, rhs_block=rhs_block, precision=precision, reliable_delta=reliable_delta)
            if want_m or want_w:
                est, _, gm, gw, _ = h.trace_inv_probe_grad(n_vectors, tol, seed, mass=want_m, coupling=want_w, **kw)
            else:
                est, _, _ = h.trace_inv_probe(n_vectors, tol, seed, **kw)
                gm = gw = None
        ctx.save_for_backward(gm, gw)
        return torch.tensor(float(est[-1].real), dtype=torch.float64, device=mass_field.device)

    @staticmethod
    def backward(ctx, grad_out):
        gm, gw = ctx.saved_tensors
        return (None if gm is None else grad_out * gm, None if gw is None else grad_out * gw,
                None, None, None, None, None, None, None, None, None, None)


def trace_inv(mass_field, coupling=None, links=None, *, dims, kind, n_vectors, tol=1e-10, seed=0,
              mask=tip.MASK_DEFAULT, precision=tip.PREC_FP64, reliable_delta=0.0, rhs_block=0):
    """Re T_s (0-d float64 tensor) with autograd through mass_field [V] and coupling [ndim, V].

    mass_field, coupling: float64 GPU tensors; links: complex128 [ndim, V, 3, 3]
    GPU tensor for the covariant operator (not differentiated).
    """
    return TraceInv.apply(mass_field, coupling, links, list(dims), int(kind), int(n_vectors), float(tol), int(seed),
                          int(mask), int(precision), float(reliable_delta), int(rhs_block))
