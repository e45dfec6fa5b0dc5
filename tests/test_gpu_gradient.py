"""Gradient of the estimate with respect to the mass field and the couplings
(trace_inv_probe_grad and the autograd wrapper) against the oracle, entry by
entry.

Tolerance.  Unlike the quadratures, the gradient is not variational: each
entry is quadratic in x, so a solve error enters to first order.  Every entry
is held to its own bound (conftest.gradient_entry_bounds): with both sides
solving to a true relative residual <= tol, the solutions differ by at most
2 tol ||b|| / lambda_min, which moves entry y by at most 2 D sqrt(|g(y)|) + D^2
(D = 2 eps for a site, 4 eps for an edge), lambda_min >= min m(x).
"""

import ctypes
import functools

import numpy as np
import pytest

from conftest import assert_gradient_entries, gpu_binding, to_dev
from oracle.gradient import dense_trace_inverse_grad, trace_inv_probe_grad as oracle_grad
from oracle.mask import MASK_NONE, MASK_Z2, MASK_Z4
from oracle.operators import Operator as OracleOp
from paper_1302_4018_amd import inputs

pytestmark = pytest.mark.gpu


def _ops(tip, dims, kind, seed, coupled=True, m0=0.1):
    mf = inputs.mass_field(dims, m0=m0, seed=seed)
    w = inputs.couplings(dims, seed=seed + 1) if coupled else None
    U = inputs.haar_links(dims, seed=seed + 2) if kind == 1 else None
    orc = OracleOp(dims, kind, mass_field=mf, coupling=w, links=U)
    gop = tip.Operator(dims, kind, mass_field=to_dev(mf), coupling=to_dev(w), links=to_dev(U))
    return orc, gop


CASES = [
    # dims, kind, n_vectors, mask, rhs_block, precision name
    ([16, 16], 0, 32, MASK_Z2, 0, "fp64"),            # one ragged block (32 of 64 lanes)
    ([8, 8], 0, 20, MASK_Z4, 8, "fp64"),              # complex scalar, n not a power of two, 3 blocks
    ([4, 4, 4, 8], 1, 11, MASK_Z4, 8, "fp64"),        # 33 covariant solves: 4 full blocks + 1 lane
    ([8, 8, 8, 8], 1, 8, MASK_Z4, 0, "fp64"),         # 24 solves, several stencil tiles
    ([4, 4, 4, 8], 1, 16, MASK_Z4, 0, "mixed"),
    ([16, 16], 0, 32, MASK_Z2, 0, "mixed"),
]


@pytest.mark.parametrize("dims,kind,n,mask,rhs_block,prec", CASES)
def test_gradient_matches_oracle(dims, kind, n, mask, rhs_block, prec):
    tip = gpu_binding()
    tol = 1e-12
    orc, gop = _ops(tip, dims, kind, seed=200 + len(dims) + kind)
    precision = tip.PREC_MIXED if prec == "mixed" else tip.PREC_FP64
    print(f"gradient parity: dims {dims} kind {kind} n {n} mask {mask} block {rhs_block} {prec}", flush=True)
    with tip.OpHandle(gop) as h:
        est, q, gm, gw, st = h.trace_inv_probe_grad(n, tol, 4018, mask=mask, rhs_block=rhs_block,
                                                    precision=precision)
        est_plain, q_plain, _ = h.trace_inv_probe(n, tol, 4018, mask=mask, rhs_block=rhs_block, precision=precision)
    T_o, gm_o, gw_o, _ = oracle_grad(orc, n, tol, 4018, mask)
    assert st["max_true_relres"] <= tol
    assert abs(est[-1] - T_o) <= 1e-10 * abs(T_o)
    # asking for the gradient changes nothing else
    assert np.array_equal(est, est_plain) and np.array_equal(q, q_plain)
    assert_gradient_entries(gm.cpu().numpy(), gw.cpu().numpy(), gm_o, gw_o, tol, orc.V,
                            float(np.min(orc.mass_at_sites())))
    assert np.all(gm.cpu().numpy() < 0) and np.all(gw.cpu().numpy() <= 0)


def test_gradient_exact_at_s_equals_V():
    """s = V: the probe gradient is the exact -Tr(A^-2 dA/dtheta) (dense inverse)."""
    tip = gpu_binding()
    orc, gop = _ops(tip, [2, 2, 4, 2], 1, seed=300, m0=0.3)
    with tip.OpHandle(gop) as h:
        est, q, gm, gw, st = h.trace_inv_probe_grad(orc.V, 1e-13, 5, mask=MASK_NONE)
    dm, dw = dense_trace_inverse_grad(orc)
    assert_gradient_entries(gm.cpu().numpy(), gw.cpu().numpy(), dm, dw, 1e-13, orc.V,
                            float(np.min(orc.mass_at_sites())))


def test_gradient_full_size_euler_identity():
    """32^4 covariant workload, 4 probes: A is linear in (m, w), T_s homogeneous of
    degree -1, so sum m dT/dm + sum w dT/dw = -T_s (w = 1: no coupling array)."""
    tip = gpu_binding()
    import torch
    dims = [32, 32, 32, 32]
    U = inputs.haar_links(dims)
    mf = inputs.mass_field(dims)
    gop = tip.Operator(dims, tip.KIND_COVARIANT, mass_field=to_dev(mf), links=to_dev(U))
    with tip.OpHandle(gop) as h:
        for prec in (tip.PREC_FP64, tip.PREC_MIXED):
            est, q, gm, gw, st = h.trace_inv_probe_grad(4, 1e-10, 4018, precision=prec)
            T = float(est[-1].real)
            euler = float(torch.dot(gm, torch.from_numpy(mf).cuda())) + float(gw.sum())
            # each quadrature moves by <= ||r||^2/lambda_min; the gradient's Euler sum by
            # <= 2 kappa tol of its size (kappa <= 16.2 / 0.04 here)
            assert abs(euler + T) <= 2.0 * (16.2 / 0.04) * 1e-10 * abs(T) * 2
            assert torch.all(gm < 0) and torch.all(gw <= 0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_gradient_full_size_one_probe_per_site(prec):
    """32^4 covariant workload (Haar links, m(x) = 0.1 + 0.02 clip(xi)), probe 0
    with its 3 diluted solves: dT/dm(y) at all 2^20 sites and dT/dw_mu(y) on
    all 2^22 edges against the oracle's CG, entry by entry (tol 1e-12)."""
    tip = gpu_binding()
    dims = [32, 32, 32, 32]
    U = inputs.haar_links(dims)
    mf = inputs.mass_field(dims)
    tol = 1e-12
    gop = tip.Operator(dims, tip.KIND_COVARIANT, mass_field=to_dev(mf), links=to_dev(U))
    precision = tip.PREC_MIXED if prec == "mixed" else tip.PREC_FP64
    print(f"gradient 32^4, one probe, {prec}", flush=True)
    with tip.OpHandle(gop) as h:
        est, q, gm, gw, st = h.trace_inv_probe_grad(1, tol, 4018, precision=precision)
    gm, gw = gm.cpu().numpy(), gw.cpu().numpy()
    del gop
    T_o, gm_o, gw_o = _oracle_grad_32to4_probe0(tol)
    assert st["max_true_relres"] <= tol
    assert abs(est[-1] - T_o) <= 1e-10 * abs(T_o)
    assert_gradient_entries(gm, gw, gm_o, gw_o, tol, mf.size, float(np.min(mf)))


@functools.lru_cache(maxsize=1)
def _oracle_grad_32to4_probe0(tol):
    """The oracle's gradient of T_1 on the 32^4 workload (three CG solves on the
    host), computed once for both precisions."""
    dims = [32, 32, 32, 32]
    orc = OracleOp(dims, 1, mass_field=inputs.mass_field(dims), links=inputs.haar_links(dims))
    T_o, gm_o, gw_o, _ = oracle_grad(orc, 1, tol, 4018, MASK_Z4)
    return T_o, gm_o, gw_o


def test_gradient_central_differences_8to4():
    """8^4 covariant operator with a mass field and couplings, 8 probes (24
    solves), probes held fixed: central differences of the GPU estimate with
    respect to m(y) and w_mu(y), h = 1e-4, at sites and edges spread over the
    lattice, against the GPU gradient.  The truncation error h^2/6 times the
    third derivative is below 1e-8 of the gradient's scale here (the random
    links keep lambda_min of order 1), far inside the 1e-6 tolerance."""
    tip = gpu_binding()
    dims = [8, 8, 8, 8]
    mf = inputs.mass_field(dims, m0=0.1, seed=350)
    w = inputs.couplings(dims, seed=351)
    U = to_dev(inputs.haar_links(dims, seed=352))
    n, tol, hstep = 8, 1e-13, 1e-4

    def estimate(m_arr, w_arr):
        op = tip.Operator(dims, tip.KIND_COVARIANT, mass_field=to_dev(m_arr), coupling=to_dev(w_arr), links=U)
        est, _, _ = tip.trace_inv_probe(op, n, tol, 17)
        return float(est[-1].real)

    gop = tip.Operator(dims, tip.KIND_COVARIANT, mass_field=to_dev(mf), coupling=to_dev(w), links=U)
    with tip.OpHandle(gop) as h:
        _, _, gm, gw, _ = h.trace_inv_probe_grad(n, tol, 17)
    gm, gw = gm.cpu().numpy(), gw.cpu().numpy()
    scale_m, scale_w = np.abs(gm).max(), np.abs(gw).max()
    for y in (0, 1, 777, 2048, 4095):
        d = np.zeros_like(mf)
        d[y] = hstep
        fd = (estimate(mf + d, w) - estimate(mf - d, w)) / (2 * hstep)
        assert abs(fd - gm[y]) <= 1e-6 * scale_m, (y, fd, gm[y])
    for mu, y in ((0, 5), (1, 1000), (2, 3333), (3, 4095)):
        d = np.zeros_like(w)
        d[mu, y] = hstep
        fd = (estimate(mf, w + d) - estimate(mf, w - d)) / (2 * hstep)
        assert abs(fd - gw[mu, y]) <= 1e-6 * scale_w, (mu, y, fd, gw[mu, y])


def test_gradient_is_reproducible():
    tip = gpu_binding()
    orc, gop = _ops(tip, [8, 8, 8, 8], 1, seed=310)
    with tip.OpHandle(gop) as h:
        a = h.trace_inv_probe_grad(8, 1e-10, 1)
        b = h.trace_inv_probe_grad(8, 1e-10, 1)
    assert np.array_equal(a[0], b[0])
    assert torch_equal(a[2], b[2]) and torch_equal(a[3], b[3])


def torch_equal(x, y):
    import torch
    return bool(torch.equal(x, y))


def test_gradient_only_mass_or_only_coupling():
    tip = gpu_binding()
    orc, gop = _ops(tip, [8, 8], 0, seed=320)
    with tip.OpHandle(gop) as h:
        _, _, gm, gw, _ = h.trace_inv_probe_grad(16, 1e-12, 3)
        _, _, gm1, gw1, _ = h.trace_inv_probe_grad(16, 1e-12, 3, coupling=False)
        _, _, gm2, gw2, _ = h.trace_inv_probe_grad(16, 1e-12, 3, mass=False)
    assert gw1 is None and gm2 is None
    assert torch_equal(gm, gm1) and torch_equal(gw, gw2)


def test_gradient_argument_errors():
    tip = gpu_binding()
    orc, gop = _ops(tip, [8, 8], 0, seed=330)
    with tip.OpHandle(gop) as h:
        est = np.zeros((8, 2))
        q = np.zeros((16, 2))
        p = tip._params(16, 1e-10, 1, tip.MASK_DEFAULT, 0, 0, 0, q, None)
        dptr = ctypes.POINTER(ctypes.c_double)
        st = tip.tip_stats()
        s = tip.lib.trace_inv_probe_grad(h._h, ctypes.byref(p), est.ctypes.data_as(dptr), None, None,
                                         ctypes.byref(st))
        assert s == tip.TIP_EINVAL and "NULL" in tip.tip_last_error()
        import torch
        g = torch.zeros(64, dtype=torch.float64, device="cuda")
        p.m_begin = 4
        s = tip.lib.trace_inv_probe_grad(h._h, ctypes.byref(p), est.ctypes.data_as(dptr),
                                         ctypes.c_void_p(g.data_ptr()), None, ctypes.byref(st))
        assert s == tip.TIP_EINVAL and "m_begin" in tip.tip_last_error()


def test_autograd_function():
    """torch.autograd through TraceInv: same value and gradients as the C entry
    point, and central finite differences of the GPU forward agree."""
    tip = gpu_binding()
    import torch
    from paper_1302_4018_amd.autograd import trace_inv
    dims = [4, 4, 4, 8]
    mf = torch.from_numpy(inputs.mass_field(dims, m0=0.2, seed=340)).cuda().requires_grad_(True)
    w = torch.from_numpy(inputs.couplings(dims, seed=341)).cuda().requires_grad_(True)
    U = torch.from_numpy(inputs.haar_links(dims, seed=342)).cuda()
    kw = dict(dims=dims, kind=tip.KIND_COVARIANT, n_vectors=8, tol=1e-12, seed=9)
    T = trace_inv(mf, w, U, **kw)
    gm, gw = torch.autograd.grad(3.0 * T, (mf, w))
    gop = tip.Operator(dims, tip.KIND_COVARIANT, mass_field=mf.detach(), coupling=w.detach(), links=U)
    with tip.OpHandle(gop) as h:
        est, _, rm, rw, _ = h.trace_inv_probe_grad(8, 1e-12, 9)
    assert float(T) == float(est[-1].real)
    assert torch.equal(gm, 3.0 * rm) and torch.equal(gw, 3.0 * rw)
    hstep = 1e-4
    with torch.no_grad():
        for y in (0, 77, 511):
            d = torch.zeros_like(mf)
            d[y] = hstep
            fd = (float(trace_inv(mf + d, w, U, **kw)) - float(trace_inv(mf - d, w, U, **kw))) / (2 * hstep)
            assert abs(fd - float(rm[y])) <= 1e-6 * float(rm.abs().max())
        for mu, y in ((0, 5), (3, 300)):
            d = torch.zeros_like(w)
            d[mu, y] = hstep
            fd = (float(trace_inv(mf, w + d, U, **kw)) - float(trace_inv(mf, w - d, U, **kw))) / (2 * hstep)
            assert abs(fd - float(rw[mu, y])) <= 1e-6 * float(rw.abs().max())
    # no gradient asked: the plain run
    with torch.no_grad():
        assert float(trace_inv(mf, w, U, **kw)) == float(T)


def test_c1_uniform_mass_gradient_closed_form():
    """16^2 free torus, m = 0.1, all 256 probes: the GPU gradient summed over
    sites is d Tr(A^-1)/dm = -sum_k lambda(k)^-2 = -231.195071582666."""
    tip = gpu_binding()
    import torch
    gop = tip.Operator([16, 16], tip.KIND_SCALAR, mass_field=torch.full((256,), 0.1, dtype=torch.float64,
                                                                        device="cuda"))
    with tip.OpHandle(gop) as h:
        est, q, gm, gw, st = h.trace_inv_probe_grad(256, 1e-13, 4018)
    assert abs(float(gm.sum()) - (-231.195071582666)) <= 1e-9 * 231.195071582666
    assert abs(est[-1].real - 116.949743403339) <= 1e-10 * 116.949743403339
