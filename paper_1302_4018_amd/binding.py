"""Thin ctypes binding of libtip.so (argument marshalling only).

Every entry point of ``include/tip.h`` has a Python function of the same name
here.  Tensors are torch tensors on the current HIP device; the binding passes
their data pointers and the current torch stream and does no arithmetic of
its own.  Importing this module raises if the library has not been built:
there is no CPU fallback.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtip.so")

TIP_OK, TIP_EINVAL, TIP_ENOMEM, TIP_ENOCONV, TIP_EBREAKDOWN, TIP_EDEVICE, TIP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "TIP_OK", -1: "TIP_EINVAL", -2: "TIP_ENOMEM", -3: "TIP_ENOCONV", -4: "TIP_EBREAKDOWN",
                -5: "TIP_EDEVICE", -6: "TIP_EUNSUPPORTED"}
KIND_SCALAR, KIND_COVARIANT = 0, 1
MASK_DEFAULT, MASK_NONE, MASK_Z2, MASK_Z4 = -1, 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1
PROBE_HIERARCHICAL, PROBE_NATURAL, PROBE_RANDOM, PROBE_STOPPED, PROBE_FOURIER = 0, 1, 2, 3, 4


class tip_operator(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dims", ctypes.c_int64 * 4), ("kind", ctypes.c_int32),
                ("mass", ctypes.c_double), ("mass_field", ctypes.c_void_p), ("coupling", ctypes.c_void_p),
                ("links", ctypes.c_void_p)]


class tip_params(ctypes.Structure):
    _fields_ = [("n_vectors", ctypes.c_int64), ("m_begin", ctypes.c_int64), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("seed", ctypes.c_uint64), ("mask", ctypes.c_int32),
                ("rhs_block", ctypes.c_int32), ("precision", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("quadratures", ctypes.POINTER(ctypes.c_double)), ("reliable_delta", ctypes.c_double),
                ("probe", ctypes.c_int32), ("round_tiles", ctypes.c_int32), ("march_tc", ctypes.c_int32),
                ("stop_levels", ctypes.c_int32), ("item_sites", ctypes.c_int32),
                ("residuals", ctypes.POINTER(ctypes.c_double))]


class tip_tuning(ctypes.Structure):
    _fields_ = [("rhs_block", ctypes.c_int32), ("round_tiles", ctypes.c_int32), ("march_tc", ctypes.c_int32),
                ("seconds_per_solve", ctypes.c_double), ("item_sites", ctypes.c_int32)]


class tip_stats(ctypes.Structure):
    _fields_ = [("solves", ctypes.c_int64), ("total_iters", ctypes.c_int64), ("max_iters", ctypes.c_int32),
                ("n_checkpoints_done", ctypes.c_int32), ("max_true_relres", ctypes.c_double),
                ("seconds", ctypes.c_double), ("stencil_launches", ctypes.c_int64),
                ("stencil_seconds", ctypes.c_double), ("stencil_bytes", ctypes.c_double),
                ("reliable_updates", ctypes.c_int64), ("max_quad_err_bound", ctypes.c_double),
                ("matvecs", ctypes.c_int64), ("matvec_seconds", ctypes.c_double), ("matvec_bytes", ctypes.c_double),
                ("even_odd", ctypes.c_int32), ("restarts", ctypes.c_int64), ("reused", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1302_4018_amd.build` "
                           "(there is no CPU fallback)")
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # so it shares torch's device context and streams (the caller's tensors
    # and streams are torch's)
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "tip_num_checkpoints": (ctypes.c_int32, [ctypes.c_int64]),
        "trace_inv_probe": (ctypes.c_int, [P(tip_operator), P(tip_params), P(ctypes.c_double), P(tip_stats)]),
        "trace_inv_probe_batch": (ctypes.c_int, [P(tip_operator), P(tip_params), ctypes.c_int32, ctypes.c_int32,
                                                 P(P(ctypes.c_double)), P(tip_stats), P(ctypes.c_int32)]),
        "tip_autotune": (ctypes.c_int, [ctypes.c_void_p, P(tip_params), ctypes.c_int64, P(tip_tuning), P(tip_tuning),
                                        ctypes.c_int32, P(ctypes.c_int32)]),
        "tip_autotune_batch": (ctypes.c_int, [P(tip_operator), P(tip_params), ctypes.c_int32, ctypes.c_int64,
                                              P(tip_tuning), P(tip_tuning), ctypes.c_int32, P(ctypes.c_int32)]),
        "tip_op_create": (ctypes.c_int, [P(tip_operator), ctypes.c_void_p, P(ctypes.c_void_p)]),
        "tip_op_destroy": (ctypes.c_int, [ctypes.c_void_p]),
        "trace_inv_probe_op": (ctypes.c_int, [ctypes.c_void_p, P(tip_params), P(ctypes.c_double), P(tip_stats)]),
        "trace_inv_probe_grad": (ctypes.c_int, [ctypes.c_void_p, P(tip_params), P(ctypes.c_double),
                                                ctypes.c_void_p, ctypes.c_void_p, P(tip_stats)]),
        "tip_solve_probe": (ctypes.c_int, [ctypes.c_void_p, P(tip_params), ctypes.c_int64, ctypes.c_int32,
                                           ctypes.c_void_p, P(ctypes.c_double), P(tip_stats)]),
        "tip_apply_operator": (ctypes.c_int, [P(tip_operator), ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]),
        "tip_apply_operator_noalloc": (ctypes.c_int, [P(tip_operator), ctypes.c_int32, ctypes.c_void_p,
                                                      ctypes.c_void_p, ctypes.c_void_p]),
        "tip_hier_perm": (ctypes.c_int, [ctypes.c_int32, P(ctypes.c_int64), ctypes.c_void_p, ctypes.c_void_p]),
        "tip_probe_vectors": (ctypes.c_int, [ctypes.c_int32, P(ctypes.c_int64), ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
        "tip_stream_ceiling": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                              P(ctypes.c_double), P(ctypes.c_double), ctypes.c_void_p]),
        "tip_set_profiling": (None, [ctypes.c_int32]),
        "tip_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class TipError(RuntimeError):
    def __init__(self, status, where):
        msg = lib.tip_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status, where):
    if status != TIP_OK:
        raise TipError(status, where)


def _stream(stream):
    """hipStream_t of a torch stream (default: the current one), or a raw handle."""
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need_cuda(t, name):
    if t is not None and (not t.is_cuda or not t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous tensor on the GPU")


class Operator:
    """Operator description holding device tensors (see tip_operator)."""

    def __init__(self, dims, kind, mass=0.0, mass_field=None, coupling=None, links=None):
        import torch
        self.dims = [int(n) for n in dims]
        self.kind = int(kind)
        self.mass = float(mass)
        self.mass_field = mass_field
        self.coupling = coupling
        if links is not None and links.dtype == torch.complex128:
            links = torch.view_as_real(links)
        self.links = links
        for t, n in ((mass_field, "mass_field"), (coupling, "coupling"), (links, "links")):
            _need_cuda(t, n)

    @property
    def ncomp(self):
        return 3 if self.kind == KIND_COVARIANT else 1

    @property
    def V(self):
        v = 1
        for n in self.dims:
            v *= n
        return v

    def c_struct(self):
        s = tip_operator()
        s.ndim = len(self.dims)
        for j, n in enumerate(self.dims):
            s.dims[j] = n
        s.kind = self.kind
        s.mass = self.mass
        s.mass_field = _ptr(self.mass_field)
        s.coupling = _ptr(self.coupling)
        s.links = _ptr(self.links)
        return s


def _params(n_vectors, tol, seed, mask, max_iter, rhs_block, m_begin, quadratures, stream, precision=PREC_FP64,
            reliable_delta=0.0, probe=PROBE_HIERARCHICAL, round_tiles=0, march_tc=0, stop_levels=0, item_sites=0):
    p = tip_params()
    p.n_vectors = int(n_vectors)
    p.m_begin = int(m_begin)
    p.tol = float(tol)
    p.max_iter = int(max_iter)
    p.seed = int(seed) & ((1 << 64) - 1)
    p.mask = int(mask)
    p.rhs_block = int(rhs_block)
    p.precision = int(precision)
    p.stream = _stream(stream)
    p.quadratures = (None if quadratures is None
                     else quadratures.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    p.reliable_delta = float(reliable_delta)
    p.probe = int(probe)
    p.round_tiles = int(round_tiles)
    p.march_tc = int(march_tc)
    p.stop_levels = int(stop_levels)
    p.item_sites = int(item_sites)
    return p


def _stats_dict(st):
    return {f: getattr(st, f) for f, _ in tip_stats._fields_}


def tip_num_checkpoints(n_vectors):
    return int(lib.tip_num_checkpoints(int(n_vectors)))


def _run(fn, first, n_vectors, tol, seed, mask, max_iter, rhs_block, m_begin, quadratures, stream, raise_on_error,
         precision=PREC_FP64, reliable_delta=0.0, probe=PROBE_HIERARCHICAL, round_tiles=0, march_tc=0,
         stop_levels=0, ncomp=1):
    nck = tip_num_checkpoints(n_vectors)
    est = np.zeros((nck, 2), dtype=np.float64)
    q = np.zeros((int(n_vectors), 2), dtype=np.float64)
    res = np.full((int(n_vectors), int(ncomp)), np.nan)
    if quadratures is not None:
        q[:m_begin] = np.asarray(quadratures, dtype=np.complex128)[:m_begin].view(np.float64).reshape(-1, 2)
    p = _params(n_vectors, tol, seed, mask, max_iter, rhs_block, m_begin, q, stream, precision, reliable_delta, probe,
                round_tiles, march_tc, stop_levels)
    p.residuals = res.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    st = tip_stats()
    status = fn(first, ctypes.byref(p), est.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(st))
    stats = _stats_dict(st)
    stats["status"] = status
    stats["residuals"] = res
    if raise_on_error:
        _check(status, fn.__name__)
    done = stats["n_checkpoints_done"]
    est_c = est[:, 0] + 1j * est[:, 1]
    return est_c[:done] if status != TIP_OK else est_c, q[:, 0] + 1j * q[:, 1], stats


def trace_inv_probe(op, n_vectors, tol, seed, mask=MASK_DEFAULT, max_iter=0, rhs_block=0, m_begin=0,
                    quadratures=None, stream=None, raise_on_error=True, precision=PREC_FP64, reliable_delta=0.0,
                    probe=PROBE_HIERARCHICAL, stop_levels=0):
    """Estimates at s = 2^k (complex numpy), quadratures q_m (complex numpy), stats dict."""
    s = op.c_struct()
    return _run(lib.trace_inv_probe, ctypes.byref(s), n_vectors, tol, seed, mask, max_iter, rhs_block, m_begin,
                quadratures, stream, raise_on_error, precision, reliable_delta, probe, stop_levels=stop_levels,
                ncomp=op.ncomp)


def _batch_structs(ops, n_vectors, tol, seed, mask, max_iter, rhs_block, precision, reliable_delta, probe,
                   stop_levels, item_sites, stream):
    count = len(ops)
    if len(n_vectors) != count:
        raise ValueError("ops and n_vectors differ in length")
    structs = (tip_operator * count)(*[op.c_struct() for op in ops])
    params = (tip_params * count)()
    qs = []
    masks = list(mask) if isinstance(mask, (list, tuple)) else [mask] * count
    for i, n in enumerate(n_vectors):
        q = np.zeros((int(n), 2))
        qs.append(q)
        params[i] = _params(n, tol, seed, masks[i], max_iter, rhs_block, 0, q, stream, precision, reliable_delta,
                            probe, stop_levels=stop_levels, item_sites=item_sites)
    return structs, params, qs


def trace_inv_probe_batch(ops, n_vectors, tol, seed, mask=MASK_DEFAULT, max_iter=0, rhs_block=0,
                          precision=PREC_FP64, reliable_delta=0.0, n_streams=0, raise_on_error=True,
                          probe=PROBE_HIERARCHICAL, stop_levels=0, item_sites=0, stream=None):
    """Independent problems solved together: ops and n_vectors (and mask, when
    a sequence) have one entry per problem.  Returns a list of (estimates complex numpy, stats dict with
    "status" and "quadratures")."""
    count = len(ops)
    structs, params, qs = _batch_structs(ops, n_vectors, tol, seed, mask, max_iter, rhs_block, precision,
                                         reliable_delta, probe, stop_levels, item_sites, stream)
    ests = [np.zeros((tip_num_checkpoints(n), 2)) for n in n_vectors]
    est_ptrs = (ctypes.POINTER(ctypes.c_double) * count)(*[e.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                                                          for e in ests])
    stats = (tip_stats * count)()
    statuses = (ctypes.c_int32 * count)()
    status = lib.trace_inv_probe_batch(structs, params, count, int(n_streams), est_ptrs, stats, statuses)
    if raise_on_error:
        _check(status, "trace_inv_probe_batch")
    out = []
    for i in range(count):
        st = _stats_dict(stats[i])
        st["status"] = statuses[i]
        st["quadratures"] = qs[i][:, 0] + 1j * qs[i][:, 1]
        out.append((ests[i][:, 0] + 1j * ests[i][:, 1], st))
    return out


def tip_autotune_batch(ops, n_vectors, tol, seed, sample_vectors=64, mask=MASK_DEFAULT, precision=PREC_FP64,
                       rhs_block=0, item_sites=0, stream=None):
    """Fastest (rhs_block, item_sites) of trace_inv_probe_batch on a sample:
    returns (best dict, list of tried dicts)."""
    count = len(ops)
    structs, params, _ = _batch_structs(ops, n_vectors, tol, seed, mask, 0, rhs_block, precision, 0.0,
                                        PROBE_HIERARCHICAL, 0, item_sites, stream)
    best = tip_tuning()
    tried = (tip_tuning * 16)()
    n_tried = ctypes.c_int32()
    _check(lib.tip_autotune_batch(structs, params, count, int(sample_vectors), ctypes.byref(best), tried, 16,
                                  ctypes.byref(n_tried)), "tip_autotune_batch")

    def d(t):
        return {"rhs_block": t.rhs_block, "item_sites": t.item_sites, "seconds_per_solve": t.seconds_per_solve}
    return d(best), [d(tried[k]) for k in range(min(n_tried.value, 16))]


class OpHandle:
    """Prepared operator (tip_op_create / tip_op_destroy)."""

    def __init__(self, op, stream=None):
        self._h = ctypes.c_void_p()
        s = op.c_struct()
        _check(lib.tip_op_create(ctypes.byref(s), _stream(stream), ctypes.byref(self._h)), "tip_op_create")
        self.op = op

    def trace_inv_probe(self, n_vectors, tol, seed, mask=MASK_DEFAULT, max_iter=0, rhs_block=0, m_begin=0,
                        quadratures=None, stream=None, raise_on_error=True, precision=PREC_FP64, reliable_delta=0.0,
                        probe=PROBE_HIERARCHICAL, round_tiles=0, march_tc=0, stop_levels=0):
        return _run(lib.trace_inv_probe_op, self._h, n_vectors, tol, seed, mask, max_iter, rhs_block, m_begin,
                    quadratures, stream, raise_on_error, precision, reliable_delta, probe, round_tiles, march_tc,
                    stop_levels, ncomp=self.op.ncomp)

    def autotune(self, tol, seed, sample_vectors=64, mask=MASK_DEFAULT, precision=PREC_FP64, probe=PROBE_HIERARCHICAL,
                 rhs_block=0, round_tiles=0, stream=None):
        """tip_autotune: (best tuning dict, list of tried dicts)."""
        p = _params(1, tol, seed, mask, 0, rhs_block, 0, None, stream, precision, 0.0, probe, round_tiles, 0)
        best = tip_tuning()
        tried = (tip_tuning * 32)()
        n = ctypes.c_int32(0)
        _check(lib.tip_autotune(self._h, ctypes.byref(p), int(sample_vectors), ctypes.byref(best), tried, 32,
                                ctypes.byref(n)), "tip_autotune")
        as_dict = lambda t: {f: getattr(t, f) for f, _ in tip_tuning._fields_}
        return as_dict(best), [as_dict(tried[i]) for i in range(min(n.value, 32))]

    def trace_inv_probe_grad(self, n_vectors, tol, seed, mask=MASK_DEFAULT, max_iter=0, rhs_block=0, stream=None,
                             precision=PREC_FP64, reliable_delta=0.0, mass=True, coupling=True,
                             probe=PROBE_HIERARCHICAL, stop_levels=0):
        """Estimates, quadratures, dT/dm [V] and dT/dw [ndim, V] of the last estimate
        (float64 tensors on the GPU, or None where not asked for), stats."""
        import torch
        op = self.op
        gm = torch.empty(op.V, dtype=torch.float64, device="cuda") if mass else None
        gw = torch.empty((len(op.dims), op.V), dtype=torch.float64, device="cuda") if coupling else None
        nck = tip_num_checkpoints(n_vectors)
        est = np.zeros((nck, 2), dtype=np.float64)
        q = np.zeros((int(n_vectors), 2), dtype=np.float64)
        p = _params(n_vectors, tol, seed, mask, max_iter, rhs_block, 0, q, stream, precision, reliable_delta, probe,
                    stop_levels=stop_levels)
        st = tip_stats()
        _check(lib.trace_inv_probe_grad(self._h, ctypes.byref(p), est.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        _ptr(gm) if gm is not None else None,
                                        _ptr(gw) if gw is not None else None, ctypes.byref(st)),
               "trace_inv_probe_grad")
        return est[:, 0] + 1j * est[:, 1], q[:, 0] + 1j * q[:, 1], gm, gw, _stats_dict(st)

    def solve_probe(self, m, comp, tol, seed, mask=MASK_DEFAULT, max_iter=0, stream=None, precision=PREC_FP64,
                    reliable_delta=0.0, probe=PROBE_HIERARCHICAL, stop_levels=0):
        """x = A^-1 b_{m,comp} (torch tensor on the GPU), q = b^H x, stats."""
        import torch
        op = self.op
        complex_solve = op.kind == KIND_COVARIANT or mask == MASK_Z4 or probe == PROBE_FOURIER
        shape = (op.V, op.ncomp, 2) if complex_solve else (op.V,)
        x = torch.empty(shape, dtype=torch.float64, device="cuda")
        q = np.zeros(2)
        p = _params(1, tol, seed, mask, max_iter, 0, 0, np.zeros((1, 2)), stream, precision, reliable_delta, probe,
                    stop_levels=stop_levels)
        st = tip_stats()
        _check(lib.tip_solve_probe(self._h, ctypes.byref(p), int(m), int(comp), _ptr(x),
                                   q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(st)),
               "tip_solve_probe")
        return (torch.view_as_complex(x) if complex_solve else x), complex(q[0], q[1]), _stats_dict(st)

    def close(self):
        if self._h:
            _check(lib.tip_op_destroy(self._h), "tip_op_destroy")
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trace_inv_probe_op(handle, *args, **kwargs):
    return handle.trace_inv_probe(*args, **kwargs)


def trace_inv_probe_grad(handle, *args, **kwargs):
    return handle.trace_inv_probe_grad(*args, **kwargs)


def tip_solve_probe(handle, *args, **kwargs):
    return handle.solve_probe(*args, **kwargs)


def tip_op_create(op, stream=None):
    return OpHandle(op, stream)


def tip_op_destroy(handle):
    handle.close()


def tip_apply_operator(op, x, stream=None):
    """y = A x; x is [nrhs, V, 3] complex128 (covariant) or [nrhs, V] float64 (scalar) on the GPU."""
    import torch
    _need_cuda(x, "x")
    xr = torch.view_as_real(x) if x.is_complex() else x
    y = torch.empty_like(xr)
    s = op.c_struct()
    _check(lib.tip_apply_operator(ctypes.byref(s), int(x.shape[0]), _ptr(xr), _ptr(y), _stream(stream)),
           "tip_apply_operator")
    return torch.view_as_complex(y) if x.is_complex() else y


def tip_apply_operator_noalloc(op, x, y=None, stream=None):
    """y = A x as tip_apply_operator, with no device allocation inside the
    library (its workspace is the library's fixed scratch); y is allocated
    here unless the caller passes it."""
    import torch
    _need_cuda(x, "x")
    xr = torch.view_as_real(x) if x.is_complex() else x
    if y is None:
        y = torch.empty_like(xr)
    else:
        _need_cuda(y, "y")
        y = torch.view_as_real(y) if y.is_complex() else y
    s = op.c_struct()
    _check(lib.tip_apply_operator_noalloc(ctypes.byref(s), int(x.shape[0]), _ptr(xr), _ptr(y), _stream(stream)),
           "tip_apply_operator_noalloc")
    return torch.view_as_complex(y) if x.is_complex() else y


def tip_hier_perm(dims, stream=None):
    """P(x) for every site as an int32 tensor (values < 2^31)."""
    import torch
    V = int(np.prod(dims))
    out = torch.empty(V, dtype=torch.int32, device="cuda")
    d = (ctypes.c_int64 * 4)(*[int(n) for n in dims])
    _check(lib.tip_hier_perm(len(dims), d, _ptr(out), _stream(stream)), "tip_hier_perm")
    return out


def tip_probe_vectors(dims, ncomp, mask, seed, m0, count, comp, stream=None, probe=PROBE_HIERARCHICAL, stop_levels=0):
    """b_{m,comp} restricted to component comp, m = m0..m0+count-1: complex128 [count, V]."""
    import torch
    V = int(np.prod(dims))
    out = torch.empty((int(count), V, 2), dtype=torch.float64, device="cuda")
    d = (ctypes.c_int64 * 4)(*[int(n) for n in dims])
    _check(lib.tip_probe_vectors(len(dims), d, int(ncomp), int(mask), int(seed) & ((1 << 64) - 1), int(m0),
                                 int(count), int(comp), int(probe), int(stop_levels), _ptr(out), _stream(stream)),
           "tip_probe_vectors")
    return torch.view_as_complex(out)


def tip_stream_ceiling(kind, nbytes, reps=10, grid=0, stream=None):
    """(seconds per pass, bytes per pass) of streaming kernel `kind` (0 read,
    1 copy, 2 three reads + one write) over `nbytes` of device memory."""
    sec, byt = ctypes.c_double(), ctypes.c_double()
    _check(lib.tip_stream_ceiling(int(kind), int(nbytes), int(reps), int(grid), ctypes.byref(sec), ctypes.byref(byt),
                                  _stream(stream)), "tip_stream_ceiling")
    return sec.value, byt.value


def tip_set_profiling(on):
    lib.tip_set_profiling(1 if on else 0)


def tip_last_error():
    return lib.tip_last_error().decode(errors="replace")


def tip_autotune(handle, *args, **kwargs):
    return handle.autotune(*args, **kwargs)
