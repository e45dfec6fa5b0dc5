"""Host-side checks of the C ABI: the library loads, exports every function
that include/tip.h declares, the ctypes structures match the C layout, and
argument validation rejects bad input before any device work (no GPU needed)."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "tip.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:tip_status|int32_t|void|const char\s*\*)\s+(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    from paper_1302_4018_amd import binding
    names = _declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(binding.lib, n), n
        assert hasattr(binding, n), f"binding lacks {n}"


def test_struct_layout_matches_c(tmp_path):
    from paper_1302_4018_amd import binding as b
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stddef.h>
#include <stdio.h>
#include "tip.h"
#define P(T, F) printf(#T "." #F " %zu\\n", offsetof(T, F));
int main(void) {
  printf("tip_operator %zu\\n", sizeof(tip_operator));
  printf("tip_params %zu\\n", sizeof(tip_params));
  printf("tip_stats %zu\\n", sizeof(tip_stats));
  P(tip_operator, dims) P(tip_operator, kind) P(tip_operator, mass) P(tip_operator, links)
  P(tip_params, tol) P(tip_params, seed) P(tip_params, mask) P(tip_params, stream) P(tip_params, quadratures)
  P(tip_params, reliable_delta) P(tip_params, probe) P(tip_params, round_tiles) P(tip_params, march_tc)
  P(tip_params, stop_levels) P(tip_params, item_sites) P(tip_params, residuals)
  printf("tip_tuning %zu\\n", sizeof(tip_tuning));
  P(tip_tuning, seconds_per_solve) P(tip_tuning, item_sites)
  P(tip_stats, max_true_relres) P(tip_stats, stencil_launches) P(tip_stats, stencil_bytes)
  P(tip_stats, reliable_updates) P(tip_stats, max_quad_err_bound) P(tip_stats, matvecs)
  P(tip_stats, matvec_seconds) P(tip_stats, matvec_bytes) P(tip_stats, even_odd) P(tip_stats, restarts) P(tip_stats, reused)
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                             check=True).stdout.split("\n") if line)
    classes = {"tip_operator": b.tip_operator, "tip_params": b.tip_params, "tip_stats": b.tip_stats,
               "tip_tuning": b.tip_tuning}
    for key, val in out.items():
        if "." in key:
            cls, field = key.split(".")
            assert getattr(classes[cls], field).offset == int(val), key
        else:
            assert ctypes.sizeof(classes[key]) == int(val), key


def test_num_checkpoints_matches_oracle():
    from oracle.estimator import checkpoint_sizes
    from paper_1302_4018_amd import binding as b
    for n in [1, 2, 3, 7, 8, 100, 256, 1000, 1024, 65536]:
        assert b.tip_num_checkpoints(n) == len(checkpoint_sizes(n))


def test_validation_rejects_bad_arguments_without_device_work():
    from paper_1302_4018_amd import binding as b
    lib = b.lib

    def call(op, **kw):
        p = b._params(kw.get("n", 4), kw.get("tol", 1e-10), 1, kw.get("mask", -1), 0, 0, kw.get("m_begin", 0),
                      np.zeros((8, 2)), 0)
        est = np.zeros((8, 2))
        return lib.trace_inv_probe(ctypes.byref(op), ctypes.byref(p),
                                   est.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None)

    op = b.tip_operator()
    op.ndim = 0
    assert call(op) == b.TIP_EINVAL and "ndim" in b.tip_last_error()
    op.ndim = 2
    op.dims[0], op.dims[1] = 0, 4
    assert call(op) == b.TIP_EINVAL and "must be >= 1" in b.tip_last_error()
    op.dims[0] = 4
    op.kind = 1                        # covariant without links
    assert call(op) == b.TIP_EINVAL and "links" in b.tip_last_error()
    op.kind = 7
    assert call(op) == b.TIP_EINVAL
    op.kind = 0
    assert call(op, n=0) == b.TIP_EINVAL and "n_vectors" in b.tip_last_error()
    assert call(op, n=17) == b.TIP_EINVAL
    d = (ctypes.c_int64 * 4)(1 << 16, 1 << 16, 1, 1)
    assert lib.tip_hier_perm(2, d, None, None) == b.TIP_EINVAL       # V > 2^31 is fine at 2^32? no: rejected
    d44 = (ctypes.c_int64 * 4)(4, 4, 0, 0)
    assert lib.tip_probe_vectors(2, d44, 2, -1, 1, 0, 1, 0, 0, 0, None, None) == b.TIP_EINVAL
    assert lib.tip_probe_vectors(2, d44, 1, 0, 1, 0, 1, 0, 2, 0, None, None) == b.TIP_EINVAL
    assert "Z2 or Z4" in b.tip_last_error()
    for kind in (b.PROBE_NATURAL, b.PROBE_STOPPED, b.PROBE_FOURIER):
        assert lib.tip_probe_vectors(2, (ctypes.c_int64 * 4)(6, 4, 0, 0), 1, 1, 1, 0, 1, 0, kind, 0, None,
                                     None) == b.TIP_EINVAL
        assert "power-of-two" in b.tip_last_error()
    assert lib.tip_probe_vectors(2, d44, 1, 1, 1, 0, 1, 0, b.PROBE_STOPPED, -1, None, None) == b.TIP_EINVAL
    assert "stop_levels" in b.tip_last_error()
    assert lib.tip_probe_vectors(2, d44, 1, 1, 1, 0, 1, 0, 5, 0, None, None) == b.TIP_EINVAL
    assert "probe kind" in b.tip_last_error()
