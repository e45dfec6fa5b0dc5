"""Writes the stored oracle quadratures that the full-probe-count parity tests
read (test infrastructure; calls nothing but oracle/ and the seeded input
generators).

Each file holds one line per probe m: the workload's label, m, Re q_m, Im q_m
with q_m = sum_c b_{m,c}^H A^-1 b_{m,c} (Sec. 1 estimator with the probes of
Alg. 5 / Sec. 3.4 and internal dilution; solves by textbook CG to a true
relative residual <= tol, Sec. 1.1.2).  The estimates at s = 2^k follow from
them with oracle.estimator.estimates_from_quadratures.

    python tests/golden/make_quadratures.py c2 | c3 | c4 | all

  c2  3-D 32^3 scalar Laplacian, w ~ U[0.5, 1.5] per forward edge, m = 0.05,
      Z2 mask seed 4018, tol 1e-10, probes 0..511 (every 3-D completion point
      up to s = 128, and s = 512)
  c3  4-D 16^4 covariant Laplacian, Haar U(3) links, m = 0.1, Z4 mask seed 4018,
      tol 1e-10, probes 0..63 (past the 4-D completion point s = 32)
  c4  the 64 uneven 3-D tori of the batch workload (sides iid in 8..48,
      m ~ U[0.02, 0.2], w ~ U[0.5, 1.5]), Z2 mask seed 4018, tol 1e-10,
      probes 0..3 of every torus
"""

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import general  # noqa: E402
from oracle.estimator import trace_inv_probe  # noqa: E402
from oracle.mask import MASK_Z2, MASK_Z4  # noqa: E402
from oracle.operators import Operator  # noqa: E402
from paper_1302_4018_amd import inputs  # noqa: E402

SEED = 4018
TOL = 1e-10


def _write(name, header, rows):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        for line in header:
            f.write(f"# {line}\n")
        for label, m, q in rows:
            f.write(f"{label} {m} {q.real:.17e} {q.imag:.17e}\n")
    print(f"wrote {path} ({len(rows)} rows)", flush=True)


def c2():
    dims = [32, 32, 32]
    op = Operator(dims, 0, mass=0.05, coupling=inputs.couplings(dims, seed=1))
    _, q, st = trace_inv_probe(op, 512, TOL, SEED, MASK_Z2)
    _write("quadratures_c2_32x32x32.txt",
           ["oracle quadratures q_m, m = 0..511: 32^3 scalar Laplacian, w = inputs.couplings(dims, seed=1),",
            "m = 0.05, Z2 mask seed 4018, CG to a true relative residual <= 1e-10 (Sec. 1 estimator,",
            "Alg. 5 probes, Sec. 1.1.2 solves); written by tests/golden/make_quadratures.py c2",
            f"CG iterations per solve: {min(st['iters'])}..{max(st['iters'])}"],
           [("c2", m, complex(v)) for m, v in enumerate(q)])


def c3():
    dims = [16, 16, 16, 16]
    op = Operator(dims, 1, mass=0.1, links=inputs.haar_links(dims, seed=3))
    _, q, st = trace_inv_probe(op, 64, TOL, SEED, MASK_Z4)
    _write("quadratures_c3_16x16x16x16.txt",
           ["oracle quadratures q_m = sum_c b_{m,c}^H A^-1 b_{m,c}, m = 0..63: 16^4 covariant Laplacian,",
            "links = inputs.haar_links(dims, seed=3), m = 0.1, Z4 mask seed 4018, full internal dilution,",
            "CG to a true relative residual <= 1e-10 (Sec. 1 estimator, Alg. 5 probes, Sec. 1.1.2 solves);",
            "written by tests/golden/make_quadratures.py c3",
            f"CG iterations per solve: {min(st['iters'])}..{max(st['iters'])}"],
           [("c3", m, complex(v)) for m, v in enumerate(q)])


def c4():
    rows = []
    for i, t in enumerate(inputs.uneven_tori()):
        dims = t["dims"]
        op = Operator(dims, 0, mass=t["mass"], coupling=inputs.uneven_torus_couplings(dims, i))
        _, q, _ = general.trace_inv_probe(op, 4, TOL, SEED, MASK_Z2)
        rows += [(f"torus{i}", m, complex(v)) for m, v in enumerate(q)]
    _write("quadratures_c4_uneven_tori.txt",
           ["oracle quadratures q_m, m = 0..3, of each of the 64 uneven 3-D tori of inputs.uneven_tori()",
            "(couplings inputs.uneven_torus_couplings(dims, i), mass t['mass']), Z2 mask seed 4018,",
            "CG to a true relative residual <= 1e-10; probes of Sec. 3.4 (binary levels, then the",
            "three-colouring level's F_3 columns, eq. Hperm-general-recursive); written by",
            "tests/golden/make_quadratures.py c4"],
           rows)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    for name, fn in (("c2", c2), ("c3", c3), ("c4", c4)):
        if which in (name, "all"):
            t = time.perf_counter()
            fn()
            print(f"{name}: {time.perf_counter() - t:.1f} s", flush=True)
