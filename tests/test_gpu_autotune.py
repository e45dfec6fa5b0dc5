"""tip_autotune and the tuning cache: candidates are timed, the best one is
among them, results under every tried configuration agree with the default
to rounding, and the cache returns the stored choice without timing again."""

import json

import numpy as np
import pytest

from conftest import gpu_binding, to_dev
from paper_1302_4018_amd import inputs

pytestmark = pytest.mark.gpu


def test_autotune_candidates_and_results(tmp_path):
    tip = gpu_binding()
    from paper_1302_4018_amd import autotune
    dims = [16, 16, 16, 16]
    U = inputs.haar_links(dims, seed=800)
    gop = tip.Operator(dims, tip.KIND_COVARIANT, mass_field=to_dev(inputs.mass_field(dims, seed=801)),
                       links=to_dev(U))
    with tip.OpHandle(gop) as h:
        best, tried = h.autotune(1e-10, 4018, sample_vectors=16)
        assert len(tried) == 15                       # 3 block sizes x 5 tile rounds
        assert best in tried
        assert best["seconds_per_solve"] == min(t["seconds_per_solve"] for t in tried)
        ref, _, _ = h.trace_inv_probe(16, 1e-10, 4018)
        for t in tried[::4]:
            est, _, st = h.trace_inv_probe(16, 1e-10, 4018, rhs_block=t["rhs_block"], round_tiles=t["round_tiles"])
            assert np.max(np.abs(est - ref) / np.abs(ref)) <= 1e-12
        path = str(tmp_path / "tune.json")
        kw = autotune.tuned(h, 1e-10, 4018, sample_vectors=16, path=path)
        table = json.load(open(path))
        assert len(table) == 1 and kw["rhs_block"] in (16, 32, 64)
        # a second call reads the cache (same answer, no new entry)
        assert autotune.tuned(h, 1e-10, 4018, sample_vectors=16, path=path) == kw
        assert len(json.load(open(path))) == 1


def test_autotune_on_an_odd_torus_tunes_the_block_only():
    tip = gpu_binding()
    dims = [12, 10, 6]
    gop = tip.Operator(dims, tip.KIND_SCALAR, mass=0.1, coupling=to_dev(inputs.couplings(dims, seed=810)))
    with tip.OpHandle(gop) as h:
        best, tried = h.autotune(1e-10, 1, sample_vectors=32)
    assert sorted(t["rhs_block"] for t in tried) == [16, 32, 64] and all(t["round_tiles"] == 0 for t in tried)


@pytest.mark.parametrize("march_tc,round_tiles", [(1, 64), (2, 128), (4, 256), (1, 512), (8, 0)])
def test_march_chunks_and_rounds_agree(march_tc, round_tiles):
    """The half-lattice stencil with chunks of 1..8 marched slices (each chunk
    starts by loading the slice its march would have carried) and rounds of
    64..512 tiles per XCD, each round through all its chunks before the next:
    every site is computed the same way, so the quadratures agree with the
    default launch shape to rounding, in FP64 and in mixed precision."""
    tip = gpu_binding()
    dims = [16, 16, 16, 16]
    U = inputs.haar_links(dims, seed=810)
    gop = tip.Operator(dims, tip.KIND_COVARIANT, mass_field=to_dev(inputs.mass_field(dims, seed=811)),
                       links=to_dev(U))
    print(f"march chunks: tc {march_tc} round_tiles {round_tiles}", flush=True)
    with tip.OpHandle(gop) as h:
        for prec in (tip.PREC_FP64, tip.PREC_MIXED):
            _, qr, _ = h.trace_inv_probe(32, 1e-11, 4018, precision=prec)
            _, q, st = h.trace_inv_probe(32, 1e-11, 4018, precision=prec, march_tc=march_tc,
                                         round_tiles=round_tiles)
            assert st["even_odd"] == 1 and st["max_true_relres"] <= 1e-11
            assert np.max(np.abs(q - qr) / np.abs(qr)) <= 1e-10
