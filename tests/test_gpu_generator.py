"""GPU parity of the probing-vector generator: bit-exact against the oracle."""

import numpy as np
import pytest

from conftest import gpu_binding
from oracle.hierperm import hier_perm
from oracle.probing import rhs

pytestmark = pytest.mark.gpu

SHAPES = [[16, 16], [32, 32, 32], [16, 16, 16, 16], [32, 32, 32, 32], [64], [4, 2, 8], [2, 8, 4, 16],
          [1, 4], [4, 1, 2], [2, 2], [1], [8, 8, 1, 4], [1024, 2, 1, 32]]


@pytest.mark.parametrize("dims", SHAPES)
def test_hier_perm_bit_exact(dims):
    tip = gpu_binding()
    got = tip.tip_hier_perm(dims).cpu().numpy().astype(np.int64)
    want = hier_perm(dims).astype(np.int64)
    assert np.array_equal(got, want)


CASES = [([16, 16], 1, 1), ([16, 16], 1, 0), ([32, 32, 32], 1, 1), ([16, 16, 16, 16], 3, 2),
         ([4, 2, 8], 3, 1), ([8, 8, 1, 4], 1, 2), ([2, 2], 3, 0), ([32, 32, 32, 32], 3, 2)]


@pytest.mark.parametrize("dims,ncomp,mask", CASES)
def test_probe_vectors_bit_exact(dims, ncomp, mask):
    tip = gpu_binding()
    V = int(np.prod(dims))
    P = hier_perm(dims)
    rng = np.random.default_rng(V + ncomp + mask)
    ms = sorted(set([0, 1, 2, 3, V - 1, V // 2] + [int(v) for v in rng.integers(0, V, 6)]))
    seed = 4018 + mask
    for comp in range(ncomp):
        for m in ms:
            got = tip.tip_probe_vectors(dims, ncomp, mask, seed, m, 1, comp)[0].cpu().numpy()
            want = rhs(dims, ncomp, m, comp, seed, mask, P)[:, comp]
            assert np.array_equal(got, want), (m, comp)
    # a contiguous range in one call equals single calls
    many = tip.tip_probe_vectors(dims, ncomp, mask, seed, 0, min(V, 8), 0).cpu().numpy()
    for m in range(min(V, 8)):
        assert np.array_equal(many[m], rhs(dims, ncomp, m, 0, seed, mask, P)[:, 0])


def test_probe_vectors_rejects_bad_range():
    tip = gpu_binding()
    with pytest.raises(tip.TipError):
        tip.tip_probe_vectors([4, 4], 1, 1, 1, 10, 10, 0)
