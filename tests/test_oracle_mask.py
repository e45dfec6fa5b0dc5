"""Pins for the bias-removing mask z0 (Sec. 4, eq. removebias) and its generator."""

import numpy as np
import pytest

from conftest import read_golden
from oracle import hadamard as hd
from oracle import mask as mk


def test_splitmix64_known_answers():
    want = [r[0] for r in read_golden("splitmix64_seed1234567.txt")]
    g = mk.SplitMix64(1234567)
    assert [g.next() for _ in range(5)] == want
    assert [int(v) for v in mk.splitmix64_at(1234567, np.arange(5))] == want


@pytest.mark.parametrize("seed", [0, 1, 4018, 2 ** 64 - 1, 0x123456789ABCDEF])
def test_counter_form_equals_sequential_generator(seed):
    g = mk.SplitMix64(seed)
    seq = [g.next() for _ in range(300)]
    assert [int(v) for v in mk.splitmix64_at(seed, np.arange(300))] == seq


def test_mask_layout_uses_site_times_ncomp_plus_c():
    seed, V, nc = 4018, 50, 3
    raw = [int(v) for v in mk.splitmix64_at(seed, np.arange(V * nc))]
    for c in range(nc):
        z2 = mk.mask_values(seed, V, nc, c, mk.MASK_Z2)
        z4 = mk.mask_values(seed, V, nc, c, mk.MASK_Z4)
        for s in range(V):
            u = raw[s * nc + c]
            assert z2[s] == (1 if (u >> 63) == 0 else -1)
            assert z4[s] == [1, 1j, -1, -1j][u >> 62]


def test_mask_statistics():
    V = 1 << 16
    z2 = mk.mask_values(7, V, 1, 0, mk.MASK_Z2).real
    assert set(np.unique(z2)) == {-1.0, 1.0}
    assert abs(z2.mean()) < 5 / np.sqrt(V)
    z4 = mk.mask_values(7, V, 3, 2, mk.MASK_Z4)
    counts = [np.sum(z4 == v) for v in (1, 1j, -1, -1j)]
    assert all(abs(c - V / 4) < 5 * np.sqrt(V * 3 / 16) for c in counts)
    assert np.all(np.abs(z4) == 1)
    assert np.all(mk.mask_values(7, 10, 1, 0, mk.MASK_NONE) == 1)


@pytest.mark.parametrize("kind", [mk.MASK_Z2, mk.MASK_Z4])
def test_bias_removal_keeps_gram_and_pattern(kind):
    """eq. removebias: V = z0 .* Z has V^H V = Z^H Z and V V^H = (z0 z0^H) .* Z Z^H."""
    N = 32
    Z = hd.hadamard_kron(N)[:, [hd.hperm(m, 5) for m in range(8)]].astype(np.complex128)
    z0 = mk.mask_values(99, N, 1, 0, kind)
    Vm = z0[:, None] * Z
    assert np.allclose(Vm.conj().T @ Vm, Z.conj().T @ Z, atol=0)
    assert np.allclose(Vm @ Vm.conj().T, np.outer(z0, z0.conj()) * (Z @ Z.conj().T), atol=0)
