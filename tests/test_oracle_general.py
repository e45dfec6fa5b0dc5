"""Pins for the probes of tori with sides that are not powers of two
(oracle/general.py): the three-colouring theorem of Sec. 3.4, the level
schedule, reduction to the power-of-two generator, the probing property of
the whole colouring, and the partial-sum identity with sweeps."""

import itertools

import numpy as np
import pytest

from oracle import general, mask
from oracle.lattice import coordinates, site_index, torus_distance, volume
from oracle.operators import Operator
from oracle.probing import rhs as rhs_pow2
from paper_1302_4018_amd import inputs


def _neighbour_pairs(dims):
    X = coordinates(dims)
    s = np.arange(volume(dims))
    for j, n in enumerate(dims):
        if n == 1:
            continue
        Y = X.copy()
        Y[:, j] = (Y[:, j] + 1) % n
        yield s, site_index(Y, dims)


@pytest.mark.parametrize("dims", [[5, 5], [7], [3, 3, 3], [7, 4], [5, 9, 2], [13, 6], [2, 3], [10, 7, 3]])
def test_three_colouring_has_no_conflicts(dims):
    C = general.three_colouring(coordinates(dims), dims)
    assert set(np.unique(C)) <= {0, 1, 2}
    for a, b in _neighbour_pairs(dims):
        assert np.all(C[a] != C[b]), dims


def test_three_colouring_5x5_class_sizes():
    C = general.three_colouring(coordinates([5, 5]), [5, 5])
    assert sorted(np.bincount(C).tolist()) == [8, 8, 9]


@pytest.mark.parametrize("dims,B,LB,has3,gamma", [
    ([6, 4], 1, 2, True, 12),
    ([12, 5, 8], 0, 0, True, 3),
    ([24, 6, 10], 1, 3, True, 24),
    ([12, 12], 2, 4, True, 48),
    ([8, 4, 2], 3, 6, False, 64),
    ([48, 8], 4, 7, True, 384),           # level 4 subdivides only the side of 48 (6 left)
])
def test_level_schedule(dims, B, LB, has3, gamma):
    lv = general.Levels(dims)
    assert (lv.B, lv.LB, lv.has3, lv.gamma) == (B, LB, has3, gamma)


@pytest.mark.parametrize("dims,ncomp,mk", [([4, 8], 1, mask.MASK_Z2), ([2, 4, 2], 3, mask.MASK_Z4),
                                           ([8], 1, mask.MASK_NONE), ([4, 2, 2, 2], 3, mask.MASK_Z4)])
def test_power_of_two_sides_reduce_to_alg5(dims, ncomp, mk):
    V = volume(dims)
    for m in range(V):
        for c in range(ncomp):
            assert np.array_equal(general.rhs(dims, ncomp, m, c, 11, mk), rhs_pow2(dims, ncomp, m, c, 11, mk))


@pytest.mark.parametrize("dims", [[6, 4], [12, 5, 8], [6, 6], [10, 2, 6], [3, 3, 3]])
def test_whole_colouring_is_a_probing_colouring(dims):
    """Sites sharing the colour (P_B, C) are not neighbours, and the gamma
    columns of one sweep satisfy sum_j z_j(x) conj(z_j(y)) = gamma [same colour]."""
    lv = general.Levels(dims)
    PB = general.binary_colour(dims, lv).astype(np.int64)
    C = general.last_level_colour(dims, lv)
    col = PB * 3 + C
    for a, b in _neighbour_pairs(dims):
        assert np.all(col[a] != col[b])
    Z = np.stack([general.probe(dims, j, lv)[0] for j in range(lv.gamma)], axis=1)
    G = Z @ Z.conj().T
    same = col[:, None] == col[None, :]
    assert np.allclose(G, lv.gamma * same, atol=1e-12)


def test_binary_levels_separate_sites_by_distance():
    """After the binary levels (L_B bits) of 12 x 12, same-colour sites are at
    least 2^B = 4 apart, as on the conformal sub-lattice of Sec. 3."""
    dims = [12, 12]
    lv = general.Levels(dims)
    PB = general.binary_colour(dims, lv).astype(np.int64)
    X = coordinates(dims)
    for a, b in itertools.combinations(range(volume(dims)), 2):
        if PB[a] == PB[b]:
            assert torus_distance(X[a], X[b], dims) >= 2 ** lv.B


@pytest.mark.parametrize("dims,kind,mk", [([6, 4], 0, mask.MASK_Z2), ([3, 6, 2], 1, mask.MASK_Z4),
                                          ([5, 3], 0, mask.MASK_Z4)])
def test_partial_sum_identity_over_two_sweeps(dims, kind, mk):
    """T at s = gamma (one sweep) equals the sum of masked A^-1 entries over
    same-colour pairs, and T at s = 2 gamma is the mean of two such sweeps
    with independent masks (probes computed here by dense solves, no CG)."""
    lv = general.Levels(dims)
    V = volume(dims)
    U = inputs.haar_links(dims, seed=60) if kind == 1 else None
    op = Operator(dims, kind, mass=0.4, coupling=inputs.couplings(dims, seed=61), links=U)
    Ainv = np.linalg.inv(op.dense())
    nc = op.ncomp
    PB = general.binary_colour(dims, lv).astype(np.int64)
    C = general.last_level_colour(dims, lv)
    same = (PB * 3 + C)[:, None] == (PB * 3 + C)[None, :]
    n = min(2 * lv.gamma, V)
    q = []
    for m in range(n):
        qm = 0.0
        for c in range(nc):
            b = general.rhs(dims, nc, m, c, 5, mk, lv).reshape(-1)
            qm += np.vdot(b, Ainv @ b)
        q.append(qm)
    ident = []
    for r in range(n // lv.gamma):
        tot = 0.0
        for c in range(nc):
            z0 = general.mask_sweep(5, V, nc, c, mk, r)
            idx = np.arange(V) * nc + c
            blk = Ainv[np.ix_(idx, idx)]
            tot += np.sum((np.conj(z0)[:, None] * blk * z0[None, :])[same])
        ident.append(tot)
    assert abs(np.mean(q[:lv.gamma]) - ident[0]) <= 1e-12 * abs(ident[0])
    if len(ident) == 2:
        assert abs(np.mean(q[:2 * lv.gamma]) - np.mean(ident)) <= 1e-12 * abs(ident[0])


def test_omega3_is_a_cube_root_of_unity():
    w = general.OMEGA3
    assert w[0] == 1 and w[2] == np.conj(w[1])
    assert abs(w[1] ** 3 - 1) < 1e-15 and abs(1 + w[1] + w[2]) < 1e-15


def test_general_estimator_matches_the_identity_on_a_3x3_torus():
    """3 x 3: no binary level and gamma = 3 colours of 3 sites each; the
    estimate after the three F_3 columns, with CG solves, equals the sum of
    masked A^-1 entries over same-colour pairs."""
    dims = [3, 3]
    op = Operator(dims, 0, mass=0.5)
    est, q, _ = general.trace_inv_probe(op, 3, 1e-13, 2, mask.MASK_Z2)
    lv = general.Levels(dims)
    C = general.last_level_colour(dims, lv)
    Ainv = np.linalg.inv(op.dense())
    z0 = general.mask_sweep(2, 9, 1, 0, mask.MASK_Z2, 0)
    same = C[:, None] == C[None, :]
    ident = np.sum((np.conj(z0)[:, None] * Ainv * z0[None, :])[same])
    assert abs(est[-1] - ident) <= 1e-11 * abs(ident)
