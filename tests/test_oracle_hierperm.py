"""Pins for the oracle's hierarchical permutation (Sec. 3 of the paper).

Each pin comes from the paper's worked examples, its lemmas and theorem, or
from brute force on small tori; none re-types the oracle's own formula.
"""

import itertools

import numpy as np
import pytest

from conftest import read_golden
from oracle import hierperm as hp
from oracle import lattice as lat


def test_rb2_is_the_papers_order_00_11_01_10():
    rows = read_golden("rb2_order.txt")
    rb = hp.rb_table_fast(2)
    for pos, bits in enumerate(rows):
        assert rb[hp.bin2dec(bits)] == pos
    assert hp.rb_table_slow(2) == rb


def test_c2_colors_from_lemma_3_1_proof():
    assert hp.rb_colors(2) == read_golden("c2_colors.txt")[0]


@pytest.mark.parametrize("d", range(1, 7))
def test_alg2_alg3_lemma_and_theorem_agree(d):
    fast = hp.rb_table_fast(d)
    assert hp.rb_table_slow(d) == fast                       # Alg. 2 == Alg. 3
    assert hp.rb_lemma(d) == fast                            # Lemma 3.3
    assert sorted(fast) == list(range(2 ** d))               # a permutation
    for m in range(1, d):
        assert hp.rb_from_larger(m, d) == hp.rb_table_fast(m)  # Theorem, Sec. 3.3


@pytest.mark.parametrize("d", range(1, 7))
def test_colour_lemmas_and_neighbour_property(d):
    c = hp.rb_colors(d)
    for i in range(2 ** (d - 1)):
        assert c[2 * i] == hp.rb_colors(d - 1)[i]            # Lemma 3.1
        assert c[2 * i] != c[2 * i + 1]                      # Lemma 3.2
    # every point of the 2-point torus has neighbours of the opposite colour
    for i in range(2 ** d):
        for j in range(d):
            assert c[i] != c[i ^ (1 << j)]
    # reds come first: positions < 2^{d-1} hold exactly the colour-0 points
    rb = hp.rb_table_fast(d)
    for i in range(2 ** d):
        assert (rb[i] < 2 ** (d - 1)) == (c[i] == 0)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_1d_permutation_is_the_binary_tree_order(k):
    """Sec. 3: split by b_1, then b_2, ...; P(x) is x's rank in that order."""
    N = 2 ** k
    key = lambda x: [(x >> t) & 1 for t in range(k)]        # (b_1, b_2, ..., b_k)
    order = sorted(range(N), key=key)
    P_tree = np.empty(N, dtype=np.int64)
    P_tree[order] = np.arange(N)
    P = hp.hier_perm([N]).astype(np.int64)
    assert np.array_equal(P, P_tree)
    assert all(hp.bitreverse_1d(x, k) == P[x] for x in range(N))


SHAPES = [[4, 4], [8, 8], [4, 4, 4], [2, 2, 2, 2], [4, 2, 8], [8, 4, 2], [2, 8],
          [4, 4, 2, 2], [2, 4, 8, 2], [16], [1, 4], [4, 1, 2], [2, 2]]


@pytest.mark.parametrize("dims", SHAPES)
def test_alg5_vectorised_equals_pointwise_and_is_bijection(dims):
    P = hp.hier_perm(dims).astype(np.int64)
    X = lat.coordinates(dims)
    for s in range(len(P)):
        assert P[s] == hp.lattice_hier_perm_point(list(X[s]), dims)
    assert np.array_equal(np.sort(P), np.arange(len(P)))


@pytest.mark.parametrize("dims", [[4, 4], [8, 8, 8], [2, 2, 2, 2], [4, 4, 4, 4]])
def test_alg4_equals_alg5_for_equal_sides(dims):
    k = lat.log2_exact(dims[0])
    P = hp.hier_perm(dims).astype(np.int64)
    X = lat.coordinates(dims)
    for s in range(len(P)):
        assert P[s] == hp.lattice_hier_perm0_point(list(X[s]), k)


def _classes(P, L, t):
    return (P.astype(np.int64) >> (L - t))


@pytest.mark.parametrize("dims", [[8, 8], [4, 8, 2], [8, 4, 4], [4, 4, 4, 4], [2, 4, 2, 8]])
def test_levels_split_into_conformal_sublattices_then_red_black(dims):
    """Sec. 3.1: after bit-levels 1..m the colour classes are the conformal
    sublattices (low min(m, k_j) bits of every coordinate fixed); one more bit
    red-blacks each sublattice by the parity of its next coordinate bits."""
    P = hp.hier_perm(dims)
    L = lat.total_levels(dims)
    X = lat.coordinates(dims)
    k = [lat.log2_exact(n) for n in dims]
    t = 0
    for m in range(1, max(k) + 1):
        sub = np.zeros(len(P), dtype=np.int64)
        for j in range(len(dims)):
            sub = sub * dims[j] + (X[:, j] % (2 ** min(m - 1, k[j])))
        par = np.zeros(len(P), dtype=np.int64)
        for j in range(len(dims)):
            if m <= k[j]:
                par ^= (X[:, j] >> (m - 1)) & 1
        # classes at t bits == sublattices of level m-1
        _same_partition(_classes(P, L, t) if t > 0 else np.zeros(len(P), np.int64), sub)
        # classes at t + 1 bits == sublattice x red/black colour
        _same_partition(_classes(P, L, t + 1), sub * 2 + par)
        t += len([j for j in range(len(dims)) if m <= k[j]])
    assert t == L


def _same_partition(a, b):
    pairs = set(zip(a.tolist(), b.tolist()))
    assert len(pairs) == len(set(a.tolist())) == len(set(b.tolist()))


def _min_same_class_distance(X, dims, cls):
    best = np.inf
    for c in np.unique(cls):
        pts = X[cls == c]
        if len(pts) < 2:
            continue
        for i in range(len(pts) - 1):
            d = lat.torus_distance(pts[i], pts[i + 1:], dims)
            best = min(best, int(d.min()))
    return best


@pytest.mark.parametrize("dims", [[16, 16], [8, 8, 8], [4, 4, 4, 4], [16, 4, 8], [4, 8, 2, 4]])
def test_distance_2m_colouring_brute_force(dims):
    """Sec. 3.3: when level m completes (t = sum_{l<=m} a_l + 1 bits), sites of
    one colour are at least 2^{m+1} apart, i.e. a distance-2^m colouring;
    before the extra bit they are at least 2^m apart."""
    P = hp.hier_perm(dims)
    L = lat.total_levels(dims)
    X = lat.coordinates(dims)
    k = [lat.log2_exact(n) for n in dims]
    t = 0
    for m in range(0, max(k)):
        a_next = len([j for j in range(len(dims)) if m + 1 <= k[j]])
        if t > 0:
            assert _min_same_class_distance(X, dims, _classes(P, L, t)) >= 2 ** m
        dist = _min_same_class_distance(X, dims, _classes(P, L, t + 1))
        assert dist >= 2 ** (m + 1)
        # where the torus is wide enough the bound is attained
        if all(n >= 2 ** (m + 2) for n in dims) and len(dims) >= 2:
            assert dist == 2 ** (m + 1)
        t += a_next


def test_4d_completion_points_2_32_512():
    """Sec. 3.3 / Sec. 5.3: 2^{dm+1} colours complete a distance-2^m colouring;
    in 4-D those are s = 2, 32, 512."""
    dims = [8, 8, 8, 8]
    a = [len(x) for x in lat.active_dims(dims)]
    points = [2 ** (sum(a[:m]) + 1) for m in range(len(a))]
    assert points == [2, 32, 512]
    P = hp.hier_perm(dims)
    L = lat.total_levels(dims)
    X = lat.coordinates(dims)
    for m, s in enumerate(points):
        t = int(np.log2(s))
        assert _min_same_class_distance(X, dims, _classes(P, L, t)) == 2 ** (m + 1)
    # one bit short of a completion point the distance has not doubled yet
    assert _min_same_class_distance(X, dims, _classes(P, L, 4)) == 2


def test_level_table():
    assert [len(a) for a in lat.active_dims([32, 32, 32, 32])] == [4] * 5
    assert [len(a) for a in lat.active_dims([16, 16])] == [2] * 4
    assert lat.active_dims([4, 2, 8]) == [[0, 1, 2], [0, 2], [2]]
    assert lat.total_levels([32, 32, 32, 32]) == 20
    with pytest.raises(ValueError):
        lat.log2_exact(12)
