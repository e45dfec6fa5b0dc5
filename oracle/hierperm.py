"""Hierarchical permutation of a toroidal lattice (test infrastructure only).

Follows Sec. 3 of the paper step by step:

* 1-D lattices: P(x) is the bit reversal of x (Sec. 3, the binary colouring
  tree traced from root to leaf).
* Red-Black order of the 2-point d-dimensional torus: Alg. 2 (slow, counting
  one-bits) and Alg. 3 (fast, colours c_j = [c_{j-1}, not c_{j-1}]).
* Alg. 4: hierarchical permutation when all k_j are equal.
* Alg. 5: general k_j; at bit-level m only the active dimensions (m <= k_j)
  contribute, and RB for that many dimensions is read off the d-dimensional
  table by the Theorem of Sec. 3.3 (scale the index by 2^{d-a}, keep the
  leading a bits of the result).

Readings taken where the paper leaves a choice (0-based indices throughout):
bin2dec of a bit list treats the FIRST listed bit as most significant, so in
Alg. 4/5 the first (active) dimension supplies the most significant bit of the
Red-Black index, and the strings appended to ``loc`` at earlier levels end up
in more significant positions of the final location.
"""

import numpy as np

from .lattice import coordinates, log2_exact, volume


def dec2bin(value, width):
    """MATLAB dec2bin as a list of bits, most significant first."""
    return [(int(value) >> (width - 1 - t)) & 1 for t in range(width)]


def bin2dec(bits):
    """MATLAB bin2dec of a bit list, first element most significant."""
    v = 0
    for b in bits:
        v = (v << 1) | int(b)
    return v


def bitreverse_1d(x, k):
    """P(x) = bin2dec(bitreverse(dec2bin(x))) on k bits (1-D case of Sec. 3)."""
    return bin2dec(list(reversed(dec2bin(x, k))))


def rb_colors(d):
    """Alg. 3 colours of the 2-point torus: c_0 = [0], c_j = [c_{j-1}, not c_{j-1}]."""
    c = [0]
    for _ in range(d):
        c = c + [1 - v for v in c]
    return c


def rb_table_fast(d):
    """Alg. 3: RB(i) for i = 0..2^d-1; reds (colour 0) fill the first half in
    the order they are met, blacks the second half."""
    c = rb_colors(d)
    reds, blacks = 0, (2 ** (d - 1) if d > 0 else 0)
    rb = []
    for i in range(2 ** d):
        if c[i] == 0:
            rb.append(reds)
            reds += 1
        else:
            rb.append(blacks)
            blacks += 1
    return rb


def rb_table_slow(d):
    """Alg. 2: same as Alg. 3 but the colour of i is whether dec2bin(i) has an
    odd number of one-bits ("even number of bits" -> red)."""
    reds, blacks = 0, (2 ** (d - 1) if d > 0 else 0)
    rb = []
    for i in range(2 ** d):
        if sum(dec2bin(i, max(d, 1))) % 2 == 0:
            rb.append(reds)
            reds += 1
        else:
            rb.append(blacks)
            blacks += 1
    return rb


def rb_lemma(d):
    """Lemma 3.3: RB_d(i) = floor(i/2) + c_d(i) 2^{d-1}."""
    c = rb_colors(d)
    return [i // 2 + c[i] * 2 ** (d - 1) for i in range(2 ** d)]


def rb_from_larger(m, d):
    """Theorem of Sec. 3.3: RB_m(i) = floor(RB_d(i 2^{d-m}) / 2^{d-m})."""
    rbd = rb_table_fast(d)
    return [rbd[i * 2 ** (d - m)] // 2 ** (d - m) for i in range(2 ** m)]


def lattice_hier_perm0_point(x, k):
    """Alg. 4 for one point x = (x_1..x_d), every side 2^k."""
    d = len(x)
    rb = rb_table_fast(d)
    table = [list(reversed(dec2bin(xj, k))) for xj in x]   # table[j][m-1] = b^j_m
    loc = []
    for m in range(1, k + 1):
        section = [table[j][m - 1] for j in range(d)]
        loc = loc + dec2bin(rb[bin2dec(section)], d)
    return bin2dec(loc)


def lattice_hier_perm_point(x, dims):
    """Alg. 5 for one point x = (x_1..x_d) on a torus with sides dims."""
    d = len(dims)
    k = [log2_exact(n) for n in dims]
    rb = rb_table_fast(d)
    table = [list(reversed(dec2bin(x[j], k[j]))) for j in range(d)]
    loc = []
    for m in range(1, max(k) + 1):
        bits = []
        active = 0
        for j in range(d):
            if m <= k[j]:
                bits.append(table[j][m - 1])
                active += 1
        index = bin2dec(bits) * 2 ** (d - active)
        s = rb[index] // 2 ** (d - active)
        loc = loc + dec2bin(s, active)
    return bin2dec(loc)


def hier_perm(dims):
    """P(x) for every site in site order (Alg. 5, vectorised over sites only).

    Each site is independent (Sec. 3.3), so the per-point steps of Alg. 5 are
    applied to whole arrays; no step is reordered.  Returns uint64 [V].
    """
    dims = [int(n) for n in dims]
    d = len(dims)
    k = [log2_exact(n) for n in dims]
    rb = np.array(rb_table_fast(d), dtype=np.int64)
    X = coordinates(dims)
    V = volume(dims)
    loc = np.zeros(V, dtype=np.int64)
    for m in range(1, max(k) + 1):
        bits = np.zeros(V, dtype=np.int64)
        active = 0
        for j in range(d):
            if m <= k[j]:
                b = (X[:, j] >> (m - 1)) & 1          # b^j_m
                bits = (bits << 1) | b                 # bin2dec: first listed is MSB
                active += 1
        index = bits * 2 ** (d - active)
        s = rb[index] // 2 ** (d - active)
        loc = (loc << active) | s                      # append the string to loc
    return loc.astype(np.uint64)
