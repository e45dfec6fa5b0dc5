"""Hadamard matrices and the hierarchical probing basis (test infrastructure only).

* eq. HadamardElements: H_N(i, j) = (-1)^{sum_k i_k j_k} over the binary
  digits of the 0-based row and column indices; H_{2n} = H_2 (x) H_n.
* eq. Hperm-recursive: Z~(1) = H_2, Z~(k) = [Z~(k-1) (x) H_2(:,1),
  Z~(k-1) (x) H_2(:,2)], Z(k) = Z~(k) (x) 1_{N/2^k}.
* eq. HpermSequence: the columns of Z(log2 N), as columns of H_N, are
  0, N/2, N/4, 3N/4, N/8, 5N/8, 3N/8, 7N/8, ...
"""

import numpy as np

H2 = np.array([[1, 1], [1, -1]], dtype=np.int64)


def hadamard_kron(N):
    """H_N by the recursion H_{2n} = H_2 (x) H_n (Sec. 1.1.4)."""
    H = np.ones((1, 1), dtype=np.int64)
    while H.shape[0] < N:
        H = np.kron(H2, H)
    if H.shape[0] != N:
        raise ValueError("N must be a power of two")
    return H


def hadamard_element(i, j):
    """eq. HadamardElements with 0-based i, j: (-1)^{popcount(i AND j)}.
    Works elementwise on integer numpy arrays."""
    i = np.asarray(i, dtype=np.uint64)
    j = np.asarray(j, dtype=np.uint64)
    a = i & j
    par = np.zeros(np.broadcast(i, j).shape, dtype=np.uint64)
    while np.any(a):
        par ^= a & np.uint64(1)
        a = a >> np.uint64(1)
    return 1 - 2 * par.astype(np.int64)


def probing_basis_recursive(N):
    """Z(log2 N) built literally from eq. Hperm-recursive ([N, N] of +-1)."""
    Zt = H2.copy()
    k = 1
    while 2 ** k < N:
        Zt = np.hstack([np.kron(Zt, H2[:, [0]]), np.kron(Zt, H2[:, [1]])])
        k += 1
    if 2 ** k != N:
        raise ValueError("N must be a power of two >= 2")
    return Zt  # Z(log2 N) = Z~(log2 N) (x) 1_1


def probing_basis_level(N, k):
    """Z(k) = Z~(k) (x) 1_{N/2^k}: the 2^k vectors of the first k levels."""
    Zt = H2.copy()
    for _ in range(1, k):
        Zt = np.hstack([np.kron(Zt, H2[:, [0]]), np.kron(Zt, H2[:, [1]])])
    return np.kron(Zt, np.ones((N // 2 ** k, 1), dtype=np.int64))


def hperm_from_basis(N):
    """Hperm read off eq. Hperm-recursive: the index of the column of H_N that
    equals each column of Z(log2 N)."""
    H = hadamard_kron(N)
    Z = probing_basis_recursive(N)
    cols = []
    for m in range(N):
        match = np.nonzero(np.all(H == Z[:, [m]], axis=0))[0]
        assert len(match) == 1
        cols.append(int(match[0]))
    return cols


def hperm(m, L):
    """Column of H_{2^L} used by probing vector m (eq. HpermSequence).

    The sequence 0, N/2, N/4, 3N/4, N/8, 5N/8, ... is the L-bit reversal of m:
    vector m = 2^{t-1} + r (0 <= r < 2^{t-1}) of level t takes column
    (N/2^t)(2 bitrev_{t-1}(r) + 1).  Written here as that level rule.
    """
    m = int(m)
    if m == 0:
        return 0
    t = m.bit_length()                 # level of vector m
    r = m - 2 ** (t - 1)
    rev = 0
    for b in range(t - 1):             # bitrev_{t-1}(r)
        if (r >> b) & 1:
            rev |= 1 << (t - 2 - b)
    return (2 ** L // 2 ** t) * (2 * rev + 1)
