"""Plain FP64 CPU oracle for hierarchical probing of Tr(A^-1) on toroidal lattices.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP path; both sides are
fed the same seeded inputs by ``paper_1302_4018_amd.inputs`` (which holds none
of the method's arithmetic) and the oracle re-derives everything else from the
paper (Stathopoulos, Laeuchli, Orginos, "Hierarchical probing for estimating
the trace of the matrix inverse on toroidal lattices", arXiv:1302.4018).

Modules, in the order the method uses them:

* ``lattice``   -- site numbering, per-level active dimensions (Sec. 3.3).
* ``hierperm``  -- Red-Black orders (Alg. 2, Alg. 3, Lemmas 3.1-3.3, Theorem
                   of Sec. 3.3) and the hierarchical lattice permutation
                   (Alg. 4, Alg. 5; 1-D bit reversal of Sec. 3).
* ``hadamard``  -- Hadamard matrices (eq. HadamardElements), the probing-basis
                   recursion (eq. Hperm-recursive) and its column order
                   (eq. HpermSequence).
* ``mask``      -- the random vector z0 of Sec. 4 (eq. removebias), drawn from
                   SplitMix64 (Steele, Lea & Flood, OOPSLA 2014).
* ``probing``   -- probing vectors z_m(i) = H(iperm(i), Hperm(m))
                   (eq. row-col-permutation), masked and colour-diluted.
* ``operators`` -- the shifted lattice Laplacians (Sec. 5 control problem and
                   the covariant 3-component variant).
* ``cg``        -- the linear solves that give the quadratures (Sec. 1.1.2).
* ``estimator`` -- the MC/probing estimator (1/s) sum_m z_m^H A^-1 z_m
                   (Sec. 1, Hutchinson) reported at s = 2^k.
* ``exact``     -- exact values used to pin the above: dense LU traces,
                   closed-form Fourier eigenvalue sums, FFT solves.
"""
