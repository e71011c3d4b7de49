"""Plain FP64 CPU oracle of spaND with the first-order, full second-order and
superfine second-order sparsification schemes.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or runs this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code with the GPU path: the only common module is
``synthetic`` (seeded input generators, none of the method's arithmetic).

Layout:

* ``nd``    - geometric nested dissection, vertex paths, clusters per step,
              block adjacency with symbolic fill, greedy interface colouring.
* ``dense`` - the early-stopping column-pivoted Householder QR (Alg. 1).
* ``spand`` - the level-by-level factorization (Alg. 2), the apply of
              ``M = L^{-T} L^{-1}`` and the memory/flop counters.
* ``pcg``   - preconditioned conjugate gradients (Sec. 4 protocol).

Readings of the paper where it is silent or garbled are listed in the module
docstrings where they are applied.
"""
