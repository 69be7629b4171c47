"""CPU oracle for the CSRC sparse matrix-vector product -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It is a plain, slow, obviously correct statement of what
the GPU path computes, written from the paper (Batista, Ainsworth Jr. and
Ribeiro, "Parallel structurally-symmetric sparse matrix-vector products on
multi-core processors"):

* ``reference``  CSR -> CSRC split (Sec. 2), the sequential product from
                 the splitting A = A_D + A_L + A_U and its transpose
                 (Sec. 5) via the C library, pure-Python
                 loops for tiny cases, greedy colouring (Sec. 3.2), the
                 nnz-guided row partition and effective ranges (Sec. 3.1),
                 reduced-precision rounding and error bounds.
* ``mlp``        FP64 forward/backward of the selector network.
* ``features``   the selector's structural features, by definition.

Every function is pinned by ``tests/test_oracle_*.py`` against what the paper
and the mathematics fix (library routines, closed forms, brute force); see the
docstrings for which pins cover which function.  The oracle shares no code
with the GPU library and never calls it.
"""
