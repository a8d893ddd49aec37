"""Plain, slow CPU oracle for the divide-and-conquer sector index and the matrix-free H*x.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check of the package entry
file and the bench's CPU-baseline leg may import or run anything in this
package.  The GPU library never calls into it, and it never calls into the GPU
library: the two share no code, no tables and no helpers.  The only shared
module is ``synth`` (seeded inputs, no arithmetic of the method).

Source: R. Schaefer and D. J. Luitz, "DanceQ: High-performance library for
number-conserving bases", SciPost Phys. Codebases 48 (2025), arXiv:2407.14591.

Contents
  sector.py       sector dimension (App. A), canonical order by brute-force sort
                  (Sec. 3.1-3.2), closed-form offsets/strides (eq. offset,
                  eq. stride), rank (Alg. i), increment (Alg. ii), unrank (Alg. iii),
                  the on-the-fly limit (Alg. on-the-fly), Cover's rank (eq. cover)
  hamiltonian.py  XXZ matrix elements, H*x by definition, dense sector and full
                  Q^L matrices (eq. H_30, App. D)
  lanczos.py      FP64 Lanczos with full re-orthogonalisation (Sec. 2.1 names it)
  gradients.py    adjoint of y = H(theta) x and the Hellmann-Feynman gradient
  observables.py  lowest few Ritz pairs and expectation values of the terms of H
                  (App. D)
  operators.py    generic number-conserving local operators (Sec. 4.1 operator
                  strings, App. C terms): y = O x term by term, and the operator on
                  the whole Q^L space from tensor contractions
  mixed.py        sectors and local operators on sites of different local
                  dimensions (Sec. 5's generalisation): dimension from the
                  generating function, order by brute-force sort, y = O x term by term
  native.py       ctypes loader of c/dcs_oracle.c (same definitions in plain C,
                  FP64, OpenMP) for sectors too large for Python

Everything floating point is FP64; everything integer is exact (Python ints or
uint64).  Pins of every function against values the paper prints, closed forms
and brute force live in tests/test_oracle_*.py.
"""
