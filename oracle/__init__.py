"""Plain FP64 CPU oracle for symmetric block-sparse tensor contraction.

TEST INFRASTRUCTURE ONLY.  Nothing in the library path imports, calls or links
this package; only the tests, the smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the HIP library: the two agree only through
the conventions stated in ``workloads`` (leg spectra, canonical block order).

Modules
  su2        Clebsch-Gordan coefficients, 6j symbols, recoupling F and swap R,
             omega / cup / cap, spin generators and group elements, all from the
             closed formulas (exact rationals, rounded to FP64 at the end).
  tensors    leg bases, allowed-block enumeration (U(1) charge rule, SU(2)
             triangle rule), dense reconstruction and block extraction.
  contract   dense contraction (numpy einsum, no BLAS reordering), pairwise
             block contraction, per-sector FP64 contraction, sampled entries.
  recouple   the SU(2) F-move + swap on reduced blocks, and the 6j-free route
             (permute the dense tensor, project on the new structural tensors).
  grad       the bilinear loss, its analytic block gradients, finite differences.
  invariance brute-force check of the invariance condition under random
             group elements.

Parity status: every function is pinned by a test under ``tests/`` that checks
it against the paper's printed values, closed forms, a library special case
(sympy's exact Wigner symbols) or brute force on tiny inputs.
"""
