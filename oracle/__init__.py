"""CPU oracle for the fused task-stream executor -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import, call, link or run anything in this package.  The product path (the
HIP library and its Python binding) never does, and this package imports
nothing from the product: the two share only the seeded input generators in
`synth`, which hold no arithmetic of the method.

Contents (every function cites the passage of the paper it follows):
  ir         the IR of section 3: stores, projections, None/Tiling/Image
             partitions, privileges, index tasks, sub-stores
  analysis   Definition 1, dependence maps, fusibility, the four fusion
             constraints of section 4.2, the temporary-store definition of
             section 5.1 and the canonical form of section 5.2, all by
             explicit enumeration (tiny inputs)
  stream     unfused op-by-op FP64 evaluation of a task stream
  workloads  the Black-Scholes, Jacobi-stencil and CG computations of
             sections 2 and 7 written out directly
  cnum       plain C (gcc -O2 -ffp-contract=off): libm loops, sequential CSR
             SpMV, exactly rounded sums

Pins (tests/test_oracle_*.py) tie it to values fixed independently of this
code: put-call parity, 40-digit mpmath prices, discrete harmonic fixed points,
exact rational CG, SciPy's solvers, the paper's worked examples.
"""
