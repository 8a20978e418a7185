"""Writes cg256_rho.txt: the oracle's conjugate-gradient residual history
rho_k = r_k . r_k, k = 0..500, on the 256^3 7-point Poisson system with the
right-hand side of seed 2002 (the CG workload of the paper's sparse Krylov
benchmark at its measured size), x0 = 0.  Calls only the oracle and the
seeded input generator.  Run from the repository root:

    python tests/golden/make_cg256_rho.py

(about half an hour of one CPU core)."""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import cnum  # noqa: E402
from oracle import workloads as wl  # noqa: E402

M, ITERS = 256, 500
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cg256_rho.txt")


def main():
    cnum.build()
    rowptr, col, val = synth.poisson_csr(M, 3)
    b = synth.rhs(M ** 3, synth.CG256_SEED)
    t0 = time.time()
    _, hist = wl.cg(rowptr, col, val, b, ITERS)
    with open(OUT, "w") as fh:
        fh.write("# rho_k = r_k.r_k of CG on the 256^3 7-point Poisson matrix, b = synth.rhs(256**3, 2002),\n")
        fh.write("# x0 = 0, k = 0..%d, from oracle.workloads.cg (exactly rounded dot products);\n" % ITERS)
        fh.write("# written by tests/golden/make_cg256_rho.py in %.0f s\n" % (time.time() - t0))
        for v in hist:
            fh.write(repr(float(v)) + "\n")


if __name__ == "__main__":
    main()
