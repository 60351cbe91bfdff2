"""Write the FP64 oracle solution of the 32^3x64 Wilson-clover system at
sampled sites (tests/golden/wilson_solution_32x64_sites.npz).

System: links U = exp(i eps H) with eps = 0.25 (seed 2001), kappa = 0.124,
c_sw = 1, antiperiodic in time, one Gaussian source (seed 2002); the even-odd
Schur system (Section III-A) solved by the oracle's CGNE to ||r|| <= 1e-12
||bhat||, the odd sites reconstructed. Only the oracle and the input
generator are called. The file holds the solution at 2048 sites drawn with
seed 11 (both parities), the sites, the iteration count and the final
FP64 residual ||b - M x|| / ||b|| over the whole lattice.

About 200 iterations of two Schur applications each: some 10 minutes on 8
host cores.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import solvers  # noqa: E402

DIMS, EPS, KAPPA, CSW = (32, 32, 32, 64), 0.25, 0.124, 1.0
OUT = os.path.join(HERE, "wilson_solution_32x64_sites.npz")


def main():
    t0 = time.time()
    U = synth.gauge_field(DIMS, EPS, 2001)
    b = synth.gaussian_spinor(DIMS, 2002)
    op = oracle.WilsonClover(DIMS, U, KAPPA, CSW, bc_t=-1)
    bhat = op.schur_source(b)
    print("fields and clover %.0f s" % (time.time() - t0), flush=True)
    xe, it, hist = solvers.cgne(op.schur, lambda v: op.schur(v, dagger=True), bhat, tol=1e-12)
    x = op.reconstruct(xe, b)
    res = float(np.linalg.norm(b - op.M(x)) / np.linalg.norm(b))
    print("CGNE %d iterations, residual %.3e, %.0f s" % (it, res, time.time() - t0), flush=True)
    rng = np.random.default_rng(11)
    V = int(np.prod(DIMS))
    sites = np.sort(rng.choice(V, size=2048, replace=False))
    np.savez(OUT, sites=sites, x=x.reshape(V, 4, 3)[sites], iterations=it, residual=res)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
