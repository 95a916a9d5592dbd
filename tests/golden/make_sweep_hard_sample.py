"""Write tests/golden/sweep_hard_job.npz: the FP64 oracle's transmitted field
(8 planes of 64x64) of a hard spectral-sweep job, patch 2 (truncation 21x21,
M = 441, 16 layers) at 1000 cm^-1 (lambda = 10 um), where the growth exponent
of the connection product is about 42: the paper's reduced route (the K
product of Eq. 27) loses its accuracy there, so the reference is the full
boundary system of Eqs. 24-26 (30,870 unknowns), solved densely by LU. The
reduced route's error against it is stored too, as evidence of the
instability. Calls only oracle/ and workloads/; a few minutes on 8 cores and
about 32 GB of memory.

    python tests/golden/make_sweep_hard_sample.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import cwt  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sweep_hard_job.npz")
PATCH = 2
NU_INDEX = 0


def main():
    jobs = W.spectral_sweep_jobs()
    nus = sorted(set(j[0] for j in jobs))
    U = [j[2] for j in jobs if j[1] == PATCH][0]
    prob, grid = W.sweep_problem(nus[NU_INDEX], PATCH, U)
    t0 = time.time()
    st = cwt.setup(prob)
    print("setup %.0f s" % (time.time() - t0), flush=True)
    sol = cwt.solve_unreduced(st, dense_limit=40000)
    print("full system %.0f s" % (time.time() - t0), flush=True)
    red = cwt.solve(st, "reduced")
    err_red = float(np.linalg.norm(red.p_trn - sol.p_trn) / np.linalg.norm(sol.p_trn))
    print("reduced route rel-L2 %.3e" % err_red, flush=True)
    E = cwt.synthesize(st, sol, grid)
    np.savez_compressed(OUT, E=E, patch=PATCH, nu_index=NU_INDEX, nu=nus[NU_INDEX], U=U,
                        p_trn=sol.p_trn, p_ref=sol.p_ref, reduced_route_rel_l2=err_red)
    print("wrote %s (%.0f s)" % (OUT, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
