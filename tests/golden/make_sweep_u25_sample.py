"""Write tests/golden/sweep_u25_job.npz: the FP64 oracle's transmitted field
(8 planes of 64x64) of the widest spectral-sweep job, patch 0 (truncation
25x25, M = 625, 16 layers; the band wraps around the 32-voxel patch since
2U - 1 = 49 > 32) at 1000 cm^-1 (lambda = 10 um). The reference is the full
boundary system of Eqs. 24-26 with its 43,750 unknowns, solved by banded LU
(oracle.cwt.solve_unreduced_banded). The reduced route's error against it is
stored too. Calls only oracle/ and workloads/; about ten minutes on 8 cores
and 15 GB of memory.

    python tests/golden/make_sweep_u25_sample.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import cwt  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sweep_u25_job.npz")
PATCH = 0
NU_INDEX = 0


def main():
    jobs = W.spectral_sweep_jobs()
    nus = sorted(set(j[0] for j in jobs))
    U = [j[2] for j in jobs if j[1] == PATCH][0]
    assert U == 25
    prob, grid = W.sweep_problem(nus[NU_INDEX], PATCH, U)
    t0 = time.time()
    st = cwt.setup(prob)
    print("setup %.0f s" % (time.time() - t0), flush=True)
    sol = cwt.solve_unreduced_banded(st)
    print("banded full system %.0f s" % (time.time() - t0), flush=True)
    red = cwt.solve(st, "reduced")
    err_red = float(np.linalg.norm(red.p_trn - sol.p_trn) / np.linalg.norm(sol.p_trn))
    print("reduced route rel-L2 %.3e" % err_red, flush=True)
    E = cwt.synthesize(st, sol, grid)
    np.savez_compressed(OUT, E=E, patch=PATCH, nu_index=NU_INDEX, nu=nus[NU_INDEX], U=U,
                        p_trn=sol.p_trn, p_ref=sol.p_ref, reduced_route_rel_l2=err_red)
    print("wrote %s (%.0f s)" % (OUT, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
