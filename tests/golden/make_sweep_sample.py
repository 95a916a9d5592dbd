"""Write tests/golden/sweep_job.npz: the FP64 oracle's transmitted field (8
planes of 64x64) of one spectral-sweep job, patch 8 (truncation 9x9) at the
129th of the 256 wavenumbers (the wavenumber bench.py solves that patch at),
using the full boundary system. Calls only oracle/ and workloads/.

    python tests/golden/make_sweep_sample.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import cwt  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sweep_job.npz")
PATCH = 8
NU_INDEX = 128


def main():
    jobs = W.spectral_sweep_jobs()
    nus = sorted(set(j[0] for j in jobs))
    U = [j[2] for j in jobs if j[1] == PATCH][0]
    prob, grid = W.sweep_problem(nus[NU_INDEX], PATCH, U)
    st = cwt.setup(prob)
    sol = cwt.solve(st, "unreduced")
    E = cwt.synthesize(st, sol, grid)
    np.savez_compressed(OUT, E=E, patch=PATCH, nu_index=NU_INDEX, nu=nus[NU_INDEX], U=U,
                        p_trn=sol.p_trn)
    print("wrote", OUT, E.shape)


if __name__ == "__main__":
    main()
