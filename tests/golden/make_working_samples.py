"""Write tests/golden/working_samples.npz: FP64 oracle values of the E field at
4096 seeded voxels of the 64x64x32 random-field workload (M = 441, grid
256x256x128), used by the GPU parity test at full size and by bench.py.

The oracle runs its reduced connection route here (the full boundary system
has 59,094 unknowns); the reduced and un-reduced routes agree on smaller
stacks of this workload (tests/test_oracle_workloads.py). Calls only oracle/
and workloads/. Takes about 5-10 minutes on 8 cores.

    python tests/golden/make_working_samples.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import cwt  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "working_samples.npz")


def main():
    prob, grid = W.random_field_config("working")
    t0 = time.time()
    st = cwt.setup(prob)
    sol = cwt.solve(st, "reduced")
    print("oracle setup+solve %.0f s" % (time.time() - t0), flush=True)
    rng = np.random.Generator(np.random.PCG64(2024))
    n = 4096
    j = rng.integers(0, grid.fz, n)
    g = rng.integers(0, grid.fy, n)
    f = rng.integers(0, grid.fx, n)
    zs = grid.z_planes()
    x = f * prob.X / grid.fx
    y = g * prob.Y / grid.fy
    E = cwt.field_at_points(st, sol, x, y, zs[j])
    p_inc, p_ref, p_trn = st.p_inc, sol.p_ref, sol.p_trn
    np.savez_compressed(OUT, j=j, g=g, f=f, E=E, fx=grid.fx, fy=grid.fy, fz=grid.fz,
                        M=st.M, p_inc=p_inc, p_ref=p_ref, p_trn=p_trn)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
