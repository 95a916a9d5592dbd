"""Write tests/golden/large_samples.npz: FP64 oracle values of the E field at
4096 seeded voxels of the 128x128x64 random-field workload (M = 961, grid
512x512x256), used by the GPU parity test at full size and by bench.py for
the per-component error of the split-precision forms.

The oracle runs its reduced connection route here (the full boundary system
has 251,782 unknowns); the reduced and un-reduced routes agree on smaller
stacks of the same family (tests/test_oracle_workloads.py), and the growth
exponent of this stack is small. Calls only oracle/ and workloads/. About an
hour on 8 cores and 20 GB of memory (64 dense eigendecompositions of order
3844).

    python tests/golden/make_large_samples.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import cwt  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "large_samples.npz")


def main():
    prob, grid = W.random_field_config("large")
    t0 = time.time()
    st = cwt.setup(prob)
    print("oracle setup %.0f s" % (time.time() - t0), flush=True)
    sol = cwt.solve(st, "reduced")
    print("oracle setup+solve %.0f s" % (time.time() - t0), flush=True)
    rng = np.random.Generator(np.random.PCG64(2025))
    n = 4096
    j = rng.integers(0, grid.fz, n)
    g = rng.integers(0, grid.fy, n)
    f = rng.integers(0, grid.fx, n)
    zs = grid.z_planes()
    x = f * prob.X / grid.fx
    y = g * prob.Y / grid.fy
    E = cwt.field_at_points(st, sol, x, y, zs[j])
    np.savez_compressed(OUT, j=j, g=g, f=f, E=E, fx=grid.fx, fy=grid.fy, fz=grid.fz,
                        M=st.M, p_inc=st.p_inc, p_ref=sol.p_ref, p_trn=sol.p_trn)
    print("wrote %s (%.0f s)" % (OUT, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
