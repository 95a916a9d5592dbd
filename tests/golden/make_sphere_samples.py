"""Write tests/golden/sphere_samples.npz: the FP64 oracle's E field of the
16x16x4 sphere workload (M = 25) at 4096 seeded voxels of its 32^3 grid, by
the full boundary system; bench.py states the FP64 synthesis error on it.
Calls only oracle/ and workloads/; a few seconds.

    python tests/golden/make_sphere_samples.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import cwt  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere_samples.npz")


def main():
    prob, grid = W.sphere_config()
    _, _, E = cwt.simulate(prob, grid)
    rng = np.random.Generator(np.random.PCG64(2026))
    n = 4096
    j = rng.integers(0, grid.fz, n)
    g = rng.integers(0, grid.fy, n)
    f = rng.integers(0, grid.fx, n)
    np.savez_compressed(OUT, j=j, g=g, f=f, E=E[:, j, g, f], fx=grid.fx, fy=grid.fy,
                        fz=grid.fz, M=prob.U * prob.V)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
