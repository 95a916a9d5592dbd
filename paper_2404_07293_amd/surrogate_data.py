"""Generate surrogate training targets with the library's CWT solver.

For patch seeds SEED0 + start .. SEED0 + start + count - 1 (the random-field
family, 8 x 32 x 32 voxels), solve the CWT problem with scw_solve and store the
transmitted coefficients [3][15][15] (complex64) with their seeds.

    python -m paper_2404_07293_amd.surrogate_data --start 0 --count 512 --out t0.npz
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--start", type=int, default=0)
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    import paper_2404_07293_amd as P
    import workloads as W
    from paper_2404_07293_amd.surrogate import cwt_targets
    ctx = P.Context(0, host_threads=a.threads)
    seeds = W.SURROGATE_SEED0 + a.start + np.arange(a.count)
    t0 = time.time()
    tg = np.empty((a.count, 3, 15, 15), np.complex64)
    for i, s in enumerate(seeds):
        tg[i] = cwt_targets(ctx, [W.surrogate_patch(int(s))])[0]
        if (i + 1) % 64 == 0:
            print("%d/%d patches, %.1f s" % (i + 1, a.count, time.time() - t0), flush=True)
    np.savez_compressed(a.out, seeds=seeds, targets=tg)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    sys.exit(main())
