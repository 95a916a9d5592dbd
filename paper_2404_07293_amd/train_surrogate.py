"""Generate CWT training pairs for the spectral-convolution surrogate, train it
and save the network.

Training pairs: the random-field patches with seeds SEED0 + 2048 + i, disjoint
from the committed pairs (seeds SEED0 .. SEED0 + 1023,
paper_2404_07293_amd/data/surrogate_targets.npz), whose last 128 are the
validation set. Their targets are the transmitted coefficients of plain CWT at
U = 15, solved with scw_solve_batch: device eigensolver, stable route with its
boundary systems on the device. Generation takes a range of pair indices so
that it can be split over processes and runs:

    python -m paper_2404_07293_amd.train_surrogate generate --first 0 \\
        --count 5000 --out pairs_0.npz
    python -m paper_2404_07293_amd.train_surrogate train --pairs pairs_*.npz \\
        --out paper_2404_07293_amd/data/surrogate_weights.npz

Training uses the library's own kernels (Adam, cosine learning rate) with bf16
matrix-core products and FP32 accumulation (set_compute(True)); the saved
network is deployed in that arithmetic. The weights file holds the flat FP32
parameters, the seed ranges, the schedule, the final training loss and the
validation rel-L2 in both product arithmetics.
"""
import argparse
import glob
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HERE = os.path.dirname(os.path.abspath(__file__))
VAL_DATA = os.path.join(HERE, "data", "surrogate_targets.npz")
TRAIN_SEED_OFFSET = 2048
N_VAL = 128


def train_seed(i):
    import workloads as W
    return W.SURROGATE_SEED0 + TRAIN_SEED_OFFSET + i


def generate(a):
    import paper_2404_07293_amd as P
    import workloads as W
    from paper_2404_07293_amd.surrogate import cwt_targets
    ctx = P.Context(0)
    seeds = np.array([train_seed(i) for i in range(a.first, a.first + a.count)], np.int64)
    targets = np.empty((a.count, 3, 15, 15), np.complex64)
    t0 = time.time()
    for c0 in range(0, a.count, a.chunk):
        patches = np.stack([W.surrogate_patch(int(s)) for s in seeds[c0:c0 + a.chunk]])
        tg = cwt_targets(ctx, patches, eig="device", chunk=a.chunk, route="stable_device")
        targets[c0:c0 + len(patches)] = tg
        print("pairs %d..%d: %d/%d, %.1f s" % (a.first, a.first + a.count,
                                              c0 + len(patches), a.count, time.time() - t0),
              flush=True)
    np.savez(a.out, seeds=seeds, targets=targets, seconds=time.time() - t0)
    print("wrote %s (%d pairs, %.0f s)" % (a.out, a.count, time.time() - t0), flush=True)


def load_pairs(patterns):
    files = sorted({f for p in patterns for f in glob.glob(p)})
    if not files:
        raise SystemExit("no pair files match %s" % patterns)
    seeds, targets, secs = [], [], 0.0
    for f in files:
        d = np.load(f, allow_pickle=False)
        seeds.append(d["seeds"])
        targets.append(d["targets"])
        secs += float(d["seconds"])
    seeds, targets = np.concatenate(seeds), np.concatenate(targets)
    order = np.argsort(seeds)
    seeds, targets = seeds[order], targets[order]
    if np.any(np.diff(seeds) == 0):
        raise SystemExit("pair files overlap")
    return seeds, targets, secs, files


def train(a):
    import torch

    import paper_2404_07293_amd as P
    import workloads as W
    from paper_2404_07293_amd.surrogate import Surrogate
    seeds, targets, t_gen, files = load_pairs(a.pairs)
    n = len(seeds)
    print("%d training pairs from %d files" % (n, len(files)), flush=True)
    ctx = P.Context(0)
    dev = torch.device("cuda", 0)
    sur = Surrogate(ctx, max_batch=max(a.batch, 512), seed=11)
    sur.set_compute(True)
    x_tr = torch.empty((n, 16, 32, 32), dtype=torch.float32, device=dev)
    step = sur.max_batch
    for c0 in range(0, n, step):
        x_tr[c0:c0 + step] = sur.encode(np.stack([W.surrogate_patch(int(s))
                                                  for s in seeds[c0:c0 + step]]))
    t_tr = torch.as_tensor(targets).to(dev)
    d = np.load(VAL_DATA, allow_pickle=False)
    vseeds, vtargets = d["seeds"][-N_VAL:], d["targets"][-N_VAL:]
    x_va = sur.encode(np.stack([W.surrogate_patch(int(s)) for s in vseeds]))
    t_va = torch.as_tensor(vtargets).to(dev)

    def val_err():
        out = sur.forward(x_va.contiguous())
        torch.cuda.synchronize()
        o, w = out.cpu().numpy(), t_va.cpu().numpy()
        return float(np.linalg.norm(o - w) / np.linalg.norm(w))

    rng = np.random.Generator(np.random.PCG64(3))
    per = n // a.batch
    steps = a.epochs * per
    k = 0
    t1 = time.time()
    loss = None
    for ep in range(a.epochs):
        perm = torch.as_tensor(rng.permutation(n), device=dev)
        for i in range(per):
            idx = perm[i * a.batch:(i + 1) * a.batch]
            lr = 0.5 * a.lr * (1 + np.cos(np.pi * k / steps))
            last = i == per - 1
            loss = sur.train_step(x_tr[idx].contiguous(), t_tr[idx].contiguous(), lr=lr,
                                  want_loss=last)
            k += 1
        print("epoch %d/%d: loss %.4e, val rel-L2 %.3e, %.1f s" % (
            ep + 1, a.epochs, loss, val_err(), time.time() - t1), flush=True)
    t_train = time.time() - t1
    err_bf16 = val_err()
    sur.set_compute(False)
    err_fp32 = val_err()
    np.savez(a.out, params=sur.get_params().astype(np.float32),
             seed_first=int(seeds[0]), seed_last=int(seeds[-1]), seed_count=int(n),
             val_seed_first=int(vseeds[0]), val_seed_count=int(N_VAL),
             epochs=a.epochs, batch=a.batch, lr=a.lr, steps=steps, final_loss=float(loss),
             products="bf16", val_rel_l2_bf16=err_bf16, val_rel_l2_fp32=err_fp32,
             target_seconds=t_gen, train_seconds=t_train)
    print("wrote %s: val rel-L2 %.3e (bf16 products), %.3e (fp32); targets %.0f s, training "
          "%.0f s" % (a.out, err_bf16, err_fp32, t_gen, t_train), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate", help="CWT targets for a range of training pairs")
    g.add_argument("--first", type=int, default=0)
    g.add_argument("--count", type=int, required=True)
    g.add_argument("--chunk", type=int, default=128, help="patches per batched solve")
    g.add_argument("--out", required=True)
    t = sub.add_parser("train", help="train on generated pairs and save the network")
    t.add_argument("--pairs", nargs="+", required=True, help="pair files (globs allowed)")
    t.add_argument("--epochs", type=int, default=500)
    t.add_argument("--batch", type=int, default=64)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "generate":
        generate(a)
    else:
        train(a)


if __name__ == "__main__":
    sys.exit(main())
