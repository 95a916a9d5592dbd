"""The HIP surrogate against its FP64 CPU reference (oracle/surrogate.py,
itself pinned by finite differences): forward outputs and every parameter
gradient, through the C ABI; plus training on CWT-generated pairs and the CWT
fallback. FP32 kernels: forward and gradients agree with the FP64 reference to
1e-5 and 1e-4 relative L2. BF16 matrix-core mode: two evaluations of the
network on bf16-rounded operands do not agree element by element, because a
relative change of 3e-7 in the values being rounded (FP32 against FP64
accumulation) already moves the output of the rounded reference
(oracle/surrogate.py, bf16=True) by about 0.6 of its own distance to the exact
network (measured on the reference alone). The test therefore checks what is
fixed: the GPU's distance to the exact network is that of the rounded
reference within a factor 2, and the GPU is closer to the rounded reference
than the rounded reference is to the exact network."""
import numpy as np
import pytest

import workloads as W
from oracle import surrogate as S

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ctx():
    _torch()
    import paper_2404_07293_amd as P
    return P.Context(0)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _net_and_data(ctx, B=3, seed=5):
    torch = _torch()
    from paper_2404_07293_amd.surrogate import Surrogate
    sur = Surrogate(ctx, max_batch=max(8, B), seed=1)
    p = S.init_params(2)
    for k in range(S.N_LAYERS):
        p["spec%d" % k] *= 4.0
    flat = S.flatten(p).astype(np.float32)
    sur.set_params(flat)
    p32 = S.unflatten(flat.astype(np.float64))
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, 16, 32, 32)).astype(np.float32)
    tgt = (rng.standard_normal((B, 3, 15, 15)) + 1j * rng.standard_normal((B, 3, 15, 15)))
    tgt = tgt.astype(np.complex64)
    xd = torch.as_tensor(x).cuda()
    td = torch.as_tensor(tgt).cuda()
    return sur, p32, x.astype(np.float64), tgt.astype(np.complex128), xd, td


def test_forward_matches_reference(ctx):
    torch = _torch()
    sur, p, x, tgt, xd, td = _net_and_data(ctx)
    got = sur.forward(xd).cpu().numpy()
    torch.cuda.synchronize()
    want = S.forward(p, x)
    err = rel(got, want)
    print("surrogate forward rel-L2 %.3e" % err)
    assert err <= 1e-5


def test_forward_matches_reference_over_several_tiles(ctx):
    """37 patches: the layer mixing takes two tiles of 32 patches (the second
    ragged) and the head's mixing ends on a partial group of 4."""
    torch = _torch()
    sur, p, x, tgt, xd, td = _net_and_data(ctx, B=37, seed=9)
    got = sur.forward(xd).cpu().numpy()
    torch.cuda.synchronize()
    want = S.forward(p, x)
    errs = [rel(got[i], want[i]) for i in range(len(x))]
    print("surrogate forward, 37 patches: max per-patch rel-L2 %.3e" % max(errs))
    assert max(errs) <= 1e-5


def test_bf16_forward_matches_rounded_reference(ctx):
    torch = _torch()
    sur, p, x, tgt, xd, td = _net_and_data(ctx)
    sur.set_compute(True)
    got = sur.forward(xd).cpu().numpy()
    torch.cuda.synchronize()
    want = S.forward(p, x, bf16=True)
    exact = S.forward(p, x)
    err, dist, ref = rel(got, want), rel(got, exact), rel(want, exact)
    print("bf16 forward rel-L2 %.3e vs rounded reference, %.3e vs exact (reference %.3e)"
          % (err, dist, ref))
    assert 0.5 * ref <= dist <= 2.0 * ref
    assert err <= ref
    sur.set_compute(False)
    back = sur.forward(xd).cpu().numpy()
    torch.cuda.synchronize()
    assert rel(back, exact) <= 1e-5


def test_bf16_forward_over_several_tiles(ctx):
    """Matrix-core inference with bf16 storage on 37 patches: the mixing's
    second tile of 32 patches and the head's second group are ragged. Every
    patch meets the bound of the rounded reference on its own."""
    torch = _torch()
    sur, p, x, tgt, xd, td = _net_and_data(ctx, B=37, seed=9)
    sur.set_compute(True)
    got = sur.forward(xd).cpu().numpy()
    torch.cuda.synchronize()
    want = S.forward(p, x, bf16=True)
    exact = S.forward(p, x)
    errs = [rel(got[i], want[i]) for i in range(len(x))]
    refs = [rel(want[i], exact[i]) for i in range(len(x))]
    dists = [rel(got[i], exact[i]) for i in range(len(x))]
    print("bf16 forward, 37 patches: max rel-L2 %.3e vs rounded reference (max reference "
          "distance %.3e)" % (max(errs), max(refs)))
    for i in range(len(x)):
        assert errs[i] <= 1.5 * refs[i], i
        assert dists[i] <= 2.5 * refs[i], i


def test_bf16_training_reduces_loss(ctx, small_set):
    torch = _torch()
    from paper_2404_07293_amd.surrogate import Surrogate
    n, tg = small_set
    sur = Surrogate(ctx, max_batch=24, seed=3)
    sur.set_compute(True)
    x = sur.encode(n)
    t = torch.as_tensor(tg.astype(np.complex64)).cuda()
    first = sur.train_step(x, t, lr=1e-3)
    for _ in range(150):
        last = sur.train_step(x, t, lr=1e-3)
    print("bf16 training loss %.4f -> %.4f" % (first, last))
    assert last < 0.5 * first


def test_gradients_match_reference(ctx):
    sur, p, x, tgt, xd, td = _net_and_data(ctx)
    loss, g = sur.loss_grad(xd, td)
    out, cache = S.forward(p, x, keep=True)
    assert abs(loss - S.loss(out, tgt)) <= 1e-5 * S.loss(out, tgt)
    gref = S.backward(p, cache, out, tgt)
    gg = S.unflatten(g.astype(np.float64))
    for name, _, _ in S.param_shapes():
        err = rel(gg[name], gref[name])
        print("grad %-7s rel-L2 %.3e" % (name, err))
        assert err <= 1e-4, name


def test_bf16_gradients_match_reference(ctx):
    """Matrix-core mode (bf16 operands, FP32 accumulation): every parameter
    group's gradient against the exact FP64 gradient of the same network and
    data (oracle/surrogate.py).

    Bound, from the arithmetic: a bf16 operand carries a relative rounding of
    up to 2^-9 (2e-3). Rounding the forward products alone moves the exact
    backward's gradients by 1-7e-3 (the rounded reference,
    forward(bf16=True) then the FP64 backward, measured per group below);
    the library also rounds the operands of its backward products, which
    adds about as much again (1.1e-2 measured on the deepest group, lift_w).
    So each group must be within 2e-2 of the exact gradient and point the
    same way (cosine above 0.9999): training in bf16 follows the true descent
    direction. A wrong adjoint (a dropped term, a missing conjugate) is off by
    O(1)."""
    sur, p, x, tgt, xd, td = _net_and_data(ctx)
    sur.set_compute(True)
    loss, g = sur.loss_grad(xd, td)
    sur.set_compute(False)
    out, cache = S.forward(p, x, keep=True)
    assert abs(loss - S.loss(out, tgt)) <= 1e-2 * S.loss(out, tgt)
    gref = S.backward(p, cache, out, tgt)
    outb, cacheb = S.forward(p, x, keep=True, bf16=True)
    grnd = S.backward(p, cacheb, outb, tgt)
    gg = S.unflatten(g.astype(np.float64))
    for name, _, _ in S.param_shapes():
        a, b, c = np.ravel(gg[name]), np.ravel(gref[name]), np.ravel(grnd[name])
        err, err_rnd = rel(a, b), rel(c, b)
        cos = float(np.real(np.vdot(b, a)) / (np.linalg.norm(a) * np.linalg.norm(b)))
        print("bf16 grad %-7s rel-L2 %.3e (rounded reference %.3e) cosine %.7f"
              % (name, err, err_rnd, cos))
        assert err <= 2e-2, name
        assert cos >= 0.9999, name


def test_encode_matches_reference(ctx):
    torch = _torch()
    from paper_2404_07293_amd.surrogate import Surrogate
    sur = Surrogate(ctx, max_batch=4)
    n = np.stack([W.surrogate_patch(W.SURROGATE_SEED0 + i) for i in range(3)])
    x = sur.encode(n).cpu().numpy()
    torch.cuda.synchronize()
    want = np.stack([S.encode(a) for a in n])
    assert np.abs(x - want).max() <= 1e-4


@pytest.fixture(scope="module")
def small_set(ctx):
    from paper_2404_07293_amd.surrogate import cwt_targets
    n = np.stack([W.surrogate_patch(W.SURROGATE_SEED0 + i) for i in range(24)])
    return n, cwt_targets(ctx, n)


def test_training_reduces_loss(ctx, small_set):
    torch = _torch()
    from paper_2404_07293_amd.surrogate import Surrogate
    n, tg = small_set
    sur = Surrogate(ctx, max_batch=24, seed=3)
    x = sur.encode(n)
    t = torch.as_tensor(tg.astype(np.complex64)).cuda()
    first = sur.train_step(x, t, lr=1e-3)
    for _ in range(150):
        last = sur.train_step(x, t, lr=1e-3)
    print("training loss %.4f -> %.4f" % (first, last))
    assert last < 0.5 * first


def test_fallback_returns_cwt_solution(ctx, small_set):
    from paper_2404_07293_amd.surrogate import Surrogate
    n, tg = small_set
    sur = Surrogate(ctx, max_batch=24, seed=3)
    # an impossible tolerance forces the fallback: every patch is solved by CWT
    out, fell, err = sur.infer_checked(n[:6], n_check=2, seed=1, tol=1e-12)
    assert fell and err > 0
    assert rel(out, tg[:6]) <= 1e-12
    # a loose tolerance keeps the surrogate's own outputs
    out2, fell2, err2 = sur.infer_checked(n[:6], n_check=2, seed=1, tol=1e9)
    torch = _torch()
    ref = sur.forward(sur.encode(n[:6])).cpu().numpy()
    torch.cuda.synchronize()
    assert not fell2 and abs(err2 - err) <= 1e-6 * err
    assert rel(out2, ref) <= 1e-6


def test_out_of_distribution_patch_triggers_fallback(ctx, small_set):
    torch = _torch()
    from paper_2404_07293_amd.surrogate import Surrogate
    n, tg = small_set
    sur = Surrogate(ctx, max_batch=24, seed=3)
    x = sur.encode(n)
    t = torch.as_tensor(tg.astype(np.complex64)).cuda()
    for _ in range(100):
        sur.train_step(x, t, lr=1e-3, want_loss=False)
    odd = np.full((2, 8, 32, 32), 2.4 + 0.3j)
    odd[:, :, 8:24, 8:24] = 1.0
    out, fell, err = sur.infer_checked(odd, n_check=2, seed=0, tol=1e-2)
    print("out-of-distribution check rel-L2 %.3e, fallback %s" % (err, fell))
    assert fell and err > 1e-2


def test_trained_network_beats_cwt_at_equal_accuracy(ctx):
    """What the learned part gains: after a short training on CWT-generated
    pairs, the surrogate's error on held-out patches is matched by plain CWT
    only at some truncation U; the surrogate is then at least 100 times faster
    per patch than that CWT run (setup and solve, which a transmitted
    spectrum needs)."""
    import os
    import time
    torch = _torch()
    from paper_2404_07293_amd.surrogate import Surrogate
    data = os.path.join(os.path.dirname(__file__), "..", "paper_2404_07293_amd", "data",
                        "surrogate_targets.npz")
    d = np.load(data, allow_pickle=False)
    seeds, targets = d["seeds"], d["targets"]
    n_tr, n_val = 512, 8
    patches = np.stack([W.surrogate_patch(int(s)) for s in seeds[:n_tr + n_val]])
    sur = Surrogate(ctx, max_batch=n_tr + n_val, seed=11)
    x = sur.encode(patches)
    t = torch.as_tensor(targets[:n_tr + n_val]).cuda()
    rng = np.random.default_rng(3)
    steps = 40 * (n_tr // 32)
    k = 0
    for ep in range(40):
        perm = torch.as_tensor(rng.permutation(n_tr)).cuda()
        for i in range(n_tr // 32):
            idx = perm[i * 32:(i + 1) * 32]
            lr = 0.5 * 2e-3 * (1 + np.cos(np.pi * k / steps))
            sur.train_step(x[idx].contiguous(), t[idx].contiguous(), lr=lr, want_loss=False)
            k += 1
    xv = x[n_tr:].contiguous()
    want = targets[n_tr:n_tr + n_val]
    out = sur.forward(xv).cpu().numpy()
    err_sur = rel(out, want)
    # surrogate time per patch at a batch of 512
    xb = x[:512].contiguous()
    sur.forward(xb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        sur.forward(xb)
    torch.cuda.synchronize()
    t_sur = (time.perf_counter() - t0) / (5 * 512)
    # plain CWT at increasing truncation until it is as accurate
    for U in range(1, 16, 2):
        got = np.zeros(want.shape, np.complex128)
        lo = 7 - U // 2
        t0 = time.perf_counter()
        for i in range(n_val):
            p = W.surrogate_problem(patches[n_tr + i])
            p = W.Problem(n=p.n, px=p.px, py=p.py, pz=p.pz, lam=p.lam, U=U, V=U, n_top=p.n_top,
                          n_bot=p.n_bot, plane_wave=p.plane_wave)
            sol = ctx.solve(p)
            got[i, :, lo:lo + U, lo:lo + U] = sol.exterior()[2].reshape(3, U, U)
            sol.free()
        t_cwt = (time.perf_counter() - t0) / n_val
        err_cwt = rel(got, want)
        if err_cwt <= err_sur:
            break
    print("surrogate rel-L2 %.3e at %.2e s/patch; CWT U=%d rel-L2 %.3e at %.2e s/patch"
          % (err_sur, t_sur, U, err_cwt, t_cwt))
    assert err_sur < 0.1
    assert err_cwt <= err_sur
    assert t_cwt > 100 * t_sur


def test_deployed_weights_meet_their_validation_error(ctx):
    """The committed network (paper_2404_07293_amd/data/surrogate_weights.npz,
    trained on 20,000 CWT pairs by train_surrogate.py) in its deployed
    arithmetic: on the 128 held-out pairs it reproduces the validation rel-L2
    recorded at training (within 5 %), which is below the checked inference's
    1e-2 threshold; on 4 of those patches it is as close to the FP64 oracle's
    bf16 network as the rounded reference is to the exact one."""
    import os
    torch = _torch()
    from paper_2404_07293_amd.surrogate import Surrogate
    here = os.path.join(os.path.dirname(__file__), "..", "paper_2404_07293_amd", "data")
    wfile = os.path.join(here, "surrogate_weights.npz")
    if not os.path.exists(wfile):
        pytest.skip("no deployed weights")
    w = np.load(wfile, allow_pickle=False)
    d = np.load(os.path.join(here, "surrogate_targets.npz"), allow_pickle=False)
    seeds, targets = d["seeds"][-128:], d["targets"][-128:]
    assert int(w["val_seed_first"]) == int(seeds[0])
    patches = np.stack([W.surrogate_patch(int(s)) for s in seeds])
    sur = Surrogate(ctx, max_batch=128, seed=0)
    sur.set_params(w["params"])
    sur.set_compute(True)
    x = sur.encode(patches)
    got = sur.forward(x).cpu().numpy()
    torch.cuda.synchronize()
    err = rel(got, targets)
    rec = float(w["val_rel_l2_bf16"])
    print("deployed weights: val rel-L2 %.4e (recorded %.4e)" % (err, rec))
    assert err <= 1.05 * rec and err < 1e-2
    p = S.unflatten(w["params"].astype(np.float64))
    xs = x[:4].cpu().numpy().astype(np.float64)
    want = S.forward(p, xs, bf16=True)
    exact = S.forward(p, xs)
    e_ref, e_gpu = rel(want, exact), rel(got[:4], exact)
    print("deployed weights, 4 patches: GPU %.3e, rounded reference %.3e from the exact network"
          % (e_gpu, e_ref))
    assert rel(got[:4], want) <= e_ref
    assert e_gpu <= 2.0 * e_ref


def test_bf16_inference_is_per_patch_at_large_batch(ctx):
    """1100 patches: the persistent inference kernels then take several patches
    per block, with the next patch's loads in flight. Every patch's output is
    bit for bit the one it gets in a batch of its own 100 (one patch per
    block), and sampled patches meet the rounded reference's bound."""
    torch = _torch()
    from paper_2404_07293_amd.surrogate import Surrogate
    sur = Surrogate(ctx, max_batch=1100, seed=1)
    p = S.init_params(4)
    for k in range(S.N_LAYERS):
        p["spec%d" % k] *= 4.0
    flat = S.flatten(p).astype(np.float32)
    sur.set_params(flat)
    sur.set_compute(True)
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    x = torch.randn((1100, 16, 32, 32), device="cuda", generator=g)
    big = sur.forward(x).clone()
    part = sur.forward(x[1000:].contiguous())
    first = sur.forward(x[:3].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(big[1000:], part)
    assert torch.equal(big[:3], first)
    p32 = S.unflatten(flat.astype(np.float64))
    idx = [0, 517, 1099]
    xs = x[idx].cpu().numpy().astype(np.float64)
    want = S.forward(p32, xs, bf16=True)
    exact = S.forward(p32, xs)
    got = big[idx].cpu().numpy()
    err, ref = rel(got, want), rel(want, exact)
    print("bf16 inference, 1100 patches: sampled rel-L2 %.3e vs rounded reference (%.3e)"
          % (err, ref))
    assert err <= ref
    assert rel(got, exact) <= 2.0 * ref


def test_bf16_inference_full_batch_is_finite_and_repeatable(ctx):
    """Batch 4096, every persistent block taking several patches, on the
    network's own random initialisation and normal inputs: all outputs are
    finite, two runs agree bit for bit, and sampled patches meet the rounded
    reference's bound. A block reading an LDS table before it is written (on
    its first patch) shows up here as non-finite or run-dependent values."""
    torch = _torch()
    from paper_2404_07293_amd.surrogate import Surrogate
    sur = Surrogate(ctx, max_batch=4096, seed=11)
    sur.set_compute(True)
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    x = torch.randn((4096, 16, 32, 32), device="cuda", generator=g)
    a = sur.forward(x).clone()
    b = sur.forward(x).clone()
    torch.cuda.synchronize()
    assert bool(torch.isfinite(torch.view_as_real(a)).all())
    assert torch.equal(a, b)
    p = S.unflatten(sur.get_params().astype(np.float64))
    idx = [0, 2049, 4095]
    xs = x[idx].cpu().numpy().astype(np.float64)
    want = S.forward(p, xs, bf16=True)
    exact = S.forward(p, xs)
    got = a[idx].cpu().numpy()
    err, ref = rel(got, want), rel(want, exact)
    print("bf16 inference, 4096 patches: sampled rel-L2 %.3e vs rounded reference (%.3e)"
          % (err, ref))
    assert err <= ref
    assert rel(got, exact) <= 2.0 * ref
