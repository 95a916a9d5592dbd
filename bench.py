#!/usr/bin/env python3
"""Field-synthesis throughput of the HIP CWT library on one MI355X.

A step is one complete synthesis of the 3-component E field on the output
grid from a solved problem whose inputs are resident in HBM: phase tables,
modal sums P_l (alpha o g(z)) for every interior plane, exterior plane waves,
and the separable inverse transform to the pixel grid. The FP64 setup
(spectra, eigensolves, boundary solve) runs once before timing and is reported
separately.

Default workload: 64x64x32 voxels of a smoothed random index field, 21x21
spatial frequencies (M = 441), NA 0.9 focused x-polarised incident image,
256x256x128 output grid, complex64 synthesis.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "field voxels/s (3-comp E) plain FP32 vs BF16+comp/batched at stated rel-L2"
HBM_PEAK = 8.0e12          # bytes/s
FP32_PEAK = 157.3e12       # flop/s (vector and matrix)
FP64_PEAK = 78.6e12
GOLDEN = os.path.join(ROOT, "tests", "golden", "working_samples.npz")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stage_model(sol_info, plan, prec):
    """Algorithmic bytes and flops of each synthesis stage for one call."""
    M, L = plan["M"], plan["L"]
    fx, fy, fz = plan["fx"], plan["fy"], plan["fz"]
    U, V = plan["U"], plan["V"]
    eb = 16 if prec == "fp64" else 8
    n2, n3 = 2 * M, 3 * M
    layers = plan["layers_touched"]
    ntask, zt = plan["ntasks"], plan["zt"]
    interior = plan["interior_planes"]
    return {
        "phase": {"bytes": ntask * 2 * zt * n2 * eb + 3 * layers * n2 * 16,
                  "flops": ntask * zt * n2 * 40},
        # P_l streamed once per task, the phase inputs and the spectra written
        "modal_sum": {"bytes": ntask * n3 * n2 * eb + 3 * layers * n2 * eb
                      + interior * n3 * eb,
                      "flops": 8 * n3 * n2 * interior},
        "exterior": {"bytes": (fz - interior) * n3 * eb, "flops": (fz - interior) * n3 * 40},
        # spectra read, field written; x pass U and y pass V complex MACs
        "idft": {"bytes": fz * n3 * eb + 3 * fx * fy * fz * eb,
                 "flops": 8 * fz * 3 * (V * U * fx + V * fx * fy)},
    }

def plan_summary(prob, grid):
    """Plane classification mirroring the library's plan (for the model)."""
    L, d = prob.nz, prob.pz
    zs = grid.z_planes()
    per = {}
    for z in zs:
        if 0.0 <= z < L * d:
            l = min(int(np.floor(z / d)), L - 1)
            per[l] = per.get(l, 0) + 1
    maxc = max(per.values()) if per else 0
    zt = 1
    while zt < min(maxc, 8):
        zt *= 2
    ntasks = sum((c + zt - 1) // zt for c in per.values())
    return {"M": prob.U * prob.V, "L": L, "U": prob.U, "V": prob.V, "fx": grid.fx,
            "fy": grid.fy, "fz": grid.fz, "layers_touched": len(per), "ntasks": ntasks,
            "zt": zt, "interior_planes": sum(per.values())}


def source_hash():
    h = hashlib.sha256()
    for f in ("kernels_synth.hip", "kernels_mfma.hip"):
        p = os.path.join(ROOT, "paper_2404_07293_amd", "csrc", f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def surrogate_source_hash():
    h = hashlib.sha256()
    for f in ("kernels_surrogate_bf16.hip", "surrogate.cpp"):
        p = os.path.join(ROOT, "paper_2404_07293_amd", "csrc", f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_surrogate_traffic():
    """HBM bytes of one bf16 inference at batch 4096 from the committed PMC
    summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_surrogate_bf16_4096.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != surrogate_source_hash():
        return None
    return rec.get("hbm_bytes_per_inference")


def measured_traffic(kernel_stage, precision, workload):
    """HBM bytes per launch from the committed PMC summary, if it was taken on
    the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s_%s.json" % (kernel_stage, workload,
                                                                     precision))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(prob_full, grid_full, n_layers=2, min_seconds=10.0):
    """The FP64 oracle on a bounded sample of the same workload: the first
    `n_layers` layers of the sample (same lateral size, truncation and
    incident field) and the output planes inside them."""
    import workloads as W
    from oracle import cwt
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    prob = W.Problem(n=prob_full.n[:n_layers].copy(), px=prob_full.px, py=prob_full.py,
                     pz=prob_full.pz, lam=prob_full.lam, U=prob_full.U, V=prob_full.V,
                     n_top=prob_full.n_top, n_bot=prob_full.n_bot, inc_ex=prob_full.inc_ex,
                     inc_ey=prob_full.inc_ey, plane_wave=prob_full.plane_wave)
    ppl = grid_full.fz // prob_full.nz
    grid = W.Grid(fx=grid_full.fx, fy=grid_full.fy, fz=ppl * n_layers, z_begin=0.0,
                  z_end=prob.thickness)
    t0 = time.perf_counter()
    st = cwt.setup(prob)
    sol = cwt.solve(st, "reduced")
    t1 = time.perf_counter()
    reps = 0
    while True:
        E = cwt.synthesize(st, sol, grid)
        reps += 1
        if time.perf_counter() - t1 >= min_seconds:
            break
    t2 = time.perf_counter()
    vox = grid.fx * grid.fy * grid.fz
    assert E.shape == (3, grid.fz, grid.fy, grid.fx)
    per = (t2 - t1) / reps
    # the same synthesis on one thread (the paper's CPU column is single-threaded)
    single = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            r1, t3 = 0, time.perf_counter()
            while True:
                cwt.synthesize(st, sol, grid)
                r1 += 1
                if time.perf_counter() - t3 >= min_seconds / 2:
                    break
            single = {"value": vox / ((time.perf_counter() - t3) / r1), "cores": 1,
                      "reps": r1}
    except ImportError:
        pass
    return {"value": vox / per, "unit": "voxels/s", "cores": int(threads),
            "kind": "oracle",
            "sample": "first %d of %d layers (%d planes of %dx%d, M=%d): oracle synthesis "
                      "repeated %d times, %.3f s each; its FP64 setup+solve took %.1f s and "
                      "is not in value" % (
                          n_layers, prob_full.nz, grid.fz, grid.fx, grid.fy,
                          prob.U * prob.V, reps, per, t1 - t0),
            "single_thread": single}


def golden_error(E, prob, grid, per_component=False, path=GOLDEN):
    """rel-L2 of the synthesised field at the stored oracle sample voxels."""
    if not os.path.exists(path):
        return None
    g = np.load(path, allow_pickle=False)
    if int(g["fx"]) != grid.fx or int(g["fz"]) != grid.fz or int(g["M"]) != prob.U * prob.V:
        return None
    j, gg, f = g["j"], g["g"], g["f"]
    import torch
    idx = torch.as_tensor(np.stack([j, gg, f]), device=E.device)
    got = E[:, idx[0], idx[1], idx[2]].cpu().numpy()
    want = g["E"]
    if per_component:
        return [float(np.linalg.norm(got[c] - want[c]) / np.linalg.norm(want[c]))
                for c in range(3)]
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


SPHERE_GOLDEN = os.path.join(ROOT, "tests", "golden", "sphere_samples.npz")


def sphere_leg(ctx, torch, dev, stream, args):
    """The 16x16x4 sphere (M = 25) on its 32^3 grid in FP64, the correctness
    workload: time per synthesis and rel-L2 against the oracle's full-system
    field at the stored sample voxels."""
    import workloads as W
    prob, grid = W.sphere_config()
    sol = ctx.solve(prob)
    E = torch.empty((3, grid.fz, grid.fy, grid.fx), dtype=torch.complex128, device=dev)
    for _ in range(3):
        sol.synthesize(grid, "fp64", out=E, stream=stream)
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for _ in range(args.steps):
        sol.synthesize(grid, "fp64", out=E, stream=stream)
    s1.record(stream)
    torch.cuda.synchronize()
    ms = s0.elapsed_time(s1) / args.steps
    err = golden_error(E, prob, grid, path=SPHERE_GOLDEN)
    vox = grid.fx * grid.fy * grid.fz
    log("sphere fp64: %.4f ms per synthesis, %.3e voxels/s, rel-L2 %s" % (
        ms, vox / (ms * 1e-3), err))
    sol.free()
    return {"workload": "sphere: 16x16x4 sample, M=25, 32x32x32 grid", "dtype": "f64",
            "value": vox / (ms * 1e-3), "ms_per_step": ms, "rel_l2_vs_oracle": err,
            "note": "launch-latency bound; correctness workload"}


def optics_leg(sol, prob, grid, E_volume, torch, dev, stream, args):
    """Lateral slice and objective image on the working workload: an x-z
    slice through all planes at y = Y/3 (n = fx), and the image through an
    NA 0.8 objective with its intensity on the whole grid. The slice is
    checked against the volume's row where the two coincide (y = Y/2 here),
    the wide-aperture image against the stored oracle samples."""
    Y = prob.ny * prob.py
    Es = torch.empty((3, grid.fz, grid.fx), dtype=torch.complex64, device=dev)
    Ei = torch.empty((3, grid.fz, grid.fy, grid.fx), dtype=torch.complex64, device=dev)
    Ii = torch.empty((grid.fz, grid.fy, grid.fx), dtype=torch.float32, device=dev)

    def timed(call):
        for _ in range(max(2, args.warmup)):
            call()
        torch.cuda.synchronize()
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        for _ in range(args.steps):
            call()
        s1.record(stream)
        torch.cuda.synchronize()
        return s0.elapsed_time(s1) / args.steps

    slice_ms = timed(lambda: sol.synthesize_slice("xz", Y / 3, grid.fx, grid.fz, grid.z_begin,
                                                  grid.z_end, "fp32", out=Es, stream=stream))
    g0 = grid.fy // 2
    sol.synthesize_slice("xz", g0 * Y / grid.fy, grid.fx, grid.fz, grid.z_begin, grid.z_end,
                         "fp32", out=Es, stream=stream)
    row = E_volume[:, :, g0, :]
    slice_vs_volume = float(torch.linalg.vector_norm(Es - row) / torch.linalg.vector_norm(row))
    image_ms = timed(lambda: sol.image(grid, 0.8, "fp32", out=Ei, intensity=Ii, stream=stream))
    sol.image(grid, 100.0, "fp32", out=Ei, intensity=Ii, stream=stream)
    torch.cuda.synchronize()
    wide_err = golden_error(Ei, prob, grid)
    vox = grid.fx * grid.fz
    log("x-z slice: %.4f ms (%d planes x %d samples), rel-L2 vs the volume row %.2e; "
        "NA 0.8 image + intensity: %.4f ms, full-aperture image rel-L2 %s" % (
            slice_ms, grid.fz, grid.fx, slice_vs_volume, image_ms, wide_err))
    return {"slice_xz": {"ms": slice_ms, "samples": vox, "planes": grid.fz,
                         "rel_l2_vs_volume_row": slice_vs_volume,
                         "note": "spectra of every plane (the modal sum) + one slice transform"},
            "image_na08": {"ms": image_ms, "voxels_per_s": grid.fx * grid.fy * grid.fz /
                           (image_ms * 1e-3),
                           "full_aperture_rel_l2_vs_oracle": wide_err,
                           "note": "synthesis with the objective's transfer function on the "
                                   "spectra, plus the intensity pass"}}


def illumination_leg(ctx, prob, grid, single_ms, torch, dev, stream, args):
    """K plane-wave illuminations of the working sample sharing one setup
    (scw_solve_illuminations): the axial x-polarised wave plus K - 1 seeded
    lattice directions with random polarisation. Times one synthesis of all
    K fields (the modal sum of every illumination on the matrix cores, then
    each field's transform) against K plain single syntheses, and the shared
    setup against one single setup. Illumination 0 is checked against the
    single-illumination path on the same solution."""
    import workloads as W
    res = {}
    for K in [int(k) for k in args.illuminations.split(",") if k]:
        rng = np.random.default_rng(41)
        h = prob.U // 2
        ws = [W.PlaneWave(0, 0, 1.0, 0.0)]
        for _ in range(K - 1):
            ex, ey = rng.standard_normal(2) + 1j * rng.standard_normal(2)
            ws.append(W.PlaneWave(int(rng.integers(-h, h + 1)), int(rng.integers(-h, h + 1)),
                                  complex(ex), complex(ey)))
        t0 = time.perf_counter()
        sol = ctx.solve(prob, waves=ws)
        setup_s = time.perf_counter() - t0
        out = torch.empty((K, 3, grid.fz, grid.fy, grid.fx), dtype=torch.complex64, device=dev)
        for _ in range(max(2, args.warmup)):
            sol.synthesize_illuminations(grid, out=out, stream=stream)
        torch.cuda.synchronize()
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        for _ in range(args.steps):
            sol.synthesize_illuminations(grid, out=out, stream=stream)
        s1.record(stream)
        torch.cuda.synchronize()
        ms = s0.elapsed_time(s1) / args.steps
        E0 = sol.synthesize(grid, "fp32", stream=stream)
        torch.cuda.synchronize()
        err = float(torch.linalg.vector_norm(out[0] - E0) / torch.linalg.vector_norm(E0))
        vox = K * grid.fx * grid.fy * grid.fz
        cols = K * grid.fz  # (illumination, plane) columns of the modal sum
        flops = 8.0 * 3 * sol.M * 2 * sol.M * cols
        log("%d illuminations: %.4f ms (%.4f ms per field vs %.4f single), %.3e voxels/s; "
            "setup %.2f s; illumination 0 vs single path rel-L2 %.2e" % (
                K, ms, ms / K, single_ms, vox / (ms * 1e-3), setup_s, err))
        res["K%d" % K] = {"illuminations": K, "ms": ms, "ms_per_field": ms / K,
                          "voxels_per_s": vox / (ms * 1e-3),
                          "speedup_vs_single_syntheses": single_ms * K / ms,
                          "setup_s": setup_s, "modal_sum_flops": flops,
                          "rel_l2_illum0_vs_single_path": err}
        del out, E0
        sol.free()
    return res


SWEEP_GOLDEN = os.path.join(ROOT, "tests", "golden", "sweep_job.npz")
LARGE_GOLDEN = os.path.join(ROOT, "tests", "golden", "large_samples.npz")


def large_leg(ctx, torch, dev, stream, args):
    """The 128x128x64 random-field sample (M = 961, 64 layers) on the
    512x512x256 grid: plain FP32 synthesis and the two split-precision forms,
    each with its rel-L2 against the oracle, per component."""
    import workloads as W
    prob, grid = W.random_field_config("large")
    import paper_2404_07293_amd as P
    route = "stable_device"
    t0 = time.perf_counter()
    try:
        sol = ctx.solve(prob, route=route)
    except P.ScwError as e:  # recorded, then the host elimination
        log("large: device elimination failed (%s); solving on the host" % e)
        route = "stable (device route failed: %s)" % e
        t0 = time.perf_counter()
        sol = ctx.solve(prob, route="stable")
    t_setup = time.perf_counter() - t0
    info = sol.info()
    log("large: setup %.1f s (eig %.1f s, boundary solve on the device %.2f s), "
        "growth exponent %.1f" % (t_setup, info["eig_seconds"], info["boundary_seconds"],
                                  info["growth_exponent"]))
    E = torch.empty((3, grid.fz, grid.fy, grid.fx), dtype=torch.complex64, device=dev)
    voxels = grid.fx * grid.fy * grid.fz
    rec = {"workload": "large: %dx%dx%d random-field sample, M=%d, %dx%dx%d grid" % (
        prob.nx, prob.ny, prob.nz, prob.U * prob.V, grid.fx, grid.fy, grid.fz),
        "voxels_per_step": voxels, "setup_s": t_setup, "eig_s": info["eig_seconds"],
        "boundary_s": info["boundary_seconds"], "route": route,
        "growth_exponent": info["growth_exponent"]}
    steps = max(3, args.steps // 5)
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    for prec in ("fp32", "bf16x3", "fp16x3"):
        tune = sol.tune(grid, prec, out=E, stream=stream, reps=2) if args.tune else None
        for _ in range(2):
            sol.synthesize(grid, prec, out=E, stream=stream)
        torch.cuda.synchronize()
        s0.record(stream)
        for _ in range(steps):
            sol.synthesize(grid, prec, out=E, stream=stream)
        s1.record(stream)
        torch.cuda.synchronize()
        ms = s0.elapsed_time(s1) / steps
        err = golden_error(E, prob, grid, path=LARGE_GOLDEN)
        per = golden_error(E, prob, grid, True, path=LARGE_GOLDEN)
        rec[prec] = {"value": voxels / (ms * 1e-3), "ms_per_step": ms,
                     "rel_l2_vs_oracle": err, "rel_l2_per_component": per,
                     "hbm_bytes_algorithmic": sol.synthesis_bytes(grid, prec),
                     "tuning": tune}
        log("large %s: ms/step %.3f, %.3e voxels/s, rel-L2 %s per component %s" % (
            prec, ms, voxels / (ms * 1e-3), err, per))
    del E
    sol.free()
    return rec


def roof_batch(jobs, grid, ms):
    """Roofline of the batched launch. Its kernel runs factored transform
    passes and is bound by writing the fields: bytes = every job's field
    (3 fz fy fx complex64) plus the coefficients its transmitted planes read
    (p_trn, 3M, and k s_z of the lower half-space, M; complex64), against the
    HBM peak. The direct-sum
    flops of the separable transform are kept as an equivalent figure only;
    the factored passes do not execute them."""
    fl = sum(8.0 * 3 * grid.fz * (u * u * grid.fx + u * grid.fx * grid.fy) for _, _, u in jobs)
    out = 8.0 * 3 * grid.fz * grid.fx * grid.fy * len(jobs)
    coef = sum(8.0 * 4 * u * u for _, _, u in jobs)
    t = ms * 1e-3
    return {"bound": "hbm", "achieved": (out + coef) / t / 1e9, "peak": HBM_PEAK / 1e9,
            "unit": "GB/s", "frac": (out + coef) / t / HBM_PEAK, "algorithmic_bytes": out + coef,
            "field_bytes": out, "coefficient_bytes": coef,
            "equivalent_direct_sum_flops": fl,
            "equivalent_direct_sum_tflops": fl / t / 1e12}


def batched_sweep(ctx, torch, dev, stream, args):
    """The spectral sweep (256 wavenumbers x 16 patches of 32x32x16 voxels,
    truncation 9..25 per patch, 8 transmitted planes of 64x64) as one batched,
    graph-captured launch. Each patch is solved once at one wavenumber (patch
    p at the (16p+1)-th); the 4096 jobs reuse the solution of their patch, so
    the launch does the synthesis work of the full sweep (the work per job
    depends only on its truncation and the grid)."""
    import workloads as W
    jobs = W.spectral_sweep_jobs()
    nus = sorted(set(j[0] for j in jobs))
    u_of = {p: u for _, p, u in jobs}
    t0 = time.perf_counter()
    solved, grid = {}, None
    for p in sorted(u_of):
        prob, grid = W.sweep_problem(nus[16 * p], p, u_of[p])
        solved[p] = ctx.solve(prob)
    t_setup = time.perf_counter() - t0
    b = ctx.batch([solved[p] for _, p, _ in jobs], grid)
    Eb = torch.empty((len(jobs), 3, grid.fz, grid.fy, grid.fx), dtype=torch.complex64,
                     device=dev)
    tune = b.tune(out=Eb, stream=stream, reps=3) if args.tune else None
    if tune:
        log("tuned batch: %s" % tune)
    for _ in range(max(2, args.warmup)):
        b.launch(out=Eb, stream=stream)
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for _ in range(args.steps):
        b.launch(out=Eb, stream=stream)
    s1.record(stream)
    torch.cuda.synchronize()
    ms = s0.elapsed_time(s1) / args.steps
    voxels = len(jobs) * grid.fz * grid.fy * grid.fx
    err = None
    if os.path.exists(SWEEP_GOLDEN):
        g = np.load(SWEEP_GOLDEN, allow_pickle=False)
        pt, k = int(g["patch"]), int(g["nu_index"])
        if k == 16 * pt:
            idx = [i for i, (nu, p, _) in enumerate(jobs) if p == pt][0]
            got = Eb[idx].cpu().numpy()
            err = float(np.linalg.norm(got - g["E"]) / np.linalg.norm(g["E"]))
    bytes_out = voxels * 3 * 8
    log("batched sweep: %d jobs, %.3f ms/launch, %.3e voxels/s, rel-L2 %s (setup %.1f s)" % (
        len(jobs), ms, voxels / (ms * 1e-3), err, t_setup))
    distinct = distinct_sweep(ctx, torch, dev, stream, args, jobs, grid, tune)
    rec = {"value": voxels / (ms * 1e-3), "ms_per_step": ms, "jobs": len(jobs),
           "voxels_per_step": voxels, "rel_l2_vs_oracle": err,
           "hbm_write_gbps": bytes_out / (ms * 1e-3) / 1e9,
           "roofline": roof_batch(jobs, grid, ms),
           "solved_jobs": len(solved), "setup_s": t_setup, "tuning": tune,
           "note": "one solve per patch; all 256 wavenumbers of a patch reuse it",
           "distinct": distinct}
    del Eb
    b.free()
    for sol in solved.values():
        sol.free()
    return rec


def distinct_sweep(ctx, torch, dev, stream, args, jobs, grid, tune):
    """Every wavenumber of the two U = 9 patches (8 and 13) solved on its own:
    512 distinct jobs. Their fields in one batched launch (the shape the
    4096-job tuner chose), against the same jobs as 512 separate
    scw_synthesize calls (the plain GPU form), both FP32; the stored oracle job
    (patch 8 at the 129th wavenumber) is one of them and gives the error of
    both forms."""
    import workloads as W
    pats = (8, 13)
    djobs = [(nu, p, u) for nu, p, u in jobs if p in pats]
    nus = sorted(set(j[0] for j in jobs))
    t0 = time.perf_counter()
    sols = [ctx.solve(W.sweep_problem(nu, p, u)[0]) for nu, p, u in djobs]
    t_setup = time.perf_counter() - t0
    b = ctx.batch(sols, grid)
    if tune:
        b.configure(tune["radix"], tune["blocks_per_cu"], tune["chunk"])
    Eb = torch.empty((len(djobs), 3, grid.fz, grid.fy, grid.fx), dtype=torch.complex64,
                     device=dev)
    Ep = torch.empty_like(Eb)
    for _ in range(max(2, args.warmup)):
        b.launch(out=Eb, stream=stream)
    for i, sol in enumerate(sols):  # plans of the plain form, built before timing
        sol.synthesize(grid, "fp32", out=Ep[i], stream=stream)
    torch.cuda.synchronize()
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for _ in range(args.steps):
        b.launch(out=Eb, stream=stream)
    s1.record(stream)
    torch.cuda.synchronize()
    ms_b = s0.elapsed_time(s1) / args.steps
    reps = max(2, args.steps // 5)
    s0.record(stream)
    for _ in range(reps):
        for i, sol in enumerate(sols):
            sol.synthesize(grid, "fp32", out=Ep[i], stream=stream)
    s1.record(stream)
    torch.cuda.synchronize()
    ms_p = s0.elapsed_time(s1) / reps
    voxels = len(djobs) * grid.fz * grid.fy * grid.fx
    err_b = err_p = None
    if os.path.exists(SWEEP_GOLDEN):
        g = np.load(SWEEP_GOLDEN, allow_pickle=False)
        key = (nus[int(g["nu_index"])], int(g["patch"]))
        idx = [i for i, (nu, p, _) in enumerate(djobs) if (nu, p) == key]
        if idx:
            want = g["E"]
            err_b = float(np.linalg.norm(Eb[idx[0]].cpu().numpy() - want) / np.linalg.norm(want))
            err_p = float(np.linalg.norm(Ep[idx[0]].cpu().numpy() - want) / np.linalg.norm(want))
    same = float(torch.linalg.vector_norm(Eb - Ep) / torch.linalg.vector_norm(Ep))
    log("distinct sweep jobs: %d solved in %.1f s; batched %.3f ms (%.3e voxels/s), plain "
        "per-job synthesis %.3f ms (%.3e voxels/s); rel-L2 vs oracle batched %s plain %s; "
        "batched vs plain %.1e" % (len(djobs), t_setup, ms_b, voxels / (ms_b * 1e-3), ms_p,
                                   voxels / (ms_p * 1e-3), err_b, err_p, same))
    rec = {"jobs": len(djobs), "patches": list(pats), "U": 9, "setup_s": t_setup,
           "batched": {"ms": ms_b, "value": voxels / (ms_b * 1e-3), "rel_l2_vs_oracle": err_b},
           "plain": {"ms": ms_p, "value": voxels / (ms_p * 1e-3), "rel_l2_vs_oracle": err_p,
                     "calls": len(djobs)},
           "batched_over_plain": ms_p / ms_b, "batched_vs_plain_rel_l2": same}
    del Eb, Ep
    b.free()
    for sol in sols:
        sol.free()
    return rec


SUR_DATA = os.path.join(ROOT, "paper_2404_07293_amd", "data", "surrogate_targets.npz")


def surrogate_flops_per_patch():
    """Arithmetic of one inference (real flops; a complex MAC is 8, a real
    by complex MAC 4): lift, four Fourier layers (row and column DFTs, per-mode
    mixing, inverse DFTs with the real part only, pointwise map) and the head."""
    n, w, cin, ky, kx, hk = 32, 32, 16, 17, 9, 15
    lift = 2 * cin * w * n * n
    layer = (w * n * kx * n * 4 + w * ky * kx * n * 8 + ky * kx * w * w * 8
             + w * n * kx * ky * 8 + w * n * n * kx * 4 + 2 * w * w * n * n)
    head = w * n * hk * n * 4 + w * hk * hk * n * 8 + hk * hk * w * 3 * 8
    return lift + 4 * layer + head


def surrogate_bytes_per_patch(elem=4):
    """Activation traffic one inference cannot avoid (activations of 32 x 32 x
    32 per patch, elem bytes each: 4 for FP32 storage, 2 for bf16): the lift
    reads its 16 FP32 input channels and writes h; each Fourier layer reads h
    and writes the next h (its spectra can stay on chip); the head reads h and
    writes 15 x 15 x 3 complex64 outputs."""
    n, w, cin, hk = 32, 32, 16, 15
    act = w * n * n * elem
    return cin * n * n * 4 + act + 4 * (2 * act) + act + hk * hk * 3 * 8


def cwt_equal_accuracy(ctx, patches, targets, err_goal):
    """Plain CWT on the surrogate's patches at truncation U = 1, 3, 5, ...:
    rel-L2 of its transmitted coefficients (zero outside its band) against the
    15 x 15 reference, and its patches/s on its fastest route (the patches
    solved together by scw_solve_batch: device eigensolver, device
    elimination). Returns the first U whose error is at most err_goal, with
    the sweep."""
    import workloads as W
    sweep = []
    for U in range(1, 16, 2):
        got = np.zeros(targets.shape, np.complex128)
        lo = 7 - U // 2
        probs = []
        for n in patches:
            prob = W.surrogate_problem(n)
            probs.append(W.Problem(n=prob.n, px=prob.px, py=prob.py, pz=prob.pz, lam=prob.lam,
                                   U=U, V=U, n_top=prob.n_top, n_bot=prob.n_bot,
                                   plane_wave=prob.plane_wave))
        t0 = time.perf_counter()
        sols = ctx.solve_batch(probs, route="stable_device", eig="device")
        for i, sol in enumerate(sols):
            got[i, :, lo:lo + U, lo:lo + U] = sol.exterior()[2].reshape(3, U, U)
        rate = len(patches) / (time.perf_counter() - t0)
        for sol in sols:
            sol.free()
        err = float(np.linalg.norm(got - targets) / np.linalg.norm(targets))
        sweep.append({"U": U, "rel_l2": err, "patches_per_s": rate})
        if err <= err_goal:
            return dict(sweep[-1], sweep=sweep)
    return {"U": None, "sweep": sweep}


SUR_WEIGHTS = os.path.join(ROOT, "paper_2404_07293_amd", "data", "surrogate_weights.npz")


def surrogate_leg(ctx, torch, dev, stream, args):
    """The spectral-convolution surrogate: the trained network when its
    weights file is present (else a short training on the committed pairs),
    validation rel-L2 on 128 held-out CWT pairs, inference at batch 4096 in
    both product arithmetics, checked inference, and plain CWT at equal
    accuracy."""
    import workloads as W
    from paper_2404_07293_amd.surrogate import Surrogate
    d = np.load(SUR_DATA, allow_pickle=False)
    seeds, targets = d["seeds"], d["targets"]
    n_val = 128
    patches = np.stack([W.surrogate_patch(int(s)) for s in seeds])
    sur = Surrogate(ctx, max_batch=4096, seed=11)
    sur.set_compute(bool(args.sur_bf16))
    x_all = sur.encode(patches)
    t_all = torch.as_tensor(targets).to(dev)
    n_tr = len(seeds) - n_val
    xtr, ttr, xva, tva = x_all[:n_tr], t_all[:n_tr], x_all[n_tr:], t_all[n_tr:]
    trained = None
    if args.sur_weights and os.path.exists(args.sur_weights):
        w = np.load(args.sur_weights, allow_pickle=False)
        sur.set_params(w["params"])
        trained = {k: (w[k].item() if w[k].ndim == 0 else None) for k in w.files if k != "params"}
        train_pairs, steps, t_train = int(w["seed_count"]), int(w["steps"]), float(
            w["train_seconds"])
    else:
        rng = np.random.Generator(np.random.PCG64(3))
        bs, epochs, lr0 = args.sur_batch, args.sur_epochs, args.sur_lr
        steps = epochs * (n_tr // bs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = 0
        for ep in range(epochs):
            perm = torch.as_tensor(rng.permutation(n_tr), device=dev)
            for i in range(n_tr // bs):
                idx = perm[i * bs:(i + 1) * bs]
                lr = 0.5 * lr0 * (1 + np.cos(np.pi * k / steps))   # cosine decay
                sur.train_step(xtr[idx].contiguous(), ttr[idx].contiguous(), lr=lr,
                               want_loss=False)
                k += 1
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        train_pairs = n_tr

    def err_on(x, t):
        out = sur.forward(x.contiguous())
        torch.cuda.synchronize()
        o, w = out.cpu().numpy(), t.cpu().numpy()
        return float(np.linalg.norm(o - w) / np.linalg.norm(w))

    val_err = err_on(xva, tva)
    # inference throughput at batch 4096 (inputs encoded and resident)
    reps = (4096 + len(seeds) - 1) // len(seeds)
    xb = x_all.repeat(reps, 1, 1, 1)[:4096].contiguous()
    out = torch.empty((4096, 3, 15, 15), dtype=torch.complex64, device=dev)
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    n_inf = max(5, args.steps // 5)

    def time_inference():
        for _ in range(3):
            sur.forward(xb, out=out)
        torch.cuda.synchronize()
        s0.record(stream)
        for _ in range(n_inf):
            sur.forward(xb, out=out)
        s1.record(stream)
        torch.cuda.synchronize()
        return s0.elapsed_time(s1) / n_inf

    ms_inf = time_inference()
    # the same parameters with the other arithmetic of the products
    sur.set_compute(not args.sur_bf16)
    other_err = err_on(xva, tva)
    ms_other = time_inference()
    sur.set_compute(bool(args.sur_bf16))
    # plain CWT at equal accuracy: the smallest truncation whose transmitted
    # coefficients are as close to the 15 x 15 reference as the surrogate's
    nq = args.sur_cwt_patches
    equal = (cwt_equal_accuracy(ctx, patches[n_tr:n_tr + nq], targets[n_tr:n_tr + nq], val_err)
             if nq > 0 else {"U": None, "sweep": []})
    full = (equal["sweep"][-1] if equal["sweep"] and equal["sweep"][-1]["U"] == 15 else None)
    # checked inference with the CWT fallback on 64 validation patches
    fell, chk, t_checked = None, None, None
    if args.sur_check:
        t2 = time.perf_counter()
        _, fell, chk = sur.infer_checked(patches[n_tr:n_tr + 64], n_check=32, seed=5, tol=1e-2)
        t_checked = time.perf_counter() - t2
    rate = 4096 / (ms_inf * 1e-3)
    mode, other = ("bf16", "fp32") if args.sur_bf16 else ("fp32", "bf16")
    log("surrogate (%s, %d training pairs): val rel-L2 %.3e; %.2f ms per 4096 = %.0f patches/s; "
        "%s products: val rel-L2 %.3e, %.2f ms" % (
            "trained weights" if trained else "short training", train_pairs, val_err, ms_inf,
            rate, other, other_err, ms_other))
    if equal.get("U"):
        log("plain CWT reaches rel-L2 %.3e at U = %d: %.2f patches/s (batched device solve); "
            "surrogate gain at equal accuracy %.0fx" % (
                equal["rel_l2"], equal["U"], equal["patches_per_s"],
                rate / equal["patches_per_s"]))
    if args.sur_check:
        log("checked inference, 64 patches, 32 solved by CWT: rel-L2 %.3e, fallback %s, "
            "%.1f s" % (chk, fell, t_checked))
    bpp = surrogate_bytes_per_patch(2 if args.sur_bf16 else 4)
    rec = {"products": mode, "storage": "bf16" if args.sur_bf16 else "fp32",
           "weights": os.path.relpath(args.sur_weights, ROOT) if trained else None,
           "train_pairs": train_pairs, "val_pairs": n_val, "train_steps": steps,
           "train_seconds": t_train, "training": trained, "rel_l2_val": val_err,
           "infer_batch": 4096, "infer_ms": ms_inf, "patches_per_s": rate,
           "roofline": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK / 1e9,
                        "achieved": bpp * rate / 1e9, "frac": bpp * rate / HBM_PEAK,
                        "traffic": (measured_surrogate_traffic() if args.sur_bf16 else None),
                        "measured_gbps": ((measured_surrogate_traffic() or 0) / (ms_inf * 1e-3)
                                          / 1e9 if args.sur_bf16 and measured_surrogate_traffic()
                                          else None),
                        "algorithmic_bytes_per_patch": bpp,
                        "direct_dft_flops_per_patch": surrogate_flops_per_patch(),
                        "direct_dft_tflops": surrogate_flops_per_patch() * rate / 1e12},
           "checked_batch": 64, "n_check": 32, "check_rel_l2": chk, "fallback_fired": fell,
           "checked_seconds": t_checked, "cwt_equal_accuracy": equal,
           "cwt_patches_per_s_full_band": full["patches_per_s"] if full else None,
           "other_products": {"products": other, "rel_l2_val": other_err, "infer_ms": ms_other,
                              "patches_per_s": 4096 / (ms_other * 1e-3)},
           "speedup_vs_cwt_equal_accuracy": (rate / equal["patches_per_s"]
                                             if equal.get("U") else None),
           "note": "CWT rates: patches solved together by scw_solve_batch (device eigensolver, "
                   "device elimination), setup included; fallback threshold 1e-2 rel-L2 on 32 "
                   "CWT-solved patches of the batch"}
    sur.free()
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16x3", "fp16x3"])
    ap.add_argument("--workload", default="working", choices=["working", "large"])
    ap.add_argument("--layers", type=int, default=None, help="keep only the first N layers")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--surrogate", type=int, default=1,
                    help="also train and time the spectral-convolution surrogate")
    ap.add_argument("--sur-epochs", type=int, default=400)
    ap.add_argument("--sur-batch", type=int, default=32)
    ap.add_argument("--sur-lr", type=float, default=2e-3)
    ap.add_argument("--sur-bf16", type=int, default=1,
                    help="surrogate matrix products in bf16 on the matrix cores with bf16 "
                         "storage (1, deployed) or FP32 (0)")
    ap.add_argument("--sur-weights", default=SUR_WEIGHTS,
                    help="trained surrogate weights (train_surrogate.py); '' trains briefly")
    ap.add_argument("--sur-cwt-patches", type=int, default=32,
                    help="validation patches solved by plain CWT for the equal-accuracy sweep "
                         "(0 skips it)")
    ap.add_argument("--sur-check", type=int, default=1,
                    help="run the checked inference (32 CWT samples of 64 patches)")
    ap.add_argument("--batched", type=int, default=1,
                    help="also time the batched spectral sweep (4096 jobs, one launch)")
    ap.add_argument("--large", type=int, default=1,
                    help="also time the 128x128x64 / M=961 / 512^2x256 workload in FP32, "
                         "BF16x3 and FP16x3")
    ap.add_argument("--variants", default="bf16x3,fp16x3",
                    help="other precisions timed in the same run ('' for none)")
    ap.add_argument("--tune", type=int, default=1,
                    help="run the library's autotuner before timing (0: built-in defaults)")
    ap.add_argument("--illuminations", default="8,16",
                    help="illumination counts timed on the working sample ('' for none)")
    ap.add_argument("--route-compare", type=int, default=1,
                    help="also solve the workload with the boundary elimination on the device")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run N plain 256 MiB device copies (PMC scale reference)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        return 2

    import torch
    import paper_2404_07293_amd as P
    import workloads as W

    prob, grid = W.random_field_config(args.workload, nz=args.layers)
    log("workload %s: sample %s, U=V=%d, grid %dx%dx%d, precision %s" % (
        args.workload, prob.n.shape, prob.U, grid.fx, grid.fy, grid.fz, args.precision))
    ctx = P.Context(0)
    t0 = time.perf_counter()
    sol = ctx.solve(prob)
    info = sol.info()
    log("setup %.1f s (eig %.1f s, boundary solve %.2f s), growth exponent %.1f" % (
        time.perf_counter() - t0, info["eig_seconds"], info["boundary_seconds"],
        info["growth_exponent"]))
    routes = None
    if args.route_compare:
        # the same setup with the boundary elimination on the device
        try:
            dsol = ctx.solve(prob, route="stable_device")
        except P.ScwError as e:
            dsol = None
            routes = {"stable_device": {"error": str(e)}}
            log("boundary solve on the device failed: %s" % e)
    if routes is None and args.route_compare:
        dinfo = dsol.info()
        hx, dx = sol.exterior(), dsol.exterior()
        diff = float(np.linalg.norm(dx[2] - hx[2]) / np.linalg.norm(hx[2]))
        routes = {"stable": {"setup_s": info["setup_seconds"],
                             "boundary_s": info["boundary_seconds"]},
                  "stable_device": {"setup_s": dinfo["setup_seconds"],
                                    "boundary_s": dinfo["boundary_seconds"]},
                  "p_trn_rel_diff": diff}
        log("boundary solve on the device: %.2f s (host %.2f s), setup %.1f s; p_trn "
            "rel diff %.1e" % (dinfo["boundary_seconds"], info["boundary_seconds"],
                               dinfo["setup_seconds"], diff))
        dsol.free()
        # the same setup with the eigendecompositions on the device
        try:
            esol = ctx.solve(prob, eig="device")
            einfo = esol.info()
            ediff = float(np.linalg.norm(esol.exterior()[2] - hx[2]) / np.linalg.norm(hx[2]))
            routes["eig_device"] = {"setup_s": einfo["setup_seconds"],
                                    "eig_s": einfo["eig_seconds"],
                                    "eig_s_host": info["eig_seconds"],
                                    "p_trn_rel_diff": ediff}
            log("eigendecompositions on the device: %.2f s (host %.2f s); p_trn rel diff %.1e"
                % (einfo["eig_seconds"], info["eig_seconds"], ediff))
            esol.free()
        except P.ScwError as e:
            routes["eig_device"] = {"error": str(e)}
            log("device eigensolver failed: %s" % e)

    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    dt = torch.complex128 if args.precision == "fp64" else torch.complex64
    E = torch.empty((3, grid.fz, grid.fy, grid.fx), dtype=dt, device=dev)
    tuning = {}
    if args.tune:
        tuning[args.precision] = sol.tune(grid, args.precision, out=E, stream=stream, reps=5)
        log("tuned %s: %s" % (args.precision, tuning[args.precision]))
    for _ in range(args.warmup):
        sol.synthesize(grid, args.precision, out=E, stream=stream)
    torch.cuda.synchronize()
    lib = ctx.lib
    import ctypes
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)

    def timed_loop(prec, out, steps):
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(steps):
            sol.synthesize(grid, prec, out=out, stream=stream)
        stop.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / steps

    # timed region: back-to-back synthesis calls on one stream
    ms = timed_loop(args.precision, E, args.steps)
    # per-kernel durations: the same loop again with HIP events recorded on the
    # synthesis stream around each kernel
    P._native.check(lib.scw_profile_begin(ctx.handle, args.steps))
    ms_marked = timed_loop(args.precision, E, args.steps)
    nst = 4
    stage_ms = (ctypes.c_double * nst)()
    calls = ctypes.c_int()
    P._native.check(lib.scw_profile_end(ctx.handle, stage_ms, nst, ctypes.byref(calls)))
    names = [lib.scw_stage_name(i).decode() for i in range(nst)]
    stages = {n: float(stage_ms[i]) for i, n in enumerate(names)}
    log("ms/step %.4f (with stage events %.4f); stages %s" % (
        ms, ms_marked, {k: round(v, 4) for k, v in stages.items()}))

    # each stage alone, back to back between two events (scw_synthesize_stages):
    # the kernel's average launch duration without the events between stages
    def stage_alone(stage):
        for _ in range(2):
            sol.synthesize_stages(grid, stage, out=E, precision=args.precision, stream=stream)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(args.steps):
            sol.synthesize_stages(grid, stage, out=E, precision=args.precision, stream=stream)
        stop.record(stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / args.steps

    alone = {"modal_sum": stage_alone("modal"), "idft": stage_alone("transform")}
    sol.synthesize(grid, args.precision, out=E, stream=stream)
    log("stages alone: %s" % {k: round(v, 4) for k, v in alone.items()})

    voxels = grid.fx * grid.fy * grid.fz
    value = voxels / (ms * 1e-3)
    err = golden_error(E, prob, grid)
    log("rel-L2 vs oracle samples: %s" % err)

    model = stage_model(info, plan_summary(prob, grid), args.precision)
    dom = max(stages, key=lambda k: stages[k])
    # the dominant kernel's duration: timed alone where it can run alone
    t = (alone.get(dom) or stages[dom]) * 1e-3
    by, fl = model[dom]["bytes"], model[dom]["flops"]
    fpeak = FP64_PEAK if args.precision == "fp64" else FP32_PEAK
    if by / HBM_PEAK >= fl / fpeak:
        roof = {"bound": "hbm", "achieved": by / t / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": fl / t / 1e12, "peak": fpeak / 1e12,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = dom
    roof["kernel_ms"] = t * 1e3
    roof["timing"] = ("the stage alone, %d back-to-back calls between two HIP events"
                      % args.steps if dom in alone else "HIP events between the stages")
    roof["traffic"] = measured_traffic(dom, args.precision, args.workload)
    roof["algorithmic_bytes"] = by
    roof["algorithmic_flops"] = fl
    # every stage, and the whole step, against the HBM roofline
    per_stage = {}
    # stages with a kernel in this configuration (the FP32 modal sum makes its
    # own phase factors, and an interior grid has no exterior planes)
    ran = [k for k in stages if not (k == "phase" and args.precision != "fp64")
           and (model[k]["bytes"] or model[k]["flops"])]
    for name in ran:
        t_ms = alone.get(name) or stages[name]
        b_, f_ = model[name]["bytes"], model[name]["flops"]
        if t_ms <= 0:
            continue
        per_stage[name] = {"ms": t_ms, "gbps": b_ / (t_ms * 1e-3) / 1e9,
                           "hbm_frac": b_ / (t_ms * 1e-3) / HBM_PEAK,
                           "tflops": f_ / (t_ms * 1e-3) / 1e12}
    tot_b = sum(model[k]["bytes"] for k in ran)
    roof_stage = {"stages": per_stage,
                  "step": {"ms": ms, "algorithmic_bytes": tot_b,
                           "gbps": tot_b / (ms * 1e-3) / 1e9,
                           "hbm_frac": tot_b / (ms * 1e-3) / HBM_PEAK,
                           "roofline_ms": tot_b / HBM_PEAK * 1e3}}

    if args.copy_calibration:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(args.copy_calibration):
            b.copy_(a)
        torch.cuda.synchronize()

    out = {
        "metric": METRIC, "value": value, "unit": "voxels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16x3": "bf16x3+f32acc",
                  "fp16x3": "fp16x3+f32acc"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "%s: %dx%dx%d random-field sample, M=%d, %dx%dx%d grid" % (
            args.workload, prob.nx, prob.ny, prob.nz, prob.U * prob.V, grid.fx, grid.fy,
            grid.fz), "precision": args.precision, "voxels_per_step": voxels},
        "rel_l2_vs_oracle": err,
        "stages_ms": stages,
        "stages_alone_ms": alone,
        "setup_s": info["setup_seconds"],
        "setup_routes": routes,
        "assembly_device_ms": info["assembly_device_ms"],
        "roofline": roof,
        "roofline_by_stage": roof_stage,
        "tuning": tuning,
    }
    if args.variants:
        variants = {}
        for prec in args.variants.split(","):
            Ev = torch.empty((3, grid.fz, grid.fy, grid.fx), dtype=torch.complex64, device=dev)
            if args.tune:
                tuning[prec] = sol.tune(grid, prec, out=Ev, stream=stream, reps=5)
                log("tuned %s: %s" % (prec, tuning[prec]))
            for _ in range(max(2, args.warmup)):
                sol.synthesize(grid, prec, out=Ev, stream=stream)
            vms = timed_loop(prec, Ev, args.steps)
            variants[prec] = {"value": voxels / (vms * 1e-3), "ms_per_step": vms,
                              "rel_l2_vs_oracle": golden_error(Ev, prob, grid),
                              "rel_l2_per_component": golden_error(Ev, prob, grid, True)}
            log("%s: ms/step %.4f rel-L2 %s" % (prec, vms, variants[prec]["rel_l2_vs_oracle"]))
            del Ev
        out["variants"] = variants
    if args.workload == "working" and args.precision == "fp32":
        out.setdefault("variants", {})["optics"] = optics_leg(sol, prob, grid, E, torch, dev,
                                                             stream, args)
        if args.illuminations:
            out["variants"]["illuminations"] = illumination_leg(ctx, prob, grid, ms, torch, dev,
                                                                stream, args)
    if args.workload == "working":
        out.setdefault("variants", {})["sphere_fp64"] = sphere_leg(ctx, torch, dev, stream, args)
    if args.large and args.workload == "working":
        out.setdefault("variants", {})["large"] = large_leg(ctx, torch, dev, stream, args)
    if args.surrogate and os.path.exists(SUR_DATA):
        out["surrogate"] = surrogate_leg(ctx, torch, dev, stream, args)
    if args.batched:
        out.setdefault("variants", {})["batched_sweep"] = batched_sweep(ctx, torch, dev, stream,
                                                                     args)
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(prob, grid)
    print(json.dumps(out), flush=True)
    sol.free()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
