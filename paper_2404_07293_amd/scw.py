"""Python binding of the HIP CWT library: argument marshalling only.

Every computation runs in libscw.so (HIP kernels on the GPU and the library's
own host FP64 setup). PyTorch supplies device memory for outputs and the
stream the synthesis is enqueued on.
"""
import ctypes

import numpy as np

from . import _native as N


def _ptr(a):
    return a.ctypes.data_as(N.c_dp) if a is not None else None


def _problem(prob, route, eig, keep):
    """A ctypes scw_problem for a ``workloads.Problem``; arrays it points to
    are appended to ``keep`` (the caller holds them through the call)."""
    n = np.ascontiguousarray(prob.n, dtype=np.complex128)
    keep.append(n)
    p = N.ScwProblem()
    p.nz, p.ny, p.nx = n.shape
    p.px, p.py, p.pz = float(prob.px), float(prob.py), float(prob.pz)
    p.n = _ptr(n)
    p.lam = float(prob.lam)
    p.n_top = float(prob.n_top)
    nb = complex(prob.n_bot)
    p.n_bot_re, p.n_bot_im = nb.real, nb.imag
    p.U, p.V = int(prob.U), int(prob.V)
    if prob.inc_ex is not None or prob.inc_ey is not None:
        ref = prob.inc_ex if prob.inc_ex is not None else prob.inc_ey
        p.inc_ny, p.inc_nx = ref.shape
        for name in ("inc_ex", "inc_ey"):
            img = getattr(prob, name)
            if img is not None:
                img = np.ascontiguousarray(img, dtype=np.complex128)
                keep.append(img)
                setattr(p, name, _ptr(img))
    pw = prob.plane_wave
    p.pw_u, p.pw_v = int(pw.u), int(pw.v)
    ex, ey = complex(pw.ex), complex(pw.ey)
    p.pw_ex[0], p.pw_ex[1] = ex.real, ex.imag
    p.pw_ey[0], p.pw_ey[1] = ey.real, ey.imag
    p.route = N.ROUTE[route]
    p.eig = N.EIG[eig]
    return p


class Context:
    """A library context on one HIP device (``scw_create``)."""

    def __init__(self, device=0, host_threads=0):
        self.lib = N.load()
        h = ctypes.c_void_p()
        N.check(self.lib.scw_create(ctypes.byref(h), int(device), int(host_threads)))
        self.handle = h
        self.device = int(device)

    def close(self):
        if self.handle:
            self.lib.scw_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def eig_batched(self, A, stream=None):
        """``scw_eig_batched`` on a CUDA complex128 tensor A [count, n, n]
        (each matrix as numpy/torch row-major A[i, j]; passed transposed so
        the library sees it column-major). Returns (w [count, n], X
        [count, n, n]) with A[b] @ X[b][:, j] = w[b, j] X[b][:, j]; A is
        left unchanged (the library works on a copy)."""
        import torch
        if A.dtype != torch.complex128 or A.dim() != 3 or A.shape[1] != A.shape[2]:
            raise ValueError("A must be a complex128 tensor [count, n, n]")
        count, n = int(A.shape[0]), int(A.shape[1])
        work = A.transpose(1, 2).contiguous()          # column-major per matrix
        w = torch.empty((count, n), dtype=torch.complex128, device=A.device)
        Xc = torch.empty((count, n, n), dtype=torch.complex128, device=A.device)
        if stream is None:
            stream = torch.cuda.current_stream(A.device)
        N.check(self.lib.scw_eig_batched(self.handle, n, count, ctypes.c_void_p(work.data_ptr()),
                                         ctypes.c_void_p(w.data_ptr()),
                                         ctypes.c_void_p(Xc.data_ptr()),
                                         ctypes.c_void_p(stream.cuda_stream)))
        return w, Xc.transpose(1, 2)

    def synthesize_composed(self, patches, px, py, grid, precision="fp32", out=None,
                            stream=None):
        """``scw_synthesize_composed``: the solutions ``patches`` (row-major,
        px x py) side by side, each over its own period, into ``out``
        [3, fz, py*fy, px*fx] (allocated when None)."""
        import torch
        if len(patches) != px * py:
            raise ValueError("need px * py patches")
        dt = torch.complex128 if precision == "fp64" else torch.complex64
        dev = torch.device("cuda", self.device)
        shape = (3, int(grid.fz), int(py) * int(grid.fy), int(px) * int(grid.fx))
        if out is None:
            out = torch.empty(shape, dtype=dt, device=dev)
        if tuple(out.shape) != shape or out.dtype != dt or not out.is_contiguous():
            raise ValueError("out must be a contiguous %s tensor of shape %s" % (dt, shape))
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        arr = (ctypes.c_void_p * len(patches))(*[p.handle for p in patches])
        N.check(self.lib.scw_synthesize_composed(self.handle, arr, int(px), int(py),
                                                 ctypes.byref(_grid(grid)),
                                                 N.PRECISION[precision],
                                                 ctypes.c_void_p(out.data_ptr()),
                                                 ctypes.c_void_p(stream.cuda_stream)))
        return out

    def solve_batch(self, probs, route="stable", eig="device"):
        """``scw_solve_batch``: solve the ``workloads.Problem`` list together
        (the device eigendecompositions of equal truncation share launches);
        returns one Solution per problem."""
        keep = []
        arr = (N.ScwProblem * len(probs))()
        for i, pr in enumerate(probs):
            arr[i] = _problem(pr, route, eig, keep)
        hs = (ctypes.c_void_p * len(probs))()
        N.check(self.lib.scw_solve_batch(self.handle, arr, len(probs), hs))
        return [Solution(self, ctypes.c_void_p(hs[i]), pr) for i, pr in enumerate(probs)]

    def solve(self, prob, route="stable", waves=None, eig="host"):
        """Run ``scw_solve`` on a ``workloads.Problem``; returns a Solution.
        With ``waves`` (a list of ``workloads.PlaneWave``) it runs
        ``scw_solve_illuminations`` instead: one illumination per wave, the
        problem's own incident field ignored. ``eig`` places the per-layer
        eigendecompositions: "host" (LAPACK) or "device" (the library's
        batched GPU eigensolver)."""
        keep = []
        p = _problem(prob, route, eig, keep)
        h = ctypes.c_void_p()
        if waves is None:
            N.check(self.lib.scw_solve(self.handle, ctypes.byref(p), ctypes.byref(h)))
            return Solution(self, h, prob)
        arr = (N.ScwPlaneWave * len(waves))()
        for i, w in enumerate(waves):
            ex, ey = complex(w.ex), complex(w.ey)
            arr[i].u, arr[i].v = int(w.u), int(w.v)
            arr[i].ex[0], arr[i].ex[1] = ex.real, ex.imag
            arr[i].ey[0], arr[i].ey[1] = ey.real, ey.imag
        N.check(self.lib.scw_solve_illuminations(self.handle, ctypes.byref(p), len(waves), arr,
                                                 ctypes.byref(h)))
        return Solution(self, h, prob, n_illuminations=len(waves))

    def batch(self, solutions, grid, precision="fp32"):
        """``scw_batch_plan`` over solved problems sharing one exterior grid."""
        arr = (ctypes.c_void_p * len(solutions))(*[s.handle.value for s in solutions])
        h = ctypes.c_void_p()
        N.check(self.lib.scw_batch_plan(self.handle, arr, len(solutions),
                                        ctypes.byref(_grid(grid)), N.PRECISION[precision],
                                        ctypes.byref(h)))
        return Batch(self, h, list(solutions), grid)


def _grid(grid):
    g = N.ScwGrid()
    g.fx, g.fy, g.fz = int(grid.fx), int(grid.fy), int(grid.fz)
    g.z_begin, g.z_end = float(grid.z_begin), float(grid.z_end)
    return g


class Solution:
    """A solved problem (``scw_solution``) living on the context's device."""

    def __init__(self, ctx, handle, prob, n_illuminations=1):
        self.ctx = ctx
        self.lib = ctx.lib
        self.handle = handle
        self.M = int(prob.U) * int(prob.V)
        self.n_illuminations = int(n_illuminations)

    def free(self):
        if self.handle:
            self.lib.scw_solution_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self):
        inf = N.ScwSolutionInfo()
        N.check(self.lib.scw_solution_info_get(self.handle, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in N.ScwSolutionInfo._fields_}

    def exterior(self):
        """(p_inc, p_ref, p_trn), each complex128 [3, M]."""
        out = [np.zeros(3 * self.M, np.complex128) for _ in range(3)]
        N.check(self.lib.scw_solution_exterior(self.handle, *[_ptr(a) for a in out]))
        return tuple(a.reshape(3, self.M) for a in out)

    def synthesis_bytes(self, grid, precision="fp32"):
        return self.lib.scw_synthesis_bytes(self.handle, ctypes.byref(_grid(grid)),
                                            N.PRECISION[precision])

    def _out(self, grid, precision, out, stream):
        import torch
        dt = torch.complex128 if precision == "fp64" else torch.complex64
        shape = (3, int(grid.fz), int(grid.fy), int(grid.fx))
        dev = torch.device("cuda", self.ctx.device)
        if out is None:
            out = torch.empty(shape, dtype=dt, device=dev)
        if tuple(out.shape) != shape or out.dtype != dt or not out.is_contiguous() \
                or out.device != dev:
            raise ValueError("out must be a contiguous %s tensor of shape %s on %s"
                             % (dt, shape, dev))
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        return out, stream

    def synthesize(self, grid, precision="fp32", out=None, stream=None):
        """Enqueue ``scw_synthesize`` into ``out`` (a CUDA tensor
        [3, fz, fy, fx]); allocates it when None. Returns the tensor."""
        out, stream = self._out(grid, precision, out, stream)
        N.check(self.lib.scw_synthesize(self.ctx.handle, self.handle,
                                        ctypes.byref(_grid(grid)), N.PRECISION[precision],
                                        ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(stream.cuda_stream)))
        return out

    def synthesize_tiled(self, grid, tx, ty, precision="fp32", out=None, stream=None):
        """Enqueue ``scw_synthesize_tiled``: the field over tx x ty lateral
        periods into ``out`` [3, fz, ty*fy, tx*fx] (allocated when None)."""
        import torch
        dt = torch.complex128 if precision == "fp64" else torch.complex64
        dev = torch.device("cuda", self.ctx.device)
        shape = (3, int(grid.fz), int(ty) * int(grid.fy), int(tx) * int(grid.fx))
        if out is None:
            out = torch.empty(shape, dtype=dt, device=dev)
        if tuple(out.shape) != shape or out.dtype != dt or not out.is_contiguous():
            raise ValueError("out must be a contiguous %s tensor of shape %s" % (dt, shape))
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        N.check(self.lib.scw_synthesize_tiled(self.ctx.handle, self.handle,
                                              ctypes.byref(_grid(grid)), int(tx), int(ty),
                                              N.PRECISION[precision],
                                              ctypes.c_void_p(out.data_ptr()),
                                              ctypes.c_void_p(stream.cuda_stream)))
        return out

    def synthesize_noalloc(self, grid, out, precision="fp32", stream=None):
        """Enqueue ``scw_synthesize_noalloc`` into the caller's ``out`` (a
        CUDA tensor [3, fz, fy, fx]): the library allocates nothing, its
        workspaces live in the device's static scratch array. Returns ``out``."""
        if out is None:
            raise ValueError("the allocation-free synthesis writes into a caller-owned out")
        out, stream = self._out(grid, precision, out, stream)
        N.check(self.lib.scw_synthesize_noalloc(self.ctx.handle, self.handle,
                                                ctypes.byref(_grid(grid)),
                                                N.PRECISION[precision],
                                                ctypes.c_void_p(out.data_ptr()),
                                                ctypes.c_void_p(stream.cuda_stream)))
        return out

    def synthesize_stages(self, grid, stages, out=None, precision="fp32", stream=None):
        """Enqueue ``scw_synthesize_stages``: only the named stages ("modal",
        "exterior", "transform", or a list of them) of the synthesis. The
        spectra stay in the plan's workspace between calls; ``out`` (allocated
        when None) is written only by the transform. Returns ``out``."""
        if isinstance(stages, str):
            stages = [stages]
        mask = 0
        for st in stages:
            mask |= N.STAGE[st]
        out, stream = self._out(grid, precision, out, stream)
        N.check(self.lib.scw_synthesize_stages(self.ctx.handle, self.handle,
                                               ctypes.byref(_grid(grid)),
                                               N.PRECISION[precision], mask,
                                               ctypes.c_void_p(out.data_ptr()),
                                               ctypes.c_void_p(stream.cuda_stream)))
        return out

    def synthesize_illuminations(self, grid, out=None, stream=None):
        """Enqueue ``scw_synthesize_illuminations`` (FP32): the field of every
        illumination into ``out`` [K, 3, fz, fy, fx] complex64, allocated
        when None. Returns the tensor."""
        import torch
        dev = torch.device("cuda", self.ctx.device)
        shape = (self.n_illuminations, 3, int(grid.fz), int(grid.fy), int(grid.fx))
        if out is None:
            out = torch.empty(shape, dtype=torch.complex64, device=dev)
        if tuple(out.shape) != shape or out.dtype != torch.complex64 \
                or not out.is_contiguous() or out.device != dev:
            raise ValueError("out must be a contiguous complex64 tensor of shape %s on %s"
                             % (shape, dev))
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        N.check(self.lib.scw_synthesize_illuminations(self.ctx.handle, self.handle,
                                                      ctypes.byref(_grid(grid)),
                                                      N.PRECISION["fp32"],
                                                      ctypes.c_void_p(out.data_ptr()),
                                                      ctypes.c_void_p(stream.cuda_stream)))
        return out

    def image(self, grid, na, precision="fp32", out=None, intensity=None, stream=None):
        """Enqueue ``scw_synthesize_image``: the field through an ideal
        objective of numerical aperture ``na`` into ``out`` [3, fz, fy, fx]
        and its intensity into ``intensity`` [fz, fy, fx] (float32, float64
        for "fp64"); both are allocated when None. Returns (out, intensity)."""
        import torch
        out, stream = self._out(grid, precision, out, stream)
        dt = torch.float64 if precision == "fp64" else torch.float32
        shape = (int(grid.fz), int(grid.fy), int(grid.fx))
        if intensity is None:
            intensity = torch.empty(shape, dtype=dt, device=out.device)
        if tuple(intensity.shape) != shape or intensity.dtype != dt \
                or not intensity.is_contiguous() or intensity.device != out.device:
            raise ValueError("intensity must be a contiguous %s tensor of shape %s on %s"
                             % (dt, shape, out.device))
        N.check(self.lib.scw_synthesize_image(self.ctx.handle, self.handle,
                                              ctypes.byref(_grid(grid)), N.PRECISION[precision],
                                              float(na), ctypes.c_void_p(out.data_ptr()),
                                              ctypes.c_void_p(intensity.data_ptr()),
                                              ctypes.c_void_p(stream.cuda_stream)))
        return out, intensity

    def filtered(self, grid, H, precision="fp32", out=None, intensity=None, stream=None):
        """Enqueue ``scw_synthesize_filtered``: the field with the transfer
        function ``H`` (M complex values in mode order, numpy or torch)
        applied to every plane's spectrum, into ``out`` [3, fz, fy, fx], and
        its intensity into ``intensity`` [fz, fy, fx]; both allocated when
        None. Returns (out, intensity)."""
        import torch
        out, stream = self._out(grid, precision, out, stream)
        dt = torch.float64 if precision == "fp64" else torch.float32
        shape = (int(grid.fz), int(grid.fy), int(grid.fx))
        if intensity is None:
            intensity = torch.empty(shape, dtype=dt, device=out.device)
        if tuple(intensity.shape) != shape or intensity.dtype != dt \
                or not intensity.is_contiguous() or intensity.device != out.device:
            raise ValueError("intensity must be a contiguous %s tensor of shape %s on %s"
                             % (dt, shape, out.device))
        h = torch.as_tensor(H).to(device=out.device, dtype=torch.complex128).contiguous()
        if h.numel() != self.info()["M"]:
            raise ValueError("H must hold one value per mode (%d)" % self.info()["M"])
        self._transfer = h  # stays alive while the enqueued kernels may read it
        N.check(self.lib.scw_synthesize_filtered(self.ctx.handle, self.handle,
                                                 ctypes.byref(_grid(grid)),
                                                 N.PRECISION[precision],
                                                 ctypes.c_void_p(h.data_ptr()),
                                                 ctypes.c_void_p(out.data_ptr()),
                                                 ctypes.c_void_p(intensity.data_ptr()),
                                                 ctypes.c_void_p(stream.cuda_stream)))
        return out, intensity

    def synthesize_slice(self, axis, position, n, fz, z_begin, z_end, precision="fp32",
                         out=None, stream=None):
        """Enqueue ``scw_synthesize_slice``: the field on an x-z ("xz", at
        y = position) or y-z ("yz", at x = position) plane with n lateral
        samples and fz planes over [z_begin, z_end), into ``out`` (a CUDA
        tensor [3, fz, n]; allocated when None). Returns the tensor."""
        import torch
        if precision not in ("fp32", "fp64"):
            raise ValueError("a slice is synthesized in fp32 or fp64")
        dt = torch.complex128 if precision == "fp64" else torch.complex64
        dev = torch.device("cuda", self.ctx.device)
        shape = (3, int(fz), int(n))
        if out is None:
            out = torch.empty(shape, dtype=dt, device=dev)
        if tuple(out.shape) != shape or out.dtype != dt or not out.is_contiguous() \
                or out.device != dev:
            raise ValueError("out must be a contiguous %s tensor of shape %s on %s"
                             % (dt, shape, dev))
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        sl = N.ScwSlice(N.SLICE_AXIS[axis], float(position), int(n), int(fz), float(z_begin),
                        float(z_end))
        N.check(self.lib.scw_synthesize_slice(self.ctx.handle, self.handle, ctypes.byref(sl),
                                              N.PRECISION[precision],
                                              ctypes.c_void_p(out.data_ptr()),
                                              ctypes.c_void_p(stream.cuda_stream)))
        return out

    def configure(self, modal_rows=0, transform="auto", fft_radix=0, tiles=0):
        """``scw_synthesis_configure``: explicit kernel configuration (0 /
        "auto" fields leave the library's choice)."""
        cfg = N.ScwSynthConfig(int(modal_rows), N.TRANSFORM[transform], int(fft_radix),
                               int(tiles))
        N.check(self.lib.scw_synthesis_configure(self.handle, ctypes.byref(cfg)))

    def tune(self, grid, precision="fp32", out=None, stream=None, reps=5):
        """``scw_tune_synthesis``: time the kernel configurations for this
        grid and precision and keep the fastest. Returns the report as a dict;
        ``out`` holds the field afterwards."""
        out, stream = self._out(grid, precision, out, stream)
        rep = N.ScwTuneReport()
        N.check(self.lib.scw_tune_synthesis(self.ctx.handle, self.handle,
                                            ctypes.byref(_grid(grid)), N.PRECISION[precision],
                                            ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(stream.cuda_stream), int(reps),
                                            ctypes.byref(rep)))
        c = rep.config
        return {"n_candidates": rep.n_candidates, "default_ms": rep.default_ms,
                "best_ms": rep.best_ms, "modal_rows": c.modal_rows,
                "transform": N.TRANSFORM_NAME.get(c.transform, "?"),
                "fft_radix": c.fft_radix, "tiles": c.tiles}


class Batch:
    """A planned batched synthesis (``scw_batch``); keeps its jobs alive."""

    def __init__(self, ctx, handle, jobs, grid):
        self.ctx = ctx
        self.lib = ctx.lib
        self.handle = handle
        self.jobs = jobs
        self.grid = grid

    def free(self):
        if self.handle:
            self.lib.scw_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def _out(self, out, stream):
        import torch
        g = self.grid
        shape = (len(self.jobs), 3, int(g.fz), int(g.fy), int(g.fx))
        dev = torch.device("cuda", self.ctx.device)
        if out is None:
            out = torch.empty(shape, dtype=torch.complex64, device=dev)
        if tuple(out.shape) != shape or out.dtype != torch.complex64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous complex64 tensor of shape %s" % (shape,))
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        return out, stream

    def launch(self, out=None, stream=None):
        """Replay the batch graph into ``out`` [njobs, 3, fz, fy, fx] complex64."""
        out, stream = self._out(out, stream)
        N.check(self.lib.scw_batch_launch(self.handle, ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(stream.cuda_stream)))
        return out

    def configure(self, radix, blocks_per_cu, chunk):
        """``scw_batch_configure``: set the persistent kernel's shape."""
        N.check(self.lib.scw_batch_configure(self.handle, int(radix), int(blocks_per_cu),
                                             int(chunk)))

    def tune(self, out=None, stream=None, reps=3):
        """``scw_batch_tune``: sweep the persistent kernel's shapes and keep
        the fastest. Returns the report as a dict."""
        out, stream = self._out(out, stream)
        rep = N.ScwTuneReport()
        N.check(self.lib.scw_batch_tune(self.handle, ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(stream.cuda_stream), int(reps),
                                        ctypes.byref(rep)))
        return {"n_candidates": rep.n_candidates, "default_ms": rep.default_ms,
                "best_ms": rep.best_ms, "radix": rep.batch_radix,
                "blocks_per_cu": rep.batch_blocks_per_cu, "chunk": rep.batch_chunk}
