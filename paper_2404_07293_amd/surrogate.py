"""Binding of the spectral-convolution surrogate (``scw_sur_*``): argument
marshalling only. Training, inference, gradients and the CWT fallback run in
libscw.so."""
import ctypes

import numpy as np

from . import _native as N

PATCH_SHAPE = (8, 32, 32)
OUT_SHAPE = (3, 15, 15)


class Surrogate:
    def __init__(self, ctx, max_batch=4096, seed=0):
        self.ctx = ctx
        self.lib = ctx.lib
        h = ctypes.c_void_p()
        N.check(self.lib.scw_sur_create(ctx.handle, int(max_batch), int(seed), ctypes.byref(h)))
        self.handle = h
        self.max_batch = int(max_batch)
        self.n_params = int(self.lib.scw_sur_param_count())

    def free(self):
        if self.handle:
            self.lib.scw_sur_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def get_params(self):
        p = np.empty(self.n_params, np.float32)
        N.check(self.lib.scw_sur_get_params(self.handle, p.ctypes.data_as(ctypes.c_void_p)))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.n_params
        N.check(self.lib.scw_sur_set_params(self.handle, p.ctypes.data_as(ctypes.c_void_p)))

    def set_compute(self, bf16):
        """``scw_sur_set_compute``: bf16 matrix-core products (True) or FP32
        vector products (False)."""
        N.check(self.lib.scw_sur_set_compute(self.handle, 1 if bf16 else 0))

    def _stream(self, stream):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(torch.device("cuda", self.ctx.device))
        return ctypes.c_void_p(stream.cuda_stream)

    def encode(self, n_patches, stream=None):
        """complex patches (numpy [B][8][32][32] or CUDA complex64 tensor) ->
        encoded float inputs (CUDA tensor [B][16][32][32])."""
        import torch
        dev = torch.device("cuda", self.ctx.device)
        t = torch.as_tensor(n_patches).to(dev, torch.complex64).contiguous()
        B = t.shape[0]
        x = torch.empty((B, 16, 32, 32), dtype=torch.float32, device=dev)
        N.check(self.lib.scw_sur_encode(self.handle, ctypes.c_void_p(t.data_ptr()), B,
                                        ctypes.c_void_p(x.data_ptr()), self._stream(stream)))
        return x

    def forward(self, x, out=None, stream=None):
        import torch
        B = x.shape[0]
        if out is None:
            out = torch.empty((B,) + OUT_SHAPE, dtype=torch.complex64, device=x.device)
        N.check(self.lib.scw_sur_forward(self.handle, ctypes.c_void_p(x.data_ptr()), B,
                                         ctypes.c_void_p(out.data_ptr()), self._stream(stream)))
        return out

    def loss_grad(self, x, target, stream=None):
        """(loss, flat FP32 gradient) for one batch."""
        g = np.empty(self.n_params, np.float32)
        loss = ctypes.c_double()
        N.check(self.lib.scw_sur_loss_grad(self.handle, ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(target.data_ptr()), x.shape[0],
                                           ctypes.byref(loss), g.ctypes.data_as(ctypes.c_void_p),
                                           self._stream(stream)))
        return loss.value, g

    def train_step(self, x, target, lr=1e-3, want_loss=True, stream=None):
        loss = ctypes.c_double()
        N.check(self.lib.scw_sur_train_step(self.handle, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(target.data_ptr()), x.shape[0],
                                            ctypes.c_float(lr),
                                            ctypes.byref(loss) if want_loss else None,
                                            self._stream(stream)))
        return loss.value if want_loss else None

    def infer_checked(self, n_patches, n_check=32, seed=0, tol=1e-2):
        """(outputs complex128 [B][3][15][15], fell_back, check rel-L2)."""
        n = np.ascontiguousarray(n_patches, dtype=np.complex128)
        B = n.shape[0]
        out = np.empty((B,) + OUT_SHAPE, np.complex128)
        fb = ctypes.c_int()
        err = ctypes.c_double()
        N.check(self.lib.scw_sur_infer_checked(self.ctx.handle, self.handle,
                                               n.ctypes.data_as(N.c_dp), B, int(n_check),
                                               int(seed), float(tol), out.ctypes.data_as(N.c_dp),
                                               ctypes.byref(fb), ctypes.byref(err)))
        return out, bool(fb.value), err.value


def cwt_targets(ctx, patches, eig="host", chunk=256, route="stable"):
    """Transmitted coefficients [B][3][15][15] of each patch by plain CWT, for
    training data and checks: one ``scw_solve`` per patch with the host
    eigensolver, or, with eig="device", ``scw_solve_batch`` over chunks of
    patches whose eigendecompositions share the device eigensolver's launches
    (route "stable_device" also keeps the boundary systems on the device)."""
    import workloads as W
    out = np.empty((len(patches),) + OUT_SHAPE, np.complex128)
    if eig == "device":
        for c0 in range(0, len(patches), chunk):
            probs = [W.surrogate_problem(n) for n in patches[c0:c0 + chunk]]
            for i, sol in enumerate(ctx.solve_batch(probs, route=route, eig="device")):
                out[c0 + i] = sol.exterior()[2].reshape(OUT_SHAPE)
                sol.free()
        return out
    for i, n in enumerate(patches):
        prob = W.surrogate_problem(n)
        sol = ctx.solve(prob)
        out[i] = sol.exterior()[2].reshape(OUT_SHAPE)
        sol.free()
    return out
