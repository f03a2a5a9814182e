"""Learned warm start: the network of ``dtm_mlp_*`` (include/dtm.h) driven
from Python.  Every arithmetic step runs in the HIP library; this module
allocates the workspace, initialises the weights, loops over mini-batches
and saves / restores checkpoints.

Typical use::

    net = WarmStartMLP(max_batch=1024, seed=0)
    (feat, shift), prior = net.features(scenes), net.flux_prior(scenes)
    net.fit(feat, targets, epochs=20, prior=prior, shift=shift)   # targets: P x 1024 (device)
    x0 = net.predict(feat, prior, shift)             # P x 1024 float32, rows sum to 1
    plan.solve(pi, infos, x0=x0.reshape(-1))         # uniform fallback is automatic

With ``prior`` (the log of the flux start lambda / sum(lambda), see
``dtm_mlp_flux_prior``) the network's logits are added to it, so it learns a
correction to the solver's flux start; without it, the whole PDF.  With
``shift`` (each scene's pulse bin) the network's outputs are rotated to
start at that bin, so it learns in a frame centred on the pulse.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import dtm

IN, IN_PAD, HIDDEN, OUT = 5, 16, 256, 1024
MAX_BATCH = 65536


class Layout(ctypes.Structure):
    _fields_ = [
        ("params", ctypes.c_size_t), ("params_bf16", ctypes.c_size_t), ("grads", ctypes.c_size_t),
        ("adam_m", ctypes.c_size_t), ("adam_v", ctypes.c_size_t), ("act", ctypes.c_size_t),
        ("partial", ctypes.c_size_t), ("total", ctypes.c_size_t),
        ("off_w1", ctypes.c_int64), ("off_b1", ctypes.c_int64), ("off_w2", ctypes.c_int64),
        ("off_b2", ctypes.c_int64), ("off_w3", ctypes.c_int64), ("off_b3", ctypes.c_int64),
        ("n_params", ctypes.c_int64), ("max_batch", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_F = ctypes.c_float
_bound = False


def _bind():
    global _bound
    if _bound:
        return dtm.lib()
    L = dtm.lib()
    sig = {
        "dtm_mlp_workspace_layout": (ctypes.c_int, [_I32, ctypes.POINTER(Layout)]),
        "dtm_mlp_features": (ctypes.c_int, [_P, _I32, _P, _P, _P]),
        "dtm_mlp_sync_bf16": (ctypes.c_int, [_P, _I32, _P]),
        "dtm_mlp_flux_prior": (ctypes.c_int, [_P, _I32, _P, _P]),
        "dtm_mlp_forward": (ctypes.c_int, [_P, _I32, _P, _P, _P, _I32, _P, _P]),
        "dtm_mlp_backward": (ctypes.c_int, [_P, _I32, _P, _P, _P, _P, _P, _I32, _P, _P]),
        "dtm_mlp_adam": (ctypes.c_int, [_P, _I32, _F, _F, _F, _F, _I32, _P]),
        "dtm_mlp_gemm_bf16": (ctypes.c_int, [_I32, _I32, _I32, _P, _I32, _I32, _P, _I32, _I32, _P,
                                             _I32, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _bound = True
    return L


def layout(max_batch):
    out = Layout()
    dtm.check(_bind().dtm_mlp_workspace_layout(max_batch, ctypes.byref(out)), "dtm_mlp_workspace_layout")
    return out


def gemm_bf16(A, B, trans_a=False, trans_b=False, stream=None):
    """C = op(A) op(B) through the library's MFMA GEMM (A, B int16 tensors
    holding bfloat16 bits, row-major); returns float32 C."""
    import torch
    M = A.shape[1] if trans_a else A.shape[0]
    K = A.shape[0] if trans_a else A.shape[1]
    N = B.shape[0] if trans_b else B.shape[1]
    C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    dtm.check(_bind().dtm_mlp_gemm_bf16(M, N, K, A.data_ptr(), A.stride(0), int(trans_a), B.data_ptr(),
                                        B.stride(0), int(trans_b), C.data_ptr(), C.stride(0),
                                        dtm._stream(stream)), "dtm_mlp_gemm_bf16")
    return C


def solve_targets(scenes, dtype="f32", chunk=16384, solve_opts=None, x0=None):
    """Stationary PDFs of many pixels with the batched solver, in chunks so the
    dense matrices of one chunk at a time sit in HBM.  Returns (pi as a P x n
    tensor for equal n, or the packed vector otherwise; SolveInfo records)."""
    import torch
    outs, infos = [], []
    ws = None
    n_all = np.asarray(scenes["n_bins"])
    for a in range(0, len(scenes), chunk):
        s = scenes[a:a + chunk]
        plan = dtm.Plan(s, dtype, solve_opts or dtm.opts(tol=1e-6))
        try:
            if ws is None or ws.numel() < plan.workspace_bytes:
                ws = None
                ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
            plan.bind(ws)
            tdt = torch.float32 if plan.dtype == dtm.DTM_F32 else torch.float64
            pi = torch.empty(plan.pi_elems, dtype=tdt, device="cuda")
            inf = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
            xa = None
            if x0 is not None:
                off = int(np.sum(n_all[:a]))
                xa = x0[off:off + plan.pi_elems]
            plan.solve(pi, inf, xa)
            torch.cuda.synchronize()
            outs.append(pi)
            infos.append(dtm.infos_to_numpy(inf))
        finally:
            plan.close()
    pi = torch.cat(outs)
    if np.all(n_all == n_all[0]):
        pi = pi.view(len(scenes), int(n_all[0]))
    return pi, np.concatenate(infos)


class WarmStartMLP:
    """zero_output: start with a zero output layer, so that with a prior the
    untrained network predicts the prior itself (the flux start)."""

    def __init__(self, max_batch=1024, seed=0, device="cuda", zero_output=False):
        import torch
        if not 1 <= max_batch <= MAX_BATCH:
            raise ValueError("max_batch out of range")
        _bind()
        self.max_batch = max_batch
        self.L = layout(max_batch)
        self.ws = torch.zeros(self.L.total, dtype=torch.uint8, device=device)
        self.step = 0
        self.init_weights(seed, zero_output)

    # ---- views into the workspace -------------------------------------------
    def _f32(self, byte_off, n):
        return self.ws[byte_off:byte_off + 4 * n].view(dtype=__import__("torch").float32)

    @property
    def params(self):
        return self._f32(self.L.params, self.L.n_params)

    @property
    def grads(self):
        return self._f32(self.L.grads, self.L.n_params)

    def tensors(self, flat):
        """Split a flat parameter-shaped vector into W1 (16x256), b1, W2, b2, W3, b3."""
        L = self.L
        return {
            "W1": flat[L.off_w1:L.off_b1].view(IN_PAD, HIDDEN), "b1": flat[L.off_b1:L.off_w2],
            "W2": flat[L.off_w2:L.off_b2].view(HIDDEN, HIDDEN), "b2": flat[L.off_b2:L.off_w3],
            "W3": flat[L.off_w3:L.off_b3].view(HIDDEN, OUT), "b3": flat[L.off_b3:L.n_params],
        }

    def init_weights(self, seed, zero_output=False):
        """Uniform(+-1/sqrt(fan_in)) weights (W3 zero with zero_output), zero
        biases, zero Adam moments (seeded NumPy PCG64); padded input rows of
        W1 stay zero."""
        import torch
        rng = np.random.default_rng(seed)
        flat = np.zeros(self.L.n_params, dtype=np.float32)
        L = self.L
        for off, fan_in, rows, cols in ((L.off_w1, IN, IN_PAD, HIDDEN), (L.off_w2, HIDDEN, HIDDEN, HIDDEN),
                                        (L.off_w3, HIDDEN, HIDDEN, OUT)):
            w = np.zeros((rows, cols), dtype=np.float32)
            a = 1.0 / math.sqrt(fan_in)
            w[:fan_in] = rng.uniform(-a, a, (fan_in, cols))
            if zero_output and off == L.off_w3:
                w[:] = 0.0
            flat[off:off + rows * cols] = w.ravel()
        self.params.copy_(torch.from_numpy(flat))
        self._f32(self.L.adam_m, self.L.n_params).zero_()
        self._f32(self.L.adam_v, self.L.n_params).zero_()
        self.step = 0
        self.sync()

    def sync(self, stream=None):
        dtm.check(_bind().dtm_mlp_sync_bf16(self.ws.data_ptr(), self.max_batch, dtm._stream(stream)),
                  "dtm_mlp_sync_bf16")

    # ---- network ----------------------------------------------------------------
    def features(self, scenes, stream=None):
        """(phi of each scene as P x 5 float32, each scene's pulse bin as P
        int32), both on the device and computed on the GPU."""
        import torch
        arr = np.ascontiguousarray(scenes)
        raw = torch.from_numpy(arr.view(np.uint8).copy()).to(self.ws.device)
        feat = torch.empty((arr.size, IN), dtype=torch.float32, device=self.ws.device)
        shift = torch.empty(arr.size, dtype=torch.int32, device=self.ws.device)
        dtm.check(_bind().dtm_mlp_features(raw.data_ptr(), arr.size, feat.data_ptr(), shift.data_ptr(),
                                           dtm._stream(stream)), "dtm_mlp_features")
        return feat, shift

    def flux_prior(self, scenes, stream=None):
        """log(lambda_j / sum lambda) at the 1024 bin centres of each scene
        (P x 1024 float32 on the device), computed on the GPU."""
        import torch
        arr = np.ascontiguousarray(scenes)
        raw = torch.from_numpy(arr.view(np.uint8).copy()).to(self.ws.device)
        prior = torch.empty((arr.size, OUT), dtype=torch.float32, device=self.ws.device)
        dtm.check(_bind().dtm_mlp_flux_prior(raw.data_ptr(), arr.size, prior.data_ptr(), dtm._stream(stream)),
                  "dtm_mlp_flux_prior")
        return prior

    def predict(self, feat, prior=None, shift=None, stream=None):
        """softmax(rotate(network(feat), shift) + prior) for any number of
        rows, in max_batch chunks (prior: P x 1024 float32, shift: P int32;
        either may be None)."""
        import torch
        P = feat.shape[0]
        out = torch.empty((P, OUT), dtype=torch.float32, device=self.ws.device)
        for a in range(0, P, self.max_batch):
            b = min(P, a + self.max_batch)
            dtm.check(_bind().dtm_mlp_forward(self.ws.data_ptr(), self.max_batch, feat[a:b].data_ptr(),
                                              None if prior is None else prior[a:b].data_ptr(),
                                              None if shift is None else shift[a:b].data_ptr(),
                                              b - a, out[a:b].data_ptr(), dtm._stream(stream)),
                      "dtm_mlp_forward")
        return out

    def backward(self, feat, target, loss=None, prior=None, shift=None, rows=None, stream=None):
        """Gradients of the mean cross-entropy into ``grads`` (one batch: the
        rows ``rows`` (int32 on the device) of feat, target, prior and shift,
        or all of their rows)."""
        B = feat.shape[0] if rows is None else rows.shape[0]
        dtm.check(_bind().dtm_mlp_backward(self.ws.data_ptr(), self.max_batch, feat.data_ptr(),
                                           None if prior is None else prior.data_ptr(),
                                           None if shift is None else shift.data_ptr(),
                                           target.data_ptr(), None if rows is None else rows.data_ptr(),
                                           B, None if loss is None else loss.data_ptr(),
                                           dtm._stream(stream)), "dtm_mlp_backward")

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step += 1
        dtm.check(_bind().dtm_mlp_adam(self.ws.data_ptr(), self.max_batch, lr, beta1, beta2, eps, self.step,
                                       dtm._stream(stream)), "dtm_mlp_adam")

    def fit(self, feat, target, epochs=20, lr=1e-3, seed=0, log=None, prior=None, shift=None):
        """Adam with cosine-decayed learning rate over shuffled mini-batches
        of max_batch rows (prior: P x 1024 prior logits, shift: P pulse bins;
        either may be None); returns the mean loss of each epoch."""
        import torch
        P = feat.shape[0]
        B = self.max_batch
        nb = P // B
        if nb < 1:
            raise ValueError("need at least one full batch")
        total = epochs * nb
        g = torch.Generator(device="cpu")
        g.manual_seed(seed)
        loss = torch.empty(nb * B, dtype=torch.float32, device=self.ws.device)
        hist = []
        for ep in range(epochs):
            # the shuffle is drawn on the host; the library reads each
            # mini-batch's rows in place
            perm = torch.randperm(P, generator=g).to(dtype=torch.int32, device=self.ws.device)
            for b in range(nb):
                self.backward(feat, target, loss[b * B:(b + 1) * B], prior=prior, shift=shift,
                              rows=perm[b * B:(b + 1) * B])
                t = self.step / max(1, total - 1)
                self.adam(lr * 0.5 * (1.0 + math.cos(math.pi * min(1.0, t))))
            hist.append(float(loss.cpu().numpy().astype(np.float64).mean()))
            if log:
                log(ep, hist[-1])
        return hist

    # ---- checkpoints -------------------------------------------------------------
    def state_dict(self):
        L = self.L
        return {
            "params": self.params.detach().cpu().clone(),
            "adam_m": self._f32(L.adam_m, L.n_params).detach().cpu().clone(),
            "adam_v": self._f32(L.adam_v, L.n_params).detach().cpu().clone(),
            "step": self.step,
        }

    def load_state_dict(self, sd):
        L = self.L
        self.params.copy_(sd["params"])
        self._f32(L.adam_m, L.n_params).copy_(sd["adam_m"])
        self._f32(L.adam_v, L.n_params).copy_(sd["adam_v"])
        self.step = int(sd["step"])
        self.sync()
