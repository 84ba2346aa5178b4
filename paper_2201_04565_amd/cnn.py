"""Python binding of the surrogate network in liblsm.so (marshalling only).

Forward, loss, backward and Adam all run in the library's HIP kernels on
device buffers; torch provides the workspace, the batch buffers and the
stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import lsm as _lsm

CNN_EXPORTS = (
    "lsm_cnn_create", "lsm_cnn_destroy", "lsm_cnn_last_error", "lsm_cnn_param_count",
    "lsm_cnn_layout", "lsm_cnn_workspace_bytes", "lsm_cnn_bind", "lsm_cnn_set_params",
    "lsm_cnn_get_params", "lsm_cnn_get_grads", "lsm_cnn_forward", "lsm_cnn_mse", "lsm_cnn_mse_noalloc",
    "lsm_cnn_backward", "lsm_cnn_adam_step", "lsm_cnn_conv_forward", "lsm_cnn_read_buffer",
)

# internal buffers readable by Network.buffer (LSM_CNN_BUF_* of lsm.h):
# name -> (id, element type, BF16 stored as uint16)
BUFFERS = {"pooled": (0, np.uint16), "mask": (1, np.uint8), "act": (2, np.uint16),
           "dact": (3, np.uint16), "dpool0": (4, np.uint16), "gap": (5, np.float32),
           "dgap": (6, np.float32), "hidden": (7, np.float32), "dhidden": (8, np.float32),
           "out": (9, np.float32), "dout": (10, np.float32)}

DEFAULT_CHANNELS = (32, 64, 128, 128, 256)


class CnnConfig(C.Structure):
    _fields_ = [("batch", C.c_int32), ("height", C.c_int32), ("width", C.c_int32),
                ("channels", C.c_int32 * 5), ("hidden", C.c_int32), ("outputs", C.c_int32)]


def _load():
    L = _lsm.load_library()
    if getattr(L, "_cnn_ready", False):
        return L
    vp, i64, fl = C.c_void_p, C.c_int64, C.c_float
    P = C.POINTER
    L.lsm_cnn_create.argtypes = [P(CnnConfig), P(vp)]
    L.lsm_cnn_destroy.argtypes = [vp]
    L.lsm_cnn_destroy.restype = None
    L.lsm_cnn_last_error.argtypes = [vp]
    L.lsm_cnn_last_error.restype = C.c_char_p
    L.lsm_cnn_param_count.argtypes = [vp, P(i64)]
    L.lsm_cnn_layout.argtypes = [vp, vp, vp, vp]
    L.lsm_cnn_workspace_bytes.argtypes = [vp, P(C.c_size_t)]
    L.lsm_cnn_bind.argtypes = [vp, vp, C.c_size_t, vp]
    for nm in ("lsm_cnn_set_params", "lsm_cnn_get_params", "lsm_cnn_get_grads"):
        getattr(L, nm).argtypes = [vp, vp]
    L.lsm_cnn_forward.argtypes = [vp, vp, i64, vp]
    L.lsm_cnn_mse.argtypes = [vp, vp, vp, vp]
    L.lsm_cnn_mse_noalloc.argtypes = [vp, vp, vp, vp]
    L.lsm_cnn_backward.argtypes = [vp, vp]
    L.lsm_cnn_adam_step.argtypes = [vp, fl, fl, fl, fl, i64]
    L.lsm_cnn_conv_forward.argtypes = [vp, C.c_int, vp, vp, i64]
    L.lsm_cnn_read_buffer.argtypes = [vp, C.c_int, C.c_int, vp, P(C.c_size_t)]
    L._cnn_ready = True
    return L


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Network:
    """One surrogate network bound to its own device workspace."""

    def __init__(self, size=128, batch=512, channels=DEFAULT_CHANNELS, hidden=256, outputs=65,
                 device="cuda:0", stream=None):
        import torch

        self.torch = torch
        L = _load()
        self._L = L
        self._h = None
        cfg = CnnConfig(batch, size, size, (C.c_int32 * 5)(*channels), hidden, outputs)
        h = C.c_void_p()
        rc = L.lsm_cnn_create(C.byref(cfg), C.byref(h))
        if rc != 0:
            raise _lsm.LsmError(rc, L.lsm_strerror(rc).decode())
        self._h = h
        self.size, self.batch, self.channels = size, batch, tuple(channels)
        self.hidden, self.outputs = hidden, outputs
        n = C.c_int64()
        L.lsm_cnn_param_count(h, C.byref(n))
        self.n_params = n.value
        nb = C.c_size_t()
        self._check(L.lsm_cnn_workspace_bytes(h, C.byref(nb)))
        self.device = torch.device(device)
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        # default: torch's current stream, so results are ordered with the
        # caller's own torch work; another stream is synchronised both ways
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._check(L.lsm_cnn_bind(h, _dptr(self.workspace), nb.value,
                                   C.c_void_p(self.stream.cuda_stream)))
        self.y = torch.empty((batch, outputs), dtype=torch.float32, device=self.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.t = 0

    def _check(self, rc):
        if rc != 0:
            msg = self._L.lsm_cnn_last_error(self._h).decode() if self._h else ""
            raise _lsm.LsmError(rc, f"{self._L.lsm_strerror(rc).decode()}: {msg}")

    def close(self):
        if self._h is not None and self._h.value:
            self._L.lsm_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- parameters
    def layout(self):
        wo = np.zeros(7, np.int64)
        bo = np.zeros(7, np.int64)
        wn = np.zeros(7, np.int64)
        self._check(self._L.lsm_cnn_layout(self._h, wo.ctypes.data_as(C.c_void_p),
                                           bo.ctypes.data_as(C.c_void_p),
                                           wn.ctypes.data_as(C.c_void_p)))
        return wo, bo, wn

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.n_params
        self._check(self._L.lsm_cnn_set_params(self._h, p.ctypes.data_as(C.c_void_p)))
        self.t = 0

    def params(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        self._check(self._L.lsm_cnn_get_params(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def grads(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        self._check(self._L.lsm_cnn_get_grads(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    # ------------------------------------------------------------- compute
    def _enter(self):
        # inputs produced on torch's current stream must be ready on ours
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _leave(self, *inputs):
        # outputs must be ready for the caller's stream, and inputs must not
        # be recycled by the caching allocator while our stream reads them
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)
            for t in inputs:
                if t is not None:
                    t.record_stream(self.stream)

    def forward(self, x_u8):
        """x_u8: uint8 CUDA tensor [B, size, size] -> FP32 [B, outputs] (a view).

        The backward pass reads x_u8 again: keep it unchanged until then."""
        B = x_u8.shape[0]
        self._enter()
        self._check(self._L.lsm_cnn_forward(self._h, _dptr(x_u8), B, _dptr(self.y)))
        self._x = x_u8
        self._leave(x_u8)
        return self.y[:B]

    def mse(self, target):
        self._enter()
        self._check(self._L.lsm_cnn_mse(self._h, _dptr(target), None, _dptr(self.loss)))
        self._leave(target)
        return self.loss

    def mse_noalloc(self, target, dy, loss):
        """lsm_cnn_mse_noalloc into caller tensors dy [batch, outputs] and
        loss [1] (float32, on the network's device)."""
        self._enter()
        self._check(self._L.lsm_cnn_mse_noalloc(self._h, _dptr(target), _dptr(dy), _dptr(loss)))
        self._leave(target, dy, loss)

    def backward(self, dy=None):
        self._enter()
        self._check(self._L.lsm_cnn_backward(self._h, _dptr(dy)))
        self._leave(dy, getattr(self, "_x", None))

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        self._enter()
        self._check(self._L.lsm_cnn_adam_step(self._h, float(lr), float(beta1), float(beta2),
                                              float(eps), self.t))
        self._leave()

    def train_step(self, x_u8, target, lr):
        self.forward(x_u8)
        loss = self.mse(target)
        self.backward()
        self.adam_step(lr)
        return loss

    def conv_forward(self, layer, x_bf16, out_bf16):
        B = x_bf16.shape[0]
        self._enter()
        self._check(self._L.lsm_cnn_conv_forward(self._h, int(layer), _dptr(x_bf16),
                                                 _dptr(out_bf16), B))
        self._leave(x_bf16, out_bf16)

    def buffer(self, name, layer=0):
        """Copy of an internal buffer of the last pass (flat array over the
        configured batch; BF16 buffers are returned as FP32 values)."""
        bid, dt = BUFFERS[name]
        n = C.c_size_t()
        self._check(self._L.lsm_cnn_read_buffer(self._h, bid, int(layer), None, C.byref(n)))
        out = np.zeros(n.value // np.dtype(dt).itemsize, dt)
        self._check(self._L.lsm_cnn_read_buffer(self._h, bid, int(layer),
                                                out.ctypes.data_as(C.c_void_p), C.byref(n)))
        if dt == np.uint16:
            return (out.astype(np.uint32) << 16).view(np.float32)
        return out

    def synchronize(self):
        self.stream.synchronize()
