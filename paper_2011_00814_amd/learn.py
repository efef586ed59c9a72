"""Thin ctypes binding of the learned coarse-grid correction (include/gpe_learn.h)
and the network object that owns its device buffers.  Argument marshalling
only: every computation runs in the HIP kernels of libgpe.so; PyTorch
provides the device memory and the stream.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

from . import gpe as G

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "gpe_learn.h")
GPE_ACT_BF16, GPE_ACT_FP32 = 0, 1
CHANNELS = (4, 32, 32, 4)

_bound = False


def header_functions():
    src = open(HEADER).read()
    return re.findall(r"^\s*(?:int|size_t|void)\s+(gpe_\w+)\s*\(", src, re.M)


def lib():
    global _bound
    L = G.lib()
    if not _bound:
        vp, sz, i32, i64, f32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        f4 = ctypes.POINTER(ctypes.c_float)
        sig = {
            "gpe_cnn_param_count": ([], sz),
            "gpe_cnn_act_bytes": ([i32], sz),
            "gpe_cnn_scratch_bytes": ([i32, i32, i32], sz),
            "gpe_restrict2d": ([vp, vp, i32, i32, i32, i32, vp], ctypes.c_int),
            "gpe_cnn_target": ([vp, vp, i32, i32, i32, f4, vp, vp], ctypes.c_int),
            "gpe_cnn_features": ([vp, i32, i32, i32, f4, i32, vp, vp], ctypes.c_int),
            "gpe_cnn_convert": ([vp, vp, i32, vp], ctypes.c_int),
            "gpe_cnn_forward": ([vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, vp], ctypes.c_int),
            "gpe_cnn_loss": ([vp, vp, vp, vp, i64, vp, sz, vp], ctypes.c_int),
            "gpe_cnn_backward": ([vp, vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, vp, sz, vp], ctypes.c_int),
            "gpe_cnn_adam": ([vp, vp, vp, vp, i64, f32, f32, f32, f32, i64, vp], ctypes.c_int),
            "gpe_cnn_apply": ([vp, vp, i32, i32, i32, f4, vp, vp], ctypes.c_int),
            "gpe_interface_position": ([vp, i32, i32, i32, vp, vp], ctypes.c_int),
            "gpe_cnn_infer_scratch_bytes": ([i32, i32, i32], sz),
            "gpe_cnn_infer": ([vp, vp, vp, i32, i32, i32, f4, f4, vp, vp, sz, vp], ctypes.c_int),
            "gpe_cnn_infer_noalloc": ([vp, vp, vp, i32, i32, i32, f4, f4, vp, vp], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _bound = True
    return L


def _check(rc, what):
    if rc:
        raise G.GpeError(rc, what)


def _f4(vals):
    return (ctypes.c_float * 4)(*[float(v) for v in vals])


def _vp(x):
    return ctypes.c_void_p(int(x))


# ---- functions with the names of the C-ABI ---------------------------------------
def gpe_cnn_param_count() -> int:
    return int(lib().gpe_cnn_param_count())


def gpe_cnn_act_bytes(act_type: int) -> int:
    return int(lib().gpe_cnn_act_bytes(int(act_type)))


def gpe_cnn_scratch_bytes(B: int, H: int, W: int) -> int:
    return int(lib().gpe_cnn_scratch_bytes(B, H, W))


def gpe_restrict2d(fine_table, coarse_table, B, ny, nx, f, stream):
    _check(lib().gpe_restrict2d(_vp(fine_table), _vp(coarse_table), B, ny, nx, f, _vp(stream)), "gpe_restrict2d")


def gpe_cnn_target(next_table, pred_table, B, H, W, out_scale, target, stream):
    _check(lib().gpe_cnn_target(_vp(next_table), _vp(pred_table), B, H, W, _f4(out_scale), _vp(target), _vp(stream)),
           "gpe_cnn_target")


def gpe_cnn_features(table, B, H, W, in_scale, act_type, x0, stream):
    _check(lib().gpe_cnn_features(_vp(table), B, H, W, _f4(in_scale), act_type, _vp(x0), _vp(stream)),
           "gpe_cnn_features")


def gpe_cnn_convert(params, params_act, act_type, stream):
    _check(lib().gpe_cnn_convert(_vp(params), _vp(params_act), act_type, _vp(stream)), "gpe_cnn_convert")


def gpe_cnn_forward(params, params_act, x0, a1, a2, out, B, H, W, act_type, stream):
    _check(lib().gpe_cnn_forward(_vp(params), _vp(params_act), _vp(x0), _vp(a1), _vp(a2), _vp(out), B, H, W, act_type,
                                 _vp(stream)), "gpe_cnn_forward")


def gpe_cnn_loss(out, target, gout, loss, n, scratch, scratch_bytes, stream):
    _check(lib().gpe_cnn_loss(_vp(out), _vp(target), _vp(gout), _vp(loss), int(n), _vp(scratch), scratch_bytes,
                              _vp(stream)), "gpe_cnn_loss")


def gpe_cnn_backward(params, params_act, x0, a1, a2, gout, grads, B, H, W, act_type, scratch, scratch_bytes, stream):
    _check(lib().gpe_cnn_backward(_vp(params), _vp(params_act), _vp(x0), _vp(a1), _vp(a2), _vp(gout), _vp(grads), B,
                                  H, W, act_type, _vp(scratch), scratch_bytes, _vp(stream)), "gpe_cnn_backward")


def gpe_cnn_adam(params, m, v, grads, n, lr, beta1, beta2, eps, t, stream):
    _check(lib().gpe_cnn_adam(_vp(params), _vp(m), _vp(v), _vp(grads), int(n), lr, beta1, beta2, eps, int(t),
                              _vp(stream)), "gpe_cnn_adam")


def gpe_cnn_apply(table, out, B, H, W, out_scale, scratch, stream):
    _check(lib().gpe_cnn_apply(_vp(table), _vp(out), B, H, W, _f4(out_scale), _vp(scratch), _vp(stream)),
           "gpe_cnn_apply")


def gpe_cnn_infer_scratch_bytes(B: int, H: int, W: int) -> int:
    return int(lib().gpe_cnn_infer_scratch_bytes(B, H, W))


def gpe_cnn_infer(table, params, params_bf16, B, H, W, in_scale, out_scale, out, scratch, scratch_bytes, stream):
    _check(lib().gpe_cnn_infer(_vp(table), _vp(params), _vp(params_bf16), B, H, W, _f4(in_scale), _f4(out_scale),
                               _vp(out), _vp(scratch), scratch_bytes, _vp(stream)), "gpe_cnn_infer")


def gpe_cnn_infer_noalloc(table, params, params_bf16, B, H, W, in_scale, out_scale, out, stream):
    _check(lib().gpe_cnn_infer_noalloc(_vp(table), _vp(params), _vp(params_bf16), B, H, W, _f4(in_scale),
                                       _f4(out_scale), _vp(out), _vp(stream)), "gpe_cnn_infer_noalloc")


def gpe_interface_position(table, B, H, W, out, stream):
    _check(lib().gpe_interface_position(_vp(table), B, H, W, _vp(out), _vp(stream)), "gpe_interface_position")


# ---- device pointer tables --------------------------------------------------------
def pointer_table(ptrs, device):
    """A device array of device pointers (int64), kept alive by the caller."""
    import torch

    return torch.tensor([int(p) for p in ptrs], dtype=torch.int64, device=device)


def state_pointers(grids):
    """(u, v, p, phi) device pointers of 2-D FP32 grid handles (Solver or
    EnsembleCase objects): what the kernels of this module read and write.
    Those kernels address a field as dense rows of nx, so the grids' device
    rows must carry no padding (FP32: nx below 64 or a multiple of 64)."""
    out = []
    for g in grids:
        nx = g.shape[-1]
        if G.gpe_field_pitch(g.h) != nx:
            raise ValueError(f"learned-correction kernels need unpadded rows: nx = {nx} has a row pitch")
        for f in (G.GPE_FIELD_U, G.GPE_FIELD_V, G.GPE_FIELD_P, G.GPE_FIELD_PHI):
            out.append(G.gpe_field_pointer(g.h, f))
    return out


def bf16_to_float(t):
    """bfloat16 bit patterns (int16 tensor or array) -> float32 numpy array."""
    a = np.asarray(t.cpu().numpy() if hasattr(t, "cpu") else t).astype(np.uint16).astype(np.uint32) << 16
    return a.view(np.float32)


class CNN:
    """The network's device buffers for batches of up to B coarse states of
    H x W cells: FP32 master parameters, the act_type copy, Adam moments,
    gradients, activations, output, gradient of the output and scratch."""

    def __init__(self, B: int, H: int, W: int, act_type: int = GPE_ACT_BF16, device="cuda:0", stream=None,
                 params: np.ndarray | None = None):
        import torch

        self.B, self.H, self.W, self.act_type = B, H, W, act_type
        self.device = torch.device(device)
        # default: torch's current stream, so that tensors torch fills and the
        # kernels launched here are ordered on one stream
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        n = gpe_cnn_param_count()
        self.n = n
        ab = gpe_cnn_act_bytes(act_type)
        adt = torch.int16 if ab == 2 else torch.float32
        f32 = dict(dtype=torch.float32, device=self.device)
        self.params = torch.zeros(n, **f32)
        if params is not None:
            self.params.copy_(torch.from_numpy(np.asarray(params, dtype=np.float32)))
        self.params_act = torch.zeros(n, dtype=adt, device=self.device)
        self.m = torch.zeros(n, **f32)
        self.v = torch.zeros(n, **f32)
        self.grads = torch.zeros(n, **f32)
        P = B * H * W
        self.x0 = torch.zeros(P * 4, dtype=adt, device=self.device)
        self.a1 = torch.zeros(P * 32, dtype=adt, device=self.device)
        self.a2 = torch.zeros(P * 32, dtype=adt, device=self.device)
        self.out = torch.zeros(P * 4, **f32)
        self.gout = torch.zeros(P * 4, **f32)
        self.target = torch.zeros(P * 4, **f32)
        self.loss_buf = torch.zeros(1, **f32)
        self.scratch_bytes = gpe_cnn_scratch_bytes(B, H, W)
        self.scratch = torch.zeros(self.scratch_bytes // 4 + 1, **f32)
        self.infer_bytes = gpe_cnn_infer_scratch_bytes(B, H, W)
        self.infer_scratch = torch.zeros(self.infer_bytes // 4 + 1, **f32)
        self.step_count = 0
        self.convert()

    @property
    def sid(self):
        return self.stream.cuda_stream

    def convert(self):
        gpe_cnn_convert(self.params.data_ptr(), self.params_act.data_ptr(), self.act_type, self.sid)

    def features(self, table, B, in_scale):
        gpe_cnn_features(table.data_ptr(), B, self.H, self.W, in_scale, self.act_type, self.x0.data_ptr(), self.sid)

    def forward(self, B):
        gpe_cnn_forward(self.params.data_ptr(), self.params_act.data_ptr(), self.x0.data_ptr(), self.a1.data_ptr(),
                        self.a2.data_ptr(), self.out.data_ptr(), B, self.H, self.W, self.act_type, self.sid)

    def loss(self, B) -> None:
        gpe_cnn_loss(self.out.data_ptr(), self.target.data_ptr(), self.gout.data_ptr(), self.loss_buf.data_ptr(),
                     B * self.H * self.W * 4, self.scratch.data_ptr(), self.scratch_bytes, self.sid)

    def backward(self, B):
        gpe_cnn_backward(self.params.data_ptr(), self.params_act.data_ptr(), self.x0.data_ptr(), self.a1.data_ptr(),
                         self.a2.data_ptr(), self.gout.data_ptr(), self.grads.data_ptr(), B, self.H, self.W,
                         self.act_type, self.scratch.data_ptr(), self.scratch_bytes, self.sid)

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        gpe_cnn_adam(self.params.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), self.grads.data_ptr(), self.n, lr,
                     beta1, beta2, eps, self.step_count, self.sid)
        self.convert()

    def apply(self, table, B, out_scale):
        gpe_cnn_apply(table.data_ptr(), self.out.data_ptr(), B, self.H, self.W, out_scale, self.scratch.data_ptr(),
                      self.sid)

    def infer(self, table, B, in_scale, out_scale):
        """Network input, forward pass and correction of B states in the
        fused BF16 kernel (the output also lands in self.out)."""
        if self.act_type != GPE_ACT_BF16:
            raise ValueError("the fused inference path uses BF16 operands")
        gpe_cnn_infer(table.data_ptr(), self.params.data_ptr(), self.params_act.data_ptr(), B, self.H, self.W,
                      in_scale, out_scale, self.out.data_ptr(), self.infer_scratch.data_ptr(), self.infer_bytes,
                      self.sid)

    def synchronize(self):
        self.stream.synchronize()


def unpack_params(flat):
    """Packed parameter vector -> [(w, b)] per layer (numpy, float64)."""
    flat = np.asarray(flat, dtype=np.float64)
    out, o = [], 0
    for layer in range(3):
        ci, co = CHANNELS[layer], CHANNELS[layer + 1]
        w = flat[o:o + co * 9 * ci].reshape(co, 3, 3, ci)
        o += co * 9 * ci
        b = flat[o:o + co]
        o += co
        out.append((w, b))
    return out


def pack_params(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])
