"""Python binding of the MI355X coprime-blurred-pair (CBP) deblurring library.

Thin ctypes marshalling over the C ABI in include/cbp.h: every step of the
method (unit-circle evaluation, per-sample Gram eigen-solves, scale fix,
assembly, Fourier division) runs in the HIP kernels of libcbp.so.  PyTorch
only provides device memory and the stream.  If libcbp.so has not been built,
every call raises -- there is no CPU fallback.

Tensors: blurred frames are CUDA (HIP) tensors of shape (H, W) or (C, H, W),
float32 (mixed precision form) or float64 (FP64 form).
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

__all__ = [
    "lib", "library_path", "CbpError", "Precision", "workspace_size", "eval_unit_circle",
    "recover_kernels", "deblur", "deblur_batch", "Deblurrer", "PreparedBatch", "decode_diag", "profile",
    "Flags", "last_tuning", "sample_grams", "deblur_noalloc", "noalloc_scratch_bytes", "MlpState", "mlp_forward",
    "mlp_blob_from_params", "load_mlp", "estimate_kernel_sizes", "draw_kernel_pairs", "encode", "quantize",
    "dequantize",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libcbp.so")

CBP_MAX_K = 32
CBP_MAX_S = 32
CBP_MAX_N = 64

STATUS = {0: "ok", 1: "invalid argument", 2: "inconsistent or unsupported shape", 3: "degenerate input",
          4: "device error", 5: "workspace too small", 6: "unsupported option"}


class Precision:
    FP64 = 0
    MIXED = 1
    MFMA32 = 2
    BF16 = 3
    MFMA64 = 4


class Flags:
    GRAPH = 1      # capture the call's launches in a HIP graph, replay on later identical calls
    AUTOTUNE = 2   # search the launch shapes of this batch class on its first call
    DIVIDE_B1 = 4  # single-channel division B1 / K1
    SCALE_K1 = 8   # scale least squares over kernel 1's equations only
    ONE_AXIS = 16  # per-sample scales of one evaluation order, fixed by the kernels' support


class CbpError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} (status {status})")


class CbpImage(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("height", ctypes.c_int32),
                ("width", ctypes.c_int32), ("channels", ctypes.c_int32), ("pitch", ctypes.c_int64),
                ("channel_stride", ctypes.c_int64)]


class CbpOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("samples", ctypes.c_int32), ("lambda_", ctypes.c_double),
                ("tau", ctypes.c_double), ("learned", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("mlp_blob", ctypes.c_void_p), ("stream", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("diag", ctypes.c_void_p)]


class CbpTuning(ctypes.Structure):
    _fields_ = [("fold_rows", ctypes.c_int32), ("strip_columns", ctypes.c_int32),
                ("workgroups_per_cu", ctypes.c_int32), ("fft_order", ctypes.c_int32), ("ms", ctypes.c_double)]


class CbpDiag(ctypes.Structure):
    _fields_ = [("k1", ctypes.c_int32), ("k2", ctypes.c_int32), ("S", ctypes.c_int32), ("n", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("refine_sample", ctypes.c_int32),
                ("refine_scale", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("sample_lambda0", ctypes.c_double * CBP_MAX_S * 2),
                ("sample_lambda1", ctypes.c_double * CBP_MAX_S * 2),
                ("sample_scale", ctypes.c_double * CBP_MAX_S * 2),
                ("scale_lambda0", ctypes.c_double), ("scale_lambda1", ctypes.c_double),
                ("scale_scale", ctypes.c_double),
                ("kernel_imag", ctypes.c_double * 2), ("kernel_outside", ctypes.c_double * 2),
                ("sample_vec", ctypes.c_double * 2 * CBP_MAX_N * CBP_MAX_S * 2),
                ("scale_vec", ctypes.c_double * 2 * (2 * CBP_MAX_S)),
                ("khat", ctypes.c_double * 2 * CBP_MAX_S * CBP_MAX_S * 2),
                ("sample_features", ctypes.c_float * 32 * CBP_MAX_S * 2),
                ("sample_weights", ctypes.c_double * (2 * CBP_MAX_S + 1)),
                ("judge", ctypes.c_double * 2)]


class CbpSizeSearch(ctypes.Structure):
    _fields_ = [("kmin", ctypes.c_int32), ("kmax", ctypes.c_int32), ("step", ctypes.c_int32),
                ("samples", ctypes.c_int32)]


class CbpSizeResult(ctypes.Structure):
    _fields_ = [("k1", ctypes.c_int32), ("k2", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("ncand", ctypes.c_int32), ("samples", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("cand", ctypes.c_int32 * CBP_MAX_K), ("score", ctypes.c_double * CBP_MAX_K),
                ("drop", ctypes.c_double * CBP_MAX_K)]


SIZE_NONE_SINGULAR = 1
SIZE_FIRST_SINGULAR = 2

_LIB = None

# every entry point declared in include/cbp.h with (restype, argtypes)
_P = ctypes.c_void_p
_SIGS = {
    "cbp_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "cbp_version": (ctypes.c_char_p, []),
    "cbp_diag_size": (ctypes.c_size_t, []),
    "cbp_workspace_size": (ctypes.c_size_t, [ctypes.c_int32] * 5 + [ctypes.POINTER(CbpOptions)]),
    "cbp_eval_unit_circle": (ctypes.c_int, [ctypes.POINTER(CbpImage), ctypes.c_int32, _P, _P,
                                            ctypes.POINTER(CbpOptions)]),
    "cbp_recover_kernels": (ctypes.c_int, [ctypes.POINTER(CbpImage), ctypes.POINTER(CbpImage), ctypes.c_int32,
                                           ctypes.c_int32, _P, _P, ctypes.POINTER(CbpOptions)]),
    "cbp_deblur": (ctypes.c_int, [ctypes.POINTER(CbpImage), ctypes.POINTER(CbpImage), ctypes.POINTER(CbpImage),
                                  _P, _P, ctypes.POINTER(CbpOptions)]),
    "cbp_deblur_batch": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(CbpImage), ctypes.POINTER(CbpImage),
                                        ctypes.POINTER(CbpImage), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(CbpOptions)]),
    "cbp_deblur_noalloc": (ctypes.c_int, [ctypes.POINTER(CbpImage), ctypes.POINTER(CbpImage),
                                          ctypes.POINTER(CbpImage), _P, _P, ctypes.POINTER(CbpOptions)]),
    "cbp_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "cbp_size_workspace_size": (ctypes.c_size_t, [ctypes.c_int32] * 4 + [ctypes.POINTER(CbpSizeSearch),
                                                                      ctypes.POINTER(CbpOptions)]),
    "cbp_estimate_kernel_sizes": (ctypes.c_int, [ctypes.POINTER(CbpImage), ctypes.POINTER(CbpImage),
                                                 ctypes.POINTER(CbpSizeSearch), _P, _P,
                                                 ctypes.POINTER(CbpOptions)]),
    "cbp_draw_kernel_pairs": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P]),
    "cbp_encode": (ctypes.c_int, [ctypes.POINTER(CbpImage), _P, ctypes.c_int32, _P, ctypes.c_int32,
                                  ctypes.POINTER(CbpImage), ctypes.POINTER(CbpImage), _P]),
    "cbp_quantize": (ctypes.c_int, [ctypes.POINTER(CbpImage), ctypes.POINTER(CbpImage), ctypes.c_int32, _P]),
    "cbp_dequantize": (ctypes.c_int, [ctypes.POINTER(CbpImage), ctypes.POINTER(CbpImage), _P]),
    "cbp_last_tuning": (ctypes.c_int, [ctypes.c_void_p]),
    "cbp_sample_grams": (ctypes.c_int, [ctypes.POINTER(CbpImage), ctypes.POINTER(CbpImage), ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(CbpOptions)]),
    "cbp_last_error": (ctypes.c_char_p, []),
    "cbp_mlp_param_count": (ctypes.c_int32, []),
    "cbp_mlp_blob_size": (ctypes.c_size_t, []),
    "cbp_mlp_state_size": (ctypes.c_size_t, [ctypes.c_int32]),
    "cbp_mlp_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "cbp_mlp_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "cbp_mlp_checkpoint_size": (ctypes.c_size_t, []),
    "cbp_mlp_save_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "cbp_mlp_load_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "cbp_mlp_gradients": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cbp_mlp_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int32, ctypes.c_float, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "cbp_mlp_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "cbp_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "cbp_profile_enable": (None, [ctypes.c_int32]),
    "cbp_profile_reset": (None, []),
    "cbp_profile_read": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.c_int32]),
    "cbp_profile_phase_name": (ctypes.c_char_p, [ctypes.c_int32]),
}


def lib() -> ctypes.CDLL:
    """Load libcbp.so (built in-tree by paper_1203_4874_amd.build)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(library_path):
            raise RuntimeError(f"HIP library not built ({library_path}); run: python -m paper_1203_4874_amd.build")
        L = ctypes.CDLL(library_path)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


# ---------------------------------------------------------------- marshalling helpers

def _torch():
    import torch
    return torch


def _image(t) -> CbpImage:
    torch = _torch()
    if not t.is_cuda:
        raise ValueError("CBP frames must be device tensors")
    if t.dtype not in (torch.float32, torch.float64):
        raise ValueError("CBP frames must be float32 or float64")
    if t.dim() == 2:
        C, (H, W) = 1, t.shape
        sc, sy, sx = t.shape[0] * t.stride(0), t.stride(0), t.stride(1)
    elif t.dim() == 3:
        C, H, W = t.shape
        sc, sy, sx = t.stride(0), t.stride(1), t.stride(2)
    else:
        raise ValueError("frames must be (H, W) or (C, H, W)")
    if sx != 1:
        raise ValueError("frames must have unit stride along x")
    return CbpImage(t.data_ptr(), 0 if t.dtype == torch.float32 else 1, H, W, C, sy, sc)


def _image_u8(t) -> CbpImage:
    torch = _torch()
    if not t.is_cuda or t.dtype != torch.uint8:
        raise ValueError("8-bit streams must be uint8 device tensors")
    if t.dim() == 2:
        C, (H, W) = 1, t.shape
        sc, sy, sx = t.shape[0] * t.stride(0), t.stride(0), t.stride(1)
    elif t.dim() == 3:
        C, H, W = t.shape
        sc, sy, sx = t.stride(0), t.stride(1), t.stride(2)
    else:
        raise ValueError("streams must be (H, W) or (C, H, W)")
    if sx != 1:
        raise ValueError("streams must have unit stride along x")
    return CbpImage(t.data_ptr(), 2, H, W, C, sy, sc)


def _precision_of(t) -> int:
    torch = _torch()
    return Precision.MIXED if t.dtype == torch.float32 else Precision.FP64


def _check(status: int, where: str):
    if status != 0:
        if status == 4:
            where = f"{where} [{lib().cbp_last_error().decode()}]"
        raise CbpError(status, where)


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def workspace_size(maxH: int, maxW: int, maxk: int, channels: int = 1, batch: int = 1,
                   precision: int = Precision.FP64, samples: int = 0) -> int:
    o = CbpOptions()
    o.precision = precision
    o.samples = samples
    return int(lib().cbp_workspace_size(maxH, maxW, maxk, channels, batch, ctypes.byref(o)))


def diag_size() -> int:
    return int(lib().cbp_diag_size())


def decode_diag(buf: np.ndarray) -> dict:
    """Decode one cbp_diag record (bytes copied from the device) to numpy."""
    d = CbpDiag.from_buffer_copy(bytes(buf[:ctypes.sizeof(CbpDiag)]))
    S, n = d.S, d.n
    sv = np.ctypeslib.as_array(d.sample_vec).reshape(2, CBP_MAX_S, CBP_MAX_N, 2)
    kh = np.ctypeslib.as_array(d.khat).reshape(2, CBP_MAX_S, CBP_MAX_S, 2)
    scv = np.ctypeslib.as_array(d.scale_vec).reshape(2 * CBP_MAX_S, 2)
    return dict(k1=d.k1, k2=d.k2, S=S, n=n, flags=d.flags, refine_sample=d.refine_sample,
                refine_scale=d.refine_scale,
                sample_lambda0=np.ctypeslib.as_array(d.sample_lambda0).reshape(2, CBP_MAX_S)[:, :S].copy(),
                sample_lambda1=np.ctypeslib.as_array(d.sample_lambda1).reshape(2, CBP_MAX_S)[:, :S].copy(),
                sample_scale=np.ctypeslib.as_array(d.sample_scale).reshape(2, CBP_MAX_S)[:, :S].copy(),
                scale_lambda0=d.scale_lambda0, scale_lambda1=d.scale_lambda1, scale_scale=d.scale_scale,
                kernel_imag=list(d.kernel_imag), kernel_outside=list(d.kernel_outside),
                sample_vec=(sv[:, :S, :n, 0] + 1j * sv[:, :S, :n, 1]).copy(),
                scale_vec=(scv[:2 * S, 0] + 1j * scv[:2 * S, 1]).copy(),
                khat=(kh[:, :S, :S, 0] + 1j * kh[:, :S, :S, 1]).copy(),
                sample_features=np.ctypeslib.as_array(d.sample_features).reshape(2, CBP_MAX_S, 32)[:, :S].copy(),
                sample_weights=np.ctypeslib.as_array(d.sample_weights)[:2 * S + 1].copy(),
                judge=list(d.judge))


@dataclass
class _Buffers:
    ws: object
    diag: object


class Deblurrer:
    """Holds a workspace (and optional diag buffer) for repeated calls on
    frames up to a maximum size, so steady-state calls allocate nothing."""

    def __init__(self, maxH: int, maxW: int, maxk: int, channels: int = 1, batch: int = 1,
                 precision: int = Precision.FP64, samples: int = 0, device="cuda", diag: bool = False):
        torch = _torch()
        self.precision = precision
        self.samples = samples
        nbytes = workspace_size(maxH, maxW, maxk, channels, batch, precision, samples)
        if nbytes == 0:
            raise CbpError(2, "workspace_size")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.diag = torch.zeros(diag_size() * batch, dtype=torch.uint8, device=device) if diag else None
        self.batch = batch

    def options(self, lam: float = 0.0, stream=None, precision=None, flags: int = 0, mlp=None) -> CbpOptions:
        o = CbpOptions()
        o.precision = self.precision if precision is None else precision
        o.samples = self.samples
        o.lambda_ = lam
        o.flags = flags
        if mlp is not None:
            o.learned = 1
            o.mlp_blob = mlp.data_ptr()
        o.stream = _stream_ptr(stream)
        o.workspace = self.ws.data_ptr()
        o.workspace_bytes = self.ws.numel()
        o.diag = self.diag.data_ptr() if self.diag is not None else None
        return o

    def read_diag(self, index: int = 0) -> dict:
        torch = _torch()
        torch.cuda.synchronize()
        raw = self.diag.cpu().numpy()
        sz = diag_size()
        return decode_diag(raw[index * sz:(index + 1) * sz])

    def recover_kernels(self, b1, b2, m: int, n: int, K1=None, K2=None, stream=None):
        torch = _torch()
        i1, i2 = _image(b1), _image(b2)
        k1, k2 = i1.height - m + 1, i2.height - m + 1
        if K1 is None:
            K1 = torch.empty((max(k1, 1), max(k1, 1)), dtype=torch.float64, device=b1.device)
        if K2 is None:
            K2 = torch.empty((max(k2, 1), max(k2, 1)), dtype=torch.float64, device=b1.device)
        o = self.options(0.0, stream, _precision_of(b1))
        _check(lib().cbp_recover_kernels(ctypes.byref(i1), ctypes.byref(i2), m, n, K1.data_ptr(), K2.data_ptr(),
                                         ctypes.byref(o)), "cbp_recover_kernels")
        return K1, K2

    def deblur(self, b1, b2, m: int, n: int, lam: float = 0.0, out=None, K1=None, K2=None, stream=None,
               flags: int = 0, mlp=None):
        """mlp: a device network blob (uint8 tensor, MlpState.export()) selects the learned form."""
        torch = _torch()
        i1, i2 = _image(b1), _image(b2)
        k1, k2 = i1.height - m + 1, i2.height - m + 1
        if out is None:
            shape = (m, n) if b1.dim() == 2 else (b1.shape[0], m, n)
            out = torch.empty(shape, dtype=b1.dtype, device=b1.device)
        if K1 is None:
            K1 = torch.empty((max(k1, 1), max(k1, 1)), dtype=torch.float64, device=b1.device)
        if K2 is None:
            K2 = torch.empty((max(k2, 1), max(k2, 1)), dtype=torch.float64, device=b1.device)
        io = _image(out)
        o = self.options(lam, stream, self.precision if self.precision >= 2 else _precision_of(b1), flags, mlp)
        _check(lib().cbp_deblur(ctypes.byref(i1), ctypes.byref(i2), ctypes.byref(io), K1.data_ptr(),
                                K2.data_ptr(), ctypes.byref(o)), "cbp_deblur")
        return out, K1, K2

    def prepare_batch(self, pairs, lam: float = 0.0, outs=None, flags: int = 0, mlp=None) -> "PreparedBatch":
        """pairs: list of (b1, b2, m, n).  Allocates the latents and kernels
        once and marshals the argument arrays once; PreparedBatch.run() then
        makes one cbp_deblur_batch call per invocation."""
        return PreparedBatch(self, pairs, lam, outs, flags, mlp)

    def deblur_batch(self, pairs, lam: float = 0.0, outs=None, stream=None, flags: int = 0):
        """pairs: list of (b1, b2, m, n).  Returns (latents, K1s, K2s, statuses)."""
        pb = self.prepare_batch(pairs, lam, outs, flags)
        st = pb.run(stream, check=True)
        return pb.latents, pb.K1s, pb.K2s, st


class PreparedBatch:
    """Marshalled arguments of one cbp_deblur_batch call (see Deblurrer.prepare_batch)."""

    def __init__(self, d: Deblurrer, pairs, lam, outs, flags, mlp=None):
        torch = _torch()
        nf = len(pairs)
        self.d, self.nf, self.lam, self.flags, self.mlp = d, nf, lam, flags, mlp
        self.I1 = (CbpImage * nf)()
        self.I2 = (CbpImage * nf)()
        self.IO = (CbpImage * nf)()
        self.k1p = (ctypes.c_void_p * nf)()
        self.k2p = (ctypes.c_void_p * nf)()
        self.st = (ctypes.c_int * nf)()
        self.latents, self.K1s, self.K2s = [], [], []
        self.pairs = pairs
        for f, (b1, b2, m, n) in enumerate(pairs):
            self.I1[f], self.I2[f] = _image(b1), _image(b2)
            k1, k2 = self.I1[f].height - m + 1, self.I2[f].height - m + 1
            out = outs[f] if outs is not None else torch.empty(
                (m, n) if b1.dim() == 2 else (b1.shape[0], m, n), dtype=b1.dtype, device=b1.device)
            K1 = torch.empty((max(k1, 1), max(k1, 1)), dtype=torch.float64, device=b1.device)
            K2 = torch.empty((max(k2, 1), max(k2, 1)), dtype=torch.float64, device=b1.device)
            self.IO[f] = _image(out)
            self.k1p[f], self.k2p[f] = K1.data_ptr(), K2.data_ptr()
            self.latents.append(out)
            self.K1s.append(K1)
            self.K2s.append(K2)
        self.precision = d.precision if d.precision >= 2 else _precision_of(pairs[0][0])

    def run(self, stream=None, check: bool = True):
        o = self.d.options(self.lam, stream, self.precision, self.flags, self.mlp)
        s = lib().cbp_deblur_batch(self.nf, self.I1, self.I2, self.IO, self.k1p, self.k2p, self.st,
                                   ctypes.byref(o))
        if check:
            _check(s, "cbp_deblur_batch")
        return list(self.st)


class MlpState:
    """Training state of the learned form's network (device memory owned
    here): FP32 master weights, Adam moments, bf16 copies and the activations
    of up to max_rows rows.  Every step runs in the library's kernels."""

    def __init__(self, max_rows: int, device="cuda"):
        torch = _torch()
        self.rows = int(max_rows)
        nbytes = int(lib().cbp_mlp_state_size(self.rows))
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.device = device

    @staticmethod
    def param_count() -> int:
        return int(lib().cbp_mlp_param_count())

    def set_params(self, params, stream=None):
        torch = _torch()
        p = torch.as_tensor(params, dtype=torch.float32, device=self.device).contiguous()
        _check(lib().cbp_mlp_set_params(self.buf.data_ptr(), self.rows, p.data_ptr(), _stream_ptr(stream)),
               "cbp_mlp_set_params")
        self._keep = p

    def get_params(self, stream=None):
        torch = _torch()
        p = torch.empty(self.param_count(), dtype=torch.float32, device=self.device)
        _check(lib().cbp_mlp_get_params(self.buf.data_ptr(), self.rows, p.data_ptr(), _stream_ptr(stream)),
               "cbp_mlp_get_params")
        return p

    def save_state(self, stream=None):
        """Checkpoint (FP32 device tensor [3][param_count]): master weights and
        both Adam moments, for resuming training."""
        torch = _torch()
        c = torch.empty(3 * self.param_count(), dtype=torch.float32, device=self.device)
        _check(lib().cbp_mlp_save_state(self.buf.data_ptr(), self.rows, c.data_ptr(), _stream_ptr(stream)),
               "cbp_mlp_save_state")
        return c

    def load_state(self, ckpt, stream=None):
        """Restore a checkpoint written by save_state (any max_rows)."""
        torch = _torch()
        c = torch.as_tensor(ckpt, dtype=torch.float32, device=self.device).contiguous()
        if c.numel() != 3 * self.param_count():
            raise ValueError(f"checkpoint holds {c.numel()} floats, expected {3 * self.param_count()}")
        _check(lib().cbp_mlp_load_state(self.buf.data_ptr(), self.rows, c.data_ptr(), _stream_ptr(stream)),
               "cbp_mlp_load_state")
        self._keep = c

    def gradients(self, X, T, stream=None):
        """(loss, grads) of the mean loss on rows X [n][32], targets T [n][2]."""
        torch = _torch()
        g = torch.empty(self.param_count(), dtype=torch.float32, device=self.device)
        _check(lib().cbp_mlp_gradients(self.buf.data_ptr(), self.rows, X.data_ptr(), T.data_ptr(), X.shape[0],
                                       self.loss.data_ptr(), g.data_ptr(), _stream_ptr(stream)),
               "cbp_mlp_gradients")
        return self.loss, g

    def train_step(self, X, T, lr: float, step: int, stream=None):
        _check(lib().cbp_mlp_train_step(self.buf.data_ptr(), self.rows, X.data_ptr(), T.data_ptr(), X.shape[0],
                                        float(lr), int(step), self.loss.data_ptr(), _stream_ptr(stream)),
               "cbp_mlp_train_step")
        return self.loss

    def export(self, stream=None):
        """The inference blob (uint8 device tensor) for the learned form."""
        torch = _torch()
        blob = torch.zeros(int(lib().cbp_mlp_blob_size()), dtype=torch.uint8, device=self.device)
        _check(lib().cbp_mlp_export(self.buf.data_ptr(), self.rows, blob.data_ptr(), _stream_ptr(stream)),
               "cbp_mlp_export")
        return blob


def mlp_forward(blob, X, stream=None):
    """Network outputs (o1, o2) [n][2] FP32 for feature rows X [n][32] (FP32 device)."""
    torch = _torch()
    out = torch.empty((X.shape[0], 2), dtype=torch.float32, device=X.device)
    _check(lib().cbp_mlp_forward(blob.data_ptr(), X.data_ptr(), X.shape[0], out.data_ptr(), _stream_ptr(stream)),
           "cbp_mlp_forward")
    return out


WEIGHTS = os.path.join(_HERE, "weights", "cbp_mlp.npz")


def load_mlp(path: str = WEIGHTS, device="cuda"):
    """The trained network (packed FP32 parameters in an .npz written by
    paper_1203_4874_amd.train_mlp) as an inference blob on the device."""
    with np.load(path, allow_pickle=False) as z:
        params = np.ascontiguousarray(z["params"], dtype=np.float32)
    if params.size != MlpState.param_count():
        raise ValueError(f"{path}: {params.size} parameters, expected {MlpState.param_count()}")
    return mlp_blob_from_params(params, device)


def mlp_blob_from_params(params, device="cuda"):
    """Inference blob from packed FP32 parameters (through a one-row state)."""
    st = MlpState(1, device)
    st.set_params(params)
    return st.export()


def last_tuning():
    """Launch shapes of the last autotune search on the current device, or None."""
    t = CbpTuning()
    if lib().cbp_last_tuning(ctypes.byref(t)) != 0:
        return None
    return dict(fold_rows=t.fold_rows, strip_columns=t.strip_columns,
                workgroups_per_cu=t.workgroups_per_cu, fft_order=t.fft_order, ms=t.ms)


def _one_shot(b1, b2, m, n, samples, diag):
    H = max(b1.shape[-2], b2.shape[-2])
    W = max(b1.shape[-1], b2.shape[-1])
    k = max(b1.shape[-2], b2.shape[-2]) - m + 1
    ch = 1 if b1.dim() == 2 else b1.shape[0]
    return Deblurrer(H, W, max(1, min(k, CBP_MAX_K)), ch, 1, _precision_of(b1), samples, b1.device, diag)


def eval_unit_circle(b, S: int, stream=None):
    """(EX, EY) complex128 device tensors of shapes (S, W) and (S, H)."""
    torch = _torch()
    im = _image(b)
    ex = torch.empty((S, im.width), dtype=torch.complex128, device=b.device)
    ey = torch.empty((S, im.height), dtype=torch.complex128, device=b.device)
    need = workspace_size(im.height, im.width, max(1, min(S, CBP_MAX_K)), 1, 1, Precision.FP64, S)
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=b.device)
    o = CbpOptions()
    o.precision = _precision_of(b)
    o.stream = _stream_ptr(stream)
    o.workspace = ws.data_ptr()
    o.workspace_bytes = ws.numel()
    _check(lib().cbp_eval_unit_circle(ctypes.byref(im), S, ex.data_ptr(), ey.data_ptr(), ctypes.byref(o)),
           "cbp_eval_unit_circle")
    return ex, ey


def sample_grams(b1, b2, m: int, n: int, precision=None, samples: int = 0, stream=None):
    """Per-sample Gram matrices, complex128 device tensor (2, S, N, N):
    [pass][sample][p][q] with unknowns ordered (u: k2 entries, v: k1)."""
    torch = _torch()
    i1, i2 = _image(b1), _image(b2)
    k1, k2 = i1.height - m + 1, i2.height - m + 1
    S = samples or max(k1, k2)
    N = k1 + k2
    prec = _precision_of(b1) if precision is None else precision
    d = Deblurrer(max(i1.height, i2.height), max(i1.width, i2.width), max(1, min(max(k1, k2), CBP_MAX_K)),
                  i1.channels, 1, prec, samples, b1.device)
    G = torch.empty((2, S, N, N), dtype=torch.complex128, device=b1.device)
    o = d.options(0.0, stream, prec)
    _check(lib().cbp_sample_grams(ctypes.byref(i1), ctypes.byref(i2), m, n, G.data_ptr(), ctypes.byref(o)),
           "cbp_sample_grams")
    return G


def recover_kernels(b1, b2, m: int, n: int, samples: int = 0, diag: bool = False):
    d = _one_shot(b1, b2, m, n, samples, diag)
    K1, K2 = d.recover_kernels(b1, b2, m, n)
    return (K1, K2, d.read_diag()) if diag else (K1, K2)


def deblur(b1, b2, m: int, n: int, samples: int = 0, lam: float = 0.0, diag: bool = False):
    d = _one_shot(b1, b2, m, n, samples, diag)
    L, K1, K2 = d.deblur(b1, b2, m, n, lam)
    return (L, K1, K2, d.read_diag()) if diag else (L, K1, K2)


def estimate_kernel_sizes(b1, b2, kmin: int = 1, kmax: int = CBP_MAX_K, step: int = 1, samples: int = 0,
                          ratios: bool = False, stream=None) -> dict:
    """cbp_estimate_kernel_sizes: blind (k1, k2) of a blurred pair (no latent
    size).  Synchronises and returns the estimate, its flags, the candidates
    with their scores and drops and (ratios=True) the per-sample ratios
    [candidate][pass][sample]."""
    torch = _torch()
    i1, i2 = _image(b1), _image(b2)
    se = CbpSizeSearch(kmin, kmax, step, samples)
    o = CbpOptions()
    o.precision = _precision_of(b1)
    d = i1.height - i2.height
    nbytes = int(lib().cbp_size_workspace_size(max(i1.height, i2.height), max(i1.width, i2.width), i1.channels,
                                               d, ctypes.byref(se), ctypes.byref(o)))
    if nbytes == 0:
        raise CbpError(2, "cbp_size_workspace_size")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=b1.device)
    res = torch.zeros(ctypes.sizeof(CbpSizeResult), dtype=torch.uint8, device=b1.device)
    rat = torch.zeros(CBP_MAX_K * 2 * CBP_MAX_S, dtype=torch.float64, device=b1.device) if ratios else None
    o.stream = _stream_ptr(stream)
    o.workspace = ws.data_ptr()
    o.workspace_bytes = ws.numel()
    _check(lib().cbp_estimate_kernel_sizes(ctypes.byref(i1), ctypes.byref(i2), ctypes.byref(se), res.data_ptr(),
                                           rat.data_ptr() if rat is not None else None, ctypes.byref(o)),
           "cbp_estimate_kernel_sizes")
    torch.cuda.synchronize()
    r = CbpSizeResult.from_buffer_copy(bytes(res.cpu().numpy()))
    nc = r.ncand
    out = dict(k1=r.k1, k2=r.k2, flags=r.flags, S=r.samples, candidates=list(r.cand[:nc]),
               scores=np.array(r.score[:nc]), drops=np.array(r.drop[:nc]))
    if rat is not None:
        out["ratios"] = rat[:nc * 2 * r.samples].cpu().numpy().reshape(nc, 2, r.samples)
    return out


def draw_kernel_pairs(seed: int, frame0: int, nframes: int, k1: int, k2: int, samples: int = 0, device="cuda",
                      stream=None):
    """cbp_draw_kernel_pairs: the encoder's coprime kernel pairs of frames
    frame0 .. frame0 + nframes - 1.  Returns (K1s [n, k1, k1], K2s, attempts,
    min_ratio) -- the last two synchronised to host numpy arrays."""
    torch = _torch()
    K1s = torch.empty((nframes, k1, k1), dtype=torch.float64, device=device)
    K2s = torch.empty((nframes, k2, k2), dtype=torch.float64, device=device)
    att = torch.empty(nframes, dtype=torch.int32, device=device)
    mr = torch.empty(nframes, dtype=torch.float64, device=device)
    _check(lib().cbp_draw_kernel_pairs(seed, frame0, nframes, k1, k2, samples, K1s.data_ptr(), K2s.data_ptr(),
                                       att.data_ptr(), mr.data_ptr(), _stream_ptr(stream)), "cbp_draw_kernel_pairs")
    return K1s, K2s, att.cpu().numpy(), mr.cpu().numpy()


def encode(L, K1, K2, b1=None, b2=None, stream=None):
    """cbp_encode: the blurred pair (B1, B2) of a latent frame."""
    torch = _torch()
    k1, k2 = K1.shape[-1], K2.shape[-1]
    m, n = L.shape[-2], L.shape[-1]
    lead = tuple(L.shape[:-2])
    if b1 is None:
        b1 = torch.empty(lead + (m + k1 - 1, n + k1 - 1), dtype=L.dtype, device=L.device)
    if b2 is None:
        b2 = torch.empty(lead + (m + k2 - 1, n + k2 - 1), dtype=L.dtype, device=L.device)
    il, i1, i2 = _image(L), _image(b1), _image(b2)
    _check(lib().cbp_encode(ctypes.byref(il), K1.data_ptr(), k1, K2.data_ptr(), k2, ctypes.byref(i1),
                            ctypes.byref(i2), _stream_ptr(stream)), "cbp_encode")
    return b1, b2


def quantize(B, drop_bits: int = 0, out=None, stream=None):
    """cbp_quantize: the 8-bit stream of a level without drop_bits low bits."""
    torch = _torch()
    if out is None:
        out = torch.empty(B.shape, dtype=torch.uint8, device=B.device)
    _check(lib().cbp_quantize(ctypes.byref(_image(B)), ctypes.byref(_image_u8(out)), drop_bits, _stream_ptr(stream)),
           "cbp_quantize")
    return out


def dequantize(q, dtype=None, out=None, stream=None):
    """cbp_dequantize: q / 255 as float32 (or dtype)."""
    torch = _torch()
    if out is None:
        out = torch.empty(q.shape, dtype=dtype or torch.float32, device=q.device)
    _check(lib().cbp_dequantize(ctypes.byref(_image_u8(q)), ctypes.byref(_image(out)), _stream_ptr(stream)),
           "cbp_dequantize")
    return out


def noalloc_scratch_bytes() -> int:
    return int(lib().cbp_noalloc_scratch_bytes())


def deblur_noalloc(b1, b2, out, K1, K2, samples: int = 0, lam: float = 0.0, precision=None, diag=None,
                   stream=None):
    """cbp_deblur_noalloc: the library's per-device scratch replaces the
    workspace.  out (the latent, whose shape gives m x n), K1 and K2 are
    caller-allocated device tensors; diag is an optional device byte tensor
    of diag_size() bytes."""
    i1, i2, io = _image(b1), _image(b2), _image(out)
    o = CbpOptions()
    o.precision = _precision_of(b1) if precision is None else precision
    o.samples = samples
    o.lambda_ = lam
    o.stream = _stream_ptr(stream)
    o.diag = diag.data_ptr() if diag is not None else None
    _check(lib().cbp_deblur_noalloc(ctypes.byref(i1), ctypes.byref(i2), ctypes.byref(io),
                                    K1.data_ptr() if K1 is not None else None,
                                    K2.data_ptr() if K2 is not None else None, ctypes.byref(o)),
           "cbp_deblur_noalloc")
    return out, K1, K2


def deblur_batch(pairs, samples: int = 0, lam: float = 0.0, flags: int = 0):
    torch = _torch()
    H = max(max(p[0].shape[-2], p[1].shape[-2]) for p in pairs)
    W = max(max(p[0].shape[-1], p[1].shape[-1]) for p in pairs)
    k = max(max(p[0].shape[-2], p[1].shape[-2]) - p[2] + 1 for p in pairs)
    ch = 1 if pairs[0][0].dim() == 2 else pairs[0][0].shape[0]
    d = Deblurrer(H, W, max(1, min(k, CBP_MAX_K)), ch, len(pairs), _precision_of(pairs[0][0]), samples,
                  pairs[0][0].device)
    return d.deblur_batch(pairs, lam, flags=flags)


class profile:
    """Context manager: per-phase GPU time (ms) of the calls made inside it."""

    def __enter__(self):
        lib().cbp_profile_reset()
        lib().cbp_profile_enable(1)
        self.result = {}
        return self

    def __exit__(self, *exc):
        L = lib()
        n = 16
        tot = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        k = L.cbp_profile_read(tot, cnt, n)
        L.cbp_profile_enable(0)
        self.result = {L.cbp_profile_phase_name(i).decode(): (tot[i], cnt[i]) for i in range(k)}
        return False
