"""Python binding of libct (ctypes): argument marshalling only.

Every transform step runs in the HIP kernels of libct.so; this module only
converts torch tensors to device pointers and sizes, allocates caller-owned
workspace, and checks return codes. There is no fallback: if the library is
missing or a call fails, an exception is raised.

Names follow the C ABI (include/ct.h): forward, inverse, quantize,
dequantize, forward_adjoint, inverse_adjoint, layout.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libct.so")

MAX_LEVELS = 6
ERRORS = {0: "CT_OK", -1: "CT_ERR_ARG", -2: "CT_ERR_GEOM", -3: "CT_ERR_WORKSPACE",
          -4: "CT_ERR_HIP", -5: "CT_ERR_UNSUPPORTED"}


class Geom(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("dirs", ctypes.c_int32 * MAX_LEVELS)]


class Layout(ctypes.Structure):
    _fields_ = [("pad_h", ctypes.c_int32), ("pad_w", ctypes.c_int32),
                ("exp2", ctypes.c_int32), ("nsub", ctypes.c_int32),
                ("ncoef", ctypes.c_int64)]


class Subband(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("k", ctypes.c_int32),
                ("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
                ("offset", ctypes.c_int64),
                ("o1", ctypes.c_int32), ("o2", ctypes.c_int32),
                ("s1", ctypes.c_int32), ("s2", ctypes.c_int32),
                ("transposed", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


class CTError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {ERRORS.get(code, code)} ({_lib().ct_strerror(code).decode()})")
        self.code = code


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(hipcc for gfx950); there is no fallback path")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        G = ctypes.POINTER(Geom)
        i32, sz = ctypes.c_int32, ctypes.c_size_t
        sig = {
            "ct_layout_query": [G, ctypes.POINTER(Layout), ctypes.POINTER(Subband), i32],
            "ct_workspace_bytes": [G, i32, ctypes.POINTER(sz)],
            "ct_forward": [G, i32, P, P, P, sz, P],
            "ct_inverse": [G, i32, P, P, P, sz, P],
            "ct_forward_adjoint": [G, i32, P, P, P, sz, P],
            "ct_inverse_adjoint": [G, i32, P, P, P, sz, P],
            "ct_quantize": [G, i32, P, P, i32, P, P, P, sz, P],
            "ct_dequantize": [G, i32, P, P, i32, P, P, P],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.ct_profile_enable.argtypes = [i32, i32]
        lib.ct_profile_enable.restype = ctypes.c_int
        lib.ct_profile_collect.argtypes = [ctypes.POINTER(KernelStat), i32, ctypes.POINTER(i32)]
        lib.ct_profile_collect.restype = ctypes.c_int
        lib.ct_strerror.argtypes = [ctypes.c_int]
        lib.ct_strerror.restype = ctypes.c_char_p
        _LIB = lib
    return _LIB


def geom(height, width, levels, dirs):
    d = list(dirs) + [0] * (MAX_LEVELS - len(dirs))
    return Geom(int(height), int(width), int(levels), (ctypes.c_int32 * MAX_LEVELS)(*d))


def _check(name, rc):
    if rc != 0:
        raise CTError(name, rc)


def layout(height, width, levels, dirs):
    """(Layout, [Subband]) of one plane; host only."""
    g = geom(height, width, levels, dirs)
    lay = Layout()
    _check("ct_layout_query", _lib().ct_layout_query(ctypes.byref(g), ctypes.byref(lay), None, 0))
    table = (Subband * lay.nsub)()
    _check("ct_layout_query", _lib().ct_layout_query(ctypes.byref(g), ctypes.byref(lay), table, lay.nsub))
    return lay, list(table)


def profile_enable(on=True, max_launches=0):
    """Record HIP events around every later launch (see ct_profile_enable)."""
    _check("ct_profile_enable", _lib().ct_profile_enable(1 if on else 0, int(max_launches)))


def profile_collect():
    """{kernel: (launches, total_ms, bytes)} since the last collect."""
    cap = 64
    out = (KernelStat * cap)()
    n = ctypes.c_int32(0)
    _check("ct_profile_collect", _lib().ct_profile_collect(out, cap, ctypes.byref(n)))
    return {out[i].name.decode(): (int(out[i].launches), float(out[i].total_ms), float(out[i].bytes))
            for i in range(min(n.value, cap))}


def workspace_bytes(height, width, levels, dirs, batch):
    g = geom(height, width, levels, dirs)
    n = ctypes.c_size_t(0)
    _check("ct_workspace_bytes", _lib().ct_workspace_bytes(ctypes.byref(g), int(batch), ctypes.byref(n)))
    return n.value


class Plan:
    """Geometry + reusable workspace for one batch size on one device."""

    def __init__(self, height, width, levels, dirs, batch, device="cuda"):
        self.height, self.width, self.levels = int(height), int(width), int(levels)
        self.dirs = [int(d) for d in dirs]
        self.batch = int(batch)
        self.g = geom(height, width, levels, dirs)
        self.layout, self.table = layout(height, width, levels, dirs)
        self.ncoef = int(self.layout.ncoef)
        self.nsub = int(self.layout.nsub)
        self.ws_bytes = workspace_bytes(height, width, levels, dirs, batch)
        self.device = torch.device(device)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _check_tensor(self, t, shape, dtype, name):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def _io(self, fn, src, src_shape, dst_shape, out=None):
        B = self.batch
        self._check_tensor(src, src_shape, torch.float32, "input")
        if out is None:
            out = torch.empty(dst_shape, dtype=torch.float32, device=src.device)
        self._check_tensor(out, dst_shape, torch.float32, "output")
        rc = getattr(_lib(), fn)(ctypes.byref(self.g), B, ctypes.c_void_p(src.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                 self.ws_bytes, self._stream())
        _check(fn, rc)
        return out

    def forward(self, planes, out=None):
        B, H, W = self.batch, self.height, self.width
        return self._io("ct_forward", planes, (B, H, W), (B, self.ncoef), out)

    def inverse(self, coeffs, out=None):
        B, H, W = self.batch, self.height, self.width
        return self._io("ct_inverse", coeffs, (B, self.ncoef), (B, H, W), out)

    def forward_adjoint(self, gcoeffs, out=None):
        B, H, W = self.batch, self.height, self.width
        return self._io("ct_forward_adjoint", gcoeffs, (B, self.ncoef), (B, H, W), out)

    def inverse_adjoint(self, gplanes, out=None):
        B, H, W = self.batch, self.height, self.width
        return self._io("ct_inverse_adjoint", gplanes, (B, H, W), (B, self.ncoef), out)

    def _steps(self, steps):
        if steps.dim() == 1:
            self._check_tensor(steps, (self.nsub,), torch.float32, "steps")
            return steps, 0
        self._check_tensor(steps, (self.batch, self.nsub), torch.float32, "steps")
        return steps, self.nsub

    def quantize(self, coeffs, steps, idx=None, side=None):
        """Returns (int16 indices [B, ncoef], side [B, 2] = lowpass (min, max))."""
        B = self.batch
        self._check_tensor(coeffs, (B, self.ncoef), torch.float32, "coeffs")
        steps, stride = self._steps(steps)
        if idx is None:
            idx = torch.empty((B, self.ncoef), dtype=torch.int16, device=coeffs.device)
        if side is None:
            side = torch.empty((B, 2), dtype=torch.float32, device=coeffs.device)
        self._check_tensor(idx, (B, self.ncoef), torch.int16, "idx")
        self._check_tensor(side, (B, 2), torch.float32, "side")
        rc = _lib().ct_quantize(ctypes.byref(self.g), B, ctypes.c_void_p(coeffs.data_ptr()),
                                ctypes.c_void_p(steps.data_ptr()), stride,
                                ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(side.data_ptr()),
                                ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes, self._stream())
        _check("ct_quantize", rc)
        return idx, side

    def dequantize(self, idx, steps, side, out=None):
        B = self.batch
        self._check_tensor(idx, (B, self.ncoef), torch.int16, "idx")
        self._check_tensor(side, (B, 2), torch.float32, "side")
        steps, stride = self._steps(steps)
        if out is None:
            out = torch.empty((B, self.ncoef), dtype=torch.float32, device=idx.device)
        self._check_tensor(out, (B, self.ncoef), torch.float32, "coeffs")
        rc = _lib().ct_dequantize(ctypes.byref(self.g), B, ctypes.c_void_p(idx.data_ptr()),
                                  ctypes.c_void_p(steps.data_ptr()), stride,
                                  ctypes.c_void_p(side.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  self._stream())
        _check("ct_dequantize", rc)
        return out


def forward(x, levels, dirs):
    """CT of x [B, H, W] float32 (device) -> coefficients [B, ncoef]."""
    B, H, W = x.shape
    return Plan(H, W, levels, dirs, B, x.device).forward(x.contiguous())


def inverse(coeffs, height, width, levels, dirs):
    B = coeffs.shape[0]
    return Plan(height, width, levels, dirs, B, coeffs.device).inverse(coeffs.contiguous())
