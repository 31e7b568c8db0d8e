"""Python binding of libct (ctypes): argument marshalling only.

Every transform step runs in the HIP kernels of libct.so; this module only
converts torch tensors to device pointers and sizes, allocates caller-owned
workspace, and checks return codes. There is no fallback: if the library is
missing or a call fails, an exception is raised.

Names follow the C ABI (include/ct.h): forward, inverse, quantize,
dequantize, forward_adjoint, inverse_adjoint, layout, rgb_to_ycocg,
ycocg_to_rgb, lowpass_diff, motion_search, mc_residual, rle_encode,
rle_decode_host, deflate_host, inflate_host.
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
                ("levels", ctypes.c_int32), ("dirs", ctypes.c_int32 * MAX_LEVELS),
                ("filters", ctypes.c_int32), ("recon", ctypes.c_int32)]


# filter pair and LP reconstruction of a geometry (ct_geom.filters / .recon)
FILTERS = {"97": 0, "53": 1}
RECON = {"dual": 0, "ba": 1}


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
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("alg_bytes", ctypes.c_double)]


class StreamDesc(ctypes.Structure):
    _fields_ = [("geom", Geom), ("batch", ctypes.c_int32),
                ("planes", ctypes.c_void_p), ("coeffs", ctypes.c_void_p),
                ("idx", ctypes.c_void_p), ("side", ctypes.c_void_p),
                ("steps", ctypes.c_void_p), ("steps_stride", ctypes.c_int32),
                ("deq", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_int32), ("stages", ctypes.c_int32),
                ("work_items", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("autotuned", ctypes.c_int32),
                ("levels_paired", ctypes.c_int32), ("levels_single", ctypes.c_int32),
                ("levels_triple", ctypes.c_int32), ("workspace_bytes", ctypes.c_int64),
                ("levels_short_blocks", ctypes.c_int32), ("levels_tall_blocks", ctypes.c_int32),
                ("levels_sized_blocks", ctypes.c_int32)]


PLAN_GRAPH = 1
PLAN_AUTOTUNE = 2
PLAN_FUSED = 4


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
            "ct_quantize_noalloc": [G, i32, P, P, i32, P, P, P],
            "ct_dequantize": [G, i32, P, P, i32, P, P, P],
            "ct_encode": [G, i32, P, P, i32, P, P, P, P, sz, P],
            "ct_decode": [G, i32, P, P, i32, P, P, P, sz, P],
            "ct_encode_rgb": [G, i32, P, P, i32, P, P, P, sz, P],
            "ct_rgb_to_ycocg": [i32, i32, i32, i32, P, P, P, P, P],
            "ct_ycocg_to_rgb": [i32, i32, i32, i32, P, P, P, P, P],
            "ct_lowpass_diff": [G, i32, P, i32, P],
            "ct_motion_search": [i32, i32, i32, i32, P, P, P, P, P],
            "ct_mc_residual": [G, i32, i32, P, P, P, i32, i32, i32, i32, P, P],
            "ct_rle_workspace_bytes": [G, i32, ctypes.POINTER(sz)],
            "ct_rle_encode": [G, i32, P, i32, P, P, P, sz, P],
            "ct_rle_decode_host": [G, P, P, i32, P],
            "ct_deflate_host": [P, P, i32, i32, i32, P, sz, P, ctypes.POINTER(sz)],
            "ct_inflate_host": [P, P, P, i32, i32, P],
            "ct_autotune": [G, i32, P, sz, P],
            "ct_autotune_clear": [],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.ct_profile_enable.argtypes = [i32, i32]
        lib.ct_profile_enable.restype = ctypes.c_int
        lib.ct_profile_collect.argtypes = [ctypes.POINTER(KernelStat), i32, ctypes.POINTER(i32)]
        lib.ct_profile_collect.restype = ctypes.c_int
        lib.ct_plan_create.argtypes = [ctypes.POINTER(StreamDesc), i32, i32, ctypes.POINTER(ctypes.c_void_p)]
        lib.ct_plan_create.restype = ctypes.c_int
        for name in ("ct_plan_run", "ct_plan_run_plain"):
            getattr(lib, name).argtypes = [ctypes.c_void_p, ctypes.c_void_p]
            getattr(lib, name).restype = ctypes.c_int
        lib.ct_plan_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(PlanInfo)]
        lib.ct_plan_info.restype = ctypes.c_int
        lib.ct_plan_destroy.argtypes = [ctypes.c_void_p]
        lib.ct_plan_destroy.restype = None
        lib.ct_strerror.argtypes = [ctypes.c_int]
        lib.ct_strerror.restype = ctypes.c_char_p
        _LIB = lib
    return _LIB


def geom(height, width, levels, dirs, filters="97", recon="dual"):
    """ct_geom; filters "97" (the 9-7 pair) or "53" (LeGall 5/3), recon "dual"
    (dual-frame LP synthesis) or "ba" (Burt-Adelson); the codes 0 / 1 work too."""
    d = list(dirs) + [0] * (MAX_LEVELS - len(dirs))
    f = FILTERS.get(filters, filters)
    r = RECON.get(recon, recon)
    return Geom(int(height), int(width), int(levels), (ctypes.c_int32 * MAX_LEVELS)(*d), int(f), int(r))


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


def profile_collect(alg=False):
    """{kernel: (launches, total_ms, compulsory bytes)} since the last collect;
    with alg=True the tuples also carry the algorithmic bytes."""
    cap = 64
    out = (KernelStat * cap)()
    n = ctypes.c_int32(0)
    _check("ct_profile_collect", _lib().ct_profile_collect(out, cap, ctypes.byref(n)))
    res = {}
    for i in range(min(n.value, cap)):
        s = out[i]
        t = (int(s.launches), float(s.total_ms), float(s.bytes))
        res[s.name.decode()] = t + (float(s.alg_bytes),) if alg else t
    return res


def autotune_clear():
    """Forget this process's tuned tile shapes (ct_autotune_clear)."""
    _check("ct_autotune_clear", _lib().ct_autotune_clear())


def workspace_bytes(height, width, levels, dirs, batch):
    g = geom(height, width, levels, dirs)
    n = ctypes.c_size_t(0)
    _check("ct_workspace_bytes", _lib().ct_workspace_bytes(ctypes.byref(g), int(batch), ctypes.byref(n)))
    return n.value


class Plan:
    """Geometry + reusable workspace for one batch size on one device."""

    def __init__(self, height, width, levels, dirs, batch, device="cuda", filters="97", recon="dual"):
        self.height, self.width, self.levels = int(height), int(width), int(levels)
        self.dirs = [int(d) for d in dirs]
        self.batch = int(batch)
        self.g = geom(height, width, levels, dirs, filters, recon)
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

    def autotune(self):
        """Tune the split passes' tile shapes for this geometry and batch
        (ct_autotune); later calls of every plan of this shape in this process
        use the choices. Returns nothing; blocks until the timing is done."""
        _check("ct_autotune", _lib().ct_autotune(ctypes.byref(self.g), self.batch,
                                                 ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                                 self._stream()))

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

    def quantize_noalloc(self, coeffs, steps, idx=None, side=None):
        """ct_quantize_noalloc: as quantize(), with the library's static scratch
        instead of the plan's workspace (at most 1024 planes)."""
        B = self.batch
        self._check_tensor(coeffs, (B, self.ncoef), torch.float32, "coeffs")
        steps, stride = self._steps(steps)
        if idx is None:
            idx = torch.empty((B, self.ncoef), dtype=torch.int16, device=coeffs.device)
        if side is None:
            side = torch.empty((B, 2), dtype=torch.float32, device=coeffs.device)
        self._check_tensor(idx, (B, self.ncoef), torch.int16, "idx")
        self._check_tensor(side, (B, 2), torch.float32, "side")
        rc = _lib().ct_quantize_noalloc(ctypes.byref(self.g), B, ctypes.c_void_p(coeffs.data_ptr()),
                                        ctypes.c_void_p(steps.data_ptr()), stride,
                                        ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(side.data_ptr()),
                                        self._stream())
        _check("ct_quantize_noalloc", rc)
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

    def lowpass_diff(self, idx, inverse=False):
        """K-frame lowpass filtering of idx [B, ncoef] int16 in place (ct_lowpass_diff)."""
        self._check_tensor(idx, (self.batch, self.ncoef), torch.int16, "idx")
        rc = _lib().ct_lowpass_diff(ctypes.byref(self.g), self.batch, ctypes.c_void_p(idx.data_ptr()),
                                    1 if inverse else 0, self._stream())
        _check("ct_lowpass_diff", rc)
        return idx

    def mc_residual(self, cur, prev, mv, n=1, group=1, inverse=False, out=None):
        """P-frame components (ct_mc_residual): cur - prediction(prev), or with
        inverse=True cur + prediction(prev); int16 [B, ncoef]. mv is the int16
        [ceil(B / group), nby, nbx, 2] output of motion_search."""
        B = self.batch
        self._check_tensor(cur, (B, self.ncoef), torch.int16, "cur")
        self._check_tensor(prev, (B, self.ncoef), torch.int16, "prev")
        if mv.dim() != 4 or mv.shape[0] != -(-B // group) or mv.shape[3] != 2:
            raise ValueError("mv must be [ceil(B / group), nby, nbx, 2]")
        self._check_tensor(mv, tuple(mv.shape), torch.int16, "mv")
        if out is None:
            out = torch.empty_like(cur)
        self._check_tensor(out, (B, self.ncoef), torch.int16, "out")
        rc = _lib().ct_mc_residual(ctypes.byref(self.g), B, int(n), ctypes.c_void_p(cur.data_ptr()),
                                   ctypes.c_void_p(prev.data_ptr()), ctypes.c_void_p(mv.data_ptr()),
                                   int(mv.shape[1]), int(mv.shape[2]), int(group), 1 if inverse else 0,
                                   ctypes.c_void_p(out.data_ptr()), self._stream())
        _check("ct_mc_residual", rc)
        return out

    def rle_encode(self, idx, p_frame, symbols=None, sub_off=None):
        """Zero-run coding (ct_rle_encode): (symbols int16 [B, 2 ncoef], sub_off
        int32 [B, nsub + 1]); plane b's stream is symbols[b, :sub_off[b, -1]]."""
        B = self.batch
        self._check_tensor(idx, (B, self.ncoef), torch.int16, "idx")
        if symbols is None:
            symbols = torch.empty((B, 2 * self.ncoef), dtype=torch.int16, device=idx.device)
        if sub_off is None:
            sub_off = torch.empty((B, self.nsub + 1), dtype=torch.int32, device=idx.device)
        self._check_tensor(symbols, (B, 2 * self.ncoef), torch.int16, "symbols")
        self._check_tensor(sub_off, (B, self.nsub + 1), torch.int32, "sub_off")
        if not hasattr(self, "_rle_ws"):
            n = ctypes.c_size_t(0)
            _check("ct_rle_workspace_bytes", _lib().ct_rle_workspace_bytes(ctypes.byref(self.g), B, ctypes.byref(n)))
            self._rle_ws = torch.empty(max(1, n.value), dtype=torch.uint8, device=self.device)
        rc = _lib().ct_rle_encode(ctypes.byref(self.g), B, ctypes.c_void_p(idx.data_ptr()), 1 if p_frame else 0,
                                  ctypes.c_void_p(symbols.data_ptr()), ctypes.c_void_p(sub_off.data_ptr()),
                                  ctypes.c_void_p(self._rle_ws.data_ptr()), self._rle_ws.numel(), self._stream())
        _check("ct_rle_encode", rc)
        return symbols, sub_off

    def rle_decode_host(self, symbols, sub_off, p_frame):
        """One plane's indices from its symbol stream (ct_rle_decode_host, host
        code): symbols int16 and sub_off int32 numpy arrays."""
        import numpy as np
        sym = np.ascontiguousarray(symbols, dtype=np.int16)
        off = np.ascontiguousarray(sub_off, dtype=np.int32)
        out = np.empty(self.ncoef, dtype=np.int16)
        rc = _lib().ct_rle_decode_host(ctypes.byref(self.g), sym.ctypes.data, off.ctypes.data,
                                       1 if p_frame else 0, out.ctypes.data)
        _check("ct_rle_decode_host", rc)
        return out

    def encode(self, x, steps, idx=None, side=None, coeffs=None):
        """Fused forward CT + quantise: (idx [B, ncoef] int16, side [B, 2]);
        `coeffs` (optional [B, ncoef] float32) also receives the coefficients."""
        B = self.batch
        self._check_tensor(x, (B, self.height, self.width), torch.float32, "planes")
        steps, stride = self._steps(steps)
        if idx is None:
            idx = torch.empty((B, self.ncoef), dtype=torch.int16, device=x.device)
        if side is None:
            side = torch.empty((B, 2), dtype=torch.float32, device=x.device)
        self._check_tensor(idx, (B, self.ncoef), torch.int16, "idx")
        self._check_tensor(side, (B, 2), torch.float32, "side")
        cptr = None
        if coeffs is not None:
            self._check_tensor(coeffs, (B, self.ncoef), torch.float32, "coeffs")
            cptr = coeffs.data_ptr()
        rc = _lib().ct_encode(ctypes.byref(self.g), B, ctypes.c_void_p(x.data_ptr()),
                              ctypes.c_void_p(steps.data_ptr()), stride, ctypes.c_void_p(idx.data_ptr()),
                              ctypes.c_void_p(side.data_ptr()), ctypes.c_void_p(cptr),
                              ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes, self._stream())
        _check("ct_encode", rc)
        return idx, side

    def encode_rgb(self, rgb, steps, idx=None, side=None):
        """Fused colour transform + forward CT + quantise of uint8 RGB frames
        rgb [F, H, W, 3] (the plan's batch is 3 F: planes Y, Co + 127,
        Cg + 127 of each frame): (idx [3 F, ncoef] int16, side [3 F, 2])."""
        B = self.batch
        if B % 3:
            raise ValueError("encode_rgb needs a plan whose batch is 3 * frames")
        F = B // 3
        self._check_tensor(rgb, (F, self.height, self.width, 3), torch.uint8, "rgb")
        steps, stride = self._steps(steps)
        if idx is None:
            idx = torch.empty((B, self.ncoef), dtype=torch.int16, device=rgb.device)
        if side is None:
            side = torch.empty((B, 2), dtype=torch.float32, device=rgb.device)
        self._check_tensor(idx, (B, self.ncoef), torch.int16, "idx")
        self._check_tensor(side, (B, 2), torch.float32, "side")
        rc = _lib().ct_encode_rgb(ctypes.byref(self.g), F, ctypes.c_void_p(rgb.data_ptr()),
                                  ctypes.c_void_p(steps.data_ptr()), stride, ctypes.c_void_p(idx.data_ptr()),
                                  ctypes.c_void_p(side.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                  self.ws_bytes, self._stream())
        _check("ct_encode_rgb", rc)
        return idx, side

    def decode(self, idx, steps, side, out=None):
        """Fused dequantise + inverse CT: planes [B, H, W] float32."""
        B = self.batch
        self._check_tensor(idx, (B, self.ncoef), torch.int16, "idx")
        self._check_tensor(side, (B, 2), torch.float32, "side")
        steps, stride = self._steps(steps)
        if out is None:
            out = torch.empty((B, self.height, self.width), dtype=torch.float32, device=idx.device)
        self._check_tensor(out, (B, self.height, self.width), torch.float32, "planes")
        rc = _lib().ct_decode(ctypes.byref(self.g), B, ctypes.c_void_p(idx.data_ptr()),
                              ctypes.c_void_p(steps.data_ptr()), stride, ctypes.c_void_p(side.data_ptr()),
                              ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                              self.ws_bytes, self._stream())
        _check("ct_decode", rc)
        return out


def forward(x, levels, dirs):
    """CT of x [B, H, W] float32 (device) -> coefficients [B, ncoef]."""
    B, H, W = x.shape
    return Plan(H, W, levels, dirs, B, x.device).forward(x.contiguous())


def inverse(coeffs, height, width, levels, dirs):
    B = coeffs.shape[0]
    return Plan(height, width, levels, dirs, B, coeffs.device).inverse(coeffs.contiguous())


def _cuda(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def chroma_shape(height, width, n):
    """(ceil(H / n), ceil(W / n)); the library checks the range of n."""
    if int(n) < 1:
        raise ValueError(f"chroma factor must be >= 1, got {n}")
    return -(-int(height) // int(n)), -(-int(width) // int(n))


def rgb_to_ycocg(rgb, n, y=None, co=None, cg=None):
    """uint8 RGB [B, H, W, 3] -> (Y [B, H, W], Co + 127, Cg + 127 [B, Hc, Wc]) float32."""
    if rgb.dim() != 4 or rgb.shape[-1] != 3:
        raise ValueError("rgb must be [B, H, W, 3]")
    B, H, W, _ = rgb.shape
    Hc, Wc = chroma_shape(H, W, n)
    _cuda(rgb, torch.uint8, (B, H, W, 3), "rgb")
    dev = rgb.device
    y = torch.empty((B, H, W), dtype=torch.float32, device=dev) if y is None else y
    co = torch.empty((B, Hc, Wc), dtype=torch.float32, device=dev) if co is None else co
    cg = torch.empty((B, Hc, Wc), dtype=torch.float32, device=dev) if cg is None else cg
    _cuda(y, torch.float32, (B, H, W), "y")
    _cuda(co, torch.float32, (B, Hc, Wc), "co")
    _cuda(cg, torch.float32, (B, Hc, Wc), "cg")
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    rc = _lib().ct_rgb_to_ycocg(B, H, W, int(n), ctypes.c_void_p(rgb.data_ptr()),
                                ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(co.data_ptr()),
                                ctypes.c_void_p(cg.data_ptr()), st)
    _check("ct_rgb_to_ycocg", rc)
    return y, co, cg


def ycocg_to_rgb(y, co, cg, n, out=None):
    """(Y [B, H, W], Co + 127, Cg + 127 [B, Hc, Wc]) -> float32 RGB [B, H, W, 3]."""
    if y.dim() != 3:
        raise ValueError("y must be [B, H, W]")
    B, H, W = y.shape
    Hc, Wc = chroma_shape(H, W, n)
    _cuda(y, torch.float32, (B, H, W), "y")
    _cuda(co, torch.float32, (B, Hc, Wc), "co")
    _cuda(cg, torch.float32, (B, Hc, Wc), "cg")
    out = torch.empty((B, H, W, 3), dtype=torch.float32, device=y.device) if out is None else out
    _cuda(out, torch.float32, (B, H, W, 3), "rgb")
    st = ctypes.c_void_p(torch.cuda.current_stream(y.device).cuda_stream)
    rc = _lib().ct_ycocg_to_rgb(B, H, W, int(n), ctypes.c_void_p(y.data_ptr()),
                                ctypes.c_void_p(co.data_ptr()), ctypes.c_void_p(cg.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), st)
    _check("ct_ycocg_to_rgb", rc)
    return out


def deflate_host(symbols, sub_off, mode=0, level=6):
    """DEFLATE of one plane's symbol stream (ct_deflate_host): (compressed
    bytes, per-part byte counts); mode 0 per component, mode 1 whole plane."""
    import numpy as np
    sym = np.ascontiguousarray(symbols, dtype=np.int16)
    off = np.ascontiguousarray(sub_off, dtype=np.int32)
    nsub = len(off) - 1
    cap = 2 * sym.nbytes + 64 * nsub + 1024
    out = np.empty(cap, dtype=np.uint8)
    parts = np.zeros(nsub if mode == 0 else 1, dtype=np.uint32)
    total = ctypes.c_size_t(0)
    rc = _lib().ct_deflate_host(sym.ctypes.data, off.ctypes.data, nsub, int(mode), int(level), out.ctypes.data,
                                cap, parts.ctypes.data, ctypes.byref(total))
    _check("ct_deflate_host", rc)
    return out[:total.value].tobytes(), parts


def inflate_host(blob, parts, sub_off, mode=0):
    """Inverse of deflate_host: the int16 symbol stream."""
    import numpy as np
    off = np.ascontiguousarray(sub_off, dtype=np.int32)
    buf = np.frombuffer(blob, dtype=np.uint8).copy()
    parts = np.ascontiguousarray(parts, dtype=np.uint32)
    sym = np.empty(int(off[-1]), dtype=np.int16)
    rc = _lib().ct_inflate_host(buf.ctypes.data, parts.ctypes.data, off.ctypes.data, len(off) - 1, int(mode),
                                sym.ctypes.data)
    _check("ct_inflate_host", rc)
    return sym


def motion_search(cur, prev, w, mv=None, ssd=None, want_ssd=True):
    """Block matching of cur [B, H, W] against prev [B, H, W] (float32 luminance):
    (mv [B, nby, nbx, 2] int16 (dy, dx), ssd [B, nby, nbx] int32 or None)."""
    if cur.dim() != 3:
        raise ValueError("cur must be [B, H, W]")
    B, H, W = cur.shape
    nby, nbx = -(-H // 16), -(-W // 16)
    _cuda(cur, torch.float32, (B, H, W), "cur")
    _cuda(prev, torch.float32, (B, H, W), "prev")
    mv = torch.empty((B, nby, nbx, 2), dtype=torch.int16, device=cur.device) if mv is None else mv
    _cuda(mv, torch.int16, (B, nby, nbx, 2), "mv")
    if want_ssd:
        ssd = torch.empty((B, nby, nbx), dtype=torch.int32, device=cur.device) if ssd is None else ssd
        _cuda(ssd, torch.int32, (B, nby, nbx), "ssd")
    else:
        ssd = None
    st = ctypes.c_void_p(torch.cuda.current_stream(cur.device).cuda_stream)
    rc = _lib().ct_motion_search(B, H, W, int(w), ctypes.c_void_p(cur.data_ptr()),
                                 ctypes.c_void_p(prev.data_ptr()), ctypes.c_void_p(mv.data_ptr()),
                                 ctypes.c_void_p(ssd.data_ptr() if ssd is not None else None), st)
    _check("ct_motion_search", rc)
    return mv, ssd


class Batched:
    """Many streams of uneven geometry in one graph launch (ct_plan_*).

    streams: list of dicts with keys height, width, levels, dirs, planes
    ([batch, H, W] float32 CUDA tensor) and steps ([nsub] or [batch, nsub]
    float32 CUDA tensor), and optionally filters and recon (see geom). Output buffers are allocated here and exposed per
    stream as coeffs, idx, side, deq, out. With fused=True the plan runs the
    fused encoder and decoder: coeffs and deq are None (not written).
    """

    def __init__(self, streams, graph=True, autotune=False, device="cuda", fused=False):
        self.device = torch.device(device)
        self.streams = []
        descs = (StreamDesc * len(streams))()
        for i, st in enumerate(streams):
            H, W, J, dirs = st["height"], st["width"], st["levels"], st["dirs"]
            planes = st["planes"]
            B = planes.shape[0]
            lay, _ = layout(H, W, J, dirs)
            n = int(lay.ncoef)
            steps = st["steps"].contiguous()
            stride = 0 if steps.dim() == 1 else int(lay.nsub)
            flt = None if fused else torch.empty((B, n), dtype=torch.float32, device=self.device)
            rec = dict(height=H, width=W, levels=J, dirs=list(dirs), batch=B, ncoef=n,
                       planes=planes.contiguous(), steps=steps,
                       coeffs=flt,
                       idx=torch.empty((B, n), dtype=torch.int16, device=self.device),
                       side=torch.empty((B, 2), dtype=torch.float32, device=self.device),
                       deq=None if fused else torch.empty((B, n), dtype=torch.float32, device=self.device),
                       out=torch.empty((B, H, W), dtype=torch.float32, device=self.device))
            self.streams.append(rec)
            d = descs[i]
            d.geom = geom(H, W, J, dirs, st.get("filters", "97"), st.get("recon", "dual"))
            d.batch = B
            d.planes = rec["planes"].data_ptr()
            d.coeffs = rec["coeffs"].data_ptr() if rec["coeffs"] is not None else None
            d.idx = rec["idx"].data_ptr()
            d.side = rec["side"].data_ptr()
            d.steps = steps.data_ptr()
            d.steps_stride = stride
            d.deq = rec["deq"].data_ptr() if rec["deq"] is not None else None
            d.out = rec["out"].data_ptr()
        flags = (PLAN_GRAPH if graph else 0) | (PLAN_AUTOTUNE if autotune else 0) | (PLAN_FUSED if fused else 0)
        handle = ctypes.c_void_p()
        torch.cuda.synchronize(self.device)
        _check("ct_plan_create", _lib().ct_plan_create(descs, len(streams), flags, ctypes.byref(handle)))
        self.handle = handle

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def run(self):
        _check("ct_plan_run", _lib().ct_plan_run(self.handle, self._stream()))

    def run_plain(self):
        _check("ct_plan_run_plain", _lib().ct_plan_run_plain(self.handle, self._stream()))

    def info(self):
        inf = PlanInfo()
        _check("ct_plan_info", _lib().ct_plan_info(self.handle, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in PlanInfo._fields_}

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            _lib().ct_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
