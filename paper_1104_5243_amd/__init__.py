"""MI355X (gfx950) cone-beam backprojection: Python binding of libfdk.so.

Thin argument marshalling over the C ABI of include/fdk.h: every step of
the backprojection runs in the library's HIP kernels.  PyTorch supplies the
device memory and the stream.  There is no CPU fallback: if libfdk.so is
missing or cannot be loaded, importing the binding's functions raises.

    import paper_1104_5243_amd as fdk
    vol = torch.zeros(N, N, N, device="cuda")
    fdk.backproject(vol, proj, P, voxel_size, origin)   # vol += B proj
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfdk.so")

FDK_OK = 0
FDK_ERR_INVALID_ARG = -1
FDK_ERR_HIP = -2
FDK_ERR_UNSUPPORTED = -3
DTYPE_F32, DTYPE_F16, DTYPE_BF16 = 0, 1, 2
KERNEL_FUSED, KERNEL_PLAIN = 0, 1

# every symbol include/fdk.h declares
EXPORTS = (
    "fdk_backproject", "fdk_backproject_ex", "fdk_backproject_noalloc", "fdk_backproject_plain",
    "fdk_forward_project", "fdk_convert_storage",
    "fdk_prefilter", "fdk_conv_rows", "fdk_conv_rows_wgrad_workspace", "fdk_conv_rows_wgrad",
    "fdk_scale_groups", "fdk_group_dot", "fdk_relu_backward", "fdk_matvec", "fdk_adam", "fdk_mse",
    "fdk_update_probe", "fdk_profile_begin", "fdk_profile_end", "fdk_set_batch",
    "fdk_set_layout", "fdk_set_row_clamp", "fdk_set_divide", "fdk_release", "fdk_last_error",
    "fdk_version",
)

_lib = None


class FdkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fdk error {code}: {msg}")
        self.code = code


def build() -> str:
    from . import buildlib as _b
    global _lib
    _lib = None
    return _b.build()


def lib():
    """The loaded libfdk.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1104_5243_amd.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, fp, dp, i, f = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                            ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_float)
        L.fdk_backproject.argtypes = [vp, i, f, fp, vp, i, i, i, dp, vp]
        L.fdk_backproject_ex.argtypes = [vp, i, f, fp, vp, i, i, i, i, dp, fp, i, vp]
        L.fdk_backproject_noalloc.argtypes = [vp, i, f, fp, vp, i, i, i, i, dp, fp, vp]
        L.fdk_backproject_plain.argtypes = [vp, i, f, fp, vp, i, i, i, dp, vp]
        L.fdk_forward_project.argtypes = [vp, i, i, i, dp, vp, i, f, fp, vp]
        L.fdk_update_probe.argtypes = [vp, ctypes.c_size_t, f, vp]
        L.fdk_convert_storage.argtypes = [vp, vp, i, i, i, i, vp, vp]
        d = ctypes.c_double
        L.fdk_prefilter.argtypes = [vp, vp, i, i, i, d, d, d, d, d, d, vp]
        sz = ctypes.c_size_t
        L.fdk_conv_rows.argtypes = [vp, vp, vp, vp, i, i, i, i, i, i, i, vp]
        L.fdk_conv_rows_wgrad_workspace.argtypes = [i, i, i]
        L.fdk_conv_rows_wgrad.argtypes = [vp, vp, vp, vp, i, i, i, i, i, i, vp, sz, vp]
        L.fdk_scale_groups.argtypes = [vp, vp, vp, sz, i, i, vp]
        L.fdk_group_dot.argtypes = [vp, vp, vp, sz, i, vp]
        L.fdk_relu_backward.argtypes = [vp, vp, vp, sz, vp]
        L.fdk_matvec.argtypes = [vp, vp, vp, i, i, i, vp]
        L.fdk_adam.argtypes = [vp, vp, vp, vp, i, f, f, f, f, i, vp]
        L.fdk_mse.argtypes = [vp, vp, vp, vp, sz, vp, sz, vp]
        L.fdk_profile_begin.argtypes = []
        L.fdk_profile_end.argtypes = [dp, ctypes.POINTER(ctypes.c_int)]
        L.fdk_set_batch.argtypes = [i]
        L.fdk_set_row_clamp.argtypes = [i]
        L.fdk_set_divide.argtypes = [i]
        L.fdk_release.argtypes = []
        L.fdk_last_error.argtypes = []
        L.fdk_last_error.restype = ctypes.c_char_p
        L.fdk_version.argtypes = []
        for name in EXPORTS:
            if name not in ("fdk_last_error",):
                getattr(L, name).restype = ctypes.c_int
        L.fdk_conv_rows_wgrad_workspace.restype = ctypes.c_size_t
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise FdkError(rc, lib().fdk_last_error().decode())
    return rc


def last_error() -> str:
    return lib().fdk_last_error().decode()


def version() -> int:
    return lib().fdk_version()


# --------------------------------------------------------------------------
# marshalling helpers
# --------------------------------------------------------------------------
def _stream_ptr(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def _mats(P, n_views: int):
    P = np.ascontiguousarray(np.asarray(P, dtype=np.float64).reshape(-1, 12))
    if P.shape[0] != n_views:
        raise ValueError(f"need {n_views} 3x4 matrices, got {P.shape[0]}")
    return P, P.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _origin(origin):
    o = np.ascontiguousarray(np.asarray(origin, dtype=np.float32).reshape(3))
    return o, o.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _dev_tensor(t, name, dtypes, ndim=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")
    return t


def _volume(volume):
    import torch
    _dev_tensor(volume, "volume", (torch.float32,), 3)
    N = volume.shape[0]
    if tuple(volume.shape) != (N, N, N):
        raise ValueError("volume must be N x N x N, indexed [z, y, x]")
    return N


# --------------------------------------------------------------------------
# entry points
# --------------------------------------------------------------------------
def backproject(volume, proj, P, voxel_size: float, origin, stream=None, kernel: str = "fused",
                view_scale=None):
    """volume[z, y, x] += sum over views of the bilinearly sampled, 1/w^2
    weighted projections (see include/fdk.h).  proj: (n_views, H, W) device
    tensor of float32, float16 or bfloat16; P: (n_views, 3, 4) FP64 on the
    host; origin: world centre of voxel (0, 0, 0).  Asynchronous on `stream`
    (default: the current stream)."""
    import torch
    N = _volume(volume)
    _dev_tensor(proj, "proj", (torch.float32, torch.float16, torch.bfloat16), 3)
    if proj.device != volume.device:
        raise ValueError("volume and proj must be on the same device")
    V, H, W = proj.shape
    Pm, Pp = _mats(P, V)
    o, op = _origin(origin)
    dtype = {torch.float32: DTYPE_F32, torch.float16: DTYPE_F16, torch.bfloat16: DTYPE_BF16}[
        proj.dtype]
    flags = {"fused": KERNEL_FUSED, "plain": KERNEL_PLAIN}[kernel]
    vs_arr, vs_ptr = None, None
    if view_scale is not None:
        vs_arr = np.ascontiguousarray(np.asarray(view_scale, dtype=np.float32).reshape(V))
        vs_ptr = vs_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    with torch.cuda.device(volume.device):
        rc = lib().fdk_backproject_ex(
            ctypes.c_void_p(volume.data_ptr()), N, float(voxel_size), op,
            ctypes.c_void_p(proj.data_ptr()), dtype, V, H, W, Pp, vs_ptr, flags,
            _stream_ptr(stream, volume.device))
    _check(rc)
    return volume


def backproject_noalloc(volume, proj, P, voxel_size: float, origin, stream=None,
                        view_scale=None):
    """As `backproject` (fused kernel), through the entry point that
    allocates nothing: the staged views go to the library's fixed scratch
    array (see fdk_backproject_noalloc in include/fdk.h)."""
    import torch
    N = _volume(volume)
    _dev_tensor(proj, "proj", (torch.float32, torch.float16, torch.bfloat16), 3)
    if proj.device != volume.device:
        raise ValueError("volume and proj must be on the same device")
    V, H, W = proj.shape
    Pm, Pp = _mats(P, V)
    o, op = _origin(origin)
    dtype = {torch.float32: DTYPE_F32, torch.float16: DTYPE_F16, torch.bfloat16: DTYPE_BF16}[
        proj.dtype]
    vs_arr, vs_ptr = None, None
    if view_scale is not None:
        vs_arr = np.ascontiguousarray(np.asarray(view_scale, dtype=np.float32).reshape(V))
        vs_ptr = vs_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    with torch.cuda.device(volume.device):
        rc = lib().fdk_backproject_noalloc(
            ctypes.c_void_p(volume.data_ptr()), N, float(voxel_size), op,
            ctypes.c_void_p(proj.data_ptr()), dtype, V, H, W, Pp, vs_ptr,
            _stream_ptr(stream, volume.device))
    _check(rc)
    return volume


def backproject_plain(volume, proj, P, voxel_size: float, origin, stream=None):
    """The plain FP32 path (one thread per voxel, the listing's arithmetic)."""
    import torch
    N = _volume(volume)
    _dev_tensor(proj, "proj", (torch.float32,), 3)
    V, H, W = proj.shape
    Pm, Pp = _mats(P, V)
    o, op = _origin(origin)
    with torch.cuda.device(volume.device):
        rc = lib().fdk_backproject_plain(
            ctypes.c_void_p(volume.data_ptr()), N, float(voxel_size), op,
            ctypes.c_void_p(proj.data_ptr()), V, H, W, Pp, _stream_ptr(stream, volume.device))
    _check(rc)
    return volume


def forward_project(proj, volume, P, voxel_size: float, origin, stream=None):
    """proj[i, k, j] += (B^T volume): the exact transpose of `backproject`."""
    import torch
    N = _volume(volume)
    _dev_tensor(proj, "proj", (torch.float32,), 3)
    V, H, W = proj.shape
    Pm, Pp = _mats(P, V)
    o, op = _origin(origin)
    with torch.cuda.device(volume.device):
        rc = lib().fdk_forward_project(
            ctypes.c_void_p(proj.data_ptr()), V, H, W, Pp, ctypes.c_void_p(volume.data_ptr()), N,
            float(voxel_size), op, _stream_ptr(stream, volume.device))
    _check(rc)
    return proj


def prefilter(out, proj, beta0: float, dbeta: float, delta: float, sid: float, sdd: float,
              pixel: float, stream=None):
    """Feldkamp pre-processing of line integrals on the GPU (cosine weight,
    Parker weight over pi + 2*delta, or 1/2 for delta < 0, Ram-Lak row
    filter, times tau * dbeta): out = filtered(proj), both (V, H, W) float32."""
    import torch
    _dev_tensor(proj, "proj", (torch.float32,), 3)
    _dev_tensor(out, "out", (torch.float32,), 3)
    if out.shape != proj.shape:
        raise ValueError("out and proj must have the same shape")
    V, H, W = proj.shape
    with torch.cuda.device(proj.device):
        rc = lib().fdk_prefilter(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(proj.data_ptr()),
                                 V, H, W, float(beta0), float(dbeta), float(delta), float(sid),
                                 float(sdd), float(pixel), _stream_ptr(stream, proj.device))
    _check(rc)
    return out


# --------------------------------------------------------------------------
# learned-filter kernels (thin wrappers; tensors are float32 CUDA tensors)
# --------------------------------------------------------------------------
CONV_RELU, CONV_ACCUMULATE, CONV_TRANSPOSE, CONV_RELU_MASK = 1, 2, 4, 8


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _f32(*ts):
    import torch
    for t in ts:
        if t is not None:
            _dev_tensor(t, "tensor", (torch.float32,))


def conv_rows(out, x, weight, bias, rows, W, cin, cout, K, pad, flags=0, stream=None):
    """out[r][co][j] = bias[co] + sum w(co,ci,t) x[r][ci][j+t-pad] (see fdk.h)."""
    _f32(out, x, weight, bias)
    with torch_device(x):
        _check(lib().fdk_conv_rows(_p(out), _p(x), _p(weight), _p(bias), rows, W, cin, cout, K,
                                   pad, flags, _stream_ptr(stream, x.device)))
    return out


def conv_rows_wgrad_workspace(cin, cout, K) -> int:
    return int(lib().fdk_conv_rows_wgrad_workspace(cin, cout, K))


def conv_rows_wgrad(dweight, dbias, dout, x, rows, W, cin, cout, K, pad, workspace, stream=None):
    _f32(dweight, dbias, dout, x)
    with torch_device(x):
        _check(lib().fdk_conv_rows_wgrad(_p(dweight), _p(dbias), _p(dout), _p(x), rows, W, cin,
                                         cout, K, pad, _p(workspace),
                                         workspace.numel() * workspace.element_size(),
                                         _stream_ptr(stream, x.device)))


def scale_groups(y, x, scale, group_len, groups, accumulate=False, stream=None):
    _f32(y, x, scale)
    with torch_device(x):
        _check(lib().fdk_scale_groups(_p(y), _p(x), _p(scale), group_len, groups,
                                      1 if accumulate else 0, _stream_ptr(stream, x.device)))
    return y


def group_dot(out, a, b, group_len, groups, stream=None):
    _f32(out, a, b)
    with torch_device(a):
        _check(lib().fdk_group_dot(_p(out), _p(a), _p(b), group_len, groups,
                                   _stream_ptr(stream, a.device)))
    return out


def relu_backward(dx, dy, y, stream=None):
    _f32(dx, dy, y)
    with torch_device(y):
        _check(lib().fdk_relu_backward(_p(dx), _p(dy), _p(y), y.numel(),
                                       _stream_ptr(stream, y.device)))
    return dx


def matvec(y, A, x, rows, cols, transpose=False, stream=None):
    _f32(y, A, x)
    with torch_device(A):
        _check(lib().fdk_matvec(_p(y), _p(A), _p(x), rows, cols, 1 if transpose else 0,
                                _stream_ptr(stream, A.device)))
    return y


def adam(param, m, v, grad, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _f32(param, m, v, grad)
    with torch_device(param):
        _check(lib().fdk_adam(_p(param), _p(m), _p(v), _p(grad), param.numel(), float(lr),
                              float(beta1), float(beta2), float(eps), int(step),
                              _stream_ptr(stream, param.device)))


def mse(grad, loss, a, b, workspace, stream=None):
    """loss[0] = mean((a-b)^2); grad = 2 (a-b)/n if grad is not None."""
    _f32(grad, loss, a, b)
    with torch_device(a):
        _check(lib().fdk_mse(_p(grad), _p(loss), _p(a), _p(b), a.numel(), _p(workspace),
                             workspace.numel() * workspace.element_size(),
                             _stream_ptr(stream, a.device)))


def torch_device(t):
    import torch
    return torch.cuda.device(t.device)


def update_probe(a, s: float = 1.0000001, stream=None):
    """a *= s in place (the paper's update benchmark)."""
    import torch
    _dev_tensor(a, "a", (torch.float32,))
    with torch.cuda.device(a.device):
        _check(lib().fdk_update_probe(ctypes.c_void_p(a.data_ptr()), a.numel(), float(s),
                                      _stream_ptr(stream, a.device)))
    return a


def to_storage(proj, dtype, stream=None):
    """Convert an FP32 (n_views, H, W) device stack to reduced-precision
    storage for `backproject` with the library's conversion kernels
    (fdk_convert_storage).  Returns (stack, view_scale): for float16 each
    view is multiplied by a power of 4 that brings its largest magnitude to
    (2^12, 2^14] before rounding, and view_scale (host float32) undoes it
    exactly inside the library; for bfloat16 view_scale is None."""
    import torch
    if dtype == torch.float32:
        return proj, None
    if dtype not in (torch.float16, torch.bfloat16):
        raise ValueError(f"unsupported storage dtype {dtype}")
    _dev_tensor(proj, "proj", (torch.float32,), 3)
    V, H, W = proj.shape
    out = torch.empty((V, H, W), dtype=dtype, device=proj.device)
    scale = torch.empty(V, dtype=torch.float32, device=proj.device) if dtype == torch.float16 \
        else None
    with torch.cuda.device(proj.device):
        _check(lib().fdk_convert_storage(
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(proj.data_ptr()), V, H, W,
            DTYPE_F16 if dtype == torch.float16 else DTYPE_BF16, _p(scale),
            _stream_ptr(stream, proj.device)))
    return out, (None if scale is None else scale.cpu().numpy())


def profile_begin():
    _check(lib().fdk_profile_begin())


def profile_end():
    """(summed milliseconds of the library's timed kernels, number of
    launches), over every host thread since profile_begin()."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int(0)
    _check(lib().fdk_profile_end(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def set_batch(views_per_pass: int) -> int:
    return _check(lib().fdk_set_batch(int(views_per_pass)))


LAYOUTS = {"rows": 0, "pairs": 1, "quads": 2, "dpairs": 3, "dquads": 4}


def set_layout(layout) -> str:
    """Staged-plane layout of the fused backprojection (a name of LAYOUTS, or
    None to read it back); returns the layout in effect."""
    code = -1 if layout is None else LAYOUTS[layout]
    got = _check(lib().fdk_set_layout(code))
    return next(k for k, v in LAYOUTS.items() if v == got)


def set_row_clamp(clamp=None) -> bool:
    """Whether the fused backprojection clamps every tap row into the staged
    plane (True) or, for FP16/BF16 storage, leaves rows outside it to the
    buffer's range check where the geometry allows (False, the default);
    None reads it back.  Results are bit-identical either way."""
    code = -1 if clamp is None else (1 if clamp else 0)
    return _check(lib().fdk_set_row_clamp(code)) == 1


DIVIDES = {"rcp": 0, "rcp_nr": 1, "ieee": 2, "rcp12": 3}


def set_divide(mode=None) -> str:
    """Reciprocal variant of the fused backprojection's part 1 (a name of
    DIVIDES, or None to read it back); returns the variant in effect."""
    code = -1 if mode is None else DIVIDES[mode]
    got = _check(lib().fdk_set_divide(code))
    return next(k for k, v in DIVIDES.items() if v == got)


def release():
    _check(lib().fdk_release())
