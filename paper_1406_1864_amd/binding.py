"""ctypes binding of libfwi (include/fwi.h): argument marshalling only.

Every function named ``fwi_*`` here calls the C entry point of the same name
with the same arguments; torch tensors are accepted wherever the C ABI takes a
device pointer, and ``synthetic.Grid`` / ``synthetic.Geometry`` wherever it
takes ``fwi_grid`` / ``fwi_geometry``.  All computation happens in the HIP
kernels of ``libfwi.so``; nothing here falls back to another implementation:
if the library is missing or fails to load, every call raises.

The helpers below the raw bindings (``workspace``, ``forward``, ``gradient``,
``hessian_diag``, ``precondition``) only allocate torch tensors for outputs and
workspace and then call the raw bindings.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfwi.so")
HEADER_PATH = os.path.join(os.path.dirname(HERE), "include", "fwi.h")

FWI_OK = 0
FWI_ERR_ARG = -1
FWI_ERR_GEOM = -2
FWI_ERR_CFL = -3
FWI_ERR_WORKSPACE = -4
FWI_ERR_HIP = -5
FWI_ERR_NONFINITE = -6
FWI_ERR_STATE = -7
FWI_CFL_LIMIT = 0.5546324796655889
FWI_STATIC_SCRATCH_BYTES = 64 << 20   # the static scratch of fwi_gradient_static, per GPU

EXEC_BATCHED, EXEC_PLAIN = 0, 1
MISFIT_L2, MISFIT_TIME_INTEGRAL = 0, 1
HESS_EQ1, HESS_OFFSET = 0, 1
RCV_PM, RCV_NONE = 0, 1
PRECOND_SHOT, PRECOND_OFFSET = 0, 1
DFT_FP32, DFT_BF16X3 = 0, 1
WS_FORWARD, WS_GRADIENT, WS_HESSIAN, WS_AUTOGRAD, WS_PRECOND, WS_EXTIMAGE, WS_BORN, WS_GNHVP = range(8)

MISFIT_EQ3_LITERAL = 2
_MISFIT = {"l2": MISFIT_L2, "int": MISFIT_TIME_INTEGRAL, "time_integral": MISFIT_TIME_INTEGRAL,
           "eq3": MISFIT_EQ3_LITERAL, 0: 0, 1: 1, 2: 2}
_RCV = {"pm": RCV_PM, "none": RCV_NONE, 0: 0, 1: 1}


class FwiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libfwi error {code}: {msg}")
        self.code = code


class fwi_grid(ctypes.Structure):
    _fields_ = [("nz", c_int32), ("nx", c_int32), ("dx", c_double), ("dt", c_double),
                ("nt_max", c_int32), ("nsponge", c_int32), ("v_ref", c_double), ("free_surface", c_int32)]


class fwi_geometry(ctypes.Structure):
    _fields_ = [("nshot", c_int32), ("src_iz", POINTER(c_int32)), ("src_ix", POINTER(c_int32)),
                ("rec_ptr", POINTER(c_int32)), ("rec_iz", POINTER(c_int32)),
                ("rec_ix", POINTER(c_int32)), ("nt", POINTER(c_int32))]


class fwi_exec(ctypes.Structure):
    _fields_ = [("mode", c_int32), ("shots_in_flight", c_int32), ("tile_rows", c_int32),
                ("graph_steps", c_int32), ("autotune", c_int32), ("prefetch", c_int32),
                ("prefetch_reverse", c_int32), ("shots_in_flight_reverse", c_int32),
                ("tile_rows_reverse", c_int32), ("reverse_steps", c_int32), ("forward_steps", c_int32),
                ("graph_branches", c_int32)]


_lib = None
_SIGS = {
    "fwi_workspace_bytes": (c_size_t, [POINTER(fwi_grid), POINTER(fwi_geometry), POINTER(fwi_exec), c_int, c_int]),
    "fwi_validate": (c_int, [POINTER(fwi_grid), POINTER(fwi_geometry)]),
    "fwi_exec_query": (c_int, [POINTER(fwi_grid), POINTER(fwi_geometry), POINTER(fwi_exec), c_int,
                               POINTER(fwi_exec)]),
    "fwi_forward": (c_int, [POINTER(fwi_grid), POINTER(fwi_geometry), POINTER(fwi_exec), c_void_p, c_void_p,
                            c_int64, c_void_p, c_void_p, c_size_t, c_void_p]),
    "fwi_gradient": (c_int, [POINTER(fwi_grid), POINTER(fwi_geometry), POINTER(fwi_exec), c_void_p, c_void_p,
                             c_int64, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p,
                             c_void_p, c_size_t, c_void_p]),
    "fwi_gradient_static": (c_int, [POINTER(fwi_grid), POINTER(fwi_geometry), POINTER(fwi_exec), c_void_p,
                                    c_void_p, c_int64, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_int, c_int,
                                    c_void_p, c_void_p]),
    "fwi_extended_image": (c_int, [POINTER(fwi_grid), POINTER(fwi_geometry), POINTER(fwi_exec), c_void_p,
                                   c_void_p, c_int64, c_void_p, c_int, c_void_p, c_void_p, c_int, c_void_p,
                                   c_void_p, c_size_t, c_void_p]),
    "fwi_misfit_value": (c_int, [POINTER(fwi_grid), POINTER(fwi_geometry), POINTER(fwi_exec), c_void_p,
                                 c_void_p, c_int64, c_void_p, c_int, c_void_p, c_void_p, c_size_t, c_void_p]),
    "fwi_born": (c_int, [POINTER(fwi_grid), POINTER(fwi_geometry), POINTER(fwi_exec), c_void_p, c_void_p,
                         c_int64, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "fwi_gn_hvp": (c_int, [POINTER(fwi_grid), POINTER(fwi_geometry), POINTER(fwi_exec), c_void_p, c_void_p,
                           c_int64, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "fwi_hessian_diag": (c_int, [POINTER(fwi_grid), POINTER(fwi_geometry), POINTER(fwi_exec), c_void_p,
                                 c_void_p, c_int64, c_int, c_int, c_int, c_void_p, c_void_p, c_size_t,
                                 c_void_p]),
    "fwi_misfit_forward": (c_int, [POINTER(fwi_grid), POINTER(fwi_geometry), POINTER(fwi_exec), c_void_p,
                                   c_void_p, c_int64, c_void_p, c_int, c_void_p, c_void_p, c_size_t,
                                   c_void_p]),
    "fwi_misfit_backward": (c_int, [POINTER(fwi_grid), POINTER(fwi_geometry), POINTER(fwi_exec), c_void_p,
                                    c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p,
                                    c_void_p, c_size_t, c_void_p]),
    "fwi_offset_diag_exact_workspace_bytes": (c_size_t, [POINTER(fwi_grid), POINTER(fwi_geometry),
                                                         POINTER(fwi_exec), c_int, ctypes.c_double, c_int]),
    "fwi_offset_diag_exact": (c_int, [POINTER(fwi_grid), POINTER(fwi_geometry), POINTER(fwi_exec), c_void_p,
                                      c_void_p, c_int64, c_int, ctypes.c_double, c_int, c_void_p, c_void_p,
                                      c_size_t, c_void_p]),
    "fwi_precondition": (c_int, [POINTER(fwi_grid), c_void_p, c_void_p, c_int, c_void_p, c_int, c_float,
                                 c_void_p, c_void_p, c_size_t, c_void_p]),
    "fwi_status": (c_int, [c_void_p, c_void_p]),
    "fwi_last_error": (ctypes.c_char_p, []),
    "fwi_tune_reset": (None, []),
}


def load():
    """Load libfwi.so (raises if it is not built or cannot be loaded)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1406_1864_amd.build` "
                           "or __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def header_functions():
    """Names of the functions declared in include/fwi.h."""
    src = open(HEADER_PATH).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fwi_[a-z_]+)\s*\(", src)))


def last_error() -> str:
    return load().fwi_last_error().decode()


def _check(rc):
    if rc != FWI_OK:
        raise FwiError(rc, last_error())
    return rc


# ------------------------------------------------------------------ marshalling
def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def make_grid(grid) -> fwi_grid:
    return fwi_grid(int(grid.nz), int(grid.nx), float(grid.dx), float(grid.dt), int(grid.nt_max),
                    int(grid.nsponge), float(grid.v_ref), int(bool(getattr(grid, "free_surface", False))))


class GeometryC:
    """fwi_geometry plus the int32 arrays it points to (kept alive here)."""

    def __init__(self, geom):
        self.arrays = [_i32(geom.src_iz), _i32(geom.src_ix), _i32(geom.rec_ptr), _i32(geom.rec_iz),
                       _i32(geom.rec_ix), _i32(geom.nt)]
        ptrs = [a.ctypes.data_as(POINTER(c_int32)) for a in self.arrays]
        self.struct = fwi_geometry(int(geom.nshot), *ptrs)


def make_exec(mode=EXEC_BATCHED, shots_in_flight=0, tile_rows=0, graph_steps=0, autotune=0,
              prefetch=0, prefetch_reverse=0, shots_in_flight_reverse=0, tile_rows_reverse=0,
              reverse_steps=0, forward_steps=0, graph_branches=0) -> fwi_exec:
    return fwi_exec(int(mode), int(shots_in_flight), int(tile_rows), int(graph_steps), int(autotune),
                    int(prefetch), int(prefetch_reverse), int(shots_in_flight_reverse), int(tile_rows_reverse),
                    int(reverse_steps), int(forward_steps), int(graph_branches))


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream)


def _ex(exec_):
    return ctypes.byref(exec_) if exec_ is not None else None


def _geo(geom):
    return geom if isinstance(geom, GeometryC) else GeometryC(geom)


# ------------------------------------------------------------------ raw ABI
def fwi_workspace_bytes(grid, geom, exec_, what, hmax=0) -> int:
    g, G = make_grid(grid), _geo(geom)
    return int(load().fwi_workspace_bytes(ctypes.byref(g), ctypes.byref(G.struct), _ex(exec_), int(what),
                                          int(hmax)))


def fwi_validate(grid, geom) -> int:
    g, G = make_grid(grid), _geo(geom)
    return int(load().fwi_validate(ctypes.byref(g), ctypes.byref(G.struct)))


def fwi_exec_query(grid, geom, exec_, what) -> dict:
    g, G = make_grid(grid), _geo(geom)
    out = fwi_exec()
    _check(load().fwi_exec_query(ctypes.byref(g), ctypes.byref(G.struct), _ex(exec_), int(what), ctypes.byref(out)))
    return {k: getattr(out, k) for k, _ in fwi_exec._fields_}


def fwi_forward(grid, geom, exec_, v, wavelet, wavelet_stride, data, workspace, ws_bytes, stream=None):
    g, G = make_grid(grid), _geo(geom)
    return _check(load().fwi_forward(ctypes.byref(g), ctypes.byref(G.struct), _ex(exec_), _ptr(v), _ptr(wavelet),
                                     int(wavelet_stride), _ptr(data), _ptr(workspace), int(ws_bytes),
                                     _stream(stream)))


def fwi_gradient(grid, geom, exec_, v, wavelet, wavelet_stride, d_obs, misfit, J, grad, illum, hmax, rcv_model,
                 offset_diag, workspace, ws_bytes, stream=None):
    g, G = make_grid(grid), _geo(geom)
    return _check(load().fwi_gradient(ctypes.byref(g), ctypes.byref(G.struct), _ex(exec_), _ptr(v),
                                      _ptr(wavelet), int(wavelet_stride), _ptr(d_obs), _MISFIT[misfit], _ptr(J),
                                      _ptr(grad), _ptr(illum), int(hmax), _RCV[rcv_model], _ptr(offset_diag),
                                      _ptr(workspace), int(ws_bytes), _stream(stream)))


def fwi_gradient_static(grid, geom, exec_, v, wavelet, wavelet_stride, d_obs, misfit, J, grad, illum, hmax,
                        rcv_model, offset_diag, stream=None):
    g, G = make_grid(grid), _geo(geom)
    return _check(load().fwi_gradient_static(ctypes.byref(g), ctypes.byref(G.struct), _ex(exec_), _ptr(v),
                                             _ptr(wavelet), int(wavelet_stride), _ptr(d_obs), _MISFIT[misfit],
                                             _ptr(J), _ptr(grad), _ptr(illum), int(hmax), _RCV[rcv_model],
                                             _ptr(offset_diag), _stream(stream)))


def fwi_extended_image(grid, geom, exec_, v, wavelet, wavelet_stride, d_obs, misfit, J, grad, hmax, image,
                       workspace, ws_bytes, stream=None):
    g, G = make_grid(grid), _geo(geom)
    return _check(load().fwi_extended_image(ctypes.byref(g), ctypes.byref(G.struct), _ex(exec_), _ptr(v),
                                            _ptr(wavelet), int(wavelet_stride), _ptr(d_obs), _MISFIT[misfit],
                                            _ptr(J), _ptr(grad), int(hmax), _ptr(image), _ptr(workspace),
                                            int(ws_bytes), _stream(stream)))


def fwi_misfit_value(grid, geom, exec_, v, wavelet, wavelet_stride, d_obs, misfit, J, workspace, ws_bytes,
                     stream=None):
    g, G = make_grid(grid), _geo(geom)
    return _check(load().fwi_misfit_value(ctypes.byref(g), ctypes.byref(G.struct), _ex(exec_), _ptr(v),
                                          _ptr(wavelet), int(wavelet_stride), _ptr(d_obs), _MISFIT[misfit], _ptr(J),
                                          _ptr(workspace), int(ws_bytes), _stream(stream)))


def fwi_born(grid, geom, exec_, v, wavelet, wavelet_stride, dv, data, workspace, ws_bytes, stream=None):
    g, G = make_grid(grid), _geo(geom)
    return _check(load().fwi_born(ctypes.byref(g), ctypes.byref(G.struct), _ex(exec_), _ptr(v), _ptr(wavelet),
                                  int(wavelet_stride), _ptr(dv), _ptr(data), _ptr(workspace), int(ws_bytes),
                                  _stream(stream)))


def fwi_gn_hvp(grid, geom, exec_, v, wavelet, wavelet_stride, dv, misfit, J, hv, workspace, ws_bytes, stream=None):
    g, G = make_grid(grid), _geo(geom)
    return _check(load().fwi_gn_hvp(ctypes.byref(g), ctypes.byref(G.struct), _ex(exec_), _ptr(v), _ptr(wavelet),
                                    int(wavelet_stride), _ptr(dv), _MISFIT[misfit], _ptr(J), _ptr(hv),
                                    _ptr(workspace), int(ws_bytes), _stream(stream)))


def fwi_hessian_diag(grid, geom, exec_, v, wavelet, wavelet_stride, kind, hmax, rcv_model, diag, workspace,
                     ws_bytes, stream=None):
    g, G = make_grid(grid), _geo(geom)
    return _check(load().fwi_hessian_diag(ctypes.byref(g), ctypes.byref(G.struct), _ex(exec_), _ptr(v),
                                          _ptr(wavelet), int(wavelet_stride), int(kind), int(hmax),
                                          _RCV[rcv_model], _ptr(diag), _ptr(workspace), int(ws_bytes),
                                          _stream(stream)))


def fwi_misfit_forward(grid, geom, exec_, v, wavelet, wavelet_stride, d_obs, misfit, J, workspace, ws_bytes,
                       stream=None):
    g, G = make_grid(grid), _geo(geom)
    return _check(load().fwi_misfit_forward(ctypes.byref(g), ctypes.byref(G.struct), _ex(exec_), _ptr(v),
                                            _ptr(wavelet), int(wavelet_stride), _ptr(d_obs), _MISFIT[misfit],
                                            _ptr(J), _ptr(workspace), int(ws_bytes), _stream(stream)))


def fwi_misfit_backward(grid, geom, exec_, v, wavelet, wavelet_stride, grad_scale, grad, illum, hmax, rcv_model,
                        offset_diag, workspace, ws_bytes, stream=None):
    g, G = make_grid(grid), _geo(geom)
    return _check(load().fwi_misfit_backward(ctypes.byref(g), ctypes.byref(G.struct), _ex(exec_), _ptr(v),
                                             _ptr(wavelet), int(wavelet_stride), _ptr(grad_scale), _ptr(grad),
                                             _ptr(illum), int(hmax), _RCV[rcv_model], _ptr(offset_diag),
                                             _ptr(workspace), int(ws_bytes), _stream(stream)))


def fwi_offset_diag_exact_workspace_bytes(grid, geom, exec_, hmax, fmax, dft=DFT_FP32) -> int:
    g, G = make_grid(grid), _geo(geom)
    return int(load().fwi_offset_diag_exact_workspace_bytes(ctypes.byref(g), ctypes.byref(G.struct), _ex(exec_),
                                                            int(hmax), float(fmax), int(dft)))


def fwi_offset_diag_exact(grid, geom, exec_, v, wavelet, wavelet_stride, hmax, fmax, dft, diag, workspace,
                          ws_bytes, stream=None):
    g, G = make_grid(grid), _geo(geom)
    return _check(load().fwi_offset_diag_exact(ctypes.byref(g), ctypes.byref(G.struct), _ex(exec_), _ptr(v),
                                               _ptr(wavelet), int(wavelet_stride), int(hmax), float(fmax),
                                               int(dft), _ptr(diag), _ptr(workspace), int(ws_bytes),
                                               _stream(stream)))


def fwi_precondition(grid, v, grad, kind, hdiag, hmax, eps, out, workspace, ws_bytes, stream=None):
    g = make_grid(grid)
    return _check(load().fwi_precondition(ctypes.byref(g), _ptr(v), _ptr(grad), int(kind), _ptr(hdiag),
                                          int(hmax), float(eps), _ptr(out), _ptr(workspace), int(ws_bytes),
                                          _stream(stream)))


def fwi_tune_reset() -> None:
    load().fwi_tune_reset()


def fwi_status(workspace, stream=None) -> int:
    return int(load().fwi_status(_ptr(workspace), _stream(stream)))


# ------------------------------------------------------------------ helpers
def _torch():
    import torch
    return torch


def workspace(grid, geom, what, exec_=None, hmax=0, device="cuda"):
    torch = _torch()
    n = fwi_workspace_bytes(grid, geom, exec_, what, hmax)
    if n == 0:
        raise FwiError(FWI_ERR_ARG, last_error())
    return torch.empty(n, dtype=torch.uint8, device=device)


def _dev(x, dtype=None, device="cuda"):
    torch = _torch()
    if isinstance(x, torch.Tensor):
        t = x.to(device=device)
    else:
        t = torch.as_tensor(np.asarray(x), device=device)
    if dtype is not None:
        t = t.to(dtype)
    return t.contiguous()


def _wavelet(wavelet, nt_max, device):
    torch = _torch()
    w = _dev(wavelet, torch.float32, device)
    if w.dim() == 1:
        if w.shape[0] < nt_max:
            w = torch.nn.functional.pad(w, (0, nt_max - w.shape[0]))
        return w, 0
    return w, w.stride(0)


def forward(v, wavelet, grid, geom, exec_=None, ws=None, device="cuda"):
    """Traces [ntrace][nt_max] (torch float32 on the device)."""
    torch = _torch()
    G = _geo(geom)
    vd = _dev(v, torch.float32, device)
    w, ws_ = _wavelet(wavelet, grid.nt_max, device)
    data = torch.empty((max(geom.ntrace, 1), grid.nt_max), dtype=torch.float32, device=device)
    ws = workspace(grid, G, WS_FORWARD, exec_, device=device) if ws is None else ws
    fwi_forward(grid, G, exec_, vd, w, ws_, data, ws, ws.numel())
    return data[:geom.ntrace]


def gradient(v, wavelet, grid, geom, d_obs, misfit="int", exec_=None, illum=True, hmax=None, rcv_model="pm",
             ws=None, device="cuda"):
    """(J, grad, H1 or None, D or None) as torch tensors on the device."""
    torch = _torch()
    G = _geo(geom)
    vd = _dev(v, torch.float32, device)
    w, ws_ = _wavelet(wavelet, grid.nt_max, device)
    dobs = _dev(d_obs, torch.float32, device)
    J = torch.empty((), dtype=torch.float64, device=device)
    grad = torch.empty((grid.nz, grid.nx), dtype=torch.float32, device=device)
    H1 = torch.empty_like(grad) if illum else None
    D = None
    if hmax is not None:
        D = torch.empty((2 * hmax + 1, grid.nz, grid.nx), dtype=torch.float32, device=device)
    ws = workspace(grid, G, WS_GRADIENT, exec_, hmax or 0, device=device) if ws is None else ws
    fwi_gradient(grid, G, exec_, vd, w, ws_, dobs, misfit, J, grad, H1, hmax or 0, rcv_model, D, ws, ws.numel())
    return J, grad, H1, D


def extended_image(v, wavelet, grid, geom, d_obs, hmax, misfit="int", exec_=None, ws=None, device="cuda"):
    """(J, grad, image[2 hmax + 1][nz][nx]) as torch tensors on the device."""
    torch = _torch()
    G = _geo(geom)
    vd = _dev(v, torch.float32, device)
    w, ws_ = _wavelet(wavelet, grid.nt_max, device)
    dobs = _dev(d_obs, torch.float32, device)
    J = torch.empty((), dtype=torch.float64, device=device)
    grad = torch.empty((grid.nz, grid.nx), dtype=torch.float32, device=device)
    image = torch.empty((2 * hmax + 1, grid.nz, grid.nx), dtype=torch.float32, device=device)
    ws = workspace(grid, G, WS_EXTIMAGE, exec_, hmax, device=device) if ws is None else ws
    fwi_extended_image(grid, G, exec_, vd, w, ws_, dobs, misfit, J, grad, hmax, image, ws, ws.numel())
    return J, grad, image


def misfit_value(v, wavelet, grid, geom, d_obs, misfit="int", exec_=None, ws=None, device="cuda"):
    """J(v) (torch float64 scalar on the device)."""
    torch = _torch()
    G = _geo(geom)
    vd = _dev(v, torch.float32, device)
    w, ws_ = _wavelet(wavelet, grid.nt_max, device)
    dobs = _dev(d_obs, torch.float32, device)
    J = torch.empty((), dtype=torch.float64, device=device)
    ws = workspace(grid, G, WS_FORWARD, exec_, device=device) if ws is None else ws
    fwi_misfit_value(grid, G, exec_, vd, w, ws_, dobs, misfit, J, ws, ws.numel())
    return J


def born(v, wavelet, grid, geom, dv, exec_=None, ws=None, device="cuda"):
    """Born data J dv [ntrace][nt_max] (torch float32 on the device)."""
    torch = _torch()
    G = _geo(geom)
    vd = _dev(v, torch.float32, device)
    dvd = _dev(dv, torch.float32, device)
    w, ws_ = _wavelet(wavelet, grid.nt_max, device)
    data = torch.empty((max(geom.ntrace, 1), grid.nt_max), dtype=torch.float32, device=device)
    ws = workspace(grid, G, WS_BORN, exec_, device=device) if ws is None else ws
    fwi_born(grid, G, exec_, vd, w, ws_, dvd, data, ws, ws.numel())
    return data[:geom.ntrace]


def gn_hvp(v, wavelet, grid, geom, dv, misfit="int", exec_=None, ws=None, device="cuda"):
    """(1/2 |W J dv|^2, J^T W^T W J dv) as torch tensors on the device."""
    torch = _torch()
    G = _geo(geom)
    vd = _dev(v, torch.float32, device)
    dvd = _dev(dv, torch.float32, device)
    w, ws_ = _wavelet(wavelet, grid.nt_max, device)
    J = torch.empty((), dtype=torch.float64, device=device)
    hv = torch.empty((grid.nz, grid.nx), dtype=torch.float32, device=device)
    ws = workspace(grid, G, WS_GNHVP, exec_, device=device) if ws is None else ws
    fwi_gn_hvp(grid, G, exec_, vd, w, ws_, dvd, misfit, J, hv, ws, ws.numel())
    return J, hv


def hessian_diag(v, wavelet, grid, geom, kind=HESS_EQ1, hmax=0, rcv_model="pm", exec_=None, ws=None,
                 device="cuda"):
    torch = _torch()
    G = _geo(geom)
    vd = _dev(v, torch.float32, device)
    w, ws_ = _wavelet(wavelet, grid.nt_max, device)
    shape = (grid.nz, grid.nx) if kind == HESS_EQ1 else (2 * hmax + 1, grid.nz, grid.nx)
    out = torch.empty(shape, dtype=torch.float32, device=device)
    ws = workspace(grid, G, WS_HESSIAN, exec_, hmax, device=device) if ws is None else ws
    fwi_hessian_diag(grid, G, exec_, vd, w, ws_, kind, hmax, rcv_model, out, ws, ws.numel())
    return out


def offset_diag_exact(v, wavelet, grid, geom, hmax, fmax=0.0, exec_=None, ws=None, device="cuda", dft=None):
    """Offset diagonal with the exact receiver term, D[2 hmax + 1][nz][nx]
    (fmax in Hz bounds the frequency band, 0 keeps every bin; dft selects
    the arithmetic of the spectra on the matrix cores, DFT_BF16X3 by default)."""
    dft = DFT_BF16X3 if dft is None else dft
    torch = _torch()
    G = _geo(geom)
    vd = _dev(v, torch.float32, device)
    w, ws_ = _wavelet(wavelet, grid.nt_max, device)
    out = torch.empty((2 * hmax + 1, grid.nz, grid.nx), dtype=torch.float32, device=device)
    if ws is None:
        n = fwi_offset_diag_exact_workspace_bytes(grid, G, exec_, hmax, fmax, dft)
        if n == 0:
            raise FwiError(FWI_ERR_ARG, last_error())
        ws = torch.empty(n, dtype=torch.uint8, device=device)
    fwi_offset_diag_exact(grid, G, exec_, vd, w, ws_, hmax, fmax, dft, out, ws, ws.numel())
    return out


def precondition(v, grad, hdiag, grid, kind=PRECOND_SHOT, hmax=0, eps=1e-2, device="cuda"):
    torch = _torch()
    out = torch.empty_like(grad)
    ws = torch.empty(256, dtype=torch.uint8, device=device)
    fwi_precondition(grid, v, grad, kind, hdiag, hmax, eps, out, ws, ws.numel())
    return out
