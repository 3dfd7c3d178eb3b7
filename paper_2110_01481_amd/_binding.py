"""ctypes binding of libabgmres (include/abgmres.h): argument marshalling only.

Torch tensors supply device memory and the current HIP stream; every computation runs
in the library's kernels. The module fails loudly when the library is missing.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libabgmres.so")

F64, F32, BF16 = 0, 1, 2
BP_HAT, BP_ADJ, BP_STRIP_T, BP_JOSEPH_T, BP_STRIP_TAU = 0, 1, 2, 3, 4
# back projectors by name: the unmatched interpolating B, the transposes of the line,
# strip and interpolation (Joseph) models, and the thresholded strip transpose B_tau
BP_KINDS = {"hat": BP_HAT, "adj": BP_ADJ, "strip_t": BP_STRIP_T, "joseph_t": BP_JOSEPH_T,
            "strip_tau": BP_STRIP_TAU}
# forward projector models (Sec. 6.1)
FP_MODELS = {"line": 0, "strip": 1, "joseph": 2}
STOP_NONE, STOP_DP, STOP_NCP = 0, 1, 2
METHOD_AB, METHOD_BA, METHOD_LSQR, METHOD_LSMR = 0, 1, 2, 3

STATUS = {0: "ok", -1: "einval", -2: "enomem", -3: "ehip", -4: "enan", -5: "edevice",
          -6: "efull", 1: "not_converged", 2: "breakdown", 3: "zero_rhs"}
EXPORTS = ["abg_create_geometry", "abg_destroy_geometry", "abg_geometry_sizes",
           "abg_fp_workspace_bytes", "abg_fp_apply", "abg_bp_apply", "abg_workspace_bytes",
           "abg_ab_gmres", "abg_ba_gmres", "abg_status_string", "abg_profile_enable",
           "abg_profile_read", "abg_request_bytes", "abg_engine_create", "abg_engine_destroy",
           "abg_engine_submit", "abg_engine_step", "abg_engine_poll", "abg_engine_set_tiles",
           "abg_engine_get_tiles", "abg_engine_autotune", "abg_batch_solve",
           "abg_mgs_force_stream", "abg_geometry_set_model", "abg_geometry_get_model",
           "abg_geometry_set_strip_threshold", "abg_lsq_workspace_bytes", "abg_lsqr", "abg_lsmr",
           "abg_gmres_error_history", "abg_release_process_resources", "abg_fp_apply_noalloc",
           "abg_ncp_force_goertzel", "abg_fp_force_block_shape", "abg_fp_force_stage_share"]


class AbgError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)}")


class Stop(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("tau", ctypes.c_double), ("noise_norm", ctypes.c_double)]


class Precision(ctypes.Structure):
    _fields_ = [("proj", ctypes.c_int), ("basis", ctypes.c_int)]


_dp = ctypes.POINTER(ctypes.c_double)


class Info(ctypes.Structure):
    _fields_ = [("k_stop", ctypes.c_int), ("k_done", ctypes.c_int), ("status", ctypes.c_int),
                ("n_literal", ctypes.c_int), ("res_norm", ctypes.c_double),
                ("ncp_dist", ctypes.c_double), ("beta", ctypes.c_double),
                ("res_hist", _dp), ("ls_hist", _dp), ("ncp_hist", _dp),
                ("hist_len", ctypes.c_int), ("H", _dp)]


class Request(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("method", ctypes.c_int), ("bp_kind", ctypes.c_int),
                ("k_max", ctypes.c_int), ("stop", Stop), ("b", ctypes.c_void_p),
                ("x0", ctypes.c_void_p), ("x", ctypes.c_void_p), ("ws", ctypes.c_void_p),
                ("ws_bytes", ctypes.c_size_t), ("info", ctypes.POINTER(Info)),
                ("tag", ctypes.c_longlong)]


_lib = None
# geometries and engines alive in this process: shutdown() releases them in order
_live: "weakref.WeakSet" = weakref.WeakSet()
_shut = False
# Objects collected during interpreter shutdown (when the HIP runtime may already be gone)
# leave their memory to the process exit instead of calling into the library: __del__
# binds sys.is_finalizing as a default argument, since module globals may be cleared by then.


def shutdown():
    """Releases every live engine and geometry, then the library's process-wide resources
    (abg_release_process_resources), while the HIP runtime is still up. Registered with
    atexit when the library is loaded; bench.py and the test session also call it at
    their end. Objects released here are closed; the library stays usable."""
    global _shut
    if _lib is None:
        return
    for o in sorted(list(_live), key=lambda o: 0 if isinstance(o, Engine) else 1):
        o.close()
    _lib.abg_release_process_resources()
    _shut = True


def load_library(path: str | None = None):
    """Loads libabgmres.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with __graft_entry__.build() "
                          "or python -m paper_2110_01481_amd.build")
    lib = ctypes.CDLL(p)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    lib.abg_create_geometry.argtypes = [i, i, d, d, _dp, i, d, ctypes.POINTER(vp)]
    lib.abg_destroy_geometry.argtypes = [vp]
    lib.abg_geometry_sizes.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]
    lib.abg_fp_workspace_bytes.argtypes = [vp, i]
    lib.abg_fp_workspace_bytes.restype = sz
    lib.abg_fp_apply.argtypes = [vp, i, vp, vp, vp, sz, vp]
    lib.abg_bp_apply.argtypes = [vp, i, i, vp, vp, vp]
    lib.abg_fp_apply_noalloc.argtypes = [vp, i, vp, vp, vp]
    lib.abg_workspace_bytes.argtypes = [vp, i, i, Precision, Stop]
    lib.abg_workspace_bytes.restype = sz
    for name in ("abg_ab_gmres", "abg_ba_gmres"):
        getattr(lib, name).argtypes = [vp, i, vp, vp, vp, i, Stop, Precision, vp, sz,
                                       ctypes.POINTER(Info), vp]
    lib.abg_status_string.argtypes = [i]
    lib.abg_status_string.restype = ctypes.c_char_p
    lib.abg_profile_enable.argtypes = [i]
    lib.abg_profile_read.argtypes = [ctypes.POINTER(ctypes.c_longlong), _dp, i]
    lib.abg_request_bytes.argtypes = [vp, i, i, Precision, Stop]
    lib.abg_request_bytes.restype = sz
    lib.abg_engine_create.argtypes = [Precision, i, vp, ctypes.POINTER(vp)]
    lib.abg_engine_destroy.argtypes = [vp]
    lib.abg_engine_submit.argtypes = [vp, ctypes.POINTER(Request)]
    lib.abg_engine_step.argtypes = [vp, ctypes.POINTER(i)]
    lib.abg_engine_poll.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(i), i,
                                    ctypes.POINTER(i)]
    lib.abg_engine_set_tiles.argtypes = [vp, i, i, i]
    lib.abg_engine_get_tiles.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]
    lib.abg_engine_autotune.argtypes = [vp, i, ctypes.POINTER(i), ctypes.POINTER(i),
                                        ctypes.POINTER(i), _dp]
    lib.abg_batch_solve.argtypes = [ctypes.POINTER(Request), i, Precision, i, i, i, vp]
    lib.abg_mgs_force_stream.argtypes = [i]
    lib.abg_ncp_force_goertzel.argtypes = [i]
    lib.abg_fp_force_block_shape.argtypes = [i]
    lib.abg_fp_force_stage_share.argtypes = [i]
    lib.abg_geometry_set_model.argtypes = [vp, i]
    lib.abg_geometry_get_model.argtypes = [vp, ctypes.POINTER(i)]
    lib.abg_geometry_set_strip_threshold.argtypes = [vp, ctypes.c_double, _dp]
    lib.abg_lsq_workspace_bytes.restype = ctypes.c_size_t
    lib.abg_lsq_workspace_bytes.argtypes = [vp, i, i]
    for name in ("abg_lsqr", "abg_lsmr"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, vp, vp, i, Stop, i, vp, ctypes.c_size_t, ctypes.POINTER(Info), vp,
                      _dp, vp]
    lib.abg_gmres_error_history.argtypes = [vp, i, i, i, Stop, Precision, vp, vp, vp, sz, i, _dp,
                                            vp]
    lib.abg_release_process_resources.argtypes = []
    _lib = lib
    atexit.register(shutdown)
    return lib


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t == torch.float64:
        return F64
    if t == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t}")


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_empty(nbytes: int, device):
    torch = _torch()
    # 256-byte alignment: torch's caching allocator returns 512-byte aligned blocks
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


def _check(rc: int, where: str, ok=(0,)):
    if rc not in ok:
        raise AbgError(rc, where)
    return rc


class Geometry:
    """2-D parallel-beam geometry owned by the library (abg_create_geometry)."""

    def __init__(self, N: int, n_ang: int, n_det: int, ang_range: float = 180.0,
                 ang_start: float = 0.0, angles_deg=None, det_spacing: float = 1.0,
                 model: str = "line"):
        lib = load_library()
        h = ctypes.c_void_p()
        arr = None
        if angles_deg is not None:
            arr = np.ascontiguousarray(angles_deg, dtype=np.float64)
            n_ang = arr.size
        ptr = arr.ctypes.data_as(_dp) if arr is not None else None
        _check(lib.abg_create_geometry(int(N), int(n_ang), float(ang_start), float(ang_range), ptr,
                                       int(n_det), float(det_spacing), ctypes.byref(h)),
               "abg_create_geometry")
        self._h = h
        _live.add(self)
        self.N, self.n_ang, self.n_det = int(N), int(n_ang), int(n_det)
        self.n = self.N * self.N
        self.m = self.n_ang * self.n_det
        self._fp_ws = {}
        self.model = "line"
        if model != "line":
            self.set_model(model)

    def set_strip_threshold(self, tau: float) -> float:
        """Threshold tau of the "strip_tau" back projector B_tau (Sec. 6.5); returns the
        largest strip-model entry (abg_geometry_set_strip_threshold)."""
        mx = ctypes.c_double()
        _check(load_library().abg_geometry_set_strip_threshold(self._h, float(tau), ctypes.byref(mx)),
               "abg_geometry_set_strip_threshold")
        return mx.value

    def set_model(self, model: str):
        """Forward projector model: "line", "strip" or "joseph" (abg_geometry_set_model)."""
        _check(load_library().abg_geometry_set_model(self._h, FP_MODELS[model]),
               "abg_geometry_set_model")
        self.model = model

    def close(self):
        if getattr(self, "_h", None):
            self._fp_ws.clear()
            load_library().abg_destroy_geometry(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def release_workspace(self):
        """Drops the cached forward-projector scratch of fp()."""
        self._fp_ws.clear()

    def fp_workspace(self, dtype_code: int, device):
        key = (dtype_code, str(device))
        ws = self._fp_ws.get(key)
        if ws is None:
            nb = load_library().abg_fp_workspace_bytes(self._h, dtype_code)
            ws = _dev_empty(nb, device)
            self._fp_ws[key] = ws
        return ws

    def fp(self, x, out=None, stream=None):
        """y = A x (the geometry's model) for a contiguous CUDA tensor x of n elements."""
        torch = _torch()
        assert x.is_cuda and x.is_contiguous() and x.numel() == self.n
        t = _dtype_code(x.dtype)
        y = out if out is not None else torch.empty(self.m, dtype=x.dtype, device=x.device)
        ws = self.fp_workspace(t, x.device)
        _check(load_library().abg_fp_apply(self._h, t, ctypes.c_void_p(x.data_ptr()),
                                           ctypes.c_void_p(y.data_ptr()),
                                           ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                           _stream_ptr(stream)), "abg_fp_apply")
        return y

    def fp_noalloc(self, x, out, stream=None):
        """y = A x through abg_fp_apply_noalloc (the library's static device scratch; no
        allocation by the library): x and the output `out` are caller-owned CUDA tensors."""
        assert x.is_cuda and x.is_contiguous() and x.numel() == self.n
        assert out.is_cuda and out.is_contiguous() and out.numel() == self.m and out.dtype == x.dtype
        _check(load_library().abg_fp_apply_noalloc(self._h, _dtype_code(x.dtype),
                                                   ctypes.c_void_p(x.data_ptr()),
                                                   ctypes.c_void_p(out.data_ptr()),
                                                   _stream_ptr(stream)), "abg_fp_apply_noalloc")
        return out

    def bp(self, y, kind: str = "hat", out=None, stream=None):
        """x = B y (kind "hat", unmatched), A_line^T y ("adj"), A_strip^T y ("strip_t"),
        A_Joseph^T y ("joseph_t") or B_tau y ("strip_tau", set_strip_threshold)."""
        torch = _torch()
        assert y.is_cuda and y.is_contiguous() and y.numel() == self.m
        t = _dtype_code(y.dtype)
        x = out if out is not None else torch.empty(self.n, dtype=y.dtype, device=y.device)
        _check(load_library().abg_bp_apply(self._h, BP_KINDS[kind], t,
                                           ctypes.c_void_p(y.data_ptr()),
                                           ctypes.c_void_p(x.data_ptr()), _stream_ptr(stream)),
               "abg_bp_apply")
        return x


@dataclass
class SolveResult:
    x: object
    status: str
    k_stop: int
    k_done: int
    res_norm: float
    ncp_dist: float
    beta: float
    n_literal: int
    res_hist: np.ndarray
    ls_hist: np.ndarray
    ncp_hist: np.ndarray
    H: np.ndarray | None = None
    extra: dict = field(default_factory=dict)
    err_hist: np.ndarray | None = None   # ||x_k - x_ref|| per k (runs given x_ref)


_DTYPES = {"f64": F64, "f32": F32, "bf16": BF16}


def workspace_bytes(g: Geometry, method: str, k_max: int, proj="f32", basis="f32",
                    stop="none") -> int:
    st = Stop({"none": STOP_NONE, "dp": STOP_DP, "ncp": STOP_NCP}[stop], 1.0, 1.0)
    return int(load_library().abg_workspace_bytes(g.handle, METHOD_AB if method == "ab" else METHOD_BA,
                                                  int(k_max), Precision(_DTYPES[proj], _DTYPES[basis]), st))


def gmres(method: str, g: Geometry, b, k_max: int, stop: str = "none", tau: float = 1.0,
          noise_norm: float = 0.0, bp: str = "hat", basis: str | None = None, x0=None,
          out=None, workspace=None, want_H: bool = False, x_ref=None,
          stream=None) -> SolveResult:
    """AB-GMRES (method "ab") or BA-GMRES ("ba") through the C ABI.

    b: CUDA tensor of m elements (float64 or float32: the projector dtype);
    basis: "f64", "f32" or "bf16" storage of the Krylov basis (default: b's dtype);
    bp: back projector "hat", "adj", "strip_t", "joseph_t" or "strip_tau" (A is the
    geometry's model);
    x_ref: optional CUDA tensor of n elements (b's dtype): the result's err_hist then holds
    ||x_k - x_ref|| for k = 1..k_done (abg_gmres_error_history on the solve's workspace).
    """
    torch = _torch()
    lib = load_library()
    assert b.is_cuda and b.is_contiguous() and b.numel() == g.m
    proj = _dtype_code(b.dtype)
    bas = proj if basis is None else _DTYPES[basis]
    st = Stop({"none": STOP_NONE, "dp": STOP_DP, "ncp": STOP_NCP}[stop], float(tau), float(noise_norm))
    prec = Precision(proj, bas)
    meth = METHOD_AB if method == "ab" else METHOD_BA
    nb = lib.abg_workspace_bytes(g.handle, meth, int(k_max), prec, st)
    if nb == 0:
        raise AbgError(-1, "abg_workspace_bytes")
    ws = workspace if workspace is not None else _dev_empty(nb, b.device)
    x = out if out is not None else torch.empty(g.n, dtype=b.dtype, device=b.device)
    res = np.zeros(k_max)
    ls = np.zeros(k_max)
    ncp = np.zeros(k_max)
    H = np.zeros((k_max, k_max + 1)) if want_H else None
    info = Info()
    info.res_hist = res.ctypes.data_as(_dp)
    info.ls_hist = ls.ctypes.data_as(_dp)
    info.ncp_hist = ncp.ctypes.data_as(_dp)
    info.hist_len = k_max
    info.H = H.ctypes.data_as(_dp) if H is not None else None
    fn = lib.abg_ab_gmres if meth == METHOD_AB else lib.abg_ba_gmres
    x0p = ctypes.c_void_p(x0.data_ptr()) if x0 is not None else None
    rc = fn(g.handle, BP_KINDS[bp], ctypes.c_void_p(b.data_ptr()), x0p,
            ctypes.c_void_p(x.data_ptr()), int(k_max), st, prec, ctypes.c_void_p(ws.data_ptr()),
            ws.numel(), ctypes.byref(info), _stream_ptr(stream))
    _check(rc, "abg_%s_gmres" % method, ok=(0, 1, 2, 3))
    kd = info.k_done
    err = None
    if x_ref is not None:
        assert x_ref.is_cuda and x_ref.dtype == b.dtype and x_ref.numel() == g.n
        x_ref = x_ref.contiguous()
        err = np.zeros(max(kd, 1))
        rc2 = lib.abg_gmres_error_history(g.handle, meth, BP_KINDS[bp], int(k_max), st, prec,
                                          x0p, ctypes.c_void_p(x_ref.data_ptr()),
                                          ctypes.c_void_p(ws.data_ptr()), ws.numel(), kd,
                                          err.ctypes.data_as(_dp), _stream_ptr(stream))
        _check(rc2, "abg_gmres_error_history")
        err = err[:kd].copy()
    Hm = None
    if H is not None:
        Hm = H.T[:kd + 1, :kd].copy()   # column-major (k_max+1) x k_max in memory
    return SolveResult(x=x, status=STATUS[rc], k_stop=info.k_stop, k_done=kd,
                       res_norm=info.res_norm, ncp_dist=info.ncp_dist, beta=info.beta,
                       n_literal=info.n_literal, res_hist=res[:kd].copy(),
                       ls_hist=ls[:kd].copy(), ncp_hist=ncp[:kd].copy(), H=Hm, err_hist=err)


def lsq_workspace_bytes(g: Geometry, method: str, dtype="f64") -> int:
    """Workspace bytes of LSQR ("lsqr") or LSMR ("lsmr") (abg_lsq_workspace_bytes)."""
    meth = METHOD_LSQR if method == "lsqr" else METHOD_LSMR
    return int(load_library().abg_lsq_workspace_bytes(g.handle, meth, _DTYPES[dtype]))


def lsq(method: str, g: Geometry, b, k_max: int, stop: str = "none", tau: float = 1.0,
        noise_norm: float = 0.0, x0=None, out=None, workspace=None, x_ref=None,
        stream=None) -> SolveResult:
    """LSQR (method "lsqr") or LSMR ("lsmr") with the geometry's model A and its exact
    transpose, through the C ABI (abg_lsqr / abg_lsmr). b: CUDA tensor of m elements
    (float64 or float32); x_ref: optional CUDA tensor of n elements (b's dtype): the
    result's err_hist then holds ||x_k - x_ref|| per step."""
    torch = _torch()
    lib = load_library()
    assert b.is_cuda and b.is_contiguous() and b.numel() == g.m
    t = _dtype_code(b.dtype)
    meth = METHOD_LSQR if method == "lsqr" else METHOD_LSMR
    st = Stop({"none": STOP_NONE, "dp": STOP_DP, "ncp": STOP_NCP}[stop], float(tau),
              float(noise_norm))
    nb = lib.abg_lsq_workspace_bytes(g.handle, meth, t)
    if nb == 0:
        raise AbgError(-1, "abg_lsq_workspace_bytes")
    ws = workspace if workspace is not None else _dev_empty(nb, b.device)
    x = out if out is not None else torch.empty(g.n, dtype=b.dtype, device=b.device)
    res = np.zeros(k_max)
    ls = np.zeros(k_max)
    ncp = np.zeros(k_max)
    info = Info()
    info.res_hist = res.ctypes.data_as(_dp)
    info.ls_hist = ls.ctypes.data_as(_dp)
    info.ncp_hist = ncp.ctypes.data_as(_dp)
    info.hist_len = k_max
    info.H = None
    fn = lib.abg_lsqr if meth == METHOD_LSQR else lib.abg_lsmr
    x0p = ctypes.c_void_p(x0.data_ptr()) if x0 is not None else None
    err = None
    xr = None
    if x_ref is not None:
        assert x_ref.is_cuda and x_ref.dtype == b.dtype and x_ref.numel() == g.n
        x_ref = x_ref.contiguous()
        xr = ctypes.c_void_p(x_ref.data_ptr())
        err = np.zeros(k_max)
    rc = fn(g.handle, ctypes.c_void_p(b.data_ptr()), x0p, ctypes.c_void_p(x.data_ptr()), int(k_max),
            st, t, ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(info), xr,
            err.ctypes.data_as(_dp) if err is not None else None, _stream_ptr(stream))
    _check(rc, "abg_" + method, ok=(0, 1, 2, 3))
    kd = info.k_done
    return SolveResult(x=x, status=STATUS[rc], k_stop=info.k_stop, k_done=kd,
                       res_norm=info.res_norm, ncp_dist=info.ncp_dist, beta=info.beta,
                       n_literal=info.n_literal, res_hist=res[:kd].copy(), ls_hist=ls[:kd].copy(),
                       ncp_hist=ncp[:kd].copy() if stop == "ncp" else np.zeros(0), H=None,
                       err_hist=err[:kd].copy() if err is not None else None)


def ab_gmres(g, b, k_max, **kw) -> SolveResult:
    return gmres("ab", g, b, k_max, **kw)


def ba_gmres(g, b, k_max, **kw) -> SolveResult:
    return gmres("ba", g, b, k_max, **kw)


def mgs_force_stream(on: bool = True):
    """Single solves of vectors longer than 2^21 elements always use the streaming
    Gram-Schmidt variant (abg_mgs_force_stream)."""
    load_library().abg_mgs_force_stream(1 if on else 0)


def ncp_force_goertzel(on: bool = True):
    """NCP periodograms by Goertzel's recurrence for every row length (abg_ncp_force_goertzel)."""
    load_library().abg_ncp_force_goertzel(1 if on else 0)


def fp_force_stage_share(eighths: int = -1):
    """Eighths (0..8) of the four-angle forward blocks that stage their band rows in LDS;
    -1 restores the automatic share (abg_fp_force_stage_share). Results are bit-identical
    for every share."""
    _check(load_library().abg_fp_force_stage_share(int(eighths)), "abg_fp_force_stage_share")


def fp_force_block_shape(lg_angles: int = -1):
    """Forward projector blocks of 2^lg_angles angles (0..2); -1 restores the automatic
    choice (abg_fp_force_block_shape). Results are bit-identical for every shape."""
    _check(load_library().abg_fp_force_block_shape(int(lg_angles)), "abg_fp_force_block_shape")


# the launch classes abg_profile_read reports, in its order (ABG_PROF_KINDS of them)
PROF_KINDS = ["forward", "back", "mgs", "combine", "ncp"]


def profile_enable(on: bool = True):
    load_library().abg_profile_enable(1 if on else 0)


def profile_read(reset: bool = True):
    counts = (ctypes.c_longlong * len(PROF_KINDS))()
    ms = (ctypes.c_double * len(PROF_KINDS))()
    load_library().abg_profile_read(counts, ms, 1 if reset else 0)
    names = PROF_KINDS
    return {nm: (int(counts[i]), float(ms[i])) for i, nm in enumerate(names)}


# ---- batched engine -----------------------------------------------------------------------

def request_bytes(g: Geometry, method: str, k_max: int, proj="f32", basis="f32",
                  stop="dp") -> int:
    """Device bytes one engine request needs (basis, Hessenberg state, scratch)."""
    st = Stop({"none": STOP_NONE, "dp": STOP_DP}[stop], 1.0, 1.0)
    return int(load_library().abg_request_bytes(g.handle, METHOD_AB if method == "ab" else METHOD_BA,
                                                int(k_max), Precision(_DTYPES[proj], _DTYPES[basis]), st))


@dataclass
class Problem:
    """One solve for the batched engine. b: CUDA tensor of m elements (engine's proj dtype)."""
    g: Geometry
    method: str
    b: object
    k_max: int
    stop: str = "dp"
    tau: float = 1.0
    noise_norm: float = 0.0
    bp: str = "hat"
    x0: object = None
    tag: int = 0


class _Pending:
    def __init__(self, prob: Problem, x, ws, k_max: int):
        self.prob = prob
        self.x = x
        self.ws = ws
        self.res = np.zeros(k_max)
        self.ls = np.zeros(k_max)
        self.info = Info()
        self.info.res_hist = self.res.ctypes.data_as(_dp)
        self.info.ls_hist = self.ls.ctypes.data_as(_dp)
        self.info.ncp_hist = None
        self.info.hist_len = k_max
        self.info.H = None

    def result(self, code: int) -> SolveResult:
        i = self.info
        kd = i.k_done
        return SolveResult(x=self.x, status=STATUS.get(code, str(code)), k_stop=i.k_stop,
                           k_done=kd, res_norm=i.res_norm, ncp_dist=0.0, beta=i.beta,
                           n_literal=i.n_literal, res_hist=self.res[:kd].copy(),
                           ls_hist=self.ls[:kd].copy(), ncp_hist=np.zeros(0),
                           extra={"tag": self.prob.tag})


class Engine:
    """Batched AB-/BA-GMRES engine (abg_engine_*): submit problems at any time, advance all
    of them one Arnoldi step per round, collect finished ones with poll()."""

    def __init__(self, proj="f32", basis="f32", max_slots=64, stream=None, device=None):
        torch = _torch()
        self.lib = load_library()
        self.proj, self.basis = proj, basis
        self.prec = Precision(_DTYPES[proj], _DTYPES[basis])
        self.device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream
        h = ctypes.c_void_p()
        _check(self.lib.abg_engine_create(self.prec, int(max_slots), _stream_ptr(stream),
                                          ctypes.byref(h)), "abg_engine_create")
        self._h = h
        _live.add(self)
        self.max_slots = int(max_slots)
        self._pending: dict[int, _Pending] = {}
        self._next_tag = 1

    def close(self):
        if getattr(self, "_h", None):
            self.lib.abg_engine_destroy(self._h)
            self._h = None
            self._pending.clear()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def set_tiles(self, rays: int, ang_block: int | None = None, sched: int | None = None):
        cur = self.get_tiles()
        ab = ang_block if ang_block is not None else cur[1]
        sc = sched if sched is not None else cur[2]
        _check(self.lib.abg_engine_set_tiles(self._h, int(rays), int(ab), int(sc)),
               "abg_engine_set_tiles")

    def get_tiles(self) -> tuple:
        r, a, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self.lib.abg_engine_get_tiles(self._h, ctypes.byref(r), ctypes.byref(a),
                                             ctypes.byref(c)), "abg_engine_get_tiles")
        return r.value, a.value, c.value

    def signature(self) -> str:
        """Key of the current mix for the tile cache: precision and the sorted shapes."""
        shapes = sorted((p.prob.g.N, p.prob.g.n_ang, p.prob.g.n_det, p.prob.method)
                        for p in self._pending.values())
        return f"{self.proj}/{self.basis}:" + ";".join("%d,%d,%d,%s" % s for s in shapes)

    def autotune(self, reps: int = 3, cache: str | None = None) -> dict:
        """Picks the projector tile shapes for the problems held now (call after submit,
        before the first step). With `cache` (a JSON file), a shape found before for the
        same device and mix is reused without timing."""
        import json
        torch = _torch()
        dev = torch.cuda.get_device_name(self.device)
        key = dev + "|" + self.signature()
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                table = json.load(fh)
        if key in table:
            e = table[key]
            self.set_tiles(e["rays"], e["ang_block"], e["sched"])
            return {"rays": e["rays"], "ang_block": e["ang_block"], "sched": e["sched"],
                    "ms": e["ms"], "cached": True}
        r, a, c, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(self.lib.abg_engine_autotune(self._h, int(reps), ctypes.byref(r), ctypes.byref(a),
                                            ctypes.byref(c), ctypes.byref(ms)),
               "abg_engine_autotune")
        out = {"rays": r.value, "ang_block": a.value, "sched": c.value, "ms": ms.value,
               "cached": False}
        if cache and ms.value > 0:
            table[key] = {k: out[k] for k in ("rays", "ang_block", "sched", "ms")}
            d = os.path.dirname(os.path.abspath(cache))
            os.makedirs(d, exist_ok=True)
            with open(cache, "w") as fh:
                json.dump(table, fh, indent=1)
        return out

    def submit(self, prob: Problem, x=None, workspace=None) -> int | None:
        """Adds a problem; returns its engine tag, or None when every slot is busy."""
        torch = _torch()
        g = prob.g
        b = prob.b
        assert b.is_cuda and b.is_contiguous() and b.numel() == g.m
        assert _dtype_code(b.dtype) == self.prec.proj, "b must be in the engine's proj dtype"
        meth = METHOD_AB if prob.method == "ab" else METHOD_BA
        st = Stop({"none": STOP_NONE, "dp": STOP_DP}[prob.stop], float(prob.tau), float(prob.noise_norm))
        nb = self.lib.abg_request_bytes(g.handle, meth, int(prob.k_max), self.prec, st)
        if nb == 0:
            raise AbgError(-1, "abg_request_bytes")
        ws = workspace if workspace is not None else _dev_empty(nb, b.device)
        x = x if x is not None else torch.empty(g.n, dtype=b.dtype, device=b.device)
        tag = self._next_tag
        self._next_tag += 1
        pend = _Pending(prob, x, ws, int(prob.k_max))
        r = Request(g.handle, meth, BP_KINDS[prob.bp], int(prob.k_max), st,
                    ctypes.c_void_p(b.data_ptr()),
                    ctypes.c_void_p(prob.x0.data_ptr()) if prob.x0 is not None else None,
                    ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                    ctypes.pointer(pend.info), tag)
        rc = self.lib.abg_engine_submit(self._h, ctypes.byref(r))
        if rc == -6:
            return None
        _check(rc, "abg_engine_submit")
        self._pending[tag] = pend
        return tag

    def step(self) -> int:
        """One round; returns the number of problems not yet finished."""
        n = ctypes.c_int()
        _check(self.lib.abg_engine_step(self._h, ctypes.byref(n)), "abg_engine_step")
        return n.value

    def poll(self) -> list:
        """Finished problems since the last poll: list of (tag, SolveResult)."""
        out = []
        cap = max(1, len(self._pending))
        tags = (ctypes.c_longlong * cap)()
        sts = (ctypes.c_int * cap)()
        n = ctypes.c_int()
        _check(self.lib.abg_engine_poll(self._h, tags, sts, cap, ctypes.byref(n)), "abg_engine_poll")
        for i in range(n.value):
            pend = self._pending.pop(int(tags[i]))
            out.append((int(tags[i]), pend.result(int(sts[i]))))
        return out

    def run(self, problems, max_rounds: int = 100000) -> list:
        """Solves the problems together; returns SolveResults in input order."""
        tags = []
        for p in problems:
            t = self.submit(p)
            if t is None:
                raise AbgError(-6, "Engine.run: more problems than slots")
            tags.append(t)
        done = {}
        rounds = 0
        while len(done) < len(tags):
            self.step()
            for t, r in self.poll():
                done[t] = r
            rounds += 1
            if rounds > max_rounds:
                raise AbgError(-5, "Engine.run: no progress")
        return [done[t] for t in tags]


def batch_solve(problems, proj="f32", basis="f32", rays: int = 0, ang_block: int = 0,
                sched: int = -1, stream=None) -> list:
    """abg_batch_solve: all problems on a new engine; returns SolveResults in input order."""
    torch = _torch()
    lib = load_library()
    prec = Precision(_DTYPES[proj], _DTYPES[basis])
    keep = []
    reqs = (Request * len(problems))()
    for i, prob in enumerate(problems):
        g, b = prob.g, prob.b
        meth = METHOD_AB if prob.method == "ab" else METHOD_BA
        st = Stop({"none": STOP_NONE, "dp": STOP_DP}[prob.stop], float(prob.tau), float(prob.noise_norm))
        nb = lib.abg_request_bytes(g.handle, meth, int(prob.k_max), prec, st)
        if nb == 0:
            raise AbgError(-1, "abg_request_bytes")
        ws = _dev_empty(nb, b.device)
        x = torch.empty(g.n, dtype=b.dtype, device=b.device)
        pend = _Pending(prob, x, ws, int(prob.k_max))
        keep.append(pend)
        reqs[i] = Request(g.handle, meth, BP_KINDS[prob.bp], int(prob.k_max),
                          st, ctypes.c_void_p(b.data_ptr()),
                          ctypes.c_void_p(prob.x0.data_ptr()) if prob.x0 is not None else None,
                          ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                          ctypes.pointer(pend.info), i)
    _check(lib.abg_batch_solve(reqs, len(problems), prec, int(rays), int(ang_block), int(sched),
                               _stream_ptr(stream)), "abg_batch_solve")
    return [p.result(p.info.status) for p in keep]
