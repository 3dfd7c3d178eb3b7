"""ctypes binding of libabgmres (include/abgmres.h): argument marshalling only.

Torch tensors supply device memory and the current HIP stream; every computation runs
in the library's kernels. The module fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libabgmres.so")

F64, F32, BF16 = 0, 1, 2
BP_HAT, BP_ADJ = 0, 1
STOP_NONE, STOP_DP, STOP_NCP = 0, 1, 2
METHOD_AB, METHOD_BA = 0, 1

STATUS = {0: "ok", -1: "einval", -2: "enomem", -3: "ehip", -4: "enan", -5: "edevice",
          1: "not_converged", 2: "breakdown", 3: "zero_rhs"}
EXPORTS = ["abg_create_geometry", "abg_destroy_geometry", "abg_geometry_sizes",
           "abg_fp_workspace_bytes", "abg_fp_apply", "abg_bp_apply", "abg_workspace_bytes",
           "abg_ab_gmres", "abg_ba_gmres", "abg_status_string", "abg_profile_enable",
           "abg_profile_read"]


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


_lib = None


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
    lib.abg_workspace_bytes.argtypes = [vp, i, i, Precision, Stop]
    lib.abg_workspace_bytes.restype = sz
    for name in ("abg_ab_gmres", "abg_ba_gmres"):
        getattr(lib, name).argtypes = [vp, i, vp, vp, vp, i, Stop, Precision, vp, sz,
                                       ctypes.POINTER(Info), vp]
    lib.abg_status_string.argtypes = [i]
    lib.abg_status_string.restype = ctypes.c_char_p
    lib.abg_profile_enable.argtypes = [i]
    lib.abg_profile_read.argtypes = [ctypes.POINTER(ctypes.c_longlong), _dp, i]
    _lib = lib
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
                 ang_start: float = 0.0, angles_deg=None, det_spacing: float = 1.0):
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
        self.N, self.n_ang, self.n_det = int(N), int(n_ang), int(n_det)
        self.n = self.N * self.N
        self.m = self.n_ang * self.n_det
        self._fp_ws = {}

    def close(self):
        if getattr(self, "_h", None):
            load_library().abg_destroy_geometry(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def fp_workspace(self, dtype_code: int, device):
        key = (dtype_code, str(device))
        ws = self._fp_ws.get(key)
        if ws is None:
            nb = load_library().abg_fp_workspace_bytes(self._h, dtype_code)
            ws = _dev_empty(nb, device)
            self._fp_ws[key] = ws
        return ws

    def fp(self, x, out=None, stream=None):
        """y = A x (line model) for a contiguous CUDA tensor x of n elements."""
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

    def bp(self, y, kind: str = "hat", out=None, stream=None):
        """x = B y (kind "hat", unmatched) or x = A^T y (kind "adj")."""
        torch = _torch()
        assert y.is_cuda and y.is_contiguous() and y.numel() == self.m
        t = _dtype_code(y.dtype)
        x = out if out is not None else torch.empty(self.n, dtype=y.dtype, device=y.device)
        _check(load_library().abg_bp_apply(self._h, BP_ADJ if kind == "adj" else BP_HAT, t,
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


_DTYPES = {"f64": F64, "f32": F32, "bf16": BF16}


def workspace_bytes(g: Geometry, method: str, k_max: int, proj="f32", basis="f32",
                    stop="none") -> int:
    st = Stop({"none": STOP_NONE, "dp": STOP_DP, "ncp": STOP_NCP}[stop], 1.0, 1.0)
    return int(load_library().abg_workspace_bytes(g.handle, METHOD_AB if method == "ab" else METHOD_BA,
                                                  int(k_max), Precision(_DTYPES[proj], _DTYPES[basis]), st))


def gmres(method: str, g: Geometry, b, k_max: int, stop: str = "none", tau: float = 1.0,
          noise_norm: float = 0.0, bp: str = "hat", basis: str | None = None, x0=None,
          out=None, workspace=None, want_H: bool = False, stream=None) -> SolveResult:
    """AB-GMRES (method "ab") or BA-GMRES ("ba") through the C ABI.

    b: CUDA tensor of m elements (float64 or float32: the projector dtype);
    basis: "f64", "f32" or "bf16" storage of the Krylov basis (default: b's dtype).
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
    rc = fn(g.handle, BP_ADJ if bp == "adj" else BP_HAT, ctypes.c_void_p(b.data_ptr()), x0p,
            ctypes.c_void_p(x.data_ptr()), int(k_max), st, prec, ctypes.c_void_p(ws.data_ptr()),
            ws.numel(), ctypes.byref(info), _stream_ptr(stream))
    _check(rc, "abg_%s_gmres" % method, ok=(0, 1, 2, 3))
    kd = info.k_done
    Hm = None
    if H is not None:
        Hm = H.T[:kd + 1, :kd].copy()   # column-major (k_max+1) x k_max in memory
    return SolveResult(x=x, status=STATUS[rc], k_stop=info.k_stop, k_done=kd,
                       res_norm=info.res_norm, ncp_dist=info.ncp_dist, beta=info.beta,
                       n_literal=info.n_literal, res_hist=res[:kd].copy(),
                       ls_hist=ls[:kd].copy(), ncp_hist=ncp[:kd].copy(), H=Hm)


def ab_gmres(g, b, k_max, **kw) -> SolveResult:
    return gmres("ab", g, b, k_max, **kw)


def ba_gmres(g, b, k_max, **kw) -> SolveResult:
    return gmres("ba", g, b, k_max, **kw)


def profile_enable(on: bool = True):
    load_library().abg_profile_enable(1 if on else 0)


def profile_read(reset: bool = True):
    counts = (ctypes.c_longlong * 4)()
    ms = (ctypes.c_double * 4)()
    load_library().abg_profile_read(counts, ms, 1 if reset else 0)
    names = ["forward", "back", "mgs", "combine"]
    return {nm: (int(counts[i]), float(ms[i])) for i, nm in enumerate(names)}
