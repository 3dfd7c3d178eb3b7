"""Geometry and FP64 projectors of the reference oracle (test infrastructure only).

The paper's operators are ASTRA's explicit matrices (Sec. 6.1); here the forward
projector A is the line model (exact ray/pixel intersection lengths), A^T its exact
transpose, and B the unmatched back projector that interpolates linearly on the
detector at each pixel centre. The strip and interpolation (Joseph) models of Sec. 6.1
and their transposes complete the paper's three discretisations (their norm-wise
differences reproduce Table 6.2). Conventions are spelled out in ``projectors.c``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# An axis-aligned ray lies on a pixel edge when its offset from the pixel centre is
# 1/2 up to this tolerance (bin positions s0 + i*ds are rounded).
EDGE_TIE = 1e-9
_LIB_PATH = os.path.join(_HERE, "liboracle_proj.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        for name in ("orc_forward", "orc_adjoint", "orc_backproject_hat"):
            f = getattr(lib, name)
            f.restype = None
            f.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_double, dp, dp]
        for name in ("orc_forward_model", "orc_transpose_model"):
            f = getattr(lib, name)
            f.restype = None
            f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int,
                          ctypes.c_double, dp, dp]
        lib.orc_model_gram.restype = None
        lib.orc_model_gram.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int,
                                       ctypes.c_double, dp]
        lib.orc_strip_max.restype = ctypes.c_double
        lib.orc_strip_max.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int,
                                      ctypes.c_double]
        lib.orc_transpose_strip_tau.restype = None
        lib.orc_transpose_strip_tau.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int,
                                                ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, dp, dp]
        lib.orc_strip_tau_sums.restype = None
        lib.orc_strip_tau_sums.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        lib.orc_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def angle_table(n_ang: int, ang_range: float = 180.0, ang_start: float = 0.0, angles_deg=None):
    """theta_a = start + a*range/n_ang degrees (Table 6.1: 0,1,..,179 and 0,0.3,..,179.7).

    cos/sin are exact (0, +-1) at multiples of 90 degrees so that axis-aligned rays are
    recognised as such.
    """
    if angles_deg is None:
        th = ang_start + (np.arange(n_ang, dtype=np.float64) * ang_range) / n_ang
    else:
        th = np.asarray(angles_deg, dtype=np.float64)
    rad = th * (np.pi / 180.0)
    c = np.cos(rad)
    s = np.sin(rad)
    for a, t in enumerate(th):
        if np.fmod(t, 90.0) == 0.0:
            quadrant = int(round(t / 90.0)) % 4
            c[a], s[a] = [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)][quadrant]
    return th, c, s


# Discretisation models of the forward projector (Sec. 6.1): codes of projectors.c.
MODELS = {"line": 0, "strip": 1, "joseph": 2}


class Geometry:
    """2-D parallel-beam scan of an N x N unit-pixel image: n = N^2, m = n_ang*n_det."""

    def __init__(self, N: int, n_ang: int, n_det: int, ang_range: float = 180.0,
                 ang_start: float = 0.0, angles_deg=None, det_spacing: float = 1.0):
        self.N = int(N)
        self.n_det = int(n_det)
        self.ds = float(det_spacing)
        self.theta, self.cos, self.sin = angle_table(n_ang, ang_range, ang_start, angles_deg)
        self.n_ang = len(self.theta)
        self.n = self.N * self.N
        self.m = self.n_ang * self.n_det

    @property
    def s(self) -> np.ndarray:
        """Detector bin centres s_i = (i - (n_det-1)/2) * ds."""
        return (np.arange(self.n_det, dtype=np.float64) - 0.5 * (self.n_det - 1)) * self.ds

    def _call(self, name, src, n_out):
        src = np.ascontiguousarray(src, dtype=np.float64)
        out = np.empty(n_out, dtype=np.float64)
        getattr(_load(), name)(self.N, self.n_ang, _ptr(self.cos), _ptr(self.sin), self.n_det,
                               self.ds, _ptr(src), _ptr(out))
        return out

    def _call_model(self, name, model, src, n_out):
        src = np.ascontiguousarray(src, dtype=np.float64)
        out = np.empty(n_out, dtype=np.float64)
        getattr(_load(), name)(MODELS[model], self.N, self.n_ang, _ptr(self.cos), _ptr(self.sin),
                               self.n_det, self.ds, _ptr(src), _ptr(out))
        return out

    def A_model(self, model: str, x: np.ndarray) -> np.ndarray:
        """y = A x for the line, strip or Joseph (interpolation) model (Sec. 6.1)."""
        assert x.size == self.n
        return self._call_model("orc_forward_model", model, x, self.m)

    def AT_model(self, model: str, y: np.ndarray) -> np.ndarray:
        """x = A^T y for the line, strip or Joseph model."""
        assert y.size == self.m
        return self._call_model("orc_transpose_model", model, y, self.n)

    def model_gram(self) -> np.ndarray:
        """3 x 3 Frobenius inner products <A_a, A_b> of the line, strip and Joseph models."""
        G = np.empty(9)
        _load().orc_model_gram(self.N, self.n_ang, _ptr(self.cos), _ptr(self.sin), self.n_det,
                               self.ds, _ptr(G))
        return G.reshape(3, 3)

    def strip_max(self) -> float:
        """Largest entry of the strip-model matrix A_s."""
        if getattr(self, "_strip_max", None) is None:
            self._strip_max = float(_load().orc_strip_max(self.N, self.n_ang, _ptr(self.cos),
                                                          _ptr(self.sin), self.n_det, self.ds))
        return self._strip_max

    def B_tau(self, tau: float):
        """x = B_tau y (Sec. 6.5): A_s^T without its entries below tau * max A_s (entries
        within 1e-6 * max of that threshold are kept)."""
        mx = self.strip_max()

        def apply(y):
            y = np.ascontiguousarray(y, dtype=np.float64)
            assert y.size == self.m
            out = np.empty(self.n)
            _load().orc_transpose_strip_tau(self.N, self.n_ang, _ptr(self.cos), _ptr(self.sin),
                                            self.n_det, self.ds, tau * mx, mx, _ptr(y), _ptr(out))
            return out
        return apply

    def strip_tau_unmatchedness(self, tau: float) -> float:
        """||B_tau - A_s^T||_F / ||A_s||_F (Table 6.4)."""
        mx = self.strip_max()
        out = np.empty(2)
        _load().orc_strip_tau_sums(self.N, self.n_ang, _ptr(self.cos), _ptr(self.sin), self.n_det,
                                   self.ds, tau * mx, mx, _ptr(out))
        return float(np.sqrt(out[1] / out[0]))

    def A(self, x: np.ndarray) -> np.ndarray:
        """Forward projection y = A x (line model)."""
        assert x.size == self.n
        return self._call("orc_forward", x, self.m)

    def AT(self, y: np.ndarray) -> np.ndarray:
        """Matched back projection x = A^T y."""
        assert y.size == self.m
        return self._call("orc_adjoint", y, self.n)

    def B_hat(self, y: np.ndarray) -> np.ndarray:
        """Unmatched back projection x = B y (linear interpolation on the detector)."""
        assert y.size == self.m
        return self._call("orc_backproject_hat", y, self.n)

    def back(self, kind: str):
        """Back projector by name: "hat" (unmatched interpolation B), "adj" (A_line^T),
        "strip_t" (A_strip^T), "joseph_t" (A_Joseph^T)."""
        if kind == "strip_t":
            return lambda y: self.AT_model("strip", y)
        if kind == "joseph_t":
            return lambda y: self.AT_model("joseph", y)
        return {"hat": self.B_hat, "adj": self.AT}[kind]

    def fwd(self, model: str):
        """Forward projector by model name ("line", "strip", "joseph")."""
        return self.A if model == "line" else (lambda x: self.A_model(model, x))

    def back_pixels(self, kind: str, y: np.ndarray, pixels) -> np.ndarray:
        """(B y)_j or (A^T y)_j for the listed pixel indices only (NumPy, vectorised over
        angles): the same closed forms as the C projectors, for spot checks at sizes
        where a full back projection on the CPU is too slow."""
        Y = np.asarray(y, dtype=np.float64).reshape(self.n_ang, self.n_det)
        s0 = -0.5 * (self.n_det - 1) * self.ds
        p = np.maximum(np.abs(self.cos), np.abs(self.sin))
        q = np.minimum(np.abs(self.cos), np.abs(self.sin))
        rows = np.arange(self.n_ang)
        out = np.empty(len(pixels))
        for idx, j in enumerate(pixels):
            r, c = divmod(int(j), self.N)
            xc, yc = c - self.N / 2 + 0.5, r - self.N / 2 + 0.5
            t0 = xc * self.cos + yc * self.sin
            u = (t0 - s0) / self.ds
            base = np.floor(u).astype(np.int64)
            acc = 0.0
            for di in (-1, 0, 1, 2):
                i = base + di
                ok = (i >= 0) & (i < self.n_det)
                ic = np.clip(i, 0, self.n_det - 1)
                if kind == "hat":
                    w = np.maximum(0.0, 1.0 - np.abs(u - i)) / self.ds
                else:
                    at = np.abs(s0 + i * self.ds - t0)
                    flat, outer = 0.5 * (p - q), 0.5 * (p + q)
                    with np.errstate(divide="ignore", invalid="ignore"):
                        slope = np.where(q > 0, (outer - at) / (p * q), 0.0)
                    w = np.where(at <= flat, 1.0 / p, np.where(at >= outer, 0.0, slope))
                    axis = q == 0
                    edge = np.abs(at - 0.5) <= EDGE_TIE
                    w = np.where(axis, np.where(edge, 0.5 / p, np.where(at < 0.5, 1.0 / p, 0.0)), w)
                acc += float(np.sum(np.where(ok, w * Y[rows, ic], 0.0)))
            out[idx] = acc
        return out


def assemble_dense(g: Geometry):
    """Explicit A (m x n), A^T-kernel and B (n x m) by applying the operators to unit
    vectors -- only for tiny geometries."""
    A = np.zeros((g.m, g.n))
    for j in range(g.n):
        e = np.zeros(g.n)
        e[j] = 1.0
        A[:, j] = g.A(e)
    AT = np.zeros((g.n, g.m))
    B = np.zeros((g.n, g.m))
    for i in range(g.m):
        e = np.zeros(g.m)
        e[i] = 1.0
        AT[:, i] = g.AT(e)
        B[:, i] = g.B_hat(e)
    return A, AT, B


def basis_storage(method: str, k: int, m: int, n: int) -> int:
    """Number of stored basis entries after k iterations: AB keeps k vectors of length
    m, BA k vectors of length n (Sec. 6.2, storage rows of Table 6.3)."""
    return k * (m if method == "ab" else n)


def num_threads() -> int:
    return int(_load().orc_num_threads())
