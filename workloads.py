"""Seeded synthetic inputs for the AB-/BA-GMRES CT reconstruction workloads.

This module holds no projector or solver arithmetic. It only draws problem sizes,
ellipse phantoms and Gaussian noise directions, so that the GPU library and the FP64
reference oracle can consume the very same arrays.

Stand-in for the paper's test data (Sec. 6.1, Table 6.1): the paper's ground truth is
the AIRtools II ``threephases`` phantom on ASTRA matrices, neither of which is
available, so every workload here is a sum of seeded random ellipses with the image
and sinogram shapes of the benchmark configurations below.

Seeds: ``numpy.random.default_rng([1000*cfg + instance, stream])`` with stream 0 for
the phantom, 1 for the noise direction and 2 for size/arrival draws.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

STREAM_PHANTOM = 0
STREAM_NOISE = 1
STREAM_DRAWS = 2


def rng(cfg: int, instance: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([1000 * cfg + instance, stream])


def n_det_for(N: int) -> int:
    """Detector bins covering the image diagonal: ceil(N*sqrt(2)), made odd.

    Gives 91, 183, 363, 725, 1449, 2897 for N = 64, 128, 256, 512, 1024, 2048.
    """
    d = math.ceil(N * math.sqrt(2.0))
    return d if d % 2 else d + 1


def ellipse_phantom(N: int, n_ellipses: int, gen: np.random.Generator) -> np.ndarray:
    """Sum of ``n_ellipses`` filled ellipses sampled at pixel centres, row-major N*N.

    Semi-axes U[N/16, 3N/8], centres U[-N/4, N/4]^2, orientation U[0, pi),
    intensity U[0.1, 1]. Pixel (r, c) has centre (c - N/2 + 1/2, r - N/2 + 1/2).
    """
    img = np.zeros((N, N), dtype=np.float64)
    yc = (np.arange(N, dtype=np.float64) - N / 2 + 0.5)[:, None]
    xc = (np.arange(N, dtype=np.float64) - N / 2 + 0.5)[None, :]
    for _ in range(n_ellipses):
        a, b = gen.uniform(N / 16, 3 * N / 8, size=2)
        cx, cy = gen.uniform(-N / 4, N / 4, size=2)
        phi = gen.uniform(0.0, math.pi)
        val = gen.uniform(0.1, 1.0)
        dx = xc - cx
        dy = yc - cy
        u = (dx * math.cos(phi) + dy * math.sin(phi)) / a
        v = (-dx * math.sin(phi) + dy * math.cos(phi)) / b
        img += val * ((u * u + v * v) <= 1.0)
    return img.ravel()


def noise_direction(m: int, gen: np.random.Generator) -> np.ndarray:
    return gen.standard_normal(m)


def add_noise(b_clean: np.ndarray, eta: float, g: np.ndarray):
    """b = b_clean + e with e = eta*||b_clean|| g/||g||, so ||e||/||b_clean|| = eta.

    Returns (b, ||e||). The paper fixes the relative noise level this way (Sec. 6.1).
    """
    e = (eta * np.linalg.norm(b_clean) / np.linalg.norm(g)) * g
    return b_clean + e, float(np.linalg.norm(e))


@dataclass(frozen=True)
class Workload:
    """One reconstruction problem: parallel-beam geometry, phantom and solver settings."""
    cfg: int
    instance: int
    N: int
    n_ang: int
    n_det: int
    ang_range: float = 180.0
    n_ellipses: int = 5
    eta: float = 0.01
    k_max: int = 30
    stop: str = "none"          # "none" | "dp" | "ncp"
    tau: float = 1.0
    method: str = "ab"          # "ab" | "ba"
    extra: dict = field(default_factory=dict, compare=False)

    @property
    def n(self) -> int:
        return self.N * self.N

    @property
    def m(self) -> int:
        return self.n_ang * self.n_det

    def phantom(self) -> np.ndarray:
        return ellipse_phantom(self.N, self.n_ellipses, rng(self.cfg, self.instance, STREAM_PHANTOM))

    def noise_dir(self) -> np.ndarray:
        return noise_direction(self.m, rng(self.cfg, self.instance, STREAM_NOISE))


# The benchmark workloads (plain FP64 case, single solve, large single solve).
CONFIG1 = Workload(cfg=1, instance=0, N=64, n_ang=90, n_det=91, n_ellipses=5, eta=0.01,
                   k_max=30, stop="none")
CONFIG2 = Workload(cfg=2, instance=0, N=512, n_ang=720, n_det=725, n_ellipses=20, eta=0.02,
                   k_max=100, stop="dp", tau=1.02)
CONFIG3 = Workload(cfg=3, instance=0, N=2048, n_ang=1800, n_det=2897, n_ellipses=50,
                   eta=0.01, k_max=60, stop="ncp", method="ba")
# Under-determined few-view scan (m < n), the regime Sec. 6.2 mentions beside the
# over-determined one: a 512^2 ellipse phantom seen from 180 angles (m = 0.5 n).
CONFIG_FEW_VIEW = Workload(cfg=6, instance=0, N=512, n_ang=180, n_det=725, n_ellipses=20,
                           eta=0.02, k_max=100, stop="dp", tau=1.02)


def batched_workloads(count: int = 64, cfg: int = 4):
    """The batched mix: N from {128,256,512,1024}, angles from {60,180,360,720},
    instances 0..count/2-1 full range [0,180), the rest limited [0,120); noise
    U[0.005, 0.03]; even instances AB, odd BA; DP stop with tau = 1.02."""
    gen = rng(cfg, 0, STREAM_DRAWS)
    out = []
    for i in range(count):
        N = int(gen.choice([128, 256, 512, 1024]))
        n_ang = int(gen.choice([60, 180, 360, 720]))
        eta = float(gen.uniform(0.005, 0.03))
        out.append(Workload(cfg=cfg, instance=i, N=N, n_ang=n_ang, n_det=n_det_for(N),
                            ang_range=180.0 if i < count // 2 else 120.0,
                            n_ellipses=10, eta=eta, k_max=100, stop="dp", tau=1.02,
                            method="ab" if i % 2 == 0 else "ba"))
    return out


def serving_requests(rate: float = 50.0, duration: float = 60.0, cfg: int = 5,
                     sizes=(256, 512, 1024, 2048)):
    """Poisson arrivals at ``rate`` per second for ``duration`` seconds.

    Each request: N from ``sizes``, angles U{180..1800}, noise U[0.01, 0.03],
    AB or BA with equal odds, k_max U{30..120}, DP stop with tau = 1.02.
    Returns a list of (arrival_time_s, Workload).
    """
    gen = rng(cfg, 0, STREAM_DRAWS)
    t = 0.0
    out = []
    i = 0
    while True:
        t += float(gen.exponential(1.0 / rate))
        if t >= duration:
            break
        N = int(gen.choice(list(sizes)))
        n_ang = int(gen.integers(180, 1801))
        eta = float(gen.uniform(0.01, 0.03))
        method = "ab" if gen.random() < 0.5 else "ba"
        k_max = int(gen.integers(30, 121))
        out.append((t, Workload(cfg=cfg, instance=i, N=N, n_ang=n_ang, n_det=n_det_for(N),
                                n_ellipses=10, eta=eta, k_max=k_max, stop="dp", tau=1.02,
                                method=method)))
        i += 1
    return out
