"""abg_fp_apply_noalloc (forward projection through the library's static device scratch,
for callers that cannot allocate) against abg_fp_apply with a caller workspace, through
the C ABI: two calls in a row, the second on a smaller geometry (the scratch then holds
the first call's larger padded copies), both bit-for-bit equal to the workspace entry
point; a third call in the other dtype; a geometry too large for the scratch is refused
with ABG_ENOMEM and leaves the output untouched."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

ENOMEM = -2


def _ws_apply(lib, g, dt, x, y, torch):
    nb = lib.abg_fp_workspace_bytes(g.handle, dt)
    ws = torch.full((nb,), 0x7F, dtype=torch.uint8, device="cuda")
    rc = lib.abg_fp_apply(g.handle, dt, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                          ctypes.c_void_p(ws.data_ptr()), nb, None)
    assert rc == 0


def _noalloc_apply(lib, g, dt, x, y):
    return lib.abg_fp_apply_noalloc(g.handle, dt, ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(y.data_ptr()), None)


@pytest.mark.parametrize("first,second", [((1024, 720, "f64"), (300, 180, "f64")),
                                          ((2048, 360, "f64"), (512, 720, "f32"))])
def test_noalloc_forward_equals_workspace_forward(gpu_lib, first, second):
    import torch
    from paper_2110_01481_amd import _binding as B
    lib = B.load_library()
    for i, (N, n_ang, dts) in enumerate((first, second)):
        tdt = torch.float64 if dts == "f64" else torch.float32
        dt = B.F64 if dts == "f64" else B.F32
        g = gpu_lib.Geometry(N, n_ang, W.n_det_for(N), ang_range=180.0 if i == 0 else 120.0)
        x = torch.tensor(W.ellipse_phantom(N, 6, W.rng(97, N, 0)), dtype=tdt, device="cuda")
        y_ws = torch.empty(g.m, dtype=tdt, device="cuda")
        y_na = torch.full((g.m,), float("nan"), dtype=tdt, device="cuda")
        _ws_apply(lib, g, dt, x, y_ws, torch)
        assert _noalloc_apply(lib, g, dt, x, y_na) == 0
        torch.cuda.synchronize()
        assert torch.equal(y_ws, y_na), (N, n_ang, dts)
        g.close()


def test_noalloc_refuses_a_geometry_beyond_the_scratch(gpu_lib):
    import torch
    from paper_2110_01481_amd import _binding as B
    lib = B.load_library()
    N = 2169      # 2 x 2169 x 2177 FP64 values exceed the 72 MiB scratch
    g = gpu_lib.Geometry(N, 4, W.n_det_for(N))
    assert lib.abg_fp_workspace_bytes(g.handle, B.F64) > 72 << 20
    x = torch.ones(g.n, dtype=torch.float64, device="cuda")
    y = torch.full((g.m,), 7.0, dtype=torch.float64, device="cuda")
    assert _noalloc_apply(lib, g, B.F64, x, y) == ENOMEM
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
    # the same geometry in FP32 fits (2 x 2169 x 2177 x 4 bytes) and matches
    x32, y32 = x.float(), torch.empty(g.m, dtype=torch.float32, device="cuda")
    assert _noalloc_apply(lib, g, B.F32, x32, y32) == 0
    y_ws = torch.empty_like(y32)
    _ws_apply(lib, g, B.F32, x32, y_ws, torch)
    torch.cuda.synchronize()
    assert torch.equal(y32, y_ws)
    g.close()
