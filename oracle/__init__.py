"""Reference oracle for AB-/BA-GMRES with an unmatched projector pair -- TEST INFRASTRUCTURE.

Plain, slow, FP64 CPU implementation of what the GPU path computes, written from
Hansen, Hayami & Morikuni, "GMRES methods for tomographic reconstruction with an
unmatched back projector" (arXiv 2110.01481). It is used only by ``tests/``, by
``__graft_entry__.smoke()`` and by the CPU-baseline leg of ``bench.py``; the product
library never imports, calls or links anything here, and this package never imports
the product.

Contents:
  geometry   angle table and detector positions (Sec. 6.1, Table 6.1 sizes)
  projectors A (line model), A^T, and the unmatched pixel-driven interpolating B
             (C, OpenMP, FP64; oracle/projectors.c)
  brute      Liang-Barsky clipping of every ray against every pixel (tiny grids)
  gmres      AB-GMRES and BA-GMRES exactly as listed in Sec. 2 (MGS Arnoldi,
             least squares on H_k by numpy.linalg.lstsq, iterate, residual,
             stopping rule)
  stopping   discrepancy principle and NCP criterion (Sec. 6.3)
  krylov     independent Krylov-subspace minimisers used to pin the GMRES code
"""
from .core import (Geometry, angle_table, assemble_dense, basis_storage)
from .brute import brute_force_matrix, chord_length_in_square
from .stopping import ncp_distance, dp_index, ncp_index
from .gmres import ab_gmres, ba_gmres, GmresResult, bf16_round
from .krylov import krylov_basis, min_residual_iterate, golub_kahan_lsqr, golub_kahan_lsmr

__all__ = [
    "Geometry", "angle_table", "assemble_dense", "basis_storage",
    "brute_force_matrix", "chord_length_in_square",
    "ncp_distance", "dp_index", "ncp_index",
    "ab_gmres", "ba_gmres", "GmresResult", "bf16_round",
    "krylov_basis", "min_residual_iterate", "golub_kahan_lsqr", "golub_kahan_lsmr",
]
