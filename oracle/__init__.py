"""FP64 CPU oracle for cone-beam backprojection (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The GPU library never calls it, and the two share
no code; their only common dependency is the seeded input generator
`synth`, which holds none of the method's arithmetic.

The C file `oracle.c` holds the plain definitions (backprojection of the
paper's Listing 1 with zero-extended taps, in FP64, and its exact
transpose).  This module wraps them and adds the error measures used to
compare a result with the oracle: relative RMSE and the PSNR of the
paper's accuracy study (Section 7.2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c (plain -O2, no FMA contraction) into liboracle.so."""
    global _lib
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               os.path.join(_HERE, "oracle.c"), "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
        _lib = None
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        ip = ctypes.POINTER(ctypes.c_int)
        i = ctypes.c_int
        lib.oracle_backproject_box.argtypes = [dp, i, ctypes.c_double, dp, fp, i, i, i, dp,
                                               i, i, i, i, i, i]
        lib.oracle_backproject_points.argtypes = [dp, ip, ctypes.c_longlong, i,
                                                  ctypes.c_double, dp, fp, i, i, i, dp]
        lib.oracle_forward_project.argtypes = [dp, i, i, i, dp, dp, i, ctypes.c_double, dp]
        lib.oracle_threads.argtypes = []
        _lib = lib
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _prep(proj, P, origin):
    proj = np.ascontiguousarray(proj, dtype=np.float32)
    if proj.ndim != 3:
        raise ValueError("proj must be (n_views, H, W)")
    P = np.ascontiguousarray(np.asarray(P, dtype=np.float64).reshape(-1, 12))
    if P.shape[0] != proj.shape[0]:
        raise ValueError("one 3x4 matrix per view is required")
    o = np.ascontiguousarray(origin, dtype=np.float64).reshape(3)
    return proj, P, o


def backproject(proj, P, N: int, voxel_size: float, origin, box=None, out=None) -> np.ndarray:
    """FP64 backprojection.  box = ((x0,nx),(y0,ny),(z0,nz)) restricts the
    output to a sub-block (shape (nz, ny, nx)); default is the whole N^3
    grid.  `out`, if given, is accumulated into."""
    proj, P, o = _prep(proj, P, origin)
    if box is None:
        box = ((0, N), (0, N), (0, N))
    (x0, nx), (y0, ny), (z0, nz) = box
    if out is None:
        out = np.zeros((nz, ny, nx), dtype=np.float64)
    assert out.dtype == np.float64 and out.shape == (nz, ny, nx) and out.flags.c_contiguous
    V, H, W = proj.shape
    rc = _load().oracle_backproject_box(_d(out), N, voxel_size, _d(o), _f(proj), V, H, W, _d(P),
                                        x0, nx, y0, ny, z0, nz)
    if rc != 0:
        raise ValueError("oracle_backproject_box: invalid arguments")
    return out


def backproject_points(proj, P, N: int, voxel_size: float, origin, xyz) -> np.ndarray:
    """FP64 backprojection at voxels xyz (n, 3) given as (x, y, z) indices."""
    proj, P, o = _prep(proj, P, origin)
    xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
    out = np.zeros(len(xyz), dtype=np.float64)
    V, H, W = proj.shape
    rc = _load().oracle_backproject_points(
        _d(out), xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(xyz), N, voxel_size,
        _d(o), _f(proj), V, H, W, _d(P))
    if rc != 0:
        raise ValueError("oracle_backproject_points: invalid arguments")
    return out


def forward_project(vol, P, H: int, W: int, voxel_size: float, origin) -> np.ndarray:
    """FP64 exact transpose of `backproject`: (n_views, H, W) projections of
    the N^3 volume `vol` (indexed [z, y, x])."""
    vol = np.ascontiguousarray(vol, dtype=np.float64)
    N = vol.shape[0]
    if vol.shape != (N, N, N):
        raise ValueError("vol must be N^3")
    P = np.ascontiguousarray(np.asarray(P, dtype=np.float64).reshape(-1, 12))
    o = np.ascontiguousarray(origin, dtype=np.float64).reshape(3)
    out = np.zeros((P.shape[0], H, W), dtype=np.float64)
    rc = _load().oracle_forward_project(_d(out), P.shape[0], H, W, _d(P), _d(vol), N,
                                        voxel_size, _d(o))
    if rc != 0:
        raise ValueError("oracle_forward_project: invalid arguments")
    return out


def threads() -> int:
    """OpenMP threads the oracle's parallel loops run on."""
    return int(_load().oracle_threads())


# --------------------------------------------------------------------------
# error measures
# --------------------------------------------------------------------------
def rel_rmse(V, R) -> float:
    """||V - R||_2 / ||R||_2, accumulated in FP64."""
    V = np.asarray(V, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    den = np.sqrt(np.sum(R * R))
    return float(np.sqrt(np.sum((V - R) ** 2)) / den) if den > 0 else float(
        np.sqrt(np.sum((V - R) ** 2)))


def psnr(V, R) -> float:
    """PSNR of the paper's accuracy study (Section 7.2): 10 log10(M^2 / MSE)
    with M the value range of the reference R (max R - min R)."""
    V = np.asarray(V, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    M = float(R.max() - R.min())
    mse = float(np.mean((V - R) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(M * M / mse)
