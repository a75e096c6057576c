"""Seeded synthetic inputs for cone-beam backprojection workloads.

The paper's benchmark reconstructs a 256 mm cube from 496 filtered C-arm
projections of 1248x960 pixels, each with its own 3x4 projection matrix
(paper, Section 3.1, "Code analysis").  The measured projections and
matrices are not available, so this module makes stand-ins with the same
shapes and value distribution:

* a circular short-scan geometry (source-isocentre 750 mm, source-detector
  1200 mm, 0.308 mm pixels, 200 degrees, seeded +-0.5 mm jitter of source
  and detector centre) and its FP64 projection matrices;
* a seeded 10-ellipsoid phantom, its analytic line integrals, and their
  Feldkamp pre-processing (cosine weight, Parker weight, Ram-Lak filter).

It holds no step of the backprojection.  Both the GPU path and the CPU
oracle take their inputs from here; neither shares any other code.

Random numbers come from splitmix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

ELL_STRIDE = 17
MASK64 = (1 << 64) - 1


def build(force: bool = True) -> str:
    """Compile synth.c into libsynth.so next to it."""
    global _lib
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               os.path.join(_HERE, "synth.c"), "-o", _LIB_PATH + ".tmp", "-lm"]
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
        lib.synth_line_integrals.argtypes = [fp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             dp, dp, dp, dp, ctypes.c_double, dp, ctypes.c_int]
        lib.synth_fdk_prefilter.argtypes = [fp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                            ctypes.c_int]
        lib.synth_voxelize.argtypes = [fp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, dp, dp, ctypes.c_int, ctypes.c_int]
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fptr(a: np.ndarray):
    assert a.dtype == np.float32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class SplitMix64:
    """splitmix64 generator (Steele, Lea, Flood 2014)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        """53-bit uniform in [lo, hi)."""
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / 9007199254740992.0))

    def normal(self) -> float:
        """Standard normal by the Box-Muller transform (one value per call)."""
        u1 = 1.0 - self.uniform()  # (0, 1]
        u2 = self.uniform()
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
@dataclass
class Geometry:
    """Per-view flat-panel cone-beam geometry (all FP64, millimetres)."""
    n_views: int
    H: int
    W: int
    sid: float
    sdd: float
    pixel: float
    arc: float          # radians
    betas: np.ndarray   # (V,)
    src: np.ndarray     # (V,3) source position
    det: np.ndarray     # (V,3) detector centre (centre of pixel ((W-1)/2,(H-1)/2))
    eu: np.ndarray      # (V,3) unit detector u axis (along a row, increasing column)
    ev: np.ndarray      # (V,3) unit detector v axis (increasing row)
    nrm: np.ndarray     # (V,3) unit detector normal, pointing from source to detector
    P: np.ndarray       # (V,3,4) row-major projection matrices

    @property
    def dbeta(self) -> float:
        return self.arc / max(self.n_views - 1, 1)


def projection_matrix(s, d, eu, ev, nrm, sid, pixel, W, H) -> np.ndarray:
    """3x4 matrix mapping homogeneous world mm to (u*w, v*w, w) in pixel
    indices, with w = depth along the detector normal / sid, so that w = 1
    at the isocentre depth."""
    cu, cv = 0.5 * (W - 1), 0.5 * (H - 1)
    D = float(np.dot(d - s, nrm))
    rho = np.concatenate([nrm, [-np.dot(nrm, s)]])
    P = np.empty((3, 4))
    P[2] = rho / sid
    for r, (e, c) in enumerate(((eu, cu), (ev, cv))):
        ee = np.concatenate([e, [-np.dot(e, s)]])
        P[r] = (D * ee + np.dot(s - d, e) * rho) / (pixel * sid) + c * P[2]
    return P


def cone_beam_geometry(n_views: int = 496, H: int = 960, W: int = 1248, sid: float = 750.0,
                       sdd: float = 1200.0, pixel: float = 0.308, arc_deg: float = 200.0,
                       jitter_mm: float = 0.5, seed: int = 1104) -> Geometry:
    """Circular scan about the world z axis, beta_i = i * arc / (V-1).

    Unjittered: source s = sid (cos b, sin b, 0), detector normal
    n = -s/sid, detector centre d = s + sdd n, eu = (-sin b, cos b, 0),
    ev = (0, 0, 1).  Source and detector centre then get i.i.d.
    U(-jitter, jitter) offsets per axis (source x,y,z then detector x,y,z
    for each view in turn); the axes stay unjittered."""
    rng = SplitMix64(seed)
    arc = math.radians(arc_deg)
    V = n_views
    betas = np.array([i * arc / (V - 1) if V > 1 else 0.0 for i in range(V)])
    src = np.empty((V, 3)); det = np.empty((V, 3)); eu = np.empty((V, 3))
    ev = np.empty((V, 3)); nrm = np.empty((V, 3)); P = np.empty((V, 3, 4))
    for i, b in enumerate(betas):
        c, s_ = math.cos(b), math.sin(b)
        s = np.array([sid * c, sid * s_, 0.0])
        n = np.array([-c, -s_, 0.0])
        d = s + sdd * n
        if jitter_mm:
            s = s + np.array([rng.uniform(-jitter_mm, jitter_mm) for _ in range(3)])
            d = d + np.array([rng.uniform(-jitter_mm, jitter_mm) for _ in range(3)])
        src[i], det[i], nrm[i] = s, d, n
        eu[i] = (-s_, c, 0.0)
        ev[i] = (0.0, 0.0, 1.0)
        P[i] = projection_matrix(s, d, eu[i], ev[i], n, sid, pixel, W, H)
    return Geometry(V, H, W, sid, sdd, pixel, arc, betas, src, det, eu, ev, nrm, P)


def ray_plane_project(geom: Geometry, i: int, X: np.ndarray):
    """Project world points X (...,3) onto view i by explicit ray/plane
    intersection.  Returns (u, v, w) with u, v in pixel indices and w the
    depth along the normal divided by sid."""
    s, d, e1, e2, n = geom.src[i], geom.det[i], geom.eu[i], geom.ev[i], geom.nrm[i]
    X = np.asarray(X, dtype=np.float64)
    depth = (X - s) @ n
    t = np.dot(d - s, n) / depth
    p = s + t[..., None] * (X - s)
    u = 0.5 * (geom.W - 1) + ((p - d) @ e1) / geom.pixel
    v = 0.5 * (geom.H - 1) + ((p - d) @ e2) / geom.pixel
    return u, v, depth / geom.sid


# --------------------------------------------------------------------------
# volume frame
# --------------------------------------------------------------------------
FOV_MM = 256.0


def volume_frame(N: int, fov_mm: float = FOV_MM):
    """(voxel_size, origin) of an N^3 grid filling a centred fov_mm cube:
    voxel centres at origin + voxel_size * index, symmetric about 0."""
    vs = fov_mm / N
    o = -0.5 * fov_mm + 0.5 * vs
    return vs, (o, o, o)


# --------------------------------------------------------------------------
# phantom
# --------------------------------------------------------------------------
def _quat_to_matrix(q):
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def ellipsoid_phantom(seed: int = 5243, n: int = 10, scale: float = 1.0) -> np.ndarray:
    """(n, 17) ellipsoid records.  Ellipsoid 0 is the body (centre 0,
    semi-axes (95, 80, 85) mm, density 0.02 /mm); the others have centres
    U([-60,60]^2 x [-36,36]) mm, semi-axes U(10,50) mm, a uniformly random
    rotation (normalised Gaussian quaternion) and density U(-0.01, 0.01).
    Per ellipsoid the draws are: centre x,y,z; semi-axes; 4 normals;
    density.  `scale` multiplies every length (for smaller fields of view)."""
    rng = SplitMix64(seed)
    E = np.zeros((n, ELL_STRIDE))
    E[0, 3:6] = (95.0, 80.0, 85.0)
    E[0, 6:15] = np.eye(3).ravel()
    E[0, 15] = 0.02
    for e in range(1, n):
        c = (rng.uniform(-60, 60), rng.uniform(-60, 60), rng.uniform(-36, 36))
        a = (rng.uniform(10, 50), rng.uniform(10, 50), rng.uniform(10, 50))
        q = np.array([rng.normal() for _ in range(4)])
        q /= np.linalg.norm(q)
        E[e, 0:3] = c
        E[e, 3:6] = a
        E[e, 6:15] = _quat_to_matrix(q).ravel()
        E[e, 15] = rng.uniform(-0.01, 0.01)
    E[:, 0:6] *= scale
    return E


def sphere_phantom(radius: float, density: float, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    E = np.zeros((1, ELL_STRIDE))
    E[0, 0:3] = center
    E[0, 3:6] = radius
    E[0, 6:15] = np.eye(3).ravel()
    E[0, 15] = density
    return E


# --------------------------------------------------------------------------
# projections
# --------------------------------------------------------------------------
def line_integrals(geom: Geometry, ell: np.ndarray, views=None) -> np.ndarray:
    """FP32 (V, H, W) analytic line integrals of the phantom."""
    lib = _load()
    idx = np.arange(geom.n_views) if views is None else np.asarray(views)
    V = len(idx)
    out = np.empty((V, geom.H, geom.W), dtype=np.float32)
    src = np.ascontiguousarray(geom.src[idx]); det = np.ascontiguousarray(geom.det[idx])
    eu = np.ascontiguousarray(geom.eu[idx]); ev = np.ascontiguousarray(geom.ev[idx])
    ell = np.ascontiguousarray(ell, dtype=np.float64)
    rc = lib.synth_line_integrals(_fptr(out), V, geom.H, geom.W, _dptr(src), _dptr(det),
                                  _dptr(eu), _dptr(ev), geom.pixel, _dptr(ell), len(ell))
    if rc != 0:
        raise RuntimeError(f"synth_line_integrals failed ({rc})")
    return out


def fft_length(W: int) -> int:
    L = 1
    while L < 2 * W - 1:
        L <<= 1
    return L


def fdk_prefilter(proj: np.ndarray, geom: Geometry, parker: bool = True, views=None) -> np.ndarray:
    """Feldkamp pre-processing of line integrals, in place (cosine weight,
    Parker short-scan weight, Ram-Lak row filter, scaled by tau * dbeta)."""
    lib = _load()
    idx = np.arange(geom.n_views) if views is None else np.asarray(views)
    betas = np.ascontiguousarray(geom.betas[idx])
    delta = 0.5 * (geom.arc - math.pi)
    rc = lib.synth_fdk_prefilter(_fptr(proj), proj.shape[0], geom.H, geom.W, _dptr(betas),
                                 delta, geom.dbeta, geom.sid, geom.sdd, geom.pixel,
                                 fft_length(geom.W), 1 if parker else 0)
    if rc != 0:
        raise RuntimeError(f"synth_fdk_prefilter failed ({rc})")
    return proj


def filtered_projections(geom: Geometry, ell: np.ndarray, views=None) -> np.ndarray:
    p = line_integrals(geom, ell, views)
    return fdk_prefilter(p, geom, views=views)


def voxelize(ell: np.ndarray, N: int, voxel_size: float, origin, sub: int = 1,
             shape=None) -> np.ndarray:
    lib = _load()
    nz, ny, nx = shape if shape is not None else (N, N, N)
    out = np.empty((nz, ny, nx), dtype=np.float32)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    ell = np.ascontiguousarray(ell, dtype=np.float64)
    rc = lib.synth_voxelize(_fptr(out), nx, ny, nz, voxel_size, _dptr(o), _dptr(ell), len(ell), sub)
    if rc != 0:
        raise RuntimeError("synth_voxelize failed")
    return out


def voxelize_torch(ell: np.ndarray, N: int, voxel_size: float, origin, device, sub: int = 1):
    """Phantom density at the N^3 voxels, the mean of sub^3 regularly spaced
    samples inside each voxel (sub = 1: the voxel centre), computed with
    torch on `device` (for generating many training volumes quickly)."""
    import torch
    vol = torch.zeros(N, N, N, dtype=torch.float64, device=device)
    for sz in range(sub):
        for sy in range(sub):
            for sx in range(sub):
                off = [(s_ + 0.5) / sub - 0.5 for s_ in (sx, sy, sz)]
                ax = [origin[k] + voxel_size * (torch.arange(N, dtype=torch.float64, device=device)
                                                + off[k]) for k in range(3)]
                z, y, x = torch.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
                for E in np.asarray(ell, dtype=np.float64):
                    R = torch.tensor(E[6:15].reshape(3, 3), device=device)
                    d = [x - E[0], y - E[1], z - E[2]]
                    q = 0.0
                    for k in range(3):
                        t = (R[0, k] * d[0] + R[1, k] * d[1] + R[2, k] * d[2]) / E[3 + k]
                        q = q + t * t
                    vol += (q <= 1.0).to(torch.float64) * E[15]
    return (vol / (sub ** 3)).float()


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
WORKLOADS = {
    # parity gate: 128^3, 2 mm voxels
    "fdk128": dict(N=128, n_views=496, H=960, W=1248, pixel=0.308),
    # main throughput workload: 512^3, 0.5 mm voxels
    "fdk512": dict(N=512, n_views=496, H=960, W=1248, pixel=0.308),
    # large volume with reduced-precision projection storage
    "fdk1024": dict(N=1024, n_views=496, H=960, W=1248, pixel=0.308),
    # differentiable pair: 256^3 volumes, 248 views of 624x480
    "fdk256x8": dict(N=256, n_views=248, H=480, W=624, pixel=0.616),
    # learned filter: 62 sparse views of 624x480
    "learn128": dict(N=128, n_views=62, H=480, W=624, pixel=0.616),
}


def workload(name: str, jitter_seed: int = 1104, phantom_seed: int = 5243):
    """(geometry, phantom, voxel_size, origin, N) of a named workload."""
    cfg = WORKLOADS[name]
    geom = cone_beam_geometry(cfg["n_views"], cfg["H"], cfg["W"], pixel=cfg["pixel"],
                              seed=jitter_seed)
    ell = ellipsoid_phantom(phantom_seed)
    vs, origin = volume_frame(cfg["N"])
    return geom, ell, vs, origin, cfg["N"]
