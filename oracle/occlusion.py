"""Visibility of straight segments for the FP64 oracle.

Test infrastructure (see ``oracle/__init__``).

Eqs. (1)-(2) gate every ray contribution by a Heaviside visibility.  A
segment is blocked by a triangle (plain C, ``occlusion.c``) or by the solid
of a sphere or of a finite vertical cylinder (closed form below) when the
crossing lies strictly inside the segment, t in (EPS, 1 - EPS).
"""
import ctypes
import os
import subprocess

import numpy as np

EPS = 1e-6
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "occlusion.c")
_LIB = os.path.join(_HERE, "_occlusion.so")
_lib = None


def build_library(force=False):
    """Compile occlusion.c with gcc (plain C, no GPU)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_library())
        lib.oracle_occlude.restype = ctypes.c_int
        lib.oracle_occlude.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_void_p]
        _lib = lib
    return _lib


def segments_vs_triangles(tri, p0, p1, brute=False):
    """Boolean per segment: does it cross any triangle?  tri is (n, 3, 3)."""
    p0 = np.ascontiguousarray(p0, dtype=np.float64).reshape(-1, 3)
    p1 = np.ascontiguousarray(p1, dtype=np.float64).reshape(-1, 3)
    hit = np.zeros(p0.shape[0], dtype=np.uint8)
    if tri is None or len(tri) == 0 or p0.shape[0] == 0:
        return hit.astype(bool)
    tri = np.ascontiguousarray(tri, dtype=np.float64).reshape(-1, 9)
    rc = _load().oracle_occlude(tri.ctypes.data, tri.shape[0], p0.ctypes.data, p1.ctypes.data,
                                p0.shape[0], EPS, int(brute), hit.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle occlusion grid allocation failed")
    return hit.astype(bool)


def _interval_overlap(lo, hi):
    return np.maximum(lo, EPS) < np.minimum(hi, 1.0 - EPS)


def segments_vs_sphere(p0, p1, sph):
    """|P0 + t d - C|^2 <= a^2 for some t in (EPS, 1-EPS)."""
    cx, cy, cz, a = sph
    d = p1 - p0
    w = p0 - np.array([cx, cy, cz])
    A = np.einsum("ij,ij->i", d, d)
    B = np.einsum("ij,ij->i", d, w)
    C = np.einsum("ij,ij->i", w, w) - a * a
    disc = B * B - A * C
    ok = (disc > 0) & (A > 0)
    sq = np.sqrt(np.where(ok, disc, 0.0))
    Asafe = np.where(A > 0, A, 1.0)
    t0 = (-B - sq) / Asafe
    t1 = (-B + sq) / Asafe
    return ok & _interval_overlap(t0, t1)


def segments_vs_cylinder(p0, p1, cyl):
    """Segment meets the solid {(x-cx)^2 + (y-cy)^2 <= a^2, z0 <= z <= z0+h}."""
    cx, cy, z0, h, a = cyl
    d = p1 - p0
    wx, wy = p0[:, 0] - cx, p0[:, 1] - cy
    A = d[:, 0] ** 2 + d[:, 1] ** 2
    B = d[:, 0] * wx + d[:, 1] * wy
    C = wx * wx + wy * wy - a * a
    disc = B * B - A * C
    Asafe = np.where(A > 0, A, 1.0)
    sq = np.sqrt(np.maximum(disc, 0.0))
    lo_r = np.where(A > 0, (-B - sq) / Asafe, np.where(C <= 0, -np.inf, np.inf))
    hi_r = np.where(A > 0, (-B + sq) / Asafe, np.where(C <= 0, np.inf, -np.inf))
    radial = np.where(A > 0, disc > 0, C <= 0)
    dz = d[:, 2]
    dzs = np.where(dz != 0, dz, 1.0)
    ta = (z0 - p0[:, 2]) / dzs
    tb = (z0 + h - p0[:, 2]) / dzs
    lo_z = np.where(dz != 0, np.minimum(ta, tb), np.where((p0[:, 2] >= z0) & (p0[:, 2] <= z0 + h), -np.inf, np.inf))
    hi_z = np.where(dz != 0, np.maximum(ta, tb), np.where((p0[:, 2] >= z0) & (p0[:, 2] <= z0 + h), np.inf, -np.inf))
    lo = np.maximum(lo_r, lo_z)
    hi = np.minimum(hi_r, hi_z)
    return radial & _interval_overlap(lo, hi)


def segments_blocked(scene, p0, p1, skip=None, bodies=True, triangles=True):
    """Blocked by any triangle or any body except the one named by ``skip``
    (('s', i) or ('c', i))."""
    p0 = np.asarray(p0, dtype=float)
    p1 = np.asarray(p1, dtype=float)
    blocked = np.zeros(p0.shape[0], dtype=bool)
    if p0.shape[0] == 0:
        return blocked
    if triangles:
        blocked |= segments_vs_triangles(scene.get("tri"), p0, p1)
    if bodies:
        for i, s in enumerate(scene.get("spheres", [])):
            if skip != ("s", i):
                blocked |= segments_vs_sphere(p0, p1, s)
        for i, c in enumerate(scene.get("cylinders", [])):
            if skip != ("c", i):
                blocked |= segments_vs_cylinder(p0, p1, c)
    return blocked
