"""CPU oracle for point-to-plane ICP, normals and k-NN (Python side).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers.  The GPU library never
imports, links or runs anything here, and nothing here imports the GPU
library.  The arithmetic lives in ``oracle.c`` (float64, written from the
definitions; see its header); this module compiles it with gcc and wraps it
with ctypes.

Parity status of each function (what pins it lives in ``tests/``):
  knn_brute           the definition itself; pinned by hand-checked cases,
                      lattices with exact ties, and sorting.
  knn_kdtree          pinned bit-equal to knn_brute.
  normals             pinned by exact planes, spheres, numpy.linalg.eigh.
  p2plane_system      pinned by identity pairs, normal-flip invariance,
                      symmetry / PSD, finite differences of the residual.
  icp                 pinned by closed-form Kabsch alignment on noiseless
                      copies, recovery of known transforms, equivariance and
                      quadratic convergence.
  rigid_fit           pinned by exact recovery of known motions, Horn's
                      quaternion method (numpy eigh), reflections, and
                      brute-force search over nearby rotations.
  icp_p2p             pinned by one-step recovery from exact correspondences
                      and convergence to the ground truth.
  combined_system     pinned to p2plane_system at weights (0, 1), to the
                      analytic point-to-point blocks, and by finite
                      differences of the weighted objective.
  icp_combined        pinned by recovery of known transforms and by equality
                      with icp at weights (0, 1).
  projective_pixels   pinned by round trips of back-projected pixels,
                      rounding at half-pixel boundaries, points behind the
                      camera and outside the image.
  icp_projective      pinned by the identity pose on a frame and itself, the
                      point-to-plane system of explicit pairs, and recovery
                      of a camera motion from noiseless views.
  normals_radius      pinned by lattice neighbourhoods counted by hand,
                      kd-tree against brute-force membership, equality with
                      k-NN normals when the radius holds exactly k points,
                      planes and spheres.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")
# a differently built copy of the same source (e.g. the sanitizer build of
# tests/test_oracle_sanitized.py) can be loaded instead
_LIB_OVERRIDE = os.environ.get("ORACLE_LIB")

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")

ICP_CONVERGED, ICP_MAXITER, ICP_DEGENERATE, ICP_NO_INLIERS = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile oracle.c into _oracle.so (gcc, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(out: str) -> str:
    """The same source built with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code, gcc), every report fatal; load it through ORACLE_LIB with the
    ASan runtime preloaded."""
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_lib = None


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            lib = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
        lib.oracle_knn_brute.argtypes = [_f32p, ctypes.c_int64, _f32p, ctypes.c_int64, ctypes.c_int,
                                         _i32p, _f32p]
        lib.oracle_knn_kdtree.argtypes = lib.oracle_knn_brute.argtypes
        lib.oracle_normals.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int, _f64p, ctypes.c_int,
                                       _f64p, _f64p, _f64p]
        lib.oracle_jacobi3.argtypes = [_f64p, _f64p, _f64p]
        lib.oracle_jacobi3.restype = None
        lib.oracle_cholesky6.argtypes = [_f64p, _f64p]
        lib.oracle_euler_zyx.argtypes = [ctypes.c_double] * 3 + [_f64p]
        lib.oracle_euler_zyx.restype = None
        lib.oracle_p2plane_system.argtypes = [_f32p, ctypes.c_int64, _f32p, _f32p, ctypes.c_int64,
                                              _f64p, ctypes.c_double, ctypes.c_int, _f64p, _f64p,
                                              _i64p, _f64p, _i32p]
        lib.oracle_icp.argtypes = [_f32p, ctypes.c_int64, _f32p, _f32p, ctypes.c_int64,
                                   ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_int, _f64p, _i32p, _i64p, _f64p, ctypes.c_void_p]
        lib.oracle_rigid_fit.argtypes = [_f64p, _f64p, ctypes.c_int64, _f64p, _f64p, _f64p, _f64p]
        lib.oracle_icp_p2p.argtypes = [_f32p, ctypes.c_int64, _f32p, ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int, _f64p,
                                       _i32p, _i64p, _f64p]
        lib.oracle_combined_system.argtypes = [_f32p, ctypes.c_int64, _f32p, _f32p, ctypes.c_int64, _f64p,
                                               ctypes.c_double, ctypes.c_double, ctypes.c_double, _f64p, _f64p,
                                               _i64p, _f64p]
        lib.oracle_icp_combined.argtypes = [_f32p, ctypes.c_int64, _f32p, _f32p, ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                            ctypes.c_double, ctypes.c_int, _f64p, _i32p, _i64p, _f64p]
        lib.oracle_projective_pixels.argtypes = [_f32p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _f64p, _f64p,
                                                 _i64p]
        lib.oracle_icp_projective.argtypes = [_f32p, ctypes.c_int64, _f32p, _f32p, ctypes.c_int, ctypes.c_int,
                                              _f64p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                                              ctypes.c_double, _f64p, _i32p, _i64p, _f64p]
        lib.oracle_normals_radius.argtypes = [_f32p, ctypes.c_int64, ctypes.c_float, ctypes.c_int, _f64p,
                                              ctypes.c_int, _f64p, _f64p, _f64p, _i32p]
        lib.oracle_num_threads.argtypes = []
        _lib = lib
    return _lib


def _pts(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("points must be (n, 3)")
    return a


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def knn(ref, qry, k: int, method: str = "brute"):
    """k nearest reference points of every query under the float32 key,
    ascending by (key, index).  Returns (idx int32 (nq,k), key float32)."""
    ref, qry = _pts(ref), _pts(qry)
    idx = np.empty((qry.shape[0], k), np.int32)
    d2 = np.empty((qry.shape[0], k), np.float32)
    fn = _load().oracle_knn_brute if method == "brute" else _load().oracle_knn_kdtree
    rc = fn(ref, ref.shape[0], qry, qry.shape[0], int(k), idx, d2)
    if rc:
        raise ValueError(f"oracle knn failed ({rc})")
    return idx, d2


def normals(xyz, k: int, viewpoint=(0.0, 0.0, 0.0), method: str = "kdtree"):
    """PCA normals, curvature and ascending covariance eigenvalues (float64)."""
    xyz = _pts(xyz)
    n = xyz.shape[0]
    nrm = np.empty((n, 3), np.float64)
    curv = np.empty(n, np.float64)
    ev = np.empty((n, 3), np.float64)
    vp = np.ascontiguousarray(viewpoint, dtype=np.float64)
    rc = _load().oracle_normals(xyz, n, int(k), vp, int(method == "kdtree"), nrm, curv, ev)
    if rc:
        raise ValueError(f"oracle normals failed ({rc})")
    return nrm, curv, ev


def jacobi3(a):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(9).copy()
    w = np.empty(3, np.float64)
    v = np.empty(9, np.float64)
    _load().oracle_jacobi3(a, w, v)
    return w, v.reshape(3, 3)


def cholesky6(A):
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(36)
    L = np.empty(36, np.float64)
    rc = _load().oracle_cholesky6(A, L)
    return None if rc else L.reshape(6, 6)


def euler_zyx(alpha: float, beta: float, gamma: float) -> np.ndarray:
    R = np.empty(9, np.float64)
    _load().oracle_euler_zyx(float(alpha), float(beta), float(gamma), R)
    return R.reshape(3, 3)


def p2plane_system(src, tgt, tgt_normals, T, d_max: float, method: str = "kdtree"):
    """Linearised point-to-plane system at pose T.
    Returns dict(A (6,6), b (6,), inliers, sum_r2, corr (ns,) int32)."""
    src, tgt, nrm = _pts(src), _pts(tgt), _pts(tgt_normals)
    T = np.ascontiguousarray(T, dtype=np.float64).reshape(16)
    A = np.empty(36, np.float64)
    b = np.empty(6, np.float64)
    inl = np.zeros(1, np.int64)
    s2 = np.zeros(1, np.float64)
    corr = np.empty(src.shape[0], np.int32)
    rc = _load().oracle_p2plane_system(src, src.shape[0], tgt, nrm, tgt.shape[0], T, float(d_max),
                                       int(method == "kdtree"), A, b, inl, s2, corr)
    if rc:
        raise ValueError(f"oracle system failed ({rc})")
    return dict(A=A.reshape(6, 6), b=b, inliers=int(inl[0]), sum_r2=float(s2[0]), corr=corr)


def icp(src, tgt, tgt_normals, T_init=None, d_max: float = 0.1, max_iters: int = 20,
        conv_tol: float = 0.0, method: str = "kdtree"):
    """Point-to-plane ICP.  Returns dict(T, status, iterations, inliers, rms, x_hist)."""
    src, tgt, nrm = _pts(src), _pts(tgt), _pts(tgt_normals)
    T0 = None
    if T_init is not None:
        T0 = np.ascontiguousarray(T_init, dtype=np.float64).reshape(16)
    T = np.empty(16, np.float64)
    si = np.zeros(2, np.int32)
    si64 = np.zeros(1, np.int64)
    sd = np.zeros(1, np.float64)
    xh = np.zeros((max(max_iters, 1), 6), np.float64)
    rc = _load().oracle_icp(src, src.shape[0], tgt, nrm, tgt.shape[0],
                            None if T0 is None else T0.ctypes.data, float(d_max), int(max_iters),
                            float(conv_tol), int(method == "kdtree"), T, si, si64, sd, xh.ctypes.data)
    if rc:
        raise ValueError(f"oracle icp failed ({rc})")
    it = int(si[1])
    return dict(T=T.reshape(4, 4), status=int(si[0]), iterations=it, inliers=int(si64[0]),
                rms=float(sd[0]), x_hist=xh[:it].copy())


def rigid_fit(p, q):
    """Least-squares rigid motion p -> q (closed form).  Returns (R (3,3),
    t (3,), top, gap): the rotation is unique when gap > 0."""
    p = np.ascontiguousarray(p, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
    R, t, top, gap = np.empty(9), np.empty(3), np.empty(1), np.empty(1)
    if _load().oracle_rigid_fit(p, q, p.shape[0], R, t, top, gap):
        raise ValueError("rigid_fit needs at least one pair")
    return R.reshape(3, 3), t, float(top[0]), float(gap[0])


def _stats(T, si, si64, sd):
    return dict(T=T.reshape(4, 4), status=int(si[0]), iterations=int(si[1]), inliers=int(si64[0]),
                rms=float(sd[0]))


def icp_p2p(src, tgt, T_init=None, d_max: float = 0.1, max_iters: int = 20, conv_tol: float = 0.0,
            method: str = "kdtree"):
    """Point-to-point ICP with the closed-form fit.  Returns dict(T, status,
    iterations, inliers, rms)."""
    src, tgt = _pts(src), _pts(tgt)
    T0 = None if T_init is None else np.ascontiguousarray(T_init, dtype=np.float64).reshape(16)
    T, si, si64, sd = np.empty(16), np.zeros(2, np.int32), np.zeros(1, np.int64), np.zeros(1)
    rc = _load().oracle_icp_p2p(src, src.shape[0], tgt, tgt.shape[0], None if T0 is None else T0.ctypes.data,
                                float(d_max), int(max_iters), float(conv_tol), int(method == "kdtree"), T, si,
                                si64, sd)
    if rc:
        raise ValueError(f"oracle icp_p2p failed ({rc})")
    return _stats(T, si, si64, sd)


def combined_system(src, tgt, tgt_normals, T, d_max: float, w_point: float, w_plane: float):
    """(A (6,6), b (6,), inliers, weighted sum of squared residuals)."""
    src, tgt = _pts(src), _pts(tgt)
    nrm = _pts(tgt_normals)
    T = np.ascontiguousarray(T, dtype=np.float64).reshape(16)
    A, b, inl, s2 = np.empty(36), np.empty(6), np.zeros(1, np.int64), np.zeros(1)
    rc = _load().oracle_combined_system(src, src.shape[0], tgt, nrm, tgt.shape[0], T, float(d_max), float(w_point),
                                        float(w_plane), A, b, inl, s2)
    if rc:
        raise ValueError(f"oracle combined_system failed ({rc})")
    return A.reshape(6, 6), b, int(inl[0]), float(s2[0])


def icp_combined(src, tgt, tgt_normals, T_init=None, w_point: float = 0.5, w_plane: float = 1.0,
                 d_max: float = 0.1, max_iters: int = 20, conv_tol: float = 0.0, method: str = "kdtree"):
    """ICP with the weighted point-to-point + point-to-plane metric."""
    src, tgt, nrm = _pts(src), _pts(tgt), _pts(tgt_normals)
    T0 = None if T_init is None else np.ascontiguousarray(T_init, dtype=np.float64).reshape(16)
    T, si, si64, sd = np.empty(16), np.zeros(2, np.int32), np.zeros(1, np.int64), np.zeros(1)
    rc = _load().oracle_icp_combined(src, src.shape[0], tgt, nrm, tgt.shape[0],
                                     None if T0 is None else T0.ctypes.data, float(w_point), float(w_plane),
                                     float(d_max), int(max_iters), float(conv_tol), int(method == "kdtree"), T, si,
                                     si64, sd)
    if rc:
        raise ValueError(f"oracle icp_combined failed ({rc})")
    return _stats(T, si, si64, sd)


def _intrinsics(K):
    """float32-rounded intrinsics as float64 (the C ABI takes float32)."""
    return np.ascontiguousarray(np.asarray(K, dtype=np.float32).astype(np.float64))


def projective_pixels(src, width: int, height: int, K, T):
    """Candidate pixel (raster index) of every source point at pose T, -1 if none."""
    src = _pts(src)
    pix = np.empty(src.shape[0], np.int64)
    _load().oracle_projective_pixels(src, src.shape[0], int(width), int(height), _intrinsics(K),
                                     np.ascontiguousarray(T, dtype=np.float64).reshape(16), pix)
    return pix


def icp_projective(src, tgt, tgt_normals, width: int, height: int, K, T_init=None, d_max: float = 0.2,
                   max_iters: int = 15, conv_tol: float = 0.0):
    """Point-to-plane ICP with projective correspondences into the organized
    target image (height*width, 3)."""
    src = _pts(src)
    tgt = np.ascontiguousarray(tgt, dtype=np.float32).reshape(-1, 3)
    nrm = np.ascontiguousarray(tgt_normals, dtype=np.float32).reshape(-1, 3)
    if tgt.shape[0] != width * height or nrm.shape[0] != width * height:
        raise ValueError("organized target must have width*height points and normals")
    T0 = None if T_init is None else np.ascontiguousarray(T_init, dtype=np.float64).reshape(16)
    T, si, si64, sd = np.empty(16), np.zeros(2, np.int32), np.zeros(1, np.int64), np.zeros(1)
    _load().oracle_icp_projective(src, src.shape[0], tgt, nrm, int(width), int(height), _intrinsics(K),
                                  None if T0 is None else T0.ctypes.data, float(d_max), int(max_iters),
                                  float(conv_tol), T, si, si64, sd)
    return _stats(T, si, si64, sd)


def normals_radius(xyz, radius: float, k: int = 0, viewpoint=(0.0, 0.0, 0.0), method: str = "kdtree"):
    """Normals from radius (k = 0) or hybrid (k nearest within the radius)
    neighbourhoods.  Returns (normals (n,3) f64, curvature (n,), eigenvalues
    (n,3), counts (n,) int32)."""
    xyz = _pts(xyz)
    n = xyz.shape[0]
    nrm, curv, ev = np.empty((n, 3)), np.empty(n), np.empty((n, 3))
    cnt = np.empty(n, np.int32)
    rc = _load().oracle_normals_radius(xyz, n, float(np.float32(radius)), int(k),
                                       np.ascontiguousarray(viewpoint, dtype=np.float64), int(method == "kdtree"),
                                       nrm, curv, ev, cnt)
    if rc:
        raise ValueError(f"oracle normals_radius failed ({rc})")
    return nrm, curv, ev, cnt
