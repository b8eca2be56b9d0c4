"""Pins for the oracle's PCA normals, curvature and Jacobi eigensolver (CPU)."""
import math

import numpy as np
import pytest

from gen import rng_for, sphere_plane
from tests.helpers import angle_between


def test_jacobi_matches_numpy_eigh(oracle_mod):
    rng = rng_for(200)
    for _ in range(300):
        M = rng.normal(size=(3, 3))
        scale = 10.0 ** rng.uniform(-6, 3, size=3)
        A = M @ np.diag(scale) @ M.T
        w, v = oracle_mod.jacobi3(A)
        we, ve = np.linalg.eigh(A)
        assert np.allclose(w, we, rtol=1e-10, atol=1e-13 * we[-1])
        # eigen-equation and orthonormality
        assert np.allclose(A @ v, v * w, atol=1e-11 * we[-1])
        assert np.allclose(v.T @ v, np.eye(3), atol=1e-12)
        # eigenvector of the smallest eigenvalue agrees with LAPACK up to sign
        if we[1] - we[0] > 1e-6 * we[2]:
            assert abs(abs(v[:, 0] @ ve[:, 0]) - 1) < 1e-9


def test_jacobi_diagonal_and_repeated(oracle_mod):
    w, v = oracle_mod.jacobi3(np.diag([3.0, 1.0, 2.0]))
    assert w.tolist() == [1.0, 2.0, 3.0]
    assert np.array_equal(np.abs(v), np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]], float))
    w, v = oracle_mod.jacobi3(np.eye(3) * 5)
    assert w.tolist() == [5.0, 5.0, 5.0]


def test_axis_plane_exact_normal(oracle_mod):
    # points exactly on z = 0.5: covariance has an exactly zero z row/column,
    # so the normal is exactly +-e_z, oriented toward the viewpoint (0,0,0)
    rng = rng_for(201)
    xy = rng.uniform(-1, 1, size=(500, 2))
    pts = np.column_stack([xy, np.full(500, 0.5)]).astype(np.float32)
    n, curv, ev = oracle_mod.normals(pts, 10, (0, 0, 0))
    assert np.all(n == np.array([0.0, 0.0, -1.0]))
    assert np.all(curv == 0) and np.all(ev[:, 0] == 0)
    n2, _, _ = oracle_mod.normals(pts, 10, (0, 0, 2.0))
    assert np.all(n2 == np.array([0.0, 0.0, 1.0]))


def test_tilted_plane_normal(oracle_mod):
    rng = rng_for(202)
    nrm = np.array([1.0, -2.0, 2.0]) / 3.0
    u = np.cross(nrm, [1.0, 0, 0]); u /= np.linalg.norm(u)
    w = np.cross(nrm, u)
    ab = rng.uniform(-1, 1, size=(800, 2))
    pts = (ab[:, :1] * u + ab[:, 1:] * w + 0.3 * nrm).astype(np.float32)
    n, curv, _ = oracle_mod.normals(pts, 12, (0, 0, 0))
    # float32 rounding of the inputs is the only deviation from the plane;
    # the viewpoint lies on the -nrm side
    ang = angle_between(n, -nrm)
    assert ang.max() < 5e-6
    assert curv.max() < 1e-10


def test_sphere_normals_radial(oracle_mod):
    rng = rng_for(203)
    g = rng.normal(size=(20000, 3))
    pts = (g / np.linalg.norm(g, axis=1, keepdims=True)).astype(np.float32)
    n, curv, _ = oracle_mod.normals(pts, 10, (0, 0, 0))
    # oriented toward the centre; neighbourhood radius ~0.03 -> tilt well under 0.05 rad
    ang = angle_between(n, -pts.astype(np.float64))
    assert np.percentile(ang, 99) < 0.05 and ang.max() < 0.2
    assert 0 < np.median(curv) < 0.01


def test_orientation_rule(oracle_mod):
    pts = sphere_plane(rng_for(204), 3000)
    vp = np.array([0.3, -2.0, 0.7])
    n, _, _ = oracle_mod.normals(pts, 10, vp)
    dots = np.sum(n * (vp - pts.astype(np.float64)), axis=1)
    assert np.all(dots >= 0)
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-12)


def test_orientation_tie_rule(oracle_mod):
    # viewpoint inside the plane z=0: n.(v-p)=0 exactly, so the first nonzero
    # component decides (e_z has only z nonzero -> +e_z)
    rng = rng_for(205)
    xy = rng.integers(-50, 51, size=(400, 2)) / 32.0
    pts = np.column_stack([xy, np.zeros(400)]).astype(np.float32)
    pts = np.unique(pts, axis=0)
    n, _, _ = oracle_mod.normals(pts, 8, (0.25, 0.5, 0.0))
    assert np.all(n == np.array([0.0, 0.0, 1.0]))


@pytest.mark.parametrize("p", [(1.0, 2.0, 3.0), (0.1, 0.2, 0.3), (-7.3, 1e3, 0.017)])
def test_degenerate_coincident_points(oracle_mod, p):
    # identical neighbours: zero covariance, so the normal is undefined and
    # reported as (0,0,0) with curvature 0, whatever the coordinates
    pts = np.vstack([np.tile([p], (12, 1)), [[5.0, 5.0, 5.0]] * 3]).astype(np.float32)
    n, curv, ev = oracle_mod.normals(pts, 10, (0, 0, 0))
    assert np.all(n[:12] == 0) and np.all(curv[:12] == 0) and np.all(ev[:12] == 0)


def test_matches_numpy_cov_eigh(oracle_mod):
    # independent path: neighbours by numpy lexsort on exact keys, numpy
    # covariance (1/k) and LAPACK eigh
    rng = rng_for(206)
    pts = (rng.integers(-64, 65, size=(600, 3)) / 64.0).astype(np.float32)
    pts = np.unique(pts, axis=0)
    k = 9
    n, curv, ev = oracle_mod.normals(pts, k, (0, 0, 0), method="brute")
    p64 = pts.astype(np.float64)
    for i in range(0, len(pts), 7):
        dd = ((p64 - p64[i]) ** 2).sum(1)
        nb = np.lexsort((np.arange(len(dd)), dd))[:k]
        C = np.cov(p64[nb].T, bias=True)
        we, ve = np.linalg.eigh(C)
        assert np.allclose(ev[i], we, rtol=1e-9, atol=1e-14)
        tr = we.sum()
        assert math.isclose(curv[i], we[0] / tr if tr > 0 else 0.0, rel_tol=1e-9, abs_tol=1e-14)
        if we[1] - we[0] > 1e-6 * we[2]:
            assert abs(abs(n[i] @ ve[:, 0]) - 1) < 1e-9


@pytest.mark.parametrize("k", [3, 10, 16, 32])
def test_kdtree_and_brute_normals_identical(oracle_mod, k):
    pts = sphere_plane(rng_for(207, k), 3000)
    a = oracle_mod.normals(pts, k, (0, 0, 0), method="brute")
    b = oracle_mod.normals(pts, k, (0, 0, 0), method="kdtree")
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
