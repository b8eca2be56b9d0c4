"""Pins for the oracle's point-to-plane system and ICP loop (CPU).

Each test is chosen so that a plausible slip in the oracle (a dropped term,
a sign, a transposed operand, a wrong composition order) fails it: the
closed-form Kabsch alignment, recovery of known transforms, exact identity
behaviour, normal-flip invariance, symmetry/PSD, the first-order model of the
residual, quadratic convergence and rigid-motion equivariance.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from gen import apply_rigid, make_workload, random_rigid, rng_for, room_scan, sphere_plane
from tests.helpers import kabsch, pose_err


def _normals(oracle_mod, pts, k=10):
    n, _, _ = oracle_mod.normals(pts, k, (0, 0, 0))
    return n.astype(np.float32)


def test_euler_zyx_matches_scipy(oracle_mod):
    rng = rng_for(300)
    for _ in range(50):
        a, b, g = rng.uniform(-0.5, 0.5, 3)
        R = oracle_mod.euler_zyx(a, b, g)
        ref = Rotation.from_euler("ZYX", [g, b, a]).as_matrix()   # Rz(g) Ry(b) Rx(a)
        assert np.allclose(R, ref, atol=1e-14)


def test_cholesky_matches_numpy(oracle_mod):
    rng = rng_for(301)
    for _ in range(50):
        M = rng.normal(size=(6, 6))
        A = M @ M.T + 1e-3 * np.eye(6)
        L = oracle_mod.cholesky6(A)
        assert np.allclose(L, np.linalg.cholesky(A), rtol=1e-10, atol=1e-12)
    A = np.diag([1, 1, 1, 1, 1, 0.0])
    assert oracle_mod.cholesky6(A) is None


def test_system_symmetric_psd_and_flip_invariant(oracle_mod):
    w = make_workload(0, size="small")
    n = _normals(oracle_mod, w.target)
    T = np.eye(4)
    s = oracle_mod.p2plane_system(w.source, w.target, n, T, w.d_max)
    A, b = s["A"], s["b"]
    assert np.array_equal(A, A.T)
    ev = np.linalg.eigvalsh(A)
    assert ev.min() >= -1e-12 * np.trace(A) and ev.min() > 0
    flip = n.copy()
    sel = rng_for(302).random(len(n)) < 0.5
    flip[sel] *= -1
    s2 = oracle_mod.p2plane_system(w.source, w.target, flip, T, w.d_max)
    assert np.array_equal(s2["A"], A) and np.array_equal(s2["b"], b)
    assert s2["inliers"] == s["inliers"] and s2["sum_r2"] == s["sum_r2"]


def test_system_is_first_order_model_of_residual(oracle_mod):
    """sum_i (r_i + J_i x)^2 = s2 + 2 b.x + x.A.x must match the true
    point-to-plane cost of the moved points, with the correspondences held,
    to first order in the twist x = (alpha, beta, gamma, tau)."""
    w = make_workload(0, size="small")
    n = _normals(oracle_mod, w.target)
    T = random_rigid(rng_for(303), 2.0, 0.01)
    s = oracle_mod.p2plane_system(w.source, w.target, n, T, w.d_max)
    corr = s["corr"]
    ok = corr >= 0
    p = w.source[ok].astype(np.float64) @ T[:3, :3].T + T[:3, 3]
    q = w.target[corr[ok]].astype(np.float64)
    nn = n[corr[ok]].astype(np.float64)
    rng = rng_for(304)
    for eps in (1e-3, 1e-4):
        x = rng.normal(size=6) * eps
        R = Rotation.from_euler("ZYX", [x[2], x[1], x[0]]).as_matrix()
        true_cost = np.sum((((p @ R.T) + x[3:] - q) * nn).sum(1) ** 2)
        model = s["sum_r2"] + 2 * s["b"] @ x + x @ s["A"] @ x
        # the model is exact up to the second-order term of the rotation
        assert abs(true_cost - model) < 50 * eps ** 2 * np.abs(s["b"]).sum() + 1e-12 + 1e-3 * eps * abs(model)
        # and its gradient is right: a wrong sign of b would double the error
        wrong = s["sum_r2"] - 2 * s["b"] @ x + x @ s["A"] @ x
        assert abs(true_cost - model) < 0.5 * abs(true_cost - wrong) + 1e-15


def test_first_step_is_normal_equation_solution(oracle_mod):
    w = make_workload(0, size="small")
    n = _normals(oracle_mod, w.target)
    s = oracle_mod.p2plane_system(w.source, w.target, n, np.eye(4), w.d_max)
    r = oracle_mod.icp(w.source, w.target, n, None, w.d_max, 1)
    x = -np.linalg.solve(s["A"], s["b"])
    assert np.allclose(r["x_hist"][0], x, rtol=1e-9, atol=1e-15)
    R = Rotation.from_euler("ZYX", [x[2], x[1], x[0]]).as_matrix()
    assert np.allclose(r["T"][:3, :3], R, atol=1e-13)
    assert np.allclose(r["T"][:3, 3], x[3:], atol=1e-15)


def test_identity_pair_stays_identity_bit_exact(oracle_mod):
    pts = sphere_plane(rng_for(305), 3000)
    n = _normals(oracle_mod, pts)
    r = oracle_mod.icp(pts, pts, n, None, 0.1, 10)
    assert np.array_equal(r["T"], np.eye(4))
    assert r["rms"] == 0.0 and r["inliers"] == 3000
    assert np.all(r["x_hist"] == 0)


def test_kabsch_equals_icp_on_noiseless_copy(oracle_mod):
    """On a noiseless exact copy the least-squares alignment of the known
    pairs (closed form) and ICP's fixed point are the same transform."""
    rng = rng_for(306)
    src = sphere_plane(rng, 4000, sigma=0.0)
    T = random_rigid(rng, 6.0, 0.04)
    tgt = apply_rigid(T, src)
    n = _normals(oracle_mod, tgt)
    r = oracle_mod.icp(src, tgt, n, None, 0.2, 30)
    K = kabsch(src, tgt)
    ea, et = pose_err(r["T"], K)
    assert ea < 1e-5 and et < 1e-6
    ga, gt = pose_err(K, T)
    assert ga < 1e-6 and gt < 1e-6


def test_gt_recovery_room_small_motion(oracle_mod):
    rng = rng_for(307)
    src = room_scan(rng, 160, 120)
    T = random_rigid(rng, 3.0, 0.03)
    tgt = apply_rigid(T, src)
    n, _, _ = oracle_mod.normals(tgt, 16, (0, 0, 0))
    r = oracle_mod.icp(src, tgt, n.astype(np.float32), None, 0.2, 40)
    ea, et = pose_err(r["T"], T)
    assert ea < 1e-5 and et < 1e-6


def test_workload0_recovers_ground_truth(oracle_mod):
    w = make_workload(0)
    n = _normals(oracle_mod, w.target, w.k)
    r = oracle_mod.icp(w.source, w.target, n, None, w.d_max, w.iters)
    ea, et = pose_err(r["T"], w.T_gt)
    assert ea < 1e-5 and et < 1e-6
    assert r["status"] == oracle_mod.ICP_MAXITER and r["iterations"] == w.iters


def test_quadratic_convergence(oracle_mod):
    rng = rng_for(308)
    src = sphere_plane(rng, 5000, sigma=0.0)
    T = random_rigid(rng, 1.0, 0.005)
    tgt = apply_rigid(T, src)
    n = _normals(oracle_mod, tgt)
    errs = []
    for it in range(1, 5):
        r = oracle_mod.icp(src, tgt, n, None, 0.2, it)
        errs.append(pose_err(r["T"], T)[0])
    # once nearest neighbours are the true partners this is Gauss-Newton on a
    # zero-residual problem: e_{k+1} <= C e_k^2 down to the float32 floor of
    # the target coordinates (a few 1e-9 rad here)
    assert errs[0] < 1e-2
    assert errs[1] < 1.0 * errs[0] ** 2
    assert errs[2] < 1e-7


def test_equivariance(oracle_mod):
    w = make_workload(0, size="small")
    n = _normals(oracle_mod, w.target)
    r = oracle_mod.icp(w.source, w.target, n, None, w.d_max, w.iters)
    G = random_rigid(rng_for(309), 30.0, 0.7)
    H = random_rigid(rng_for(310), 25.0, 0.3)
    # moving the source by H and the target by G maps the answer to G T H^-1
    src2 = apply_rigid(H, w.source)
    tgt2 = apply_rigid(G, w.target)
    n2 = (n.astype(np.float64) @ G[:3, :3].T).astype(np.float32)
    T0 = G @ np.eye(4) @ np.linalg.inv(H)
    r2 = oracle_mod.icp(src2, tgt2, n2, T0, w.d_max, w.iters)
    ea, et = pose_err(r2["T"], G @ r["T"] @ np.linalg.inv(H))
    assert ea < 1e-5 and et < 1e-5


def test_degenerate_plane(oracle_mod):
    rng = rng_for(311)
    xy = rng.uniform(-1, 1, size=(2000, 2))
    pts = np.column_stack([xy, np.zeros(2000)]).astype(np.float32)
    n = np.tile(np.array([[0, 0, 1]], np.float32), (2000, 1))
    r = oracle_mod.icp(pts, pts, n, None, 0.1, 5)
    assert r["status"] == oracle_mod.ICP_DEGENERATE and r["iterations"] == 0
    assert np.array_equal(r["T"], np.eye(4))


def test_no_inliers_and_few_inliers(oracle_mod):
    pts = sphere_plane(rng_for(312), 500)
    n = _normals(oracle_mod, pts)
    far = pts + np.float32(10.0)
    r = oracle_mod.icp(far, pts, n, None, 0.1, 5)
    assert r["status"] == oracle_mod.ICP_NO_INLIERS and r["inliers"] == 0 and r["rms"] == 0.0
    r = oracle_mod.icp(np.vstack([far, pts[:4]]), pts, n, None, 0.1, 5)
    assert r["status"] == oracle_mod.ICP_DEGENERATE and r["iterations"] == 0


def test_zero_normals_are_rejected(oracle_mod):
    w = make_workload(0, size="small")
    n = _normals(oracle_mod, w.target)
    n0 = n.copy()
    n0[::3] = 0
    s = oracle_mod.p2plane_system(w.source, w.target, n0, np.eye(4), w.d_max)
    s_full = oracle_mod.p2plane_system(w.source, w.target, n, np.eye(4), w.d_max)
    assert s["inliers"] < s_full["inliers"]
    assert np.all(n0[s["corr"][s["corr"] >= 0]].any(axis=1))


def test_convergence_tolerance_stops_early(oracle_mod):
    w = make_workload(0, size="small")
    n = _normals(oracle_mod, w.target)
    r = oracle_mod.icp(w.source, w.target, n, None, w.d_max, 50, conv_tol=1e-9)
    assert r["status"] == oracle_mod.ICP_CONVERGED and r["iterations"] < 50
    assert np.abs(r["x_hist"][-1]).max() < 1e-9


@pytest.mark.parametrize("size", ["small"])
def test_kdtree_and_brute_systems_identical(oracle_mod, size):
    w = make_workload(1, size=size)
    n = _normals(oracle_mod, w.target, 16)
    for T in (np.eye(4), w.T_gt, random_rigid(rng_for(313), 2.0, 0.02) @ w.T_gt):
        a = oracle_mod.p2plane_system(w.source, w.target, n, T, w.d_max, method="brute")
        b = oracle_mod.p2plane_system(w.source, w.target, n, T, w.d_max, method="kdtree")
        assert np.array_equal(a["corr"], b["corr"])
        assert np.array_equal(a["A"], b["A"]) and np.array_equal(a["b"], b["b"])
