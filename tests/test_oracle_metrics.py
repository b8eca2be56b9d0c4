"""Pins for the oracle's point-to-point fit and ICP and its combined
(point-to-point + point-to-plane) metric (CPU).

The closed-form fit is held to Horn's quaternion method (a different
published solution of the same problem, via numpy's eigh), to exact motions,
to local optimality against nearby rotations and to its degenerate case; the
combined system to the point-to-plane system at weights (0, 1), to the
analytic point-to-point blocks at weights (1, 0), and to finite differences
of the weighted objective; both ICP loops to known transforms.
"""
import numpy as np
from scipy.spatial.transform import Rotation

from gen import apply_rigid, random_rigid, rng_for, sphere_plane
from tests.helpers import pose_err


def _horn(p, q):
    """Rotation maximising sum (q - qbar) . R (p - pbar) from the top
    eigenvector of Horn's 4x4 matrix (Horn 1987), and its two top
    eigenvalues."""
    p = p - p.mean(0)
    q = q - q.mean(0)
    S = p.T @ q
    Sxx, Sxy, Sxz = S[0]
    Syx, Syy, Syz = S[1]
    Szx, Szy, Szz = S[2]
    N = np.array([[Sxx + Syy + Szz, Syz - Szy, Szx - Sxz, Sxy - Syx],
                  [Syz - Szy, Sxx - Syy - Szz, Sxy + Syx, Szx + Sxz],
                  [Szx - Sxz, Sxy + Syx, -Sxx + Syy - Szz, Syz + Szy],
                  [Sxy - Syx, Szx + Sxz, Syz + Szy, -Sxx - Syy + Szz]])
    w, V = np.linalg.eigh(N)
    qw, qx, qy, qz = V[:, -1]
    R = Rotation.from_quat([qx, qy, qz, qw]).as_matrix()
    return R, w[-1], w[-1] - w[-2]


def test_rigid_fit_recovers_exact_motions(oracle_mod):
    rng = rng_for(400)
    for ang in (0.0, 1e-6, 5.0, 90.0, 179.0):
        p = rng.normal(size=(60, 3)) * rng.uniform(0.1, 10.0)
        T = random_rigid(rng, ang, 2.0)
        q = p @ T[:3, :3].T + T[:3, 3]
        R, t, top, gap = oracle_mod.rigid_fit(p, q)
        assert np.abs(R - T[:3, :3]).max() < 1e-12 * max(1.0, np.abs(p).max())
        assert np.abs(t - T[:3, 3]).max() < 1e-11 * max(1.0, np.abs(p).max())
        assert gap > 0


def test_rigid_fit_matches_horn_quaternion(oracle_mod):
    rng = rng_for(401)
    for _ in range(30):
        p = rng.normal(size=(40, 3))
        q = p @ Rotation.random(random_state=int(rng.integers(1 << 30))).as_matrix().T
        q += rng.normal(scale=0.3, size=q.shape) + rng.normal(size=3)
        R, t, top, gap = oracle_mod.rigid_fit(p, q)
        Rh, lam, lgap = _horn(p, q)
        assert np.abs(R - Rh).max() < 1e-10
        assert abs(top - lam) < 1e-10 * abs(lam) and abs(gap - lgap) < 1e-9 * abs(lam)
        assert abs(np.linalg.det(R) - 1.0) < 1e-12


def test_rigid_fit_reflection_gives_a_rotation(oracle_mod):
    # q is a mirror image of p: the best proper rotation, not the reflection
    rng = rng_for(402)
    p = rng.normal(size=(30, 3)) * np.array([3.0, 2.0, 0.2])
    q = p * np.array([1.0, 1.0, -1.0])
    R, t, top, gap = oracle_mod.rigid_fit(p, q)
    Rh, _, _ = _horn(p, q)
    assert abs(np.linalg.det(R) - 1.0) < 1e-12
    assert np.abs(R - Rh).max() < 1e-10


def test_rigid_fit_is_locally_optimal(oracle_mod):
    rng = rng_for(403)
    p = rng.normal(size=(50, 3))
    q = p @ random_rigid(rng, 30.0, 1.0)[:3, :3].T + rng.normal(scale=0.2, size=(50, 3))
    R, t, _, _ = oracle_mod.rigid_fit(p, q)

    def cost(Rx):
        tx = q.mean(0) - Rx @ p.mean(0)
        return np.sum((p @ Rx.T + tx - q) ** 2)

    c0 = cost(R)
    for _ in range(200):
        d = Rotation.from_rotvec(rng.normal(size=3) * 1e-3).as_matrix()
        assert cost(d @ R) >= c0 - 1e-12


def _near_line(rng, spread):
    """50 points on a unit-direction line through a, each moved off it by
    N(0, spread^2) per axis (float64, before any rounding)."""
    s = np.sort(rng.uniform(-1.0, 1.0, 50))
    d = np.array([0.6, -0.3, 0.74])
    d /= np.linalg.norm(d)
    return np.array([0.3, 1.1, 2.0]) + s[:, None] * d + rng.normal(size=(50, 3)) * spread, d


def test_p2p_degeneracy_threshold_is_where_float32_data_stop_fixing_the_rotation(oracle_mod):
    # The inputs are float32 points.  For a nearly collinear pair set the
    # rotation about the line is fixed only by the off-line spread, so the
    # float32 rounding of the inputs moves it by about 2^-24 / spread while
    # Horn's gap/top is about spread^2.  Two float32 roundings of the same
    # exact motion (the set moved along its own line by 3.3e-8 first) show
    # it, with numpy's eigh (Horn's method, independent of the oracle):
    # at gap/top ~ 1e-7 the rotation moves by more than the 1e-5 rad pose
    # tolerance (undetermined by the data: the loop must stop, DEGENERATE);
    # at gap/top ~ 1e-3 it is fixed well within it (the loop must step).
    # A threshold of 1e-12 would accept the first set and apply a rotation
    # that is rounding noise at the tolerance.
    rng = rng_for(404)
    for spread, undetermined in ((1e-4, True), (1e-2, False)):
        exact, d = _near_line(rng, spread)
        T = random_rigid(rng, 10.0, 0.2)
        Rs = []
        for shift in (0.0, 3.3e-8):
            e = exact + d * shift
            p = e.astype(np.float32).astype(np.float64)
            q = (e @ T[:3, :3].T + T[:3, 3]).astype(np.float32).astype(np.float64)
            R, lam, gap = _horn(p, q)
            Rs.append(R)
        moved = pose_err(np.block([[Rs[0], np.zeros((3, 1))], [np.zeros((1, 3)), 1.0]]),
                         np.block([[Rs[1], np.zeros((3, 1))], [np.zeros((1, 3)), 1.0]]))[0]
        src = exact.astype(np.float32)
        tgt = (exact @ T[:3, :3].T + T[:3, 3]).astype(np.float32)
        _, _, top, g = oracle_mod.rigid_fit(src.astype(np.float64), tgt.astype(np.float64))
        r = oracle_mod.icp_p2p(src, tgt, T, d_max=1.0, max_iters=1)
        if undetermined:
            assert 1e-12 < g / top < 1e-6 and moved > 1e-5, (g / top, moved)
            assert r["status"] == oracle_mod.ICP_DEGENERATE
        else:
            assert g / top > 1e-6 and moved < 1e-5, (g / top, moved)
            assert r["status"] == oracle_mod.ICP_MAXITER and r["iterations"] == 1


def test_rigid_fit_degenerate_when_collinear(oracle_mod):
    s = np.linspace(-1.0, 1.0, 20)[:, None]
    p = s * np.array([[1.0, 2.0, 0.5]])
    q = p + np.array([0.3, 0.0, 0.1])
    _, _, top, gap = oracle_mod.rigid_fit(p, q)
    assert gap <= 1e-12 * top
    p2 = np.vstack([p, [[0.0, 0.0, 1.0]]])           # one point off the line: unique again
    _, _, top, gap = oracle_mod.rigid_fit(p2, p2 + 0.1)
    assert gap > 1e-6 * top


def test_icp_p2p_one_step_from_exact_correspondences(oracle_mod):
    # a motion much smaller than the point spacing: every nearest neighbour
    # is the true partner, so the closed form lands on the motion at once
    rng = rng_for(404)
    src = (rng.uniform(-1.0, 1.0, size=(300, 3))).astype(np.float32)
    T = random_rigid(rng, 0.01, 1e-4)
    tgt = apply_rigid(T, src)
    r = oracle_mod.icp_p2p(src, tgt, None, 0.5, 1)
    assert r["status"] == oracle_mod.ICP_MAXITER and r["iterations"] == 1 and r["inliers"] == 300
    ea, et = pose_err(r["T"], T)
    assert ea < 1e-7 and et < 1e-7        # float32 rounding of the target


def test_icp_p2p_converges_to_ground_truth(oracle_mod):
    rng = rng_for(405)
    src = sphere_plane(rng, 3000)
    T = random_rigid(rng, 6.0, 0.05)
    tgt = apply_rigid(T, src)
    r = oracle_mod.icp_p2p(src, tgt, None, 0.3, 60, conv_tol=1e-12)
    ea, et = pose_err(r["T"], T)
    assert ea < 1e-6 and et < 1e-6 and r["inliers"] == 3000
    # fewer than 3 inliers: degenerate, pose kept
    far = random_rigid(rng, 0.0, 10.0)
    r2 = oracle_mod.icp_p2p(src[:2], apply_rigid(far, src[:2]), None, 30.0, 5)
    assert r2["status"] == oracle_mod.ICP_DEGENERATE and r2["iterations"] == 0
    assert np.array_equal(r2["T"], np.eye(4))


def _cloud(oracle_mod, seed):
    rng = rng_for(seed)
    src = sphere_plane(rng, 1500)
    T = random_rigid(rng, 4.0, 0.03)
    tgt = apply_rigid(T, src)
    nrm = oracle_mod.normals(tgt, 10, (0, 0, 0))[0].astype(np.float32)
    return rng, src, tgt, nrm, T


def test_combined_system_reduces_to_point_to_plane(oracle_mod):
    rng, src, tgt, nrm, _ = _cloud(oracle_mod, 406)
    T0 = random_rigid(rng, 1.0, 0.01)
    A, b, inl, s2 = oracle_mod.combined_system(src, tgt, nrm, T0, 0.2, 0.0, 1.0)
    ref = oracle_mod.p2plane_system(src, tgt, nrm, T0, 0.2, method="brute")
    assert inl == ref["inliers"] and s2 == ref["sum_r2"]
    assert np.array_equal(A, ref["A"]) and np.array_equal(b, ref["b"])


def test_combined_system_point_blocks(oracle_mod):
    # at weights (1, 0): A = sum [[|p|^2 I - p p^T, [p]x], [-[p]x, I]] and
    # b = sum [p x r; r] with r = p' - q, written here from the block formula
    rng, src, tgt, nrm, _ = _cloud(oracle_mod, 407)
    T0 = random_rigid(rng, 1.0, 0.01)
    A, b, inl, s2 = oracle_mod.combined_system(src, tgt, nrm, T0, 0.2, 1.0, 0.0)
    p = src.astype(np.float64) @ T0[:3, :3].T + T0[:3, 3]
    _, idx = __import__("scipy.spatial", fromlist=["cKDTree"]).cKDTree(tgt.astype(np.float64)).query(p)
    q = tgt.astype(np.float64)[idx]
    keep = np.sum((p - q) ** 2, axis=1) <= 0.2 ** 2
    p, q = p[keep], q[keep]
    r = p - q
    Aref = np.zeros((6, 6))
    bref = np.zeros(6)
    for pi, ri in zip(p, r):
        X = np.array([[0, -pi[2], pi[1]], [pi[2], 0, -pi[0]], [-pi[1], pi[0], 0]])
        Aref[:3, :3] += pi @ pi * np.eye(3) - np.outer(pi, pi)
        Aref[:3, 3:] += X
        Aref[3:, :3] -= X
        Aref[3:, 3:] += np.eye(3)
        bref[:3] += np.cross(pi, ri)
        bref[3:] += ri
    assert inl == keep.sum()
    assert np.allclose(A, Aref, rtol=1e-12, atol=1e-9) and np.allclose(b, bref, rtol=1e-12, atol=1e-9)
    assert np.isclose(s2, np.sum(r * r), rtol=1e-12)


def test_combined_system_gradient_by_finite_differences(oracle_mod):
    # with the correspondences fixed, the weighted objective f(x) at the
    # moved points p'' = Rz Ry Rx p' + tau has gradient 2 b at x = 0
    rng, src, tgt, nrm, _ = _cloud(oracle_mod, 408)
    wpt, wpl = 0.4, 1.3
    A, b, inl, s2 = oracle_mod.combined_system(src, tgt, nrm, np.eye(4), 0.2, wpt, wpl)
    p = src.astype(np.float64)
    d2, idx = __import__("scipy.spatial", fromlist=["cKDTree"]).cKDTree(tgt.astype(np.float64)).query(p)
    keep = d2 <= 0.2
    p, q, n = p[keep], tgt.astype(np.float64)[idx[keep]], nrm.astype(np.float64)[idx[keep]]

    def f(x):
        R = Rotation.from_euler("ZYX", [x[2], x[1], x[0]]).as_matrix()
        pp = p @ R.T + x[3:]
        e = pp - q
        return wpl * np.sum(np.sum(e * n, axis=1) ** 2) + wpt * np.sum(e * e)

    assert np.isclose(f(np.zeros(6)), s2, rtol=1e-12)
    h = 1e-6
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        g = (f(e) - f(-e)) / (2 * h)
        assert abs(g - 2 * b[k]) <= 1e-5 * max(1.0, abs(2 * b[k])), (k, g, 2 * b[k])


def test_icp_combined_recovers_transforms(oracle_mod):
    rng, src, tgt, nrm, T = _cloud(oracle_mod, 409)
    for wpt, wpl in ((0.0, 1.0), (0.5, 1.0), (1.0, 0.0), (2.0, 0.3)):
        r = oracle_mod.icp_combined(src, tgt, nrm, None, wpt, wpl, 0.2, 40, conv_tol=1e-13)
        ea, et = pose_err(r["T"], T)
        assert ea < 1e-7 and et < 1e-7, (wpt, wpl, ea, et)
    # weights (0, 1) are the point-to-plane loop itself
    a = oracle_mod.icp_combined(src, tgt, nrm, None, 0.0, 1.0, 0.2, 7)
    b = oracle_mod.icp(src, tgt, nrm, None, 0.2, 7)
    assert np.array_equal(a["T"], b["T"]) and a["inliers"] == b["inliers"] and a["rms"] == b["rms"]
