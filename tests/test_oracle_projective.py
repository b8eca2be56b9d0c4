"""Pins for the oracle's projective data association and its ICP loop (CPU).

Pixels are checked by round trips of back-projected pixels (a pinhole
camera maps its own depth image back to itself), by the rounding rule at
half-pixel boundaries and by the rejection cases; the loop by the identity
on a frame and itself and by recovery of a known camera motion from
noiseless views (projective association is exact only in the limit, so the
recovery bound shrinks with the image size)."""
import numpy as np

from gen.scenes import room_views, rng_for
from tests.helpers import pose_err


def test_pixels_round_trip(oracle_mod):
    _, tgt, _, K = room_views(rng_for(600), 160, 120, depth_noise=0.0)
    pix = oracle_mod.projective_pixels(tgt, 160, 120, K, np.eye(4))
    assert np.array_equal(pix, np.arange(160 * 120))


def test_pixels_rounding_and_rejection(oracle_mod):
    # fx = fy = 1, cx = cy = 0: u = x / z exactly for these values
    K = (1.0, 1.0, 0.0, 0.0)
    pts = np.array([[2.5, 0.0, 1.0],      # u = 2.5 -> pixel 3
                    [2.4999, 1.0, 1.0],   # u < 2.5 -> 2, v = 1
                    [-0.5, 0.0, 1.0],     # u = -0.5 -> floor(0) = 0, inside
                    [-0.5001, 0.0, 1.0],  # -> -1, outside
                    [3.5, 0.0, 1.0],      # u = 3.5 -> 4 = width: outside
                    [1.0, 1.0, -1.0],     # behind the camera
                    [1.0, 1.0, 0.0],      # on the camera plane
                    [1.0, 2.25, 0.5]],    # u = 2, v = 4.5 -> 5: outside (height 5)
                   np.float32)
    pix = oracle_mod.projective_pixels(pts, 4, 5, K, np.eye(4))
    assert pix.tolist() == [3, 4 + 2, 0, -1, -1, -1, -1, -1]
    # the pose is applied first: a translation moves the point by whole pixels
    T = np.eye(4)
    T[0, 3] = 1.0
    assert oracle_mod.projective_pixels(pts[:1], 4, 5, K, T).tolist() == [-1]      # u = 3.5
    T[0, 3] = -1.0
    assert oracle_mod.projective_pixels(pts[:1], 4, 5, K, T).tolist() == [2]       # u = 1.5 -> 2


def test_icp_identity_on_a_frame_and_itself(oracle_mod):
    _, tgt, _, K = room_views(rng_for(601), 160, 120)
    nrm = oracle_mod.normals(tgt, 16, (0, 0, 0))[0].astype(np.float32)
    r = oracle_mod.icp_projective(tgt, tgt, nrm, 160, 120, K, None, 0.05, 3)
    assert np.array_equal(r["T"], np.eye(4))
    assert r["inliers"] == int(np.any(nrm != 0, axis=1).sum()) and r["rms"] == 0.0


def test_icp_invalid_pixels_are_skipped(oracle_mod):
    src, tgt, C, K = room_views(rng_for(602), 160, 120, depth_noise=0.0)
    nrm = oracle_mod.normals(tgt, 16, (0, 0, 0))[0].astype(np.float32)
    bad = tgt.copy()
    bad[::3] = np.nan                      # every third pixel invalid
    a = oracle_mod.icp_projective(src, bad, nrm, 160, 120, K, None, 0.2, 1)
    good = oracle_mod.icp_projective(src, tgt, nrm, 160, 120, K, None, 0.2, 1)
    assert 0 < a["inliers"] < good["inliers"]
    zero = tgt.copy()
    zero[:, 2] = 0.0                       # z = 0 everywhere: no valid pixel
    z = oracle_mod.icp_projective(src, zero, nrm, 160, 120, K, None, 0.2, 4)
    assert z["status"] == oracle_mod.ICP_NO_INLIERS and z["iterations"] == 0


def test_icp_recovers_camera_motion_from_noiseless_views(oracle_mod):
    src, tgt, C, K = room_views(rng_for(603), 320, 240, 3.0, 0.03, depth_noise=0.0)
    nrm = oracle_mod.normals(tgt, 16, (0, 0, 0))[0].astype(np.float32)
    r = oracle_mod.icp_projective(src, tgt, nrm, 320, 240, K, None, 0.2, 30)
    ea, et = pose_err(r["T"], C)
    assert ea < 2e-4 and et < 1e-3, (ea, et)        # from 0.052 rad / 0.03
