"""Small numerical helpers shared by the tests (metrics only, no method code)."""
import numpy as np


def rot_angle(Ra, Rb):
    """Angle of Ra Rb^T: atan2(|vee(M - M^T)|/2, (tr M - 1)/2)."""
    M = np.asarray(Ra, np.float64) @ np.asarray(Rb, np.float64).T
    v = np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
    return float(np.arctan2(0.5 * np.linalg.norm(v), 0.5 * (np.trace(M) - 1.0)))


def pose_err(Ta, Tb):
    Ta, Tb = np.asarray(Ta), np.asarray(Tb)
    return rot_angle(Ta[:3, :3], Tb[:3, :3]), float(np.linalg.norm(Ta[:3, 3] - Tb[:3, 3]))


def angle_between(a, b):
    """Signed-orientation angle between rows of a and b: atan2(|a x b|, a.b)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=-1), np.sum(a * b, axis=-1))


def kabsch(p, q):
    """Least-squares rigid map p -> q (no scale) by SVD of the cross-covariance
    (Arun, Huang and Blostein 1987): H = sum (p - pbar)(q - qbar)^T = U S V^T,
    R = V diag(1, 1, sign det(V U^T)) U^T, t = qbar - R pbar."""
    p = np.asarray(p, np.float64)
    q = np.asarray(q, np.float64)
    pb, qb = p.mean(0), q.mean(0)
    H = (p - pb).T @ (q - qb)
    U, _, Vt = np.linalg.svd(H)
    d = np.sign(np.linalg.det(Vt.T @ U.T))
    R = Vt.T @ np.diag([1.0, 1.0, d]) @ U.T
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = qb - R @ pb
    return T
