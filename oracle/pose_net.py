"""CPU oracle of the learned pose initialiser and of multi-start ICP.

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers; the GPU library never
imports it.

Neither the encoder nor the multi-start rule comes from the paper (its ICP
starts from one given pose, Section 3); they are this build's readings of an
initialiser in front of the paper's ICP:

  * encoder (per cloud): points are centred on their centroid and scaled by
    the inverse RMS distance to it; per point x -> ReLU(W1^T x + b1) (64)
    -> ReLU(W2^T . + b2) (128) -> ReLU(W3^T . + b3) (256); the cloud's
    feature is the per-channel maximum over its points.  The activations that
    feed the second and third layers are rounded to bfloat16, as are W2 and
    W3 (the GPU runs those two layers on bfloat16 matrix cores with float32
    accumulation); everything else is float64 here.
  * head (per pair): h = ReLU(W4^T [f_src; f_tgt] + b4) (256),
    q = W5^T h + b5 (4), the unit quaternion q / |q| (w, x, y, z) is the
    rotation R; the initial pose is T0 = [R, c_tgt - R c_src] with c the
    centroids.
  * training loss of a pair: |R(q) - R_label|_F^2, weighted per pair and
    summed; its gradient (loss_and_grad) is the dense chain rule over every
    point of every cloud, with the bfloat16 roundings taken as the identity
    (straight-through) and the rounded W2, W3 standing in for W2, W3.
  * learned registration: ICP from the predicted pose; a result counts as
    accepted when its status is converged or max-iterations, it has inliers
    and its RMS is at most the accepted RMS; otherwise multi-start ICP
    decides.
  * multi-start ICP: point-to-plane ICP (oracle.icp) from the identity
    rotation and from 7 rotations of 60 degrees about Fibonacci-sphere axes,
    each about the source centroid onto the target centroid; the result with
    the smallest final RMS is kept (ties: the lower start index).

Pinned in tests/test_oracle_pose_net.py: the forward against an explicit
per-point loop, the rounding rule, the quaternion map against scipy, the
start rotations' angles and axes, multi-start selection on pairs whose
basins are known, and the gradient (without rounding) against central
finite differences of the loss.
"""
from __future__ import annotations

import math

import numpy as np

C1, C2, C3, H = 64, 128, 256, 256
SHAPES = (("W1", (3, C1)), ("b1", (C1,)), ("W2", (C1, C2)), ("b2", (C2,)), ("W3", (C2, C3)), ("b3", (C3,)),
          ("W4", (2 * C3, H)), ("b4", (H,)), ("W5", (H, 4)), ("b5", (4,)))


def param_count() -> int:
    return int(sum(np.prod(s) for _, s in SHAPES))


def unpack(flat):
    """Named views of the flat float32 parameter vector (row-major, in SHAPES order)."""
    flat = np.asarray(flat)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = flat[o:o + n].reshape(shp)
        o += n
    assert o == flat.size
    return out


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def normalise(pts):
    """(centred and scaled points (float32), centroid (float64), scale)."""
    p = np.asarray(pts, dtype=np.float64)
    c = p.mean(axis=0)
    d = p - c
    rms = math.sqrt(float(np.mean(np.sum(d * d, axis=1))))
    s = 1.0 / rms if rms > 0 else 1.0
    return (d * s).astype(np.float32), c, s


def encode(params, pts):
    """(feature (256,), argmax point index per channel (256,), centroid)."""
    P = unpack(params)
    x, c, _ = normalise(pts)
    x = x.astype(np.float64)
    a1 = np.maximum(x @ P["W1"].astype(np.float64) + P["b1"], 0.0)
    a1 = bf16(a1.astype(np.float32))
    a2 = np.maximum(a1 @ bf16(P["W2"]) + P["b2"], 0.0)
    a2 = bf16(a2.astype(np.float32))
    a3 = np.maximum(a2 @ bf16(P["W3"]) + P["b3"], 0.0)
    return a3.max(axis=0), a3.argmax(axis=0), c


def _encoder(P, pts, round_bf16=True):
    """Per-point activations of one cloud (float64): x, pre-activations
    z1..z3, activations a1..a3, the weights used for layers 2, 3, the
    feature and arg-max."""
    rnd = bf16 if round_bf16 else (lambda v: np.asarray(v, np.float64))
    x, c, _ = normalise(pts)
    x = x.astype(np.float64)
    W2 = rnd(P["W2"])
    W3 = rnd(P["W3"])
    z1 = x @ np.asarray(P["W1"], np.float64) + P["b1"]
    a1 = rnd(np.maximum(z1, 0.0).astype(np.float32)) if round_bf16 else np.maximum(z1, 0.0)
    z2 = a1 @ W2 + P["b2"]
    a2 = rnd(np.maximum(z2, 0.0).astype(np.float32)) if round_bf16 else np.maximum(z2, 0.0)
    z3 = a2 @ W3 + P["b3"]
    a3 = np.maximum(z3, 0.0)
    return dict(x=x, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, W2=W2, W3=W3, f=a3.max(axis=0),
                arg=a3.argmax(axis=0), c=c)


def _quat_loss_grad(q, R_label):
    """|R(q/|q|) - R_label|_F^2 and its gradient in q, from
    R(u) = (w^2 - v.v) I + 2 v v^T + 2 w [v]_x with u = (w, v)."""
    q = np.asarray(q, np.float64)
    nq = np.linalg.norm(q)
    if not nq > 0:
        return 0.0, np.zeros(4)
    u = q / nq
    w, v = u[0], u[1:]
    D = 2.0 * (quat_to_R(u) - R_label)          # dL/dR
    L = float(np.sum((quat_to_R(u) - R_label) ** 2))
    cross = np.array([D[2, 1] - D[1, 2], D[0, 2] - D[2, 0], D[1, 0] - D[0, 1]])
    du = np.empty(4)
    du[0] = 2.0 * w * np.trace(D) + 2.0 * (v @ cross)
    du[1:] = -2.0 * v * np.trace(D) + 2.0 * (D + D.T) @ v + 2.0 * w * cross
    return L, (du - u * (u @ du)) / nq


def loss_and_grad(params, pairs, labels, weights=None, round_bf16=True):
    """Sum over pairs of weight * |R(q) - R_label|^2 and its gradient in the
    flat parameters.  pairs: list of (src, tgt) point arrays; labels: 3x3
    rotations (or 4x4 poses); weights: per pair, default 1."""
    params = np.asarray(params)
    P = unpack(params.astype(np.float64))
    G = {k: np.zeros_like(v, dtype=np.float64) for k, v in P.items()}
    total = 0.0
    for p, (src, tgt) in enumerate(pairs):
        wgt = 1.0 if weights is None else float(weights[p])
        if wgt == 0.0:
            continue
        enc = [_encoder(P, src, round_bf16), _encoder(P, tgt, round_bf16)]
        fcat = np.concatenate([enc[0]["f"], enc[1]["f"]])
        z4 = fcat @ P["W4"] + P["b4"]
        h = np.maximum(z4, 0.0)
        q = h @ P["W5"] + P["b5"]
        L, dq = _quat_loss_grad(q, np.asarray(labels[p], np.float64)[:3, :3])
        total += wgt * L
        dq = wgt * dq
        G["W5"] += np.outer(h, dq)
        G["b5"] += dq
        dz4 = (P["W5"] @ dq) * (z4 > 0)
        G["W4"] += np.outer(fcat, dz4)
        G["b4"] += dz4
        dfcat = P["W4"] @ dz4
        for side, e in enumerate(enc):
            df = dfcat[side * C3:(side + 1) * C3]
            dz3 = np.zeros_like(e["z3"])
            cols = np.arange(C3)
            dz3[e["arg"], cols] = np.where(e["f"] > 0, df, 0.0)
            G["W3"] += e["a2"].T @ dz3
            G["b3"] += dz3.sum(axis=0)
            dz2 = (dz3 @ e["W3"].T) * (e["z2"] > 0)
            G["W2"] += e["a1"].T @ dz2
            G["b2"] += dz2.sum(axis=0)
            dz1 = (dz2 @ e["W2"].T) * (e["z1"] > 0)
            G["W1"] += e["x"].T @ dz1
            G["b1"] += dz1.sum(axis=0)
    return total, np.concatenate([G[name].ravel() for name, _ in SHAPES])


def quat_to_R(q):
    """Rotation of the unit quaternion q / |q| (w, x, y, z); q = 0 gives the identity."""
    q = np.asarray(q, np.float64)
    nq = np.linalg.norm(q)
    if not nq > 0:
        return np.eye(3)
    w, x, y, z = q / nq
    return np.array([[w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z]])


def head(params, f_src, f_tgt):
    P = unpack(params)
    h = np.maximum(np.concatenate([f_src, f_tgt]) @ P["W4"].astype(np.float64) + P["b4"], 0.0)
    return h @ P["W5"].astype(np.float64) + P["b5"]


def predict(params, src, tgt):
    """Initial pose T0 (4x4 float64) of one pair."""
    fs, _, cs = encode(params, src)
    ft, _, ct = encode(params, tgt)
    R = quat_to_R(head(params, fs, ft))
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = ct - R @ cs
    return T


def fibonacci_axes(n: int = 7):
    """n unit axes on the Fibonacci sphere: z_i = 1 - (2i + 1)/n, azimuth i * golden angle."""
    g = math.pi * (3.0 - math.sqrt(5.0))
    out = []
    for i in range(n):
        z = 1.0 - (2.0 * i + 1.0) / n
        r = math.sqrt(max(0.0, 1.0 - z * z))
        out.append((r * math.cos(i * g), r * math.sin(i * g), z))
    return np.array(out)


def axis_angle(axis, angle):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def start_rotations():
    """Identity and 7 rotations of 60 degrees about the Fibonacci axes."""
    return [np.eye(3)] + [axis_angle(a, math.radians(60.0)) for a in fibonacci_axes(7)]


def start_poses(src, tgt):
    cs = np.asarray(src, np.float64).mean(axis=0)
    ct = np.asarray(tgt, np.float64).mean(axis=0)
    out = []
    for R in start_rotations():
        T = np.eye(4)
        T[:3, :3] = R
        T[:3, 3] = ct - R @ cs
        out.append(T)
    return out


def multi_start_icp(oracle_mod, src, tgt, tgt_normals, d_max, iters):
    """Best of the 8 starts by final RMS (ties: lower start).  Returns
    (result dict of oracle.icp, start index)."""
    best, bi = None, -1
    for i, T0 in enumerate(start_poses(src, tgt)):
        r = oracle_mod.icp(src, tgt, tgt_normals, T0, d_max, iters)
        if best is None or (r["inliers"] > 0 and (best["inliers"] == 0 or r["rms"] < best["rms"])):
            best, bi = r, i
    return best, bi


def learned_icp(oracle_mod, params, src, tgt, tgt_normals, d_max, iters, accept_rms):
    """(result dict, start index: -1 = the learned start was kept)."""
    r = oracle_mod.icp(src, tgt, tgt_normals, predict(params, src, tgt), d_max, iters)
    ok = r["status"] in (oracle_mod.ICP_CONVERGED, oracle_mod.ICP_MAXITER) and r["inliers"] > 0
    if ok and r["rms"] <= accept_rms:
        return r, -1
    return multi_start_icp(oracle_mod, src, tgt, tgt_normals, d_max, iters)
