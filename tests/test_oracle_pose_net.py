"""Pins for the oracle of the learned initialiser (CPU): the forward pass
against an explicit per-point loop, the bfloat16 rounding rule, the
quaternion map and start rotations against scipy, and multi-start selection
on a pair whose basins are known."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from gen import apply_rigid, random_rigid, rng_for, sphere_plane
from oracle import pose_net as pn
from tests.helpers import pose_err, rot_angle


def _params(seed):
    rng = np.random.default_rng(seed)
    out = []
    for name, shp in pn.SHAPES:
        fan_in = shp[0] if len(shp) == 2 else 1
        scale = math.sqrt(2.0 / fan_in) if name.startswith("W") else 0.1
        out.append((rng.standard_normal(int(np.prod(shp))) * scale).astype(np.float32))
    return np.concatenate(out)


def test_bf16_rounding_rule():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, 3.0 + 2 ** -7, -2.5, 0.0], np.float32)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert pn.bf16(x).tolist() == [1.0, 1.0, 1.0 + 2 ** -7, 3.0, -2.5, 0.0]   # ulp at 1 is 2^-7
    r = np.random.default_rng(1).standard_normal(10000).astype(np.float32)
    b = pn.bf16(r)
    assert np.all(np.abs(b - r) <= np.abs(r) * 2 ** -8 + 1e-38)
    assert np.all((b.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)


def test_encoder_matches_per_point_loop():
    params = _params(2)
    P = pn.unpack(params)
    pts = sphere_plane(rng_for(800), 300)
    f, arg, c = pn.encode(params, pts)
    x, c2, s = pn.normalise(pts)
    assert np.allclose(c, pts.astype(np.float64).mean(0)) and np.array_equal(c, c2)
    W2, W3 = pn.bf16(P["W2"]), pn.bf16(P["W3"])
    best = np.full(256, -1.0)
    bi = np.zeros(256, int)
    for i in range(len(x)):
        a1 = [max(0.0, sum(float(x[i, k]) * float(P["W1"][k, j]) for k in range(3)) + float(P["b1"][j]))
              for j in range(64)]
        a1 = pn.bf16(np.array(a1, np.float32))
        a2 = pn.bf16(np.maximum(a1 @ W2 + P["b2"], 0.0).astype(np.float32))
        a3 = np.maximum(a2 @ W3 + P["b3"], 0.0)
        up = a3 > best
        best[up] = a3[up]
        bi[up] = i
    assert np.allclose(f, best, rtol=1e-12, atol=1e-12) and np.array_equal(arg, bi)


def test_quaternion_map_and_start_rotations():
    rng = np.random.default_rng(3)
    for _ in range(20):
        q = rng.standard_normal(4)
        R = pn.quat_to_R(q)
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()      # scipy: (x, y, z, w)
        assert np.allclose(R, ref, atol=1e-14)
    rots = pn.start_rotations()
    assert len(rots) == 8 and np.array_equal(rots[0], np.eye(3))
    ax = pn.fibonacci_axes(7)
    assert np.allclose(np.linalg.norm(ax, axis=1), 1.0)
    for R, a in zip(rots[1:], ax):
        rv = Rotation.from_matrix(R).as_rotvec()
        assert abs(np.linalg.norm(rv) - math.radians(60)) < 1e-12
        assert np.allclose(rv / np.linalg.norm(rv), a, atol=1e-12)


def test_multi_start_picks_the_right_basin(oracle_mod):
    # an asymmetric room subsample turned by start rotation 3 and 8 degrees
    # more: the identity start is far outside the basin, start 3 inside it,
    # and the exact copy gives rms ~ 0 there
    from gen.scenes import room_scan
    rng = rng_for(801)
    pix = np.sort(rng.choice(640 * 480, size=4096, replace=False))
    src = room_scan(rng, pixels=pix)
    R = pn.axis_angle(rng.standard_normal(3), math.radians(8.0)) @ pn.start_rotations()[3]
    cs = src.astype(np.float64).mean(0)
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = cs - R @ cs + np.array([0.05, -0.02, 0.03])
    tgt = apply_rigid(T, src)
    nrm = oracle_mod.normals(tgt, 10, (0, 0, 0))[0].astype(np.float32)
    best, bi = pn.multi_start_icp(oracle_mod, src, tgt, nrm, 0.2, 40)
    assert bi == 3
    ea, et = pose_err(best["T"], T)
    assert ea < 1e-6 and et < 1e-6 and best["rms"] < 1e-5
    plain = oracle_mod.icp(src, tgt, nrm, pn.start_poses(src, tgt)[0], 0.2, 40)
    assert plain["rms"] > best["rms"] and rot_angle(plain["T"][:3, :3], T[:3, :3]) > 0.1


def _pair_set(seed, n=150, count=2):
    rng = rng_for(seed)
    out, labels = [], []
    for _ in range(count):
        src = sphere_plane(rng, n)
        T = random_rigid(rng, 40.0, 0.1)
        out.append((src, apply_rigid(T, src)))
        labels.append(T)
    return out, labels


def test_gradient_matches_finite_differences():
    params = _params(4).astype(np.float64)
    pairs, labels = _pair_set(802)
    w = [1.0, 0.5]
    L, g = pn.loss_and_grad(params, pairs, labels, w, round_bf16=False)
    assert L > 0.1
    rng = np.random.default_rng(5)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in pn.SHAPES])
    idx = []
    for a, b in zip(offs[:-1], offs[1:]):          # every tensor, largest |g| and random entries
        seg = np.abs(g[a:b])
        idx += [a + int(np.argmax(seg))] + list(a + rng.integers(0, b - a, 3))
    for i in idx:
        h = 1e-6 * max(1.0, abs(params[i]))
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (pn.loss_and_grad(pp, pairs, labels, w, round_bf16=False)[0] -
              pn.loss_and_grad(pm, pairs, labels, w, round_bf16=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-7, (i, fd, g[i])


def test_gradient_zero_weight_and_exact_label():
    params = _params(5)
    pairs, labels = _pair_set(803)
    L, g = pn.loss_and_grad(params, pairs, labels, [0.0, 0.0])
    assert L == 0.0 and not g.any()
    # the network's own prediction as the label: zero loss, zero gradient
    Rp = [pn.predict(params, s, t)[:3, :3] for s, t in pairs]
    L, g = pn.loss_and_grad(params, pairs, Rp)
    assert L < 1e-20 and np.abs(g).max() < 1e-8
    # loss value: the rotation angle theta between prediction and label gives 8 sin^2(theta / 2)
    lab = [pn.axis_angle([0, 0, 1], 0.7) @ R for R in Rp]
    L, _ = pn.loss_and_grad(params, pairs[:1], lab[:1])
    assert abs(L - 8 * math.sin(0.35) ** 2) < 1e-12


def test_learned_icp_keeps_or_falls_back(oracle_mod):
    # a zero head output predicts the identity rotation about the centroids:
    # on a pair turned by 5 degrees ICP converges from it (kept); turned by
    # start 3 and 8 degrees more it does not, and multi-start takes over
    from gen.scenes import room_scan
    rng = rng_for(804)
    pix = np.sort(rng.choice(640 * 480, size=3000, replace=False))
    src = room_scan(rng, pixels=pix)
    params = _params(6)
    P = pn.unpack(params)
    P["W5"][:] = 0.0
    P["b5"][:] = 0.0
    cs = src.astype(np.float64).mean(0)
    for R, kept in ((pn.axis_angle([0.3, 1.0, 0.2], math.radians(5.0)), True),
                    (pn.axis_angle(rng.standard_normal(3), math.radians(8.0)) @ pn.start_rotations()[3], False)):
        T = np.eye(4)
        T[:3, :3] = R
        T[:3, 3] = cs - R @ cs
        tgt = apply_rigid(T, src)
        nrm = oracle_mod.normals(tgt, 10, (0, 0, 0))[0].astype(np.float32)
        r, start = pn.learned_icp(oracle_mod, params, src, tgt, nrm, 0.3, 30, 0.004)
        assert (start == -1) == kept, start
        ea, et = pose_err(r["T"], T)
        assert ea < 1e-6 and et < 1e-6 and r["rms"] < 1e-5


def test_straight_through_gradient_matches_autograd():
    # The training gradient with the bfloat16 roundings in place: the forward
    # rounds a1, a2, W2 and W3 to bfloat16, the backward takes each rounding
    # as the identity.  torch's autograd (float64, CPU) computes the same
    # thing independently: every rounding written as v + (round(v) - v)
    # detached, the max-pool, ReLUs, head and quaternion loss written out.
    import torch
    params = _params(9)
    pairs = [(sphere_plane(rng_for(810, j), 200), sphere_plane(rng_for(811, j), 180)) for j in range(2)]
    labels = [random_rigid(rng_for(812, j), 40.0, 0.0) for j in range(2)]
    weights = [1.0, 0.5]
    L, g = pn.loss_and_grad(params, pairs, labels, weights, round_bf16=True)

    def rnd(v):
        # bfloat16 of the float32 value of v, held fixed by autograd
        r = torch.from_numpy(pn.bf16(v.detach().numpy().astype(np.float32)))
        return v + (r - v).detach()

    T = {}
    o = 0
    for name, shp in pn.SHAPES:
        n = int(np.prod(shp))
        T[name] = torch.tensor(params[o:o + n].astype(np.float64).reshape(shp), requires_grad=True)
        o += n
    total = torch.zeros((), dtype=torch.float64)
    for (src, tgt), lab, wgt in zip(pairs, labels, weights):
        feats = []
        for pts in (src, tgt):
            x = torch.from_numpy(pn.normalise(pts)[0].astype(np.float64))
            a1 = rnd(torch.relu(x @ T["W1"] + T["b1"]))
            a2 = rnd(torch.relu(a1 @ rnd(T["W2"]) + T["b2"]))
            a3 = torch.relu(a2 @ rnd(T["W3"]) + T["b3"])
            feats.append(a3.max(dim=0).values)
        h = torch.relu(torch.cat(feats) @ T["W4"] + T["b4"])
        q = h @ T["W5"] + T["b5"]
        w, xq, yq, zq = q / torch.linalg.norm(q)
        R = torch.stack([torch.stack([w * w + xq * xq - yq * yq - zq * zq, 2 * (xq * yq - w * zq),
                                      2 * (xq * zq + w * yq)]),
                         torch.stack([2 * (xq * yq + w * zq), w * w - xq * xq + yq * yq - zq * zq,
                                      2 * (yq * zq - w * xq)]),
                         torch.stack([2 * (xq * zq - w * yq), 2 * (yq * zq + w * xq),
                                      w * w - xq * xq - yq * yq + zq * zq])])
        total = total + wgt * torch.sum((R - torch.from_numpy(np.asarray(lab)[:3, :3])) ** 2)
    total.backward()
    ga = np.concatenate([T[name].grad.numpy().ravel() for name, _ in pn.SHAPES])
    assert abs(total.item() - L) <= 1e-12 * max(1.0, L)
    assert np.linalg.norm(ga - g) <= 1e-10 * np.linalg.norm(ga), np.linalg.norm(ga - g) / np.linalg.norm(ga)
    # and the roundings matter: the gradient without them differs
    _, g0 = pn.loss_and_grad(params, pairs, labels, weights, round_bf16=False)
    assert np.linalg.norm(g0 - g) > 1e-4 * np.linalg.norm(g)
