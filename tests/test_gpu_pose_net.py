"""GPU parity of the learned initialiser and of multi-start ICP through the
C ABI: the predicted pose against the oracle (float32 / bfloat16 matrix-core
arithmetic against float64 with the same bfloat16 roundings), the training
gradient against the oracle's dense gradient, the Adam update against its
formula, determinism, multi-start ICP against the oracle's 8-start
selection, and the consistency of the three initialisation modes."""
import math

import numpy as np
import pytest

from gen import POSE_CONFIG, pose_net_init, pose_pairs, random_rigid, rng_for
from oracle import pose_net as pn
from tests.helpers import pose_err, rot_angle

pytestmark = pytest.mark.gpu

# forward: both sides round the same activations and weights to bfloat16,
# but the GPU accumulates in float32 where the oracle uses float64 (relative
# error ~1e-6 in the features; observed up to 2e-6 rad in the rotation on
# the pairs of test_forward_matches_oracle): held to 10x the observed error
FWD_ROT_TOL = 2e-5
# an activation whose pre-activation lies within the float32 error of a
# bfloat16 rounding midpoint is rounded one way by the GPU and the other by
# the oracle; where that point carries a channel's maximum, the feature moves
# by a fraction of one bfloat16 step.  On 160 pairs of 1 to 2,600 points
# (test_encoder_tile_runs_match_single_pair_calls) 89-91 % of the poses
# agree within FWD_ROT_TOL and the rest within 1e-4 to 2e-4 rad: the bulk is
# held to FWD_ROT_TOL and every pair to 10x the worst such case
FLIP_ROT_TOL = 2e-3
FLIP_SHARE_MIN = 0.85
# gradient: float32 sums against float64 ones, observed up to 7e-6 relative
# L2 error per parameter tensor: held to about 10x that
GRAD_REL_TOL = 1e-4


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_00399_amd import pcgpu
    return pcgpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _say(*a):
    print(*a, flush=True)


def _uneven(sizes, seed):
    """Pairs of the learned-initialiser workload with the given sizes."""
    pairs = []
    for j, n in enumerate(sizes):
        pairs += pose_pairs(4, 1, n_points=n, first=seed + j).pairs
    return pairs


def _pack(pairs):
    src = np.ascontiguousarray(np.vstack([w.source for w in pairs]).astype(np.float32))
    tgt = np.ascontiguousarray(np.vstack([w.target for w in pairs]).astype(np.float32))
    off = np.concatenate([[0], np.cumsum([w.n for w in pairs])]).astype(np.int64)
    return src, tgt, off


def _params(seed):
    rng = np.random.default_rng(seed)
    p = pose_net_init(rng)
    # non-zero biases so that every ReLU sees both signs
    P = pn.unpack(p)
    for name in ("b1", "b2", "b3", "b4"):
        P[name][:] = (rng.standard_normal(P[name].size) * 0.1).astype(np.float32)
    return p


def test_forward_matches_oracle(gpu):
    pairs = _uneven([1, 127, 128, 129, 700, 4096], 100)
    params = _params(1)
    src, tgt, off = _pack(pairs)
    _say(f"forward sizes={[w.n for w in pairs]}")
    T = gpu.pose_net_predict(_dev(params), _dev(src), off, _dev(tgt), off).cpu().numpy()
    worst = 0.0
    for w, Tg in zip(pairs, T):
        To = pn.predict(params, w.source, w.target)
        ea = rot_angle(Tg[:3, :3], To[:3, :3])
        et = np.linalg.norm(Tg[:3, 3] - To[:3, 3])
        worst = max(worst, ea)
        assert np.allclose(Tg[3], [0, 0, 0, 1])
        assert ea < FWD_ROT_TOL, (w.name, w.n, ea)
        assert et < FWD_ROT_TOL * (1.0 + np.linalg.norm(w.source, axis=1).max()), (w.name, et)
    _say(f"forward worst rotation difference {worst:.3g} rad")


def test_forward_empty_cloud_and_zero_quaternion(gpu):
    pairs = _uneven([300, 200], 110)
    params = _params(2)
    src, tgt, _ = _pack(pairs)
    # pair 0 has an empty source: zero feature, centroid 0
    so = np.array([0, 0, 300 + 200], np.int64)
    to = np.array([0, 300, 500], np.int64)
    s2 = np.vstack([pairs[0].source, pairs[1].source]).astype(np.float32)
    t2 = np.vstack([pairs[0].target, pairs[1].target]).astype(np.float32)
    T = gpu.pose_net_predict(_dev(params), _dev(s2), so, _dev(t2), to).cpu().numpy()
    _, _, ct = pn.encode(params, t2[:300])
    ft = pn.encode(params, t2[:300])[0]
    R = pn.quat_to_R(pn.head(params, np.zeros(256), ft))
    # with a zero source feature the head's output is small, so the same
    # float32 error in it turns the normalised quaternion further (observed
    # 5.4e-5 rad): held to 2x that
    assert rot_angle(T[0][:3, :3], R) < 1e-4
    assert np.linalg.norm(T[0][:3, 3] - ct) < 1e-3
    # a zero head output gives the identity rotation
    z = params.copy()
    P = pn.unpack(z)
    P["W5"][:] = 0.0
    P["b5"][:] = 0.0
    T = gpu.pose_net_predict(_dev(z), _dev(src), np.array([0, 300, 500]), _dev(tgt),
                             np.array([0, 300, 500])).cpu().numpy()
    assert np.array_equal(T[0][:3, :3], np.eye(3)) and np.array_equal(T[1][:3, :3], np.eye(3))


def _train_case(seed):
    pairs = _uneven([300, 513, 129], seed)
    rng = rng_for(41, seed)
    labels = [random_rigid(rng, rng.uniform(0, 90), 0.1) for _ in pairs]
    return pairs, labels


def test_gradient_matches_oracle(gpu):
    import torch
    pairs, labels = _train_case(120)
    params = _params(3)
    w = np.array([1.0, 0.5, 2.0], np.float32)
    src, tgt, off = _pack(pairs)
    _say(f"gradient sizes={[p.n for p in pairs]}")
    loss, grad = gpu.pose_net_train_step(_dev(params), None, None, 1, 0.0, _dev(src), off, _dev(tgt), off,
                                         np.stack(labels), pair_weight=w, want_grad=True)
    torch.cuda.synchronize()
    L, g = pn.loss_and_grad(params, [(p.source, p.target) for p in pairs], labels, w)
    lg = loss.cpu().numpy().astype(np.float64)
    assert abs(lg.sum() - L) <= 1e-4 * L, (lg.sum(), L)
    gg = grad.cpu().numpy().astype(np.float64)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in pn.SHAPES])
    for (name, _), a, b in zip(pn.SHAPES, offs[:-1], offs[1:]):
        ref = np.linalg.norm(g[a:b])
        err = np.linalg.norm(gg[a:b] - g[a:b])
        _say(f"  {name}: |g| {ref:.4g}, relative error {err / max(ref, 1e-30):.3g}")
        assert err <= GRAD_REL_TOL * ref + 1e-9, (name, err, ref)


def _tile_run_case():
    # 160 pairs of 1 to 2,600 points: about 1,000 encoder tiles of 512
    # points, so each of the 256 workgroups takes a run of several tiles,
    # and clouds of up to 6 tiles straddle the runs' boundaries
    rng = np.random.default_rng(21)
    return _uneven(rng.integers(1, 2600, 160).tolist(), 600)


def test_encoder_tile_runs_match_single_pair_calls(gpu):
    # each pose of the batched call equals the pose of the same pair
    # predicted alone (one tile per workgroup there): the maxima are exact,
    # so how tiles are grouped into runs cannot change a bit; two empty
    # sources and two empty targets sit inside runs; every other pair
    # against the oracle (FLIP_ROT_TOL)
    pairs = _tile_run_case()
    params = _params(5)
    srcs = [w.source.astype(np.float32) for w in pairs]
    tgts = [w.target.astype(np.float32) for w in pairs]
    for j in (7, 90):
        srcs[j] = srcs[j][:0]
    for j in (8, 91):
        tgts[j] = tgts[j][:0]
    so = np.concatenate([[0], np.cumsum([len(a) for a in srcs])]).astype(np.int64)
    to = np.concatenate([[0], np.cumsum([len(a) for a in tgts])]).astype(np.int64)
    tiles = sum(-(-len(a) // 512) for a in srcs + tgts)
    _say(f"tile runs: pairs={len(pairs)} points={so[-1] + to[-1]} tiles={tiles}")
    assert tiles > 3 * 256
    P = _dev(params)
    T = gpu.pose_net_predict(P, _dev(np.vstack(srcs)), so, _dev(np.vstack(tgts)), to).cpu().numpy()
    for j in range(len(pairs)):
        Tj = gpu.pose_net_predict(P, _dev(srcs[j].reshape(-1, 3)), np.array([0, len(srcs[j])], np.int64),
                                  _dev(tgts[j].reshape(-1, 3)), np.array([0, len(tgts[j])], np.int64)).cpu().numpy()
        assert np.array_equal(T[j], Tj[0]), (j, len(srcs[j]), len(tgts[j]))
    errs = []
    for j, w in enumerate(pairs):
        if len(srcs[j]) and len(tgts[j]):
            To = pn.predict(params, w.source, w.target)
            errs.append(rot_angle(T[j][:3, :3], To[:3, :3]))
    errs = np.array(errs)
    share = float(np.mean(errs < FWD_ROT_TOL))
    _say(f"  against the oracle: {share:.3f} of {errs.size} pairs within {FWD_ROT_TOL}, worst {errs.max():.3g} rad")
    assert share >= FLIP_SHARE_MIN and errs.max() < FLIP_ROT_TOL, (share, errs.max())


def test_layout_over_many_clouds_matches_single_pair_calls(gpu):
    # 700 pairs (1,400 clouds): the device-side layout (rows and tile
    # offsets from the uploaded pair offsets) takes its prefix sum in two
    # chunks of 1,024 clouds; sampled poses, and the last pair's, against
    # the same pairs predicted alone, bit for bit
    rng = np.random.default_rng(23)
    pairs = _uneven(rng.integers(1, 300, 700).tolist(), 900)
    params = _dev(_params(7))
    src, tgt, off = _pack(pairs)
    _say(f"many clouds: pairs={len(pairs)} points={off[-1]}")
    T = gpu.pose_net_predict(params, _dev(src), off, _dev(tgt), off).cpu().numpy()
    for j in list(range(0, 700, 37)) + [510, 511, 512, 513, 699]:
        w = pairs[j]
        o = np.array([0, w.n], np.int64)
        Tj = gpu.pose_net_predict(params, _dev(w.source.astype(np.float32)), o, _dev(w.target.astype(np.float32)),
                                  o).cpu().numpy()
        assert np.array_equal(T[j], Tj[0]), (j, w.n)


def test_gradient_over_tile_runs_matches_single_pair_calls(gpu):
    # the training forward's arg-max over runs of several tiles per
    # workgroup (the case above): each pair's loss equals that of the pair
    # trained alone, bit for bit, and the batch's gradient equals the sum of
    # the single-pair gradients up to float32 summation order (a maximum
    # routed to a wrong point would move it by orders of magnitude more).
    # The single-pair path is the one test_gradient_matches_oracle checks
    # against the oracle.  Against the oracle directly this batch's first-
    # layer gradient differs by 1.6e-3 (one pair of 2,501 points by 12 %):
    # there a bfloat16 rounding decision or a near-tie moves a channel's
    # arg-max point, and the oracle's own gradient jumps the same way when
    # its inputs move by 1e-7 to 3e-6 relative (0.3 to 4 % for that pair;
    # for another, the GPU's 0.47 % exactly), so the oracle is not a
    # tighter reference than this at these sizes.
    import torch
    pairs = _tile_run_case()
    params = _dev(_params(6))
    labels = np.stack([random_rigid(rng_for(43, j), 60, 0.1) for j in range(len(pairs))])
    src, tgt, off = _pack(pairs)
    loss, grad = gpu.pose_net_train_step(params, None, None, 1, 0.0, _dev(src), off, _dev(tgt), off, labels,
                                         want_grad=True)
    loss, grad = loss.cpu().numpy(), grad.cpu().numpy().astype(np.float64)
    gsum = np.zeros_like(grad)
    for j, w in enumerate(pairs):
        o = np.array([0, w.n], np.int64)
        lj, gj = gpu.pose_net_train_step(params, None, None, 1, 0.0, _dev(w.source.astype(np.float32)), o,
                                         _dev(w.target.astype(np.float32)), o, labels[j:j + 1], want_grad=True)
        assert lj.cpu().numpy()[0] == loss[j], j
        gsum += gj.cpu().numpy()
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in pn.SHAPES])
    for (name, _), a, b in zip(pn.SHAPES, offs[:-1], offs[1:]):
        ref = np.linalg.norm(gsum[a:b])
        err = np.linalg.norm(grad[a:b] - gsum[a:b])
        _say(f"  {name}: |g| {ref:.4g}, batched against summed single-pair: relative {err / max(ref, 1e-30):.3g}")
        assert err <= 1e-5 * ref + 1e-9, (name, err, ref)


def test_adam_step_and_determinism(gpu):
    import torch
    pairs, labels = _train_case(130)
    params = _params(4)
    src, tgt, off = _pack(pairs)
    args = (_dev(src), off, _dev(tgt), off, np.stack(labels))
    p0 = _dev(params)
    l1, g1 = gpu.pose_net_train_step(p0, None, None, 1, 0.0, *args, want_grad=True)
    l2, g2 = gpu.pose_net_train_step(p0, None, None, 1, 0.0, *args, want_grad=True)
    assert torch.equal(l1, l2) and torch.equal(g1, g2)          # bitwise: no atomics
    assert torch.equal(p0.cpu(), torch.from_numpy(params))      # lr = 0 leaves params alone
    m = torch.zeros_like(p0)
    v = torch.zeros_like(p0)
    lr = 1e-3
    _, g = gpu.pose_net_train_step(p0, m, v, 1, lr, *args, want_grad=True)
    g = g.cpu().numpy().astype(np.float64) / len(pairs)
    # step 1 from zero moments: m_hat = g, v_hat = g^2
    want = params - lr * g / (np.abs(g) + 1e-8)
    got = p0.cpu().numpy()
    assert np.abs(got - want).max() <= 1e-6 * lr + 2e-7 * np.abs(params).max()
    assert np.allclose(m.cpu().numpy(), 0.1 * g, rtol=1e-5, atol=1e-12)
    assert np.allclose(v.cpu().numpy(), 0.001 * g * g, rtol=1e-4, atol=1e-20)


def test_training_reduces_the_loss(gpu):
    import torch
    pairs, labels = _train_case(140)
    params = _dev(_params(5))
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    src, tgt, off = _pack(pairs)
    args = (_dev(src), off, _dev(tgt), off, np.stack(labels))
    first = None
    for step in range(1, 61):
        loss, _ = gpu.pose_net_train_step(params, m, v, step, 1e-3, *args)
        if first is None:
            first = float(loss.sum())
    last = float(gpu.pose_net_train_step(params, None, None, 1, 0.0, *args)[0].sum())
    _say(f"loss {first:.4g} -> {last:.4g} after 60 steps")
    assert last < 0.5 * first


def _normals(oracle_mod, pairs):
    return np.ascontiguousarray(np.vstack([oracle_mod.normals(p.target, POSE_CONFIG["k"], (0, 0, 0))[0]
                                           for p in pairs]).astype(np.float32))


def test_multi_start_matches_oracle(gpu, oracle_mod):
    pairs = _uneven([1500, 1100, 1800], 150)
    src, tgt, off = _pack(pairs)
    nrm = _normals(oracle_mod, pairs)
    d, it = POSE_CONFIG["d_max"], POSE_CONFIG["iters"]
    _say(f"multi-start sizes={[p.n for p in pairs]}")
    T, st, start = gpu.icp_learned_batched(gpu.PC_INIT_MULTI_START, None, _dev(src), off, _dev(tgt), _dev(nrm), off,
                                           d, it)
    T, start = T.cpu().numpy(), start.cpu().numpy()
    for j, p in enumerate(pairs):
        tn = nrm[off[j]:off[j + 1]]
        dm = float(np.float32(d))
        runs = [oracle_mod.icp(p.source, p.target, tn, T0, dm, it) for T0 in pn.start_poses(p.source, p.target)]
        ro, bi = pn.multi_start_icp(oracle_mod, p.source, p.target, tn, dm, it)
        g = int(start[j])
        _say(f"  {p.name}: oracle start {bi} rms {ro['rms']:.3g}; gpu start {g} rms {st[j]['rms']:.3g}; "
             f"oracle rms per start {[round(r['rms'], 4) for r in runs]}")
        assert ro["rms"] < POSE_CONFIG["accept_rms"]          # the case has a converged start
        # several starts may reach the same optimum, their RMS equal up to
        # rounding: the pose is unique, the start index need not be
        ea, et = pose_err(runs[g]["T"], ro["T"])
        assert ea <= 1e-5 and et <= 1e-6, ("gpu start is not equivalent", g, bi, ea, et)
        ea, et = pose_err(T[j], ro["T"])
        assert ea <= 1e-5 and et <= 1e-6, (ea, et)
        assert st[j]["status"] == runs[g]["status"] and st[j]["iterations_run"] == runs[g]["iterations"]


def test_init_modes_are_consistent(gpu, oracle_mod):
    import torch
    pairs = _uneven([2000, 900, 1500, 1200], 160)
    src, tgt, off = _pack(pairs)
    nrm = _normals(oracle_mod, pairs)
    params = _dev(_params(6))
    S, Tt, N = _dev(src), _dev(tgt), _dev(nrm)
    d, it = POSE_CONFIG["d_max"], POSE_CONFIG["iters"]
    run = lambda mode, acc: gpu.icp_learned_batched(mode, params, S, off, Tt, N, off, d, it, accept_rms=acc,
                                                    read_stats=False)
    T2, s2, b2 = run(gpu.PC_INIT_LEARNED_ONLY, 0.0)
    T0 = gpu.pose_net_predict(params, S, off, Tt, off)
    Tb, sb = gpu.icp_point_to_plane_batched(S, off, Tt, N, off, init_T=T0, max_corr_dist=d, max_iters=it,
                                            read_stats=False)
    assert torch.equal(T2, Tb) and torch.equal(s2, sb) and bool((b2 == -1).all())
    Ta, sa, ba = run(gpu.PC_INIT_LEARNED, float("inf"))          # every learned result accepted
    assert torch.equal(Ta, T2) and torch.equal(sa, s2) and bool((ba == -1).all())
    Tm, sm, bm = run(gpu.PC_INIT_MULTI_START, 0.0)
    Tf, sf, bf = run(gpu.PC_INIT_LEARNED, -1.0)                  # every pair falls back
    assert torch.equal(Tf, Tm) and torch.equal(sf, sm) and torch.equal(bf, bm)
    assert bool((bm >= 0).all()) and bool((bm < 8).all())
    # the learned path keeps exactly the pairs whose refinement is accepted
    acc = float(np.median([r["rms"] for r in gpu.decode_stats_batched(s2)]))
    Tx, sx, bx = run(gpu.PC_INIT_LEARNED, acc)
    rec2 = gpu.decode_stats_batched(s2)
    for j in range(len(pairs)):
        kept = rec2[j]["status"] in (0, 1) and rec2[j]["inliers"] > 0 and rec2[j]["rms"] <= acc
        assert (int(bx[j]) == -1) == kept
        src_T = T2 if kept else Tm
        assert torch.equal(Tx[j], src_T[j])


def test_learned_pipeline_matches_oracle(gpu, oracle_mod):
    # trained weights on evaluation pairs: the same keep-or-fall-back
    # decision as the oracle's composition, and the same pose
    from paper_1807_00399_amd.train_pose_net import load_params
    pairs = pose_pairs(4, 6, n_points=2048).pairs
    params = load_params()
    src, tgt, off = _pack(pairs)
    nrm = _normals(oracle_mod, pairs)
    d, it, acc = POSE_CONFIG["d_max"], POSE_CONFIG["iters"], POSE_CONFIG["accept_rms"]
    T, st, start = gpu.icp_learned_batched(gpu.PC_INIT_LEARNED, _dev(params), _dev(src), off, _dev(tgt), _dev(nrm),
                                           off, d, it, accept_rms=acc)
    T, start = T.cpu().numpy(), start.cpu().numpy()
    kept = 0
    for j, p in enumerate(pairs):
        tn = nrm[off[j]:off[j + 1]]
        ro, bo = pn.learned_icp(oracle_mod, params, p.source, p.target, tn, float(np.float32(d)), it, acc)
        _say(f"  {p.name}: oracle start {bo} rms {ro['rms']:.3g}; gpu start {start[j]} rms {st[j]['rms']:.3g}")
        assert (start[j] == -1) == (bo == -1)
        kept += int(bo == -1)
        if bo == -1:
            ea, et = pose_err(T[j], ro["T"])
            assert ea <= 1e-5 and et <= 1e-6, (ea, et)
        elif ro["rms"] < acc:
            # multi-start: the pose is unique when a start converged
            ea, et = pose_err(T[j], ro["T"])
            assert ea <= 1e-5 and et <= 1e-6, (ea, et)
    _say(f"  learned start kept on {kept} of {len(pairs)} pairs")


def test_learned_full_workload_sampled(gpu, oracle_mod):
    # the benchmark's learned leg as it runs: all 512 pairs of 4096 points,
    # the targets' normals on the GPU, the learned start with 8-start
    # fallback, in the launch tuning the benchmark applies; sampled pairs
    # against the oracle's composition given the same normals
    import os
    import torch
    from paper_1807_00399_amd import autotune
    from paper_1807_00399_amd.train_pose_net import load_params
    cfg = POSE_CONFIG
    b = pose_pairs(cfg["eval_config"])
    off = b.offsets
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1807_00399_amd",
                        "tuning_cache.json")
    hit = autotune.load_cache(path).get(autotune.cache_key(autotune._device_name(None), "pose_pairs_512", b.n))
    params = load_params()
    d, it, acc = cfg["d_max"], cfg["iters"], cfg["accept_rms"]
    _say(f"full learned workload {b.name} pairs={b.n_pairs} n={b.n} tuned {hit and hit['tuning']}")
    src, tgt = _dev(b.source), _dev(b.target)
    try:
        if hit is not None:
            t = hit["tuning"]
            gpu.set_tuning(t["icp_block_threads"], t["icp_leaf"], t["node_budget"], t["sort_queries"],
                           t.get("icp_persistent", 0))
        nrm, _ = gpu.estimate_normals_batched(tgt, off, cfg["k"], curvature=False)
        T, st, start = gpu.icp_learned_batched(gpu.PC_INIT_LEARNED, torch.from_numpy(params).cuda(), src, off, tgt,
                                               nrm, off, d, it, accept_rms=acc)
    finally:
        gpu.set_tuning(128, 16, 1.0, 1)
    T, start, nrm = T.cpu().numpy(), start.cpu().numpy(), nrm.cpu().numpy()
    sample = sorted(np.random.default_rng(13).choice(b.n_pairs, 6, replace=False).tolist())
    for j in sample:
        p = b.pairs[j]
        ro, bo = pn.learned_icp(oracle_mod, params, p.source, p.target, nrm[off[j]:off[j + 1]], float(np.float32(d)),
                                it, acc)
        _say(f"  pair {j}: oracle start {bo} rms {ro['rms']:.3g}; gpu start {start[j]} rms {st[j]['rms']:.3g}")
        assert (start[j] == -1) == (bo == -1), j
        if bo == -1 or ro["rms"] < acc:
            ea, et = pose_err(T[j], ro["T"])
            assert ea <= 1e-5 and et <= 1e-6, (j, ea, et)
