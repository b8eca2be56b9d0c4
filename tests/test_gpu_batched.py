"""GPU parity of the batched entry points (many uneven clouds / pairs in one
call) through the C ABI.

Every cloud and pair of a batch is computed exactly as the single form
computes it alone, so the batched results must equal the single-call results
bit for bit; the single calls are themselves held to the oracle elsewhere,
and here the oracle is also run directly on each small pair (normals within
1e-5 rad on well-conditioned points, pose within 1e-5 rad / 1e-6)."""
import numpy as np
import pytest

from gen import batch_workload, sphere_plane, rng_for, random_rigid, apply_rigid
from tests.helpers import angle_between, pose_err

pytestmark = pytest.mark.gpu

ROT_TOL = 1e-5
TRANS_TOL = 1e-6
NORMAL_TOL_RAD = 1e-5
GAP_GATE = 1e-3


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


@pytest.fixture(scope="module")
def small_batch():
    return batch_workload(3, "small")


def _batched_normals(gpu, b):
    off = b.offsets
    n, c = gpu.estimate_normals_batched(_dev(b.target), off, b.param("k").astype(np.int32))
    return n.cpu().numpy(), c.cpu().numpy()


def test_batched_normals_equal_single_and_oracle(gpu, oracle_mod, small_batch):
    b = small_batch
    _say(f"batched normals {b.name} pairs={b.n_pairs} n={b.n}")
    bn, bc = _batched_normals(gpu, b)
    off = b.offsets
    for j, w in enumerate(b.pairs):
        sn, sc = gpu.estimate_normals(_dev(w.target), w.k)
        sn, sc = sn.cpu().numpy(), sc.cpu().numpy()
        assert np.array_equal(bn[off[j]:off[j + 1]], sn), f"pair {j}: normals differ from the single call"
        assert np.array_equal(bc[off[j]:off[j + 1]], sc), f"pair {j}: curvature differs from the single call"
        en, ec, ev = oracle_mod.normals(w.target, w.k, (0.0, 0.0, 0.0), method="kdtree")
        gate = (ev[:, 1] - ev[:, 0]) >= GAP_GATE * ev[:, 2]
        zero = ~np.any(en != 0, axis=1)
        ang = angle_between(sn.astype(np.float64), en)
        g = gate & ~zero
        assert (float(ang[g].max()) if g.any() else 0.0) <= NORMAL_TOL_RAD, f"pair {j}"


def _single_icp(gpu, w, nrm, T0=None, d_max=None, iters=None):
    T, st = gpu.icp_point_to_plane(_dev(w.source), _dev(w.target), _dev(nrm), T0,
                                   w.d_max if d_max is None else d_max, w.iters if iters is None else iters)
    return T.cpu().numpy(), st


def test_batched_icp_equal_single_and_oracle(gpu, oracle_mod, small_batch):
    b = small_batch
    off = b.offsets
    # the same target normals on every side: the oracle's, in float32
    nrms = [oracle_mod.normals(w.target, w.k, (0, 0, 0))[0].astype(np.float32) for w in b.pairs]
    _say(f"batched icp {b.name} pairs={b.n_pairs}")
    T, stats = gpu.icp_point_to_plane_batched(_dev(b.source), off, _dev(b.target), _dev(np.vstack(nrms)), off,
                                              None, b.param("d_max").astype(np.float32),
                                              b.param("iters").astype(np.int32))
    T = T.cpu().numpy()
    for j, w in enumerate(b.pairs):
        Ts, ss = _single_icp(gpu, w, nrms[j])
        assert np.array_equal(T[j], Ts), f"pair {j}: pose differs from the single call"
        assert stats[j] == ss, (j, stats[j], ss)
        ro = oracle_mod.icp(w.source, w.target, nrms[j], None, float(np.float32(w.d_max)), w.iters)
        ea, et = pose_err(T[j], ro["T"])
        assert ea <= ROT_TOL and et <= TRANS_TOL, f"pair {j}: {ea:.3g} rad, {et:.3g}"
        assert stats[j]["status"] == ro["status"] and stats[j]["iterations_run"] == ro["iterations"]


def test_batched_icp_with_normals_equal_single_and_oracle(gpu, oracle_mod, small_batch):
    """One pyramid for the targets' normals and the registrations: every
    pair's pose, statistics and normals equal the single fused call's; the
    pose is held to the oracle run on the GPU's own normals."""
    import torch
    b = small_batch
    off = b.offsets
    _say(f"batched icp with normals {b.name} pairs={b.n_pairs}")
    nrm = torch.empty((b.target.shape[0], 3), dtype=torch.float32, device="cuda")
    T, stats = gpu.icp_point_to_plane_with_normals_batched(_dev(b.source), off, _dev(b.target), off,
                                                           b.param("k").astype(np.int32), (0.0, 0.0, 0.0), None,
                                                           b.param("d_max").astype(np.float32),
                                                           b.param("iters").astype(np.int32), out_normals=nrm)
    T, nrm = T.cpu().numpy(), nrm.cpu().numpy()
    for j, w in enumerate(b.pairs):
        Ts, ss, ns = gpu.icp_point_to_plane_with_normals(_dev(w.source), _dev(w.target), w.k, (0.0, 0.0, 0.0), None,
                                                         w.d_max, w.iters, return_normals=True)
        assert np.array_equal(T[j], Ts.cpu().numpy()), f"pair {j}: pose differs from the single call"
        assert stats[j] == ss, (j, stats[j], ss)
        assert np.array_equal(nrm[off[j]:off[j + 1]], ns.cpu().numpy()), f"pair {j}: normals differ"
        ro = oracle_mod.icp(w.source, w.target, nrm[off[j]:off[j + 1]], None, float(np.float32(w.d_max)), w.iters)
        ea, et = pose_err(T[j], ro["T"])
        assert ea <= ROT_TOL and et <= TRANS_TOL, f"pair {j}: {ea:.3g} rad, {et:.3g}"
        assert stats[j]["inliers"] == ro["inliers"]


def test_batched_icp_edge_pairs(gpu, oracle_mod):
    # a normal pair, an empty source, an empty target, a pair with no
    # iterations, a tiny pair and a pair with its own d_max and init pose
    rng = rng_for(99, 0)
    a = sphere_plane(rng, 1500)
    Ta = random_rigid(rng, 8.0, 0.03)
    c = sphere_plane(rng, 900)
    Tc = random_rigid(rng, 6.0, 0.02)
    tiny = sphere_plane(rng, 7)
    Ti = random_rigid(rng, 2.0, 0.01)
    empty = np.zeros((0, 3), np.float32)
    srcs = [a, empty, a, a, tiny, c]
    tgts = [apply_rigid(Ta, a), apply_rigid(Ta, a), empty, apply_rigid(Ta, a), apply_rigid(Ti, tiny),
            apply_rigid(Tc, c)]
    d_max = np.array([0.1, 0.1, 0.1, 0.1, 0.5, 0.07], np.float32)
    iters = np.array([15, 15, 15, 0, 10, 12], np.int32)
    T0 = np.tile(np.eye(4), (6, 1, 1))
    T0[5, :3, 3] = (0.01, -0.005, 0.002)
    nrms = [oracle_mod.normals(t, min(6, len(t)), (0, 0, 0))[0].astype(np.float32) if len(t) else
            np.zeros((0, 3), np.float32) for t in tgts]
    so = np.concatenate([[0], np.cumsum([len(s) for s in srcs])]).astype(np.int64)
    to = np.concatenate([[0], np.cumsum([len(t) for t in tgts])]).astype(np.int64)
    _say("batched icp edge pairs", so.tolist(), to.tolist())
    T, stats = gpu.icp_point_to_plane_batched(_dev(np.vstack(srcs)), so, _dev(np.vstack(tgts)),
                                              _dev(np.vstack(nrms)), to, T0, d_max, iters)
    T = T.cpu().numpy()
    for j in range(6):
        Ts, ss = gpu.icp_point_to_plane(_dev(srcs[j]), _dev(tgts[j]), _dev(nrms[j]), T0[j], float(d_max[j]),
                                        int(iters[j]))
        assert np.array_equal(T[j], Ts.cpu().numpy()), j
        assert stats[j] == ss, (j, stats[j], ss)
    assert stats[1]["status"] == 3 and stats[2]["status"] == 3          # no source / no target
    assert np.array_equal(T[1], T0[1]) and np.array_equal(T[2], T0[2])
    assert stats[3]["iterations_run"] == 0 and np.array_equal(T[3], T0[3])
    for j in (0, 4, 5):
        ro = oracle_mod.icp(srcs[j], tgts[j], nrms[j], T0[j], float(d_max[j]), int(iters[j]))
        ea, et = pose_err(T[j], ro["T"])
        assert ea <= ROT_TOL and et <= TRANS_TOL, (j, ea, et)


def test_batched_icp_with_normals_edge_pairs(gpu, oracle_mod):
    """The fused batched call on the edge pairs: each pair equals the single
    fused call, including an empty source, an empty target, a pair with no
    iterations and a 7-point pair (k = 6), and the non-empty registrations
    match the oracle run on the GPU's own normals."""
    import torch
    rng = rng_for(99, 1)
    a = sphere_plane(rng, 1500)
    Ta = random_rigid(rng, 8.0, 0.03)
    tiny = sphere_plane(rng, 7)
    Ti = random_rigid(rng, 2.0, 0.01)
    empty = np.zeros((0, 3), np.float32)
    srcs = [a, empty, a, a, tiny]
    tgts = [apply_rigid(Ta, a), apply_rigid(Ta, a), empty, apply_rigid(Ta, a), apply_rigid(Ti, tiny)]
    kk = np.array([10, 10, 10, 10, 6], np.int32)
    d_max = np.array([0.1, 0.1, 0.1, 0.1, 0.5], np.float32)
    iters = np.array([15, 15, 15, 0, 10], np.int32)
    so = np.concatenate([[0], np.cumsum([len(x) for x in srcs])]).astype(np.int64)
    to = np.concatenate([[0], np.cumsum([len(x) for x in tgts])]).astype(np.int64)
    _say("batched icp with normals edge pairs", so.tolist(), to.tolist())
    nrm = torch.empty((int(to[-1]), 3), dtype=torch.float32, device="cuda")
    T, stats = gpu.icp_point_to_plane_with_normals_batched(_dev(np.vstack(srcs)), so, _dev(np.vstack(tgts)), to, kk,
                                                           (0.0, 0.0, 0.0), None, d_max, iters, out_normals=nrm)
    T, nrm = T.cpu().numpy(), nrm.cpu().numpy()
    for j in range(5):
        if len(tgts[j]) == 0:
            continue     # the single fused call needs at least k target points
        Ts, ss, ns = gpu.icp_point_to_plane_with_normals(_dev(srcs[j]), _dev(tgts[j]), int(kk[j]), (0.0, 0.0, 0.0),
                                                         None, float(d_max[j]), int(iters[j]), return_normals=True)
        assert np.array_equal(T[j], Ts.cpu().numpy()), j
        assert stats[j] == ss, (j, stats[j], ss)
        assert np.array_equal(nrm[to[j]:to[j + 1]], ns.cpu().numpy()), j
    assert stats[1]["status"] == 3 and stats[2]["status"] == 3          # no source / no target
    assert np.array_equal(T[2], np.eye(4))
    assert stats[3]["iterations_run"] == 0 and np.array_equal(T[3], np.eye(4))
    for j in (0, 4):
        ro = oracle_mod.icp(srcs[j], tgts[j], nrm[to[j]:to[j + 1]], None, float(d_max[j]), int(iters[j]))
        ea, et = pose_err(T[j], ro["T"])
        assert ea <= ROT_TOL and et <= TRANS_TOL, (j, ea, et)
        assert stats[j]["inliers"] == ro["inliers"]


def test_batched_rejects_bad_offsets(gpu):
    import torch
    x = torch.zeros((10, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        gpu.estimate_normals_batched(x, [0, 5, 9], 3)            # does not end at len(xyz)
    with pytest.raises(gpu.PcgpuError):
        gpu.estimate_normals_batched(x, [0, 6, 5, 10], 3)        # decreasing
    with pytest.raises(gpu.PcgpuError):
        gpu.estimate_normals_batched(x, [0, 2, 10], [3, 3])      # k above a cloud's size


@pytest.mark.slow
def test_batched_full_workload_sampled(gpu, oracle_mod):
    b = batch_workload(3)
    off = b.offsets
    _say(f"full batched workload {b.name} n={b.n}")
    tgt = _dev(b.target)
    bn, _ = gpu.estimate_normals_batched(tgt, off, b.param("k").astype(np.int32), curvature=False)
    T, stats = gpu.icp_point_to_plane_batched(_dev(b.source), off, tgt, bn, off, None,
                                              b.param("d_max").astype(np.float32),
                                              b.param("iters").astype(np.int32))
    T, bn = T.cpu().numpy(), bn.cpu().numpy()
    sizes = np.diff(off)
    rng = np.random.default_rng(7)
    sample = sorted(set(rng.choice(b.n_pairs, 12, replace=False).tolist()) | {int(np.argmin(sizes)),
                                                                              int(np.argmax(sizes))})
    for j in sample:
        w = b.pairs[j]
        sn, _ = gpu.estimate_normals(_dev(w.target), w.k, curvature=False)
        assert np.array_equal(bn[off[j]:off[j + 1]], sn.cpu().numpy()), f"pair {j} normals"
        Ts, ss = _single_icp(gpu, w, bn[off[j]:off[j + 1]])
        assert np.array_equal(T[j], Ts) and stats[j] == ss, f"pair {j} pose"
    # the oracle on the smallest sampled pairs, with the same normals
    for j in sorted(sample, key=lambda q: sizes[q])[:4]:
        w = b.pairs[j]
        ro = oracle_mod.icp(w.source, w.target, bn[off[j]:off[j + 1]], None, float(np.float32(w.d_max)), w.iters)
        ea, et = pose_err(T[j], ro["T"])
        assert ea <= ROT_TOL and et <= TRANS_TOL, (j, ea, et)


def test_batched_full_workload_fused_bench_tuning(gpu, oracle_mod):
    # the benchmark's batch step as it runs: the fused normals+ICP batched
    # call over the full 256 uneven pairs, in the launch tuning the benchmark
    # applies (the autotuner's cached choice); sampled pairs against the
    # single fused call in the default tuning (same correspondences, sums
    # regrouped) and the oracle on the smallest of them
    import os
    import torch
    from paper_1807_00399_amd import autotune
    b = batch_workload(3)
    off = b.offsets
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1807_00399_amd",
                        "tuning_cache.json")
    hit = autotune.load_cache(path).get(autotune.cache_key(autotune._device_name(None), "uneven_pairs_256", b.n))
    if hit is None:
        pytest.skip("no cached tuning for this device")
    tun = hit["tuning"]
    _say(f"full fused batch {b.name} n={b.n} tuned {tun}")
    nrm = torch.empty((b.target.shape[0], 3), dtype=torch.float32, device="cuda")
    try:
        gpu.set_tuning(tun["icp_block_threads"], tun["icp_leaf"], tun["node_budget"], tun["sort_queries"],
                       tun.get("icp_persistent", 0))
        T, stats = gpu.icp_point_to_plane_with_normals_batched(_dev(b.source), off, _dev(b.target), off,
                                                               b.param("k").astype(np.int32), (0.0, 0.0, 0.0), None,
                                                               b.param("d_max").astype(np.float32),
                                                               b.param("iters").astype(np.int32), out_normals=nrm)
    finally:
        gpu.set_tuning(128, 16, 1.0, 1)
    T, nrm = T.cpu().numpy(), nrm.cpu().numpy()
    sizes = np.diff(off)
    rng = np.random.default_rng(11)
    sample = sorted(set(rng.choice(b.n_pairs, 10, replace=False).tolist()) | {int(np.argmin(sizes)),
                                                                              int(np.argmax(sizes))})
    for j in sample:
        w = b.pairs[j]
        Ts, ss, ns = gpu.icp_point_to_plane_with_normals(_dev(w.source), _dev(w.target), w.k, (0.0, 0.0, 0.0),
                                                         None, w.d_max, w.iters, return_normals=True)
        assert np.array_equal(nrm[off[j]:off[j + 1]], ns.cpu().numpy()), f"pair {j}: normals differ"
        assert np.abs(T[j] - Ts.cpu().numpy()).max() < 1e-10, f"pair {j}: pose differs"
        assert stats[j]["inliers"] == ss["inliers"] and stats[j]["status"] == ss["status"], (j, stats[j], ss)
    for j in sorted(sample, key=lambda q: sizes[q])[:3]:
        w = b.pairs[j]
        ro = oracle_mod.icp(w.source, w.target, nrm[off[j]:off[j + 1]], None, float(np.float32(w.d_max)), w.iters)
        ea, et = pose_err(T[j], ro["T"])
        assert ea <= ROT_TOL and et <= TRANS_TOL, (j, ea, et)
        assert stats[j]["inliers"] == ro["inliers"], (j, stats[j]["inliers"], ro["inliers"])


def test_batched_full_workload_every_pair_vs_oracle(gpu):
    # the benchmark's batch step as it runs (fused normals + ICP over one
    # pyramid, the launch tuning the benchmark applies) against the oracle's
    # end-to-end result for every one of the 256 pairs: its own kd-tree
    # normals and float64 ICP, stored with input digests by
    # tests/golden/make_icp_golden.py (oracle only)
    import hashlib
    import json
    import os
    from paper_1807_00399_amd import autotune
    b = batch_workload(3)
    off = b.offsets
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "icp_batch256.json")
    g = json.load(open(path))

    def digest(a):
        return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()

    assert g["sha256_source"] == digest(b.source) and g["sha256_target"] == digest(b.target) \
        and g["sha256_offsets"] == digest(off), "stored oracle results are for other inputs"
    cache = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1807_00399_amd",
                         "tuning_cache.json")
    hit = autotune.load_cache(cache).get(autotune.cache_key(autotune._device_name(None), "uneven_pairs_256", b.n))
    tun = hit["tuning"] if hit else gpu.get_tuning()
    _say(f"full fused batch {b.name} n={b.n} every pair vs oracle, tuning {tun}")
    try:
        gpu.set_tuning(tun["icp_block_threads"], tun["icp_leaf"], tun["node_budget"], tun["sort_queries"],
                       tun.get("icp_persistent", 0))
        T, stats = gpu.icp_point_to_plane_with_normals_batched(_dev(b.source), off, _dev(b.target), off,
                                                               b.param("k").astype(np.int32), (0.0, 0.0, 0.0), None,
                                                               b.param("d_max").astype(np.float32),
                                                               b.param("iters").astype(np.int32))
    finally:
        gpu.set_tuning(128, 16, 1.0, 1)
    T = T.cpu().numpy()
    bad = []
    worst = (0.0, 0.0)
    for j, p in enumerate(g["pairs"]):
        ea, et = pose_err(T[j], np.array(p["T"]).reshape(4, 4))
        worst = (max(worst[0], ea), max(worst[1], et))
        s = stats[j]
        if not (ea <= ROT_TOL and et <= TRANS_TOL and s["inliers"] == p["inliers"] and s["status"] == p["status"]
                and s["iterations_run"] == p["iterations"]):
            bad.append((j, ea, et, s["inliers"], p["inliers"], s["status"], p["status"]))
    _say(f"worst pose error {worst[0]:.3g} rad {worst[1]:.3g}; {len(bad)} pairs off")
    assert not bad, bad[:8]


def test_tunings_give_the_same_results(gpu, oracle_mod, small_batch):
    # every launch shape, pyramid depth and query order finds the same
    # correspondences; the block size and the query order only regroup the
    # compensated sums (~1e-14 relative)
    b = small_batch
    off = b.offsets
    nrms = np.vstack([oracle_mod.normals(w.target, w.k, (0, 0, 0))[0].astype(np.float32) for w in b.pairs])
    args = (_dev(b.source), off, _dev(b.target), _dev(nrms), off, None, b.param("d_max").astype(np.float32),
            b.param("iters").astype(np.int32))
    ref_T, ref_st = None, None
    try:
        for tb in (64, 128, 256):
            for leaf in (8, 16, 32):
                for nb, sq in ((0.25, 0), (1.0, 1), (1.0, 0)):
                    gpu.set_tuning(tb, leaf, nb, sq)
                    _say(f"tuning {tb} {leaf} {nb} {sq}")
                    T, st = gpu.icp_point_to_plane_batched(*args)
                    T = T.cpu().numpy()
                    nn, _ = gpu.estimate_normals_batched(_dev(b.target), off, b.param("k").astype(np.int32))
                    if ref_T is None:
                        ref_T, ref_st, ref_n = T, st, nn.cpu().numpy()
                        continue
                    assert np.array_equal(nn.cpu().numpy(), ref_n)
                    assert np.abs(T - ref_T).max() < 1e-10, (tb, leaf, nb, sq)
                    assert [s["inliers"] for s in st] == [s["inliers"] for s in ref_st]
                    assert [s["status"] for s in st] == [s["status"] for s in ref_st]
    finally:
        gpu.set_tuning(128, 16, 1.0)


_PERSISTENT_OFF = ("the persistent ICP loop is switched off (pc_set_tuning rejects it): after the search's "
                   "register allocation changed, a run of it stopped making progress on the GPU and the cause is "
                   "not established; not run again until it is")


@pytest.mark.skip(reason="stopped making progress on the GPU while timing its persistent-loop candidate; "
                         "not run again until the cause is shown (" + _PERSISTENT_OFF + ")")
def test_autotune_on_device(gpu, small_batch, tmp_path):
    from paper_1807_00399_amd import autotune
    b = small_batch
    off = b.offsets
    src, tgt = _dev(b.source), _dev(b.target)
    kc, dm, it = b.param("k").astype(np.int32), b.param("d_max").astype(np.float32), b.param("iters").astype(np.int32)

    def step():
        nrm, _ = gpu.estimate_normals_batched(tgt, off, kc, curvature=False)
        gpu.icp_point_to_plane_batched(src, off, tgt, nrm, off, None, dm, it, read_stats=False)

    try:
        r = autotune.tune(step, "test_small", b.n, cache_file=str(tmp_path / "t.json"), reps=1,
                          candidates=autotune.CANDIDATES[:4])
        assert not r["from_cache"] and gpu.get_tuning() == r["tuning"]
    finally:
        gpu.set_tuning(128, 16, 1.0)


@pytest.mark.skip(reason=_PERSISTENT_OFF)
def test_persistent_loop_equals_lockstep(gpu, oracle_mod, small_batch):
    # the whole ICP loop as one cooperative launch computes exactly what the
    # three launches per iteration compute: same blocks, groups and pairs,
    # same merge order, so poses and statistics are bit-identical
    b = small_batch
    off = b.offsets
    kc, dm, it = b.param("k").astype(np.int32), b.param("d_max").astype(np.float32), b.param("iters").astype(np.int32)
    src, tgt = _dev(b.source), _dev(b.target)
    try:
        for tb, leaf in ((64, 8), (128, 16), (256, 32)):
            res = []
            for pe in (0, 1):
                gpu.set_tuning(tb, leaf, 1.0, 1, pe)
                _say(f"persistent={pe} block {tb} leaf {leaf}")
                T, st = gpu.icp_point_to_plane_with_normals_batched(src, off, tgt, off, kc, (0.0, 0.0, 0.0), None, dm,
                                                                    it)
                res.append((T.cpu().numpy(), st))
            assert np.array_equal(res[0][0], res[1][0]), (tb, leaf)
            assert res[0][1] == res[1][1]
        # a single pair too, with an early stop from conv_tol
        w = b.pairs[0]
        nrm = oracle_mod.normals(w.target, w.k, (0, 0, 0))[0].astype(np.float32)
        out = []
        for pe in (0, 1):
            gpu.set_tuning(128, 16, 1.0, 1, pe)
            T, st = gpu.icp_point_to_plane(_dev(w.source), _dev(w.target), _dev(nrm), None, w.d_max, w.iters, 1e-9)
            out.append((T.cpu().numpy(), st))
        assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]
    finally:
        gpu.set_tuning(128, 16, 1.0, 1, 0)


@pytest.mark.skip(reason=_PERSISTENT_OFF)
def test_persistent_loop_full_batch_equals_lockstep(gpu):
    # the benchmark's batch step with the persistent loop: bit-identical to
    # the lockstep launches in the same launch shape
    b = batch_workload(3)
    off = b.offsets
    kc, dm, it = b.param("k").astype(np.int32), b.param("d_max").astype(np.float32), b.param("iters").astype(np.int32)
    src, tgt = _dev(b.source), _dev(b.target)
    res = []
    try:
        for pe in (0, 1):
            gpu.set_tuning(64, 8, 0.5, 1, pe)
            _say(f"full batch persistent={pe}")
            T, st = gpu.icp_point_to_plane_with_normals_batched(src, off, tgt, off, kc, (0.0, 0.0, 0.0), None, dm, it)
            res.append((T.cpu().numpy(), st))
    finally:
        gpu.set_tuning(128, 16, 1.0, 1, 0)
    assert np.array_equal(res[0][0], res[1][0])
    assert res[0][1] == res[1][1]


@pytest.mark.parametrize("n_clouds", [1, 2, 300])
def test_batched_normals_sort_passes(gpu, n_clouds):
    # the batch's radix sort runs one pass per byte of the (cloud, Morton
    # key): 6 passes for one cloud, 7 for up to 256 clouds, 8 for 300; an
    # odd count leaves the sorted keys in the alternate buffers.  Each cloud
    # of the batch must still get exactly the single call's normals.
    rng = rng_for(90, n_clouds)
    sizes = rng.integers(16, 48, size=n_clouds)
    clouds = [sphere_plane(rng, int(m)) for m in sizes]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    k = np.full(n_clouds, 8, np.int32)
    _say(f"sort passes: {n_clouds} clouds, {off[-1]} points")
    bn, bc = gpu.estimate_normals_batched(_dev(np.vstack(clouds)), off, k)
    bn, bc = bn.cpu().numpy(), bc.cpu().numpy()
    for j, c in enumerate(clouds):
        sn, sc = gpu.estimate_normals(_dev(c), 8)
        assert np.array_equal(bn[off[j]:off[j + 1]], sn.cpu().numpy()), f"cloud {j}"
        assert np.array_equal(bc[off[j]:off[j + 1]], sc.cpu().numpy()), f"cloud {j}"
