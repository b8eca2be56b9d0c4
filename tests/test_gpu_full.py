"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times: the depth-camera room (307,200 points, k=16, d_max 0.05,
30 iterations) and the LiDAR street (2,097,152 points, k=16, d_max 1.0,
40 iterations).

- k-NN: bit-exact on every query against the oracle's kd-tree (itself held
  bit-equal to brute force), and on 10,000 sampled queries against brute
  force directly.
- normals: every point, against the oracle (kd-tree, itself pinned to brute
  force), <= 1e-5 rad where the eigen-gap makes the normal well defined.
- ICP: pose within 1e-5 rad / 1e-6 of the oracle.  The oracle's full-size
  result is stored in tests/golden/icp_workloads.json by
  tests/golden/make_icp_golden.py (oracle only); it is used when the inputs
  hash to the same digests, otherwise the oracle runs here.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from gen import make_workload, rng_for
from tests.helpers import angle_between, pose_err

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "icp_workloads.json")


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_00399_amd import pcgpu
    return pcgpu


@pytest.fixture(scope="module", params=[1, 2], ids=["room307200", "street2097152"])
def work(request, oracle_mod):
    w = make_workload(request.param)
    nrm, curv, ev = oracle_mod.normals(w.target, w.k, (0.0, 0.0, 0.0), method="kdtree")
    return w, nrm, curv, ev


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_full_knn_bit_exact(gpu, oracle_mod, work):
    w = work[0]
    print(f"knn full {w.name}", flush=True)
    ref = _dev(w.target)
    idx, d2 = gpu.knn_search(ref, ref, w.k)
    gi, gd = idx.cpu().numpy(), d2.cpu().numpy()
    # every query against the oracle's exact kd-tree
    ei, ed = oracle_mod.knn(w.target, w.target, w.k, "kdtree")
    bad = np.flatnonzero(np.any(gi != ei, axis=1) | np.any(gd.view(np.uint32) != ed.view(np.uint32), axis=1))
    assert bad.size == 0, f"{bad.size} queries differ, first {bad[:5].tolist()}"
    # and a sample against the definition itself (brute force)
    sample = rng_for(700, w.n).choice(w.n, 10_000, replace=False)
    bi, bd = oracle_mod.knn(w.target, w.target[sample], w.k, "brute")
    assert np.array_equal(gi[sample], bi) and np.array_equal(gd[sample].view(np.uint32), bd.view(np.uint32))


def test_full_normals(gpu, work):
    w, en, ec, ev = work
    print(f"normals full {w.name}", flush=True)
    n, c = gpu.estimate_normals(_dev(w.target), w.k)
    gn = n.cpu().numpy().astype(np.float64)
    gate = (ev[:, 1] - ev[:, 0]) >= 1e-2 * ev[:, 2]
    ang = angle_between(gn, en)
    assert gate.mean() > 0.9
    assert ang[gate].max() <= 1e-5, ang[gate].max()
    assert np.allclose(c.cpu().numpy(), ec, rtol=1e-5, atol=1e-7)
    # the paper-facing statistic: how many points are outside the gate and
    # how far they are (reported, not gated)
    print(f"gated {gate.mean():.4f}; ungated max angle {ang[~gate].max() if (~gate).any() else 0:.3g} rad")


def test_full_icp_pose(gpu, oracle_mod, work):
    w, en, _, _ = work
    nrm = en.astype(np.float32)
    print(f"icp full {w.name}", flush=True)
    T, st = gpu.icp_point_to_plane(_dev(w.source), _dev(w.target), _dev(nrm), None, w.d_max, w.iters)
    Tg = T.cpu().numpy()
    ref = json.load(open(GOLDEN)).get(w.name) if os.path.exists(GOLDEN) else None
    if ref and ref["sha256_source"] == _digest(w.source) and ref["sha256_target"] == _digest(w.target) \
            and ref["sha256_normals"] == _digest(nrm):
        To, inl, status, its = np.array(ref["T"]).reshape(4, 4), ref["inliers"], ref["status"], ref["iterations"]
    else:
        ro = oracle_mod.icp(w.source, w.target, nrm, None, float(np.float32(w.d_max)), w.iters)
        To, inl, status, its = ro["T"], ro["inliers"], ro["status"], ro["iterations"]
    ea, et = pose_err(Tg, To)
    print(f"pose vs oracle {ea:.3g} rad {et:.3g}; inliers {st['inliers']} vs {inl}", flush=True)
    assert st["status"] == status and st["iterations_run"] == its
    assert ea <= 1e-5 and et <= 1e-6
    assert st["inliers"] == inl


def test_full_icp_with_normals(gpu, oracle_mod, work):
    # the fused call (normals and ICP over one target pyramid, the path the
    # benchmark times) at full size: bit-identical to estimate_normals
    # followed by icp_point_to_plane, and its pose within the same bar as
    # the oracle's pose from the oracle's normals
    import torch
    w, en, _, _ = work
    print(f"icp with normals full {w.name}", flush=True)
    S, T = _dev(w.source), _dev(w.target)
    Tf, sf, nf = gpu.icp_point_to_plane_with_normals(S, T, w.k, (0.0, 0.0, 0.0), None, w.d_max, w.iters,
                                                     return_normals=True, read_stats=False)
    n2, _ = gpu.estimate_normals(T, w.k, curvature=False)
    Ts, ss = gpu.icp_point_to_plane(S, T, n2, None, w.d_max, w.iters, read_stats=False)
    assert torch.equal(nf, n2) and torch.equal(Tf, Ts) and torch.equal(sf, ss)
    nrm = en.astype(np.float32)
    ref = json.load(open(GOLDEN)).get(w.name) if os.path.exists(GOLDEN) else None
    if not (ref and ref["sha256_source"] == _digest(w.source) and ref["sha256_target"] == _digest(w.target)
            and ref["sha256_normals"] == _digest(nrm)):
        pytest.skip("no stored oracle pose for this workload")
    st = gpu.decode_stats(sf)
    ea, et = pose_err(Tf.cpu().numpy(), np.array(ref["T"]).reshape(4, 4))
    print(f"fused pose vs oracle {ea:.3g} rad {et:.3g}; inliers {st['inliers']} vs {ref['inliers']}", flush=True)
    assert st["status"] == ref["status"]
    assert ea <= 1e-5 and et <= 1e-6
    assert st["inliers"] == ref["inliers"]


def _bench_tuning(tag, n):
    """The launch tuning the benchmark applies to this workload (its cached
    autotuner choice for this device), or None."""
    from paper_1807_00399_amd import autotune
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1807_00399_amd",
                        "tuning_cache.json")
    hit = autotune.load_cache(path).get(autotune.cache_key(autotune._device_name(None), tag, n))
    return hit["tuning"] if hit else None


def test_full_icp_with_normals_bench_tuning(gpu, oracle_mod, work):
    # the benchmark's exact launch configuration (block size, leaf size, node
    # budget, query order from the tuning cache) at full size: the same
    # correspondences as the default launch, sums regrouped only, and the
    # pose held to the oracle's
    w, en, _, _ = work
    tun = _bench_tuning(w.name, w.n)
    if tun is None:
        pytest.skip("no cached tuning for this device")
    print(f"icp with normals full {w.name} tuned {tun}", flush=True)
    S, T = _dev(w.source), _dev(w.target)
    Td, sd = gpu.icp_point_to_plane_with_normals(S, T, w.k, (0.0, 0.0, 0.0), None, w.d_max, w.iters)
    try:
        gpu.set_tuning(tun["icp_block_threads"], tun["icp_leaf"], tun["node_budget"], tun["sort_queries"],
                       tun.get("icp_persistent", 0))
        Tt, st = gpu.icp_point_to_plane_with_normals(S, T, w.k, (0.0, 0.0, 0.0), None, w.d_max, w.iters)
    finally:
        gpu.set_tuning(128, 16, 1.0, 1)
    Tt, Td = Tt.cpu().numpy(), Td.cpu().numpy()
    assert np.abs(Tt - Td).max() < 1e-10
    assert st["inliers"] == sd["inliers"] and st["status"] == sd["status"]
    assert st["iterations_run"] == sd["iterations_run"]
    nrm = en.astype(np.float32)
    ref = json.load(open(GOLDEN)).get(w.name) if os.path.exists(GOLDEN) else None
    if not (ref and ref["sha256_source"] == _digest(w.source) and ref["sha256_target"] == _digest(w.target)
            and ref["sha256_normals"] == _digest(nrm)):
        pytest.skip("no stored oracle pose for this workload")
    ea, et = pose_err(Tt, np.array(ref["T"]).reshape(4, 4))
    print(f"tuned pose vs oracle {ea:.3g} rad {et:.3g}; inliers {st['inliers']} vs {ref['inliers']}", flush=True)
    assert st["status"] == ref["status"]
    assert ea <= 1e-5 and et <= 1e-6
    assert st["inliers"] == ref["inliers"]
