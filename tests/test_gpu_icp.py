"""GPU parity: point-to-plane ICP through the C ABI against the oracle.

Both sides get the same target normals (the oracle's, rounded to float32)
so the comparison isolates the ICP loop; the end-to-end test gives each side
its own normals.  Bar: rotation within 1e-5 rad and translation within 1e-6
of the oracle's pose."""
import numpy as np
import pytest

from gen import apply_rigid, make_workload, random_rigid, rng_for, sphere_plane
from tests.helpers import pose_err

pytestmark = pytest.mark.gpu

ROT_TOL = 1e-5
TRANS_TOL = 1e-6


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


def _oracle_normals(oracle_mod, pts, k):
    n, _, _ = oracle_mod.normals(pts, k, (0, 0, 0))
    return n.astype(np.float32)


def _run_gpu(gpu, src, tgt, nrm, T0, d_max, iters, tol=0.0):
    T, st = gpu.icp_point_to_plane(_dev(src), _dev(tgt), _dev(nrm), T0, d_max, iters, tol)
    return T.cpu().numpy(), st


def _parity(gpu, oracle_mod, src, tgt, nrm, T0, d_max, iters, tol=0.0, label=""):
    _say(f"icp {label} n_src={len(src)} n_tgt={len(tgt)} d_max={d_max} iters={iters}")
    Tg, sg = _run_gpu(gpu, src, tgt, nrm, T0, d_max, iters, tol)
    # the ABI takes d_max as float32; the oracle gets that same value
    ro = oracle_mod.icp(src, tgt, nrm, T0, float(np.float32(d_max)), iters, tol)
    ea, et = pose_err(Tg, ro["T"])
    assert sg["status"] == ro["status"], (sg, ro["status"])
    assert sg["iterations_run"] == ro["iterations"]
    assert ea <= ROT_TOL and et <= TRANS_TOL, f"pose differs: {ea:.3g} rad, {et:.3g}"
    # every correspondence decision equals the float64 one at the GPU's own
    # pose, and that pose agrees with the oracle's to ~1e-11: a count could
    # differ only through a point that close to d_max or to a tie, and the
    # seeded inputs have none, so the counts are held equal
    assert sg["inliers"] == ro["inliers"], (sg["inliers"], ro["inliers"])
    return Tg, sg, ro


@pytest.mark.parametrize("cfg,size", [(0, "small"), (0, "full"), (1, "small"), (2, "small")])
def test_icp_workloads(gpu, oracle_mod, cfg, size):
    w = make_workload(cfg, size=size)
    nrm = _oracle_normals(oracle_mod, w.target, w.k)
    _parity(gpu, oracle_mod, w.source, w.target, nrm, None, w.d_max, w.iters, label=w.name)


def test_icp_recovers_ground_truth_workload0(gpu, oracle_mod):
    w = make_workload(0)
    nrm = _oracle_normals(oracle_mod, w.target, w.k)
    Tg, sg = _run_gpu(gpu, w.source, w.target, nrm, None, w.d_max, w.iters)
    ea, et = pose_err(Tg, w.T_gt)
    assert ea < 1e-5 and et < 1e-6


def test_icp_end_to_end_own_normals(gpu, oracle_mod):
    # each side estimates its own normals (GPU kernels vs oracle)
    w = make_workload(0)
    n_gpu, _ = gpu.estimate_normals(_dev(w.target), w.k)
    T, sg = gpu.icp_point_to_plane(_dev(w.source), _dev(w.target), n_gpu, None, w.d_max, w.iters)
    ro = oracle_mod.icp(w.source, w.target, _oracle_normals(oracle_mod, w.target, w.k), None,
                        float(np.float32(w.d_max)), w.iters)
    ea, et = pose_err(T.cpu().numpy(), ro["T"])
    assert ea <= ROT_TOL and et <= TRANS_TOL


@pytest.mark.parametrize("cfg,size", [(0, "full"), (1, "small"), (2, "small")])
def test_icp_with_normals_equals_two_calls(gpu, cfg, size):
    # one pyramid for normals and correspondences gives exactly the result
    # of estimate_normals followed by icp_point_to_plane
    import torch
    w = make_workload(cfg, size=size)
    _say(f"icp_with_normals {w.name} n={w.n}")
    S, T = _dev(w.source), _dev(w.target)
    n2, _ = gpu.estimate_normals(T, w.k, curvature=False)
    Ta, sa = gpu.icp_point_to_plane(S, T, n2, None, w.d_max, w.iters, read_stats=False)
    Tb, sb, nb = gpu.icp_point_to_plane_with_normals(S, T, w.k, init_T=None, max_corr_dist=w.d_max,
                                                     max_iters=w.iters, return_normals=True, read_stats=False)
    assert torch.equal(nb, n2) and torch.equal(Ta, Tb) and torch.equal(sa, sb)
    # without the normals output, and with an empty target
    Tc, sc = gpu.icp_point_to_plane_with_normals(S, T, w.k, max_corr_dist=w.d_max, max_iters=w.iters,
                                                 read_stats=False)
    assert torch.equal(Tc, Ta) and torch.equal(sc, sa)
    Te, se = gpu.icp_point_to_plane_with_normals(S, T[:0], 1, max_corr_dist=w.d_max, max_iters=3)
    assert se["status"] == 3 and np.array_equal(Te.cpu().numpy(), np.eye(4))


def test_icp_identity_pair_bit_exact(gpu, oracle_mod):
    pts = sphere_plane(rng_for(600), 3000)
    nrm = _oracle_normals(oracle_mod, pts, 10)
    Tg, sg = _run_gpu(gpu, pts, pts, nrm, None, 0.1, 10)
    assert np.array_equal(Tg, np.eye(4))
    assert sg["rms"] == 0.0 and sg["inliers"] == 3000


def test_icp_init_pose_and_equivariance(gpu, oracle_mod):
    w = make_workload(0, size="small")
    nrm = _oracle_normals(oracle_mod, w.target, w.k)
    T0 = random_rigid(rng_for(601), 3.0, 0.02) @ w.T_gt
    _parity(gpu, oracle_mod, w.source, w.target, nrm, T0, w.d_max, 15, label="init")
    G = random_rigid(rng_for(602), 40.0, 2.0)
    tgt2 = apply_rigid(G, w.target)
    n2 = (nrm.astype(np.float64) @ G[:3, :3].T).astype(np.float32)
    Tg, _ = _run_gpu(gpu, w.source, tgt2, n2, G, w.d_max, w.iters)
    To = oracle_mod.icp(w.source, w.target, nrm, None, w.d_max, w.iters)["T"]
    ea, et = pose_err(Tg, G @ To)
    assert ea < 1e-5 and et < 1e-5


def test_icp_degenerate_plane(gpu):
    rng = rng_for(603)
    xy = rng.uniform(-1, 1, size=(2000, 2))
    pts = np.column_stack([xy, np.zeros(2000)]).astype(np.float32)
    nrm = np.tile(np.array([[0, 0, 1]], np.float32), (2000, 1))
    Tg, sg = _run_gpu(gpu, pts, pts, nrm, None, 0.1, 5)
    assert sg["status"] == gpu.PC_ICP_DEGENERATE and sg["iterations_run"] == 0
    assert np.array_equal(Tg, np.eye(4))


def test_icp_no_inliers_and_few_inliers(gpu, oracle_mod):
    pts = sphere_plane(rng_for(604), 500)
    nrm = _oracle_normals(oracle_mod, pts, 10)
    far = pts + np.float32(10.0)
    Tg, sg = _run_gpu(gpu, far, pts, nrm, None, 0.1, 5)
    assert sg["status"] == gpu.PC_ICP_NO_INLIERS and sg["inliers"] == 0 and sg["rms"] == 0.0
    Tg, sg = _run_gpu(gpu, np.vstack([far, pts[:4]]), pts, nrm, None, 0.1, 5)
    assert sg["status"] == gpu.PC_ICP_DEGENERATE and sg["iterations_run"] == 0


def test_icp_empty_source(gpu):
    import torch
    tgt = _dev(sphere_plane(rng_for(605), 100))
    src = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    T0 = random_rigid(rng_for(606), 5.0, 0.1)
    T, st = gpu.icp_point_to_plane(src, tgt, tgt, T0, 0.1, 5)
    assert np.array_equal(T.cpu().numpy(), T0)
    assert st["status"] == gpu.PC_ICP_NO_INLIERS


def test_icp_zero_iterations_reports_initial_pose(gpu, oracle_mod):
    w = make_workload(0, size="small")
    nrm = _oracle_normals(oracle_mod, w.target, w.k)
    _parity(gpu, oracle_mod, w.source, w.target, nrm, None, w.d_max, 0, label="zero-iter")


def test_icp_convergence_tolerance(gpu, oracle_mod):
    w = make_workload(0, size="small")
    nrm = _oracle_normals(oracle_mod, w.target, w.k)
    Tg, sg, ro = _parity(gpu, oracle_mod, w.source, w.target, nrm, None, w.d_max, 50, tol=1e-7, label="tol")
    assert sg["status"] == gpu.PC_ICP_CONVERGED


def test_icp_deterministic(gpu, oracle_mod):
    w = make_workload(1, size="small")
    nrm = _oracle_normals(oracle_mod, w.target, w.k)
    a, sa = _run_gpu(gpu, w.source, w.target, nrm, None, w.d_max, w.iters)
    b, sb = _run_gpu(gpu, w.source, w.target, nrm, None, w.d_max, w.iters)
    assert np.array_equal(a, b) and sa == sb


@pytest.mark.parametrize("fused", [False, True])
def test_icp_match_certificate_duplicates(gpu, oracle_mod, fused):
    """A converged point keeps its previous match without a search when it
    lies within half the distance from that match to the nearest other
    target point.  A target with exact duplicates (that distance is 0: always
    searched) and 2 um near-duplicates (the certificate at its margin), with
    the source an exact copy started at the true pose, so that iterations 1..
    and the final pass run on certificates: the final statistics must equal
    the oracle's evaluated at the returned pose.  Residuals are ~1e-7 here, so
    a single wrong near-duplicate match would move the rms by far more than
    the tolerance."""
    rng = rng_for(0, 77)
    base = sphere_plane(rng, 3000)
    dup = base[rng.choice(3000, 200, replace=False)]
    near = base[rng.choice(3000, 200, replace=False)] + rng.normal(size=(200, 3)) * 2e-6
    tgt = np.vstack([base, dup, near]).astype(np.float32)
    G = random_rigid(rng, 3.0, 0.02)
    src = apply_rigid(np.linalg.inv(G), tgt).astype(np.float32)
    d_max = 0.1
    _say(f"icp certificate fused={fused} n={len(tgt)}")
    if fused:
        T, st, nrm = gpu.icp_point_to_plane_with_normals(_dev(src), _dev(tgt), 10, (0.0, 0.0, 0.0), G, d_max, 4,
                                                         return_normals=True)
        nrm = nrm.cpu().numpy()
    else:
        nrm = _oracle_normals(oracle_mod, tgt, 10)
        T, st = gpu.icp_point_to_plane(_dev(src), _dev(tgt), _dev(nrm), G, d_max, 4)
    T = T.cpu().numpy()
    sysm = oracle_mod.p2plane_system(src, tgt, nrm, T, float(np.float32(d_max)))
    assert st["inliers"] == sysm["inliers"] == len(src)
    rms_o = np.sqrt(sysm["sum_r2"] / sysm["inliers"])
    assert rms_o < 1e-6
    assert abs(st["rms"] - rms_o) <= 1e-3 * rms_o, (st["rms"], rms_o)
    ro = oracle_mod.icp(src, tgt, nrm, G, float(np.float32(d_max)), 4)
    ea, et = pose_err(T, ro["T"])
    assert ea <= ROT_TOL and et <= TRANS_TOL
