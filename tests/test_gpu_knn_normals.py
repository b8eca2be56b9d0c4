"""GPU parity: k-NN (bit-exact against the oracle) and PCA normals
(<= 1e-5 rad on well-conditioned points), called through the C ABI."""
import numpy as np
import pytest

from gen import lattice_cloud, make_workload, rng_for, sphere_plane, uniform_cloud
from tests.helpers import angle_between

pytestmark = pytest.mark.gpu

NORMAL_TOL_RAD = 1e-5
GAP_GATE = 1e-2     # normals compared where (l1 - l0) >= GAP_GATE * l2 (oracle eigenvalues)


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


def _knn_parity(gpu, oracle_mod, ref, qry, k, method="brute", same=False):
    _say(f"knn n_ref={len(ref)} n_qry={len(qry)} k={k}")
    r = _dev(ref)
    q = r if same else _dev(qry)
    idx, d2 = gpu.knn_search(r, q, k)
    ei, ed = oracle_mod.knn(ref, qry, k, method)
    gi, gd = idx.cpu().numpy(), d2.cpu().numpy()
    bad = np.nonzero((gi != ei).any(1) | (gd != ed).any(1))[0]
    assert bad.size == 0, f"{bad.size} rows differ; first row {bad[0]}: gpu {gi[bad[0]]} {gd[bad[0]]} oracle {ei[bad[0]]} {ed[bad[0]]}"


@pytest.mark.parametrize("k", [1, 2, 5, 10, 16, 17, 32])
def test_knn_random_self(gpu, oracle_mod, k):
    pts = uniform_cloud(rng_for(500, k), 5000)
    _knn_parity(gpu, oracle_mod, pts, pts, k, same=True)


@pytest.mark.parametrize("k", [1, 10, 32])
def test_knn_distinct_queries_inside_and_outside(gpu, oracle_mod, k):
    rng = rng_for(501, k)
    ref = uniform_cloud(rng, 4000)
    qry = uniform_cloud(rng, 1500, -2.5, 2.5)       # many queries outside the bounding box
    _knn_parity(gpu, oracle_mod, ref, qry, k)


@pytest.mark.parametrize("k", [1, 7, 19, 27, 32])
def test_knn_lattice_exact_ties(gpu, oracle_mod, k):
    pts = lattice_cloud(12, 0.25, (0.5, -1.0, 3.0))
    _knn_parity(gpu, oracle_mod, pts, pts, k, same=True)


def test_knn_duplicates_and_clusters(gpu, oracle_mod):
    rng = rng_for(502)
    base = uniform_cloud(rng, 200)
    ref = base[rng.integers(0, 200, 3000)]
    c = rng.normal(size=(10, 3))
    cl = (c[rng.integers(0, 10, 2000)] + 1e-4 * rng.normal(size=(2000, 3))).astype(np.float32)
    ref = np.vstack([ref, cl])
    _knn_parity(gpu, oracle_mod, ref, ref, 16, same=True)


def test_knn_k_equals_n_and_tiny_clouds(gpu, oracle_mod):
    for n in (1, 2, 3, 17, 32):
        pts = uniform_cloud(rng_for(503, n), n)
        _knn_parity(gpu, oracle_mod, pts, pts, min(n, 32), same=True)


def test_knn_empty_queries(gpu):
    import torch
    ref = _dev(uniform_cloud(rng_for(504), 100))
    q = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    idx, d2 = gpu.knn_search(ref, q, 4)
    assert idx.shape == (0, 4)


@pytest.mark.parametrize("cfg,size", [(0, "full"), (1, "small"), (2, "small")])
def test_knn_workload_clouds(gpu, oracle_mod, cfg, size):
    w = make_workload(cfg, size=size)
    _knn_parity(gpu, oracle_mod, w.target, w.target, w.k, method="kdtree", same=True)


def _normals_parity(gpu, oracle_mod, pts, k, vp=(0.0, 0.0, 0.0)):
    _say(f"normals n={len(pts)} k={k} vp={vp}")
    n, c = gpu.estimate_normals(_dev(pts), k, vp)
    gn, gc = n.cpu().numpy().astype(np.float64), c.cpu().numpy().astype(np.float64)
    en, ec, ev = oracle_mod.normals(pts, k, vp, method="kdtree")
    gate = (ev[:, 1] - ev[:, 0]) >= GAP_GATE * ev[:, 2]
    zero = ~np.any(en != 0, axis=1)
    ang = angle_between(gn, en)
    assert np.all(~np.any(gn[zero] != 0, axis=1)), "zero-covariance points must get a zero normal"
    g = gate & ~zero
    worst = float(ang[g].max()) if g.any() else 0.0
    assert worst <= NORMAL_TOL_RAD, f"max angle {worst:.3g} rad on gated points"
    assert np.allclose(gc, ec, rtol=1e-5, atol=1e-7)
    return float(g.mean()), worst, float(ang[~g & ~zero].max()) if (~g & ~zero).any() else 0.0


def test_normals_sphere_plane_10k(gpu, oracle_mod):
    w = make_workload(0)
    frac, worst, _ = _normals_parity(gpu, oracle_mod, w.target, w.k)
    assert frac > 0.95


@pytest.mark.parametrize("k", [3, 8, 10, 16, 32])
def test_normals_k_variants(gpu, oracle_mod, k):
    pts = sphere_plane(rng_for(505, k), 4000)
    _normals_parity(gpu, oracle_mod, pts, k, (0.2, -0.1, 0.3))


@pytest.mark.parametrize("cfg", [1, 2])
def test_normals_workload_small(gpu, oracle_mod, cfg):
    w = make_workload(cfg, size="small")
    _normals_parity(gpu, oracle_mod, w.target, w.k)


def test_normals_exact_plane_and_coincident(gpu, oracle_mod):
    rng = rng_for(506)
    xy = rng.uniform(-1, 1, size=(600, 2))
    plane = np.column_stack([xy, np.full(600, 0.5)]).astype(np.float32)
    n, _ = gpu.estimate_normals(_dev(plane), 10, (0, 0, 0))
    assert np.all(n.cpu().numpy() == np.array([0, 0, -1], np.float32))
    pts = np.vstack([np.tile([[0.1, 0.2, 0.3]], (12, 1)), uniform_cloud(rng, 50)]).astype(np.float32)
    _normals_parity(gpu, oracle_mod, pts, 10)
