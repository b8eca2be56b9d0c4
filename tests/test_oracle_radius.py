"""Pins for the oracle's radius and hybrid neighbourhoods (CPU): lattice
counts by hand, the kd-tree against brute-force membership, hybrid with an
unbounded radius against the k-NN normals, planes and spheres."""
import numpy as np

from gen import lattice_cloud, rng_for, sphere_plane, uniform_cloud
from tests.helpers import angle_between


def test_lattice_counts_by_hand(oracle_mod):
    x = lattice_cloud(6, 1.0)
    _, _, _, cnt = oracle_mod.normals_radius(x, 1.0)        # key 1 <= r^2 = 1: face neighbours count
    ijk = np.rint(x).astype(int)
    on_face = ((ijk == 0) | (ijk == 5)).sum(axis=1)         # 0 interior, 1 face, 2 edge, 3 corner
    assert np.array_equal(cnt, 7 - on_face)
    n, c, _, cnt = oracle_mod.normals_radius(x, 0.999)
    assert np.all(cnt == 1) and np.all(n == 0) and np.all(c == 0)   # fewer than 3: no normal


def test_kdtree_matches_brute_force(oracle_mod):
    for seed, r in ((700, 0.08), (701, 0.2)):
        p = uniform_cloud(rng_for(seed), 3000)
        a = oracle_mod.normals_radius(p, r)
        b = oracle_mod.normals_radius(p, r, method="brute")
        for u, v in zip(a, b):
            assert np.array_equal(u, v)


def test_hybrid_with_unbounded_radius_is_knn(oracle_mod):
    p = sphere_plane(rng_for(702), 3000)
    n, c, ev, cnt = oracle_mod.normals_radius(p, 1e6, k=12)
    en, ec, eev = oracle_mod.normals(p, 12, (0, 0, 0))
    assert np.all(cnt == 12)
    gate = (eev[:, 1] - eev[:, 0]) >= 1e-3 * eev[:, 2]
    assert np.abs(ev - eev).max() <= 1e-12 * np.abs(eev).max()
    assert angle_between(n[gate], en[gate]).max() < 1e-9
    # a finite radius keeps only the nearest ones inside it
    n2, _, _, cnt2 = oracle_mod.normals_radius(p, 0.05, k=12)
    assert cnt2.max() <= 12 and cnt2.min() >= 1 and (cnt2 < 12).any()


def test_plane_and_sphere(oracle_mod):
    rng = rng_for(703)
    xy = rng.uniform(-1, 1, size=(4000, 2))
    plane = np.column_stack([xy, np.zeros(4000)]).astype(np.float32)
    n, c, _, cnt = oracle_mod.normals_radius(plane, 0.1, viewpoint=(0, 0, 5))
    ok = cnt >= 3
    assert ok.mean() > 0.99 and np.all(n[ok] == [0, 0, 1]) and np.all(c[ok] == 0)
    g = rng.normal(size=(20000, 3))
    sph = (g / np.linalg.norm(g, axis=1, keepdims=True)).astype(np.float32)
    n, c, ev, cnt = oracle_mod.normals_radius(sph, 0.1, viewpoint=(0, 0, 0))
    good = (cnt >= 10) & ((ev[:, 1] - ev[:, 0]) >= 1e-3 * ev[:, 2])
    ang = angle_between(n[good], -sph[good].astype(np.float64))     # oriented toward the centre
    assert good.mean() > 0.95 and ang.max() < 0.05
