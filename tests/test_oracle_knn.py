"""Pins for the oracle's k-NN (CPU only).

The brute-force search *is* the definition, so it is pinned against things
outside the oracle: hand-worked cases, closed-form lattice neighbourhoods
with exact ties, and numpy's lexicographic sort on inputs whose squared
distances are exact in float32.  The kd-tree is then held bit-equal to it.
"""
import numpy as np
import pytest

from gen import lattice_cloud, rng_for, uniform_cloud


def test_hand_worked_line(oracle_mod):
    # points on the x axis at 0,1,2,3,5; query at 2.25 (all values exact)
    ref = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0], [5, 0, 0]], np.float32)
    q = np.array([[2.25, 0, 0]], np.float32)
    idx, d2 = oracle_mod.knn(ref, q, 5)
    # distances^2: 5.0625, 1.5625, 0.0625, 0.5625, 7.5625
    assert idx.tolist() == [[2, 3, 1, 0, 4]]
    assert d2.tolist() == [[0.0625, 0.5625, 1.5625, 5.0625, 7.5625]]


def test_hand_worked_tie_goes_to_lower_index(oracle_mod):
    # query exactly between points 3 and 1 (both at distance 1): lower index first
    ref = np.array([[9, 9, 9], [0, 1, 0], [5, 5, 5], [0, -1, 0]], np.float32)
    q = np.zeros((1, 3), np.float32)
    idx, d2 = oracle_mod.knn(ref, q, 2)
    assert idx.tolist() == [[1, 3]] and d2.tolist() == [[1.0, 1.0]]
    # a duplicate of the query point with a lower index beats the query itself
    ref = np.array([[1, 1, 1], [0, 0, 0], [0, 0, 0]], np.float32)
    idx, _ = oracle_mod.knn(ref, ref[2:3], 2)
    assert idx.tolist() == [[1, 2]]


def _lattice_expected(n, k):
    """Closed form for an n^3 unit lattice (index = x*n*n + y*n + z), k <= 7:
    the point itself at distance 0, then its face neighbours at distance 1
    in increasing index order (they tie exactly)."""
    out = []
    for x in range(n):
        for y in range(n):
            for z in range(n):
                i = x * n * n + y * n + z
                nb = []
                for dx, dy, dz in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
                    a, b, c = x + dx, y + dy, z + dz
                    if 0 <= a < n and 0 <= b < n and 0 <= c < n:
                        nb.append(a * n * n + b * n + c)
                out.append([i] + sorted(nb)[: k - 1])
    return out


@pytest.mark.parametrize("k", [1, 3, 4, 7])
def test_lattice_ties_closed_form(oracle_mod, k):
    n = 6
    pts = lattice_cloud(n)
    exp = _lattice_expected(n, k)
    idx, d2 = oracle_mod.knn(pts, pts, k)
    checked = 0
    for i, row in enumerate(exp):
        if len(row) == k:          # corners have only 3 face neighbours
            assert idx[i].tolist() == row
            assert d2[i, 0] == 0 and np.all(d2[i, 1:] == 1)
            checked += 1
    assert checked >= (n - 2) ** 3


def test_lattice_interior_k19(oracle_mod):
    # interior points: 1 self + 6 faces (d^2=1) + 12 edges (d^2=2) -> k=19 fully determined as a set
    n = 5
    pts = lattice_cloud(n)
    idx, d2 = oracle_mod.knn(pts, pts, 19)
    for x in range(1, n - 1):
        for y in range(1, n - 1):
            for z in range(1, n - 1):
                i = x * n * n + y * n + z
                faces, edges = [], []
                for dx in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dz in (-1, 0, 1):
                            s = abs(dx) + abs(dy) + abs(dz)
                            j = (x + dx) * n * n + (y + dy) * n + (z + dz)
                            if s == 1:
                                faces.append(j)
                            elif s == 2:
                                edges.append(j)
                assert idx[i].tolist() == [i] + sorted(faces) + sorted(edges)
                assert d2[i].tolist() == [0.0] + [1.0] * 6 + [2.0] * 12


def _exact_grid_cloud(rng, n):
    # coordinates j/64 with |j| <= 64: differences, squares and sums of three
    # squares are all exact in float32 and float64, so the float32 key equals
    # the true squared distance
    return (rng.integers(-64, 65, size=(n, 3)) / 64.0).astype(np.float32)


@pytest.mark.parametrize("k", [1, 5, 16, 32])
def test_brute_matches_numpy_lexsort(oracle_mod, k):
    rng = rng_for(100, k)
    ref = _exact_grid_cloud(rng, 700)
    qry = _exact_grid_cloud(rng, 200)
    idx, d2 = oracle_mod.knn(ref, qry, k)
    r64, q64 = ref.astype(np.float64), qry.astype(np.float64)
    for i in range(qry.shape[0]):
        dd = ((r64 - q64[i]) ** 2).sum(1)
        order = np.lexsort((np.arange(len(dd)), dd))[:k]
        assert idx[i].tolist() == order.tolist()
        assert np.array_equal(d2[i].astype(np.float64), dd[order])


def test_brute_key_is_float32_fma(oracle_mod):
    # the returned key is fmaf(dz,dz, fmaf(dy,dy, dx*dx)) of float32 differences;
    # with float64 products (exact for float32 inputs) and one final rounding
    # the value can differ only by double rounding, i.e. at most 1 ulp
    rng = rng_for(101)
    ref = uniform_cloud(rng, 300)
    qry = uniform_cloud(rng, 50)
    idx, d2 = oracle_mod.knn(ref, qry, 8)
    for i in range(qry.shape[0]):
        d = (ref[idx[i]] - qry[i]).astype(np.float32).astype(np.float64)
        ex = (d * d).sum(1).astype(np.float32)
        ulp = np.spacing(ex)
        assert np.all(np.abs(d2[i] - ex) <= ulp)
        assert np.all(np.diff(d2[i]) >= 0)


def _round_f32(x):
    """Exact rounding of a rational to the nearest float32 (ties to even),
    subnormals and overflow included, written out from the IEEE 754
    definition on exact fractions."""
    from fractions import Fraction
    if x == 0:
        return np.float32(0.0)
    sign = -1 if x < 0 else 1
    a = abs(Fraction(x))
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    q = max(e, -126) - 23                     # the float32 quantum at a
    m = a / Fraction(2) ** q
    n = m.numerator // m.denominator
    rem = m - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    v = Fraction(n) * Fraction(2) ** q
    if v > Fraction(int(np.finfo(np.float32).max)):
        return np.float32(sign * np.inf)
    return np.float32(sign * float(v))       # n has at most 24 bits: exact


def _key_exact(r, q):
    """The ranking key of the definition: float32 differences, then
    fmaf(dz, dz, fmaf(dy, dy, dx * dx)), each operation rounded once."""
    from fractions import Fraction
    F = Fraction
    dx, dy, dz = (_round_f32(F(float(r[a])) - F(float(q[a]))) for a in range(3))
    p = _round_f32(F(float(dx)) * F(float(dx)))
    s = _round_f32(F(float(dy)) * F(float(dy)) + F(float(p)))
    return _round_f32(F(float(dz)) * F(float(dz)) + F(float(s)))


def test_round_f32_against_numpy():
    # the exact rounding agrees with numpy's float64 -> float32 cast where
    # that cast is itself a single rounding (inputs exactly representable)
    rng = rng_for(103)
    x = rng.standard_normal(2000) * np.exp2(rng.integers(-140, 120, 2000))
    for v in x:
        assert _round_f32(float(v)) == np.float32(v) or (np.isinf(_round_f32(float(v))) and np.isinf(np.float32(v)))


@pytest.mark.parametrize("scale", [1e-3, 1.0, 37.0, 4e3])
def test_brute_key_bit_exact(oracle_mod, scale):
    # every key the oracle returns equals the exactly rounded sequence of
    # the definition, bit for bit (so ties, order and the k-th key are
    # pinned to the last bit), at several coordinate magnitudes
    rng = rng_for(104, int(scale * 1000))
    ref = (uniform_cloud(rng, 32) * np.float32(scale)).astype(np.float32)
    qry = (uniform_cloud(rng, 60, -1.3, 1.3) * np.float32(scale)).astype(np.float32)
    # a few queries sharing coordinates with reference points (exact zeros)
    qry[:4, :2] = ref[:4, :2]
    idx, d2 = oracle_mod.knn(ref, qry, 32)
    for i in range(qry.shape[0]):
        keys = np.array([_key_exact(ref[j], qry[i]) for j in range(32)], np.float32)
        order = sorted(range(32), key=lambda j: (keys[j], j))
        assert idx[i].tolist() == order
        assert np.array_equal(d2[i].view(np.uint32), keys[order].view(np.uint32))


@pytest.mark.parametrize("case", ["uniform", "clustered", "duplicates", "lattice", "plane"])
@pytest.mark.parametrize("k", [1, 10, 16, 32])
def test_kdtree_bit_equal_to_brute(oracle_mod, case, k):
    rng = rng_for(102, k)
    if case == "uniform":
        ref = uniform_cloud(rng, 3000)
        qry = uniform_cloud(rng, 500, -1.2, 1.2)
    elif case == "clustered":
        c = rng.normal(size=(20, 3))
        ref = (c[rng.integers(0, 20, 3000)] + 0.01 * rng.normal(size=(3000, 3))).astype(np.float32)
        qry = ref[rng.integers(0, 3000, 400)]
    elif case == "duplicates":
        base = uniform_cloud(rng, 300)
        ref = base[rng.integers(0, 300, 2000)]
        qry = base[:200]
    elif case == "lattice":
        ref = lattice_cloud(12, 0.5)
        qry = ref[rng.integers(0, ref.shape[0], 400)]
    else:
        xy = rng.uniform(-1, 1, size=(3000, 2))
        ref = np.column_stack([xy, np.zeros(3000)]).astype(np.float32)
        qry = ref[:300]
    a, da = oracle_mod.knn(ref, qry, k, "brute")
    b, db = oracle_mod.knn(ref, qry, k, "kdtree")
    assert np.array_equal(a, b)
    assert np.array_equal(da, db)


def test_self_query_first_when_tie_free(oracle_mod):
    rng = rng_for(103)
    pts = uniform_cloud(rng, 2000)
    idx, d2 = oracle_mod.knn(pts, pts, 4, "kdtree")
    assert np.array_equal(idx[:, 0], np.arange(2000))
    assert np.all(d2[:, 0] == 0)
