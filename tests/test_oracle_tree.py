"""Pins of the oracle's tree and cell properties (CPU only).

Tree: space-filling binary tree by bisecting the longest axis, buckets of at
most N_B particles (Sec. 2.2, 2.3).  Properties: volume-weighted density
sum(m)/sum(m/rho) (Sec. 2.3), centre of luminosity and far-vertex distance
(Sec. 2.2.1, 2.3), directional alpha_min / alpha_max (Sec. 2.2.3).
"""
import math

import numpy as np
import pytest

import _brute as B
from oracle.oracle import OracleTree


def _clustered(n, seed):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    # a tight cluster and exact duplicates exercise deep and depth-capped cells
    pos[: n // 8] = 0.3 + 1e-6 * rng.random((n // 8, 3))
    pos[n // 8: n // 8 + 12] = pos[0]
    rho = np.exp(rng.standard_normal(n))
    kappa = rng.uniform(0.5, 2.0, n)
    lum = np.where(rng.random(n) < 0.3, 10 ** rng.standard_normal(n), 0.0)
    mass = rng.uniform(0.5, 1.5, n)
    mass[rng.random(n) < 0.1] = 0.0  # pure sources, no absorbing mass
    return pos, rho, kappa, lum, mass


@pytest.mark.parametrize("nb", [1, 8])
@pytest.mark.parametrize("box", [((0, 0, 0), (1, 1, 1)), ((0, 0, 0), (2, 1, 1)),
                                 ((-1, 0, 0), (1, 0.5, 4))])
def test_tree_definition(nb, box):
    lo, hi = np.array(box[0], float), np.array(box[1], float)
    pos, rho, kappa, lum, mass = _clustered(3000, 11)
    pos = lo + pos * (hi - lo)
    t = OracleTree(pos, rho, kappa, lum, mass, lo, hi, nb)
    e = t.export()
    m = t.m
    assert sorted(e["perm"].tolist()) == list(range(3000))
    # level axes: longest width of the level's cell shape, ties to the lowest
    w = hi - lo
    for d in range(64):
        a = int(np.argmax(w))
        assert t.axes()[d] == a
        w[a] *= 0.5
    for i in range(m):
        leaf, cnt, dep = e["leaf"][i], e["count"][i], e["depth"][i]
        if leaf:
            assert cnt <= nb or dep == 63
            assert e["right"][i] == -1 and e["skip"][i] == i + 1
            ps = e["perm"][e["first"][i]: e["first"][i] + cnt]
            assert np.all(e["leaf_of"][ps] == i)
            for a in range(3):
                assert np.all(pos[ps, a] >= e["lo%d" % a][i])
                assert np.all(pos[ps, a] < e["hi%d" % a][i])
        else:
            assert cnt > nb and dep < 63
            l, r = i + 1, e["right"][i]
            assert e["parent"][l] == i and e["parent"][r] == i
            assert r == e["skip"][l]
            assert e["count"][l] + e["count"][r] == cnt
            assert e["first"][l] == e["first"][i]
            assert e["first"][r] == e["first"][i] + e["count"][l]
            a = e["axis"][i]
            s = 0.5 * (e["lo%d" % a][i] + e["hi%d" % a][i])
            assert e["split"][i] == s
            assert e["hi%d" % a][l] == s and e["lo%d" % a][r] == s
            for b in range(3):
                assert e["lo%d" % b][l] == e["lo%d" % b][i]
                assert e["hi%d" % b][r] == e["hi%d" % b][i]
                if b != a:
                    assert e["hi%d" % b][l] == e["hi%d" % b][i]
                    assert e["lo%d" % b][r] == e["lo%d" % b][i]
            assert e["depth"][l] == dep + 1
    # skip = pre-order index after the subtree
    size = np.ones(m, np.int64)
    for i in range(m - 1, -1, -1):
        if not e["leaf"][i]:
            size[i] = 1 + size[i + 1] + size[e["right"][i]]
    assert np.all(e["skip"] == np.arange(m) + size)
    # the path keys of the nodes are the prefixes of their particles' keys
    keys = B.path_keys(pos, lo, hi)
    order = np.lexsort((np.arange(3000), keys))
    assert np.array_equal(order, e["perm"])


@pytest.mark.parametrize("nb", [1, 3, 8])
def test_tree_matches_independent_splitter(nb):
    pos, rho, kappa, lum, mass = _clustered(2000, 5)
    lo, hi = np.zeros(3), np.array([2.0, 1.0, 0.5])
    pos = pos * hi
    t = OracleTree(pos, rho, kappa, lum, mass, lo, hi, nb)
    e = t.export()
    ref = B.split_tree(pos, nb, lo, hi, mass, rho, kappa)
    assert len(ref) == t.m
    for i, nd in enumerate(ref):  # both are in depth-first pre-order
        assert e["depth"][i] == nd["depth"]
        assert bool(e["leaf"][i]) == (nd["children"] is None)
        got = np.sort(e["perm"][e["first"][i]: e["first"][i] + e["count"][i]])
        assert np.array_equal(got, np.sort(nd["idx"]))
        for a in range(3):
            assert e["lo%d" % a][i] == nd["lo"][a] and e["hi%d" % a][i] == nd["hi"][a]
        assert math.isclose(e["alpha"][i], nd["alpha"], rel_tol=1e-13)


def test_properties_recomputed_per_node():
    pos, rho, kappa, lum, mass = _clustered(2500, 7)
    t = OracleTree(pos, rho, kappa, lum, mass, (0, 0, 0), (1, 1, 1), 8)
    e = t.export()
    for i in range(t.m):
        ps = e["perm"][e["first"][i]: e["first"][i] + e["count"][i]]
        ab = ps[mass[ps] > 0]
        A = np.sum(mass[ab] * kappa[ab])
        Bv = np.sum(mass[ab] / rho[ab])
        SL = np.sum(lum[ps])
        assert math.isclose(e["A"][i], A, rel_tol=1e-13, abs_tol=0)
        assert math.isclose(e["B"][i], Bv, rel_tol=1e-13, abs_tol=0)
        assert math.isclose(e["SL"][i], SL, rel_tol=1e-13, abs_tol=0)
        if Bv > 0:
            assert math.isclose(e["alpha"][i], A / Bv, rel_tol=1e-13)
        else:
            assert e["alpha"][i] == e["alpha"][e["parent"][i]]
        if SL > 0:
            xl = (lum[ps, None] * pos[ps]).sum(0) / SL
            lo = np.array([e["lo%d" % a][i] for a in range(3)])
            hi = np.array([e["hi%d" % a][i] for a in range(3)])
            verts = np.array([[(hi if (v >> a) & 1 else lo)[a] for a in range(3)] for v in range(8)])
            lfar = np.sqrt(np.max(np.sum((verts - xl) ** 2, axis=1)))
            assert math.isclose(e["lc"][i], SL, rel_tol=1e-13)
            for a in range(3):
                assert math.isclose(e["xl%d" % a][i], xl[a], rel_tol=1e-12, abs_tol=1e-15)
                assert lo[a] <= e["xl%d" % a][i] <= hi[a]
            assert math.isclose(e["lfar"][i], lfar, rel_tol=1e-12, abs_tol=1e-14)
        else:
            assert e["lc"][i] == 0.0
    # directional bounds from an independent recursion over the tree
    amin = np.zeros((t.m, 3))
    amax = np.zeros((t.m, 3))
    for i in range(t.m - 1, -1, -1):
        if e["leaf"][i]:
            amin[i] = amax[i] = e["alpha"][i]
        else:
            l, r, s = i + 1, e["right"][i], e["axis"][i]
            for b in range(3):
                if b == s:  # tau of both children over twice the width
                    amin[i, b] = (amin[l, b] * 1.0 + amin[r, b] * 1.0) / 2.0
                    amax[i, b] = (amax[l, b] + amax[r, b]) / 2.0
                else:
                    amin[i, b] = min(amin[l, b], amin[r, b])
                    amax[i, b] = max(amax[l, b], amax[r, b])
    assert np.array_equal(e["alpha_min"], amin.min(1))
    assert np.array_equal(e["alpha_max"], amax.max(1))
    assert np.array_equal(e["dalpha"], amax.max(1) - amin.min(1))
    # bounds bracket every cell average; leaves have no spread
    assert np.all(e["alpha_min"] <= e["alpha"] * (1 + 1e-15))
    assert np.all(e["alpha"] <= e["alpha_max"] * (1 + 1e-15))
    assert np.all(e["dalpha"][e["leaf"] == 1] == 0)


def _two(kappas, pts, nb=1):
    pts = np.asarray(pts, float)
    n = len(pts)
    return OracleTree(pts, np.ones(n), np.asarray(kappas, float), np.zeros(n),
                      np.ones(n), (0, 0, 0), (1, 1, 1), nb).export()


def test_alpha_bounds_hand_cases():
    # (i) two buckets side by side along x, alpha 1 and 3
    e = _two([1.0, 3.0], [[0.25, 0.5, 0.5], [0.75, 0.5, 0.5]])
    assert e["leaf"].tolist() == [0, 1, 1]
    assert e["alpha"][0] == 2.0
    assert e["alpha_min"][0] == 1.0 and e["alpha_max"][0] == 3.0 and e["dalpha"][0] == 2.0
    # (ii) checkerboard 1 3 / 3 1: x-split root, y-split children
    e = _two([1.0, 3.0, 3.0, 1.0], [[0.25, 0.25, 0.5], [0.25, 0.75, 0.5],
                                     [0.75, 0.25, 0.5], [0.75, 0.75, 0.5]])
    assert e["depth"].tolist() == [0, 1, 2, 2, 1, 2, 2]
    assert e["alpha_min"][0] == 1.0 and e["alpha_max"][0] == 3.0
    assert e["alpha_min"][1] == 1.0 and e["alpha_max"][1] == 3.0
    # a y-ray through the left column sees 1 then 3: mean 2 along y
    # (iii) stacked along y only (x-split root leaves one half empty)
    e = _two([1.0, 3.0], [[0.25, 0.25, 0.5], [0.25, 0.75, 0.5]])
    assert e["count"][0] == 2 and e["count"][1] == 2 and e["count"][e["right"][0]] == 0
    right = e["right"][0]
    assert e["leaf"][right] == 1 and e["alpha"][right] == e["alpha"][0] == 2.0
    # (iv) uniform medium: no spread anywhere
    rng = np.random.default_rng(3)
    n = 4096
    t = OracleTree(rng.random((n, 3)), np.ones(n), np.ones(n), np.zeros(n),
                   np.full(n, 2.0 ** -12), (0, 0, 0), (1, 1, 1), 8).export()
    assert np.all(t["dalpha"] == 0.0) and np.all(t["alpha"] == 1.0)


def test_mirror32_rounds_transport_only():
    pos, rho, kappa, lum, mass = _clustered(1000, 9)
    pos = pos.astype(np.float32).astype(np.float64)
    lum = lum.astype(np.float32).astype(np.float64)
    a = OracleTree(pos, rho, kappa, lum, mass, (0, 0, 0), (1, 1, 1), 8, mirror32=False).export()
    b = OracleTree(pos, rho, kappa, lum, mass, (0, 0, 0), (1, 1, 1), 8, mirror32=True).export()
    for k in a:
        assert np.array_equal(a[k], b[k])  # the binary64 tree is identical


def test_rejects_invalid_input():
    pos = np.array([[0.5, 0.5, 0.5], [1.0, 0.2, 0.2]])
    with pytest.raises(ValueError):
        OracleTree(pos, np.ones(2), np.ones(2), np.ones(2))
    pos = np.array([[0.5, 0.5, 0.5], [0.2, 0.2, 0.2]])
    with pytest.raises(ValueError):
        OracleTree(pos, np.array([1.0, 0.0]), np.ones(2), np.ones(2))
    with pytest.raises(ValueError):
        OracleTree(pos, np.ones(2), np.array([1.0, -1.0]), np.ones(2))
    with pytest.raises(ValueError):
        OracleTree(pos, np.ones(2), np.ones(2), np.array([1.0, np.nan]))
    # a massless particle may have any positive or zero density
    OracleTree(pos, np.array([1.0, 0.0]), np.ones(2), np.ones(2), mass=np.array([1.0, 0.0]))
