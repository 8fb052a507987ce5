"""Pins of the oracle's walk variants (CPU only).

  * per-bucket opening: every other source is covered exactly once; each
    merged cell passes eq. openangle with r measured from the sink's bucket
    box, and each of its ancestors fails it; two sinks of one bucket merge the
    same cells;
  * Gasoline's opening radius: coverage as above; each merged cell lies
    outside r_open = 2 l_far / (sqrt(3) theta) of its x_L and does not hold the
    sink, and each ancestor fails that;
  * top-down ray walk: with tau_ref = infinity every ray's tau is the meeting
    cell's alpha times r (brute-force lowest common ancestor); with tau_ref < 0
    it is the walk-up trace's fully refined tau; in a uniform medium it is
    kappa rho r;
  * early termination: the flux is the ray log's sum over rays with
    tau <= tau_max, and tau_max = infinity is the plain flux bit for bit.
"""
import math

import numpy as np
import pytest

from oracle.oracle import OracleTree


def _rand(n, seed, n_src=None):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    rho = np.exp(0.8 * rng.standard_normal(n))
    kappa = rng.uniform(0.2, 3.0, n)
    lum = np.zeros(n)
    src = rng.choice(n, size=n if n_src is None else n_src, replace=False)
    lum[src] = 10 ** (0.5 * rng.standard_normal(src.size))
    mass = rng.uniform(0.5, 1.5, n)
    return pos, rho, kappa, lum, mass


def _box(e, c):
    return (np.array([e["lo%d" % a][c] for a in range(3)]),
            np.array([e["hi%d" % a][c] for a in range(3)]))


def _gap(lo1, hi1, lo2, hi2):
    g = np.maximum(np.maximum(lo1 - hi2, lo2 - hi1), 0.0)
    return float(np.sqrt(g @ g))


def _coverage(t, e, lum, i, log, n):
    covered = np.zeros(n, int)
    for C, src in zip(log["C"], log["src"]):
        if src >= 0:
            covered[src] += 1
        else:
            covered[e["perm"][e["first"][C]: e["first"][C] + e["count"][C]]] += 1
    others = (lum > 0) & (np.arange(n) != i)
    assert np.all(covered[others] == 1) and covered[i] == 0 and np.all(covered <= 1)


@pytest.mark.parametrize("theta", [0.5, 0.75, 1.0])
def test_bucket_opening(theta):
    n = 3000
    pos, rho, kappa, lum, mass = _rand(n, 41, n_src=n)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=8)
    e = t.export()
    merged = {}
    for i in (0, 17, 1234, 2999):
        log = t.ray_log_variant(theta, 0.1, i, open_mode=1)
        _coverage(t, e, lum, i, log, n)
        S = e["leaf_of"][i]
        slo, shi = _box(e, S)
        for C in log["C"][log["src"] < 0]:
            lo, hi = _box(e, C)
            assert e["lfar"][C] < theta * _gap(lo, hi, slo, shi)
            p = e["parent"][C]
            while p >= 0:
                lo, hi = _box(e, p)
                assert not (e["lfar"][p] < theta * _gap(lo, hi, slo, shi))
                p = e["parent"][p]
        merged[i] = set(log["C"][log["src"] < 0].tolist())
    # another sink of sink 17's bucket merges the same cells
    S = e["leaf_of"][17]
    mates = [j for j in e["perm"][e["first"][S]: e["first"][S] + e["count"][S]] if j != 17]
    assert mates
    log = t.ray_log_variant(theta, 0.1, mates[0], open_mode=1)
    assert set(log["C"][log["src"] < 0].tolist()) == merged[17]


@pytest.mark.parametrize("theta", [0.5, 0.75, 1.0])
def test_gasoline_opening(theta):
    n = 3000
    pos, rho, kappa, lum, mass = _rand(n, 42, n_src=n)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=8)
    e = t.export()

    def accepts(c, xi):
        lo, hi = _box(e, c)
        inside = np.all(xi >= lo) and np.all(xi <= hi)
        xl = np.array([e["xl%d" % a][c] for a in range(3)])
        d = np.linalg.norm(xi - xl)
        return (not inside) and d > 2.0 * e["lfar"][c] / (math.sqrt(3.0) * theta)

    for i in (3, 555, 2100):
        log = t.ray_log_variant(theta, 0.1, i, open_mode=2)
        _coverage(t, e, lum, i, log, n)
        for C in log["C"][log["src"] < 0]:
            assert accepts(C, pos[i])
            p = e["parent"][C]
            while p >= 0:
                assert not accepts(p, pos[i])
                p = e["parent"][p]


def _lca(e, a, b):
    anc = set()
    while a >= 0:
        anc.add(int(a))
        a = e["parent"][a]
    while int(b) not in anc:
        b = e["parent"][b]
    return int(b)


@pytest.mark.parametrize("theta", [0.0, 0.75])
def test_top_down_walk(theta):
    n = 2500
    pos, rho, kappa, lum, mass = _rand(n, 43, n_src=400)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=8)
    e = t.export()
    for i in (0, 99, 2400):
        S = e["leaf_of"][i]
        log = t.ray_log_variant(theta, math.inf, i, ray_mode=1)
        r = np.linalg.norm(log["y"] - pos[i], axis=1)
        for C, tau, rr in zip(log["C"], log["tau"], r):
            A = _lca(e, S, C)
            assert abs(tau - e["alpha"][A] * rr) <= 1e-13 * max(1.0, tau)
        full_td = t.ray_log_variant(theta, -1.0, i, ray_mode=1)
        full_up = t.ray_log(theta, -1.0, i)
        np.testing.assert_allclose(full_td["tau"], full_up["tau"], rtol=1e-12, atol=1e-15)
    # uniform medium: kappa rho r for every ray at any tau_ref
    m = 4096
    rng = np.random.default_rng(9)
    p2 = rng.random((m, 3))
    l2 = np.where(rng.random(m) < 0.25, rng.uniform(0.5, 1.0, m), 0.0)
    t2 = OracleTree(p2, np.ones(m), np.full(m, 2.5), l2, np.full(m, 2.0 ** -12))
    for tau_ref in (0.0, 0.1, math.inf):
        log = t2.ray_log_variant(theta, tau_ref, 5, ray_mode=1)
        r = np.linalg.norm(log["y"] - p2[5], axis=1)
        np.testing.assert_allclose(log["tau"], 2.5 * r, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("tau_max", [0.5, 1.5, 3.0])
def test_early_termination(tau_max):
    n = 3000
    pos, rho, kappa, lum, mass = _rand(n, 44, n_src=600)
    kappa *= 3.0
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=8)
    sinks = np.array([1, 400, 1999, 2998])
    F, C = t.flux_variant(0.75, 0.1, tau_max=tau_max, sinks=sinks)
    F0, C0 = t.flux(0.75, 0.1, sinks=sinks)
    assert np.array_equal(C, C0)
    cut = 0
    for q, i in enumerate(sinks):
        log = t.ray_log(0.75, 0.1, i)
        keep = log["tau"] <= tau_max
        assert keep.sum() > 0
        cut += keep.size - keep.sum()
        assert abs(F[q] - log["f"][keep].sum()) <= 1e-13 * F0[q]
    assert cut > 0
    Fi, Ci = t.flux_variant(0.75, 0.1, tau_max=math.inf, sinks=sinks)
    assert np.array_equal(Fi, F0) and np.array_equal(Ci, C0)
    # the other variants with their defaults are the plain flux, bit for bit
    Fd, Cd = t.flux_variant(0.75, 0.1, sinks=sinks)
    assert np.array_equal(Fd, F0) and np.array_equal(Cd, C0)
