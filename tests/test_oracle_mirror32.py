"""Pins of the oracle's binary32 mirror mode (CPU only).

In binary32 transport the library stores the values its walk reads rounded
once (round to nearest even) from the binary64 build values, and does every
operation in binary64.  The oracle's mirror mode must read exactly those
values:

  * every transport field equals binary32 of its binary64 value -- the cell
    box, split plane, centre of luminosity, luminosity, far-vertex distance,
    alpha, and the spread alpha_max - alpha_min rounded from its binary64
    value (not the difference of the rounded bounds); positions and
    luminosities are the binary32 inputs;
  * optically thin, theta_open = 0: the all-pairs sum of L / (4 pi r^2) over
    the binary32 positions and luminosities (eq. simpint);
  * uniform medium with kappa rho exact in binary32: tau = kappa rho r per ray;
  * theta_open = 0 with refinement always on: tau is the exact integral of the
    bucket-wise constant field, each bucket at binary32 of its alpha (brute
    force over buckets);
  * tau_ref = infinity: the walk-up field with binary32 alphas (brute force);
  * against the binary64 oracle on the same binary32-valued inputs at
    theta_open = 0 and tau_ref < 0 (identical decisions), the flux differs by
    no more than the rounding of alpha allows: |tau32 - tau64| <= 2^-24 tau,
    so |F32 / F64 - 1| <= exp(2^-24 tau_max) - 1;
  * every merged cell passes eq. openangle, and each of its ancestors fails
    it, on the binary32 values; every unrefined piece of a cell that is not a
    bucket passes eq. refcrit with the binary32 spread.
Each brute-force reference is built from the rounded inputs by numpy, with no
call into the oracle.
"""
import math

import numpy as np
import pytest

import _brute as B
from oracle.oracle import OracleTree, TRANSPORT_FIELDS

F32 = lambda a: np.asarray(a, np.float64).astype(np.float32).astype(np.float64)  # noqa: E731


def _field(n, seed, n_src, f32_pos=False):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    pos[: n // 10] = 0.6 + 0.01 * rng.random((n // 10, 3))  # a cluster: deep cells
    if f32_pos:
        pos = F32(pos)
    rho = np.exp(0.9 * rng.standard_normal(n))
    kappa = rng.uniform(0.2, 3.0, n)
    lum = np.zeros(n)
    src = rng.choice(n, size=n_src, replace=False)
    lum[src] = 10 ** (0.5 * rng.standard_normal(n_src))
    mass = rng.uniform(0.5, 1.5, n)
    mass[rng.random(n) < 0.05] = 0.0  # pure sources: empty cells inherit alpha
    return pos, rho, kappa, lum, mass


@pytest.mark.parametrize("box", [((0, 0, 0), (1, 1, 1)), ((-0.3, 0, 0.1), (1.7, 1.1, 0.9))])
def test_transport_fields_are_binary32_of_binary64(box):
    lo, hi = np.array(box[0], float), np.array(box[1], float)
    pos, rho, kappa, lum, mass = _field(3000, 31, 700)
    pos = lo + pos * (hi - lo)
    m32 = OracleTree(pos, rho, kappa, lum, mass, lo, hi, 8, mirror32=True)
    e = m32.export()  # binary64 cell values (the build is identical in both modes)
    t = m32.export_transport()
    for f in TRANSPORT_FIELDS:
        assert np.array_equal(t[f], F32(e[f])), f
    assert np.array_equal(t["pos"], F32(pos))
    assert np.array_equal(t["lum"], F32(lum))
    # the spread is rounded from its binary64 value: the plausible alternative,
    # the difference of the rounded bounds, differs in many cells here
    alt = F32(e["alpha_max"]) - F32(e["alpha_min"])
    assert np.count_nonzero(alt != t["dalpha"]) > 50
    # binary64 mode reads the build's own values
    m64 = OracleTree(F32(pos), rho, kappa, F32(lum), mass, lo, hi, 8, mirror32=False)
    e64, t64 = m64.export(), m64.export_transport()
    for f in TRANSPORT_FIELDS:
        assert np.array_equal(t64[f], e64[f]), f
    # the mirror builds its tree from the binary32 positions
    for f in ("perm", "first", "count", "right", "lo0", "hi2", "alpha", "dalpha"):
        assert np.array_equal(e64[f], e[f]), f


def test_mirror32_thin_all_pairs():
    pos, rho, kappa, lum, mass = _field(1200, 32, 300)
    t = OracleTree(pos, rho, 0 * kappa, lum, mass, bucket_size=8, mirror32=True)
    F, C = t.flux(0.0, 0.1)
    ref = B.all_pairs_flux(F32(pos), F32(lum))
    np.testing.assert_allclose(F, ref, rtol=1e-13, atol=0)
    # the unrounded sum is farther away than that: the test sees the rounding
    raw = B.all_pairs_flux(pos, lum)
    assert np.max(np.abs(raw / F - 1.0)) > 1e-9
    assert np.array_equal(C[:, 1], C[:, 2])


@pytest.mark.parametrize("theta,tau_ref", [(0.0, 0.1), (0.5, -1.0), (0.75, 0.1), (1.0, math.inf)])
def test_mirror32_uniform_medium(theta, tau_ref):
    rng = np.random.default_rng(33)
    n = 3000
    pos = rng.random((n, 3))
    lum = np.where(rng.random(n) < 0.3, rng.uniform(0.5, 1.0, n), 0.0)
    kr = 2.5  # kappa rho, exact in binary32
    t = OracleTree(pos, np.ones(n), np.full(n, kr), lum, np.full(n, 2.0 ** -12), mirror32=True)
    p32 = F32(pos)
    for i in (0, 9, 1500, 2999):
        log = t.ray_log(theta, tau_ref, i)
        r = np.linalg.norm(log["y"] - p32[i], axis=1)
        np.testing.assert_allclose(log["tau"], kr * r, rtol=1e-13, atol=1e-15)
    if theta == 0.0:
        s = np.arange(0, n, 41)
        F, _ = t.flux(theta, tau_ref, sinks=s)
        np.testing.assert_allclose(F, B.all_pairs_flux(p32, F32(lum), kr, sinks=s), rtol=1e-12)


def _leaf_field(pos32, nb, mass, rho, kappa, round_alpha):
    ref = B.split_tree(pos32, nb, np.zeros(3), np.ones(3), mass, rho, kappa)
    if round_alpha:
        for nd in ref:
            nd["alpha"] = float(np.float32(nd["alpha"]))
    return ref


@pytest.mark.parametrize("nb", [1, 6])
def test_mirror32_full_limit_exact_leaf_integration(nb):
    pos, rho, kappa, lum, mass = _field(300, 34, 60)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=nb, mirror32=True)
    p32, l32 = F32(pos), F32(lum)
    ref = _leaf_field(p32, nb, mass, rho, kappa, round_alpha=True)
    lv = B.leaves(ref)
    llo = np.array([nd["lo"] for nd in lv])
    lhi = np.array([nd["hi"] for nd in lv])
    lal = np.array([nd["alpha"] for nd in lv])
    lal64 = np.array([nd["alpha"] for nd in B.leaves(
        _leaf_field(p32, nb, mass, rho, kappa, round_alpha=False))])
    F, C = t.flux(0.0, -1.0)
    worst64 = 0.0
    for i in range(0, 300, 7):
        log = t.ray_log(0.0, -1.0, i)
        f = 0.0
        nseg = 0
        for src, tau in zip(log["src"], log["tau"]):
            ex, k = B.exact_tau_leaf_field(p32[i], p32[src], llo, lhi, lal)
            assert math.isclose(tau, ex, rel_tol=1e-12, abs_tol=1e-14)
            ex64, _ = B.exact_tau_leaf_field(p32[i], p32[src], llo, lhi, lal64)
            worst64 = max(worst64, abs(tau - ex64) / ex64)
            nseg += k
            f += l32[src] * math.exp(-ex) / (4 * math.pi * np.sum((p32[src] - p32[i]) ** 2))
        assert C[i, 3] == nseg
        assert math.isclose(F[i], f, rel_tol=1e-12)
    assert worst64 > 1e-10  # the binary64 alphas would not pass the 1e-12 check


@pytest.mark.parametrize("theta", [0.0, 0.75])
def test_mirror32_never_refine_limit(theta):
    pos, rho, kappa, lum, mass = _field(400, 35, 80)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=4, mirror32=True)
    p32 = F32(pos)
    e = t.export()
    ref = _leaf_field(p32, 4, mass, rho, kappa, round_alpha=True)
    assert len(ref) == t.m
    for i in range(0, 400, 13):
        log = t.ray_log(theta, math.inf, i)
        S = e["leaf_of"][i]
        for C, y, tau in zip(log["C"], log["y"], log["tau"]):
            ex = B.walk_up_tau(ref, S, C, p32[i], y)
            assert math.isclose(tau, ex, rel_tol=1e-12, abs_tol=1e-14)


def test_mirror32_against_binary64_within_alpha_rounding():
    pos, rho, kappa, lum, mass = _field(1500, 36, 400, f32_pos=True)
    lum = F32(lum)
    sinks = np.arange(0, 1500, 5)
    o32 = OracleTree(pos, rho, kappa, lum, mass, bucket_size=8, mirror32=True)
    o64 = OracleTree(pos, rho, kappa, lum, mass, bucket_size=8, mirror32=False)
    F32_, C32 = o32.flux(0.0, -1.0, sinks=sinks)
    F64_, C64, G = o64.flux(0.0, -1.0, sinks=sinks, with_g=True)
    assert np.array_equal(C32, C64)  # theta 0 and tau_ref < 0: no decision depends on rounding
    rel = np.abs(F32_ / F64_ - 1.0)
    taus = np.concatenate([o64.ray_log(0.0, -1.0, int(i))["tau"] for i in sinks])
    bound = math.expm1(2.0 ** -24 * float(np.max(taus))) + 1e-14
    assert np.all(rel <= bound), (rel.max(), bound)
    assert rel.max() > 1e-12  # the mirror does round alpha


@pytest.mark.parametrize("theta,tau_ref", [(0.5, 0.05), (0.75, 0.1), (1.0, 0.3)])
def test_mirror32_decisions_use_binary32_values(theta, tau_ref):
    pos, rho, kappa, lum, mass = _field(2500, 37, 2500)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=8, mirror32=True)
    e = t.export()
    tt = t.export_transport()
    p32 = F32(pos)
    lo = np.stack([F32(e["lo%d" % a]) for a in range(3)], 1)
    hi = np.stack([F32(e["hi%d" % a]) for a in range(3)], 1)
    xl = np.stack([F32(e["xl%d" % a]) for a in range(3)], 1)
    lfar, lc, dal = F32(e["lfar"]), F32(e["lc"]), F32(e["dalpha"])

    def rdist(c, x):
        g = np.maximum(np.maximum(lo[c] - x, x - hi[c]), 0.0)
        return (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]

    pieces = 0
    for i in (1, 333, 1700, 2499):
        x = p32[i]
        log = t.ray_log(theta, tau_ref, i)
        for k, (C, src, y, L) in enumerate(zip(log["C"], log["src"], log["y"], log["L"])):
            if src < 0:  # a merged cell: its binary32 point and luminosity
                assert np.array_equal(y, xl[C]) and L == lc[C]
                assert lfar[C] * lfar[C] < theta * theta * rdist(C, x)
                p = e["parent"][C]
                while p >= 0:
                    assert not (lfar[p] * lfar[p] < theta * theta * rdist(p, x))
                    p = e["parent"][p]
            else:
                assert np.array_equal(y, p32[src]) and L == F32(lum)[src]
            if k % 17 == 0:
                pc = t.ray_pieces(theta, tau_ref, i, k)
                for nd, ln in zip(pc["node"], pc["len"]):
                    assert e["leaf"][nd] or not (dal[nd] * ln > tau_ref)
                    pieces += 1
    assert pieces > 100
    assert np.array_equal(tt["dalpha"], dal)
