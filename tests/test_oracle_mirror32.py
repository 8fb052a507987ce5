"""Pins of the oracle's binary32 mirror mode (CPU only).

In binary32 transport the library stores the values its walk reads rounded
once (round to nearest even) from the binary64 build values, computes each
ray's geometry -- direction, 1/d, r^2, r, plane crossings
t = (s - x) (1/d), piece lengths l = r (t_b - t_a) -- in binary32, and forms
the refinement criterion's product and every term alpha l as exact binary64
products, summed in binary64.  The oracle's mirror mode must do exactly that:

  * every transport field equals binary32 of its binary64 value -- the cell
    box, split plane, centre of luminosity, luminosity, far-vertex distance,
    alpha, and the spread alpha_max - alpha_min rounded from its binary64
    value (not the difference of the rounded bounds); positions and
    luminosities are the binary32 inputs;
  * optically thin, theta_open = 0: the all-pairs sum of L / (4 pi r^2) with
    r^2 the binary32 sum of binary32 squares of binary32 differences
    (eq. simpint), to 1e-13;
  * theta_open = 0 with refinement always on: the pieces are the buckets the
    segment crosses, each from the largest binary32 crossing of its entry
    faces to the smallest of its exit faces (clamped to [0, 1]), l the
    binary32 r (t_b - t_a), alpha the bucket's binary32 alpha (brute force over
    buckets, eq. tauint), to 1e-12;
  * uniform medium with kappa rho exact in binary32: the binary32 pieces tile
    the ray, so tau = kappa rho r to within the rounding of r and of each
    piece (6 units of 2^-24 plus a margin);
  * tau_ref = infinity: the walk-up field with binary32 alphas (brute force),
    to within the shift of each piece boundary by binary32 rounding;
  * against the binary64 oracle on the same binary32-valued inputs at
    theta_open = 0 and tau_ref < 0 (the same refinement), each ray's tau
    differs by no more than binary32 rounding allows: 2^-24 tau from alpha,
    and from the geometry 7 u tau plus 5 u r times the total variation of
    alpha along the ray (u = 2^-24);
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
U = 2.0 ** -24


def _r2_f32(x, y):
    """r^2 of the segment x -> y as binary32 does it: binary32 differences,
    squares and sums, ((d0 d0 + d1 d1) + d2 d2)."""
    d = np.asarray(y, np.float32) - np.asarray(x, np.float32)
    dd = d * d
    return (dd[..., 0] + dd[..., 1]) + dd[..., 2], d


def _all_pairs_f32(pos, lum, sinks=None):
    """sum over other sources of L / (4 pi r^2), r^2 in binary32."""
    p32 = np.asarray(pos, np.float32)
    l32 = F32(lum)
    src = np.nonzero(l32 > 0)[0]
    sinks = np.arange(p32.shape[0]) if sinks is None else np.asarray(sinks)
    out = np.zeros(sinks.size)
    for q, i in enumerate(sinks):
        r2, _ = _r2_f32(p32[i], p32[src])
        ok = r2 > 0
        out[q] = np.sum(l32[src][ok] / (4.0 * math.pi * r2[ok].astype(np.float64)))
    return out


def _leaf_pieces_f32(x, y, leaf_lo, leaf_hi):
    """Each bucket's piece of the segment x -> y in binary32: t = (face - x)
    (1/d) per face, entry the largest entry crossing (and 0), exit the smallest
    exit crossing (and 1); l = r (t_b - t_a).  Returns (t_a, t_b, l) per bucket
    (l = 0 where not crossed)."""
    x32 = np.asarray(x, np.float32)
    r2, d = _r2_f32(x32, np.asarray(y, np.float32))
    assert np.all(d != 0)
    inv = np.float32(1.0) / d
    r = np.sqrt(r2)
    lo = np.asarray(leaf_lo, np.float32)
    hi = np.asarray(leaf_hi, np.float32)
    t_lo = (lo - x32) * inv
    t_hi = (hi - x32) * inv
    ent = np.where(d > 0, t_lo, t_hi)
    ext = np.where(d > 0, t_hi, t_lo)
    ta = np.maximum(np.float32(0), ent.max(axis=1))
    tb = np.minimum(np.float32(1), ext.min(axis=1))
    l = np.where(tb > ta, r * (tb - ta), np.float32(0))
    return ta, tb, l.astype(np.float64), float(r)


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
    ref = _all_pairs_f32(pos, lum)
    np.testing.assert_allclose(F, ref, rtol=1e-13, atol=0)
    # binary64 geometry on the rounded inputs is farther away than that, and
    # so are the unrounded inputs: the test sees each rounding
    assert np.max(np.abs(B.all_pairs_flux(F32(pos), F32(lum)) / F - 1.0)) > 1e-9
    assert np.max(np.abs(B.all_pairs_flux(pos, lum) / F - 1.0)) > 1e-9
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
        # binary32 r: 3.5 u; each piece r (t_b - t_a): 2 u; the pieces tile [0, 1]
        np.testing.assert_allclose(log["tau"], kr * r, rtol=8 * U, atol=1e-15)
    if theta == 0.0:
        s = np.arange(0, n, 41)
        F, _ = t.flux(theta, tau_ref, sinks=s)
        rmax = math.sqrt(3.0)
        ref = B.all_pairs_flux(p32, F32(lum), kr, sinks=s)
        np.testing.assert_allclose(F, ref, rtol=8 * U * (1 + kr * rmax) + 4 * U)


def _leaf_field(pos32, nb, mass, rho, kappa, round_alpha):
    ref = B.split_tree(pos32, nb, np.zeros(3), np.ones(3), mass, rho, kappa)
    if round_alpha:
        for nd in ref:
            nd["alpha"] = float(np.float32(nd["alpha"]))
    return ref


@pytest.mark.parametrize("nb", [1, 6])
def test_mirror32_full_limit_binary32_leaf_pieces(nb):
    pos, rho, kappa, lum, mass = _field(300, 34, 60)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=nb, mirror32=True)
    p32, l32 = F32(pos), F32(lum)
    ref = _leaf_field(p32, nb, mass, rho, kappa, round_alpha=True)
    lv = B.leaves(ref)
    llo = np.array([nd["lo"] for nd in lv])
    lhi = np.array([nd["hi"] for nd in lv])
    assert np.array_equal(F32(llo), llo) and np.array_equal(F32(lhi), lhi)
    lal = np.array([nd["alpha"] for nd in lv])
    lal64 = np.array([nd["alpha"] for nd in B.leaves(
        _leaf_field(p32, nb, mass, rho, kappa, round_alpha=False))])
    F, C = t.flux(0.0, -1.0)
    worst_alpha = worst_geom = 0.0
    for i in range(0, 300, 7):
        log = t.ray_log(0.0, -1.0, i)
        f = 0.0
        nseg = 0
        for src, tau in zip(log["src"], log["tau"]):
            _, _, l, _ = _leaf_pieces_f32(p32[i], p32[src], llo, lhi)
            ex = float(np.sum(lal * l))
            assert math.isclose(tau, ex, rel_tol=1e-12, abs_tol=1e-14)
            # binary64 alphas, or binary64 geometry, would not pass that check
            worst_alpha = max(worst_alpha, abs(tau - float(np.sum(lal64 * l))) / tau)
            ex64, _ = B.exact_tau_leaf_field(p32[i], p32[src], llo, lhi, lal)
            worst_geom = max(worst_geom, abs(tau - ex64) / tau)
            nseg += int(np.count_nonzero(l > 0))
            r2, _ = _r2_f32(p32[i], p32[src])
            f += l32[src] * math.exp(-ex) / (4 * math.pi * float(r2))
        assert C[i, 3] == nseg
        assert math.isclose(F[i], f, rel_tol=1e-12)
    assert worst_alpha > 1e-10 and worst_geom > 1e-10


@pytest.mark.parametrize("theta", [0.0, 0.75])
def test_mirror32_never_refine_limit(theta):
    pos, rho, kappa, lum, mass = _field(400, 35, 80)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=4, mirror32=True)
    p32 = F32(pos)
    e = t.export()
    ref = _leaf_field(p32, 4, mass, rho, kappa, round_alpha=True)
    assert len(ref) == t.m
    amax = max(nd["alpha"] for nd in ref)
    worst = 0.0
    for i in range(0, 400, 13):
        log = t.ray_log(theta, math.inf, i)
        S = e["leaf_of"][i]
        C_ = t.flux(theta, math.inf, sinks=[i])[1][0]
        for C, y, tau in zip(log["C"], log["y"], log["tau"]):
            ex = B.walk_up_tau(ref, S, C, p32[i], y)
            r = float(np.linalg.norm(y - p32[i]))
            # each piece boundary t moves by at most 4 u, each length by 5.5 u
            bound = 6 * U * ex + 2 * 4 * U * r * amax * (C_[3] + 2)
            assert abs(tau - ex) <= bound, (tau, ex, bound)
            worst = max(worst, abs(tau - ex) / ex)
    assert worst > 1e-12


def test_mirror32_against_binary64_within_binary32_rounding():
    pos, rho, kappa, lum, mass = _field(800, 36, 200, f32_pos=True)
    lum = F32(lum)
    o32 = OracleTree(pos, rho, kappa, lum, mass, bucket_size=8, mirror32=True)
    o64 = OracleTree(pos, rho, kappa, lum, mass, bucket_size=8, mirror32=False)
    ref = _leaf_field(pos, 8, mass, rho, kappa, round_alpha=False)
    lv = B.leaves(ref)
    llo = np.array([nd["lo"] for nd in lv])
    lhi = np.array([nd["hi"] for nd in lv])
    lal = np.array([nd["alpha"] for nd in lv])
    worst = 0.0
    for i in range(0, 800, 23):
        g32 = o32.ray_log(0.0, -1.0, i)
        g64 = o64.ray_log(0.0, -1.0, i)
        assert np.array_equal(g32["src"], g64["src"])  # theta 0: the same rays
        for src, t32, t64 in zip(g32["src"], g32["tau"], g64["tau"]):
            ta, tb, l, r = _leaf_pieces_f32(pos[i], pos[src], llo, lhi)
            on = l > 0
            a_seq = lal[on][np.argsort(ta[on])]
            tv = float(np.sum(np.abs(np.diff(np.r_[0.0, a_seq, 0.0]))))
            bound = U * t64 + 7 * U * t64 + 5 * U * r * tv + 1e-15
            assert abs(t32 - t64) <= bound, (t32, t64, bound)
            worst = max(worst, abs(t32 - t64) / t64)
    assert worst > 1e-12  # the mirror does round


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
