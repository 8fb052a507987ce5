"""Pins of the oracle's per-sink flux against what the paper and the
mathematics fix (CPU only).

  * optically thin: kappa = 0 gives tau = 0, and theta_open = 0 gives the
    all-pairs sum of L / (4 pi r^2) (eq. simpint summed over sources);
  * uniform medium: every cell has alpha = kappa rho and no spread, so every
    ray has tau = kappa rho r at any theta_open and tau_ref (eqs. taui, tausum);
  * theta_open = 0 with refinement always on: tau is the exact integral of the
    bucket-wise constant field along the segment (eq. tauint), brute force;
  * an emitting thin shell: the closed form of the shell flux;
  * source merging covers every source exactly once (Sec. 2.2.1);
  * the refinement bound, eq. (reffrac);
  * the Stromgren radius and photon balance of an equilibrium H II region.
"""
import math

import numpy as np
import pytest

import _brute as B
from oracle.oracle import OracleTree
from paper_1902_08083_amd import workloads as W


def _rand(n, seed, n_src=None, kappa_law="random"):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    if kappa_law == "random":
        rho = np.exp(0.8 * rng.standard_normal(n))
        kappa = rng.uniform(0.2, 3.0, n)
    else:
        rho = np.ones(n)
        kappa = np.ones(n)
    lum = np.zeros(n)
    src = rng.choice(n, size=n if n_src is None else n_src, replace=False)
    lum[src] = 10 ** (0.5 * rng.standard_normal(src.size))
    mass = rng.uniform(0.5, 1.5, n)
    return pos, rho, kappa, lum, mass


@pytest.mark.parametrize("theta", [0.0])
def test_thin_all_pairs_closed_form(theta):
    pos, rho, kappa, lum, mass = _rand(1500, 21, n_src=300)
    pos[7] = pos[3]  # a coincident pair is skipped, not divided by zero
    t = OracleTree(pos, rho, 0 * kappa, lum, mass, bucket_size=8)
    F, C = t.flux(theta, 0.1)
    ref = B.all_pairs_flux(pos, lum)
    np.testing.assert_allclose(F, ref, rtol=1e-13, atol=0)
    n_src = np.count_nonzero(lum > 0)
    self_src = (lum > 0).astype(int)
    self_src[7] = self_src[3] = int(lum[3] > 0) + int(lum[7] > 0)
    assert np.array_equal(C[:, 1], n_src - self_src)  # every other source is a ray
    assert np.array_equal(C[:, 1], C[:, 2])


@pytest.mark.parametrize("theta", [0.3, 0.75, 1.0])
def test_merging_covers_every_source_once(theta):
    pos, rho, kappa, lum, mass = _rand(3000, 4, n_src=3000)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=8)
    e = t.export()
    for i in (0, 17, 1234, 2999):
        log = t.ray_log(theta, 0.1, i)
        covered = np.zeros(3000, int)
        xi = pos[i]
        for C, src, y, L in zip(log["C"], log["src"], log["y"], log["L"]):
            if src >= 0:
                covered[src] += 1
                assert L == lum[src] and np.array_equal(y, pos[src])
            else:
                ps = e["perm"][e["first"][C]: e["first"][C] + e["count"][C]]
                covered[ps] += 1
                assert L == e["lc"][C]
                assert np.array_equal(y, [e["xl0"][C], e["xl1"][C], e["xl2"][C]])
                lo = np.array([e["lo%d" % a][C] for a in range(3)])
                hi = np.array([e["hi%d" % a][C] for a in range(3)])
                r = np.linalg.norm(np.maximum(np.maximum(lo - xi, xi - hi), 0))
                assert e["lfar"][C] < theta * r  # eq. openangle holds for merged cells
                # and failed for every ancestor (parents of the sink always open)
                p = e["parent"][C]
                while p >= 0:
                    lo = np.array([e["lo%d" % a][p] for a in range(3)])
                    hi = np.array([e["hi%d" % a][p] for a in range(3)])
                    rp = np.linalg.norm(np.maximum(np.maximum(lo - xi, xi - hi), 0))
                    assert not (e["lfar"][p] < theta * rp)
                    p = e["parent"][p]
        others = (lum > 0) & (np.arange(3000) != i)
        assert np.all(covered[others] == 1)  # every other source exactly once
        assert covered[i] == 0  # cells holding the sink are never merged
        assert np.all(covered <= 1)


@pytest.mark.parametrize("theta,tau_ref", [(0.0, 0.1), (0.5, -1.0), (0.75, 0.1), (1.0, 0.0),
                                           (0.75, math.inf)])
def test_uniform_medium_every_ray(theta, tau_ref):
    rng = np.random.default_rng(8)
    n = 4096
    pos = rng.random((n, 3))
    lum = np.where(rng.random(n) < 0.25, rng.uniform(0.5, 1.0, n), 0.0)
    kr = 2.5  # kappa rho, exact in binary64 with m = 2^-12
    t = OracleTree(pos, np.ones(n), np.full(n, kr), lum, np.full(n, 2.0 ** -12))
    for i in (0, 5, 77, 4095):
        log = t.ray_log(theta, tau_ref, i)
        r = np.linalg.norm(log["y"] - pos[i], axis=1)
        np.testing.assert_allclose(log["tau"], kr * r, rtol=1e-13, atol=1e-15)
    if theta == 0.0:
        F, _ = t.flux(theta, tau_ref, sinks=np.arange(0, n, 37))
        ref = B.all_pairs_flux(pos, lum, kr, sinks=np.arange(0, n, 37))
        np.testing.assert_allclose(F, ref, rtol=1e-12)


@pytest.mark.parametrize("nb", [1, 4])
def test_full_limit_matches_exact_leaf_integration(nb):
    pos, rho, kappa, lum, mass = _rand(300, 13, n_src=60)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=nb)
    ref = B.split_tree(pos, nb, np.zeros(3), np.ones(3), mass, rho, kappa)
    lv = B.leaves(ref)
    llo = np.array([nd["lo"] for nd in lv])
    lhi = np.array([nd["hi"] for nd in lv])
    lal = np.array([nd["alpha"] for nd in lv])
    F, C = t.flux(0.0, -1.0)
    n_src = np.count_nonzero(lum > 0)
    for i in range(0, 300, 7):
        log = t.ray_log(0.0, -1.0, i)
        assert len(log["tau"]) == n_src - (lum[i] > 0)
        nseg = 0
        f = 0.0
        for src, tau in zip(log["src"], log["tau"]):
            ex, k = B.exact_tau_leaf_field(pos[i], pos[src], llo, lhi, lal)
            assert math.isclose(tau, ex, rel_tol=1e-12, abs_tol=1e-14)
            nseg += k
            d2 = np.sum((pos[src] - pos[i]) ** 2)
            f += lum[src] * math.exp(-ex) / (4 * math.pi * d2)
        assert C[i, 3] == nseg  # one piece per bucket crossed
        assert math.isclose(F[i], f, rel_tol=1e-12)


def test_shell_closed_form():
    """Background shell (Sec. 2.2.4): M sources on a golden-angle spiral of
    radius R, total luminosity 1, optically thin; flux at radius r."""
    M, R = 10000, 0.5
    centre = np.array([0.55, 0.55, 0.55])
    shell = B.fibonacci_sphere(M, R, centre)
    rs = np.linspace(0.0, 0.4, 41)
    rng = np.random.default_rng(2)
    u = rng.standard_normal((rs.size, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    probes = centre + rs[:, None] * u
    pos = np.vstack([shell, probes])
    n = pos.shape[0]
    lum = np.r_[np.full(M, 1.0 / M), np.zeros(rs.size)]
    t = OracleTree(pos, np.ones(n), np.zeros(n), lum, np.ones(n), (0, 0, 0), (1.1, 1.1, 1.1), 8)
    sinks = np.arange(M, n)
    F0, _ = t.flux(0.0, 0.1, sinks=sinks)
    ref = B.shell_flux(rs, R, 1.0)
    np.testing.assert_allclose(F0, ref, rtol=3e-5)
    assert abs(F0[0] * 4 * math.pi * R * R - 1.0) < 1e-5  # constant flux at the centre
    F75, _ = t.flux(0.75, 0.1, sinks=sinks)
    # merging moves the centre of luminosity inward: the flux is over-estimated
    assert np.all(F75 >= F0 * (1 - 1e-3))
    np.testing.assert_allclose(F75, ref, rtol=0.15)


def test_refinement_error_bound():
    """Eq. (reffrac): per piece the flux error is below 1 - exp(-(tau_max -
    tau_min)) <~ tau_ref; the RMS over sinks stays below tau_ref."""
    w = W.c2(n=1 << 13)
    pos = w["pos"].astype(np.float64)
    t = OracleTree(pos, w["rho"], w["kappa"], np.where(np.arange(pos.shape[0]) % 2 == 0, 1.0, 0.0),
                   w["mass"], bucket_size=8)
    sinks = np.arange(0, pos.shape[0], 11)
    Fref, Cref = t.flux(0.75, -1.0, sinks=sinks)
    prev_cost = None
    for tau_ref in (0.2, 0.1, 0.05, 0.01):
        F, C = t.flux(0.75, tau_ref, sinks=sinks)
        rms = math.sqrt(np.mean((F / Fref - 1.0) ** 2))
        assert rms < tau_ref
        cost = C[:, 3].sum()
        assert cost <= Cref[:, 3].sum()
        if prev_cost is not None:
            assert cost >= prev_cost  # a smaller tolerance refines more
        prev_cost = cost
    Fno, Cno = t.flux(0.75, math.inf, sinks=sinks)
    assert Cno[:, 3].sum() < Cref[:, 3].sum()


def _stromgren_1d(ndot, sigma, alpha_B, rmax=0.9, nstep=100000):
    """Exact spherically symmetric equilibrium: d tau / dr = sigma n_H x(r),
    x from x sigma F = alpha_B n_H (1 - x)^2 with F = Ndot e^-tau / (4 pi r^2)
    (midpoint rule, n_H = 1)."""
    r = np.linspace(1e-6, rmax, nstep + 1)
    h = r[1] - r[0]

    def xeq(rr, tau):
        q = sigma * ndot * math.exp(-tau) / (4.0 * math.pi * rr * rr) / alpha_B
        return ((2.0 + q) - math.sqrt((2.0 + q) ** 2 - 4.0)) / 2.0 if q < 1e12 else 1.0 / q

    xs = np.empty_like(r)
    tau = 0.0
    for k in range(nstep + 1):
        xs[k] = xeq(r[k], tau)
        if k < nstep:
            tau += h * sigma * xeq(r[k] + 0.5 * h, tau + 0.5 * h * sigma * xs[k])
    return r, xs


def _stromgren_run(n1, RS=0.25, mfp_spacings=2.0):
    rng = np.random.default_rng(6)
    g = (np.stack(np.meshgrid(*[np.arange(n1)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5
         + 0.3 * (rng.random((n1 ** 3, 3)) - 0.5)) / n1
    centre = np.array([0.5, 0.5, 0.5])
    pos = np.vstack([g, centre[None]])
    n = pos.shape[0]
    ngas = n - 1
    alpha_B = 1.0
    ndot = 4.0 * math.pi / 3.0 * RS ** 3 * alpha_B  # Stromgren radius RS at n_H = 1
    sigma = n1 / mfp_spacings
    lum = np.zeros(n)
    lum[-1] = ndot
    mass = np.r_[np.full(ngas, 1.0 / ngas), 0.0]  # the source absorbs nothing
    r = np.linalg.norm(g - centre, axis=1)
    x = np.where(r < RS, 1e-3, 1.0)
    for _ in range(200):
        t = OracleTree(pos, np.ones(n), np.r_[sigma * x, 0.0], lum, mass)
        # refinement always on keeps the flux continuous in x (fixed point)
        F, _ = t.flux(0.75, -1.0, sinks=np.arange(ngas))
        q = sigma * F / alpha_B
        xe = ((2.0 + q) - np.sqrt((2.0 + q) ** 2 - 4.0)) / 2.0
        dx = np.max(np.abs(xe - x))
        x = 0.5 * x + 0.5 * xe
        if dx < 1e-7:
            break
    R1, X1 = _stromgren_1d(ndot, sigma, alpha_B)
    inner = r < 0.4
    err = np.mean(np.abs(x - np.interp(r, R1, X1))[inner])
    bins = np.linspace(0.5 * RS, 1.5 * RS, 41)
    mid = 0.5 * (bins[1:] + bins[:-1])
    prof = np.array([np.mean(x[(r >= a) & (r < b)]) for a, b in zip(bins[:-1], bins[1:])])
    r_half = np.interp(0.5, prof, mid)
    r_half_1d = np.interp(0.5, X1, R1)
    balance = np.sum(alpha_B * (1.0 - x) ** 2) / ngas / ndot
    return dx, err, r_half / r_half_1d - 1.0, balance


@pytest.mark.slow
def test_stromgren_equilibrium():
    """Ionisation equilibrium around one source in uniform hydrogen (Sec. 3.3,
    the Stromgren radius R_S = (3 Ndot / (4 pi alpha_B n_H^2))^(1/3)):
    kappa_i = sigma x_i, rho = n_H = 1, on-the-spot x sigma F = alpha_B (1-x)^2,
    iterated to a fixed point.  The particle profile must approach the exact
    spherically symmetric solution as the resolution grows, and the
    recombinations must balance the source's photon rate."""
    dx24, err24, rh24, bal24 = _stromgren_run(24)
    dx32, err32, rh32, bal32 = _stromgren_run(32)
    assert dx24 < 1e-6 and dx32 < 1e-6
    assert err32 < 0.016 and err32 < 0.8 * err24  # mean |x - x_exact(r)|
    assert abs(rh32) < 0.03 and abs(rh32) < abs(rh24)  # x = 0.5 radius
    assert 0.9 < bal32 < 1.0 and bal24 < bal32  # photons absorbed inside the box


@pytest.mark.parametrize("theta", [0.0, 0.75])
def test_never_refine_limit_walks_up_the_tree(theta):
    """tau_ref = infinity: the chain cells' own averages are used between the
    sink bucket and the source cell (the walk-up reading of Sec. 2.2.2 and
    the algorithm figure), checked against a brute force over buckets."""
    pos, rho, kappa, lum, mass = _rand(400, 17, n_src=80)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=4)
    e = t.export()
    ref = B.split_tree(pos, 4, np.zeros(3), np.ones(3), mass, rho, kappa)
    assert len(ref) == t.m
    for i in range(0, 400, 9):
        log = t.ray_log(theta, math.inf, i)
        S = e["leaf_of"][i]
        for C, y, tau in zip(log["C"], log["y"], log["tau"]):
            ex = B.walk_up_tau(ref, S, C, pos[i], y)
            assert math.isclose(tau, ex, rel_tol=1e-12, abs_tol=1e-14)


@pytest.mark.parametrize("tau_ref", [0.02, 0.1, 0.5])
def test_pieces_tile_the_ray_and_obey_the_criterion(tau_ref):
    """Eq. (refcrit): a piece uses an unrefined cell only where
    (alpha_max - alpha_min) l <= tau_ref, or the cell is a bucket; the pieces
    tile [0, 1] and lie inside their cells."""
    w = W.c2(n=1 << 12)
    pos = w["pos"].astype(np.float64)
    t = OracleTree(pos, w["rho"], w["kappa"], w["lum"], w["mass"], bucket_size=8)
    e = t.export()
    refined = 0
    for i in (3, 500, 4000):
        log = t.ray_log(0.75, tau_ref, i)
        for k in range(0, len(log["C"]), max(1, len(log["C"]) // 40)):
            pc = t.ray_pieces(0.75, tau_ref, i, k)
            order = np.argsort(pc["ta"], kind="stable")
            ta, tb = pc["ta"][order], pc["tb"][order]
            assert ta[0] == 0.0 and tb[-1] == 1.0
            assert np.array_equal(tb[:-1], ta[1:])  # shared boundaries, no gaps
            assert np.all(tb >= ta)
            y = log["y"][k]
            for nd, a, b, ln in zip(pc["node"], pc["ta"], pc["tb"], pc["len"]):
                leaf = e["leaf"][nd]
                # a chain cell's piece was tested on the chain cell itself
                assert leaf or e["dalpha"][nd] * ln <= tau_ref
                refined += int(not leaf and e["dalpha"][nd] > 0)
                for t_ in (a, b, 0.5 * (a + b)):
                    p = pos[i] + t_ * (y - pos[i])
                    for ax in range(3):
                        assert e["lo%d" % ax][nd] - 1e-12 <= p[ax] <= e["hi%d" % ax][nd] + 1e-12
    assert refined > 0
