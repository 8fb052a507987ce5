"""Pins of the oracle's sub-bucket particle trace (an SPH-style trace below
the buckets: each absorber adds m kappa times its smoothing kernel's integral
along the ray piece, the receiving particle excluded), on the CPU.

  * the kernel's line integral: the column through the centre is
    3 / (2 pi h^2) (closed form of the M4 spline), the columns integrate to one
    over the impact plane (the kernel's volume normalisation, by scipy's
    quad), scipy's quad of the textbook spline along random segments, and
    additivity and symmetry in the segment ends;
  * each bucket's absorber list equals a brute-force search (every absorber
    whose support sphere, radius 2h, reaches the bucket's box), and its
    decision spread is the max - min of kappa rho over its particles;
  * tau_ref = infinity never refines below a bucket: the plain flux and
    counters, bit for bit;
  * tau_ref < 0 refines every piece below its bucket, so every ray's tau is the
    brute-force column of all absorbers but the receiver along the whole ray,
    at theta_open 0 and 0.75;
  * three particles in a row: the absorber in the middle gives
    tau = m kappa 3 / (2 pi h^2), and the receiver's own opacity never counts.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle.oracle import OracleTree, sph_line


def _m4(q):
    """Monaghan's cubic spline, w(q) / (pi h^3) with support 2h."""
    if q < 1.0:
        return 1.0 - 1.5 * q * q + 0.75 * q ** 3
    if q < 2.0:
        return 0.25 * (2.0 - q) ** 3
    return 0.0


def _rand(n, seed, n_src):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    rho = np.exp(0.8 * rng.standard_normal(n))
    kappa = rng.uniform(0.2, 3.0, n)
    kappa[::11] = 0.0
    lum = np.zeros(n)
    lum[rng.choice(n, size=n_src, replace=False)] = 10 ** (0.5 * rng.standard_normal(n_src))
    mass = rng.uniform(0.5, 1.5, n) / n
    mass[::13] = 0.0
    # smoothing lengths from the particle volumes, about 60 within 2h
    h = 1.2 * (np.mean(rho) / (n * rho)) ** (1.0 / 3.0)
    return pos, rho, kappa, lum, mass, h


@pytest.mark.parametrize("h", [0.03, 0.2, 1.0])
def test_central_column(h):
    assert abs(sph_line(0.0, h, -2.5 * h, 3.0 * h) - 1.5 / (np.pi * h * h)) <= \
        1e-14 / (h * h)


def test_columns_integrate_to_one():
    h = 0.37
    val, err = integrate.quad(lambda b: 2.0 * np.pi * b * sph_line(b, h, -3 * h, 3 * h),
                              0.0, 2.0 * h, points=[h], epsabs=1e-13, epsrel=1e-13)
    assert abs(val - 1.0) <= 1e-10


def test_line_integral_against_quad():
    rng = np.random.default_rng(5)
    for _ in range(200):
        h = rng.uniform(0.05, 2.0)
        b = h * rng.choice([0.0, rng.uniform(0, 1e-3), rng.uniform(0, 2.2)])
        u0, u1 = np.sort(h * rng.uniform(-2.5, 2.5, 2))
        ref, _ = integrate.quad(lambda u: _m4(np.hypot(b, u) / h) / (np.pi * h ** 3), u0, u1,
                                points=[x for x in (-np.sqrt(max(4 * h * h - b * b, 0)),
                                                    -np.sqrt(max(h * h - b * b, 0)), 0.0,
                                                    np.sqrt(max(h * h - b * b, 0)),
                                                    np.sqrt(max(4 * h * h - b * b, 0)))
                                        if u0 < x < u1] or None,
                                epsabs=1e-14 / (h * h), epsrel=1e-13, limit=200)
        got = sph_line(b, h, u0, u1)
        assert abs(got - ref) <= 1e-12 / (h * h), (b, h, u0, u1)
        m = rng.uniform(u0, u1)
        assert abs(sph_line(b, h, u0, m) + sph_line(b, h, m, u1) - got) <= 1e-13 / (h * h)
        assert abs(sph_line(b, h, -u1, -u0) - got) <= 1e-13 / (h * h)


def test_neighbour_lists_and_spread_brute_force():
    pos, rho, kappa, lum, mass, h = _rand(700, 31, 60)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=4)
    t.set_sph(h)
    e = t.export()
    dp = t.sph_spread()
    absorber = (mass * kappa) > 0
    for node in range(t.m):
        if not e["leaf"][node]:
            assert dp[node] == -1.0
            continue
        lo = np.array([e["lo0"][node], e["lo1"][node], e["lo2"][node]])
        hi = np.array([e["hi0"][node], e["hi1"][node], e["hi2"][node]])
        gap = np.maximum(np.maximum(lo - pos, pos - hi), 0.0)
        d2 = (gap ** 2).sum(axis=1)
        want = set(np.nonzero(absorber & (d2 < 4 * h * h))[0].tolist())
        got = t.sph_neighbours(node)
        assert set(got.tolist()) == want and len(got) == len(want), node
        mine = e["perm"][e["first"][node]:e["first"][node] + e["count"][node]]
        a = (kappa * rho)[mine[mass[mine] > 0]]
        assert dp[node] == (a.max() - a.min() if a.size else 0.0)


@pytest.mark.parametrize("theta", [0.0, 0.75])
def test_never_below_the_bucket_is_the_plain_flux(theta):
    pos, rho, kappa, lum, mass, h = _rand(1500, 32, 200)
    t = OracleTree(pos, rho, kappa, lum, mass)
    t.set_sph(h)
    F, C = t.flux(theta, np.inf)
    Fs, Cs = t.flux_sph(theta, np.inf)
    assert np.array_equal(F, Fs) and np.array_equal(C, Cs)


@pytest.mark.parametrize("theta", [0.0, 0.75])
def test_full_refinement_is_the_all_particle_column(theta):
    pos, rho, kappa, lum, mass, h = _rand(400, 33, 80)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=3)
    t.set_sph(h)
    mk = np.where(mass > 0, mass * kappa, 0.0)
    for i in (0, 57, 311):
        log = t.ray_log_sph(theta, -1.0, i)
        assert log["tau"].size > 10
        xi = pos[i]
        for y, tau in zip(log["y"], log["tau"]):
            d = y - xi
            r2 = d @ d
            r = np.sqrt(r2)
            want = 0.0
            for j in np.nonzero(mk > 0)[0]:
                if j == i:
                    continue
                dl = pos[j] - xi
                ts = (dl @ d) / r2
                b = np.linalg.norm(dl - ts * d)
                want += mk[j] * sph_line(b, h[j], -ts * r, (1.0 - ts) * r)
            assert abs(tau - want) <= 1e-12 * max(1.0, want), (i, tau, want)


def test_three_particles_in_a_row():
    pos = np.array([[0.1, 0.5, 0.5], [0.5, 0.5, 0.5], [0.9, 0.5, 0.5]])
    rho = np.ones(3)
    kappa = np.array([1e6, 2.0, 0.0])  # the receiver is opaque; the source is not absorbing
    mass = np.array([1.0, 0.005, 1.0])
    lum = np.array([0.0, 0.0, 3.0])
    h = np.array([0.3, 0.05, 0.1])
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=1)
    t.set_sph(h)
    F, _ = t.flux_sph(0.0, -1.0, sinks=np.array([0]))
    tau = 0.005 * 2.0 * 1.5 / (np.pi * 0.05 ** 2)
    assert abs(F[0] - 3.0 * np.exp(-tau) / (4 * np.pi * 0.8 ** 2)) <= 1e-14 * F[0]
