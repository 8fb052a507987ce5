"""Pins of the oracle's vector flux (each ray's flux along its direction of
travel at the sink, summed over rays; the radiation-pressure direction) on
the CPU.

  * optically thin and theta_open = 0: the all-pairs sum of
    L (x_i - x_j) / (4 pi r^3), brute force;
  * a uniform medium at theta_open = 0: the same with exp(-kappa rho r);
  * six equal sources placed symmetrically about a sink: the vector flux
    cancels;
  * one source behind absorbers: the vector flux is the flux times the unit
    vector from the source to the sink;
  * merged sources (theta_open > 0): the sum of the ray log's f (x_i - y) / r in
    walk order, and |Fv| <= F.
"""
import numpy as np
import pytest

import _brute as B
from oracle.oracle import OracleTree


def _rand(n, seed, n_src):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    rho = np.exp(0.8 * rng.standard_normal(n))
    kappa = rng.uniform(0.2, 3.0, n)
    lum = np.zeros(n)
    lum[rng.choice(n, size=n_src, replace=False)] = 10 ** (0.5 * rng.standard_normal(n_src))
    return pos, rho, kappa, lum, rng.uniform(0.5, 1.5, n)


def test_thin_all_pairs():
    pos, rho, kappa, lum, mass = _rand(1200, 61, 200)
    t = OracleTree(pos, rho, 0 * kappa, lum, mass, bucket_size=8)
    F, Fv = t.flux_vector(0.0, 0.1)
    F1, _ = t.flux(0.0, 0.1)
    assert np.array_equal(F, F1)
    ref = B.all_pairs_vector_flux(pos, lum)
    assert np.all(np.abs(Fv - ref) <= 1e-13 * F[:, None])


def test_uniform_medium_all_pairs():
    rng = np.random.default_rng(62)
    n = 2048
    pos = rng.random((n, 3))
    lum = np.where(rng.random(n) < 0.2, rng.uniform(0.5, 1.0, n), 0.0)
    kr = 2.5  # kappa rho, exact in binary64 with m = 2^-12
    t = OracleTree(pos, np.ones(n), np.full(n, kr), lum, np.full(n, 2.0 ** -12))
    sinks = np.arange(0, n, 29)
    for tau_ref in (-1.0, 0.1):
        F, Fv = t.flux_vector(0.0, tau_ref, sinks=sinks)
        ref = B.all_pairs_vector_flux(pos, lum, kr, sinks=sinks)
        assert np.all(np.abs(Fv - ref) <= 1e-12 * F[:, None])


def test_symmetric_sources_cancel():
    c = np.array([0.5, 0.5, 0.5])
    h = 0.25
    src = np.array([c + s * h * e for e in np.eye(3) for s in (1.0, -1.0)])
    pos = np.vstack([c, src])
    lum = np.array([0.0] + [1.0] * 6)
    t = OracleTree(pos, np.ones(7), np.zeros(7), lum, np.ones(7), bucket_size=1)
    F, Fv = t.flux_vector(0.0, 0.1, sinks=[0])
    assert F[0] == pytest.approx(6.0 / (4.0 * np.pi * h * h), rel=1e-15)
    assert np.all(np.abs(Fv[0]) <= 1e-15 * F[0])


def test_single_source_through_absorbers():
    pos, rho, kappa, lum, mass = _rand(1500, 64, 1)
    j = int(np.nonzero(lum)[0][0])
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=8)
    for theta, tau_ref in ((0.0, -1.0), (0.75, 0.1)):
        F, Fv = t.flux_vector(theta, tau_ref)
        d = pos - pos[j]
        r = np.linalg.norm(d, axis=1)
        ok = r > 0
        err = np.abs(Fv[ok] - F[ok, None] * d[ok] / r[ok, None])
        assert np.all(err <= 1e-14 * F[ok, None])
        assert np.all(Fv[~ok] == 0) and np.all(F[~ok] == 0)


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_merged_sources_from_the_ray_log(theta):
    pos, rho, kappa, lum, mass = _rand(3000, 65, 600)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=8)
    sinks = np.array([0, 17, 999, 2999])
    F, Fv = t.flux_vector(theta, 0.1, sinks=sinks)
    for q, i in enumerate(sinks):
        log = t.ray_log(theta, 0.1, int(i))
        d = pos[i] - log["y"]
        r = np.sqrt(np.sum(d * d, axis=1))
        acc = np.zeros(3)
        for k in range(r.size):  # walk order, as the oracle sums
            acc += log["f"][k] * (d[k] / r[k])
        np.testing.assert_allclose(Fv[q], acc, rtol=1e-13, atol=1e-13 * F[q])
        assert np.linalg.norm(Fv[q]) <= F[q] * (1 + 1e-12)


# ---- second moment (radiation pressure tensor times c) ----

def test_second_moment_thin_all_pairs_and_trace():
    pos, rho, kappa, lum, mass = _rand(1000, 66, 150)
    t = OracleTree(pos, rho, 0 * kappa, lum, mass, bucket_size=8)
    F, Fv, Pm = t.flux_moments(0.0, 0.1)
    F1, Fv1 = t.flux_vector(0.0, 0.1)
    assert np.array_equal(F, F1) and np.array_equal(Fv, Fv1)
    ref = B.all_pairs_second_moment(pos, lum)
    assert np.all(np.abs(Pm - ref) <= 1e-13 * F[:, None])


@pytest.mark.parametrize("theta,tau_ref", [(0.75, 0.1), (1.0, -1.0)])
def test_second_moment_trace_is_the_flux(theta, tau_ref):
    # n is a unit vector: P_xx + P_yy + P_zz = F ray by ray
    pos, rho, kappa, lum, mass = _rand(3000, 67, 500)
    t = OracleTree(pos, rho, kappa, lum, mass, bucket_size=8)
    F, _, Pm = t.flux_moments(theta, tau_ref)
    assert np.all(np.abs(Pm[:, 0] + Pm[:, 1] + Pm[:, 2] - F) <= 1e-13 * F)
    # positive semi-definite: P_aa >= 0 and P_aa P_bb >= P_ab^2
    assert np.all(Pm[:, :3] >= 0)
    for a, b, k in ((0, 1, 3), (0, 2, 4), (1, 2, 5)):
        assert np.all(Pm[:, k] ** 2 <= Pm[:, a] * Pm[:, b] * (1 + 1e-12) + 1e-300)


def test_second_moment_isotropic_sources():
    c = np.array([0.5, 0.5, 0.5])
    h = 0.25
    src = np.array([c + s * h * e for e in np.eye(3) for s in (1.0, -1.0)])
    pos = np.vstack([c, src])
    lum = np.array([0.0] + [1.0] * 6)
    t = OracleTree(pos, np.ones(7), np.zeros(7), lum, np.ones(7), bucket_size=1)
    F, _, Pm = t.flux_moments(0.0, 0.1, sinks=[0])
    np.testing.assert_allclose(Pm[0, :3], F[0] / 3.0, rtol=1e-15)
    assert np.all(np.abs(Pm[0, 3:]) <= 1e-16 * F[0])
