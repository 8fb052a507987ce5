"""Pins of the oracle's multi-band flux (several opacity fields on one
traversal, refined where any band asks for it) on the CPU.

  * one band equal to the tree's own opacity: the plain flux and counters,
    bit for bit;
  * bands (kappa, 0): band 0 is the plain flux and band 1 the optically thin
    flux, bit for bit, with the plain traversal;
  * bands (kappa, 2 kappa): decisions follow the larger spread, so band 1 is the
    plain flux of a tree with 2 kappa, bit for bit, counters included;
  * a uniform medium with one opacity per band: every band is the brute-force
    all-pairs flux with alpha = kappa_b at theta_open = 0.
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
    mass = rng.uniform(0.5, 1.5, n)
    mass[::13] = 0.0
    return pos, rho, kappa, lum, mass


@pytest.mark.parametrize("theta,tau_ref", [(0.75, 0.1), (0.5, -1.0), (1.0, 0.05)])
def test_one_band_is_the_plain_flux(theta, tau_ref):
    pos, rho, kappa, lum, mass = _rand(2500, 101, 400)
    t = OracleTree(pos, rho, kappa, lum, mass)
    F, C = t.flux(theta, tau_ref)
    Fb, Cb = t.flux_bands(theta, tau_ref, kappa[None, :])
    assert np.array_equal(Fb[:, 0], F) and np.array_equal(Cb, C)


def test_thin_band_beside_the_plain_one():
    pos, rho, kappa, lum, mass = _rand(2500, 102, 400)
    t = OracleTree(pos, rho, kappa, lum, mass)
    F, C = t.flux(0.75, 0.1)
    Fthin, _ = OracleTree(pos, rho, 0 * kappa, lum, mass).flux(0.75, 0.1)
    Fb, Cb = t.flux_bands(0.75, 0.1, np.stack([kappa, 0 * kappa]))
    assert np.array_equal(Fb[:, 0], F) and np.array_equal(Cb, C)
    assert np.array_equal(Fb[:, 1], Fthin)


def test_decisions_follow_the_largest_spread():
    pos, rho, kappa, lum, mass = _rand(2500, 103, 400)
    t = OracleTree(pos, rho, kappa, lum, mass)
    F2, C2 = OracleTree(pos, rho, 2 * kappa, lum, mass).flux(0.75, 0.1)
    Fb, Cb = t.flux_bands(0.75, 0.1, np.stack([kappa, 2 * kappa]))
    assert np.array_equal(Fb[:, 1], F2) and np.array_equal(Cb, C2)


def test_uniform_medium_per_band():
    rng = np.random.default_rng(104)
    n = 2048
    pos = rng.random((n, 3))
    lum = np.where(rng.random(n) < 0.2, rng.uniform(0.5, 1.0, n), 0.0)
    kb = np.array([0.5, 2.5, 7.0])
    t = OracleTree(pos, np.ones(n), np.ones(n), lum, np.full(n, 2.0 ** -12))
    sinks = np.arange(0, n, 31)
    Fb, _ = t.flux_bands(0.0, 0.1, np.repeat(kb[:, None], n, axis=1), sinks=sinks)
    for b, k in enumerate(kb):
        ref = B.all_pairs_flux(pos, lum, k, sinks=sinks)
        np.testing.assert_allclose(Fb[:, b], ref, rtol=1e-12)
