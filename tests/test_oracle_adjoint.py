"""Pins of the oracle's adjoint (CPU only).

The forward is F_i = sum over rays of L e^-tau / (4 pi r^2) (eq. simpint)
with tau = sum alpha l (eqs. taui, tausum), alpha = kappa rho_cell with the
volume-weighted density (Sec. 2.3) and merged sources at the centre of
luminosity (Sec. 2.2.1).  With every decision held fixed:
  * F is homogeneous of degree 1 in all L, so sum_j L_j dF/dL_j = F;
  * alpha is homogeneous of degree 1 in all kappa and in all rho, so
    sum_p kappa_p dF/dkappa_p = sum_p rho_p dF/drho_p = -sum_rays f tau;
  * one ray in one bucket has a closed form;
  * central finite differences in binary64 agree where no decision flips.
"""
import math

import numpy as np
import pytest

from oracle.oracle import OracleTree


def _inst(n, seed, n_src):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    pos[: n // 4] = 0.6 + 0.05 * rng.random((n // 4, 3))  # a dense clump
    rho = np.exp(rng.standard_normal(n))
    kappa = rng.uniform(0.5, 3.0, n)
    lum = np.zeros(n)
    src = rng.choice(n, size=n_src, replace=False)
    lum[src] = 10 ** rng.standard_normal(n_src)
    mass = np.full(n, 1.0 / n)
    mass[rng.choice(n, size=n // 20, replace=False)] = 0.0
    return pos, rho, kappa, lum, mass


@pytest.mark.parametrize("theta,tau_ref", [(0.75, 0.1), (0.5, -1.0), (1.0, math.inf)])
def test_euler_identities(theta, tau_ref):
    pos, rho, kappa, lum, mass = _inst(3000, 1, 400)
    t = OracleTree(pos, rho, kappa, lum, mass)
    F, C, G = t.flux(theta, tau_ref, with_g=True)
    w = np.random.default_rng(2).standard_normal(F.size)
    gr, gk, gl = t.adjoint(theta, tau_ref, w)
    lhs_L = np.dot(lum, gl)
    assert math.isclose(lhs_L, np.dot(w, F), rel_tol=1e-11)
    rhs = -np.dot(w, G)
    assert math.isclose(np.dot(kappa, gk), rhs, rel_tol=1e-11)
    assert math.isclose(np.dot(rho, gr), rhs, rel_tol=1e-11)
    assert np.all(gr[mass == 0] == 0) and np.all(gk[mass == 0] == 0)


def test_single_ray_closed_form():
    pos = np.array([[0.2, 0.3, 0.4], [0.7, 0.6, 0.45]])
    rho = np.array([1.5, 0.7])
    kappa = np.array([2.0, 1.1])
    lum = np.array([0.0, 3.0])
    mass = np.array([0.4, 0.9])
    t = OracleTree(pos, rho, kappa, lum, mass)  # one bucket holds both
    F, C = t.flux(0.0, 0.1, sinks=[0])
    Bv = mass[0] / rho[0] + mass[1] / rho[1]
    alpha = (mass[0] * kappa[0] + mass[1] * kappa[1]) / Bv
    r = np.linalg.norm(pos[1] - pos[0])
    f = lum[1] * math.exp(-alpha * r) / (4 * math.pi * r * r)
    assert math.isclose(F[0], f, rel_tol=1e-14)
    gr, gk, gl = t.adjoint(0.0, 0.1, [1.0], sinks=[0])
    for p in (0, 1):
        assert math.isclose(gk[p], -f * r * mass[p] / Bv, rel_tol=1e-13)
        assert math.isclose(gr[p], -f * r * alpha * mass[p] / (Bv * rho[p] ** 2), rel_tol=1e-13)
    assert gl[0] == 0.0 and math.isclose(gl[1], f / lum[1], rel_tol=1e-14)


def _fd_case(which, theta=0.75, tau_ref=0.1, n=1500, seed=3):
    pos, rho, kappa, lum, mass = _inst(n, seed, 300)
    arrays = {"rho": rho, "kappa": kappa, "lum": lum}
    w = np.random.default_rng(4).standard_normal(n)

    def loss(arr):
        a = dict(arrays)
        a[which] = arr
        t = OracleTree(pos, a["rho"], a["kappa"], a["lum"], mass)
        F, C = t.flux(theta, tau_ref)
        return float(np.dot(w, F)), C

    F0, _ = OracleTree(pos, rho, kappa, lum, mass).flux(theta, tau_ref)
    magnitude = float(np.sum(np.abs(w * F0)))

    t = OracleTree(pos, rho, kappa, lum, mass)
    g = dict(zip(("rho", "kappa", "lum"), t.adjoint(theta, tau_ref, w)))[which]
    base_loss, base_C = loss(arrays[which])
    rng = np.random.default_rng(7)
    cand = np.nonzero(arrays[which] > 0)[0] if which == "lum" else np.nonzero(mass > 0)[0]
    checked = 0
    for p in rng.choice(cand, size=32, replace=False):
        h = 1e-5 * arrays[which][p]
        up = arrays[which].copy()
        dn = arrays[which].copy()
        up[p] += h
        dn[p] -= h
        lu, Cu = loss(up)
        ld, Cd = loss(dn)
        if not (np.array_equal(Cu, base_C) and np.array_equal(Cd, base_C)):
            continue  # a decision flipped between the two points
        fd = (lu - ld) / (2 * h)
        # truncation O(h^2) plus the round-off of the two loss sums
        tol = 1e-6 * abs(g[p]) + 4 * np.finfo(float).eps * magnitude / h
        assert abs(fd - g[p]) <= tol, (which, p, fd, g[p], tol)
        checked += 1
    assert checked >= 24


@pytest.mark.parametrize("which", ["rho", "kappa", "lum"])
def test_finite_differences(which):
    _fd_case(which)
