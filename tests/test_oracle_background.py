"""Pins of the oracle's background shell (Sec. 2.2.4: sources on a golden-angle
spiral on a sphere, merged background sources moved onto the sphere), CPU.

  * theta_open = 0 merges nothing: the plain flux bit for bit;
  * at the shell's centre every merged source lies exactly R away, so an
    optically thin flux is L / (4 pi R^2) at any theta_open (the plain walk,
    whose merged centres fall inside the sphere, over-estimates it);
  * every moved cell's point lies on the sphere in the direction of its x_L,
    a cell holding a luminous non-background particle is not moved, and a cell
    with one background source radiates from that source;
  * away from the centre the moved sources follow eq. cosmof (R14) more
    closely than the plain merged ones.
"""
import math

import numpy as np
import pytest

import _brute as B
from oracle.oracle import OracleTree


def _shell_case(M=6000, R=0.5, n_gas=600, kappa=0.0, seed=3):
    centre = np.array([0.55, 0.55, 0.55])
    shell = B.fibonacci_sphere(M, R, centre)
    rng = np.random.default_rng(seed)
    gas = centre + 0.35 * (rng.random((n_gas, 3)) * 2 - 1) / math.sqrt(3)
    rs = np.linspace(0.0, 0.4, 21)
    u = rng.standard_normal((rs.size, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    probes = centre + rs[:, None] * u
    pos = np.vstack([shell, gas, probes])
    n = pos.shape[0]
    lum = np.r_[np.full(M, 1.0 / M), np.zeros(n_gas + rs.size)]
    lum[M + 5] = 0.3  # one local star among the gas
    mass = np.r_[np.zeros(M), np.full(n_gas + rs.size, 1.0 / n_gas)]
    flags = np.r_[np.ones(M, np.uint8), np.zeros(n_gas + rs.size, np.uint8)]
    t = OracleTree(pos, np.ones(n), np.full(n, kappa), lum, mass, (0, 0, 0), (1.1, 1.1, 1.1), 8)
    t.set_background(centre, R, flags)
    return t, pos, lum, flags, centre, R, rs, np.arange(M + n_gas, n)


def test_no_merging_is_the_plain_flux():
    t, pos, lum, flags, c, R, rs, probes = _shell_case(kappa=2.0)
    F, C = t.flux_background(0.0, 0.1, sinks=probes)
    F0, C0 = t.flux(0.0, 0.1, sinks=probes)
    assert np.array_equal(F, F0) and np.array_equal(C, C0)


@pytest.mark.parametrize("theta", [0.5, 0.75, 1.0])
def test_centre_flux_is_exact(theta):
    t, pos, lum, flags, c, R, rs, probes = _shell_case()
    lum = lum.copy()
    # the probe at r = 0 sits at the centre; the local star is switched off by
    # a separate tree without it
    pos2 = pos.copy()
    pos2[probes[0]] = c
    lum[lum == 0.3] = 0.0
    n = pos2.shape[0]
    t2 = OracleTree(pos2, np.ones(n), np.zeros(n), lum, np.ones(n), (0, 0, 0), (1.1, 1.1, 1.1), 8)
    t2.set_background(c, R, flags)
    F, _ = t2.flux_background(theta, 0.1, sinks=probes[:1])
    F0, _ = t2.flux(theta, 0.1, sinks=probes[:1])
    exact = 1.0 / (4 * math.pi * R * R)
    assert abs(F[0] - exact) <= 1e-13 * exact
    assert F0[0] > exact * (1 + 1e-4)  # plain merged centres fall inside the sphere


def test_moved_cells():
    t, pos, lum, flags, c, R, rs, probes = _shell_case()
    e = t.export()
    moved, ypos = t.background_cells()
    assert moved.sum() > 0
    for cell in range(t.m):
        members = e["perm"][e["first"][cell]: e["first"][cell] + e["count"][cell]]
        lum_m = members[lum[members] > 0]
        want = lum_m.size > 0 and bool(np.all(flags[lum_m] == 1))
        assert moved[cell] == want
        if not want:
            continue
        xl = np.array([e["xl%d" % a][cell] for a in range(3)])
        v = ypos[cell] - c
        assert abs(np.linalg.norm(v) - R) <= 1e-14
        w = xl - c
        assert np.linalg.norm(np.cross(v, w)) <= 1e-13 * np.linalg.norm(w) * R
        if lum_m.size == 1:
            assert np.allclose(ypos[cell], pos[lum_m[0]], rtol=0, atol=1e-15)


def test_follows_the_shell_solution_more_closely():
    t, pos, lum, flags, c, R, rs, probes = _shell_case(M=10000)
    # the local star would add its own flux: compare the shell part only
    lum2 = lum.copy()
    lum2[lum2 == 0.3] = 0.0
    n = pos.shape[0]
    t2 = OracleTree(pos, np.ones(n), np.zeros(n), lum2, np.ones(n), (0, 0, 0), (1.1, 1.1, 1.1), 8)
    t2.set_background(c, R, flags)
    r = np.linalg.norm(pos[probes] - c, axis=1)
    ref = B.shell_flux(r, R, 1.0)
    F, _ = t2.flux_background(0.75, 0.1, sinks=probes)
    F0, _ = t2.flux(0.75, 0.1, sinks=probes)
    e_bg = np.abs(F / ref - 1)
    e_plain = np.abs(F0 / ref - 1)
    assert e_bg.mean() < 0.5 * e_plain.mean()
    assert e_bg.max() < 0.05
