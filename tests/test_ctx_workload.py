"""The paper-context particle set (Sec. 3.1.1, App. A) on the CPU: the mode
table the generator uses is the one the paper prints (tests/golden), the
Jacobian determinant that sets the gas density matches finite differences of
the position map, the stars are the coordinate-rotated glass, and the set
has the stated masses, opacities, luminosities and box."""
import os

import numpy as np

from paper_1902_08083_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tab_modes.txt")


def test_mode_table_is_the_printed_one():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert [int(r[0]) for r in rows] == list(range(1, 25))
    tab = np.array([[float(v) for v in r[1:]] for r in rows])
    assert np.array_equal(tab, W.TAB_MODES)
    assert W.MODE_AMPLITUDE == 1.0 / 275.0


def test_density_is_the_jacobian_of_the_map():
    rng = np.random.default_rng(0)
    r0 = rng.random((64, 3))
    _, det = W.perturb_modes(r0)
    h = 1e-6
    for i in range(r0.shape[0]):
        J = np.empty((3, 3))
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            p, _ = W.perturb_modes(np.stack([r0[i] + e, r0[i] - e]))
            J[:, a] = (p[0] - p[1]) / (2 * h)
        assert abs(np.linalg.det(J) - det[i]) < 1e-8
    # the displacement is the same scalar on every axis
    p, _ = W.perturb_modes(r0)
    d = p - r0
    assert np.allclose(d[:, 0], d[:, 1], rtol=0, atol=1e-15)
    assert np.allclose(d[:, 0], d[:, 2], rtol=0, atol=1e-15)
    assert np.abs(d).max() <= 24 / 275


def test_gas_stars_and_box():
    w = W.ctx_lattice(n_side=8, prec="f64")
    n = w["n_gas"]
    assert n == 512 and w["pos"].shape == (2 * n, 3)
    gas, stars = w["pos"][:n], w["pos"][n:]
    # undo the common displacement: star glass = gas glass with (x, y, z) -> (y, z, x)
    rng = np.random.default_rng(61)
    g = (np.arange(8) + 0.5) / 8
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    glass = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1) + rng.uniform(-0.25, 0.25, (n, 3)) / 8
    assert np.allclose(gas, W.perturb_modes(glass)[0], rtol=0, atol=1e-15)
    assert np.allclose(stars, W.perturb_modes(glass[:, [1, 2, 0]])[0], rtol=0, atol=1e-15)
    assert np.isclose(w["mass"][:n].sum(), 1.0) and not w["mass"][n:].any()
    assert np.all(w["kappa"][:n] == 1) and not w["kappa"][n:].any()
    assert not w["lum"][:n].any() and np.all(w["lum"][n:] == 1)
    _, det = W.perturb_modes(glass)
    assert np.allclose(w["rho"][:n], 1.0 / det)
    assert np.all(w["pos"] > -0.05) and np.all(w["pos"] < 1.05)
