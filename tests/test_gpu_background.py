"""GPU: the background shell (trevr_set_background,
trevr_compute_flux_background) through the C ABI, against the oracle.

  * a spiral shell of 6000 background sources around absorbing gas with a
    local star: the flux within 1e-12 (binary64) or 1e-5 (binary32) of the
    oracle's, counters identical;
  * at the shell's centre an optically thin flux is exactly L / (4 pi R^2);
  * theta_open = 0 merges nothing: the plain flux;
  * refusals (none set, radius <= 0) and a refit dropping the shell.
"""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1902_08083_amd as P  # noqa: E402
import _brute as B  # noqa: E402
from oracle.oracle import OracleTree  # noqa: E402

NTHREADS = min(16, os.cpu_count() or 1)
CENTRE = np.array([0.55, 0.55, 0.55])
R = 0.5


def _note(msg):
    print(msg, flush=True)


def _case(prec, kappa=2.0, M=6000, n_gas=3000, seed=4, centre_probe=False):
    shell = B.fibonacci_sphere(M, R, CENTRE)
    rng = np.random.default_rng(seed)
    gas = CENTRE + 0.35 * (rng.random((n_gas, 3)) * 2 - 1) / math.sqrt(3)
    if centre_probe:
        gas[0] = CENTRE
    pos = np.vstack([shell, gas])
    n = pos.shape[0]
    lum = np.r_[np.full(M, 1.0 / M), np.zeros(n_gas)]
    if not centre_probe:
        lum[M + 5] = 0.3
    mass = np.r_[np.zeros(M), np.full(n_gas, 1.0 / n_gas)]
    rho = np.exp(0.5 * rng.standard_normal(n))
    kap = np.full(n, kappa)
    flags = np.r_[np.ones(M, np.uint8), np.zeros(n_gas, np.uint8)]
    npdt = np.float64 if prec == "f64" else np.float32
    arrs = [a.astype(npdt) for a in (pos, rho, kap, lum, mass)]
    dt = torch.float64 if prec == "f64" else torch.float32
    d = lambda a: torch.as_tensor(a, dtype=dt, device="cuda")  # noqa: E731
    box = (0.0, 0.0, 0.0), (1.1, 1.1, 1.1)
    tg = P.build_tree(*[d(a) for a in arrs], box[0], box[1], 8)
    tg.set_background(CENTRE, R, flags)
    g = lambda a: np.asarray(a, np.float64)  # noqa: E731
    to = OracleTree(*[g(a) for a in arrs], box[0], box[1], 8, mirror32=(prec == "f32"))
    to.set_background(CENTRE, R, flags)
    return arrs, tg, to, np.arange(M, n)


@pytest.mark.parametrize("prec,theta,tau_ref", [("f64", 0.75, 0.1), ("f32", 0.75, 0.1),
                                                ("f64", 1.0, -1.0), ("f32", 0.5, 0.3)])
def test_background_matches_oracle(prec, theta, tau_ref):
    _note("background %s theta %g tau_ref %g" % (prec, theta, tau_ref))
    arrs, tg, to, gas = _case(prec)
    F, C = tg.flux_background(theta, tau_ref, counters=True)
    Fo, Co = to.flux_background(theta, tau_ref, nthreads=NTHREADS)
    assert np.array_equal(C.cpu().numpy().astype(np.int64), Co)
    tol = 1e-12 if prec == "f64" else 1e-5
    Fg = F.double().cpu().numpy()
    ok = Fo > 0
    rel = np.abs(Fg[ok] - Fo[ok]) / Fo[ok]
    _note("worst rel err %.3g" % rel.max())
    assert rel.max() <= tol and np.all(Fg[~ok] == 0)


def test_centre_is_exact_and_theta_zero_is_plain():
    _note("background centre, theta 0")
    arrs, tg, to, gas = _case("f64", kappa=0.0, centre_probe=True)
    s = torch.tensor([int(gas[0])], dtype=torch.int32, device="cuda")
    exact = 1.0 / (4 * math.pi * R * R)
    for theta in (0.5, 0.75, 1.0):
        F = float(tg.flux_background(theta, 0.1, sinks=s)[0])
        assert abs(F - exact) <= 1e-13 * exact
    arrs, tg, to, gas = _case("f64")
    F, C = tg.flux_background(0.0, 0.1, counters=True)
    F0, C0 = tg.flux(0.0, 0.1, counters=True)
    assert torch.equal(C, C0) and torch.allclose(F, F0, rtol=1e-12, atol=0)


def test_refusals():
    _note("background refusals")
    arrs, tg, to, gas = _case("f64", M=500, n_gas=500)
    d = lambda a: torch.as_tensor(a, device="cuda")  # noqa: E731
    fresh = P.build_tree(*[d(a) for a in arrs], (0.0, 0.0, 0.0), (1.1, 1.1, 1.1), 8)
    with pytest.raises(P.TrevrError) as e:
        fresh.flux_background(0.75, 0.1)
    assert e.value.status == -5
    flags = np.zeros(1000, np.uint8)
    for bad in (0.0, -1.0, float("nan")):
        with pytest.raises(P.TrevrError) as e:
            fresh.set_background(CENTRE, bad, flags)
        assert e.value.status == -1
    tg.refit(*[d(a) for a in arrs])
    with pytest.raises(P.TrevrError) as e:
        tg.flux_background(0.75, 0.1)
    assert e.value.status == -5
