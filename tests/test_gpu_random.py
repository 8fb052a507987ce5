"""GPU: seeded random configurations against the oracle -- particle count,
precision, bucket size, theta_open, tau_ref, geometry (uniform, lattice
points, clusters, dyadic points on split planes of many levels), masses with
zeros, opacities from zero -- for the flux (with counters), one walk variant
and the particle trace below the buckets; and for both adjoints, two bands,
the background shell and the second moment.  Within 1e-12 (binary64) or 1e-5
(binary32) of the oracle, counters identical.
"""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1902_08083_amd as P  # noqa: E402
from oracle.oracle import OracleTree  # noqa: E402

NTHREADS = min(16, os.cpu_count() or 1)


@pytest.mark.parametrize("case", range(16))
def test_random_configuration(case):
    rng = np.random.default_rng(2000 + case)
    n = int(rng.integers(2, 2500))
    prec = "f64" if case % 2 == 0 else "f32"
    bucket = int(rng.choice([1, 2, 4, 8, 16]))
    theta = float(rng.choice([0.0, 0.3, 0.5, 0.75, 1.0, 1.3]))
    tau_ref = float(rng.choice([-1.0, 0.0, 0.02, 0.1, 0.5, math.inf]))
    geom = case % 4
    if geom == 0:
        pos = rng.random((n, 3))
    elif geom == 1:
        k = int(round(n ** (1 / 3))) + 1
        pos = rng.integers(0, k, (n, 3)) / k
    elif geom == 2:
        c = rng.random((5, 3))
        pos = np.clip(c[rng.integers(0, 5, n)] + 0.02 * rng.standard_normal((n, 3)), 0,
                      0.999999)
    else:
        pos = rng.integers(0, 64, (n, 3)) / 64.0
    print("case %d n %d %s N_B %d theta %g tau_ref %g geometry %d" % (case, n, prec, bucket,
                                                                       theta, tau_ref, geom),
          flush=True)
    rho = np.exp(rng.standard_normal(n))
    kappa = rng.uniform(0.0, 4.0, n)
    lum = np.where(rng.random(n) < rng.uniform(0.05, 0.6), 10 ** rng.standard_normal(n), 0.0)
    mass = rng.uniform(0.0, 2.0, n) / n
    mass[rng.random(n) < 0.1] = 0.0
    npdt = np.float64 if prec == "f64" else np.float32
    arrs = [a.astype(npdt) for a in (pos, rho, kappa, lum, mass)]
    dt = torch.float64 if prec == "f64" else torch.float32
    d = lambda a: torch.as_tensor(a, dtype=dt, device="cuda")  # noqa: E731
    tol = 1e-12 if prec == "f64" else 1e-5
    tg = P.build_tree(*[d(a) for a in arrs], bucket_size=bucket)
    f = lambda a: np.asarray(a, np.float64)  # noqa: E731
    to = OracleTree(*[f(a) for a in arrs], bucket_size=bucket, mirror32=(prec == "f32"))
    F, C = tg.flux(theta, tau_ref, counters=True)
    Fo, Co = to.flux(theta, tau_ref, nthreads=NTHREADS)
    assert np.array_equal(C.cpu().numpy().astype(np.int64), Co)
    assert np.all(np.abs(F.double().cpu().numpy() - Fo) <= tol * Fo)
    om, rm = int(rng.integers(0, 3)), int(rng.integers(0, 2))
    Fv = tg.flux_variant(theta, tau_ref, om, rm).double().cpu().numpy()
    Fvo, _ = to.flux_variant(theta, tau_ref, om, rm, nthreads=NTHREADS)
    assert np.all(np.abs(Fv - Fvo) <= tol * Fvo)
    h = (1.2 * (np.maximum(mass, 1e-6 / n) / rho) ** (1 / 3)).astype(npdt)
    tg.set_sph(d(h))
    to.set_sph(h.astype(np.float64))
    Fs = tg.flux_sph(theta, tau_ref).double().cpu().numpy()
    Fso, _ = to.flux_sph(theta, tau_ref, nthreads=NTHREADS)
    assert np.all(np.abs(Fs - Fso) <= tol * Fso)


@pytest.mark.parametrize("case", range(8))
def test_random_configuration_adjoint_bands_background(case):
    """Seeded random sets: both adjoints (binary64), two opacity bands, the
    background shell and the second moment against the oracle."""
    rng = np.random.default_rng(5000 + case)
    n = int(rng.integers(2, 2500))
    prec = "f32" if case % 3 == 0 else "f64"
    bucket = int(rng.choice([1, 2, 4, 8, 16]))
    theta = float(rng.choice([0.0, 0.3, 0.5, 0.75, 1.0]))
    tau_ref = float(rng.choice([-1.0, 0.0, 0.02, 0.1, 0.5, math.inf]))
    geom = case % 4
    if geom == 0:
        pos = rng.random((n, 3))
    elif geom == 1:
        k = int(round(n ** (1 / 3))) + 1
        pos = rng.integers(0, k, (n, 3)) / k
    elif geom == 2:
        c = rng.random((5, 3))
        pos = np.clip(c[rng.integers(0, 5, n)] + 0.02 * rng.standard_normal((n, 3)), 0,
                      0.999999)
    else:
        pos = rng.integers(0, 64, (n, 3)) / 64.0
    print("case %d n %d %s N_B %d theta %g tau_ref %g geometry %d" % (case, n, prec, bucket,
                                                                       theta, tau_ref, geom),
          flush=True)
    rho = np.exp(rng.standard_normal(n))
    kappa = rng.uniform(0.0, 4.0, n)
    lum = np.where(rng.random(n) < rng.uniform(0.05, 0.6), 10 ** rng.standard_normal(n), 0.0)
    mass = rng.uniform(0.0, 2.0, n) / n
    mass[rng.random(n) < 0.1] = 0.0
    npdt = np.float64 if prec == "f64" else np.float32
    arrs = [a.astype(npdt) for a in (pos, rho, kappa, lum, mass)]
    dt = torch.float64 if prec == "f64" else torch.float32
    d = lambda a: torch.as_tensor(a, dtype=dt, device="cuda")  # noqa: E731
    tol = 1e-12 if prec == "f64" else 1e-5
    tg = P.build_tree(*[d(a) for a in arrs], bucket_size=bucket)
    f = lambda a: np.asarray(a, np.float64)  # noqa: E731
    to = OracleTree(*[f(a) for a in arrs], bucket_size=bucket, mirror32=(prec == "f32"))
    if prec == "f64":
        gF = rng.uniform(0.5, 1.5, n)
        go = to.adjoint(theta, tau_ref, gF, nthreads=NTHREADS)
        ga = tg.adjoint(theta, tau_ref, torch.as_tensor(gF, device="cuda"))
        tg.flux(theta, tau_ref, tape=True)
        gt = tg.adjoint_taped(torch.as_tensor(gF, device="cuda"))
        for a_, t_, o in zip(ga, gt, go):
            sc = max(np.max(np.abs(o)), 1e-300)
            assert np.max(np.abs(a_.cpu().numpy() - o)) <= 1e-10 * sc
            assert np.max(np.abs(t_.cpu().numpy() - o)) <= 1e-10 * sc
    kb = np.stack([arrs[2], (arrs[2] * rng.uniform(0.2, 3.0, n)).astype(npdt)])
    tg.set_bands(torch.as_tensor(kb, device="cuda"))
    Fb = tg.flux_bands(theta, tau_ref).double().cpu().numpy()
    Fbo, _ = to.flux_bands(theta, tau_ref, kb.astype(np.float64), nthreads=NTHREADS)
    assert np.all(np.abs(Fb - Fbo) <= tol * Fbo)
    flags = (rng.random(n) < 0.3).astype(np.uint8)
    tg.set_background((0.5, 0.5, 0.5), 0.4, torch.as_tensor(flags, device="cuda"))
    to.set_background(np.array([0.5, 0.5, 0.5]), 0.4, flags)
    Fg = tg.flux_background(theta, tau_ref).double().cpu().numpy()
    Fgo, _ = to.flux_background(theta, tau_ref, nthreads=NTHREADS)
    assert np.all(np.abs(Fg - Fgo) <= tol * Fgo)
    Pm = tg.flux_moments(theta, tau_ref)[2].double().cpu().numpy()
    Fo, _, Pmo = to.flux_moments(theta, tau_ref, nthreads=NTHREADS)
    assert np.all(np.abs(Pm - Pmo) <= tol * Fo[:, None])
