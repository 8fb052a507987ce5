"""GPU regression: sources exactly on split planes with refinement always on.

When a merged source's point lies on the meeting cell's plane, the ray's
source-side interval is empty; the sink-side refinement jobs left on the
lane's stack must still be traced.  Flux, adjoint (plain and taped), vector
flux and bands against the oracle on a jittered grid with sources at cell
corners of the tree (0.5, 0.25, 0.75 coordinates), binary64 and binary32;
and an unjittered 16^3 lattice (every particle on split planes of many
levels, rays inside planes): flux, top-down walk and taped adjoint.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1902_08083_amd as P  # noqa: E402
from oracle.oracle import OracleTree  # noqa: E402

NTHREADS = min(16, os.cpu_count() or 1)


def _note(msg):
    print(msg, flush=True)


def _case(prec, n1=14, seed=12):
    rng = np.random.default_rng(seed)
    g = (np.stack(np.meshgrid(*[np.arange(n1)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5
         + 0.3 * (rng.random((n1 ** 3, 3)) - 0.5)) / n1
    corners = np.array([[0.5, 0.5, 0.5], [0.25, 0.5, 0.75], [0.75, 0.25, 0.5],
                        [0.5, 0.75, 0.25]])
    pos = np.vstack([g, corners])
    n = pos.shape[0]
    lum = np.r_[np.zeros(n1 ** 3), [1.0, 0.5, 2.0, 0.7]]
    lum[rng.choice(n1 ** 3, 20, replace=False)] = 0.3
    rho = np.exp(0.5 * rng.standard_normal(n))
    kappa = rng.uniform(2.0, 6.0, n)
    mass = np.r_[np.full(n1 ** 3, 1.0 / n1 ** 3), np.zeros(4)]
    npdt = np.float64 if prec == "f64" else np.float32
    arrs = [a.astype(npdt) for a in (pos, rho, kappa, lum, mass)]
    dt = torch.float64 if prec == "f64" else torch.float32
    d = lambda a: torch.as_tensor(a, dtype=dt, device="cuda")  # noqa: E731
    tg = P.build_tree(*[d(a) for a in arrs])
    f = lambda a: np.asarray(a, np.float64)  # noqa: E731
    to = OracleTree(*[f(a) for a in arrs], mirror32=(prec == "f32"))
    return arrs, tg, to, n


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("theta,tau_ref", [(0.75, -1.0), (1.0, -1.0), (0.5, 0.0)])
def test_sources_on_planes(prec, theta, tau_ref):
    _note("sources on split planes %s theta %g tau_ref %g" % (prec, theta, tau_ref))
    arrs, tg, to, n = _case(prec)
    tol = 1e-12 if prec == "f64" else 1e-5
    F, C = tg.flux(theta, tau_ref, counters=True)
    Fo, Co = to.flux(theta, tau_ref, nthreads=NTHREADS)
    assert np.array_equal(C.cpu().numpy().astype(np.int64), Co)
    assert np.max(np.abs(F.double().cpu().numpy() - Fo) / Fo) <= tol
    Fv = tg.flux_vector(theta, tau_ref)[1].double().cpu().numpy()
    Fvo = to.flux_vector(theta, tau_ref, nthreads=NTHREADS)[1]
    assert np.max(np.abs(Fv - Fvo) / Fo[:, None]) <= tol
    kb = np.stack([arrs[2], 2 * arrs[2]])
    tg.set_bands(torch.as_tensor(kb, device="cuda"))
    Fb = tg.flux_bands(theta, tau_ref).double().cpu().numpy()
    Fbo, _ = to.flux_bands(theta, tau_ref, kb.astype(np.float64), nthreads=NTHREADS)
    assert np.max(np.abs(Fb - Fbo) / Fbo) <= tol
    if prec == "f64":
        gF = np.random.default_rng(1).uniform(0.5, 1.5, n)
        go = to.adjoint(theta, tau_ref, gF, nthreads=NTHREADS)
        gd = torch.as_tensor(gF, device="cuda")
        ga = tg.adjoint(theta, tau_ref, gd)
        tg.flux(theta, tau_ref, tape=True)
        gt = tg.adjoint_taped(gd)
        for a, t_, o in zip(ga, gt, go):
            scale = np.max(np.abs(o))
            assert np.max(np.abs(a.cpu().numpy() - o)) <= 1e-10 * scale
            assert np.max(np.abs(t_.cpu().numpy() - o)) <= 1e-10 * scale


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("theta,tau_ref,bucket", [(0.75, -1.0, 8), (0.75, 0.1, 8),
                                                  (1.0, -1.0, 1), (0.0, 0.05, 4)])
def test_regular_lattice(prec, theta, tau_ref, bucket):
    """Every particle on split planes of many levels (an unjittered 16^3
    lattice): rays inside planes, sources and sinks on cell faces and corners."""
    _note("regular lattice %s theta %g tau_ref %g N_B %d" % (prec, theta, tau_ref, bucket))
    n1 = 16
    g = np.stack(np.meshgrid(*[np.arange(n1)] * 3, indexing="ij"), -1).reshape(-1, 3) / n1
    n = g.shape[0]
    rng = np.random.default_rng(21)
    lum = np.zeros(n)
    lum[rng.choice(n, 150, replace=False)] = 10 ** rng.standard_normal(150)
    rho = np.exp(0.5 * rng.standard_normal(n))
    kappa = rng.uniform(1.0, 5.0, n)
    mass = np.full(n, 1.0 / n)
    npdt = np.float64 if prec == "f64" else np.float32
    arrs = [a.astype(npdt) for a in (g, rho, kappa, lum, mass)]
    dt = torch.float64 if prec == "f64" else torch.float32
    d = lambda a: torch.as_tensor(a, dtype=dt, device="cuda")  # noqa: E731
    tg = P.build_tree(*[d(a) for a in arrs], bucket_size=bucket)
    f = lambda a: np.asarray(a, np.float64)  # noqa: E731
    to = OracleTree(*[f(a) for a in arrs], bucket_size=bucket, mirror32=(prec == "f32"))
    F, C = tg.flux(theta, tau_ref, counters=True)
    Fo, Co = to.flux(theta, tau_ref, nthreads=NTHREADS)
    assert np.array_equal(C.cpu().numpy().astype(np.int64), Co)
    tol = 1e-12 if prec == "f64" else 1e-5
    assert np.max(np.abs(F.double().cpu().numpy() - Fo) / Fo) <= tol
    Ft = tg.flux_variant(theta, tau_ref, 0, 1).double().cpu().numpy()
    Fto, _ = to.flux_variant(theta, tau_ref, 0, 1, nthreads=NTHREADS)
    assert np.max(np.abs(Ft - Fto) / Fto) <= tol
    if prec == "f64":
        gF = rng.uniform(0.5, 1.5, n)
        go = to.adjoint(theta, tau_ref, gF, nthreads=NTHREADS)
        tg.flux(theta, tau_ref, tape=True)
        gt = tg.adjoint_taped(torch.as_tensor(gF, device="cuda"))
        for t_, o in zip(gt, go):
            assert np.max(np.abs(t_.cpu().numpy() - o)) <= 1e-10 * np.max(np.abs(o))
