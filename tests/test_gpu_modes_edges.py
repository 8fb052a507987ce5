"""GPU: small, empty and degenerate inputs for the modes beyond the plain
flux -- the particle trace below the buckets, the walk variants, the
background shell and the ionisation update -- against the oracle.

  * trees of 0, 1, 2 and 65 particles (an empty tree has one empty cell);
  * an empty sink list;
  * a coincident cluster exactly on split planes and a plane of points, with
    merged sources and refinement always on.
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


def _arrays(n, seed, degenerate=False):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    if degenerate and n >= 100:
        pos[:30] = 0.5       # a coincident cluster on three split planes
        pos[30:60, 1] = 0.25  # a plane of points
    rho = np.exp(rng.standard_normal(n))
    kappa = rng.uniform(0.5, 3.0, n)
    lum = np.where(rng.random(n) < 0.4, 10 ** rng.standard_normal(n), 0.0)
    mass = np.full(n, 1.0 / max(n, 1))
    h = 1.2 * (mass / rho) ** (1.0 / 3.0)
    flags = (rng.random(n) < 0.3).astype(np.uint8)
    return pos, rho, kappa, lum, mass, h, flags


def _trees(n, seed, degenerate=False, bucket=8):
    pos, rho, kappa, lum, mass, h, flags = _arrays(n, seed, degenerate)
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")  # noqa: E731
    tg = P.build_tree(d(pos), d(rho), d(kappa), d(lum), d(mass), bucket_size=bucket)
    tg.set_sph(d(h))
    tg.set_background((0.5, 0.5, 0.5), 0.45, torch.as_tensor(flags, device="cuda"))
    to = None
    if n > 0:
        to = OracleTree(pos, rho, kappa, lum, mass, bucket_size=bucket)
        to.set_sph(h)
        to.set_background(np.array([0.5, 0.5, 0.5]), 0.45, flags)
    return tg, to


def _close(F, Fo):
    F = F.double().cpu().numpy()
    assert np.all(np.abs(F - Fo) <= 1e-12 * np.abs(Fo) + 1e-300)


@pytest.mark.parametrize("n", [0, 1, 2, 65])
def test_small_trees(n):
    _note("modes on a tree of %d particles" % n)
    tg, to = _trees(n, 40 + n)
    for theta, tau_ref in ((0.75, 0.1), (0.5, -1.0)):
        F = tg.flux_sph(theta, tau_ref)
        Fv = tg.flux_variant(theta, tau_ref, 2, 1, 3.0)
        Fb = tg.flux_background(theta, tau_ref)
        assert F.numel() == Fv.numel() == Fb.numel() == n
        if n == 0:
            continue
        _close(F, to.flux_sph(theta, tau_ref)[0])
        _close(Fv, to.flux_variant(theta, tau_ref, 2, 1, 3.0)[0])
        _close(Fb, to.flux_background(theta, tau_ref)[0])
    x = torch.full((n,), 0.5, dtype=torch.float64, device="cuda")
    k = torch.empty_like(x)
    dx = P.ionisation_update(torch.zeros_like(x), x, k, 2.0, 1.0)
    assert float(dx.item()) == (0.5 if n > 0 else 0.0)


def test_empty_sink_lists():
    _note("modes with an empty sink list")
    tg, to = _trees(500, 7)
    s = torch.empty(0, dtype=torch.int32, device="cuda")
    assert tg.flux_sph(0.75, 0.1, sinks=s).numel() == 0
    assert tg.flux_variant(0.75, 0.1, 1, 0, sinks=s).numel() == 0
    assert tg.flux_background(0.75, 0.1, sinks=s).numel() == 0


@pytest.mark.parametrize("bucket", [1, 8])
def test_degenerate_geometry(bucket):
    _note("modes on degenerate geometry, N_B %d" % bucket)
    tg, to = _trees(1500, 9, degenerate=True, bucket=bucket)
    for theta, tau_ref in ((0.75, -1.0), (1.0, 0.1)):
        F, C = tg.flux(theta, tau_ref, counters=True)
        Fo, Co = to.flux(theta, tau_ref, nthreads=NTHREADS)
        assert np.array_equal(C.cpu().numpy().astype(np.int64), Co)
        _close(F, Fo)
        _close(tg.flux_sph(theta, tau_ref), to.flux_sph(theta, tau_ref, nthreads=NTHREADS)[0])
        for om, rm in ((1, 0), (2, 1), (0, 1)):
            _close(tg.flux_variant(theta, tau_ref, om, rm),
                   to.flux_variant(theta, tau_ref, om, rm, nthreads=NTHREADS)[0])
        _close(tg.flux_background(theta, tau_ref),
               to.flux_background(theta, tau_ref, nthreads=NTHREADS)[0])
