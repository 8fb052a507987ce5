"""GPU: a tree far deeper than the wave-shared part of the sink chain.

512 particles in a cube of side 1e-4 inside 3000 spread ones: the cluster's
cells lie about 40 levels deep, so the 64 sinks of a wave inside it share
ancestors below depth 31, past the wave-shared prefix of the sink chain, and
the trace finds those levels by descending from the prefix.  Flux and
counters at every sink against the oracle (binary64 and binary32 mirror), and
the taped adjoint in binary64.
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


def _deep_case(prec, seed=31):
    rng = np.random.default_rng(seed)
    spread = rng.random((3000, 3))
    cluster = np.array([0.4137, 0.6021, 0.2893]) + 1e-4 * rng.random((512, 3))
    pos = np.vstack([spread, cluster])
    n = pos.shape[0]
    rho = np.exp(0.4 * rng.standard_normal(n))
    kappa = rng.uniform(1.0, 4.0, n)
    lum = np.zeros(n)
    lum[rng.choice(n, 300, replace=False)] = rng.uniform(0.5, 2.0, 300)
    lum[3000:3100] = 1.0  # sources inside the cluster too
    mass = np.full(n, 1.0 / n)
    npdt = np.float64 if prec == "f64" else np.float32
    arrs = [a.astype(npdt) for a in (pos, rho, kappa, lum, mass)]
    dt = torch.float64 if prec == "f64" else torch.float32
    d = lambda a: torch.as_tensor(a, dtype=dt, device="cuda")  # noqa: E731
    tg = P.build_tree(*[d(a) for a in arrs])
    f = lambda a: np.asarray(a, np.float64)  # noqa: E731
    to = OracleTree(*[f(a) for a in arrs], mirror32=(prec == "f32"))
    return arrs, tg, to, n


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("theta,tau_ref", [(0.75, 0.1), (0.75, -1.0)])
def test_deep_cluster_flux_and_counters(prec, theta, tau_ref):
    _note("deep cluster %s theta %g tau_ref %g" % (prec, theta, tau_ref))
    _, tg, to, n = _deep_case(prec)
    info = tg.info()
    assert info["max_depth"] >= 40, info["max_depth"]
    Fg, Cg = tg.flux(theta, tau_ref, counters=True)
    Fo, Co = to.flux(theta, tau_ref, nthreads=NTHREADS)
    Fg = Fg.double().cpu().numpy()
    rel = np.abs(Fg - Fo) / Fo
    tol = 1e-12 if prec == "f64" else 1e-5
    assert rel.max() <= tol, (int(np.argmax(rel)), float(rel.max()))
    assert np.array_equal(Cg.cpu().numpy().astype(np.int64), Co)


def test_deep_cluster_taped_adjoint():
    _note("deep cluster taped adjoint f64")
    _, tg, to, n = _deep_case("f64")
    gF = np.random.default_rng(32).standard_normal(n)
    tg.flux(0.75, 0.1, tape=True)
    gr, gk, gl = tg.adjoint_taped(torch.as_tensor(gF, dtype=torch.float64, device="cuda"))
    orr, ok, ol = to.adjoint(0.75, 0.1, gF, nthreads=NTHREADS)
    for name, g, o in (("rho", gr, orr), ("kappa", gk, ok), ("lum", gl, ol)):
        g = g.cpu().numpy()
        scale = np.max(np.abs(o))
        err = np.abs(g - o) / (np.abs(o) + 1e-6 * scale)
        assert err.max() <= 1e-10, (name, float(err.max()))
