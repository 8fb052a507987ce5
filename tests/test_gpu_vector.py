"""GPU: the vector flux (each ray's flux along its direction of travel at the
sink, summed over the sink's rays) through the C ABI, against the oracle.

  * binary64 and binary32 transport, merged sources and refinement, within
    1e-12 (binary64) or 1e-5 (binary32) of the sink's scalar flux;
  * the scalar flux and counters of the vector call equal the plain call's;
  * six equal sources about a sink cancel;
  * sink subsets with invalid indices (NaN), and launch shapes above four
    waves per SIMD (the vector kernel then runs at four);
  * the second moment (sum f n_a n_b) against the oracle, its trace equal to
    the flux, and F/3 on the diagonal for six symmetric sources.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1902_08083_amd as P  # noqa: E402
from paper_1902_08083_amd import workloads as W  # noqa: E402
from oracle.oracle import OracleTree  # noqa: E402

NTHREADS = min(16, os.cpu_count() or 1)


def _note(msg):
    print(msg, flush=True)


def _tree(w):
    dt = torch.float64 if w["prec"] == "f64" else torch.float32
    f = lambda k: torch.as_tensor(w[k], dtype=dt, device="cuda")  # noqa: E731
    return P.build_tree(f("pos"), f("rho"), f("kappa"), f("lum"),
                        None if w.get("mass") is None else f("mass"),
                        w["box_lo"], w["box_hi"], w["bucket_size"])


def _oracle(w):
    f = lambda a: None if a is None else np.asarray(a, np.float64)  # noqa: E731
    return OracleTree(f(w["pos"]), f(w["rho"]), f(w["kappa"]), f(w["lum"]), f(w.get("mass")),
                      w["box_lo"], w["box_hi"], w["bucket_size"], mirror32=(w["prec"] == "f32"))


@pytest.mark.parametrize("prec,theta,tau_ref", [("f64", 0.75, 0.1), ("f64", 0.0, -1.0),
                                                ("f32", 0.75, 0.1), ("f32", 1.0, 0.05)])
def test_vector_flux_matches_oracle(prec, theta, tau_ref):
    _note("vector flux %s theta %g tau_ref %g" % (prec, theta, tau_ref))
    arrs = W.lognormal_box(1 << 13, 400, 8.0, 71)
    w = W._pack("vec", *arrs, prec=prec)
    tg = _tree(w)
    F, Fv, C = tg.flux_vector(theta, tau_ref, counters=True)
    F0, C0 = tg.flux(theta, tau_ref, counters=True)
    assert torch.equal(F, F0) and torch.equal(C, C0)
    Fo, Fvo = _oracle(w).flux_vector(theta, tau_ref, nthreads=NTHREADS)
    tol = 1e-12 if prec == "f64" else 1e-5
    err = np.abs(Fv.double().cpu().numpy() - Fvo)
    worst = float(np.max(err / Fo[:, None]))
    _note("worst |Fv - oracle| / F = %.3g" % worst)
    assert worst <= tol


def test_vector_flux_symmetric_sources_cancel():
    _note("vector flux: six symmetric sources")
    c = np.array([0.5, 0.5, 0.5])
    h = 0.25
    src = np.array([c + s * h * e for e in np.eye(3) for s in (1.0, -1.0)])
    pos = np.vstack([c, src])
    dev = "cuda"
    t = P.build_tree(torch.tensor(pos, dtype=torch.float64, device=dev),
                     torch.ones(7, dtype=torch.float64, device=dev),
                     torch.zeros(7, dtype=torch.float64, device=dev),
                     torch.tensor([0.0] + [1.0] * 6, dtype=torch.float64, device=dev),
                     torch.ones(7, dtype=torch.float64, device=dev), bucket_size=1)
    sinks = torch.tensor([0], dtype=torch.int32, device=dev)
    F, Fv = t.flux_vector(0.0, 0.1, sinks=sinks)
    F, Fv = float(F[0]), Fv[0].cpu().numpy()
    assert abs(F - 6.0 / (4.0 * np.pi * h * h)) <= 1e-14 * F
    assert np.all(np.abs(Fv) <= 1e-15 * F)


def test_vector_flux_subset_and_launch_shapes():
    _note("vector flux: sink subset, invalid index, launch shapes")
    arrs = W.lognormal_box(5000, 200, 6.0, 72)
    w = W._pack("vec2", *arrs, prec="f64")
    tg = _tree(w)
    sinks = torch.tensor([4, -1, 4999, 12, 5000, 77], dtype=torch.int32, device="cuda")
    F, Fv = tg.flux_vector(0.75, 0.1, sinks=sinks)
    Fv = Fv.cpu().numpy()
    assert np.isnan(Fv[[1, 4]]).all() and np.isnan(F.cpu().numpy()[[1, 4]]).all()
    Fo, Fvo = _oracle(w).flux_vector(0.75, 0.1, sinks=np.array([4, 4999, 12, 77]),
                                      nthreads=NTHREADS)
    ok = [0, 2, 3, 5]
    assert np.all(np.abs(Fv[ok] - Fvo) <= 1e-12 * Fo[:, None])
    ref = tg.flux_vector(0.75, 0.1)[1].clone()
    for launch in [(8, 4, 64), (3, 4, 128), (2, 2, 64)]:
        tg.set_launch(*launch)
        assert torch.equal(tg.flux_vector(0.75, 0.1)[1], ref), launch


# ---- second moment (radiation pressure tensor times c) ----

@pytest.mark.parametrize("prec,theta,tau_ref", [("f64", 0.75, 0.1), ("f32", 0.75, 0.1),
                                                ("f64", 0.0, -1.0)])
def test_second_moment_matches_oracle(prec, theta, tau_ref):
    _note("second moment %s theta %g tau_ref %g" % (prec, theta, tau_ref))
    arrs = W.lognormal_box(1 << 13, 400, 8.0, 73)
    w = W._pack("mom", *arrs, prec=prec)
    tg = _tree(w)
    F, Fv, Pm = tg.flux_moments(theta, tau_ref)
    # another kernel variant: a refined chain piece is deferred or refined at
    # once depending on the LDS stack room, so tau's summation order (and its
    # last bits) may differ from the plain call's
    rt = 1e-12 if prec == "f64" else 3e-7
    F0 = tg.flux(theta, tau_ref)
    assert torch.allclose(F, F0, rtol=rt, atol=0)
    Fv0 = tg.flux_vector(theta, tau_ref)[1]
    assert float((Fv - Fv0).abs().max(dim=1).values.div(F0).max()) <= rt
    Fo, Fvo, Pmo = _oracle(w).flux_moments(theta, tau_ref, nthreads=NTHREADS)
    tol = 1e-12 if prec == "f64" else 1e-5
    Pm = Pm.double().cpu().numpy()
    worst = float(np.max(np.abs(Pm - Pmo) / Fo[:, None]))
    _note("worst |P - oracle| / F = %.3g" % worst)
    assert worst <= tol
    # the trace is the flux
    tr = Pm[:, 0] + Pm[:, 1] + Pm[:, 2]
    tol_tr = 1e-12 if prec == "f64" else 1e-6
    assert np.all(np.abs(tr - F.double().cpu().numpy()) <= tol_tr * Fo)


def test_second_moment_isotropic_and_launch_shapes():
    _note("second moment: isotropic sources, launch shapes")
    c = np.array([0.5, 0.5, 0.5])
    h = 0.25
    pos = np.vstack([c] + [c + s * h * e for e in np.eye(3) for s in (1.0, -1.0)])
    dev = "cuda"
    d64 = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)  # noqa: E731
    t = P.build_tree(d64(pos), d64(np.ones(7)), d64(np.zeros(7)), d64([0.0] + [1.0] * 6),
                     d64(np.ones(7)), bucket_size=1)
    F, _, Pm = t.flux_moments(0.0, 0.1, sinks=torch.tensor([0], dtype=torch.int32, device=dev))
    F, Pm = float(F[0]), Pm[0].cpu().numpy()
    assert np.all(np.abs(Pm[:3] - F / 3.0) <= 1e-15 * F)
    assert np.all(np.abs(Pm[3:]) <= 1e-16 * F)
    arrs = W.lognormal_box(4000, 150, 6.0, 74)
    tg = _tree(W._pack("mom2", *arrs, prec="f32"))
    ref = tg.flux_moments(0.75, 0.1)[2].clone()
    for launch in [(8, 4, 64), (4, 4, 64), (1, 1, 128)]:
        tg.set_launch(*launch)
        assert torch.equal(tg.flux_moments(0.75, 0.1)[2], ref), launch
