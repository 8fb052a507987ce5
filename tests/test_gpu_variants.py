"""GPU: the walk variants (trevr_compute_flux_variant) through the C ABI,
against the oracle.

  * each opening test (sink point, bucket box, Gasoline's opening radius) and
    each ray walk (up the tree, top down from the meeting cell): the flux
    within 1e-12 (binary64) or 1e-5 (binary32) of the oracle's, counters
    identical (integer work);
  * early termination: the flux within the same bounds (a ray's cut is
    decided on its full optical depth in both), counters never above the
    plain walk's;
  * modes 0 / 0 / infinity: the plain flux and counters;
  * refusals of modes out of range and of tau_max <= 0.
"""
import math
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


def _setup(prec, n, seed):
    arrs = W.lognormal_box(n, n // 10, 8.0, seed)
    w = W._pack("variants", *arrs, prec=prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    f = lambda k: torch.as_tensor(w[k], dtype=dt, device="cuda")  # noqa: E731
    tg = P.build_tree(f("pos"), f("rho"), f("kappa"), f("lum"), f("mass"), w["box_lo"],
                      w["box_hi"], w["bucket_size"])
    g = lambda a: np.asarray(a, np.float64)  # noqa: E731
    to = OracleTree(g(w["pos"]), g(w["rho"]), g(w["kappa"]), g(w["lum"]), g(w["mass"]),
                    w["box_lo"], w["box_hi"], w["bucket_size"], mirror32=(prec == "f32"))
    return w, tg, to


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("open_mode,ray_mode,theta,tau_ref", [
    (1, 0, 0.75, 0.1), (2, 0, 0.75, 0.1), (0, 1, 0.75, 0.1), (0, 1, 0.5, -1.0),
    (2, 1, 1.0, 0.05), (1, 1, 0.75, float("inf"))])
def test_variants_match_oracle(prec, open_mode, ray_mode, theta, tau_ref):
    _note("variant %s open %d ray %d theta %g tau_ref %g" % (prec, open_mode, ray_mode, theta,
                                                            tau_ref))
    w, tg, to = _setup(prec, 1 << 13, 301)
    F, C = tg.flux_variant(theta, tau_ref, open_mode, ray_mode, counters=True)
    Fo, Co = to.flux_variant(theta, tau_ref, open_mode, ray_mode, nthreads=NTHREADS)
    assert np.array_equal(C.cpu().numpy().astype(np.int64), Co)
    tol = 1e-12 if prec == "f64" else 1e-5
    rel = np.abs(F.double().cpu().numpy() - Fo) / Fo
    _note("worst rel err %.3g" % rel.max())
    assert rel.max() <= tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_early_termination_matches_oracle(prec):
    _note("early termination %s" % prec)
    w, tg, to = _setup(prec, 1 << 13, 302)
    F0, C0 = tg.flux(0.75, 0.1, counters=True)
    for tau_max, ray_mode in ((2.0, 0), (0.7, 1)):
        F, C = tg.flux_variant(0.75, 0.1, 0, ray_mode, tau_max, counters=True)
        Fo, _ = to.flux_variant(0.75, 0.1, 0, ray_mode, tau_max, nthreads=NTHREADS)
        # rays whose tau sits within rounding of tau_max may be cut on one side
        # only; each carries at most L e^-tau_max / (4 pi r^2)
        tol = 1e-12 if prec == "f64" else 1e-5
        err = np.abs(F.double().cpu().numpy() - Fo)
        _note("tau_max %g: %d sinks with every ray cut" % (tau_max, int((Fo == 0).sum())))
        assert np.all(err <= tol * Fo)  # zero where every ray is cut
        Fm = tg.flux_variant(0.75, 0.1, 0, ray_mode)  # the same walk without the cut
        assert bool((F <= Fm * (1 + 1e-6)).all())
        if ray_mode == 0:
            assert bool((C[:, 4] <= C0[:, 4]).all()) and bool((C[:, :3] == C0[:, :3]).all())
            assert int(C[:, 4].sum()) < int(C0[:, 4].sum())


def test_defaults_and_refusals():
    _note("variant defaults and refusals")
    w, tg, to = _setup("f32", 5000, 303)
    F0, C0 = tg.flux(0.75, 0.1, counters=True)
    F, C = tg.flux_variant(0.75, 0.1, counters=True)
    assert torch.equal(C, C0)
    assert torch.allclose(F, F0, rtol=3e-7, atol=0)
    for args in ((3, 0, 1.0), (0, 2, 1.0), (0, 0, 0.0), (0, 0, float("nan")), (-1, 0, 1.0)):
        with pytest.raises(P.TrevrError) as e:
            tg.flux_variant(0.75, 0.1, *args)
        assert e.value.status == -1
    sinks = torch.tensor([3, -2, 4999], dtype=torch.int32, device="cuda")
    F = tg.flux_variant(0.75, 0.1, 1, 1, 3.0, sinks=sinks).cpu().numpy()
    assert np.isnan(F[1]) and np.isfinite(F[[0, 2]]).all()
