"""GPU: several opacity bands on one traversal (trevr_set_bands,
trevr_compute_flux_bands) through the C ABI, against the oracle.

  * three bands, binary64 and binary32 transport: each band's flux within
    1e-12 (binary64) or 1e-5 (binary32) of the oracle's, and the traversal's
    counters identical (decisions on the largest band spread);
  * one band equal to the tree's opacity: the plain flux up to summation
    order, with identical counters;
  * refusals: more than four bands, a negative opacity, no bands set, bands
    dropped by a refit.
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


def _setup(prec, n, seed, k):
    arrs = W.lognormal_box(n, n // 20, 8.0, seed)
    w = W._pack("bands", *arrs, prec=prec)
    rng = np.random.default_rng(seed + 7)
    kb = np.asarray(w["kappa"], np.float64)[None, :] * rng.uniform(0.2, 3.0, (k, 1))
    kb[-1] *= rng.uniform(0.5, 1.5, n)  # one band with its own spatial structure
    npdt = np.float64 if prec == "f64" else np.float32
    kb = kb.astype(npdt)
    dt = torch.float64 if prec == "f64" else torch.float32
    f = lambda key: torch.as_tensor(w[key], dtype=dt, device="cuda")  # noqa: E731
    tg = P.build_tree(f("pos"), f("rho"), f("kappa"), f("lum"), f("mass"), w["box_lo"],
                      w["box_hi"], w["bucket_size"])
    g = lambda a: np.asarray(a, np.float64)  # noqa: E731
    to = OracleTree(g(w["pos"]), g(w["rho"]), g(w["kappa"]), g(w["lum"]), g(w["mass"]),
                    w["box_lo"], w["box_hi"], w["bucket_size"], mirror32=(prec == "f32"))
    return w, tg, to, kb


@pytest.mark.parametrize("prec,theta,tau_ref", [("f64", 0.75, 0.1), ("f32", 0.75, 0.1),
                                                ("f64", 0.5, -1.0)])
def test_bands_match_oracle(prec, theta, tau_ref):
    _note("bands %s theta %g tau_ref %g" % (prec, theta, tau_ref))
    w, tg, to, kb = _setup(prec, 1 << 13, 111, 3)
    tg.set_bands(torch.as_tensor(kb, device="cuda"))
    Fb, C = tg.flux_bands(theta, tau_ref, counters=True)
    Fbo, Co = to.flux_bands(theta, tau_ref, kb.astype(np.float64), nthreads=NTHREADS)
    assert np.array_equal(C.cpu().numpy().astype(np.int64), Co)
    tol = 1e-12 if prec == "f64" else 1e-5
    rel = np.abs(Fb.double().cpu().numpy() - Fbo) / Fbo
    _note("worst band rel err %.3g" % rel.max())
    assert rel.max() <= tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_one_band_is_the_plain_flux(prec):
    _note("one band = the plain flux, %s" % prec)
    w, tg, to, kb = _setup(prec, 6000, 112, 1)
    dt = torch.float64 if prec == "f64" else torch.float32
    tg.set_bands(torch.as_tensor(np.asarray(w["kappa"])[None, :], dtype=dt, device="cuda"))
    Fb, Cb = tg.flux_bands(0.75, 0.1, counters=True)
    F, C = tg.flux(0.75, 0.1, counters=True)
    assert torch.equal(Cb, C)
    rt = 1e-12 if prec == "f64" else 3e-7
    assert torch.allclose(Fb[:, 0], F, rtol=rt, atol=0)


def test_band_refusals():
    _note("band refusals")
    w, tg, to, kb = _setup("f64", 3000, 113, 2)
    with pytest.raises(P.TrevrError) as e:
        tg.flux_bands(0.75, 0.1)
    assert e.value.status == -5
    with pytest.raises(P.TrevrError) as e:
        tg.set_bands(torch.ones((5, 3000), dtype=torch.float64, device="cuda"))
    assert e.value.status == -1
    bad = kb.copy()
    bad[1, 17] = -1.0
    with pytest.raises(P.TrevrError) as e:
        tg.set_bands(torch.as_tensor(bad, device="cuda"))
    assert e.value.status == -4
    tg.set_bands(torch.as_tensor(kb, device="cuda"))
    Fb = tg.flux_bands(0.75, 0.1)
    assert Fb.shape == (3000, 2) and bool(torch.isfinite(Fb).all())
    d = lambda k: torch.as_tensor(w[k], dtype=torch.float64, device="cuda")  # noqa: E731
    tg.refit(d("pos"), d("rho"), d("kappa"), d("lum"), d("mass"))
    with pytest.raises(P.TrevrError) as e:
        tg.flux_bands(0.75, 0.1)
    assert e.value.status == -5
