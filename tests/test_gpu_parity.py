"""GPU parity: the HIP library against the oracle, through the C ABI.

  * tree export (order, topology, binary64 cell data) bit-exact;
  * fluxes within 1e-12 relative in binary64 and within 1e-5 relative
    (stored binary32) in binary32 transport, against the oracle reading the
    same binary32-rounded cell data ("mirror"); the walk's integer counters
    identical;
  * at the full 2^21-particle size, sampled sinks of the same launch the
    benchmark times;
  * edge cases: empty and single-particle sets, ragged sink counts,
    coincident particles (depth cap), no sources, bucket size 1, refinement
    always / never, theta_open = 0, several boxes, sink subsets;
  * the adjoint against the oracle's adjoint.
"""
import math
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1902_08083_amd as P  # noqa: E402
from oracle.oracle import OracleTree  # noqa: E402
from paper_1902_08083_amd import workloads as W  # noqa: E402

NTHREADS = min(16, os.cpu_count() or 1)


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_tree(w, bucket=None):
    dt = torch.float64 if w["prec"] == "f64" else torch.float32
    dev = "cuda"
    t = P.build_tree(torch.as_tensor(w["pos"], dtype=dt, device=dev),
                     torch.as_tensor(w["rho"], dtype=dt, device=dev),
                     torch.as_tensor(w["kappa"], dtype=dt, device=dev),
                     torch.as_tensor(w["lum"], dtype=dt, device=dev),
                     None if w.get("mass") is None else torch.as_tensor(w["mass"], dtype=dt,
                                                                       device=dev),
                     w["box_lo"], w["box_hi"], bucket or w["bucket_size"])
    return t


def oracle_tree(w, bucket=None):
    f = lambda a: None if a is None else np.asarray(a, np.float64)  # noqa: E731
    return OracleTree(f(w["pos"]), f(w["rho"]), f(w["kappa"]), f(w["lum"]), f(w.get("mass")),
                      w["box_lo"], w["box_hi"], bucket or w["bucket_size"],
                      mirror32=(w["prec"] == "f32"))


def assert_flux_close(Fg, Fo, prec, what=""):
    Fg = np.asarray(Fg, np.float64)
    Fo = np.asarray(Fo, np.float64)
    if prec == "f64":
        tol = 1e-12
    else:
        tol = 1e-5
    denom = np.where(Fo != 0, np.abs(Fo), 1.0)
    rel = np.abs(Fg - Fo) / denom
    worst = int(np.argmax(rel)) if rel.size else 0
    assert rel.size == 0 or rel.max() <= tol, (what, worst, Fg[worst], Fo[worst], rel.max())
    return float(rel.max()) if rel.size else 0.0


def small_lognormal(n, n_src, tau_box, seed, all_sources=False, prec="f32"):
    arrs = W.lognormal_box(n, n_src, tau_box, seed, all_sources=all_sources)
    return W._pack("lognormal%d" % n, *arrs, prec=prec)


# ---------------------------------------------------------------- tree ----

@pytest.mark.parametrize("case", ["c1", "c2_2e15", "clustered_nb1", "box2x1x1"])
def test_tree_export_bit_exact(case):
    _note("tree export %s" % case)
    if case == "c1":
        w, nb = W.c1(), None
    elif case == "c2_2e15":
        w, nb = small_lognormal(1 << 15, 1024, 5.0, 2), None
    elif case == "clustered_nb1":
        w = small_lognormal(5000, 100, 5.0, 9, prec="f64")
        w["pos"][:50] = w["pos"][0]  # coincident points: depth-capped bucket
        nb = 1
    else:
        w = small_lognormal(20000, 300, 3.0, 4, prec="f64")
        w["pos"] = w["pos"] * np.array([2.0, 1.0, 1.0])
        w["box_hi"] = (2.0, 1.0, 1.0)
        nb = 4
    g = gpu_tree(w, nb).export()
    o = oracle_tree(w, nb).export()
    assert set(g) == set(o)
    for k in o:
        assert g[k].shape == o[k].shape, k
        if o[k].dtype == np.float64:
            same = (g[k] == o[k]) | (np.isnan(g[k]) & np.isnan(o[k]))
            assert np.all(same), (k, np.argmin(same))
        else:
            assert np.array_equal(g[k], o[k]), k


# ---------------------------------------------------------------- flux ----

def _parity(w, theta=None, tau_ref=None, sinks=None, bucket=None, check_counters=True):
    theta = w["theta"] if theta is None else theta
    tau_ref = w["tau_ref"] if tau_ref is None else tau_ref
    tg = gpu_tree(w, bucket)
    Fg, Cg = tg.flux(theta, tau_ref, sinks=None if sinks is None else torch.as_tensor(
        sinks, dtype=torch.int32, device="cuda"), counters=True)
    to = oracle_tree(w, bucket)
    Fo, Co = to.flux(theta, tau_ref, sinks=sinks, nthreads=NTHREADS)
    err = assert_flux_close(Fg.cpu().numpy(), Fo, w["prec"], (w["name"], theta, tau_ref))
    if check_counters:
        Cg = Cg.cpu().numpy().astype(np.int64)
        bad = np.nonzero(np.any(Cg != Co, axis=1))[0]
        assert bad.size == 0, ("counters differ", bad[:5], Cg[bad[:5]], Co[bad[:5]])
    return err, Fg, Cg


def test_flux_c1_fp64():
    _note("flux c1 fp64")
    err, _, C = _parity(W.c1())
    assert err <= 1e-12


def test_flux_c2_full_fp32():
    _note("flux c2 fp32, 2^18 particles, all sinks")
    _parity(W.c2())


@pytest.mark.parametrize("theta,tau_ref", W.C3_SWEEP)
def test_flux_c3_sweep_points_small(theta, tau_ref):
    _note("flux c3 recipe at 2^15, theta %g tau_ref %g" % (theta, tau_ref))
    w = small_lognormal(1 << 15, 0, 10.0, 3, all_sources=True)
    _parity(w, theta, tau_ref)


def test_flux_c3_full_size_sampled():
    """2^21 particles, every particle a source, all sinks in one launch (the
    benchmark's launch); the oracle evaluates a seeded sample of sinks."""
    _note("flux c3 full size (2^21), sampled")
    w = W.c3()
    tg = gpu_tree(w)
    Fg, Cg = tg.flux(w["theta"], w["tau_ref"], counters=True)
    Fg, Cg = Fg.cpu().numpy(), Cg.cpu().numpy()
    to = oracle_tree(w)
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(w["pos"].shape[0], size=384, replace=False))
    Fo, Co = to.flux(w["theta"], w["tau_ref"], sinks=sample, nthreads=NTHREADS)
    assert_flux_close(Fg[sample], Fo, "f32", "c3 sampled")
    assert np.array_equal(Cg[sample].astype(np.int64), Co)
    assert np.all(Fg > 0) and np.all(np.isfinite(Fg))


@pytest.mark.parametrize("theta,tau_ref", [(0.0, 0.1), (0.75, -1.0), (0.75, math.inf),
                                           (0.75, 0.0), (2.0, 0.1)])
def test_flux_limits_fp64(theta, tau_ref):
    _note("flux limits theta %g tau_ref %g" % (theta, tau_ref))
    w = small_lognormal(3000, 400, 5.0, 12, prec="f64")
    _parity(w, theta, tau_ref)


# Launch shapes selecting each register-budget variant of the walk kernel
# (waves per SIMD 3, 4, 5, 6, 8); their refinement stacks hold 10..2 entries
# in LDS, so full refinement (tau_ref < 0) runs past them into the private
# spill and, on the smallest, refines chain pieces at once instead of
# deferring them.
VARIANT_LAUNCHES = [(3, 4, 64), (4, 4, 64), (5, 4, 64), (6, 4, 64), (8, 4, 64)]


@pytest.mark.parametrize("launch", VARIANT_LAUNCHES)
def test_flux_every_kernel_variant_full_refinement_fp64(launch):
    _note("flux variant %s, full refinement, fp64" % (launch,))
    w = small_lognormal(1 << 13, 300, 8.0, 21, prec="f64")
    tg = gpu_tree(w)
    tg.set_launch(*launch)
    Fg, Cg = tg.flux(0.75, -1.0, counters=True)
    to = oracle_tree(w)
    Fo, Co = to.flux(0.75, -1.0, nthreads=NTHREADS)
    assert_flux_close(Fg.cpu().numpy(), Fo, "f64", ("variant", launch))
    assert np.array_equal(Cg.cpu().numpy().astype(np.int64), Co)


@pytest.mark.parametrize("launch", [(3, 4, 64), (4, 4, 64), (8, 4, 64)])
def test_adjoint_kernel_variants_full_refinement_fp64(launch):
    _note("adjoint variant %s, full refinement, fp64" % (launch,))
    w = small_lognormal(1 << 12, 200, 8.0, 22, prec="f64")
    gF = np.random.default_rng(23).standard_normal(w["pos"].shape[0])
    tg = gpu_tree(w)
    tg.set_launch(*launch, adjoint=True)
    assert tg.get_launch(adjoint=True) == dict(zip(("blocks_per_cu", "waves_per_block", "chunk"),
                                                   launch))
    gr, gk, gl = tg.adjoint(0.75, -1.0, torch.as_tensor(gF, dtype=torch.float64, device="cuda"))
    orr, ok, ol = oracle_tree(w).adjoint(0.75, -1.0, gF, nthreads=NTHREADS)
    for name, g, o in (("rho", gr, orr), ("kappa", gk, ok), ("lum", gl, ol)):
        g = g.cpu().numpy()
        scale = np.max(np.abs(o))
        err = np.abs(g - o) / (np.abs(o) + 1e-6 * scale)
        assert err.max() <= 1e-10, (name, launch, float(err.max()))


@pytest.mark.parametrize("launch", [(3, 4, 64), (4, 4, 64), (6, 4, 64), (8, 4, 64)])
def test_adjoint_kernel_variants_fp32(launch):
    """Binary32 transport on every adjoint table size: 256 slots at 3 waves per
    SIMD, 128 at 4, 64 at 6 and 8, where most of a round's cells miss the
    table and take slots over from each other."""
    _note("adjoint variant %s, fp32" % (launch,))
    w = small_lognormal(1 << 14, 400, 10.0, 24, prec="f32")
    gF = np.random.default_rng(25).standard_normal(w["pos"].shape[0])
    tg = gpu_tree(w)
    tg.set_launch(*launch, adjoint=True)
    gr, gk, gl = tg.adjoint(0.75, 0.1, torch.as_tensor(gF, dtype=torch.float32, device="cuda"))
    gF = gF.astype(np.float32).astype(np.float64)
    orr, ok, ol = oracle_tree(w).adjoint(0.75, 0.1, gF, nthreads=NTHREADS)
    for name, g, o in (("rho", gr, orr), ("kappa", gk, ok), ("lum", gl, ol)):
        g = g.cpu().numpy().astype(np.float64)
        scale = np.max(np.abs(o))
        err = np.abs(g - o) / (np.abs(o) + 1e-6 * scale)
        assert err.max() <= 2e-6, (name, launch, float(err.max()))


def test_flux_sink_subset_and_order():
    _note("flux sink subset")
    w = small_lognormal(40000, 2000, 5.0, 13)
    rng = np.random.default_rng(3)
    sinks = rng.choice(40000, size=1000, replace=True)  # any order, repeats allowed
    _parity(w, sinks=sinks)
    tg = gpu_tree(w)
    full = tg.flux(0.75, 0.1).cpu().numpy()
    sub = tg.flux(0.75, 0.1, sinks=torch.as_tensor(sinks, dtype=torch.int32,
                                                   device="cuda")).cpu().numpy()
    assert np.array_equal(sub, full[sinks])


@pytest.mark.parametrize("n", [0, 1, 2, 63, 65, 1000])
def test_flux_small_and_ragged(n):
    _note("flux n = %d" % n)
    rng = np.random.default_rng(n + 1)
    w = W._pack("ragged%d" % n, rng.random((n, 3)), np.exp(rng.standard_normal(n)),
                rng.uniform(0.5, 2, n), np.where(rng.random(n) < 0.5, 1.0, 0.0),
                np.full(n, 1.0), prec="f64")
    if n == 0:
        tg = gpu_tree(w)
        assert tg.info()["m"] == 1
        assert tg.flux(0.75, 0.1).numel() == 0
        return
    _parity(w)


def test_flux_degenerate_inputs():
    _note("flux degenerate inputs")
    rng = np.random.default_rng(5)
    n = 2000
    pos = rng.random((n, 3))
    pos[:40] = 0.5  # coincident cluster exactly on split planes
    pos[40:80, 0] = 0.25  # a plane of points
    lum = np.where(rng.random(n) < 0.3, 1.0, 0.0)
    mass = rng.uniform(0.5, 1.5, n)
    mass[::7] = 0.0  # pure sources
    w = W._pack("degenerate", pos, np.exp(rng.standard_normal(n)), rng.uniform(0, 2, n), lum,
                mass, prec="f64")
    for nb in (1, 8):
        _parity(w, bucket=nb)
        _parity(w, 0.0, -1.0, bucket=nb)
    w0 = dict(w, lum=np.zeros(n))
    tg = gpu_tree(w0)
    assert np.all(tg.flux(0.75, 0.1).cpu().numpy() == 0.0)


def test_flux_forest_matches_single_boxes():
    _note("forest of 12 boxes")
    boxes = W.c4(n_boxes=12, max_log2=13)
    n_off = np.cumsum([0] + [b["pos"].shape[0] for b in boxes])
    cat = lambda k: np.concatenate([b[k] for b in boxes])  # noqa: E731
    # shift each box to its own corner region to check per-box geometry
    lo = np.array([[2.0 * b, 0.0, 0.0] for b in range(12)])
    hi = lo + 1.0
    pos = np.concatenate([b["pos"].astype(np.float64) + lo[i] for i, b in enumerate(boxes)])
    dt = torch.float32
    t = P.Tree().build(torch.as_tensor(pos.astype(np.float32), device="cuda"),
                       torch.as_tensor(cat("rho"), device="cuda"),
                       torch.as_tensor(cat("kappa"), device="cuda"),
                       torch.as_tensor(cat("lum"), device="cuda"),
                       torch.as_tensor(cat("mass"), device="cuda"), lo, hi, 8, n_off)
    Fg, Cg = t.flux(0.75, 0.1, counters=True)
    Fg, Cg = Fg.cpu().numpy(), Cg.cpu().numpy()
    for i, b in enumerate(boxes):
        bb = dict(b, pos=(b["pos"].astype(np.float64) + lo[i]).astype(np.float32),
                  box_lo=tuple(lo[i]), box_hi=tuple(hi[i]))
        Fo, Co = oracle_tree(bb).flux(0.75, 0.1, nthreads=NTHREADS)
        sl = slice(n_off[i], n_off[i + 1])
        assert_flux_close(Fg[sl], Fo, "f32", "box %d" % i)
        assert np.array_equal(Cg[sl].astype(np.int64), Co)


def test_flux_repeatable():
    _note("flux repeatable")
    w = small_lognormal(1 << 16, 2000, 5.0, 21)
    tg = gpu_tree(w)
    a = tg.flux(0.75, 0.1)
    b = tg.flux(0.75, 0.1)
    assert torch.equal(a, b)
    tg2 = gpu_tree(small_lognormal(5000, 100, 5.0, 22))  # handle reuse with other sizes
    tg.build(*[torch.as_tensor(x, device="cuda") for x in
               (w["pos"], w["rho"], w["kappa"], w["lum"], w["mass"])])
    assert torch.equal(tg.flux(0.75, 0.1), a)
    del tg2


@pytest.mark.parametrize("bad,status", [("outside", -2), ("nan", -3), ("neg_kappa", -4),
                                        ("zero_rho", -4)])
def test_build_rejects_bad_input(bad, status):
    n = 100
    rng = np.random.default_rng(1)
    pos = rng.random((n, 3))
    rho, kappa, lum = np.ones(n), np.ones(n), np.ones(n)
    if bad == "outside":
        pos[5, 1] = 1.0
    elif bad == "nan":
        lum[3] = np.nan
    elif bad == "neg_kappa":
        kappa[7] = -1.0
    else:
        rho[9] = 0.0
    t = P.Tree()
    with pytest.raises(P.TrevrError) as e:
        t.build(*[torch.as_tensor(x, device="cuda") for x in (pos, rho, kappa, lum)])
    assert e.value.status == status
    with pytest.raises(P.TrevrError) as e:
        t.flux(0.75, 0.1)
    assert e.value.status == -5  # no tree after a failed build


# ------------------------------------------------------------- adjoint ----

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_matches_oracle(prec):
    _note("adjoint parity %s" % prec)
    w = small_lognormal(1 << 14, 500, 10.0, 5, prec=prec)
    w["mass"] = w["mass"].copy()
    w["mass"][::13] = 0
    rng = np.random.default_rng(8)
    gF = rng.standard_normal(w["pos"].shape[0])
    tg = gpu_tree(w)
    dt = tg.dtype
    gr, gk, gl = tg.adjoint(0.75, 0.1, torch.as_tensor(gF, dtype=dt, device="cuda"))
    to = oracle_tree(w)
    if prec == "f32":
        gF = gF.astype(np.float32).astype(np.float64)
    orr, ok, ol = to.adjoint(0.75, 0.1, gF, nthreads=NTHREADS)
    tol = 1e-10 if prec == "f64" else 2e-6
    errs = {}
    for name, g, o in (("rho", gr, orr), ("kappa", gk, ok), ("lum", gl, ol)):
        g = g.cpu().numpy().astype(np.float64)
        scale = np.max(np.abs(o))
        err = np.abs(g - o) / (np.abs(o) + 1e-6 * scale)
        errs[name] = (float(err.max()), int(np.argmax(err)))
    _note("adjoint errors %s" % errs)
    assert all(e <= tol for e, _ in errs.values()), errs
    # Euler identity on the GPU's own outputs: sum L dF/dL = sum w F
    Fg = tg.flux(0.75, 0.1).double().cpu().numpy()
    lhs = float(np.dot(np.asarray(w["lum"], np.float64), gl.double().cpu().numpy()))
    assert math.isclose(lhs, float(np.dot(gF, Fg)), rel_tol=1e-9 if prec == "f64" else 1e-4)


def test_autograd_function_c5_recipe():
    _note("autograd on the c5 recipe at 2^15")
    w = W.c5(n=1 << 15)
    dev = "cuda"
    pos = torch.as_tensor(w["pos"], device=dev)
    mass = torch.as_tensor(w["mass"], device=dev)
    kappa = torch.as_tensor(w["kappa"], device=dev).requires_grad_(True)
    lum = torch.as_tensor(w["lum"], device=dev).requires_grad_(True)
    rho = torch.as_tensor(w["rho"], device=dev).requires_grad_(True)
    with torch.no_grad():
        target = P.flux(pos, torch.as_tensor(w["rho_target"], device=dev), kappa, lum, mass)
    F = P.flux(pos, rho, kappa, lum, mass)
    loss = ((F.double().log() - target.double().log()) ** 2).sum()
    loss.backward()
    # the oracle's adjoint for the same d loss / d F
    gF = (2.0 * (F.double().log() - target.double().log()) / F.double()).detach()
    gF32 = gF.float().cpu().numpy().astype(np.float64)
    orr, ok, ol = oracle_tree(w).adjoint(0.75, 0.1, gF32, nthreads=NTHREADS)
    for name, g, o in (("rho", rho.grad, orr), ("kappa", kappa.grad, ok), ("lum", lum.grad, ol)):
        g = g.cpu().numpy().astype(np.float64)
        scale = np.max(np.abs(o))
        err = np.abs(g - o) / (np.abs(o) + 1e-6 * scale)
        assert err.max() <= 2e-6, (name, err.max())


def test_out_of_range_sink_index_is_flagged():
    w = small_lognormal(3000, 100, 5.0, 31)
    tg = gpu_tree(w)
    sinks = torch.tensor([5, -1, 3000, 7, 1 << 30], dtype=torch.int32, device="cuda")
    F, C = tg.flux(0.75, 0.1, sinks=sinks, counters=True)
    F, C = F.cpu().numpy(), C.cpu().numpy()
    assert np.isnan(F[[1, 2, 4]]).all() and np.all(C[[1, 2, 4]] == -1)
    full = tg.flux(0.75, 0.1).cpu().numpy()
    assert F[0] == full[5] and F[3] == full[7]
    g = tg.adjoint(0.75, 0.1, torch.ones(5, dtype=tg.dtype, device="cuda"), sinks=sinks)
    assert all(torch.isfinite(x).all() for x in g)
