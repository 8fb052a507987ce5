"""GPU: the adjoint's modes and caller scratch through the C ABI, the counter
totals, the differentiable flux on a shared tree, and the ionisation step's
opacity-only form.

  * TREVR_ADJ_RECOMPUTE (each ray traced twice) and TREVR_ADJ_STORE (one tau
    per ray recorded), with the tree's scratch and with the caller's, give
    the oracle's gradients (binary64 1e-10, binary32 2e-6 of each entry with
    a floor of 1e-6 of the largest) and agree with each other;
  * trevr_adjoint_scratch_size gives 8 (5 m + n) bytes (256-aligned parts) for
    RECOMPUTE and more for STORE; a smaller scratch is refused; STORE in the
    caller's scratch leaves the tree's recording as it was;
  * both modes with caller scratch are captured in a HIP graph and replayed,
    with eager work in between, each replay equal to the eager gradients;
  * trevr_sum_counters equals the host sum (invalid sinks skipped);
  * two differentiable forwards on one tree before their backwards each get
    their own gradients (the tree is refit and re-recorded for the older);
  * the ionisation step with no flux writes kappa = sigma x only.
"""
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


def _workload(n, prec, seed=5):
    w = W._pack("lognormal%d" % n, *W.lognormal_box(n, n // 30, 10.0, seed), prec=prec)
    w["mass"] = w["mass"].copy()
    w["mass"][::13] = 0
    return w


def _trees(w):
    dt = torch.float64 if w["prec"] == "f64" else torch.float32
    d = lambda k: torch.as_tensor(w[k], dtype=dt, device="cuda")  # noqa: E731
    t = P.build_tree(d("pos"), d("rho"), d("kappa"), d("lum"), d("mass"), w["box_lo"],
                     w["box_hi"], w["bucket_size"])
    f = lambda a: np.asarray(a, np.float64)  # noqa: E731
    o = OracleTree(f(w["pos"]), f(w["rho"]), f(w["kappa"]), f(w["lum"]), f(w["mass"]),
                   w["box_lo"], w["box_hi"], w["bucket_size"], mirror32=(w["prec"] == "f32"))
    return t, o


def _rel(g, o):
    g = g.double().cpu().numpy()
    scale = np.max(np.abs(o))
    return float(np.max(np.abs(g - o) / (np.abs(o) + 1e-6 * scale)))


def _scratch(t, mode, ns=None):
    b = t.adjoint_scratch_size(mode, ns)
    return torch.empty(b, dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_modes_and_scratch_match_the_oracle(prec):
    _note("adjoint modes %s" % prec)
    w = _workload(1 << 13, prec)
    t, o = _trees(w)
    n = w["pos"].shape[0]
    gF = np.random.default_rng(3).standard_normal(n)
    if prec == "f32":
        gF = gF.astype(np.float32).astype(np.float64)
    go = o.adjoint(0.75, 0.1, gF, nthreads=NTHREADS)
    g = torch.as_tensor(gF, dtype=t.dtype, device="cuda")
    tol = 1e-10 if prec == "f64" else 2e-6
    results = {}
    for mode in (P.ADJ_RECOMPUTE, P.ADJ_STORE):
        for own in (True, False):
            got = t.adjoint(0.75, 0.1, g, mode=mode, scratch=None if own else _scratch(t, mode))
            errs = [_rel(a, b) for a, b in zip(got, go)]
            _note("mode %d own %s errors %s" % (mode, own, errs))
            assert max(errs) <= tol, (mode, own, errs)
            results[(mode, own)] = got
    ref = results[(P.ADJ_RECOMPUTE, True)]
    for key, got in results.items():  # device atomics: equal up to summation order
        for a, b in zip(got, ref):
            assert torch.allclose(a, b, rtol=1e-9 if prec == "f64" else 1e-5,
                                  atol=1e-9 * float(b.abs().max())), key


def test_scratch_sizes_and_a_short_scratch():
    w = _workload(3000, "f32", seed=7)
    t, _ = _trees(w)
    info = t.info()
    m, n = info["m"], info["n"]
    al = lambda v: (v + 255) // 256 * 256  # noqa: E731
    assert t.adjoint_scratch_size(P.ADJ_RECOMPUTE) == al(40 * m) + al(8 * n)
    assert t.adjoint_scratch_size(P.ADJ_AUTO) == 0
    st = t.adjoint_scratch_size(P.ADJ_STORE)
    assert st > t.adjoint_scratch_size(P.ADJ_RECOMPUTE)
    g = torch.ones(n, dtype=t.dtype, device="cuda")
    for mode in (P.ADJ_RECOMPUTE, P.ADJ_STORE):
        short = torch.empty(t.adjoint_scratch_size(P.ADJ_RECOMPUTE) - 256 if mode == 1
                            else t.adjoint_scratch_size(P.ADJ_RECOMPUTE) + 1024,
                            dtype=torch.uint8, device="cuda")
        with pytest.raises(P.TrevrError) as e:
            t.adjoint(0.75, 0.1, g, mode=mode, scratch=short)
        assert e.value.status == -6
    with pytest.raises(P.TrevrError) as e:  # AUTO takes no caller scratch
        t.adjoint(0.75, 0.1, g, mode=P.ADJ_AUTO, scratch=_scratch(t, P.ADJ_RECOMPUTE))
    assert e.value.status == -1


def test_store_in_caller_scratch_keeps_the_recording():
    _note("store mode in caller scratch keeps the tree's recording")
    w = _workload(1 << 12, "f32", seed=9)
    t, _ = _trees(w)
    n = w["pos"].shape[0]
    gA = torch.ones(n, dtype=t.dtype, device="cuda")
    gB = torch.linspace(-1.0, 2.0, n, dtype=t.dtype, device="cuda")
    F = t.flux(0.75, 0.1, tape=True)
    before = t.adjoint_taped(gA)
    # another adjoint (other weights) with its tape in the caller's scratch
    t.adjoint(0.75, -1.0, gB, mode=P.ADJ_STORE, scratch=_scratch(t, P.ADJ_STORE))
    after = t.adjoint_taped(gA)
    for a, b in zip(before, after):
        assert torch.allclose(a, b, rtol=1e-5, atol=1e-9 * float(a.abs().max()))
    assert torch.equal(t.flux(0.75, 0.1), F)


@pytest.mark.parametrize("mode", [1, 2])
def test_graph_captured_adjoint_replays(mode):
    _note("graph-captured adjoint, mode %d" % mode)
    w = _workload(1 << 13, "f32", seed=11)
    t, _ = _trees(w)
    n = w["pos"].shape[0]
    g = torch.as_tensor(np.random.default_rng(4).standard_normal(n), dtype=t.dtype, device="cuda")
    scratch = _scratch(t, mode)
    outs = [torch.empty(n, dtype=t.dtype, device="cuda") for _ in range(3)]
    eager = [x.clone() for x in t.adjoint(0.75, 0.1, g, mode=mode, scratch=scratch)]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on a side stream, as capture wants
        t.adjoint(0.75, 0.1, g, mode=mode, scratch=scratch, out=outs)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        t.adjoint(0.75, 0.1, g, mode=mode, scratch=scratch, out=outs)
    for rep in range(3):
        for x in outs:
            x.fill_(float("nan"))
        t.flux(0.75, 0.1)  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(outs, eager):
            assert torch.isfinite(a).all()
            assert torch.allclose(a, b, rtol=1e-5, atol=1e-9 * float(b.abs().max())), rep


def test_counter_totals():
    w = _workload(5000, "f32", seed=13)
    t, _ = _trees(w)
    sinks = torch.tensor([3, -1, 4999, 5000, 17, 17], dtype=torch.int32, device="cuda")
    _, C = t.flux(0.75, 0.1, sinks=sinks, counters=True)
    tot = P.sum_counters(C).cpu().numpy()
    c = C.cpu().numpy().astype(np.int64)
    assert np.array_equal(tot, c[c[:, 0] >= 0].sum(0))
    _, Call = t.flux(0.75, 0.1, counters=True)
    assert np.array_equal(P.sum_counters(Call).cpu().numpy(),
                          Call.cpu().numpy().astype(np.int64).sum(0))
    empty = P.sum_counters(torch.empty((0, 5), dtype=torch.int32, device="cuda"))
    assert np.array_equal(empty.cpu().numpy(), np.zeros(5))


def test_two_forwards_on_one_tree_before_backward():
    _note("two differentiable forwards on one tree")
    dt = torch.float64
    w = _workload(3000, "f64", seed=15)
    d = lambda a: torch.as_tensor(np.asarray(a), dtype=dt, device="cuda")  # noqa: E731
    pos, rho, kappa, lum, mass = d(w["pos"]), d(w["rho"]), d(w["kappa"]), d(w["lum"]), d(w["mass"])
    shared = P.Tree().build(pos, rho, kappa, lum, mass)

    def run(scale, tree):
        r = (rho * scale).requires_grad_(True)
        k = kappa.clone().requires_grad_(True)
        L = lum.clone().requires_grad_(True)
        F = P.flux(pos, r, k, L, mass, tree=tree)
        return F, (r, k, L)

    F1, v1 = run(1.3, shared)
    F2, v2 = run(0.6, shared)  # overwrites the shared tree's recording
    with torch.no_grad():  # and a plain flux in between
        shared.flux(0.75, 0.1)
    F1.log().sum().backward()
    F2.log().sum().backward()
    for F, v, scale in ((F1, v1, 1.3), (F2, v2, 0.6)):
        Fp, vp = run(scale, None)  # a private tree per forward
        Fp.log().sum().backward()
        assert torch.allclose(F, Fp, rtol=1e-13)
        for a, b in zip(v, vp):
            assert torch.allclose(a.grad, b.grad, rtol=1e-11, atol=1e-11 * float(b.grad.abs().max()))


def test_ionisation_opacity_only():
    x = torch.linspace(0.0, 1.0, 1001, dtype=torch.float64, device="cuda")
    kappa = torch.empty_like(x)
    x0 = x.clone()
    d = P.ionisation_update(None, x, kappa, 7.5, 1.0)
    assert torch.equal(x, x0) and torch.equal(kappa, 7.5 * x0) and float(d.item()) == 0.0
