"""GPU: the recording flux and the taped adjoint, through the C ABI.

  * the recording flux returns exactly the plain flux (and counters);
  * the taped adjoint equals the two-pass adjoint (up to the order of the
    device atomics that sum the gradients), in binary32 and binary64, for
    all sinks and for a permuted subset;
  * a tape too small for the recording: the taped adjoint falls back to
    tracing twice with the same result; the next automatically sized
    recording is complete;
  * tape blocks taken eight at a time (a large tape) or one at a time give
    the same recording and gradients;
  * the taped adjoint without a recording, or after a rebuild, is refused
    with TREVR_E_STATE;
  * the taped adjoint against the oracle's adjoint.
"""
import ctypes
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1902_08083_amd as P  # noqa: E402
from paper_1902_08083_amd import workloads as W  # noqa: E402
from paper_1902_08083_amd.trevr import _ptr, _stream  # noqa: E402
from oracle.oracle import OracleTree  # noqa: E402

NTHREADS = min(16, os.cpu_count() or 1)


def _note(msg):
    print(msg, flush=True)


def _workload(n, n_src, tau_box, seed, prec):
    arrs = W.lognormal_box(n, n_src, tau_box, seed)
    return W._pack("lognormal%d" % n, *arrs, prec=prec)


def _tree(w):
    dt = torch.float64 if w["prec"] == "f64" else torch.float32
    f = lambda k: torch.as_tensor(w[k], dtype=dt, device="cuda")  # noqa: E731
    return P.build_tree(f("pos"), f("rho"), f("kappa"), f("lum"),
                        None if w.get("mass") is None else f("mass"),
                        w["box_lo"], w["box_hi"], w["bucket_size"])


def _grads_close(ga, gb, tol, what):
    for name, a, b in zip(("rho", "kappa", "lum"), ga, gb):
        a = a.double().cpu().numpy()
        b = b.double().cpu().numpy()
        scale = max(float(np.max(np.abs(b))), 1e-300)
        err = np.abs(a - b) / (np.abs(b) + 1e-6 * scale)
        assert err.max() <= tol, (what, name, float(err.max()))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_taped_flux_and_adjoint_match_untaped(prec):
    _note("taped flux and adjoint, all sinks, %s" % prec)
    w = _workload(1 << 14, 500, 10.0, 41, prec)
    tg = _tree(w)
    gF = torch.as_tensor(np.random.default_rng(42).standard_normal(w["pos"].shape[0]),
                         dtype=tg.dtype, device="cuda")
    F0, C0 = tg.flux(0.75, 0.1, counters=True)
    F1, C1 = tg.flux(0.75, 0.1, counters=True, tape=True)
    assert torch.equal(F0, F1) and torch.equal(C0, C1)
    g_two = tg.adjoint(0.75, 0.1, gF)
    g_tape = tg.adjoint_taped(gF)
    _grads_close(g_tape, g_two, 1e-12 if prec == "f64" else 2e-6, "taped vs two-pass")
    # a second adjoint from the same recording gives the same gradients
    _grads_close(tg.adjoint_taped(gF), g_tape, 1e-12 if prec == "f64" else 2e-6, "repeat")


def test_taped_adjoint_sink_subset_overflow_and_resize():
    _note("taped adjoint: sink subset, tape overflow fallback, automatic resize")
    w = _workload(6000, 300, 8.0, 43, "f64")
    tg = _tree(w)
    rng = np.random.default_rng(44)
    sinks = torch.as_tensor(rng.permutation(6000)[:1000].astype(np.int32), device="cuda")
    gF = torch.as_tensor(rng.standard_normal(1000), dtype=tg.dtype, device="cuda")
    g_two = tg.adjoint(0.75, 0.1, gF, sinks=sinks)
    tg.reserve_tape(1)  # far too small: the recording is incomplete
    F = tg.flux(0.75, 0.1, sinks=sinks, tape=True)
    assert torch.equal(F, tg.flux(0.75, 0.1, sinks=sinks))
    _grads_close(tg.adjoint_taped(gF), g_two, 1e-12, "overflowed tape")
    tg.reserve_tape(0)  # sized from the overflowed recording's count
    torch.cuda.synchronize()
    tg.flux(0.75, 0.1, sinks=sinks, tape=True)
    _grads_close(tg.adjoint_taped(gF), g_two, 1e-12, "resized tape")
    with pytest.raises(P.TrevrError):
        tg.reserve_tape(-1)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_tape_blocks_taken_in_chunks(prec):
    """A tape with room for eight leftover blocks per wave many times over
    makes each wave take its blocks eight at a time; the recording and the
    taped adjoint are the same as with one block per atomic."""
    _note("tape blocks eight at a time, %s" % prec)
    w = _workload(1 << 13, 400, 10.0, 47, prec)
    tg = _tree(w)
    tg.set_launch(1, 1, 64)  # 256 waves: chunks of 8 need >= 16 x 8 x 256 blocks
    n = w["pos"].shape[0]
    gF = torch.as_tensor(np.random.default_rng(48).standard_normal(n), dtype=tg.dtype,
                         device="cuda")
    tol = 1e-12 if prec == "f64" else 2e-6
    F0, C0 = tg.flux(0.75, 0.1, counters=True)
    g_two = tg.adjoint(0.75, 0.1, gF, mode=P.ADJ_RECOMPUTE)
    for blocks in (16 * 8 * 256 - 1, 16 * 8 * 256, 100000):  # one at a time, then chunks
        tg.reserve_tape(blocks)
        F1, C1 = tg.flux(0.75, 0.1, counters=True, tape=True)
        assert torch.equal(F0, F1) and torch.equal(C0, C1), blocks
        _grads_close(tg.adjoint_taped(gF), g_two, tol, "tape of %d blocks" % blocks)


def test_taped_adjoint_refused_without_recording():
    _note("taped adjoint without a recording, and after a rebuild")
    w = _workload(2000, 50, 4.0, 45, "f32")
    tg = _tree(w)
    out = [torch.empty(tg.n, dtype=tg.dtype, device="cuda") for _ in range(3)]
    gF = torch.ones(2000, dtype=tg.dtype, device="cuda")
    L = P.lib()

    def call():
        return L.trevr_compute_flux_adjoint_taped(tg._h, _ptr(gF), _ptr(out[0]), _ptr(out[1]),
                                                  _ptr(out[2]), _stream())
    assert call() == -5
    tg.flux(0.75, 0.1, tape=True)
    assert call() == 0
    torch.cuda.synchronize()
    f = lambda k: torch.as_tensor(w[k], dtype=tg.dtype, device="cuda")  # noqa: E731
    tg.build(f("pos"), f("rho"), f("kappa"), f("lum"), f("mass"), w["box_lo"], w["box_hi"],
             w["bucket_size"])
    assert call() == -5


def test_taped_adjoint_matches_oracle():
    _note("taped adjoint against the oracle, f64")
    w = _workload(1 << 13, 300, 10.0, 46, "f64")
    w["mass"] = w["mass"].copy()
    w["mass"][::11] = 0
    gF = np.random.default_rng(47).standard_normal(w["pos"].shape[0])
    tg = _tree(w)
    tg.flux(0.75, 0.1, tape=True)
    g = tg.adjoint_taped(torch.as_tensor(gF, dtype=tg.dtype, device="cuda"))
    f = lambda a: None if a is None else np.asarray(a, np.float64)  # noqa: E731
    to = OracleTree(f(w["pos"]), f(w["rho"]), f(w["kappa"]), f(w["lum"]), f(w["mass"]),
                    w["box_lo"], w["box_hi"], w["bucket_size"], mirror32=False)
    o = to.adjoint(0.75, 0.1, gF, nthreads=NTHREADS)
    _grads_close(g, [torch.as_tensor(x) for x in o], 1e-10, "taped vs oracle")
