"""GPU: trevr_refit_tree (new mass, rho, kappa and lum on the build's
positions) through the C ABI.

  * a refit tree equals a fresh build from the same arrays: the exported tree
    (order, topology, binary64 cell data) and the flux bit for bit, binary32
    and binary64, one box and several;
  * a moved position, an invalid value or another particle count is refused,
    and the tree keeps its previous properties;
  * a refit invalidates the tape of the recording flux.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_1902_08083_amd as P  # noqa: E402
from paper_1902_08083_amd import workloads as W  # noqa: E402
from paper_1902_08083_amd.trevr import _ptr, _stream  # noqa: E402


def _note(msg):
    print(msg, flush=True)


def _arrays(n, seed, dt):
    pos, rho, kappa, lum, mass = W.lognormal_box(n, n // 10, 6.0, seed)
    rng = np.random.default_rng(seed + 1000)
    mass = mass * rng.uniform(0.5, 1.5, n)
    mass[::17] = 0.0
    f = lambda a: torch.as_tensor(np.asarray(a), dtype=dt, device="cuda")  # noqa: E731
    return f(pos), f(rho), f(kappa), f(lum), f(mass)


def _same_tree(ta, tb):
    ea, eb = ta.export(), tb.export()
    for k in ea:
        a, b = np.asarray(ea[k]), np.asarray(eb[k])
        assert a.shape == b.shape and np.array_equal(a, b, equal_nan=True), k


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_refit_equals_fresh_build(dt):
    _note("refit against a fresh build, %s" % dt)
    pos, rho, kappa, lum, mass = _arrays(6000, 81, dt)
    _, rho2, kappa2, lum2, mass2 = _arrays(6000, 82, dt)
    t = P.Tree().build(pos, rho, kappa, lum, mass)
    t.refit(pos, rho2, kappa2, lum2, mass2)
    fresh = P.Tree().build(pos, rho2, kappa2, lum2, mass2)
    _same_tree(t, fresh)
    assert torch.equal(t.flux(0.75, 0.1), fresh.flux(0.75, 0.1))


def test_refit_forest_equals_fresh_build():
    _note("refit of a forest of three boxes")
    dt = torch.float64
    parts = [_arrays(n, 83 + k, dt) for k, n in enumerate((1500, 700, 2300))]
    cat = [torch.cat([p[i] for p in parts]) for i in range(5)]
    lo = [[0.0, 0.0, 0.0]] * 3
    hi = [[1.0, 1.0, 1.0]] * 3
    off = [0, 1500, 2200, 4500]
    t = P.Tree().build(cat[0], cat[1], cat[2], cat[3], cat[4], lo, hi, 8, off)
    g = torch.Generator(device="cuda").manual_seed(5)
    rho2 = cat[1] * (0.5 + torch.rand(4500, generator=g, device="cuda", dtype=dt))
    t.refit(cat[0], rho2, cat[2], cat[3], cat[4])
    fresh = P.Tree().build(cat[0], rho2, cat[2], cat[3], cat[4], lo, hi, 8, off)
    _same_tree(t, fresh)


def test_refit_refusals_keep_the_tree():
    _note("refit refusals")
    dt = torch.float64
    pos, rho, kappa, lum, mass = _arrays(3000, 91, dt)
    t = P.Tree().build(pos, rho, kappa, lum, mass)
    F0 = t.flux(0.75, 0.1)
    moved = pos.clone()
    moved[123, 1] = torch.nextafter(moved[123, 1], torch.tensor(1.0, dtype=dt, device="cuda"))
    with pytest.raises(P.TrevrError) as e:
        t.refit(moved, rho * 2, kappa, lum, mass)
    assert e.value.status == -1
    bad = kappa.clone()
    bad[7] = -1.0
    with pytest.raises(P.TrevrError) as e:
        t.refit(pos, rho, bad, lum, mass)
    assert e.value.status == -4
    with pytest.raises(P.TrevrError) as e:
        t.refit(pos[:2999], rho[:2999], kappa[:2999], lum[:2999], mass[:2999])
    assert e.value.status == -1
    assert torch.equal(t.flux(0.75, 0.1), F0)


def test_refit_invalidates_the_tape():
    _note("refit invalidates the tape")
    dt = torch.float32
    pos, rho, kappa, lum, mass = _arrays(2000, 92, dt)
    t = P.Tree().build(pos, rho, kappa, lum, mass)
    t.flux(0.75, 0.1, tape=True)
    t.refit(pos, rho * 1.5, kappa, lum, mass)
    out = [torch.empty(2000, dtype=dt, device="cuda") for _ in range(3)]
    gF = torch.ones(2000, dtype=dt, device="cuda")
    rc = P.lib().trevr_compute_flux_adjoint_taped(t._h, _ptr(gF), _ptr(out[0]), _ptr(out[1]),
                                                  _ptr(out[2]), _stream())
    assert rc == -5


def test_autograd_with_a_reused_tree():
    _note("autograd flux with a refit tree")
    dt = torch.float64
    pos, rho, kappa, lum, mass = _arrays(4000, 93, dt)
    t = P.Tree().build(pos, rho, kappa, lum, mass)
    grads = []
    for reuse in (False, True):
        r = (rho * 1.3).requires_grad_(True)
        k = kappa.clone().requires_grad_(True)
        L = lum.clone().requires_grad_(True)
        F = P.flux(pos, r, k, L, mass, tree=t if reuse else None)
        (F.log().sum()).backward()
        grads.append((F.detach(), r.grad, k.grad, L.grad))
    # gradients are sums of device atomics (order varies): compare to their scale
    for a, b in zip(*grads):
        assert torch.allclose(a, b, rtol=1e-12, atol=1e-12 * float(b.abs().max())), \
            "reused tree differs"


def test_autograd_two_forwards_on_one_tree_before_backward():
    """Forwards A and B share a tree, and a target flux under no_grad uses it
    too, all before either backward: each backward still returns its own
    forward's gradients (the tree's recording is B's, then the target's, so
    both backwards refit and record again)."""
    _note("autograd: two forwards and a no_grad flux on one tree before backward")
    dt = torch.float64
    pos, rho, kappa, lum, mass = _arrays(4000, 95, dt)
    t = P.Tree().build(pos, rho, kappa, lum, mass)
    vals = {"A": (rho * 1.3, kappa * 0.7, lum), "B": (rho * 0.6, kappa * 1.9, lum * 2.0)}
    leaves, outs = {}, {}
    for name, (r0, k0, l0) in vals.items():
        leaves[name] = [v.clone().requires_grad_(True) for v in (r0, k0, l0)]
        outs[name] = P.flux(pos, *leaves[name], mass, tree=t)
    with torch.no_grad():
        P.flux(pos, rho, kappa, lum, mass, tree=t)
    for name in ("A", "B"):
        (outs[name].log().sum()).backward()
        fresh = [v.clone().requires_grad_(True) for v in vals[name]]
        F = P.flux(pos, *fresh, mass)  # its own tree
        (F.log().sum()).backward()
        assert torch.allclose(outs[name].detach(), F.detach(), rtol=1e-13, atol=0.0), name
        for got, want in zip(leaves[name], fresh):
            g, w = got.grad, want.grad
            assert torch.allclose(g, w, rtol=1e-12, atol=1e-12 * float(w.abs().max())), name
