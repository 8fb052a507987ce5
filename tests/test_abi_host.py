"""The C ABI's argument checks, on the host only (no GPU needed).

Every entry point validates its host-side arguments before it touches a tree
or the device, so each bad argument below returns its status code and a
message without any HIP call: the particle set's sizes, boxes and offsets
(trevr_build_tree, trevr_refit_tree), the walk's theta_open, tau_ref and sink
count (trevr_compute_flux and the other walks), the walk variants' modes, the
adjoint's mode and scratch, launch shapes, the ionisation step's constants,
and the counter totals.
"""
import ctypes
import math
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1902_08083_amd", "libtrevr.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")

E_ARG, E_NONFINITE, E_CAPACITY = -1, -3, -6
P, D, I64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int64


@pytest.fixture(scope="module")
def L():
    from paper_1902_08083_amd import trevr
    return trevr.lib()


def _err(L):
    return L.trevr_last_error().decode()


def _particles(n=16, n_boxes=1, prec=0, bucket=8, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
               offsets=None, arrays=True):
    from paper_1902_08083_amd import trevr
    p = trevr._Particles()
    p.n = n
    p.prec = prec
    fake = ctypes.c_void_p(0x1000) if arrays else None  # never dereferenced on these paths
    p.x = p.y = p.z = p.rho = p.kappa = p.lum = fake
    p.mass = None
    p.n_boxes = n_boxes
    keep = []
    if offsets is not None:
        off = (ctypes.c_int64 * len(offsets))(*offsets)
        keep.append(off)
        p.box_offsets = ctypes.cast(off, ctypes.POINTER(ctypes.c_int64))
    if lo is not None:
        blo = (ctypes.c_double * len(lo))(*lo)
        bhi = (ctypes.c_double * len(hi))(*hi)
        keep += [blo, bhi]
        p.box_lo = ctypes.cast(blo, ctypes.POINTER(ctypes.c_double))
        p.box_hi = ctypes.cast(bhi, ctypes.POINTER(ctypes.c_double))
    p.bucket_size = bucket
    p._keep = keep
    return p


@pytest.mark.parametrize("kw,status,msg", [
    (dict(n=-1), E_ARG, "n < 0"),
    (dict(n=1 << 31), E_CAPACITY, "2^31"),
    (dict(prec=7), E_ARG, "precision"),
    (dict(n_boxes=0), E_ARG, "n_boxes"),
    (dict(bucket=0), E_ARG, "bucket_size"),
    (dict(lo=None), E_ARG, "box corners"),
    (dict(n_boxes=2, lo=(0.0,) * 6, hi=(1.0,) * 6), E_ARG, "box_offsets is NULL"),
    (dict(arrays=False), E_ARG, "particle array"),
    (dict(lo=(0.0, math.nan, 0.0)), E_NONFINITE, "non-finite"),
    (dict(hi=(1.0, 0.0, 1.0)), E_ARG, "hi <= lo"),
    (dict(n_boxes=2, lo=(0.0,) * 6, hi=(1.0,) * 6, offsets=(0, 4, 15)), E_ARG, "from 0 to n"),
    (dict(n_boxes=2, lo=(0.0,) * 6, hi=(1.0,) * 6, offsets=(1, 4, 16)), E_ARG, "from 0 to n"),
    (dict(n_boxes=3, lo=(0.0,) * 9, hi=(1.0,) * 9, offsets=(0, 9, 4, 16)), E_ARG,
     "must not decrease"),
])
def test_particle_set_checks(L, kw, status, msg):
    p = _particles(**kw)
    for fn in (L.trevr_build_tree, L.trevr_refit_tree):
        assert fn(None, ctypes.byref(p), None) == status
        assert msg in _err(L)
    # a NULL particle set is an argument error too
    assert L.trevr_build_tree(None, None, None) == E_ARG and "particles is NULL" in _err(L)


def test_valid_particles_then_the_tree(L):
    p = _particles(n=16, n_boxes=2, lo=(0.0,) * 6, hi=(1.0,) * 6, offsets=(0, 5, 16))
    assert L.trevr_build_tree(None, ctypes.byref(p), None) == E_ARG
    assert "tree is NULL" in _err(L)


@pytest.mark.parametrize("theta,tau_ref,ns,status,msg", [
    (-0.1, 0.1, 0, E_ARG, "theta_open"),
    (math.nan, 0.1, 0, E_ARG, "theta_open"),
    (math.inf, 0.1, 0, E_ARG, "theta_open"),
    (0.75, math.nan, 0, E_ARG, "tau_ref"),
    (0.75, 0.1, -1, E_ARG, "n_sinks < 0"),
    (0.75, 0.1, 1 << 31, E_CAPACITY, "too many sinks"),
    (0.75, -1.0, 0, E_ARG, "tree is NULL"),          # tau_ref < 0 and inf are valid
    (0.0, math.inf, 0, E_ARG, "tree is NULL"),
])
def test_walk_checks(L, theta, tau_ref, ns, status, msg):
    calls = [
        lambda: L.trevr_compute_flux(None, theta, tau_ref, None, ns, None, None, None),
        lambda: L.trevr_compute_flux_vector(None, theta, tau_ref, None, ns, None, None, None, None),
        lambda: L.trevr_compute_flux_moments(None, theta, tau_ref, None, ns, None, None, None,
                                             None, None),
        lambda: L.trevr_compute_flux_bands(None, theta, tau_ref, None, ns, None, None, None),
        lambda: L.trevr_compute_flux_sph(None, theta, tau_ref, None, ns, None, None, None),
        lambda: L.trevr_compute_flux_background(None, theta, tau_ref, None, ns, None, None, None),
        lambda: L.trevr_compute_flux_taped(None, theta, tau_ref, None, ns, None, None, None),
        lambda: L.trevr_compute_flux_variant(None, theta, tau_ref, 0, 0, math.inf, None, ns, None,
                                             None, None),
        lambda: L.trevr_compute_flux_adjoint(None, theta, tau_ref, None, ns, None, None, None,
                                             None, 1, None, 0, None),
    ]
    for c in calls:
        assert c() == status
        assert msg in _err(L)


@pytest.mark.parametrize("om,rm,tmax,msg", [
    (3, 0, math.inf, "open_mode"), (-1, 0, math.inf, "open_mode"), (0, 2, math.inf, "ray_mode"),
    (0, 0, 0.0, "tau_max"), (0, 0, -1.0, "tau_max"), (0, 0, math.nan, "tau_max"),
])
def test_variant_mode_checks(L, om, rm, tmax, msg):
    assert L.trevr_compute_flux_variant(None, 0.75, 0.1, om, rm, tmax, None, 0, None, None,
                                        None) == E_ARG
    assert msg in _err(L)


def test_adjoint_mode_and_scratch_checks(L):
    buf = ctypes.create_string_buffer(4096)
    base = ctypes.addressof(buf)
    aligned = base + (-base) % 8
    cases = [
        (dict(mode=3), "mode must be"),
        (dict(mode=-1), "mode must be"),
        (dict(mode=0, scratch=aligned), "takes no caller scratch"),
        (dict(mode=1, scratch=aligned + 4), "8-byte aligned"),
        (dict(mode=1, ns=4, grad=None), "grad_flux is NULL"),
        (dict(mode=2, scratch=aligned), "tree is NULL"),
    ]
    for kw, msg in cases:
        rc = L.trevr_compute_flux_adjoint(None, 0.75, 0.1, None, kw.get("ns", 0), kw.get("grad"),
                                          None, None, None, kw["mode"], kw.get("scratch"), 4000,
                                          None)
        assert rc == E_ARG and msg in _err(L), (kw, _err(L))
    sz = ctypes.c_size_t(0)
    assert L.trevr_adjoint_scratch_size(None, 1, 0, ctypes.byref(sz)) == E_ARG


@pytest.mark.parametrize("shape,msg", [
    ((0, 4, 64), "blocks_per_cu"), ((33, 4, 64), "blocks_per_cu"), ((4, 0, 64), "waves_per_block"),
    ((4, 17, 64), "waves_per_block"), ((4, 4, 32), "chunk"), ((4, 4, 96), "chunk"),
    ((4, 4, 8192), "chunk"), ((4, 4, 64), "NULL"),
])
def test_launch_shape_checks(L, shape, msg):
    from paper_1902_08083_amd import trevr
    c = trevr._Launch(*shape)
    for fn in (L.trevr_set_launch, L.trevr_set_adjoint_launch):
        assert fn(None, ctypes.byref(c)) == E_ARG
        assert msg in _err(L)


@pytest.mark.parametrize("n,prec,sigma,ab,damp,dxmax,msg", [
    (-1, 0, 1.0, 1.0, 0.5, True, "negative n"),
    (4, 0, 1.0, 1.0, 0.5, False, "NULL"),
    (4, 5, 1.0, 1.0, 0.5, True, "precision"),
    (4, 0, -1.0, 1.0, 0.5, True, "sigma"),
    (4, 0, math.inf, 1.0, 0.5, True, "sigma"),
    (4, 0, 1.0, 0.0, 0.5, True, "alpha_B"),
    (4, 0, 1.0, 1.0, 0.0, True, "damping"),
    (4, 0, 1.0, 1.0, 1.5, True, "damping"),
])
def test_ionisation_checks(L, n, prec, sigma, ab, damp, dxmax, msg):
    fake = ctypes.c_void_p(0x1000)
    d = ctypes.c_void_p(0x2000) if dxmax else None
    assert L.trevr_ionisation_update(n, prec, fake, None, sigma, ab, damp, fake, fake, d,
                                     None) == E_ARG
    assert msg in _err(L)


def test_other_null_checks(L):
    assert L.trevr_sum_counters(None, 4, ctypes.c_void_p(0x1000), None) == E_ARG
    assert L.trevr_sum_counters(None, -1, ctypes.c_void_p(0x1000), None) == E_ARG
    assert L.trevr_sum_counters(None, 0, None, None) == E_ARG
    assert L.trevr_reserve_tape(None, 4) == E_ARG
    assert L.trevr_export_tree(None, None, None, None, None, None, None) == E_ARG
    assert L.trevr_tree_info(None, None) == E_ARG
    assert L.trevr_tree_create(None) == E_ARG
    assert L.trevr_export_sph(None, None, None, None, None, None) == E_ARG
    assert L.trevr_compute_flux_adjoint_taped(None, None, None, None, None, None) == E_ARG
    for code in (0, -1, -2, -3, -4, -5, -6, -100, 17):
        assert L.trevr_status_string(code)


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is visible here")
def test_tree_create_without_a_device_reports_hip(L):
    h = ctypes.c_void_p()
    assert L.trevr_tree_create(ctypes.byref(h)) == -100
    assert "HIP error" in _err(L) and not h.value
