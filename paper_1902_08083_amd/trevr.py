"""Python binding of ``libtrevr.so`` (ctypes).

Argument marshalling only: every step of the radiation-field path runs in the
library's HIP kernels; torch provides device memory and the current stream.
The names follow the C ABI in ``include/trevr.h``:

    tree = build_tree(pos, rho, kappa, lum, mass=None, ...)
    F = compute_flux(tree, theta_open, tau_ref, sinks=None)
    g_rho, g_kappa, g_lum = compute_flux_adjoint(tree, theta_open, tau_ref, grad_flux)

If the library has not been built the import of this module succeeds but
every call raises ``TrevrNotBuilt``; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtrevr.so")

TREVR_F32, TREVR_F64 = 0, 1
COUNTER_FIELDS = ("n_open", "n_rays", "n_psrc", "n_seg", "n_trace")


class TrevrNotBuilt(RuntimeError):
    pass


class TrevrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("trevr status %d: %s" % (status, msg))
        self.status = status


class _Particles(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("prec", ctypes.c_int),
        ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
        ("mass", ctypes.c_void_p), ("rho", ctypes.c_void_p), ("kappa", ctypes.c_void_p),
        ("lum", ctypes.c_void_p), ("n_boxes", ctypes.c_int32),
        ("box_offsets", ctypes.POINTER(ctypes.c_int64)),
        ("box_lo", ctypes.POINTER(ctypes.c_double)), ("box_hi", ctypes.POINTER(ctypes.c_double)),
        ("bucket_size", ctypes.c_int32),
    ]


class _Launch(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("chunk", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("n_boxes", ctypes.c_int32),
                ("max_depth", ctypes.c_int32), ("prec", ctypes.c_int),
                ("bucket_size", ctypes.c_int32)]


_lib = None

EXPORTED = (
    "trevr_status_string", "trevr_last_error", "trevr_tree_create", "trevr_tree_destroy",
    "trevr_build_tree", "trevr_tree_info", "trevr_compute_flux", "trevr_compute_flux_adjoint",
    "trevr_set_launch", "trevr_get_launch", "trevr_set_adjoint_launch",
    "trevr_get_adjoint_launch", "trevr_export_tree", "trevr_compute_flux_taped",
    "trevr_compute_flux_adjoint_taped", "trevr_reserve_tape", "trevr_compute_flux_vector",
    "trevr_refit_tree", "trevr_compute_flux_moments", "trevr_set_bands",
    "trevr_compute_flux_bands", "trevr_set_sph", "trevr_compute_flux_sph", "trevr_export_sph",
    "trevr_compute_flux_variant", "trevr_set_background", "trevr_compute_flux_background",
    "trevr_ionisation_update", "trevr_adjoint_scratch_size", "trevr_sum_counters",
    "trevr_compute_flux_adjoint_noalloc",
)

ADJ_AUTO, ADJ_RECOMPUTE, ADJ_STORE = 0, 1, 2


def lib():
    """Load the library (raises TrevrNotBuilt if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise TrevrNotBuilt("%s is missing: build it with `python -m paper_1902_08083_amd.build`"
                            % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    L.trevr_status_string.restype = ctypes.c_char_p
    L.trevr_status_string.argtypes = [I]
    L.trevr_last_error.restype = ctypes.c_char_p
    L.trevr_last_error.argtypes = []
    L.trevr_tree_create.restype = I
    L.trevr_tree_create.argtypes = [ctypes.POINTER(P)]
    L.trevr_tree_destroy.restype = None
    L.trevr_tree_destroy.argtypes = [P]
    L.trevr_build_tree.restype = I
    L.trevr_build_tree.argtypes = [P, ctypes.POINTER(_Particles), P]
    L.trevr_tree_info.restype = I
    L.trevr_tree_info.argtypes = [P, ctypes.POINTER(_Info)]
    L.trevr_compute_flux.restype = I
    L.trevr_compute_flux.argtypes = [P, D, D, P, I64, P, P, P]
    L.trevr_compute_flux_adjoint.restype = I
    L.trevr_compute_flux_adjoint.argtypes = [P, D, D, P, I64, P, P, P, P, ctypes.c_int32, P,
                                             ctypes.c_size_t, P]
    L.trevr_adjoint_scratch_size.restype = I
    L.trevr_adjoint_scratch_size.argtypes = [P, ctypes.c_int32, I64, ctypes.POINTER(ctypes.c_size_t)]
    L.trevr_sum_counters.restype = I
    L.trevr_sum_counters.argtypes = [P, I64, P, P]
    L.trevr_compute_flux_adjoint_noalloc.restype = I
    L.trevr_compute_flux_adjoint_noalloc.argtypes = [P, D, D, P, I64, P, P, P, P, P]
    L.trevr_compute_flux_taped.restype = I
    L.trevr_compute_flux_taped.argtypes = [P, D, D, P, I64, P, P, P]
    L.trevr_compute_flux_adjoint_taped.restype = I
    L.trevr_compute_flux_adjoint_taped.argtypes = [P, P, P, P, P, P]
    L.trevr_refit_tree.restype = I
    L.trevr_refit_tree.argtypes = [P, ctypes.POINTER(_Particles), P]
    L.trevr_set_bands.restype = I
    L.trevr_set_bands.argtypes = [P, ctypes.c_int32, P, P]
    L.trevr_compute_flux_bands.restype = I
    L.trevr_compute_flux_bands.argtypes = [P, D, D, P, I64, P, P, P]
    L.trevr_compute_flux_variant.restype = I
    L.trevr_compute_flux_variant.argtypes = [P, D, D, ctypes.c_int32, ctypes.c_int32, D, P, I64,
                                             P, P, P]
    L.trevr_ionisation_update.restype = I
    L.trevr_ionisation_update.argtypes = [I64, ctypes.c_int, P, P, D, D, D, P, P, P, P]
    L.trevr_set_background.restype = I
    L.trevr_set_background.argtypes = [P, P, D, P, P]
    L.trevr_compute_flux_background.restype = I
    L.trevr_compute_flux_background.argtypes = [P, D, D, P, I64, P, P, P]
    L.trevr_set_sph.restype = I
    L.trevr_set_sph.argtypes = [P, P, P]
    L.trevr_compute_flux_sph.restype = I
    L.trevr_compute_flux_sph.argtypes = [P, D, D, P, I64, P, P, P]
    L.trevr_export_sph.restype = I
    L.trevr_export_sph.argtypes = [P, P, P, P, P, P]
    L.trevr_compute_flux_moments.restype = I
    L.trevr_compute_flux_moments.argtypes = [P, D, D, P, I64, P, P, P, P, P]
    L.trevr_compute_flux_vector.restype = I
    L.trevr_compute_flux_vector.argtypes = [P, D, D, P, I64, P, P, P, P]
    L.trevr_reserve_tape.restype = I
    L.trevr_reserve_tape.argtypes = [P, I64]
    L.trevr_set_launch.restype = I
    L.trevr_set_launch.argtypes = [P, ctypes.POINTER(_Launch)]
    L.trevr_get_launch.restype = I
    L.trevr_get_launch.argtypes = [P, ctypes.POINTER(_Launch)]
    L.trevr_set_adjoint_launch.restype = I
    L.trevr_set_adjoint_launch.argtypes = [P, ctypes.POINTER(_Launch)]
    L.trevr_get_adjoint_launch.restype = I
    L.trevr_get_adjoint_launch.argtypes = [P, ctypes.POINTER(_Launch)]
    L.trevr_export_tree.restype = I
    L.trevr_export_tree.argtypes = [P, P, P, P, P, P, P]
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        msg = lib().trevr_last_error().decode(errors="replace")
        raise TrevrError(rc, msg)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_array(a, dtype, device):
    t = torch.as_tensor(a, device=device)
    if t.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, t.dtype))
    return t.contiguous()


class Tree:
    """A radiation tree (one or more boxes) held on the GPU."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().trevr_tree_create(ctypes.byref(h)))
        self._h = h
        self.n = 0
        # bumped by every call that changes the cell properties or the tape
        # (build, refit, a recording flux, an adjoint on the tree's tape)
        self.generation = 0
        self.prec = None
        self.dtype = None
        self.device = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.trevr_tree_destroy(h)
            self._h = None

    # -- build -----------------------------------------------------------
    def build(self, pos, rho, kappa, lum, mass=None, box_lo=(0.0, 0.0, 0.0),
              box_hi=(1.0, 1.0, 1.0), bucket_size=8, box_offsets=None, device="cuda"):
        """pos: (n, 3) tensor; rho, kappa, lum, mass: (n,) of the same float dtype
        (float32 -> binary32 transport, float64 -> binary64).  box_lo/box_hi:
        one corner triple, or (n_boxes, 3) with box_offsets (n_boxes + 1)."""
        p, keep = self._particles(pos, rho, kappa, lum, mass, box_lo, box_hi, bucket_size,
                                  box_offsets, device)
        _check(lib().trevr_build_tree(self._h, ctypes.byref(p), _stream()))
        self.generation += 1
        self._layout = (box_lo, box_hi, bucket_size, box_offsets)
        self._n_bands = 0  # a build drops the bands
        self.n = p.n
        self.dtype = keep[0].dtype
        self.prec = p.prec
        self.device = keep[0].device
        self.n_boxes = p.n_boxes
        return self

    def refit(self, pos, rho, kappa, lum, mass=None):
        """New rho, kappa, lum (and mass) on the positions the tree was built
        from: the cell properties are recomputed, the topology kept."""
        box_lo, box_hi, bucket_size, box_offsets = self._layout
        p, keep = self._particles(pos, rho, kappa, lum, mass, box_lo, box_hi, bucket_size,
                                  box_offsets, self.device)
        _check(lib().trevr_refit_tree(self._h, ctypes.byref(p), _stream()))
        self.generation += 1
        self._n_bands = 0  # so does a refit
        return self

    @staticmethod
    def _particles(pos, rho, kappa, lum, mass, box_lo, box_hi, bucket_size, box_offsets,
                   device):
        pos = torch.as_tensor(pos, device=device)
        dtype = pos.dtype
        if dtype not in (torch.float32, torch.float64):
            raise TypeError("positions must be float32 or float64")
        n = int(pos.shape[0])
        keep = [pos[:, 0].contiguous(), pos[:, 1].contiguous(), pos[:, 2].contiguous(),
                None if mass is None else _dev_array(mass, dtype, pos.device),
                _dev_array(rho, dtype, pos.device), _dev_array(kappa, dtype, pos.device),
                _dev_array(lum, dtype, pos.device)]
        lo = torch.as_tensor(box_lo, dtype=torch.float64).reshape(-1, 3).contiguous()
        hi = torch.as_tensor(box_hi, dtype=torch.float64).reshape(-1, 3).contiguous()
        nbox = int(lo.shape[0])
        if box_offsets is None:
            if nbox != 1:
                raise ValueError("box_offsets are needed for several boxes")
            off = None
        else:
            off = torch.as_tensor(box_offsets, dtype=torch.int64).contiguous()
        p = _Particles()
        p.n = n
        p.prec = TREVR_F64 if dtype == torch.float64 else TREVR_F32
        p.x, p.y, p.z, p.mass, p.rho, p.kappa, p.lum = [
            None if t is None else t.data_ptr() for t in keep]
        p.n_boxes = nbox
        p.box_offsets = (None if off is None else
                         ctypes.cast(off.data_ptr(), ctypes.POINTER(ctypes.c_int64)))
        p.box_lo = ctypes.cast(lo.data_ptr(), ctypes.POINTER(ctypes.c_double))
        p.box_hi = ctypes.cast(hi.data_ptr(), ctypes.POINTER(ctypes.c_double))
        p.bucket_size = int(bucket_size)
        p._keep = (keep, lo, hi, off)  # alive until the call returns
        return p, keep

    def info(self):
        i = _Info()
        _check(lib().trevr_tree_info(self._h, ctypes.byref(i)))
        return {"n": i.n, "m": i.m, "n_boxes": i.n_boxes, "max_depth": i.max_depth,
                "prec": i.prec, "bucket_size": i.bucket_size}

    def set_launch(self, blocks_per_cu=4, waves_per_block=4, chunk=64, adjoint=False):
        """Launch shape of later flux calls, or of adjoint calls if `adjoint`."""
        c = _Launch(int(blocks_per_cu), int(waves_per_block), int(chunk))
        fn = lib().trevr_set_adjoint_launch if adjoint else lib().trevr_set_launch
        _check(fn(self._h, ctypes.byref(c)))

    def get_launch(self, adjoint=False):
        c = _Launch()
        fn = lib().trevr_get_adjoint_launch if adjoint else lib().trevr_get_launch
        _check(fn(self._h, ctypes.byref(c)))
        return {"blocks_per_cu": c.blocks_per_cu, "waves_per_block": c.waves_per_block,
                "chunk": c.chunk}

    # -- walks -----------------------------------------------------------
    def _sinks(self, sinks):
        if sinks is None:
            return None, self.n
        s = torch.as_tensor(sinks, device=self.device).to(torch.int32).contiguous()
        return s, int(s.shape[0])

    def flux(self, theta_open, tau_ref, sinks=None, counters=False, out=None, tape=False):
        """Flux at the sinks.  With `tape`, each ray's optical depth is also
        recorded for a later adjoint_taped call."""
        s, ns = self._sinks(sinks)
        F = out if out is not None else torch.empty(ns, dtype=self.dtype, device=self.device)
        C = torch.empty((ns, 5), dtype=torch.int32, device=self.device) if counters else None
        fn = lib().trevr_compute_flux_taped if tape else lib().trevr_compute_flux
        _check(fn(self._h, float(theta_open), float(tau_ref), _ptr(s), ns, _ptr(F), _ptr(C),
                  _stream()))
        if tape:
            self.generation += 1
            self._tape_sinks = s  # the recording reads it again in adjoint_taped
            self._tape_ns = ns
        return (F, C) if counters else F

    def flux_vector(self, theta_open, tau_ref, sinks=None, counters=False):
        """(F, Fv): the flux and the vector flux (n_sinks x 3; each ray's flux
        along its direction of travel at the sink)."""
        s, ns = self._sinks(sinks)
        F = torch.empty(ns, dtype=self.dtype, device=self.device)
        Fv = torch.empty((3, ns), dtype=self.dtype, device=self.device)
        C = torch.empty((ns, 5), dtype=torch.int32, device=self.device) if counters else None
        _check(lib().trevr_compute_flux_vector(self._h, float(theta_open), float(tau_ref),
                                               _ptr(s), ns, _ptr(F), _ptr(Fv), _ptr(C),
                                               _stream()))
        return (F, Fv.t(), C) if counters else (F, Fv.t())

    def flux_moments(self, theta_open, tau_ref, sinks=None, counters=False):
        """(F, Fv, Pm): flux, vector flux (n_sinks x 3) and the second moment
        sum f n_a n_b (n_sinks x 6: xx, yy, zz, xy, xz, yz)."""
        s, ns = self._sinks(sinks)
        F = torch.empty(ns, dtype=self.dtype, device=self.device)
        Fv = torch.empty((3, ns), dtype=self.dtype, device=self.device)
        Pm = torch.empty((6, ns), dtype=self.dtype, device=self.device)
        C = torch.empty((ns, 5), dtype=torch.int32, device=self.device) if counters else None
        _check(lib().trevr_compute_flux_moments(self._h, float(theta_open), float(tau_ref),
                                                _ptr(s), ns, _ptr(F), _ptr(Fv), _ptr(Pm),
                                                _ptr(C), _stream()))
        out = (F, Fv.t(), Pm.t())
        return out + (C,) if counters else out

    def set_bands(self, kappa_bands):
        """Opacity bands: kappa_bands (k, n), 1 <= k <= 4, in input order."""
        kb = torch.as_tensor(kappa_bands, dtype=self.dtype, device=self.device).contiguous()
        if kb.dim() != 2 or kb.shape[1] != self.n:
            raise ValueError("kappa_bands must be (k, n)")
        _check(lib().trevr_set_bands(self._h, int(kb.shape[0]), _ptr(kb), _stream()))
        self._n_bands = int(kb.shape[0])

    def flux_bands(self, theta_open, tau_ref, sinks=None, counters=False):
        """Flux per band (n_sinks x k) on one traversal (see set_bands)."""
        s, ns = self._sinks(sinks)
        k = getattr(self, "_n_bands", 0)
        Fb = torch.empty((max(k, 1), ns), dtype=self.dtype, device=self.device)
        C = torch.empty((ns, 5), dtype=torch.int32, device=self.device) if counters else None
        _check(lib().trevr_compute_flux_bands(self._h, float(theta_open), float(tau_ref),
                                              _ptr(s), ns, _ptr(Fb), _ptr(C), _stream()))
        return (Fb.t(), C) if counters else Fb.t()

    def flux_variant(self, theta_open, tau_ref, open_mode=0, ray_mode=0,
                     tau_max=float("inf"), sinks=None, counters=False, out=None):
        """Flux with a walk variant: open_mode 0 (sink point), 1 (the sink's
        bucket box), 2 (Gasoline's opening radius); ray_mode 0 (up the tree),
        1 (top down from the meeting cell); rays past tau_max contribute nothing."""
        s, ns = self._sinks(sinks)
        F = out if out is not None else torch.empty(ns, dtype=self.dtype, device=self.device)
        C = torch.empty((ns, 5), dtype=torch.int32, device=self.device) if counters else None
        _check(lib().trevr_compute_flux_variant(self._h, float(theta_open), float(tau_ref),
                                                int(open_mode), int(ray_mode), float(tau_max),
                                                _ptr(s), ns, _ptr(F), _ptr(C), _stream()))
        return (F, C) if counters else F

    def set_background(self, centre, radius, flags):
        """Background sources (flags (n,), non-zero = background) on the sphere
        (centre, radius): merged cells of them radiate from the sphere."""
        c = (ctypes.c_double * 3)(*[float(v) for v in centre])
        f = torch.as_tensor(flags, device=self.device).to(torch.uint8).contiguous()
        if f.shape != (self.n,):
            raise ValueError("flags must have one entry per particle")
        _check(lib().trevr_set_background(self._h, c, float(radius), _ptr(f), _stream()))

    def flux_background(self, theta_open, tau_ref, sinks=None, counters=False, out=None):
        """Flux with merged background sources on the shell's sphere."""
        s, ns = self._sinks(sinks)
        F = out if out is not None else torch.empty(ns, dtype=self.dtype, device=self.device)
        C = torch.empty((ns, 5), dtype=torch.int32, device=self.device) if counters else None
        _check(lib().trevr_compute_flux_background(self._h, float(theta_open), float(tau_ref),
                                                   _ptr(s), ns, _ptr(F), _ptr(C), _stream()))
        return (F, C) if counters else F

    def set_sph(self, h):
        """Smoothing lengths h (n,), input order, for the particle trace below
        the buckets (see flux_sph)."""
        hv = torch.as_tensor(h, dtype=self.dtype, device=self.device).contiguous()
        if hv.shape != (self.n,):
            raise ValueError("h must have one entry per particle")
        _check(lib().trevr_set_sph(self._h, _ptr(hv), _stream()))

    def flux_sph(self, theta_open, tau_ref, sinks=None, counters=False, out=None):
        """Flux with the SPH-style particle trace below the buckets."""
        s, ns = self._sinks(sinks)
        F = out if out is not None else torch.empty(ns, dtype=self.dtype, device=self.device)
        C = torch.empty((ns, 5), dtype=torch.int32, device=self.device) if counters else None
        _check(lib().trevr_compute_flux_sph(self._h, float(theta_open), float(tau_ref), _ptr(s),
                                            ns, _ptr(F), _ptr(C), _stream()))
        return (F, C) if counters else F

    def export_sph(self):
        """The absorber lists: (offsets[m + 1], neighbours (input indices), spread[m])."""
        import numpy as np
        m = self.info()["m"]
        ne = ctypes.c_int64(0)
        _check(lib().trevr_export_sph(self._h, ctypes.byref(ne), None, None, None, _stream()))
        off = np.empty(m + 1, np.int64)
        nb = np.empty(max(ne.value, 1), np.int64)
        sp = np.empty(max(m, 1), np.float64)
        _check(lib().trevr_export_sph(self._h, ctypes.byref(ne), off.ctypes.data_as(ctypes.c_void_p),
                                      nb.ctypes.data_as(ctypes.c_void_p),
                                      sp.ctypes.data_as(ctypes.c_void_p), _stream()))
        return off, nb[:ne.value], sp[:m]

    def adjoint_taped(self, grad_flux):
        """The adjoint for the arguments of the last flux(..., tape=True)."""
        ns = getattr(self, "_tape_ns", None)
        if ns is None:
            raise TrevrError(-5, "no recording flux call on this tree")
        g = grad_flux.to(device=self.device, dtype=self.dtype).contiguous()
        if g.shape[0] != ns:
            raise ValueError("grad_flux has %d entries, expected %d" % (g.shape[0], ns))
        outs = [torch.empty(self.n, dtype=self.dtype, device=self.device) for _ in range(3)]
        _check(lib().trevr_compute_flux_adjoint_taped(self._h, _ptr(g), _ptr(outs[0]),
                                                      _ptr(outs[1]), _ptr(outs[2]), _stream()))
        return tuple(outs)

    def reserve_tape(self, blocks):
        """Tape capacity of later recordings in blocks of 64 rays (0: automatic)."""
        _check(lib().trevr_reserve_tape(self._h, int(blocks)))

    def adjoint_scratch_size(self, mode, n_sinks=None):
        """Bytes of caller scratch the adjoint needs in `mode` (ADJ_RECOMPUTE or
        ADJ_STORE) for n_sinks sinks (default: every particle)."""
        b = ctypes.c_size_t(0)
        ns = self.n if n_sinks is None else int(n_sinks)
        _check(lib().trevr_adjoint_scratch_size(self._h, int(mode), ns, ctypes.byref(b)))
        return int(b.value)

    def adjoint(self, theta_open, tau_ref, grad_flux, sinks=None, mode=ADJ_AUTO, scratch=None,
                out=None):
        """Gradients (rho, kappa, lum) of sum_k grad_flux[k] F_k.  mode: ADJ_AUTO,
        ADJ_RECOMPUTE (each ray traced twice) or ADJ_STORE (one tau per ray
        recorded); scratch: a device tensor of at least adjoint_scratch_size
        bytes (then nothing is allocated and the call can be graph-captured)."""
        s, ns = self._sinks(sinks)
        g = grad_flux.to(device=self.device, dtype=self.dtype).contiguous()
        if g.shape[0] != ns:
            raise ValueError("grad_flux has %d entries, expected %d" % (g.shape[0], ns))
        outs = out if out is not None else [
            torch.empty(self.n, dtype=self.dtype, device=self.device) for _ in range(3)]
        nbytes = 0 if scratch is None else scratch.numel() * scratch.element_size()
        _check(lib().trevr_compute_flux_adjoint(self._h, float(theta_open), float(tau_ref),
                                                _ptr(s), ns, _ptr(g), _ptr(outs[0]),
                                                _ptr(outs[1]), _ptr(outs[2]), int(mode),
                                                _ptr(scratch), nbytes, _stream()))
        if scratch is None and mode != ADJ_RECOMPUTE:
            self.generation += 1  # the tree's tape served as scratch
        return tuple(outs)

    def export(self):
        """Host copy of the tree, in the oracle's field layout (numpy)."""
        import numpy as np
        info = self.info()
        n, m = info["n"], info["m"]
        perm = np.empty(n, np.int64)
        leaf_of = np.empty(n, np.int64)
        node_i = np.empty((m, 8), np.int64)
        node_key = np.empty(m, np.uint64)
        node_f = np.empty((m, 22), np.float64)
        c = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(lib().trevr_export_tree(self._h, c(perm), c(leaf_of), c(node_i), c(node_key),
                                       c(node_f), _stream()))
        from . import NODE_F_FIELDS, NODE_I_FIELDS
        out = {"perm": perm, "leaf_of": leaf_of, "key": node_key}
        for j, f in enumerate(NODE_I_FIELDS):
            out[f] = node_i[:, j].copy()
        for j, f in enumerate(NODE_F_FIELDS):
            out[f] = node_f[:, j].copy()
        return out


def build_tree(pos, rho, kappa, lum, mass=None, box_lo=(0.0, 0.0, 0.0), box_hi=(1.0, 1.0, 1.0),
               bucket_size=8, box_offsets=None, device="cuda", tree=None):
    t = tree if tree is not None else Tree()
    return t.build(pos, rho, kappa, lum, mass, box_lo, box_hi, bucket_size, box_offsets, device)


def compute_flux(tree, theta_open, tau_ref, sinks=None, counters=False, out=None):
    return tree.flux(theta_open, tau_ref, sinks, counters, out)


def compute_flux_adjoint(tree, theta_open, tau_ref, grad_flux, sinks=None, mode=ADJ_AUTO,
                         scratch=None):
    return tree.adjoint(theta_open, tau_ref, grad_flux, sinks, mode, scratch)


def sum_counters(counters):
    """Totals over the sinks of per-sink counters ([n_sinks, 5] int32, as the
    flux calls return them): a device int64 tensor of 5 (n_open, n_rays,
    n_psrc, n_seg, n_trace), invalid sinks skipped."""
    c = counters.contiguous()
    if c.dtype != torch.int32 or c.dim() != 2 or c.shape[1] != 5:
        raise ValueError("counters must be int32 [n_sinks, 5]")
    tot = torch.empty(5, dtype=torch.int64, device=c.device)
    _check(lib().trevr_sum_counters(_ptr(c), int(c.shape[0]), _ptr(tot), _stream()))
    return tot


class TrevrFlux(torch.autograd.Function):
    """F = flux(rho, kappa, lum) at fixed positions; backward runs the adjoint
    kernel over the same traversal (decisions held fixed), with each ray's
    optical depth taken from the forward's recording.  A shared tree may be
    refit, recorded or used by other calls between this forward and its
    backward: backward then refits it with this forward's values and records
    again before the adjoint (the tree holds them afterwards)."""

    @staticmethod
    def forward(ctx, rho, kappa, lum, pos, mass, theta_open, tau_ref, bucket_size, sinks,
                tree=None):
        vals = (rho.detach(), kappa.detach(), lum.detach())
        if tree is None:
            tree = build_tree(pos, *vals, mass, bucket_size=bucket_size, device=pos.device)
        else:  # a tree built earlier on these positions: new cell properties only
            tree.refit(pos, *vals, mass)
        F = tree.flux(theta_open, tau_ref, sinks, tape=True)
        ctx.tree = tree
        ctx.generation = tree.generation
        ctx.args = (pos, mass, theta_open, tau_ref, sinks) + vals
        return F

    @staticmethod
    def backward(ctx, gF):
        tree = ctx.tree
        if tree.generation != ctx.generation:  # the recording is not this forward's
            pos, mass, theta_open, tau_ref, sinks, rho, kappa, lum = ctx.args
            tree.refit(pos, rho, kappa, lum, mass)
            tree.flux(theta_open, tau_ref, sinks, tape=True)
        g_rho, g_kappa, g_lum = tree.adjoint_taped(gF.contiguous())
        ctx.tree = None
        ctx.args = None
        return g_rho, g_kappa, g_lum, None, None, None, None, None, None, None


def flux(pos, rho, kappa, lum, mass=None, theta_open=0.75, tau_ref=0.1, bucket_size=8,
         sinks=None, tree=None):
    """Differentiable flux at the sinks with respect to rho, kappa and lum.  With
    `tree` (a Tree built on the same positions and boxes), the tree is refit
    with the new values instead of built anew; it then holds them afterwards."""
    return TrevrFlux.apply(rho, kappa, lum, pos, mass, theta_open, tau_ref, bucket_size, sinks,
                           tree)


# ---------------------------------------------------------------- batching ---

def _concat_boxes(boxes, device):
    """boxes: list of dicts with pos (n,3), rho, kappa, lum, mass (optional),
    box_lo, box_hi.  Returns device tensors and host box tables."""
    import numpy as np
    pos = np.concatenate([np.asarray(b["pos"]) for b in boxes])
    cat = lambda k: np.concatenate([np.asarray(b[k]) for b in boxes])  # noqa: E731
    off = np.cumsum([0] + [int(np.asarray(b["pos"]).shape[0]) for b in boxes]).astype(np.int64)
    lo = np.array([b.get("box_lo", (0.0, 0.0, 0.0)) for b in boxes], np.float64)
    hi = np.array([b.get("box_hi", (1.0, 1.0, 1.0)) for b in boxes], np.float64)
    has_mass = all(b.get("mass") is not None for b in boxes)
    t = lambda a: torch.as_tensor(a, device=device)  # noqa: E731
    return (t(pos), t(cat("rho")), t(cat("kappa")), t(cat("lum")),
            t(cat("mass")) if has_mass else None, lo, hi, off)


_TUNE_CACHE = {}

DEFAULT_CANDIDATES = tuple((bpc, wpb, chunk)
                           for wpb in (4, 2, 1)
                           for bpc in (1, 2, 3, 4, 6, 8)
                           for chunk in (64, 128, 256)
                           if 2 <= bpc * wpb <= 16)

# Bumped when the candidate space or the meaning of a stored record changes.
_TUNE_FORMAT = 2


def tune_cache_path():
    """The JSON file that keeps autotuning results across processes:
    $TREVR_TUNE_CACHE, else ~/.cache/trevr/autotune.json."""
    return os.environ.get("TREVR_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "trevr", "autotune.json")


_LIB_DIGEST = None


def _lib_digest():
    """SHA-256 (first 16 hex digits) of the loaded library file: a rebuilt
    kernel invalidates the stored launch shapes."""
    global _LIB_DIGEST
    if _LIB_DIGEST is None:
        import hashlib
        h = hashlib.sha256()
        with open(LIB_PATH, "rb") as f:
            for block in iter(lambda: f.read(1 << 20), b""):
                h.update(block)
        _LIB_DIGEST = h.hexdigest()[:16]
    return _LIB_DIGEST


def tune_key(info, theta_open, tau_ref, n_sinks, device_name, lib_digest):
    """The cache key of one tuning: the tree's shape (particles, cells, boxes,
    depth, value type), the walk parameters, the sink count, the GPU and the
    library build."""
    return "|".join([
        "v%d" % _TUNE_FORMAT, str(device_name), str(lib_digest),
        "n=%d" % info["n"], "m=%d" % info["m"], "boxes=%d" % info["n_boxes"],
        "depth=%d" % info["max_depth"], "prec=%s" % info["prec"],
        "theta=%r" % float(theta_open), "tau_ref=%r" % float(tau_ref),
        "sinks=%s" % ("all" if n_sinks is None else int(n_sinks))])


def tune_cache_load(path):
    """The stored tunings ({} if the file is missing or unreadable)."""
    import json
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return {}
    if not isinstance(d, dict) or d.get("format") != _TUNE_FORMAT:
        return {}
    e = d.get("entries")
    return e if isinstance(e, dict) else {}


def tune_cache_store(path, key, record):
    """Add one tuning to the file: read, merge, write a temporary file and
    rename it over the old one (a concurrent writer loses at most its own
    entry, never the file)."""
    import json
    entries = tune_cache_load(path)
    entries[key] = record
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    tmp = "%s.tmp%d" % (path, os.getpid())
    with open(tmp, "w") as f:
        json.dump({"format": _TUNE_FORMAT, "entries": entries}, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(tree, theta_open, tau_ref, sinks=None, candidates=DEFAULT_CANDIDATES, reps=3,
             key=None, cache_path=None, persist=True):
    """Time the flux launch under each (workgroups per CU, waves per
    workgroup, sinks per queue grab) candidate and keep the fastest on the
    tree.  The shape also picks the kernel's occupancy variant, and with it
    how the LDS is split between the per-lane refinement stack, the
    sink-ancestor window and the queue.  Results are cached in memory and,
    with `persist`, in the JSON file `cache_path` (default tune_cache_path()),
    keyed by tune_key(); a hit sets the stored shape without timing
    anything.  Returns {"launch", "ms", "table", "source"}."""
    import numpy as np
    info = tree.info()
    if key is None:
        key = tune_key(info, theta_open, tau_ref, None if sinks is None else len(sinks),
                       torch.cuda.get_device_name(tree.device), _lib_digest())
    path = cache_path or tune_cache_path()
    best = _TUNE_CACHE.get(key)
    if best is None and persist:
        rec = tune_cache_load(path).get(key)
        if rec is not None and tuple(rec.get("launch", ())) in {tuple(c) for c in candidates}:
            best = {"launch": tuple(rec["launch"]), "ms": float(rec["ms"]),
                    "table": [(float(t), tuple(c)) for t, c in rec.get("table", [])],
                    "source": "file"}
            _TUNE_CACHE[key] = best
    if best is not None:
        tree.set_launch(*best["launch"])
        return best
    s, ns = tree._sinks(sinks)
    out = torch.empty(ns, dtype=tree.dtype, device=tree.device)
    st = torch.cuda.current_stream()
    table = []
    for cand in candidates:
        tree.set_launch(*cand)
        tree.flux(theta_open, tau_ref, s, out=out)  # warm-up
        ms = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            tree.flux(theta_open, tau_ref, s, out=out)
            e1.record(st)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        table.append((float(np.median(ms)), tuple(cand)))
    table.sort()
    best = {"launch": table[0][1], "ms": table[0][0], "table": table, "source": "timed"}
    tree.set_launch(*best["launch"])
    _TUNE_CACHE[key] = best
    if persist:
        try:
            tune_cache_store(path, key, {"launch": list(best["launch"]), "ms": best["ms"],
                                         "table": [[t, list(c)] for t, c in table]})
        except OSError as e:  # an unwritable cache costs a re-tune later, nothing else
            import warnings
            warnings.warn("autotune: could not write %s: %s" % (path, e))
    return best


class BatchedPlan:
    """Many independent boxes of uneven size evaluated as one forest: one
    tree build, then one persistent flux launch (queue reset + walk kernel)
    captured in a HIP graph and replayed.  The launch shape is autotuned
    before capture."""

    def __init__(self, boxes, theta_open=0.75, tau_ref=0.1, bucket_size=8, device="cuda",
                 tune=True, candidates=DEFAULT_CANDIDATES, tune_cache=None, persist_tuning=True):
        pos, rho, kappa, lum, mass, lo, hi, off = _concat_boxes(boxes, device)
        self.offsets = off
        self.theta_open = float(theta_open)
        self.tau_ref = float(tau_ref)
        self.tree = Tree().build(pos, rho, kappa, lum, mass, lo, hi, bucket_size, off, device)
        self.flux = torch.empty(pos.shape[0], dtype=pos.dtype, device=pos.device)
        self.tuning = (autotune(self.tree, self.theta_open, self.tau_ref, candidates=candidates,
                                cache_path=tune_cache, persist=persist_tuning)
                       if tune else None)
        self.graph = None

    def eager(self):
        return self.tree.flux(self.theta_open, self.tau_ref, out=self.flux)

    def capture(self):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.eager()
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.eager()
        self.graph = g
        return self

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()
        return self.flux

    def per_box(self, F=None):
        F = self.flux if F is None else F
        return [F[int(self.offsets[b]):int(self.offsets[b + 1])]
                for b in range(len(self.offsets) - 1)]


# ---- ionisation-equilibrium coupling ----------------------------------------

def ionisation_update(flux, x, kappa, sigma, alpha_b, damping=0.5, n_h=None, dx_max=None):
    """One damped on-the-spot equilibrium step per particle (trevr_ionisation_update):
    x and kappa (= sigma x) are updated in place; returns the device scalar
    max |x_eq - x_old|.  With flux None only kappa = sigma x is written."""
    dt = x.dtype
    prec = 1 if dt == torch.float64 else 0
    for a in (x, kappa) + tuple(v for v in (flux, n_h) if v is not None):
        if a.dtype != dt or not a.is_contiguous() or a.shape != x.shape:
            raise ValueError("flux, x, kappa (and n_h) must be contiguous, same dtype and shape")
    d = dx_max if dx_max is not None else torch.empty(1, dtype=torch.float64, device=x.device)
    _check(lib().trevr_ionisation_update(int(x.shape[0]), prec, _ptr(flux), _ptr(n_h),
                                         float(sigma), float(alpha_b), float(damping), _ptr(x),
                                         _ptr(kappa), _ptr(d), _stream()))
    return d


def ionisation_equilibrium(pos, rho, lum, mass, x, sigma, alpha_b, theta_open=0.75,
                           tau_ref=-1.0, damping=0.5, tol=1e-7, max_iter=200, box_lo=(0.0,) * 3,
                           box_hi=(1.0,) * 3, bucket_size=8):
    """Photoionisation equilibrium with the flux as its source term: kappa =
    sigma x, the flux at every particle, a damped update of x towards the
    on-the-spot equilibrium for n_H = rho; repeated until max |x_eq - x| < tol.
    The tree is built once and refit with the new opacities each step.
    Returns (x, flux, iterations, last max |x_eq - x|)."""
    x = x.clone().contiguous()
    kappa = torch.empty_like(x)
    ionisation_update(None, x, kappa, sigma, alpha_b)  # kappa = sigma x
    tree = Tree().build(pos, rho, kappa, lum, mass, box_lo, box_hi, bucket_size)
    F = torch.empty_like(x)
    d = torch.empty(1, dtype=torch.float64, device=x.device)
    dx = float("inf")
    it = 0
    while it < max_iter:
        tree.flux(theta_open, tau_ref, out=F)
        ionisation_update(F, x, kappa, sigma, alpha_b, damping, n_h=rho, dx_max=d)
        it += 1
        dx = float(d.item())
        if dx < tol:
            break
        tree.refit(pos, rho, kappa, lum, mass)
    return x, F, it, dx
