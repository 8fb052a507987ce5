"""ctypes wrapper of the TREVR reference oracle (``trevr_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the product library never does.  Everything here
is argument marshalling; the arithmetic is in the C file, in binary64.

``mirror32=True`` makes the oracle read every value the walk reads (cell
boxes, split planes, centres of luminosity, luminosities, far-vertex
distances, alpha and alpha_max - alpha_min, particle positions and
luminosities) rounded to binary32, as the GPU library stores them in its
binary32 transport mode, and compute each ray's geometry (direction, 1/d,
r^2, r, plane crossings, piece lengths) in binary32 as that mode does; the
criterion products, the alpha l terms and the sums stay binary64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "trevr_oracle.c")
# TREVR_ORACLE_LIB names another build of the same source (the sanitizer tests
# load an instrumented one); it is loaded as it is, never rebuilt
_LIB_ENV = os.environ.get("TREVR_ORACLE_LIB")
_LIB = _LIB_ENV or os.path.join(_HERE, "liboracle.so")

NODE_F_FIELDS = (
    "lo0", "lo1", "lo2", "hi0", "hi1", "hi2", "split", "A", "B", "SL",
    "SLx0", "SLx1", "SLx2", "alpha", "alpha_min", "alpha_max", "dalpha",
    "xl0", "xl1", "xl2", "lc", "lfar",
)
TRANSPORT_FIELDS = (
    "lo0", "lo1", "lo2", "hi0", "hi1", "hi2", "split", "xl0", "xl1", "xl2", "lc", "lfar",
    "alpha", "dalpha",
)
NODE_I_FIELDS = ("first", "count", "depth", "leaf", "parent", "right", "skip", "axis")
COUNTER_FIELDS = ("n_open", "n_rays", "n_psrc", "n_seg", "n_trace")


GCC_FLAGS = ["-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-fno-fast-math"]


def build_library(force: bool = False, path: str = None, extra=("-O2",)) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no FMA contraction);
    `path` and `extra` make another build (e.g. with sanitizers)."""
    out = path or _LIB
    if path is None and _LIB_ENV:
        return _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc"] + list(extra) + GCC_FLAGS + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_library()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.oracle_build.restype = P
        L.oracle_build.argtypes = [ctypes.c_int64] + [P] * 9 + [ctypes.c_int, ctypes.c_int]
        L.oracle_free.argtypes = [P]
        L.oracle_num_nodes.restype = ctypes.c_int64
        L.oracle_num_nodes.argtypes = [P]
        L.oracle_axis.restype = ctypes.c_int
        L.oracle_axis.argtypes = [P, ctypes.c_int]
        L.oracle_export.argtypes = [P] * 6
        L.oracle_export_transport.restype = ctypes.c_int
        L.oracle_export_transport.argtypes = [P] * 4
        L.oracle_flux.restype = ctypes.c_int
        L.oracle_flux.argtypes = [P, ctypes.c_double, ctypes.c_double, P, ctypes.c_int64,
                                  ctypes.c_int, P, P, P]
        L.oracle_flux_vec.restype = ctypes.c_int
        L.oracle_flux_vec.argtypes = [P, ctypes.c_double, ctypes.c_double, P, ctypes.c_int64,
                                      ctypes.c_int, P, P]
        L.oracle_flux_moments.restype = ctypes.c_int
        L.oracle_flux_moments.argtypes = [P, ctypes.c_double, ctypes.c_double, P, ctypes.c_int64,
                                          ctypes.c_int, P, P, P]
        L.oracle_set_bands.restype = ctypes.c_int
        L.oracle_set_bands.argtypes = [P, ctypes.c_int, P]
        L.oracle_flux_bands.restype = ctypes.c_int
        L.oracle_flux_bands.argtypes = [P, ctypes.c_double, ctypes.c_double, P, ctypes.c_int64,
                                        ctypes.c_int, P, P]
        L.oracle_sph_line.restype = ctypes.c_double
        L.oracle_sph_line.argtypes = [ctypes.c_double] * 4
        L.oracle_set_sph.restype = ctypes.c_int
        L.oracle_set_sph.argtypes = [P, P]
        L.oracle_sph_neighbours.restype = ctypes.c_int64
        L.oracle_sph_neighbours.argtypes = [P, ctypes.c_int64, ctypes.c_int64, P]
        L.oracle_sph_spread.restype = ctypes.c_int
        L.oracle_sph_spread.argtypes = [P, P]
        L.oracle_flux_sph.restype = ctypes.c_int
        L.oracle_flux_sph.argtypes = [P, ctypes.c_double, ctypes.c_double, P, ctypes.c_int64,
                                      ctypes.c_int, P, P]
        L.oracle_ray_log_sph.restype = ctypes.c_int64
        L.oracle_ray_log_sph.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                         ctypes.c_int64] + [P] * 6
        L.oracle_flux_variant.restype = ctypes.c_int
        L.oracle_flux_variant.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_double, P, ctypes.c_int64,
                                          ctypes.c_int, P, P]
        L.oracle_ray_log_variant.restype = ctypes.c_int64
        L.oracle_ray_log_variant.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int64, ctypes.c_int64] + [P] * 6
        L.oracle_set_background.restype = ctypes.c_int
        L.oracle_set_background.argtypes = [P, P, ctypes.c_double, P]
        L.oracle_flux_background.restype = ctypes.c_int
        L.oracle_flux_background.argtypes = [P, ctypes.c_double, ctypes.c_double, P,
                                             ctypes.c_int64, ctypes.c_int, P, P]
        L.oracle_background_cells.restype = ctypes.c_int
        L.oracle_background_cells.argtypes = [P, P, P]
        L.oracle_ray_log.restype = ctypes.c_int64
        L.oracle_ray_log.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                     ctypes.c_int64] + [P] * 6
        L.oracle_ray_pieces.restype = ctypes.c_int64
        L.oracle_ray_pieces.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int64, P, P]
        L.oracle_adjoint.restype = ctypes.c_int
        L.oracle_adjoint.argtypes = [P, ctypes.c_double, ctypes.c_double, P, ctypes.c_int64, P,
                                     ctypes.c_int, P, P, P]
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleTree:
    """The oracle's tree over one box of particles."""

    def __init__(self, pos, rho, kappa, lum, mass=None, box_lo=(0.0, 0.0, 0.0),
                 box_hi=(1.0, 1.0, 1.0), bucket_size=8, mirror32=False):
        pos = _d(pos)
        self.n = int(pos.shape[0])
        self._keep = [_d(pos[:, 0]), _d(pos[:, 1]), _d(pos[:, 2]),
                      None if mass is None else _d(mass), _d(rho), _d(kappa), _d(lum),
                      _d(box_lo), _d(box_hi)]
        k = self._keep
        h = lib().oracle_build(self.n, _ptr(k[0]), _ptr(k[1]), _ptr(k[2]), _ptr(k[3]),
                               _ptr(k[4]), _ptr(k[5]), _ptr(k[6]), _ptr(k[7]), _ptr(k[8]),
                               int(bucket_size), int(bool(mirror32)))
        if not h:
            raise ValueError("oracle rejected the particle set")
        self._h = ctypes.c_void_p(h)
        self.m = int(lib().oracle_num_nodes(self._h))
        self.mirror32 = bool(mirror32)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.oracle_free(h)
            self._h = None

    def axes(self):
        return np.array([lib().oracle_axis(self._h, d) for d in range(64)], dtype=np.int64)

    def export(self):
        perm = np.empty(self.n, np.int64)
        leaf_of = np.empty(self.n, np.int64)
        node_i = np.empty((self.m, 8), np.int64)
        node_key = np.empty(self.m, np.uint64)
        node_f = np.empty((self.m, len(NODE_F_FIELDS)), np.float64)
        lib().oracle_export(self._h, _ptr(perm), _ptr(leaf_of), _ptr(node_i), _ptr(node_key),
                            _ptr(node_f))
        out = {"perm": perm, "leaf_of": leaf_of, "key": node_key}
        for j, f in enumerate(NODE_I_FIELDS):
            out[f] = node_i[:, j].copy()
        for j, f in enumerate(NODE_F_FIELDS):
            out[f] = node_f[:, j].copy()
        return out

    def export_transport(self):
        """The values the walk reads: per cell the box, split plane, centre of
        luminosity, luminosity, far-vertex distance, alpha and its spread, and
        per particle the position and luminosity -- binary64, or each rounded
        once to binary32 in mirror mode."""
        node_t = np.empty((self.m, len(TRANSPORT_FIELDS)), np.float64)
        pos = np.empty((self.n, 3), np.float64)
        lum = np.empty(self.n, np.float64)
        lib().oracle_export_transport(self._h, _ptr(node_t), _ptr(pos), _ptr(lum))
        out = {f: node_t[:, j].copy() for j, f in enumerate(TRANSPORT_FIELDS)}
        out["pos"] = pos
        out["lum"] = lum
        return out

    def flux(self, theta, tau_ref, sinks=None, nthreads=0, with_g=False):
        """Return (F, counters[ns,5]) (and G = sum f tau if with_g)."""
        s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
        ns = self.n if s is None else int(s.shape[0])
        F = np.empty(ns, np.float64)
        C = np.empty((ns, 5), np.int64)
        G = np.empty(ns, np.float64) if with_g else None
        rc = lib().oracle_flux(self._h, float(theta), float(tau_ref), _ptr(s), ns,
                               int(nthreads), _ptr(F), _ptr(C), _ptr(G))
        if rc != 0:
            raise ValueError("oracle_flux rejected its arguments")
        return (F, C, G) if with_g else (F, C)

    def flux_vector(self, theta, tau_ref, sinks=None, nthreads=0):
        """Return (F, Fv[ns, 3]): the flux and the vector flux, each ray's
        flux along its direction of travel at the sink, summed in walk order."""
        s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
        ns = self.n if s is None else int(s.shape[0])
        F = np.empty(ns, np.float64)
        Fv = np.empty((ns, 3), np.float64)
        rc = lib().oracle_flux_vec(self._h, float(theta), float(tau_ref), _ptr(s), ns,
                                   int(nthreads), _ptr(F), _ptr(Fv))
        if rc != 0:
            raise ValueError("oracle_flux_vec rejected its arguments")
        return F, Fv

    def flux_moments(self, theta, tau_ref, sinks=None, nthreads=0):
        """Return (F, Fv[ns, 3], P[ns, 6]): flux, vector flux and the second
        moment sum f n_a n_b (xx, yy, zz, xy, xz, yz), in walk order."""
        s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
        ns = self.n if s is None else int(s.shape[0])
        F = np.empty(ns, np.float64)
        Fv = np.empty((ns, 3), np.float64)
        Pm = np.empty((ns, 6), np.float64)
        rc = lib().oracle_flux_moments(self._h, float(theta), float(tau_ref), _ptr(s), ns,
                                       int(nthreads), _ptr(F), _ptr(Fv), _ptr(Pm))
        if rc != 0:
            raise ValueError("oracle_flux_moments rejected its arguments")
        return F, Fv, Pm

    def flux_bands(self, theta, tau_ref, kappa_bands, sinks=None, nthreads=0):
        """Flux per opacity band on one traversal (refined where any band's
        criterion holds).  kappa_bands: (k, n).  Returns (Fb[ns, k], counters)."""
        kb = np.ascontiguousarray(kappa_bands, dtype=np.float64)
        if kb.ndim != 2 or kb.shape[1] != self.n:
            raise ValueError("kappa_bands must be (k, n)")
        if lib().oracle_set_bands(self._h, int(kb.shape[0]), _ptr(kb)) != 0:
            raise ValueError("oracle_set_bands rejected its arguments")
        s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
        ns = self.n if s is None else int(s.shape[0])
        Fb = np.empty((ns, kb.shape[0]), np.float64)
        C = np.empty((ns, 5), np.int64)
        rc = lib().oracle_flux_bands(self._h, float(theta), float(tau_ref), _ptr(s), ns,
                                     int(nthreads), _ptr(Fb), _ptr(C))
        if rc != 0:
            raise ValueError("oracle_flux_bands rejected its arguments")
        return Fb, C

    # ---- background shell ----
    def set_background(self, centre, radius, flags):
        """Background sources (flags[n], input order) on the sphere (centre,
        radius): merged cells of them radiate from the sphere."""
        self._bg_c = _d(centre)
        self._bg_f = np.ascontiguousarray(flags, dtype=np.uint8)
        if self._bg_f.shape != (self.n,):
            raise ValueError("flags must have one entry per particle")
        if lib().oracle_set_background(self._h, _ptr(self._bg_c), float(radius),
                                       _ptr(self._bg_f)) != 0:
            raise ValueError("oracle_set_background rejected its arguments")

    def flux_background(self, theta, tau_ref, sinks=None, nthreads=0):
        s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
        ns = self.n if s is None else int(s.shape[0])
        F = np.empty(ns, np.float64)
        C = np.empty((ns, 5), np.int64)
        rc = lib().oracle_flux_background(self._h, float(theta), float(tau_ref), _ptr(s), ns,
                                          int(nthreads), _ptr(F), _ptr(C))
        if rc != 0:
            raise ValueError("oracle_flux_background rejected its arguments")
        return F, C

    def background_cells(self):
        flag = np.empty(self.m, np.uint8)
        pos = np.empty((self.m, 3), np.float64)
        if lib().oracle_background_cells(self._h, _ptr(flag), _ptr(pos)) != 0:
            raise ValueError("set_background first")
        return flag.astype(bool), pos

    # ---- walk variants ----
    def flux_variant(self, theta, tau_ref, open_mode=0, ray_mode=0, tau_max=np.inf, sinks=None,
                     nthreads=0):
        """Flux with a walk variant: open_mode 0 (sink point, eq. openangle), 1 (the
        sink's bucket box), 2 (Gasoline's r_open about x_L); ray_mode 0 (up the
        tree), 1 (top down from the meeting cell); rays with tau > tau_max
        contribute nothing.  Returns (F, counters[ns, 5])."""
        s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
        ns = self.n if s is None else int(s.shape[0])
        F = np.empty(ns, np.float64)
        C = np.empty((ns, 5), np.int64)
        rc = lib().oracle_flux_variant(self._h, float(theta), float(tau_ref), int(open_mode),
                                       int(ray_mode), float(tau_max), _ptr(s), ns,
                                       int(nthreads), _ptr(F), _ptr(C))
        if rc != 0:
            raise ValueError("oracle_flux_variant rejected its arguments")
        return F, C

    def ray_log_variant(self, theta, tau_ref, sink, open_mode=0, ray_mode=0, cap=1 << 20):
        C = np.empty(cap, np.int64)
        src = np.empty(cap, np.int64)
        y = np.empty((cap, 3), np.float64)
        L = np.empty(cap, np.float64)
        tau = np.empty(cap, np.float64)
        f = np.empty(cap, np.float64)
        nr = lib().oracle_ray_log_variant(self._h, float(theta), float(tau_ref), int(open_mode),
                                          int(ray_mode), int(sink), cap, _ptr(C), _ptr(src),
                                          _ptr(y), _ptr(L), _ptr(tau), _ptr(f))
        k = min(nr, cap)
        return {"C": C[:k], "src": src[:k], "y": y[:k], "L": L[:k], "tau": tau[:k], "f": f[:k]}

    # ---- sub-bucket particle trace ----
    def set_sph(self, h):
        """Smoothing lengths (input order) for the sub-bucket particle trace."""
        h = _d(h)
        if h.shape != (self.n,):
            raise ValueError("h must have one entry per particle")
        self._h_sph = h
        if lib().oracle_set_sph(self._h, _ptr(h)) != 0:
            raise ValueError("oracle_set_sph rejected the smoothing lengths")

    def flux_sph(self, theta, tau_ref, sinks=None, nthreads=0):
        """Flux with the sub-bucket particle trace: (F, counters[ns, 5])."""
        s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
        ns = self.n if s is None else int(s.shape[0])
        F = np.empty(ns, np.float64)
        C = np.empty((ns, 5), np.int64)
        rc = lib().oracle_flux_sph(self._h, float(theta), float(tau_ref), _ptr(s), ns,
                                   int(nthreads), _ptr(F), _ptr(C))
        if rc != 0:
            raise ValueError("oracle_flux_sph rejected its arguments (set_sph first)")
        return F, C

    def sph_neighbours(self, node):
        n = int(lib().oracle_sph_neighbours(self._h, int(node), 0, None))
        out = np.empty(max(n, 1), np.int64)
        lib().oracle_sph_neighbours(self._h, int(node), n, _ptr(out))
        return out[:n]

    def sph_spread(self):
        dp = np.empty(self.m, np.float64)
        if lib().oracle_sph_spread(self._h, _ptr(dp)) != 0:
            raise ValueError("set_sph first")
        return dp

    def ray_log_sph(self, theta, tau_ref, sink, cap=1 << 20):
        return self.ray_log(theta, tau_ref, sink, cap, sph=True)

    def ray_log(self, theta, tau_ref, sink, cap=1 << 20, sph=False):
        C = np.empty(cap, np.int64)
        src = np.empty(cap, np.int64)
        y = np.empty((cap, 3), np.float64)
        L = np.empty(cap, np.float64)
        tau = np.empty(cap, np.float64)
        f = np.empty(cap, np.float64)
        fn = lib().oracle_ray_log_sph if sph else lib().oracle_ray_log
        nr = fn(self._h, float(theta), float(tau_ref), int(sink), cap,
                _ptr(C), _ptr(src), _ptr(y), _ptr(L), _ptr(tau), _ptr(f))
        k = min(nr, cap)
        return {"C": C[:k], "src": src[:k], "y": y[:k], "L": L[:k], "tau": tau[:k], "f": f[:k]}

    def ray_pieces(self, theta, tau_ref, sink, ray_index, cap=4096):
        """Pieces of one ray: node, ta, tb, alpha, length (in the order added)."""
        node = np.empty(cap, np.int64)
        tp = np.empty((cap, 4), np.float64)
        k = lib().oracle_ray_pieces(self._h, float(theta), float(tau_ref), int(sink),
                                    int(ray_index), cap, _ptr(node), _ptr(tp))
        k = min(k, cap)
        return {"node": node[:k], "ta": tp[:k, 0], "tb": tp[:k, 1], "alpha": tp[:k, 2],
                "len": tp[:k, 3]}

    def adjoint(self, theta, tau_ref, grad_flux, sinks=None, nthreads=0):
        """Gradients (rho, kappa, lum) of sum_i grad_flux[i] * F_i."""
        s = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
        ns = self.n if s is None else int(s.shape[0])
        g = _d(grad_flux)
        assert g.shape[0] == ns
        gr = np.empty(self.n, np.float64)
        gk = np.empty(self.n, np.float64)
        gl = np.empty(self.n, np.float64)
        lib().oracle_adjoint(self._h, float(theta), float(tau_ref), _ptr(s), ns, _ptr(g),
                             int(nthreads), _ptr(gr), _ptr(gk), _ptr(gl))
        return gr, gk, gl


def sph_line(b, h, u0, u1):
    """Integral of the M4 kernel W(sqrt(b^2 + u^2), h) over u in [u0, u1]."""
    return float(lib().oracle_sph_line(float(b), float(h), float(u0), float(u1)))
