"""Seeded synthetic particle sets for the TREVR radiation-field workloads.

This module only draws inputs (positions, densities, opacities,
luminosities); it holds none of the method's arithmetic and is shared by the
tests, the benchmark and the smoke check.

The paper's own test particle sets (a perturbed glass, isothermal spheres)
are stand-ins here for the clustered media it describes (Sec. 3.1: dense
filaments, under-dense voids, box optical depth of order unity): a log-normal
density field with a power-law spectrum, sampled by particles.

Recipe (all draws from ``numpy.random.default_rng(seed)``, binary64):
  * field: 64^3 white noise -> FFT -> times k^(-3/2) (k = 0 removed) ->
    inverse FFT -> normalised to unit variance g; rho_grid = exp(s g - s^2/2),
    s = 1.5 (volume mean close to 1);
  * positions: a cell is drawn with probability proportional to rho_grid
    (the same distribution as accept/reject against rho_grid / max rho_grid)
    and a uniform point inside it;
  * rho_i = rho_grid at the particle's cell, m_i = 1/N,
    kappa_i = tau_box / mean(rho_grid) (box-crossing optical depth tau_box
    for a unit box);
  * luminosities: log10 L ~ N(0, 1) for the chosen sources, 0 elsewhere.
Binary32 workloads round positions to binary32 (kept inside [0, 1)) and pass
every array as binary32; the oracle reads the same binary32 values.
"""
from __future__ import annotations

import numpy as np

GRID = 64
SIGMA_LN_RHO = 1.5

CONFIG_NAMES = ("c1_uniform4096_f64", "c2_lognormal2e18_f32", "c3_lognormal2e21_all_sources_f32",
                "c4_batched64_f32", "c5_adjoint2e20_f32")


def lognormal_field(rng, n=GRID, sigma=SIGMA_LN_RHO):
    noise = rng.standard_normal((n, n, n))
    fk = np.fft.rfftn(noise)
    kx = np.fft.fftfreq(n) * n
    kz = np.fft.rfftfreq(n) * n
    k = np.sqrt(kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2)
    amp = np.zeros_like(k)
    amp[k > 0] = k[k > 0] ** -1.5
    g = np.fft.irfftn(fk * amp, s=(n, n, n), axes=(0, 1, 2))
    g = (g - g.mean()) / g.std()
    return np.exp(sigma * g - 0.5 * sigma * sigma)


def _clip_unit(x, dtype):
    x = x.astype(dtype)
    top = np.nextafter(dtype(1.0), dtype(0.0))
    return np.clip(x, dtype(0.0), top)


def sample_field(rng, rho_grid, n):
    g = rho_grid.shape[0]
    p = rho_grid.ravel() / rho_grid.sum()
    cell = rng.choice(p.size, size=n, p=p)
    ijk = np.stack(np.unravel_index(cell, rho_grid.shape), axis=1).astype(np.float64)
    pos = (ijk + rng.random((n, 3))) / g
    return pos, rho_grid.ravel()[cell]


def _pack(name, pos, rho, kappa, lum, mass, prec, theta=0.75, tau_ref=0.1, bucket=8, **extra):
    dt = np.float64 if prec == "f64" else np.float32
    w = {
        "name": name, "prec": prec,
        "pos": _clip_unit(pos, dt),
        "rho": rho.astype(dt), "kappa": kappa.astype(dt), "lum": lum.astype(dt),
        "mass": mass.astype(dt),
        "box_lo": (0.0, 0.0, 0.0), "box_hi": (1.0, 1.0, 1.0),
        "bucket_size": bucket, "theta": theta, "tau_ref": tau_ref,
    }
    w.update(extra)
    return w


def uniform_box(n, n_src, tau_box=1.0, seed=1, prec="f64", lum_law="uniform"):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    rho = np.ones(n)
    kappa = np.full(n, float(tau_box))
    lum = np.zeros(n)
    src = rng.choice(n, size=n_src, replace=False)
    if lum_law == "uniform":
        lum[src] = rng.uniform(0.5, 1.0, n_src)
    else:
        lum[src] = 10.0 ** rng.standard_normal(n_src)
    return pos, rho, kappa, lum, np.full(n, 1.0 / n)


def lognormal_box(n, n_src, tau_box, seed, all_sources=False):
    rng = np.random.default_rng(seed)
    grid = lognormal_field(rng)
    pos, rho = sample_field(rng, grid, n)
    kappa = np.full(n, tau_box / grid.mean())
    lum = np.zeros(n)
    if all_sources:
        lum[:] = 10.0 ** rng.standard_normal(n)
    else:
        src = rng.choice(n, size=n_src, replace=False)
        lum[src] = 10.0 ** rng.standard_normal(n_src)
    return pos, rho, kappa, lum, np.full(n, 1.0 / n)


def c1(seed=1):
    """4096 uniform particles, rho = kappa = 1 (box-crossing tau = 1), 16 sources
    with L ~ U[0.5, 1], N_B = 8, theta = 0.75, tau_ref = 0.1, binary64."""
    return _pack("c1_uniform4096_f64", *uniform_box(4096, 16, 1.0, seed), prec="f64")


def c2(seed=2, n=1 << 18):
    """2^18 particles in the log-normal field, 1024 sources, tau_box = 5, binary32."""
    return _pack("c2_lognormal2e18_f32", *lognormal_box(n, 1024, 5.0, seed), prec="f32")


def c3(seed=3, n=1 << 21, theta=0.75, tau_ref=0.1):
    """2^21 particles in the log-normal field, every particle a source,
    tau_box = 10, binary32 (the headline configuration)."""
    return _pack("c3_lognormal2e21_all_sources_f32",
                 *lognormal_box(n, n, 10.0, seed, all_sources=True), prec="f32",
                 theta=theta, tau_ref=tau_ref)


C3_SWEEP = [(th, tr) for th in (0.5, 0.75, 1.0) for tr in (0.05, 0.1, 0.2)]


def c4(n_boxes=64, base_seed=4000, max_log2=17):
    """64 independent unit boxes: N_b = round(2^U(12, 17)), uniform or log-normal
    density (coin), 1..512 sources with log-normal L, tau_box ~ U(0.1, 20)."""
    boxes = []
    for b in range(n_boxes):
        rng = np.random.default_rng(base_seed + b)
        nb = int(round(2.0 ** rng.uniform(12.0, max_log2)))
        lognormal = bool(rng.integers(0, 2))
        n_src = int(rng.integers(1, 513))
        tau_box = float(rng.uniform(0.1, 20.0))
        sub = int(rng.integers(0, 2 ** 31))
        if lognormal:
            arrs = lognormal_box(nb, n_src, tau_box, sub)
        else:
            arrs = uniform_box(nb, n_src, tau_box, sub, lum_law="lognormal")
        boxes.append(_pack("c4_box%02d" % b, *arrs, prec="f32", tau_box=tau_box,
                           lognormal=lognormal))
    return boxes


def c5(seed=5, target_seed=55, n=1 << 20):
    """2^20 particles in the log-normal field, 4096 sources, tau_box = 10,
    binary32; target densities rho' = rho exp(0.2 xi), xi ~ N(0, 1)."""
    w = _pack("c5_adjoint2e20_f32", *lognormal_box(n, 4096, 10.0, seed), prec="f32")
    rng = np.random.default_rng(target_seed)
    w["rho_target"] = (w["rho"].astype(np.float64) * np.exp(0.2 * rng.standard_normal(n))
                       ).astype(np.float32)
    return w


def scaled(w_fn, n, **kw):
    """A smaller instance of a configuration's recipe (parity tests)."""
    return w_fn(n=n, **kw)


# Table tab:modes (App. A): wave vector (k_x, k_y, k_z) and phase phi of the
# 24 sinusoidal modes of eq. manfft.
TAB_MODES = np.array([
    [-3.918398, +1.727743, -4.476095, 0.829776],  # 01
    [-3.681821, -4.619688, +4.865007, 3.891157],  # 02
    [-4.831801, +3.769470, +0.567451, 3.668730],  # 03
    [-2.298279, +1.501757, +4.716946, 1.528348],  # 04
    [-0.289974, -3.097958, +1.270028, 4.113001],  # 05
    [+1.262943, -1.661726, -2.600413, 4.481799],  # 06
    [+1.588224, +4.072259, +0.616444, 2.971965],  # 07
    [-2.253394, -2.806478, +2.749155, 0.442241],  # 08
    [-1.432569, +3.324710, +4.842991, 2.871989],  # 09
    [+1.287742, -4.575517, -4.001723, 1.727810],  # 10
    [+4.769704, +0.540096, -4.203839, 5.872117],  # 11
    [-3.013200, -1.871251, -2.514416, 1.574008],  # 12
    [-4.588620, +4.384224, +1.246849, 1.985715],  # 13
    [-0.372817, +0.195243, +4.074056, 6.248739],  # 14
    [-1.842232, +0.901598, -4.453613, 6.273336],  # 15
    [+1.986937, -1.037650, +1.958888, 2.177783],  # 16
    [-1.748485, -1.386029, +3.755833, 0.532604],  # 17
    [+4.852406, -3.272506, +0.826504, 5.525470],  # 18
    [+3.663293, -4.597598, -0.890135, 4.528870],  # 19
    [-1.720903, +2.726011, +3.192427, 3.875610],  # 20
    [+4.973332, +4.777182, -2.515792, 0.406737],  # 21
    [+0.057238, -2.972427, -1.828550, 4.125258],  # 22
    [+0.938234, -0.487023, -2.755097, 1.335299],  # 23
    [+1.943361, +0.388178, -3.783953, 4.774938],  # 24
])
MODE_AMPLITUDE = 1.0 / 275.0


def perturb_modes(r0):
    """eq. manfft, read as printed: every coordinate of a particle moves by the
    same scalar, sum_i A sin(k_i . r0 + phi_i) with A = 1/275, evaluated at
    the unperturbed position.  Returns the moved positions and the Jacobian
    determinant of the map, det(I + 1 grad f) = 1 + sum_i A (k_x + k_y +
    k_z)_i cos(k_i . r0 + phi_i), so that rho = rho0 / det."""
    ph = r0 @ TAB_MODES[:, :3].T + TAB_MODES[:, 3]
    f = MODE_AMPLITUDE * np.sin(ph).sum(axis=1)
    det = 1.0 + MODE_AMPLITUDE * (np.cos(ph) * TAB_MODES[:, :3].sum(axis=1)).sum(axis=1)
    return r0 + f[:, None], det


def ctx_lattice(n_side=64, jitter=0.25, seed=61, prec="f32"):
    """Paper-context workload (Sec. 3.1.1, App. A): N gas and N star
    particles, N = n_side^3.  The 16^3 glass the paper tiles is replaced by a
    lattice of cell centres with a seeded uniform jitter of +-jitter spacings
    per coordinate; the stars take the glass with coordinates reassigned
    (x, y, z)_star = (y, z, x)_gas; both are then moved by the 24 modes
    (perturb_modes).  Gas: total mass 1 (m = 1/N), kappa = 1, rho = 1 / det of
    the map (the exact density of a unit-density medium under it), L = 0.
    Stars: L = 1, mass 0 (they do not absorb).  Particles [0, N) are gas (the
    sinks, "resolution elements"), [N, 2N) stars.  The box is [-0.05, 1.05]^3,
    which holds every moved particle (|f| <= 24/275)."""
    rng = np.random.default_rng(seed)
    g = (np.arange(n_side) + 0.5) / n_side
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    glass = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    glass = glass + rng.uniform(-jitter, jitter, glass.shape) / n_side
    n = glass.shape[0]
    gas, det = perturb_modes(glass)
    stars, _ = perturb_modes(glass[:, [1, 2, 0]])
    pos = np.concatenate([gas, stars])
    rho = np.concatenate([1.0 / det, np.ones(n)])
    kappa = np.concatenate([np.ones(n), np.zeros(n)])
    lum = np.concatenate([np.zeros(n), np.ones(n)])
    mass = np.concatenate([np.full(n, 1.0 / n), np.zeros(n)])
    dt = np.float64 if prec == "f64" else np.float32
    return {"name": "ctx_lattice%d_f%s" % (n_side, "64" if prec == "f64" else "32"),
            "prec": prec, "pos": pos.astype(dt), "rho": rho.astype(dt),
            "kappa": kappa.astype(dt), "lum": lum.astype(dt), "mass": mass.astype(dt),
            "box_lo": (-0.05, -0.05, -0.05), "box_hi": (1.05, 1.05, 1.05), "bucket_size": 8,
            "theta": 0.75, "tau_ref": 0.1, "n_gas": n, "det_min": float(det.min()),
            "det_max": float(det.max())}
