"""Independent brute-force checks for the oracle (plain numpy / Python).

Nothing here calls the oracle: these are separate, direct computations of
what the paper's method must give in cases with a plain definition.
"""
from __future__ import annotations

import math

import numpy as np


def split_tree(pos, nb, lo, hi, mass=None, rho=None, kappa=None):
    """Recursive geometric bisection of each cell's longest axis (ties to the
    lowest axis), points on a plane going to the upper half, both halves kept
    (space-filling), buckets of at most nb points.  Returns a list of node
    dicts in depth-first pre-order (left first)."""
    pos = np.asarray(pos, np.float64)
    n = pos.shape[0]
    mass = np.ones(n) if mass is None else np.asarray(mass, np.float64)
    nodes = []

    def rec(idx, clo, chi, depth, parent):
        me = len(nodes)
        node = {"idx": idx, "lo": clo.copy(), "hi": chi.copy(), "depth": depth,
                "parent": parent, "children": None}
        nodes.append(node)
        if idx.size > nb and depth < 63:
            w = chi - clo
            a = int(np.argmax(w))
            s = 0.5 * (clo[a] + chi[a])
            up = pos[idx, a] >= s
            lhi = chi.copy()
            lhi[a] = s
            rlo = clo.copy()
            rlo[a] = s
            l = rec(idx[~up], clo, lhi, depth + 1, me)
            r = rec(idx[up], rlo, chi, depth + 1, me)
            node["children"] = (l, r)
            node["axis"] = a
            node["split"] = s
        return me

    rec(np.arange(n), np.asarray(lo, np.float64), np.asarray(hi, np.float64), 0, -1)
    if rho is not None:
        rho = np.asarray(rho, np.float64)
        kappa = np.asarray(kappa, np.float64)
        for nd in nodes:
            idx = nd["idx"][mass[nd["idx"]] > 0]
            B = float(np.sum(mass[idx] / rho[idx]))
            A = float(np.sum(mass[idx] * kappa[idx]))
            if B > 0:
                nd["alpha"] = A / B
            else:
                nd["alpha"] = 0.0 if nd["parent"] < 0 else nodes[nd["parent"]]["alpha"]
    return nodes


def leaves(nodes):
    return [nd for nd in nodes if nd["children"] is None]


def segment_box_lengths(p0, p1, lo, hi):
    """Length of the segment p0 -> p1 inside each box [lo_k, hi_k] (k rows)."""
    d = p1 - p0
    r = math.sqrt(float(np.dot(d, d)))
    t0 = np.zeros(lo.shape[0])
    t1 = np.ones(lo.shape[0])
    for a in range(3):
        if d[a] != 0.0:
            ta = (lo[:, a] - p0[a]) / d[a]
            tb = (hi[:, a] - p0[a]) / d[a]
            t0 = np.maximum(t0, np.minimum(ta, tb))
            t1 = np.minimum(t1, np.maximum(ta, tb))
        else:
            inside = (lo[:, a] <= p0[a]) & (p0[a] <= hi[:, a])
            t1 = np.where(inside, t1, -1.0)
    return r * np.maximum(t1 - t0, 0.0)


def exact_tau_leaf_field(p0, p1, leaf_lo, leaf_hi, leaf_alpha):
    """Optical depth of the segment through the piecewise-constant field that
    takes each bucket's alpha inside the bucket (eq. tauint, exactly)."""
    ls = segment_box_lengths(p0, p1, leaf_lo, leaf_hi)
    return float(np.sum(leaf_alpha * ls)), int(np.count_nonzero(ls > 0))


def all_pairs_flux(pos, lum, alpha_const=0.0, sinks=None):
    """F_i = sum_{j != i, L_j > 0} L_j exp(-alpha r) / (4 pi r^2) (eq. simpint)."""
    pos = np.asarray(pos, np.float64)
    lum = np.asarray(lum, np.float64)
    src = np.nonzero(lum > 0)[0]
    sinks = np.arange(pos.shape[0]) if sinks is None else np.asarray(sinks)
    out = np.zeros(sinks.size)
    for q, i in enumerate(sinks):
        d = pos[src] - pos[i]
        r2 = np.sum(d * d, axis=1)
        ok = r2 > 0
        r = np.sqrt(r2[ok])
        out[q] = np.sum(lum[src][ok] * np.exp(-alpha_const * r) / (4.0 * math.pi * r2[ok]))
    return out


def all_pairs_vector_flux(pos, lum, alpha_const=0.0, sinks=None):
    """Fv_i = sum_{j != i, L_j > 0} L_j exp(-alpha r) (x_i - x_j) / (4 pi r^3): each
    source's flux (eq. simpint) along its direction of travel at the sink."""
    pos = np.asarray(pos, np.float64)
    lum = np.asarray(lum, np.float64)
    src = np.nonzero(lum > 0)[0]
    sinks = np.arange(pos.shape[0]) if sinks is None else np.asarray(sinks)
    out = np.zeros((sinks.size, 3))
    for q, i in enumerate(sinks):
        d = pos[i] - pos[src]
        r2 = np.sum(d * d, axis=1)
        ok = r2 > 0
        r = np.sqrt(r2[ok])
        w = lum[src][ok] * np.exp(-alpha_const * r) / (4.0 * math.pi * r2[ok] * r)
        out[q] = np.sum(w[:, None] * d[ok], axis=0)
    return out


def all_pairs_second_moment(pos, lum, alpha_const=0.0, sinks=None):
    """P_i = sum_j L_j exp(-alpha r)/(4 pi r^2) n n^T with n = (x_i - x_j)/r, as
    (xx, yy, zz, xy, xz, yz)."""
    pos = np.asarray(pos, np.float64)
    lum = np.asarray(lum, np.float64)
    src = np.nonzero(lum > 0)[0]
    sinks = np.arange(pos.shape[0]) if sinks is None else np.asarray(sinks)
    out = np.zeros((sinks.size, 6))
    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    for q, i in enumerate(sinks):
        d = pos[i] - pos[src]
        r2 = np.sum(d * d, axis=1)
        ok = r2 > 0
        r = np.sqrt(r2[ok])
        n = d[ok] / r[:, None]
        w = lum[src][ok] * np.exp(-alpha_const * r) / (4.0 * math.pi * r2[ok])
        out[q] = [np.sum(w * n[:, a] * n[:, b]) for a, b in pairs]
    return out


def fibonacci_sphere(m, radius, centre):
    """m points on a sphere by the golden-angle spiral."""
    k = np.arange(m) + 0.5
    z = 1.0 - 2.0 * k / m
    phi = math.pi * (3.0 - math.sqrt(5.0)) * k
    s = np.sqrt(1.0 - z * z)
    u = np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)
    return np.asarray(centre) + radius * u


def shell_flux(r, R, L):
    """Flux at radius r inside an emitting, optically thin shell of radius R
    and total luminosity L: (L / (8 pi R r)) ln((R + r)/(R - r)), which tends
    to L / (4 pi R^2) at the centre."""
    r = np.asarray(r, np.float64)
    out = np.empty_like(r)
    small = r < 1e-8 * R
    rr = r[~small]
    out[~small] = L / (8.0 * math.pi * R * rr) * np.log((R + rr) / (R - rr))
    out[small] = L / (4.0 * math.pi * R * R)
    return out


def path_keys(pos, lo, hi):
    """63-level path keys by repeated midpoint narrowing along the level axes
    (longest current width, ties to the lowest axis), vectorised numpy."""
    pos = np.asarray(pos, np.float64)
    n = pos.shape[0]
    clo = np.tile(np.asarray(lo, np.float64), (n, 1))
    chi = np.tile(np.asarray(hi, np.float64), (n, 1))
    w = np.asarray(hi, np.float64) - np.asarray(lo, np.float64)
    key = np.zeros(n, np.uint64)
    for d in range(63):
        a = int(np.argmax(w))
        w[a] *= 0.5
        s = 0.5 * (clo[:, a] + chi[:, a])
        up = pos[:, a] >= s
        key |= up.astype(np.uint64) << np.uint64(62 - d)
        clo[up, a] = s[up]
        chi[~up, a] = s[~up]
    return key


def walk_up_tau(nodes, sink_leaf, src_cell, p0, p1):
    """Optical depth with refinement never triggered (tau_ref = infinity):
    the ray walks up from the sink's bucket S and from the source cell C to
    their meeting cell A.  A point of the ray inside C uses C's average; any
    other point uses the average of the deepest cell that holds both the
    point's bucket and S (on S's side of A's plane) or C (on C's side).
    Brute force over all buckets crossed by the segment."""
    def ancestors(k):
        out = []
        while k >= 0:
            out.append(k)
            k = nodes[k]["parent"]
        return out

    anc_S = ancestors(sink_leaf)
    anc_C = ancestors(src_cell)
    lv = [k for k, nd in enumerate(nodes) if nd["children"] is None]
    lo = np.array([nodes[k]["lo"] for k in lv])
    hi = np.array([nodes[k]["hi"] for k in lv])
    ls = segment_box_lengths(np.asarray(p0, float), np.asarray(p1, float), lo, hi)
    tau = 0.0
    for k, l in zip(lv, ls):
        if l <= 0:
            continue
        anc_k = ancestors(k)
        if src_cell in anc_k:  # the bucket lies inside the source cell
            cell = src_cell
        else:
            sk = set(anc_k)
            dS = next(a for a in anc_S if a in sk)
            dC = next(a for a in anc_C if a in sk)
            # the meeting cell of S and C is an ancestor of both candidates;
            # the deeper of the two is on the bucket's side
            cell = dS if nodes[dS]["depth"] > nodes[dC]["depth"] else dC
        tau += nodes[cell]["alpha"] * l
    return tau
