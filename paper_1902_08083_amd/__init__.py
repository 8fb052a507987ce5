"""MI355X (gfx950) implementation of the TREVR per-sink radiation field.

Grond, Woods, Wadsley & Couchman (2019), "TREVR: A general N log^2 N
radiative transfer algorithm".  The computation runs in ``libtrevr.so``
(hand-written HIP); this package holds its Python binding and the seeded
synthetic workload generators.
"""
NODE_F_FIELDS = (
    "lo0", "lo1", "lo2", "hi0", "hi1", "hi2", "split", "A", "B", "SL",
    "SLx0", "SLx1", "SLx2", "alpha", "alpha_min", "alpha_max", "dalpha",
    "xl0", "xl1", "xl2", "lc", "lfar",
)
NODE_I_FIELDS = ("first", "count", "depth", "leaf", "parent", "right", "skip", "axis")

from .trevr import (  # noqa: E402
    ADJ_AUTO, ADJ_RECOMPUTE, ADJ_STORE, COUNTER_FIELDS, BatchedPlan, Tree, TrevrError, TrevrFlux,
    TrevrNotBuilt, autotune, build_tree, compute_flux, compute_flux_adjoint, flux,
    ionisation_equilibrium, ionisation_update, lib, sum_counters,
)

__all__ = ["ADJ_AUTO", "ADJ_RECOMPUTE", "ADJ_STORE", "BatchedPlan", "autotune", "Tree",
           "TrevrError", "TrevrFlux", "TrevrNotBuilt", "build_tree", "compute_flux",
           "compute_flux_adjoint", "flux", "ionisation_equilibrium", "ionisation_update", "lib",
           "sum_counters", "COUNTER_FIELDS", "NODE_F_FIELDS", "NODE_I_FIELDS"]
