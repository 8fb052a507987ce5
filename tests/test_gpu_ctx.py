"""GPU: the paper-context particle set (64^3 gas + 64^3 stars, Sec. 3.1.1,
App. A; theta_open 0.75, tau_ref 0.1) with the gas as sinks.  A seeded
2048-sink sample is checked against the oracle (binary32 mirror): counters
identical, flux within 1e-5.  The mean rays and pieces per gas particle are
written to ctx_counts.json in the run's output folder beside the paper's figures (about 200
rays, Sec. 3.1.2, and 850 segments, Sec. 3.1.3, per element) as context: the
paper's glass is replaced by a jittered lattice."""
import json
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

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_ctx_counts_and_parity():
    print("ctx lattice 64^3 + 64^3", flush=True)
    sys.stdout.flush()
    w = W.ctx_lattice()
    n = w["n_gas"]
    d = lambda k: torch.as_tensor(w[k], device="cuda")  # noqa: E731
    t = P.build_tree(d("pos"), d("rho"), d("kappa"), d("lum"), d("mass"), w["box_lo"],
                     w["box_hi"], w["bucket_size"])
    sinks = torch.arange(n, dtype=torch.int32, device="cuda")
    F, C = t.flux(w["theta"], w["tau_ref"], sinks=sinks, counters=True)
    F, C = F.double().cpu().numpy(), C.cpu().numpy().astype(np.int64)
    assert np.all(np.isfinite(F)) and np.all(F > 0)
    f64 = lambda a: np.asarray(a, np.float64)  # noqa: E731
    o = OracleTree(f64(w["pos"]), f64(w["rho"]), f64(w["kappa"]), f64(w["lum"]), f64(w["mass"]),
                   w["box_lo"], w["box_hi"], w["bucket_size"], mirror32=True)
    sample = np.sort(np.random.default_rng(17).choice(n, size=2048, replace=False))
    Fo, Co = o.flux(w["theta"], w["tau_ref"], sinks=sample, nthreads=min(16, os.cpu_count() or 1))
    rel = np.abs(F[sample] - Fo) / Fo
    assert rel.max() <= 1e-5, rel.max()
    assert np.array_equal(C[sample], Co)
    rep = {"workload": w["name"], "elements": n, "sources": n, "theta_open": w["theta"],
           "tau_ref": w["tau_ref"], "density_contrast": [1 / w["det_max"], 1 / w["det_min"]],
           "rays_per_element": float(C[:, 1].mean()),
           "single_particle_rays_per_element": float(C[:, 2].mean()),
           "segments_per_element": float(C[:, 3].mean()),
           "cells_tested_per_element": float(C[:, 0].mean()),
           "paper": {"rays_per_element": 200, "segments_per_element": 850,
                     "note": "64^3 perturbed glass, theta 0.75, tau_ref 0.1 (Sec. 3.1.2-3.1.3)"}}
    print(json.dumps(rep), flush=True)
    os.makedirs(os.path.join(ROOT, "gpurun_out"), exist_ok=True)
    with open(os.path.join(ROOT, "gpurun_out", "ctx_counts.json"), "w") as f:
        json.dump(rep, f, indent=1)
