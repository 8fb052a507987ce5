"""Batched boxes: 64 independent boxes of uneven size (2^12..2^17 particles,
uniform or log-normal media, 1..512 sources, box optical depth 0.1..20) as
one forest, one persistent flux launch captured in a HIP graph and replayed;
the launch shape picked by the autotuner."""
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


def test_batched_graph_replays_match_eager_and_oracle():
    print("batched c4: build + autotune", flush=True)
    boxes = W.c4()
    plan = P.BatchedPlan(boxes, candidates=[(3, 4, 64), (2, 4, 128), (4, 2, 64)])
    eager = plan.eager().clone()
    plan.capture()
    for rep in range(3):
        F = plan.replay().clone()
        torch.cuda.synchronize()
        assert torch.equal(F, eager), "replay %d differs from the eager launch" % rep
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
    Fb = plan.per_box(eager)
    sizes = [b["pos"].shape[0] for b in boxes]
    check = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 31, 50})
    for b in check:
        bx = boxes[b]
        f64 = lambda a: np.asarray(a, np.float64)  # noqa: E731
        o = OracleTree(f64(bx["pos"]), f64(bx["rho"]), f64(bx["kappa"]), f64(bx["lum"]),
                       f64(bx["mass"]), bucket_size=8, mirror32=True)
        Fo, _ = o.flux(0.75, 0.1, nthreads=NTHREADS)
        g = Fb[b].cpu().numpy().astype(np.float64)
        rel = np.abs(g - Fo) / np.where(Fo > 0, Fo, 1.0)
        print("box %d (%d particles): max rel %.2e" % (b, sizes[b], rel.max()), flush=True)
        assert rel.max() <= 1e-5


def test_autotune_keeps_results_identical():
    w = W._pack("tune", *W.lognormal_box(1 << 14, 0, 10.0, 3, all_sources=True), prec="f32")
    t = P.build_tree(*[torch.as_tensor(w[k], device="cuda") for k in
                       ("pos", "rho", "kappa", "lum", "mass")])
    ref = t.flux(0.75, 0.1).clone()
    best = P.autotune(t, 0.75, 0.1, candidates=[(1, 1, 64), (2, 4, 256), (8, 2, 128)], reps=1)
    assert tuple(best["launch"]) in [(1, 1, 64), (2, 4, 256), (8, 2, 128)]
    # every register-budget variant of the walk kernel (3..8 waves per SIMD)
    for cand in [(1, 1, 64), (2, 4, 256), (8, 2, 128), (3, 4, 4096), (5, 4, 64), (6, 4, 64),
                 (8, 4, 64), (16, 2, 128)]:
        t.set_launch(*cand)
        assert torch.equal(t.flux(0.75, 0.1), ref), cand


def test_autotune_json_cache(tmp_path):
    """A tuning is written to the JSON cache, and a later process (here: an
    emptied in-memory cache) takes the stored launch without timing; a
    candidate list without the stored launch tunes again."""
    w = W._pack("tunecache", *W.lognormal_box(1 << 13, 0, 10.0, 5, all_sources=True), prec="f32")
    t = P.build_tree(*[torch.as_tensor(w[k], device="cuda") for k in
                       ("pos", "rho", "kappa", "lum", "mass")])
    path = str(tmp_path / "tune.json")
    cands = [(1, 1, 64), (2, 4, 128), (4, 4, 64)]
    first = P.autotune(t, 0.75, 0.1, candidates=cands, reps=1, cache_path=path)
    assert first["source"] == "timed"
    stored = P.trevr.tune_cache_load(path)
    assert len(stored) == 1
    (key, rec), = stored.items()
    assert tuple(rec["launch"]) == tuple(first["launch"]) and len(rec["table"]) == 3
    P.trevr._TUNE_CACHE.clear()
    t.set_launch(1, 1, 64)
    again = P.autotune(t, 0.75, 0.1, candidates=cands, reps=1, cache_path=path)
    assert again["source"] == "file" and tuple(again["launch"]) == tuple(first["launch"])
    lo = t.get_launch()
    assert (lo["blocks_per_cu"], lo["waves_per_block"], lo["chunk"]) == tuple(first["launch"])
    P.trevr._TUNE_CACHE.clear()
    other = [c for c in [(3, 4, 64), (2, 2, 64)] if c != tuple(first["launch"])]
    third = P.autotune(t, 0.75, 0.1, candidates=other, reps=1, cache_path=path)
    assert third["source"] == "timed" and tuple(third["launch"]) in other
