"""The committed result files agree with themselves: the held-out ranked-plan
summary is the summary of its own per-room records (and the gaps are scored
on the full matrix, so each one is the plan's objective against the full
LP's), and the floor-plan record is a converged LP.  CPU only."""
import json
import os

import pytest

from paper_2103_14137_amd import ranker

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _load(*parts):
    with open(os.path.join(ROOT, *parts)) as f:
        return json.load(f)


def test_heldout_summary_matches_its_rooms():
    d = _load("paper_2103_14137_amd", "weights", "ranker_tower8_batchrooms_eval_heldout200.json")
    rooms = d["rooms"]
    assert len(rooms) == 200 and len({r["room"] for r in rooms}) == 200
    s = ranker.summarize(rooms, ("mlp", "area"))
    for mode in ("mlp", "area"):
        for k in ("gap_max", "gap_le_2pct", "fallback_rate", "ms_total", "speedup_vs_full"):
            assert d["summary"][mode][k] == pytest.approx(s[mode][k], rel=1e-12), (mode, k)
    assert d["summary"]["full_ms_total"] == pytest.approx(s["full_ms_total"], rel=1e-12)
    for r in rooms:
        for mode in ("mlp", "area"):
            m = r[mode]
            assert m["gap"] == pytest.approx((m["objective"] - r["full_objective"]) / r["full_objective"], abs=1e-15)
            assert m["n_kept"] <= r["K"] and (m["fell_back"] == 0 or m["n_kept"] == r["K"])


def test_floorplan_record_is_a_converged_lp():
    d = _load("profiles", "floorplan_csr_lp.json")
    c, lp = d["csr"], d["lp"]
    assert c["K"] == 20000 and c["N"] == 487652 and c["counted_launch_identical"]
    assert c["nnz"] <= c["K"] * c["N"] and c["rays"] > 0
    assert lp["converged"] and max(lp["primal_residual"], lp["dual_residual"], lp["gap"]) <= 1e-9
    assert 0 < lp["working_poses"] < c["K"] and lp["n_visible"] <= c["N"]
    assert lp["dwell_s"] <= 3.6e5 * (1 + 1e-9)
    assert d["command"].startswith("rocprofv3 ") and "bench.py --mode floorplan" in d["command"]
