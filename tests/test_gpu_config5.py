"""The learned 15-puzzle heuristic at the configuration's stated scale.

10^7 training states (random walks of 0-200 moves) labelled by the paper's
classic sliding-tile heuristic, the 7-8 additive PDB, minus Manhattan distance
(Experimental Setup: the sliding-tile model learns what a PDB adds to Manhattan
distance); the config-2 network trained by the library's own kernels (BF16
operands, FP32 master weights, Adam, batch 8192) and served as
MD + max(0, floor(y - delta)) (Manhattan fallback).  The run itself is
bench.config5; this test checks its outcome against the oracle: IDA* with
Manhattan distance and with the PDB return the oracle's optimal costs, the
learned heuristic exceeds the PDB label on at most 0.5% of held-out states,
expands fewer nodes than IDA*(MD) on 20 starts and returns a longer path on at
most two of them.
"""
import json

import pytest
import torch

import bench
import oracle as O
import paper_2507_11916_amd as hb
import synth

pytestmark = pytest.mark.gpu


def test_config5_learned_heuristic_at_full_scale(tmp_path):
    r = bench.config5(hb, synth, torch, str(tmp_path), progress=lambda m: print(m, flush=True))
    tr, ho, se = r["train"], r["held_out"], r["search"]
    print("config5 result:", json.dumps(r))
    assert tr["steps"] == tr["epochs"] * 10_000_000 // 8192 and tr["epochs"] >= 2
    assert tr["loss_last"] < 0.5 * tr["loss_first"]
    assert ho["h_below_md"] == 0  # Manhattan fallback
    assert ho["over_estimate_rate_vs_pdb"] <= 0.005
    assert ho["mean_h"] > ho["mean_md"] + 1.0
    assert se["all_solved"]
    starts = synth.stp_walks(4, synth.config_seeds(5, se["starts"]), lengths=se["walk_moves"])
    for row, s in zip(se["per_start"], starts):
        o = O.ida(1, s, hkind=O.H_MD)
        assert row["cost_md"] == o["cost"] and row["cost_pdb"] == o["cost"]
        assert row["cost_learned"] >= o["cost"]
    assert len(se["cost_differs"]) <= 2
    assert se["expanded"]["learned"] < se["expanded"]["md"]
