"""Pins of the oracle's blocksize-search rules (Sections 3.3, 3.6, 3.7)."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import tuner

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_pgrid_matches_paper_example():
    g = json.load(open(os.path.join(GOLDEN, "pgrid_paper_example.json")))
    for S, expect in zip(g["S"], g["lists"]):
        assert oracle.pgrid(S, g["P"]) == expect
    for P, nC in g["nC_by_P"].items():
        assert len(oracle.pgrid_candidates(200, 200, 800, int(P))) == nC
        assert len(oracle.pgrid_candidates(300, 300, 800, int(P))) == nC
        assert len(oracle.pgrid_candidates(250, 250, 1500, int(P))) == nC


def test_gap_matches_table5_percentages():
    g = json.load(open(os.path.join(GOLDEN, "table5_gap.json")))
    for row in g["rows"]:
        pct = 100.0 * oracle.gap(row["min_time"], row["actual_time"])
        assert round(pct, 1) == row["gap_percent"], row


def test_selection_hand_cases():
    # One node, two cores (= replicates), three candidates (ids 10, 11, 12).
    t = [[[3.0, 1.0, 2.0],
          [2.0, 5.0, 0.5]]]
    ids = [[10, 11, 12]]
    # Stage 1: core 0 -> id 11 (1.0), core 1 -> id 12 (0.5).
    assert oracle.select_block(t, ids, "min") == (12, 0.5)     # Eq. 1
    assert oracle.select_block(t, ids, "worst") == (11, 1.0)   # Eq. 2
    # Eq. 3: mean 0.75; both at distance 0.25 -> lowest core wins.
    assert oracle.select_block(t, ids, "avg") == (11, 1.0)
    assert oracle.select_block(t, ids, "ob") == (12, 0.5)


def test_selection_three_stages_two_nodes():
    # Node 0 owns ids 0,1; node 1 owns ids 2,3; three cores each.
    t = [[[4.0, 5.0], [6.0, 5.5], [4.5, 7.0]],
         [[5.2, 3.0], [5.1, 9.0], [8.0, 4.9]]]
    ids = [[0, 1], [2, 3]]
    # Stage 1 node 0: (id0 4.0), (id1 5.5), (id0 4.5); node 1: (id3 3.0), (id2 5.1), (id3 4.9).
    # MWMB: node 0 worst = id1 5.5, node 1 worst = id2 5.1 -> stage 3 picks id2.
    assert oracle.select_block(t, ids, "worst") == (2, 5.1)
    # MMMB: node 0 -> id0 4.0, node 1 -> id3 3.0 -> id3.
    assert oracle.select_block(t, ids, "min") == (3, 3.0)
    # MAMB: node 0 mean 4.667 -> 4.5 (id0); node 1 mean 4.333 -> 4.9 (id3) -> id0 4.5.
    assert oracle.select_block(t, ids, "avg") == (0, 4.5)
    # OB: global min 3.0 -> id3.
    assert oracle.select_block(t, ids, "ob") == (3, 3.0)


def _brute(t, ids, policy):
    """Enumerate candidate answers directly from the equations' definitions."""
    if policy == "ob":
        entries = [(v, i, k, j) for i, tab in enumerate(t) for k, row in enumerate(tab) for j, v in enumerate(row)]
        v, i, k, j = min(entries)
        return ids[i][j], v
    per_node = []
    for i, tab in enumerate(t):
        wins = []
        for k, row in enumerate(tab):
            j = min(range(len(row)), key=lambda jj: (row[jj], jj))
            wins.append((row[j], k, j))
        if policy == "min":
            v, k, j = min(wins, key=lambda w: (w[0], w[1]))
        elif policy == "worst":
            v, k, j = max(wins, key=lambda w: (w[0], -w[1]))
        else:
            mean = sum(w[0] for w in wins) / len(wins)
            v, k, j = min(wins, key=lambda w: (abs(w[0] - mean), w[1]))
        per_node.append((v, i, ids[i][j]))
    v, i, cid = min(per_node)
    return cid, v


@pytest.mark.parametrize("policy", tuner.POLICIES)
def test_selection_vs_brute_force(policy):
    rng = np.random.default_rng(7)
    for trial in range(200):
        nn = int(rng.integers(1, 4))
        nk = int(rng.integers(1, 5))
        nc = int(rng.integers(1, 6))
        # Small integer times make ties frequent.
        t = rng.integers(1, 6, size=(nn, nk, nc)).astype(float).tolist()
        ids = [list(range(i * nc, (i + 1) * nc)) for i in range(nn)]
        assert oracle.select_block(t, ids, policy) == _brute(t, ids, policy), (trial, t)
