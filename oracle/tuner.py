"""Reference rules of the paper's blocksize search (Section 3.2-3.3, 3.7).

TEST INFRASTRUCTURE ONLY (see the package docstring). Pure functions of a
timing table; no timing is done here.

Selection (Section 3.3). Nodes i = 0..N-1 each own a disjoint list of
candidate blocks; every core k of node i times every candidate of its node,
in the same order, giving t[i][k][j] (time of nI iterations of candidate j on
core k).

* Stage 1: each core keeps its fastest candidate,
  b_{k,i} = argmin_j t[i][k][j].
* Stage 2 (per node), over the stage-1 winners and their times
  T_{k,i} = t[i][k][b_{k,i}]:
  - "min"   (Eq. 1, MMMB): the winner with the smallest T_{k,i};
  - "worst" (Eq. 2, MWMB): the winner with the largest T_{k,i};
  - "avg"   (Eq. 3, MAMB): the winner whose T_{k,i} is closest to the mean
    of the node's T_{k,i} (Eq. 3's printed sum index is garbled; this is the
    reading taken).
* Stage 3: among the per-node choices, the one with the smallest stage-2
  time (recorded times, no re-timing).

"ob" (Original Block) ignores the node/core structure: the single fastest
(process, candidate) entry of the whole table.

Eqs. 1-3 are written with min/max over times but name a block; they are read
as argmin/argmax. Ties go to the lowest node, then core, then candidate index.
"""
from __future__ import annotations

from typing import Sequence

POLICIES = ("min", "worst", "avg", "ob")


def _argmin(vals: Sequence[float]) -> int:
    best = 0
    for i in range(1, len(vals)):
        if vals[i] < vals[best]:
            best = i
    return best


def _argmax(vals: Sequence[float]) -> int:
    best = 0
    for i in range(1, len(vals)):
        if vals[i] > vals[best]:
            best = i
    return best


def select_block(tables, candidate_ids, policy: str = "worst"):
    """Return (chosen candidate id, its selection-phase time = MinTime).

    ``tables[i]`` is node i's [cores][candidates] list of times;
    ``candidate_ids[i][j]`` is the global id of node i's j-th candidate.
    A single GPU is one node whose "cores" are repeated passes over the same
    candidate list.
    """
    if policy not in POLICIES:
        raise ValueError(f"unknown policy {policy!r}")
    if policy == "ob":
        best = None
        for i, tab in enumerate(tables):
            for k, row in enumerate(tab):
                for j, t in enumerate(row):
                    if best is None or t < best[0]:
                        best = (t, candidate_ids[i][j])
        return best[1], best[0]

    node_choice = []  # (time, candidate id) per node
    for i, tab in enumerate(tables):
        # Stage 1: each core's fastest candidate.
        winners = [_argmin(row) for row in tab]
        times = [tab[k][winners[k]] for k in range(len(tab))]
        # Stage 2: one of the core winners, by the policy.
        if policy == "min":
            k = _argmin(times)
        elif policy == "worst":
            k = _argmax(times)
        else:
            mean = sum(times) / len(times)
            k = _argmin([abs(t - mean) for t in times])
        node_choice.append((times[k], candidate_ids[i][winners[k]]))
    # Stage 3: the fastest node choice.
    i = _argmin([t for t, _ in node_choice])
    return node_choice[i][1], node_choice[i][0]


def pgrid(S: int, P: int):
    """Section 3.7's per-dimension list for a dimension of size S cut in P
    parts: 1 + j*S/(P-1) for j = 0..P-1. The division is read as floor, the
    last entry is clamped to S (the paper prints 200, not 201, for S=200,
    P=5), and repeated values (only when S < P-1) are kept once."""
    if S < 1 or P < 2:
        raise ValueError("need S >= 1 and P >= 2")
    out = []
    for j in range(P):
        b = min(S, 1 + (j * S) // (P - 1))
        if not out or out[-1] != b:
            out.append(b)
    return out


def pgrid_candidates(Si: int, Sj: int, Sk: int, P: int):
    """All (bi, bj, bk) of the three lists, bi fastest-varying last; nC is the
    product of the list lengths (P^3 when every S >= P-1)."""
    return [(a, b, c) for a in pgrid(Si, P) for b in pgrid(Sj, P) for c in pgrid(Sk, P)]


def gap(min_time: float, actual_time: float) -> float:
    """Section 3.6's quality measure: the relative difference between the
    verification-phase time (ActualTime) and the selection-phase time
    (MinTime), (ActualTime - MinTime) / MinTime. Near zero means the chosen
    block behaves in production as it did when it was selected."""
    return (actual_time - min_time) / min_time
