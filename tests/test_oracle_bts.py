"""Pins of the oracle's Budgeted Tree Search (orc_bts, orc_bts_real) against
what the paper states about BTS and what brute force fixes.

* Background (search algorithms): BTS is IDA* when the iterations grow by a
  suitable constant factor.  With h = 0 on the cube the tree grows about 13x
  per bound; with c2 = 16 every bound from h(root) + 1 (Batch BTS
  enhancements: the first bound) is accepted in one probe, so BTS takes
  exactly IDA*'s iterations after the first, with the closed-form counts.
* Batch BTS enhancements: the node budget grows exponentially, and the
  worst-case overhead is O(N log C*).  A real-valued heuristic with distinct
  fractional parts on every state (h = max(0, MD - 1 + u_s), u_s distinct in
  [0, 1)) is IDA*'s worst case: nearly every bound adds a handful of nodes.
  BTS's budgets must grow by at least c1 per acceptance and its total work
  must stay within a small multiple of N log2 C*, far below IDA*'s.
* Every probe, complete or exceeded, is checked against a brute-force count of
  the cost-bounded tree written here (a plain stack over the tree, capped at
  the probe's limit).
A BTS that degenerates to IDA*, never bisects, or accepts an iteration that
did not reach c1 times the budget fails one of these.
"""
import numpy as np
import pytest

import oracle as O
import synth

CUBE_LEVELS = [1, 18, 243, 3240, 43254, 577368]  # canonical sequences of each length


def test_bts_equals_ida_when_the_tree_grows_geometrically():
    starts = O.apply_moves(2, synth.rc_walk_moves_array([31, 32, 33], lengths=4))
    for s in starts:
        ida = O.ida(O.RUBIK, s, hkind=O.H_ZERO, complete_final=True)
        bts = O.bts(O.RUBIK, s, hkind=O.H_ZERO, b0=2, c1=2, c2=16)
        cost = ida["cost"]
        assert bts["cost"] == cost and cost >= 2
        # IDA* starts at h(root) = 0; BTS at h(root) + 1 and then follows it bound for bound
        assert [i["bound"] for i in ida["iters"]] == list(range(cost + 1))
        assert [(i["bound"], i["expanded"], i["generated"], i["complete"]) for i in bts["iters"]] == \
               [(i["bound"], i["expanded"], i["generated"], 1) for i in ida["iters"][1:]]
        for i in bts["iters"][:-1]:  # below the optimum every node up to the bound is expanded
            assert i["expanded"] == sum(CUBE_LEVELS[:i["bound"] + 1])


# ------------------------------------------------- slow-growth real-valued h
def _distinct_fraction_table(seed=77):
    allst = O.all8()
    md = O.manhattan(0, allst)
    u = np.random.default_rng(seed).permutation(allst.shape[0]) / allst.shape[0]
    h = np.where(md == 0, 0.0, np.maximum(0.0, md - 1 + u)).astype(np.float32)
    table = np.zeros(362880, dtype=np.float32)
    table[O.perm9_rank(allst)] = h
    hmap = {bytes(s): float(v) for s, v in zip(allst.astype(np.uint8), h)}
    return table, hmap


GOAL8 = bytes(range(9))


def _tree_count(start, hmap, bound, cap):
    """Nodes expanded by a cost-bounded DFS at `bound` (f = g + h <= bound, the
    goal is not expanded, children exclude the parent's inverse move), counting
    stops at cap + 1."""
    n = 0
    stack = [(bytes(start), 0, -1)]
    while stack:
        s, g, prev = stack.pop()
        if g + hmap[s] > bound or s == GOAL8:
            continue
        n += 1
        if n > cap:
            return n
        b = s.index(0)
        r, c = divmod(b, 3)
        for a, (dr, dc) in enumerate(((-1, 0), (0, -1), (0, 1), (1, 0))):  # up, left, right, down
            if prev >= 0 and a == 3 - prev:
                continue
            rr, cc = r + dr, c + dc
            if 0 <= rr < 3 and 0 <= cc < 3:
                t = bytearray(s)
                t[b], t[rr * 3 + cc] = t[rr * 3 + cc], 0
                stack.append((bytes(t), g + 1, a))
    return n


@pytest.fixture(scope="module")
def slow_h():
    return _distinct_fraction_table()


def test_bts_probes_match_brute_force_tree_counts(slow_h):
    table, hmap = slow_h
    bfs, _ = O.bfs8()
    for s in synth.stp_walks(3, [0, 2, 6], lengths=26):
        r = O.bts_real(s, table, b0=10, c1=2, c2=8)
        assert r["status"] == 1 and r["cost"] == bfs[O.perm9_rank(s[None])[0]]
        for i in r["iters"]:
            lim = i["limit"] if i["limit"] >= 0 else 10 ** 9
            cnt = _tree_count(s, hmap, i["bound"], lim)
            if i["complete"]:
                assert cnt <= lim and i["expanded"] == cnt
            else:  # exceeded: the tree really is larger than the limit, and the search stopped at it
                assert cnt > lim and i["expanded"] == lim


def test_bts_budget_grows_geometrically_and_total_work_is_n_log_c(slow_h):
    table, _ = slow_h
    c1, c2 = 2, 8
    checked = 0
    for s in synth.stp_walks(3, range(40), lengths=40):
        ida = O.ida_real(s, table, complete_final=True, max_iters=5000)
        N = ida["iters"][-1]["expanded"]
        if N < 2000:
            continue
        bts = O.bts_real(s, table, b0=10, c1=c1, c2=c2)
        assert bts["cost"] == ida["cost"]
        limits = []
        for i in bts["iters"]:
            if i["limit"] >= 0 and (not limits or i["limit"] != limits[-1]):
                limits.append(i["limit"])
        # a new budget only after an accepted iteration of at least c1 times the last one
        assert all(b >= c1 * a for a, b in zip(limits, limits[1:])), limits
        total_bts = sum(i["expanded"] for i in bts["iters"])
        total_ida = sum(i["expanded"] for i in ida["iters"])
        assert total_bts <= 4 * c2 * N * np.log2(ida["cost"] + 1), (total_bts, N)
        # IDA* pays about N squared over its thousands of bounds (8.6x to 111x here)
        assert total_ida >= 5 * total_bts, (total_ida, total_bts)
        checked += 1
    assert checked >= 3


@pytest.mark.parametrize("b0", [1, 10000])
def test_integer_bts_probes_match_brute_force_tree_counts(b0):
    """The integer BTS with Manhattan distance: every probe's count equals the
    brute-force tree size (or the tree exceeds the probe's limit), budgets grow
    by at least c1 per acceptance, and the cost is the breadth-first distance."""
    allst = O.all8()
    hmap = {bytes(s): float(v) for s, v in zip(allst.astype(np.uint8), O.manhattan(0, allst))}
    bfs, _ = O.bfs8()
    for s in synth.stp3_instances(8):
        r = O.bts(O.STP3, s, hkind=O.H_MD, b0=b0)
        assert r["status"] == 1 and r["cost"] == bfs[O.perm9_rank(s[None])[0]]
        limits = []
        for i in r["iters"]:
            lim = i["limit"] if i["limit"] >= 0 else 10 ** 9
            cnt = _tree_count(s, hmap, i["bound"], lim)
            if i["complete"]:
                assert cnt <= lim and i["expanded"] == cnt
            else:
                assert cnt > lim and i["expanded"] == lim
            if i["limit"] >= 0 and (not limits or i["limit"] != limits[-1]):
                limits.append(i["limit"])
        assert all(b >= 2 * a for a, b in zip(limits, limits[1:]))
