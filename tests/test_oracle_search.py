"""Pins of the oracle's serial IDA* and Budgeted Tree Search.

Optimal costs against breadth-first distances (8-puzzle, exhaustive table) and
against brute-force search with a zero heuristic (cube); path validity;
admissibility of min(floor(net), Manhattan); the BTS growth property.
"""
import numpy as np
import pytest

import oracle as O
import synth


@pytest.fixture(scope="module")
def bfs():
    d, _ = O.bfs8()
    return d


def _rank(s):
    return O.lib().orc_perm9_rank(np.ascontiguousarray(s, dtype=np.uint8).ctypes.data)


def _follow(domain, start, path):
    s = np.array(start, dtype=np.uint8)
    for m in path:
        s = O.apply(domain, s, m)
        assert s is not None
    return s


def test_ida_manhattan_costs_equal_bfs_distances(bfs):
    st = synth.stp3_instances(100)
    for s in st:
        r = O.ida(O.STP3, s, hkind=O.H_MD)
        assert r["status"] == 1
        assert r["cost"] == bfs[_rank(s)]
        assert len(r["path"]) == r["cost"]
        assert np.array_equal(_follow(O.STP3, s, r["path"]), O.goal(O.STP3))


def test_ida_with_net_min_manhattan_is_optimal(bfs, net_files):
    net = O.Net(net_files["stp3_small"])
    allst = O.all8()
    y = net.forward(allst)
    h = net.h(y, 0, classic=O.manhattan(O.STP3, allst))
    ranks = np.array([_rank(s) for s in allst])
    table = np.zeros(362880, dtype=np.int32)
    table[ranks] = h
    assert np.all(h <= bfs[ranks])  # admissible on every state
    for s in synth.stp3_instances(100):
        r = O.ida(O.STP3, s, hkind=O.H_TABLE8, table8=table)
        assert r["cost"] == bfs[_rank(s)]


def test_ida_iteration_bounds_increase_and_complete_final_counts_dominate(bfs):
    for s in synth.stp3_instances(20):
        a = O.ida(O.STP3, s, hkind=O.H_MD)
        b = O.ida(O.STP3, s, hkind=O.H_MD, complete_final=True)
        assert [i["bound"] for i in a["iters"]] == [i["bound"] for i in b["iters"]]
        bounds = [i["bound"] for i in a["iters"]]
        assert all(x < y for x, y in zip(bounds, bounds[1:]))
        for x, y in zip(a["iters"][:-1], b["iters"][:-1]):
            assert (x["expanded"], x["generated"]) == (y["expanded"], y["generated"])
        assert a["iters"][-1]["expanded"] <= b["iters"][-1]["expanded"]
        assert b["cost"] == a["cost"]


def test_rc_corner_pdb_ida_matches_brute_force():
    tab, _ = O.corner_pdb(4)
    mv = synth.rc_walk_moves_array(synth.config_seeds(8, 12), length_base=2, length_span=4)
    st = O.apply_moves(O.RUBIK, mv)
    for s, m in zip(st, mv):
        a = O.ida(O.RUBIK, s, hkind=O.H_PDB, pdb=tab, pdb_k=4)
        b = O.ida(O.RUBIK, s, hkind=O.H_ZERO)
        assert a["cost"] == b["cost"] <= (m >= 0).sum()
        assert np.array_equal(_follow(O.RUBIK, s, a["path"]), O.goal(O.RUBIK))


def test_stp4_walk_costs_respect_parity_and_length():
    st = synth.stp_walks(4, range(10), lengths=30)
    for s in st:
        r = O.ida(O.STP4, s, hkind=O.H_MD)
        assert r["status"] == 1 and r["cost"] <= 30 and r["cost"] % 2 == 0


def test_bts_finds_optimal_costs(bfs):
    for s in synth.stp3_instances(40):
        for b0 in (1, 50, 10000):
            r = O.bts(O.STP3, s, hkind=O.H_MD, b0=b0)
            assert r["status"] == 1 and r["cost"] == bfs[_rank(s)]
            assert np.array_equal(_follow(O.STP3, s, r["path"]), O.goal(O.STP3))


def test_bts_respects_its_limits_and_finds_ida_costs_on_stp4():
    # growth of the accepted iterations is pinned in test_oracle_bts.py
    st = synth.stp_walks(4, range(6), lengths=44)
    for s in st:
        r = O.bts(O.STP4, s, hkind=O.H_MD, b0=1, c1=2, c2=8)
        assert r["status"] == 1
        it = r["iters"]
        # every limited search respects its limit when it reports completion
        for i in it:
            if i["limit"] >= 0 and i["complete"]:
                assert i["expanded"] <= i["limit"]
            if not i["complete"]:
                assert i["expanded"] == i["limit"]
        ida = O.ida(O.STP4, s, hkind=O.H_MD)
        assert r["cost"] == ida["cost"]


def _table8(values_by_state):
    allst = O.all8()
    ranks = np.array([O.lib().orc_perm9_rank(np.ascontiguousarray(s).ctypes.data) for s in allst])
    t = np.zeros(362880, dtype=np.float32)
    t[ranks] = values_by_state
    return t, ranks


def test_real_valued_search_reduces_to_integer_search():
    """With integer values in the real-valued table, the real-valued IDA* takes
    exactly the integer search's iterations, and BTS reaches the same cost."""
    allst = O.all8()
    md = O.manhattan(0, allst)
    tf, ranks = _table8(md.astype(np.float32))
    ti = np.zeros(362880, dtype=np.int32)
    ti[ranks] = md
    for s in synth.stp3_instances(20):
        a = O.ida_real(s, tf, complete_final=True)
        b = O.ida(0, s, hkind=O.H_TABLE8, table8=ti, complete_final=True)
        assert a["cost"] == b["cost"]
        assert [(i["bound"], i["expanded"], i["generated"]) for i in a["iters"]] == \
               [(float(i["bound"]), i["expanded"], i["generated"]) for i in b["iters"]]
        # BTS bisects over real bounds (midpoints need not be integers), so only
        # the outcome and the counts at integer probes are shared
        c = O.bts_real(s, tf, b0=50)
        d = O.bts(0, s, hkind=O.H_TABLE8, table8=ti, b0=50)
        assert c["cost"] == d["cost"]
        at_int = {i["bound"]: i["expanded"] for i in d["iters"] if i["complete"]}
        for i in c["iters"]:
            if i["complete"] and i["bound"] == int(i["bound"]) and i["bound"] in at_int:
                assert i["expanded"] == at_int[i["bound"]]


def test_real_valued_admissible_heuristic_is_optimal():
    """h = max(0, MD/2 - 1/4) is admissible and not integer: IDA* and BTS find
    the breadth-first distance; IDA*'s bounds rise strictly and need more
    iterations than with Manhattan distance."""
    allst = O.all8()
    md = O.manhattan(0, allst)
    tf, _ = _table8(np.maximum(0.0, 0.5 * md - 0.25).astype(np.float32))
    bfs, _ = O.bfs8()
    for s in synth.stp3_instances(20):
        opt = bfs[O.lib().orc_perm9_rank(np.ascontiguousarray(s).ctypes.data)]
        a = O.ida_real(s, tf)
        assert a["cost"] == opt
        bounds = [i["bound"] for i in a["iters"]]
        assert all(x < y for x, y in zip(bounds, bounds[1:]))
        assert len(bounds) > len(O.ida(0, s, hkind=O.H_MD)["iters"])
        assert O.bts_real(s, tf, b0=100)["cost"] == opt
