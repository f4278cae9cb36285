"""Pins of the oracle's domain models against facts fixed by mathematics.

Sliding tile: the 8-puzzle's reachable half of S_9 and its known diameter;
Manhattan distance admissible and consistent; walk-parity of the state graph;
level counts of the parent-pruned tree from a blank-position recurrence.
Rubik's cube: group identities, centre and colour invariants, and the
closed-form level counts of the canonically pruned tree.
"""
import itertools

import numpy as np
import pytest

import oracle as O
import synth


def test_bfs8_reaches_half_the_permutations_with_diameter_31():
    d, n = O.bfs8()
    assert n == 181440  # 9!/2: exactly the even-parity half
    assert d.max() == 31  # known 8-puzzle diameter for a corner-blank goal
    assert (d >= 0).sum() == 181440


def test_manhattan_is_admissible_and_consistent_on_all_8puzzle_states():
    d, _ = O.bfs8()
    st = O.all8()
    md = O.manhattan(O.STP3, st)
    dist = d[O.perm9_rank(st[:2000])]
    assert np.all(md[:2000] <= dist)
    ranks = np.array([O.lib().orc_perm9_rank(s.ctypes.data) for s in st], dtype=np.int64)
    assert np.all(md <= d[ranks])
    assert np.all((md % 2) == (d[ranks] % 2))  # both change parity with every move
    # consistency: |MD(s) - MD(s')| == 1 across every edge
    for s in st[::97]:
        for m in range(4):
            c = O.apply(O.STP3, s, m)
            if c is not None:
                assert abs(int(O.manhattan(O.STP3, c)[0]) - int(O.manhattan(O.STP3, s)[0])) == 1


def test_walk_parity_and_bound():
    d, _ = O.bfs8()
    st = synth.stp3_instances(100)
    s = synth.Stream(1000)
    for i in range(100):
        L = 30 + synth.Stream(1000 + i).next() % 31
        r = O.lib().orc_perm9_rank(np.ascontiguousarray(st[i]).ctypes.data)
        assert d[r] <= L and d[r] % 2 == L % 2
    del s


def _stp_level_counts(n, depth, blank=0):
    """Number of parent-pruned move sequences of each length from a state with
    the blank at `blank`, by dynamic programming over (blank cell, previous move)."""
    moves = {0: (-1, 0), 1: (0, -1), 2: (0, 1), 3: (1, 0)}
    cnt = {(blank, -1): 1}
    out = []
    for _ in range(depth):
        nxt = {}
        for (b, prev), c in cnt.items():
            r, col = divmod(b, n)
            for m, (dr, dc) in moves.items():
                if prev >= 0 and m == 3 - prev:
                    continue
                rr, cc = r + dr, col + dc
                if 0 <= rr < n and 0 <= cc < n:
                    key = (rr * n + cc, m)
                    nxt[key] = nxt.get(key, 0) + c
        cnt = nxt
        out.append(sum(cnt.values()))
    return out


def test_stp_zero_heuristic_counts_match_level_recurrence():
    st = synth.stp_walks(4, [777], lengths=40)[0]
    r = O.ida(O.STP4, st, hkind=O.H_ZERO, max_iters=9)
    lv = _stp_level_counts(4, 10, blank=int(np.argmin(st)))
    for it in r["iters"]:
        T = it["bound"]
        assert it["expanded"] == 1 + sum(lv[:T])
        assert it["generated"] == sum(lv[:T + 1])


def _rc_level_counts(depth):
    a, b = 9, 9
    out = [18]
    for _ in range(depth - 1):
        a, b = 6 * (a + b), 9 * a + 6 * b
        out.append(a + b)
    return out


def test_rc_level_recurrence_values():
    assert _rc_level_counts(6) == [18, 243, 3240, 43254, 577368, 7706988]


def test_rc_zero_heuristic_counts_match_closed_form():
    mv = synth.rc_walk_moves([4242], lengths=12)
    st = O.apply_moves(O.RUBIK, np.array(mv, dtype=np.int8))[0]
    r = O.ida(O.RUBIK, st, hkind=O.H_ZERO, max_iters=4, node_limit=-1)
    lv = _rc_level_counts(5)
    assert [it["bound"] for it in r["iters"]] == [0, 1, 2, 3]
    for it in r["iters"]:
        T = it["bound"]
        assert it["expanded"] == 1 + sum(lv[:T])
        assert it["generated"] == sum(lv[:T + 1])


def _seq(ms):
    return O.apply_moves(O.RUBIK, np.array(ms, dtype=np.int8))[0]


def test_rc_group_identities():
    g = O.goal(O.RUBIK)
    for f in range(6):
        cw, ccw, half = 3 * f, 3 * f + 1, 3 * f + 2
        assert not np.array_equal(_seq([cw]), g)
        assert np.array_equal(_seq([cw] * 4), g)
        assert np.array_equal(_seq([cw, ccw]), g)
        assert np.array_equal(_seq([cw, cw]), _seq([half]))
        assert np.array_equal(_seq([half, half]), g)
    R, Rp, U, Up = 9, 10, 0, 1
    assert np.array_equal(_seq([R, U, Rp, Up] * 6), g)
    assert not np.array_equal(_seq([R, U, Rp, Up] * 3), g)
    cur = g
    order = None
    for k in range(1, 200):
        cur = O.apply(O.RUBIK, O.apply(O.RUBIK, cur, R), U)
        if np.array_equal(cur, g):
            order = k
            break
    assert order == 105
    # opposite faces commute, adjacent ones do not
    assert np.array_equal(_seq([0, 3]), _seq([3, 0]))
    assert not np.array_equal(_seq([0, 9]), _seq([9, 0]))


def test_rc_invariants_under_random_walks():
    mv = synth.rc_walk_moves_array(synth.config_seeds(3, 200), length_base=14, length_span=5)
    st = O.apply_moves(O.RUBIK, mv)
    for s in st:
        assert [s[9 * f + 4] for f in range(6)] == list(range(6))
        assert np.all(np.bincount(s, minlength=6) == 9)


def test_rc_u_turn_moves_front_top_row_to_left():
    # Looking down at U, a clockwise turn carries the front face's top row to
    # the left face (standard Singmaster convention).
    s = _seq([0])
    assert list(s[18:21]) == [4, 4, 4]  # L top row now shows F's colour
    assert list(s[36:39]) == [3, 3, 3]  # F top row now shows R's colour


def test_corner_pdb_size_admissible_consistent():
    k = 4
    tab, reached = O.corner_pdb(k)
    assert reached == 8 * 7 * 6 * 5 * 3 ** 4  # every placement and twist is reachable
    assert tab[O.corner_index(O.goal(O.RUBIK), k)[0]] == 0
    mv = synth.rc_walk_moves_array(synth.config_seeds(7, 300), length_base=1, length_span=8)
    st = O.apply_moves(O.RUBIK, mv)
    h = tab[O.corner_index(st, k)]
    lengths = (mv >= 0).sum(axis=1)
    assert np.all(h <= lengths)  # walk length bounds the true distance
    for s in st[:60]:
        hs = int(tab[O.corner_index(s, k)[0]])
        for m in range(18):
            c = O.apply(O.RUBIK, s, m)
            assert abs(int(tab[O.corner_index(c, k)[0]]) - hs) <= 1


def test_apply_rejects_off_board_moves():
    g = O.goal(O.STP4)
    assert O.apply(O.STP4, g, 0) is None  # blank at the top-left corner
    assert O.apply(O.STP4, g, 1) is None
    assert O.apply(O.STP4, g, 2) is not None
    assert O.apply(O.STP4, g, 3) is not None


def test_permutation_rank_is_a_bijection_on_small_sample():
    seen = set()
    for p in itertools.islice(itertools.permutations(range(9)), 5000):
        seen.add(O.lib().orc_perm9_rank(np.array(p, dtype=np.uint8).ctypes.data))
    assert len(seen) == 5000 and max(seen) < 362880


# ------------------------------------------------ 15-puzzle additive PDB
def test_additive_pdb_of_single_tiles_is_manhattan_distance():
    """A one-tile pattern with free blank moves costs exactly the tile's
    Manhattan distance, so fifteen singleton groups give MD itself."""
    spec = O.apdb([[t] for t in range(1, 16)])
    st = synth.stp_walks(4, synth.config_seeds(8, 300), lengths=200)
    np.testing.assert_array_equal(O.apdb_h(st, spec), O.manhattan(O.STP4, st))


def test_additive_pdb_counts_a_linear_conflict():
    """Tiles 1 and 2 swapped in their goal row: each is one step from home, but
    one must leave the row and come back, so the two-tile pattern costs MD + 2."""
    g = O.goal(O.STP4).copy()
    g[1], g[2] = g[2], g[1]
    spec = O.apdb([[1, 2]])
    assert O.manhattan(O.STP4, g[None])[0] == 2
    assert O.apdb_h(g[None], spec)[0] == 4


def test_additive_pdb_dominates_md_and_keeps_its_parity():
    """Each pattern's cost counts its own tiles' moves, each of which changes
    those tiles' Manhattan distance by one: h >= MD, h = MD (mod 2), and one move
    changes h by an odd amount.  (Minimised over the blank's cell the table is
    admissible but not consistent: a move can change it by 3.)"""
    spec = O.apdb([range(1, 5), range(5, 9), range(9, 13), range(13, 16)])
    st = synth.stp_walks(4, synth.config_seeds(8, 200), lengths=200)
    h, md = O.apdb_h(st, spec), O.manhattan(O.STP4, st)
    assert np.all(h >= md) and np.all((h - md) % 2 == 0)
    assert O.apdb_h(O.goal(O.STP4)[None], spec)[0] == 0
    for s in st[:60]:
        hs = O.apdb_h(s[None], spec)[0]
        for m in range(4):
            c = O.apply(O.STP4, s, m)
            if c is not None:
                assert (int(O.apdb_h(c[None], spec)[0]) - int(hs)) % 2 == 1


def test_additive_pdb_is_admissible_and_keeps_ida_optimal():
    """On short walks: h <= the optimal cost (IDA* with Manhattan distance), and
    IDA* with the additive PDB finds the same cost expanding no more nodes."""
    spec = O.apdb([range(1, 5), range(5, 9), range(9, 13), range(13, 16)])
    for s in synth.stp_walks(4, synth.config_seeds(8, 12), lengths=36):
        r_md = O.ida(O.STP4, s, hkind=O.H_MD)
        r_pd = O.ida(O.STP4, s, hkind=O.H_APDB, apdb=spec)
        assert r_md["status"] == 1 and r_pd["status"] == 1
        assert O.apdb_h(s[None], spec)[0] <= r_md["cost"]
        assert r_pd["cost"] == r_md["cost"]
        assert sum(i["expanded"] for i in r_pd["iters"]) <= sum(i["expanded"] for i in r_md["iters"])


# ------------------------------------------------ 6-tile pattern groups
@pytest.fixture(scope="module")
def group_1_6():
    return O.apdb_group_table(range(1, 7))


@pytest.mark.slow
def test_six_tile_pattern_table_pins(group_1_6):
    """The oracle's 6-tile table (0-1 breadth-first search over 16^7 dense
    codes): every placement of the six tiles is reached (16!/10!), it dominates
    the sum of its two disjoint 3-tile halves (a path for the six tiles is a
    path for each half, and its six-tile moves split between them), it has the
    parity of its tiles' Manhattan distance and lies above it, and it never
    exceeds the optimal cost of short walks."""
    ts, t = group_1_6
    assert int((t < 255).sum()) == 16 * 15 * 14 * 13 * 12 * 11
    st = synth.stp_walks(4, synth.config_seeds(9, 4000), lengths=200)
    h6 = O.apdb_group_lookup(group_1_6, st)
    h_a = O.apdb_group_lookup(O.apdb_group_table([1, 2, 3]), st)
    h_b = O.apdb_group_lookup(O.apdb_group_table([4, 5, 6]), st)
    assert np.all(h6 >= h_a + h_b) and np.any(h6 > h_a + h_b)
    where = np.argsort(st, axis=1)  # cell of each tile
    md6 = sum(np.abs(where[:, t] // 4 - t // 4) + np.abs(where[:, t] % 4 - t % 4) for t in range(1, 7))
    assert np.all(h6 >= md6) and np.all((h6 - md6) % 2 == 0)
    assert O.apdb_group_lookup(group_1_6, O.goal(O.STP4)[None])[0] == 0
    for s in synth.stp_walks(4, synth.config_seeds(9, 8), lengths=34):
        assert O.apdb_group_lookup(group_1_6, s[None])[0] <= O.ida(O.STP4, s, hkind=O.H_MD)["cost"]
