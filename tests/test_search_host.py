"""cbdfs_solve (parallel Batch IDA* / Batch BTS) against the serial oracle on
the CPU: the classic heuristic, computed directly or by the batch thread through
the batching machinery, needs no GPU.

Parity contract: for every iteration that ran to completion, (bound, expanded,
generated) equal the oracle's; costs are optimal (8-puzzle: breadth-first
distance); returned paths are valid.
"""
import numpy as np
import pytest

import oracle as O
import paper_2507_11916_amd as hb
import synth

MODES = [hb.HB_H_CLASSIC, hb.HB_H_CLASSIC_BATCHED]


def _follow(dom, start, path):
    s = np.array(start, dtype=np.uint8)
    for m in path:
        s = O.apply(dom, s, m)
        assert s is not None
    return s


def _complete_counts(iters):
    return [(i["bound"], i["expanded"], i["generated"]) for i in iters if i["complete"]]


@pytest.fixture(scope="module")
def bfs():
    d, _ = O.bfs8()
    return d


@pytest.mark.parametrize("mode", MODES)
def test_8puzzle_ida_matches_oracle(bfs, mode):
    for s in synth.stp3_instances(30):
        p = hb.default_params(batch_size=64, work_num=4, complete_final_iter=1, timeout_us=2000)
        r = hb.cbdfs_solve(0, s, combine=mode, classic=hb.HB_CLASSIC_MD, threads=4, params=p)
        o = O.ida(0, s, hkind=O.H_MD, complete_final=True)
        assert r["status"] == hb.HB_OK
        assert r["cost"] == o["cost"] == bfs[O.lib().orc_perm9_rank(np.ascontiguousarray(s).ctypes.data)]
        assert _complete_counts(r["iters"]) == _complete_counts(o["iters"])
        assert np.array_equal(_follow(0, s, r["path"]), O.goal(0))


@pytest.mark.parametrize("threads,work_num,d_init,batch,flush", [(1, 1, 0, 1, 1), (3, 2, 2, 7, 1), (8, 8, -1, 500, 1),
                                                                  (16, 3, 6, 64, 1), (8, 8, -1, 500, 2),
                                                                  (4, 4, -1, 100, 0)])
def test_stp4_counts_independent_of_parallel_shape(threads, work_num, d_init, batch, flush):
    st = synth.stp_walks(4, [11, 12, 13], lengths=44)
    for s in st:
        p = hb.default_params(batch_size=batch, work_num=work_num, d_init=d_init, timeout_us=1000,
                              flush_when_idle=flush)
        r = hb.cbdfs_solve(1, s, combine=hb.HB_H_CLASSIC_BATCHED, classic=hb.HB_CLASSIC_MD, threads=threads, params=p)
        o = O.ida(1, s, hkind=O.H_MD)
        assert r["cost"] == o["cost"]
        # every non-final iteration is complete and must match exactly
        assert _complete_counts(r["iters"]) == _complete_counts(o["iters"][:-1])
        fin_r, fin_o = r["iters"][-1], o["iters"][-1]
        assert fin_r["bound"] == fin_o["bound"] and fin_r["found"]


def test_cube_pdb_ida_matches_oracle():
    k = 4
    pdb = hb.Pdb(k, threads=4)
    tab, _ = O.corner_pdb(k)
    mv = synth.rc_walk_moves_array(synth.config_seeds(3, 8), length_base=5, length_span=3)
    st = O.apply_moves(2, mv)
    for s in st:
        p = hb.default_params(batch_size=4000, work_num=4, complete_final_iter=1)
        r = hb.cbdfs_solve(2, s, combine=hb.HB_H_CLASSIC_BATCHED, classic=hb.HB_CLASSIC_PDB, pdb=pdb, threads=8, params=p)
        o = O.ida(2, s, hkind=O.H_PDB, pdb=tab, pdb_k=k, complete_final=True)
        assert r["cost"] == o["cost"]
        assert _complete_counts(r["iters"]) == _complete_counts(o["iters"])
        assert np.array_equal(_follow(2, s, r["path"]), O.goal(2))
        assert r["generated"] / max(1, r["expanded"]) < 18


def test_stp4_additive_pdb_ida_and_bts_match_oracle():
    """Batch IDA* and Batch BTS pruning with the additive 15-puzzle PDB (the
    paper's classic sliding-tile heuristic) against the oracle's searches with
    its own table of the same tile groups: costs and per-iteration counts."""
    groups = [range(1, 5), range(5, 9), range(9, 13), range(13, 16)]
    pdb = hb.Pdb(groups=groups, threads=4)
    spec = O.apdb(groups)
    for s in synth.stp_walks(4, synth.config_seeds(2, 5), lengths=60):
        p = hb.default_params(batch_size=1000, work_num=8, complete_final_iter=1)
        r = hb.cbdfs_solve(1, s, combine=hb.HB_H_CLASSIC_BATCHED, classic=hb.HB_CLASSIC_PDB, pdb=pdb, threads=8,
                           params=p)
        o = O.ida(1, s, hkind=O.H_APDB, apdb=spec, complete_final=True)
        assert r["cost"] == o["cost"]
        assert _complete_counts(r["iters"]) == _complete_counts(o["iters"])
        assert np.array_equal(_follow(1, s, r["path"]), O.goal(1))
        p = hb.default_params(batch_size=1000, work_num=8, bts_b0=500)
        rb = hb.cbdfs_solve(1, s, combine=hb.HB_H_CLASSIC_BATCHED, classic=hb.HB_CLASSIC_PDB, pdb=pdb,
                            algo=hb.HB_BTS, threads=8, params=p)
        ob = O.bts(1, s, hkind=O.H_APDB, apdb=spec, b0=500)
        assert rb["cost"] == ob["cost"] == o["cost"]
        assert [(i["bound"], i["limit"], i["complete"]) for i in rb["iters"]] == \
               [(i["bound"], i["limit"], i["complete"]) for i in ob["iters"]]
    pdb.close()


def test_per_iteration_batch_statistics():
    """Batches and evaluations per iteration: within the totals (the initial
    tree's evaluation counts only there), each batch within the batch size,
    and no more states evaluated in an iteration than it generated."""
    s = synth.stp_walks(4, [11], lengths=44)[0]
    p = hb.default_params(batch_size=500, work_num=8)
    r = hb.cbdfs_solve(1, s, combine=hb.HB_H_CLASSIC_BATCHED, classic=hb.HB_CLASSIC_MD, threads=4, params=p)
    its = r["iters"]
    assert sum(i["batches"] for i in its) <= r["batches"] and sum(i["evals"] for i in its) <= r["evals"]
    for i in its:
        assert 0 <= i["evals"] <= i["generated"]
        assert i["batches"] * 500 >= i["evals"] and (i["evals"] > 0) == (i["batches"] > 0)
    assert its[-1]["batches"] > 0


def test_flush_mode_out_of_range_is_rejected():
    s = synth.stp_walks(4, [11], lengths=20)[0]
    r = hb.cbdfs_solve(1, s, combine=hb.HB_H_CLASSIC_BATCHED, classic=hb.HB_CLASSIC_MD, threads=2,
                       params=hb.default_params(flush_when_idle=3), raise_on_error=False)
    assert r["status"] == hb.HB_E_INVAL


def test_pdb_kind_must_match_domain():
    pdb = hb.Pdb(groups=[range(1, 5), range(5, 9), range(9, 13), range(13, 16)], threads=4)
    r = hb.cbdfs_solve(2, O.goal(2), combine=hb.HB_H_CLASSIC_BATCHED, classic=hb.HB_CLASSIC_PDB, pdb=pdb,
                       threads=2, raise_on_error=False)
    assert r["status"] == hb.HB_E_INVAL
    pdb.close()


@pytest.mark.parametrize("b0", [1, 100, 10000])
def test_bts_matches_oracle_search_sequence(bfs, b0):
    for s in synth.stp3_instances(12):
        p = hb.default_params(batch_size=64, work_num=4, bts_b0=b0)
        r = hb.cbdfs_solve(0, s, combine=hb.HB_H_CLASSIC_BATCHED, classic=hb.HB_CLASSIC_MD, algo=hb.HB_BTS,
                           threads=4, params=p)
        o = O.bts(0, s, hkind=O.H_MD, b0=b0)
        assert r["status"] == hb.HB_OK and r["cost"] == o["cost"]
        ours = [(i["bound"], i["limit"], i["complete"]) for i in r["iters"]]
        ref = [(i["bound"], i["limit"], i["complete"]) for i in o["iters"]]
        assert ours == ref
        assert _complete_counts(r["iters"]) == _complete_counts(o["iters"])


def test_bts_stp4_sequence_and_overshoot():
    st = synth.stp_walks(4, range(4), lengths=46)
    for s in st:
        p = hb.default_params(batch_size=256, work_num=4, bts_b0=50)
        r = hb.cbdfs_solve(1, s, combine=hb.HB_H_CLASSIC, classic=hb.HB_CLASSIC_MD, algo=hb.HB_BTS, threads=6, params=p)
        o = O.bts(1, s, hkind=O.H_MD, b0=50)
        assert r["cost"] == o["cost"]
        assert [(i["bound"], i["complete"]) for i in r["iters"]] == [(i["bound"], i["complete"]) for i in o["iters"]]
        for i in r["iters"]:
            if not i["complete"]:
                # an iteration is declared exceeded only once the expansions
                # observed across threads reach its limit (the node about to be
                # expanded would pass it), and it stops within a constant of it
                assert i["expanded"] >= i["limit"]
                assert i["expanded"] <= i["limit"] + 6 * 64 + 1


def test_start_equals_goal():
    for dom in (0, 1):
        r = hb.cbdfs_solve(dom, O.goal(dom), combine=hb.HB_H_CLASSIC, classic=hb.HB_CLASSIC_MD, threads=2)
        assert r["status"] == hb.HB_OK and r["cost"] == 0 and r["path"] == []


def test_unsolvable_and_invalid_starts_rejected():
    s = np.arange(9, dtype=np.uint8)
    s[[1, 2]] = s[[2, 1]]  # one swap of two tiles: odd permutation with the blank home
    with pytest.raises(hb.HBError, match="unreachable"):
        hb.cbdfs_solve(0, s, combine=hb.HB_H_CLASSIC, classic=hb.HB_CLASSIC_MD)
    with pytest.raises(hb.HBError):
        hb.cbdfs_solve(0, np.zeros(9, dtype=np.uint8), combine=hb.HB_H_CLASSIC, classic=hb.HB_CLASSIC_MD)
    cube = O.goal(2).copy()
    # twist one corner in place: colours rotate on the three stickers of URF
    idx = [8, 27, 38]  # U bottom-right, R top-left, F top-right
    cube[idx] = cube[[idx[1], idx[2], idx[0]]]
    with pytest.raises(hb.HBError, match="twisted"):
        hb.cbdfs_solve(2, cube, combine=hb.HB_H_CLASSIC, classic=hb.HB_CLASSIC_ZERO)
    with pytest.raises(hb.HBError, match="model"):
        hb.cbdfs_solve(0, O.goal(0), combine=hb.HB_H_NN)


def test_node_limit_reports_budget_with_statistics():
    s = synth.stp_walks(4, [99], lengths=120)[0]
    p = hb.default_params(node_limit=20000, batch_size=128)
    r = hb.cbdfs_solve(1, s, combine=hb.HB_H_CLASSIC_BATCHED, classic=hb.HB_CLASSIC_MD, threads=4, params=p)
    assert r["status"] == hb.HB_E_BUDGET
    assert r["expanded"] >= 20000 and len(r["iters"]) >= 1


def test_timeout_flush_with_one_thread_and_huge_batch():
    # batch of 8000 that one thread with one subtree can never fill: progress
    # relies on the flush rules (timeout or all-threads-waiting)
    s = synth.stp3_instances(3)[2]
    for idle in (0, 1):
        p = hb.default_params(batch_size=8000, work_num=1, timeout_us=200, flush_when_idle=idle)
        r = hb.cbdfs_solve(0, s, combine=hb.HB_H_CLASSIC_BATCHED, classic=hb.HB_CLASSIC_MD, threads=1, params=p)
        o = O.ida(0, s, hkind=O.H_MD)
        assert r["cost"] == o["cost"]
        assert r["mean_batch"] < 8000


def test_memory_bound_and_statistics():
    s = synth.stp_walks(4, [5], lengths=50)[0]
    threads, k = 4, 3
    p = hb.default_params(batch_size=100, work_num=k)
    r = hb.cbdfs_solve(1, s, combine=hb.HB_H_CLASSIC_BATCHED, classic=hb.HB_CLASSIC_MD, threads=threads, params=p)
    d = max(i["bound"] for i in r["iters"]) + 2
    assert r["peak_nodes"] <= threads * k * d * 4  # O(d n k) node records (b <= 4)
    # initial-tree nodes are evaluated once but generated in every iteration
    assert 0 < r["evals"] <= r["generated"] + 10 ** 5 and r["batches"] >= 1
    assert r["frontier"] >= 1
