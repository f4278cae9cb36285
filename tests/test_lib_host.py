"""Host-side library checks that need no GPU: the C ABI loads and exports every
declared symbol; the library's domain code agrees with the oracle's
independent models; packing round-trips; input validation rejects bad states."""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle as O
import paper_2507_11916_amd as hb
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "hb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(hb_[a-z0-9_]+|cbdfs_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    hb.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", hb.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [s for s in _declared_symbols() if s not in exported]
    assert not missing, missing
    assert len(_declared_symbols()) >= 20


def test_sizes():
    assert [hb.state_bytes(d) for d in (0, 1, 2)] == [9, 16, 54]
    assert [hb.packed_bytes(d) for d in (0, 1, 2)] == [8, 8, 24]
    assert hb.state_bytes(7) == -1


@pytest.mark.parametrize("domain", [0, 1])
def test_stp_moves_and_manhattan_agree_with_oracle(domain):
    n = 3 if domain == 0 else 4
    st = synth.stp_walks(n, range(500), lengths=80)
    np.testing.assert_array_equal(hb.hb_manhattan(domain, st), O.manhattan(domain, st))


def test_cube_moves_agree_with_oracle_on_10000_sequences():
    mv = synth.rc_walk_moves_array(range(10000), length_base=1, length_span=30)
    a = hb.hb_apply_moves(2, mv)
    b = O.apply_moves(2, mv)
    np.testing.assert_array_equal(a, b)
    # every single move too, including the ones canonical pruning never draws
    for m in range(18):
        np.testing.assert_array_equal(hb.hb_apply_moves(2, [m]), O.apply_moves(2, np.array([m], dtype=np.int8)))


def test_stp_move_sequences_agree_with_oracle():
    rng = np.random.default_rng(9)
    for n, dom in ((3, 0), (4, 1)):
        # random legal move sequences built by walking the blank
        seqs = []
        for _ in range(300):
            b, seq = 0, []
            for _ in range(int(rng.integers(0, 60))):
                r, c = divmod(b, n)
                opts = [m for m, ok in enumerate([r > 0, c > 0, c < n - 1, r < n - 1]) if ok]
                m = int(rng.choice(opts))
                seq.append(m)
                b += [-n, -1, 1, n][m]
            seqs.append(seq + [-1] * (60 - len(seq)))
        mv = np.array(seqs, dtype=np.int8)
        np.testing.assert_array_equal(hb.hb_apply_moves(dom, mv), O.apply_moves(dom, mv))


def test_apply_moves_rejects_off_board():
    with pytest.raises(hb.HBError):
        hb.hb_apply_moves(1, [0])


@pytest.mark.parametrize("domain", [0, 1, 2])
def test_encode_decode_round_trip(domain):
    if domain == 2:
        st = O.apply_moves(2, synth.rc_walk_moves_array(range(300), length_base=0, length_span=25))
    else:
        st = synth.stp_walks(3 if domain == 0 else 4, range(300), lengths=100)
    p = hb.hb_encode(domain, st)
    assert p.shape == (300, hb.packed_bytes(domain))
    np.testing.assert_array_equal(hb.hb_decode(domain, p), st)


def test_encode_layout_is_documented_bit_layout():
    st = synth.stp_walks(4, [5], lengths=50)
    w = int.from_bytes(hb.hb_encode(1, st)[0].tobytes(), "little")
    assert [(w >> (4 * p)) & 15 for p in range(16)] == list(st[0])
    cube = O.apply_moves(2, np.array([[0, 9, 14]], dtype=np.int8))[0]
    words = np.frombuffer(hb.hb_encode(2, cube)[0].tobytes(), dtype="<u8")
    nc = [p for p in range(54) if p % 9 != 4]
    for q, p in enumerate(nc):
        assert (int(words[q // 16]) >> (3 * (q % 16))) & 7 == cube[p]


def test_encode_rejects_invalid_states():
    bad = np.arange(16, dtype=np.uint8)
    bad[3] = 2
    with pytest.raises(hb.HBError, match="state 1"):
        hb.hb_encode(1, np.stack([np.arange(16, dtype=np.uint8), bad]))
    cube = O.goal(2).copy()
    cube[4] = 1
    with pytest.raises(hb.HBError):
        hb.hb_encode(2, cube)
    assert hb.hb_encode(1, np.zeros((0, 16), dtype=np.uint8)).shape == (0, 8)


def test_corner_pdb_agrees_with_oracle():
    k = 4
    ours = hb.Pdb(k, threads=4)
    tab, _ = O.corner_pdb(k)
    st = O.apply_moves(2, synth.rc_walk_moves_array(range(2000), length_base=0, length_span=20))
    np.testing.assert_array_equal(ours.lookup(st), tab[O.corner_index(st, k)])


def test_model_load_without_gpu_reports_device_error(net_files):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(hb.HBError) as e:
        hb.Model(net_files["stp3_small"])
    assert e.value.status in (hb.HB_E_DEVICE, hb.HB_E_INVAL)


def test_model_load_rejects_bad_files(tmp_path):
    p = tmp_path / "bad.hbw"
    p.write_bytes(b"XXXX" + bytes(40))
    with pytest.raises(hb.HBError, match="magic"):
        hb.Model(str(p))


def _golden(name):
    """key value pairs of a fixture under tests/golden (comments after '#')."""
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    out = {}
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = line.split()
            out[k] = float(v)
    return out


def test_corner_pdb_statistics_match_published_values():
    """The library's 8-corner PDB against the published entry count, largest
    value and mean; a wrong move table or corner index changes all three."""
    g = _golden("corner_pdb_8.txt")
    pdb = hb.Pdb(8)
    counts, vmax = pdb.value_counts(16)
    pdb.close()
    assert counts.sum() == g["entries"]
    assert vmax == g["max_value"]
    mean = (counts * np.arange(16)).sum() / counts.sum()
    assert round(mean, 3) == g["mean_value"]
    assert counts[0] == 1 and counts[1] == 18  # the goal; one entry per face turn


def test_corner_pdb_distribution_matches_oracle_table():
    """4-corner PDB: the library's value distribution equals the oracle's table."""
    tab, reached = O.corner_pdb(4)
    pdb = hb.Pdb(4)
    counts, vmax = pdb.value_counts(16)
    pdb.close()
    ref = np.bincount(tab[tab != 255].astype(np.int64), minlength=16)
    np.testing.assert_array_equal(counts, ref[:16])
    assert counts.sum() == reached and vmax == int(tab[tab != 255].max())


def test_defaults_follow_paper_settings():
    g = _golden("paper_settings.txt")
    p = hb.default_params()
    assert p.timeout_us == g["batch_timeout_us"]
    assert p.batch_size == g["target_batch_cube"]
    pdb = hb.Pdb(int(g["classic_cube_pdb_corners"]))  # the largest corner PDB the library builds
    pdb.close()
    with pytest.raises(hb.HBError):
        hb.Pdb(int(g["classic_cube_pdb_corners"]) + 1)


def test_additive_stp_pdb_matches_oracle():
    """The library's additive 15-puzzle PDB (its own ranking and level-parallel
    build) equals the oracle's (dense codes, 0-1 breadth-first search)."""
    groups = [range(1, 5), range(5, 9), range(9, 13), range(13, 16)]
    spec = O.apdb(groups)
    st = synth.stp_walks(4, synth.throughput_seeds(3000, 31), lengths=200)
    pdb = hb.Pdb(groups=groups)
    np.testing.assert_array_equal(pdb.lookup(st), O.apdb_h(st, spec))
    counts, vmax = pdb.value_counts(64)
    assert counts.sum() == 3 * 16 * 15 * 14 * 13 + 16 * 15 * 14  # placements of 4-4-4-3 tiles
    pdb.close()


@pytest.mark.slow
def test_additive_stp_pdb_663_matches_oracle():
    """The library's 6-6-3 split (the benchmark's and the training labels'
    PDB) equals the sum of the oracle's three group tables on 10^5 states."""
    groups = [range(1, 7), range(7, 13), range(13, 16)]
    st = synth.stp_walks(4, synth.throughput_seeds(100000, 63), lengths=200)
    ref = sum(O.apdb_group_lookup(O.apdb_group_table(g), st) for g in groups)
    pdb = hb.Pdb(groups=groups)
    np.testing.assert_array_equal(pdb.lookup(st), ref)
    counts, _ = pdb.value_counts(128)
    assert counts.sum() == 2 * 16 * 15 * 14 * 13 * 12 * 11 + 16 * 15 * 14
    pdb.close()


def test_additive_stp_pdb_rejects_bad_groupings():
    with pytest.raises(hb.HBError):
        hb.Pdb(groups=[range(1, 10), range(10, 16)])  # a group of 9 tiles
    with pytest.raises(hb.HBError):
        hb.Pdb(groups=[range(1, 8)])  # tiles 8..15 in no group


def test_pdb_entry_points_reject_bad_arguments():
    """Error statuses of the PDB calls, through the C ABI with raw arguments."""
    import ctypes as C
    L = hb.lib()
    out = C.c_void_p()
    assert L.hb_pdb_build_stp_additive(None, 1, C.byref(out)) == hb.HB_E_INVAL
    g = np.full(16, -1, dtype=np.int32)
    g[1:] = 0  # fifteen tiles in one group: more than 8
    assert L.hb_pdb_build_stp_additive(g.ctypes.data, 1, C.byref(out)) == hb.HB_E_INVAL
    assert "groups" in L.hb_last_error().decode()
    counts = np.zeros(4, dtype=np.int64)
    assert L.hb_pdb_value_counts(None, counts.ctypes.data, 4, None) == hb.HB_E_INVAL
    pdb = hb.Pdb(3, threads=2)
    assert L.hb_pdb_value_counts(pdb.handle, counts.ctypes.data, 0, None) == hb.HB_E_INVAL
    assert L.hb_pdb_value_counts(pdb.handle, None, 4, None) == hb.HB_E_INVAL
    # a short buffer counts only the values that fit
    assert L.hb_pdb_value_counts(pdb.handle, counts.ctypes.data, 4, None) == hb.HB_OK
    full, vmax = pdb.value_counts(32)
    np.testing.assert_array_equal(counts, full[:4])
    assert vmax >= 4 and full.sum() == 8 * 7 * 6 * 27
    # lookups of states that are not 15-puzzle permutations are rejected
    apdb = hb.Pdb(groups=[range(1, 5), range(5, 9), range(9, 13), range(13, 16)], threads=2)
    with pytest.raises(hb.HBError):
        apdb.lookup(np.zeros((1, 16), dtype=np.uint8))
    apdb.close()
    pdb.close()


def _md_of(st, tiles):
    where = np.argsort(st, axis=1)  # cell of each tile
    return sum(np.abs(where[:, t] // 4 - t // 4) + np.abs(where[:, t] % 4 - t % 4) for t in tiles)


def _big_group_pins(group, six, n_tiles):
    """Pins of a library pattern table over `group` (7 or 8 tiles) built with
    every other tile as its own group (so h = PDB(group) + MD(others)):
    every placement of the group is reached (16!/(16-k)!); it dominates the
    oracle's table over the first six of its tiles plus the Manhattan distance
    of the rest (a path for the k tiles is a path for those six, and the other
    tiles' moves are at least their Manhattan distance), strictly somewhere;
    it has MD's parity; and it never exceeds optimal costs of short walks."""
    others = [t for t in range(1, 16) if t not in group]
    pdb = hb.Pdb(groups=[group] + [[t] for t in others])
    counts, _ = pdb.value_counts(128)
    placements = 1
    for i in range(n_tiles):
        placements *= 16 - i
    assert counts.sum() == placements + 16 * len(others)
    st = synth.stp_walks(4, synth.throughput_seeds(20000, 78), lengths=200)
    h = pdb.lookup(st)
    pk = h - _md_of(st, others)
    lower = O.apdb_group_lookup(O.apdb_group_table(six), st) + _md_of(st, [t for t in group if t not in six])
    assert np.all(pk >= lower) and np.any(pk > lower)
    md = _md_of(st, range(1, 16))
    assert np.all(h >= md) and np.all((h - md) % 2 == 0)
    assert pdb.lookup(O.goal(O.STP4)[None])[0] == 0
    for s in synth.stp_walks(4, synth.config_seeds(9, 8), lengths=34):
        assert pdb.lookup(s[None])[0] <= O.ida(O.STP4, s, hkind=O.H_MD)["cost"]
    pdb.close()


@pytest.mark.slow
def test_seven_tile_group_of_the_paper_split():
    """Tiles 1-7, the first half of the paper's 7-8 additive PDB."""
    _big_group_pins(list(range(1, 8)), range(1, 7), 7)


@pytest.mark.slow
def test_eight_tile_group_of_the_paper_split():
    """Tiles 8-15, the second half of the paper's 7-8 additive PDB (518,918,400
    placements: index arithmetic at the library's largest group size)."""
    _big_group_pins(list(range(8, 16)), range(8, 14), 8)


def test_walk_moves_reproduce_the_walks():
    """synth.stp_walk_moves (blank-only tracking, used to build millions of
    training states) takes exactly stp_walks' walks: applying its rows to the
    goal with the library gives the same states, serially and in parallel."""
    seeds = synth.throughput_seeds(3000, 31337)
    ref = synth.stp_walks(4, seeds, length_base=0, length_span=201)
    mv = synth.stp_walk_moves(4, seeds, length_base=0, length_span=201)
    assert mv.shape[1] == 200 and np.all((mv >= -1) & (mv <= 3))
    np.testing.assert_array_equal(hb.hb_apply_moves(hb.HB_STP4, mv), ref)
    ref3 = synth.stp_walks(3, seeds[:500], lengths=40)
    np.testing.assert_array_equal(hb.hb_apply_moves(hb.HB_STP3, synth.stp_walk_moves(3, seeds[:500], lengths=40)), ref3)
    big = synth.throughput_seeds(70000, 4)
    np.testing.assert_array_equal(synth.stp_walk_moves_parallel(4, big, 0, 201, 2),
                                  synth.stp_walk_moves(4, big, length_base=0, length_span=201))
