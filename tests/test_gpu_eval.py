"""GPU parity of hb_eval_batch against the double-precision oracle.

Inputs are seeded (synth); both sides compute independently; the library is
called through its C ABI.  Tolerances:
  every stored activation, layer by layer, within the float32 summation bound
  of the oracle's layer applied to the library's own input of that layer
  (tests/layerwise.py): exact wherever no rounding boundary is that close;
  the head's output within its own float32 bound of the oracle's head on the
  library's last activation; integer h equal wherever that value is farther
  than the bound from a decision boundary (an integer for floor, q for the
  quantile); whole forward pass: rows without a rounding flip equal the
  oracle's quantised pass to the head's bound, rows with one stay within twice
  the oracle's rounding envelope plus TOL[prec] (FP32 1e-5, BF16 2e-3,
  FP8 2e-2, relative).
"""
import numpy as np
import pytest

import oracle as O
import paper_2507_11916_amd as hb
import synth
from tests import layerwise

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {hb.HB_FP32: 1e-5, hb.HB_BF16: 2e-3, hb.HB_FP8_E4M3: 2e-2}


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda") if dtype is None else t.to("cuda", dtype)


def _eval(model, packed, n_out):
    d_p = _dev(packed)
    d_h = torch.zeros(packed.shape[0], dtype=torch.int32, device="cuda")
    d_y = torch.zeros(packed.shape[0] * n_out, dtype=torch.float32, device="cuda")
    model.eval_batch(d_p, d_h, d_y)
    torch.cuda.synchronize()
    return d_h.cpu().numpy(), d_y.cpu().numpy().reshape(-1, n_out)


def _cube_states(count, seed_base=9009, lo=20, span=11):
    mv = synth.rc_walk_moves_array(synth.throughput_seeds(count, seed_base), length_base=lo, length_span=span)
    return hb.hb_apply_moves(2, mv)


def _floor_ambiguous(y, tol):
    fr = y - np.floor(y)
    return np.minimum(fr, 1 - fr) <= tol * np.maximum(1, np.abs(y))


def test_8puzzle_all_states_fp32(net_files):
    st = O.all8()
    net = O.Net(net_files["stp3_small"])
    y_ref = net.forward(st)[:, 0]
    md = O.manhattan(0, st)
    h_ref = net.h(y_ref, 0, classic=md)
    m = hb.Model(net_files["stp3_small"], prec=hb.HB_FP32, combine_md=True)
    h, y = _eval(m, hb.hb_encode(0, st), 1)
    err = np.abs(y[:, 0] - y_ref) / np.maximum(1, np.abs(y_ref))
    print("8-puzzle fp32 max rel err", err.max())
    assert err.max() <= TOL[hb.HB_FP32]
    amb = _floor_ambiguous(y_ref, TOL[hb.HB_FP32]) & (np.floor(y_ref) < md)
    mism = (h != h_ref) & ~amb
    print("ambiguous", amb.sum(), "mismatch", (h != h_ref).sum())
    assert mism.sum() == 0
    # states within the tolerance window of an integer: about 2 * window * n
    window = TOL[hb.HB_FP32] * np.abs(y_ref).max()
    assert amb.sum() <= 4 * window * len(st) + 10


def _flip_envelope(y, y_q, y_exact, e_head, flip_rows, tol):
    """Rows with no flip in any layer must match the oracle's quantised
    forward pass (y_q) to the head's float32 bound; rows with a flip may drift
    but stay within twice the oracle's own rounding envelope |y_q - y_exact|
    (plus tol).  Returns the fraction of rows with a flip."""
    d = np.abs(y - y_q)
    assert np.all(d[~flip_rows] <= e_head[~flip_rows] + 1e-9 * np.abs(y_q[~flip_rows])), \
        (d[~flip_rows].max(), np.argwhere(d[~flip_rows] > e_head[~flip_rows])[:5])
    scale = np.maximum(1, np.abs(y_q).max(axis=1))
    dr = d.max(axis=1) / scale
    env = np.abs(y_q - y_exact).max(axis=1) / scale
    assert np.all(dr[flip_rows] <= 2 * env[flip_rows] + tol), (dr[flip_rows].max(), env[flip_rows])
    return flip_rows.mean()


@pytest.mark.parametrize("prec", [hb.HB_FP32, hb.HB_BF16, hb.HB_FP8_E4M3])
def test_stp4_residual_net_parity(net_files, prec):
    """Layer by layer against the oracle (tests/layerwise.py), then the head,
    the output rule and the whole forward pass."""
    n = 300  # three 128-row tiles with a ragged tail
    st = synth.stp_walks(4, synth.throughput_seeds(n), lengths=200)
    path = net_files["stp4_res"]
    net = O.Net(path)
    m = hb.Model(path, prec=prec, combine_md=True)
    packed = hb.hb_encode(1, st)
    d_packed = _dev(packed)
    scales = None
    if prec == hb.HB_FP8_E4M3:
        calib = synth.stp_walks(4, synth.throughput_seeds(1024, 4242), lengths=200)
        m.calibrate(_dev(hb.hb_encode(1, calib)))
        scales = net.calibrate(calib)
        np.testing.assert_array_equal(m.act_scales(), scales.astype(np.float32))
    tf = layerwise.teacher_forced(m, net, st, d_packed, int(prec), scales)
    h, y = _eval(m, packed, 1)
    y_tf, e_head = tf["y_tf"], tf["e_head"]
    # the head on the library's own last activation
    assert np.all(np.abs(y - y_tf) <= e_head), np.abs(y - y_tf).max()
    # the output rule on that value: floor, clamp, min with Manhattan distance
    md = O.manhattan(1, st)
    h_tf = net.h(y_tf[:, 0], 0, classic=md)
    # the library's h is the rule on its own y, which differs from y_tf by the
    # observed error (bounded by e_head above): the rule may differ only where
    # y_tf is that close to an integer
    d = np.abs(y[:, 0] - y_tf[:, 0])
    fr = y_tf[:, 0] - np.floor(y_tf[:, 0])
    amb = (np.minimum(fr, 1 - fr) <= d) & (np.floor(y_tf[:, 0]) < md)
    assert np.all((h == h_tf) | amb), np.argwhere((h != h_tf) & ~amb)[:5]
    # the whole forward pass against the oracle's
    y_q = net.forward(st, mode=int(prec), act_scale=scales)
    y_exact = net.forward(st) if prec != hb.HB_FP32 else y_q
    frac = _flip_envelope(y, y_q, y_exact, e_head, tf["flip_rows"], TOL[prec])
    print("stp4 prec", prec, "per-layer (act, elements, two-valued, flips):", tf["stats"],
          "rows with a flip", frac, "ambiguous h", amb.sum())
    m.close()


@pytest.mark.parametrize("prec", [hb.HB_FP32, hb.HB_BF16, hb.HB_FP8_E4M3])
def test_cube_classifier_parity(net_files, prec):
    """Layer by layer against the oracle, then the logits, the quantile rule and
    the whole forward pass (nine matrix layers)."""
    n = 200
    st = _cube_states(n)
    path = net_files["rc_cls"]
    net = O.Net(path)
    m = hb.Model(path, prec=prec, out=hb.HB_OUT_CLS_QUANTILE, q=0.99)
    d_packed = _dev(hb.hb_encode(2, st))
    scales = None
    if prec == hb.HB_FP8_E4M3:
        calib = _cube_states(512, 777)
        m.calibrate(_dev(hb.hb_encode(2, calib)))
        scales = net.calibrate(calib)
        np.testing.assert_array_equal(m.act_scales(), scales.astype(np.float32))
    tf = layerwise.teacher_forced(m, net, st, d_packed, int(prec), scales)
    h, z = _eval(m, hb.hb_encode(2, st), 21)
    z_tf, e_head = tf["y_tf"], tf["e_head"]
    assert np.all(np.abs(z - z_tf) <= e_head), np.abs(z - z_tf).max()
    # The library applies the rule to its own logits, which differ from z_tf by
    # at most D = max |z - z_tf| per row (bounded by e_head above).  A change of
    # at most D in every logit moves each cumulative softmax probability by at
    # most 2D; float32 softmax and cumulative sums add at most about 1e-6.  The
    # quantile decision may differ only within that margin of q.
    h_tf = net.h(z_tf, 3, q=0.99)
    p = np.exp(z_tf - z_tf.max(axis=1, keepdims=True))
    cdf = np.cumsum(p / p.sum(axis=1, keepdims=True), axis=1)
    margin = np.abs(cdf - 0.99).min(axis=1)
    amb = margin <= 2 * np.abs(z - z_tf).max(axis=1) + 1e-6
    assert np.all((h == h_tf) | amb)
    z_q = net.forward(st, mode=int(prec), act_scale=scales)
    z_exact = net.forward(st) if prec != hb.HB_FP32 else z_q
    frac = _flip_envelope(z, z_q, z_exact, e_head, tf["flip_rows"], TOL[prec])
    print("cube prec", prec, "per-layer (act, elements, two-valued, flips):", tf["stats"],
          "rows with a flip", frac, "ambiguous h", amb.sum())
    m.close()


@pytest.mark.parametrize("n", [0, 1, 2, 63, 64, 65, 127, 129, 1000])
def test_batch_sizes_and_position_independence(net_files, n):
    path = net_files["stp4_res"]
    m = hb.Model(path, prec=hb.HB_BF16)
    st = synth.stp_walks(4, synth.throughput_seeds(1000), lengths=200)
    packed = hb.hb_encode(1, st)
    h_all, y_all = _eval(m, packed, 1)
    if n == 0:
        d_h = torch.zeros(1, dtype=torch.int32, device="cuda")
        m.eval_batch(_dev(packed[:1]), d_h, n=0)
        return
    h, y = _eval(m, packed[1000 - n:], 1)
    # a state's output does not depend on the batch around it
    np.testing.assert_array_equal(y[:, 0], y_all[1000 - n:, 0])
    np.testing.assert_array_equal(h, h_all[1000 - n:])


@pytest.mark.parametrize("prec", [hb.HB_FP32, hb.HB_BF16, hb.HB_FP8_E4M3])
def test_tile_shapes_give_identical_results(net_files, prec):
    """Every tile shape (register-staged LDS tiles, the one-wave small-batch
    kernel, the direct-load LDS ring) runs the same MFMA sequence per output:
    results are bitwise equal, so a state's h does not depend on the batch size
    or the tile that the autotuner picks (the wide-block ring tiles 15-17
    and 20 included)."""
    path = net_files["stp4_res"]
    st = synth.stp_walks(4, synth.throughput_seeds(700), lengths=200)
    packed = hb.hb_encode(1, st)
    calib = _dev(hb.hb_encode(1, synth.stp_walks(4, synth.throughput_seeds(1024, 4242), lengths=200)))
    outs = []
    for tile in list(range(1, 11)) + [15, 16, 17, 18, 19, 20]:
        m = hb.Model(path, prec=prec)
        if prec == hb.HB_FP8_E4M3:
            m.calibrate(calib)
        m.set_tile(tile)
        outs.append(_eval(m, packed, 1))
    for o in outs[1:]:
        np.testing.assert_array_equal(outs[0][1], o[1])
        np.testing.assert_array_equal(outs[0][0], o[0])


def test_chunking_beyond_max_batch(net_files):
    path = net_files["stp4_res"]
    st = synth.stp_walks(4, synth.throughput_seeds(700), lengths=200)
    packed = hb.hb_encode(1, st)
    a = _eval(hb.Model(path, prec=hb.HB_BF16, max_batch=256), packed, 1)
    b = _eval(hb.Model(path, prec=hb.HB_BF16), packed, 1)
    np.testing.assert_array_equal(a[1], b[1])


@pytest.mark.parametrize("tile", [0, 1, 5, 6, 9, 10, 15, 16, 17, 18, 19, 20])
def test_device_count_variant_matches(net_files, tile):
    """The device-count entry point (grid sized for max_n, tiles strided on the
    device) equals the host-count evaluation, for each kernel family."""
    path = net_files["rc_cls"]
    m = hb.Model(path, prec=hb.HB_BF16, out=hb.HB_OUT_CLS_QUANTILE, q=0.99, max_batch=4096)
    m.set_tile(tile)
    st = _cube_states(333)
    packed = hb.hb_encode(2, st)
    h0, z0 = _eval(m, packed, 21)
    d_p = _dev(packed)
    d_n = torch.tensor([333], dtype=torch.int32, device="cuda")
    d_h = torch.zeros(4096, dtype=torch.int32, device="cuda")
    d_z = torch.zeros(4096 * 21, dtype=torch.float32, device="cuda")
    buf = torch.zeros((4096, 24), dtype=torch.uint8, device="cuda")
    buf[:333] = d_p
    m.eval_batch_dev_n(buf, d_n, 4096, d_h, d_z)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(d_h[:333].cpu().numpy(), h0)
    np.testing.assert_array_equal(d_z[:333 * 21].cpu().numpy().reshape(-1, 21), z0)
    assert int(d_h[333:].abs().sum()) == 0  # rows past n untouched (zero-initialised)


def test_hipgraph_replay_uneven_batches(net_files):
    """One captured graph (launch shape fixed at 16384 rows, count read on the
    device) serves every batch size; each replay equals the eager evaluation."""
    path = net_files["stp4_res"]
    cap = 16384
    m = hb.Model(path, prec=hb.HB_BF16, combine_md=True, max_batch=cap)
    st = synth.stp_walks(4, synth.throughput_seeds(cap, 2024), lengths=200)
    packed = torch.from_numpy(hb.hb_encode(1, st)).cuda()
    s = torch.cuda.Stream()
    d_p = torch.zeros((cap, 8), dtype=torch.uint8, device="cuda")
    d_n = torch.zeros(1, dtype=torch.int32, device="cuda")
    d_h = torch.zeros(cap, dtype=torch.int32, device="cuda")
    with torch.cuda.stream(s):
        m.eval_batch_dev_n(d_p, d_n, cap, d_h, stream=s)  # allocates the stream's workspace before capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        m.eval_batch_dev_n(d_p, d_n, cap, d_h, stream=s)
    sizes = synth.uneven_batch_sizes(77, 6)
    for size in sizes:
        d_p[:size] = packed[:size]
        d_n.fill_(size)
        d_h.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        eager = torch.zeros(size, dtype=torch.int32, device="cuda")
        m.eval_batch(packed[:size].contiguous(), eager)  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(d_h[:size], eager), size
        assert int((d_h[size:] != -7).sum()) == 0, size  # rows past n untouched


def test_persistent_grids_take_every_tile_once(net_files):
    """Tiles 18 and 19 (persistent grids taking tiles off the stream's atomic
    counter) at batches with more tiles than blocks, several launches in a row
    (each launch's last block resets the counter): bitwise equal to the
    one-block-per-tile kernels, including the rows of the last partial tile."""
    path = net_files["stp4_res"]
    st = synth.stp_walks(4, synth.throughput_seeds(16384, 909), lengths=200)
    packed = hb.hb_encode(1, st)
    ref = hb.Model(path, prec=hb.HB_BF16, max_batch=16384)
    ref.set_tile(15)
    for n in (16384, 12345, 16384):
        h0, y0 = _eval(ref, packed[:n], 1)
        for tile in (18, 19):
            m = hb.Model(path, prec=hb.HB_BF16, max_batch=16384)
            m.set_tile(tile)
            for _ in range(3):
                h, y = _eval(m, packed[:n], 1)
                np.testing.assert_array_equal(y, y0)
                np.testing.assert_array_equal(h, h0)
            m.close()
    ref.close()


@pytest.mark.parametrize("tile", [15, 18])
def test_hipgraph_replays_match_oracle(net_files, tile):
    """The captured graph against the oracle, not only against the eager path:
    FP32 replays at uneven sizes (the wide-block 256-row tile forced, so a
    partial last tile and the device-side tile count are exercised; tile 18 as a
    persistent grid taking tiles off the counter on every replay), 40 sampled
    rows per replay against the FP64 forward pass and the output rule."""
    path = net_files["stp4_res"]
    cap = 16384
    m = hb.Model(path, prec=hb.HB_FP32, combine_md=True, max_batch=cap)
    m.set_tile(tile)
    net = O.Net(path)
    st = synth.stp_walks(4, synth.throughput_seeds(cap, 2025), lengths=200)
    packed = torch.from_numpy(hb.hb_encode(1, st)).cuda()
    s = torch.cuda.Stream()
    d_p = torch.zeros((cap, 8), dtype=torch.uint8, device="cuda")
    d_n = torch.zeros(1, dtype=torch.int32, device="cuda")
    d_h = torch.zeros(cap, dtype=torch.int32, device="cuda")
    d_y = torch.zeros(cap, dtype=torch.float32, device="cuda")
    with torch.cuda.stream(s):
        m.eval_batch_dev_n(d_p, d_n, cap, d_h, d_y, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        m.eval_batch_dev_n(d_p, d_n, cap, d_h, d_y, stream=s)
    rng = np.random.default_rng(5)
    for size in synth.uneven_batch_sizes(78, 4) + [257, 8000]:
        d_p[:size] = packed[:size]
        d_n.fill_(size)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        idx = np.unique(np.concatenate([rng.choice(size, min(size, 38), replace=False), [0, size - 1]]))
        y = d_y[:size].cpu().numpy().astype(np.float64)[idx]
        y_ref = net.forward(st[idx])[:, 0]
        assert np.max(np.abs(y - y_ref) / np.maximum(1, np.abs(y_ref))) <= TOL[hb.HB_FP32], size
        h_ref = net.h(y_ref, 0, classic=O.manhattan(1, st[idx]))
        amb = np.abs(y_ref - np.round(y_ref)) < 1e-4  # an output within rounding of an integer may floor either way
        assert np.array_equal(d_h[:size].cpu().numpy()[idx][~amb], h_ref[~amb]), size
    m.close()


def test_full_size_sampled_rows(net_files):
    """B = 16384 (the largest batch) in the benchmark's launch shape; 48 sampled
    rows against the oracle."""
    path = net_files["stp4_res"]
    B = 16384
    st = synth.stp_walks(4, synth.throughput_seeds(B, 31337), lengths=200)
    m = hb.Model(path, prec=hb.HB_FP32, combine_md=True)
    h, y = _eval(m, hb.hb_encode(1, st), 1)
    idx = np.random.default_rng(0).choice(B, 48, replace=False)
    net = O.Net(path)
    y_ref = net.forward(st[idx])[:, 0]
    err = np.abs(y[idx, 0] - y_ref) / np.maximum(1, np.abs(y_ref))
    assert err.max() <= TOL[hb.HB_FP32]


def test_fp8_requires_calibration(net_files):
    m = hb.Model(net_files["stp4_res"], prec=hb.HB_FP8_E4M3)
    st = synth.stp_walks(4, [1, 2], lengths=10)
    with pytest.raises(hb.HBError, match="calibrate"):
        _eval(m, hb.hb_encode(1, st), 1)


def test_autotuner_table_and_tuning_cache(net_files, tmp_path):
    """Bucket autotuner: one row per power-of-two batch, the model then uses the
    tuned tile per bucket, the table survives a save/load round trip, a file for
    another precision is refused, and outputs do not depend on the table."""
    path = net_files["stp4_res"]
    st = synth.stp_walks(4, synth.throughput_seeds(1500, 31), lengths=200)
    d = _dev(hb.hb_encode(1, st))
    m = hb.Model(path, prec=hb.HB_BF16, max_batch=2048)
    ref = _eval(m, hb.hb_encode(1, st), 1)
    table, rec = m.autotune(d)
    print("autotune", [(e["batch"], e["tile"], round(e["us"], 1)) for e in table], "recommended", rec)
    assert [e["batch"] for e in table] == [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 1500]
    assert all(1 <= e["tile"] <= 10 and e["us"] > 0 for e in table)
    assert rec in [e["batch"] for e in table]
    best = max(e["evals_per_s"] for e in table)
    assert next(e for e in table if e["batch"] == rec)["evals_per_s"] >= 0.9 * best
    for e in table[:-2]:  # rows 1024 and 1500 share a bucket: the later row holds it
        assert m.tile_for(e["batch"]) == e["tile"]
    assert m.tile_for(1024) == m.tile_for(1500) == table[-1]["tile"]
    f = str(tmp_path / "tuning.txt")
    m.save_tuning(f)
    m2 = hb.Model(path, prec=hb.HB_BF16, max_batch=2048)
    m2.load_tuning(f)
    for b in (1, 3, 100, 700, 1500):
        assert m2.tile_for(b) == m.tile_for(b)
    out = _eval(m2, hb.hb_encode(1, st), 1)
    np.testing.assert_array_equal(out[1], ref[1])
    with pytest.raises(hb.HBError, match="another network or precision"):
        hb.Model(path, prec=hb.HB_FP32, max_batch=2048).load_tuning(f)


@pytest.mark.parametrize("prec", [hb.HB_FP32, hb.HB_BF16])
def test_ragged_width_parity(tmp_path, prec):
    """A hidden width that is not a multiple of the tile (320, padded to 384 on
    the device), as in the model-size sweep, against the oracle."""
    path = str(tmp_path / "w320.hbw")
    synth.write_weights(path, "stp4_res", spec=synth.widened("stp4_res", 320), seed=22, head_bias=40.0)
    st = synth.stp_walks(4, synth.throughput_seeds(300, 808), lengths=200)
    net = O.Net(path)
    m = hb.Model(path, prec=prec, combine_md=True)
    packed = hb.hb_encode(1, st)
    tf = layerwise.teacher_forced(m, net, st, _dev(packed), int(prec))
    h, y = _eval(m, packed, 1)
    assert np.all(np.abs(y - tf["y_tf"]) <= tf["e_head"])
    y_ref = net.forward(st, mode=int(prec))
    y_exact = net.forward(st) if prec != hb.HB_FP32 else y_ref
    _flip_envelope(y, y_ref, y_exact, tf["e_head"], tf["flip_rows"], TOL[prec])


def test_switched_off_fused_tiles_are_refused(net_files):
    """Tile ids 11-14 (the fused persistent forward kernel) are refused while
    that kernel is switched off; the autotuner never picks them."""
    m = hb.Model(net_files["stp4_res"], prec=hb.HB_BF16, max_batch=1024)
    for t in (11, 12, 13, 14):
        with pytest.raises(hb.HBError) as e:
            m.set_tile(t)
        assert e.value.status == hb.HB_E_UNSUPPORTED
    st = synth.stp_walks(4, synth.throughput_seeds(300, 5), lengths=200)
    report = m.tune(_dev(hb.hb_encode(1, st)))
    assert report and all(1 <= t <= 10 or 15 <= t <= 20 for t, _ in report)
    m.close()
