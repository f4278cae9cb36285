"""The fused persistent forward kernel (tile ids 11-14: the whole forward pass
in one launch whose one-wave blocks pull 32 x 32 tiles off a counter) against
the kernel-per-layer path and the oracle.

Its tiles run the same arithmetic as the separate kernels, so outputs must be
bitwise equal to theirs at every precision and batch size; the counters it
leaves zero must let any sequence of launches, sizes and graph replays follow.
"""
import numpy as np
import pytest

import oracle as O
import paper_2507_11916_amd as hb
import synth

torch = pytest.importorskip("torch")
# Launches of the fused kernel did not return within 90-120 s on the GPU (no
# fault); the library switches the kernel off (set_tile 11-14 is refused) until
# the cause is shown, and these tests stay skipped meanwhile.
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="fused persistent forward kernel switched off: its launches did not "
                                      "return on the GPU; cause not yet shown")]

FUSED = (11, 12, 13, 14)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _eval(model, packed, n_out):
    d_p = _dev(packed)
    d_h = torch.full((packed.shape[0],), -7, dtype=torch.int32, device="cuda")
    d_y = torch.zeros(packed.shape[0] * n_out, dtype=torch.float32, device="cuda")
    model.eval_batch(d_p, d_h, d_y)
    torch.cuda.synchronize()
    return d_h.cpu().numpy(), d_y.cpu().numpy().reshape(-1, n_out)


def _cube_states(count, seed_base=9009):
    mv = synth.rc_walk_moves_array(synth.throughput_seeds(count, seed_base), length_base=20, length_span=11)
    return hb.hb_apply_moves(2, mv)


def _net_case(net_files, name, n):
    if name == "rc_cls":
        return net_files[name], 2, _cube_states(n), dict(out=hb.HB_OUT_CLS_QUANTILE, q=0.99), 21
    if name == "stp3_small":
        return net_files[name], 0, synth.stp3_instances(n), dict(combine_md=True), 1
    return net_files[name], 1, synth.stp_walks(4, synth.throughput_seeds(n), lengths=200), dict(combine_md=True), 1


@pytest.mark.parametrize("name", ["stp4_res", "rc_cls", "stp3_small"])
@pytest.mark.parametrize("prec", [hb.HB_FP32, hb.HB_BF16, hb.HB_FP8_E4M3])
def test_fused_equals_kernel_per_layer(net_files, name, prec):
    path, dom, st, kw, n_out = _net_case(net_files, name, 1000)
    packed = hb.hb_encode(dom, st)
    calib = _dev(packed)
    ref = hb.Model(path, prec=prec, **kw)
    if prec == hb.HB_FP8_E4M3:
        ref.calibrate(calib)
    ref.set_tile(5)  # one-wave 32 x 32 tile, a launch per layer
    fused = [hb.Model(path, prec=prec, **kw) for _ in FUSED]
    for m, t in zip(fused, FUSED):
        if prec == hb.HB_FP8_E4M3:
            m.set_act_scales(ref.act_scales())
        m.set_tile(t)
    for n in (1, 31, 32, 33, 300, 1000):
        h0, y0 = _eval(ref, packed[:n], n_out)
        for m, t in zip(fused, FUSED):
            h, y = _eval(m, packed[:n], n_out)
            np.testing.assert_array_equal(y.view(np.uint32), y0.view(np.uint32), err_msg=f"tile {t} n {n}")
            np.testing.assert_array_equal(h, h0, err_msg=f"tile {t} n {n}")
    for m in fused + [ref]:
        m.close()


def test_fused_against_oracle_and_auto_tiles(net_files):
    """FP32 15-puzzle net: fused output within float32 summation error of the
    oracle, and equal to the automatic (large-tile) path."""
    path, dom, st, kw, _ = _net_case(net_files, "stp4_res", 300)
    packed = hb.hb_encode(dom, st)
    m = hb.Model(path, prec=hb.HB_FP32, **kw)
    m.set_tile(13)
    h, y = _eval(m, packed, 1)
    y_ref = O.Net(path).forward(st)[:, 0]
    assert np.all(np.abs(y[:, 0] - y_ref) <= 1e-5 * np.maximum(1, np.abs(y_ref)))
    auto = hb.Model(path, prec=hb.HB_FP32, **kw)
    auto.set_tile(1)
    h1, y1 = _eval(auto, packed, 1)
    np.testing.assert_array_equal(y, y1)
    np.testing.assert_array_equal(h, h1)


def test_fused_ensemble_equals_members(tmp_path):
    paths = []
    for sd in (31, 32, 33):
        p = str(tmp_path / f"m{sd}.hbw")
        synth.write_weights(p, "stp4_res", seed=sd, head_bias=40.0, spec=synth.widened("stp4_res", 256))
        paths.append(p)
    st = synth.stp_walks(4, synth.throughput_seeds(500, 505), lengths=200)
    packed = hb.hb_encode(1, st)
    for rule in (hb.HB_ENSEMBLE_MIN, hb.HB_ENSEMBLE_SUM):
        ref = hb.Model(paths, prec=hb.HB_BF16, out=hb.HB_OUT_REG_REAL, ensemble_rule=rule)
        ref.set_tile(5)
        m = hb.Model(paths, prec=hb.HB_BF16, out=hb.HB_OUT_REG_REAL, ensemble_rule=rule)
        m.set_tile(12)
        a, b = _eval(ref, packed, 1), _eval(m, packed, 1)
        np.testing.assert_array_equal(a[1], b[1])
        np.testing.assert_array_equal(a[0], b[0])


def test_fused_device_count_and_graph_replays(net_files):
    """Graph-captured fused launches (state count read on the device) over
    uneven sizes, with eager fused launches between replays: every replay
    equals the eager result, rows past n are untouched, and the counters the
    kernel leaves zero keep every later launch correct."""
    path = net_files["stp4_res"]
    cap = 4096
    m = hb.Model(path, prec=hb.HB_BF16, combine_md=True, max_batch=cap)
    m.set_tile(13)
    st = synth.stp_walks(4, synth.throughput_seeds(cap, 2024), lengths=200)
    packed = _dev(hb.hb_encode(1, st))
    ref = hb.Model(path, prec=hb.HB_BF16, combine_md=True, max_batch=cap)
    ref.set_tile(5)
    s = torch.cuda.Stream()
    d_p = torch.zeros((cap, 8), dtype=torch.uint8, device="cuda")
    d_n = torch.zeros(1, dtype=torch.int32, device="cuda")
    d_h = torch.zeros(cap, dtype=torch.int32, device="cuda")
    with torch.cuda.stream(s):
        m.eval_batch_dev_n(d_p, d_n, cap, d_h, stream=s)  # the stream's workspace, before capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        m.eval_batch_dev_n(d_p, d_n, cap, d_h, stream=s)
    for size in list(synth.uneven_batch_sizes(91, 6)) + [1, 4096, 33, 0, 2000]:
        size = min(int(size), cap)
        d_p[:size] = packed[:size]
        d_n.fill_(size)
        d_h.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        if size:
            want = torch.zeros(size, dtype=torch.int32, device="cuda")
            ref.eval_batch(packed[:size].contiguous(), want)
            eager = torch.zeros(size, dtype=torch.int32, device="cuda")
            m.eval_batch(packed[:size].contiguous(), eager)
            torch.cuda.synchronize()
            assert torch.equal(d_h[:size], want), size
            assert torch.equal(eager, want), size
        assert int((d_h[size:] != -7).sum()) == 0, size
