"""Pins of the oracle network, output rules and rounding emulation.

Each pin is independent of the oracle's own code path: a dense one-hot matrix
product for the gather-sum, a hand-designed network with a closed-form output,
torch's CPU conversions for bfloat16 and e4m3, exhaustive code round trips, and
hand-built outputs on either side of every decision boundary.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests import nets


def _onehot(states, S):
    n, P = states.shape
    x = np.zeros((n, P * S))
    x[np.arange(n)[:, None], np.arange(P)[None, :] * S + states] = 1.0
    return x


def test_gather_sum_equals_dense_onehot_product(net_files, tmp_path):
    # A one-layer net whose head is the identity exposes ReLU(layer 1).
    rng = np.random.default_rng(5)
    W0 = rng.standard_normal((256, 7)).astype(np.float32)
    b0 = rng.standard_normal(7).astype(np.float32)
    path = str(tmp_path / "l1.hbw")
    synth.write_weights_arrays(path, 1, 256, [7], 0, 7, 0, [W0, b0, np.eye(7), np.zeros(7)])
    net = O.Net(path)
    st = synth.stp_walks(4, range(50), lengths=60)
    y = net.forward(st)
    ref = np.maximum(_onehot(st.astype(np.int64), 16) @ W0.astype(np.float64) + b0, 0.0)
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [3, 4])
def test_closed_form_network(n, tmp_path):
    path = str(tmp_path / "md.hbw")
    nets.write_md_net(path, n)
    net = O.Net(path)
    st = synth.stp_walks(n, range(300), lengths=41)
    md = O.manhattan(n - 3, st)
    assert md.min() >= 1
    y = net.forward(st)
    np.testing.assert_array_equal(y[:, 0], 3.5)
    np.testing.assert_array_equal(y[:, 1], 2 * md - 2)


def test_bf16_forward_is_exact_on_representable_values(tmp_path):
    # Small integers are exact in bfloat16, so the bf16 forward of this net equals
    # the unrounded one (the rounding itself is pinned by hand-built nets in
    # test_oracle_precision.py).
    path = str(tmp_path / "md.hbw")
    nets.write_md_net(path, 3)
    net = O.Net(path)
    st = synth.stp_walks(3, range(200), lengths=5)
    st = st[O.manhattan(0, st) >= 1]
    y0 = net.forward(st, mode=0)
    y1 = net.forward(st, mode=1)
    np.testing.assert_array_equal(y0, y1)


def test_fp8_weight_quantisation_bounds(net_files):
    net = O.Net(net_files["stp4_res"])
    # per-column scales: max|W|/448 as a float32 quotient
    W = np.fromfile(net_files["stp4_res"], dtype="<f4", offset=4 * 10)
    W0 = W[:256 * 1000]
    W1 = W[256 * 1000 + 1000:256 * 1000 + 1000 + 1000 * 1000].reshape(1000, 1000)
    s = net.fp8_col_scales(2)[:1000]
    expect = (np.abs(W1).max(axis=0).astype(np.float64) / 448.0).astype(np.float32)
    np.testing.assert_array_equal(s, expect)
    del W0


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(20000) * 10 ** rng.uniform(-6, 6, 20000),
                        [0.0, -0.0, 1.0, 3.0e38, -1e-40, 65504.0]])
    x32 = x.astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(x32).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(O.bf16_round(x32), ref)


def test_bf16_ties_round_to_even():
    # 1 + 2^-8 lies exactly half-way between 1 and 1 + 2^-7: ties go to the even code (1.0)
    assert O.bf16_round(1.0 + 2 ** -8) == 1.0
    # 1 + 3*2^-8 lies half-way between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert O.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    assert O.bf16_round(1.0 + 2 ** -8 + 2 ** -20) == 1.0 + 2 ** -7


def test_e4m3_codes_round_trip_exhaustively():
    vals = []
    for c in range(256):
        v = O.e4m3_decode(c)
        if math.isnan(v):
            assert c in (0x7F, 0xFF)
            continue
        assert O.e4m3_round(np.array([v]))[0] == v
        vals.append(v)
    pos = sorted(set(abs(v) for v in vals))
    assert max(pos) == 448.0 and len(pos) == 127  # 0 plus 126 positive finite values
    assert min(p for p in pos if p > 0) == 2.0 ** -9


def test_e4m3_matches_torch_in_range_and_saturates():
    rng = np.random.default_rng(2)
    x = rng.uniform(-448, 448, 50000) * 10 ** rng.uniform(-4, 0, 50000)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = O.e4m3_round(x.astype(np.float32).astype(np.float64))
    np.testing.assert_array_equal(got, ref)
    assert O.e4m3_round(np.array([500.0, -1e6, 449.0]))[:].tolist() == [448.0, -448.0, 448.0]
    # the midpoint of 448 and the first value past it (480) rounds to 448
    assert O.e4m3_round(np.array([464.0]))[0] == 448.0


def test_e4m3_ties_to_even():
    # between 1.0 (code 0x38) and 1.125 (0x39): midpoint -> even code 0x38
    assert O.e4m3_round(np.array([1.0625]))[0] == 1.0
    # between 1.125 (0x39) and 1.25 (0x3A): midpoint -> 0x3A
    assert O.e4m3_round(np.array([1.1875]))[0] == 1.25


def test_regression_output_rule_at_integer_boundaries():
    net = O.Net.__new__(O.Net)
    lib = O.lib()
    f = lib.orc_h_regression
    f.argtypes = [O.C.c_double, O.C.c_int, O.C.c_double, O.C.c_int]
    for k in [0, 1, 7, 30]:
        up = np.nextafter(float(k), np.inf)
        dn = np.nextafter(float(k), -np.inf)
        assert f(float(k), 0, 0.0, -1) == k
        assert f(up, 0, 0.0, -1) == k
        assert f(dn, 0, 0.0, -1) == max(k - 1, 0)
    assert f(-3.2, 0, 0.0, -1) == 0  # clamped at zero
    assert f(12.7, 0, 0.0, 9) == 9  # min with the classic heuristic
    assert f(12.7, 0, 2.2, -1) == 10  # constant offset
    assert f(2.5, 1, 0.0, -1) == 2 and f(3.5, 1, 0.0, -1) == 4  # half to even
    assert f(float("nan"), 0, 0.0, 5) == 5
    del net


def test_classifier_output_rule_around_q():
    f = O.lib().orc_h_classifier
    f.argtypes = [O.C.c_void_p, O.C.c_int, O.C.c_int, O.C.c_double]
    p = np.array([0.25, 0.5, 0.25])
    z = np.log(p)
    cdf = np.cumsum(np.exp(z - z.max()) / np.exp(z - z.max()).sum())
    zz = np.ascontiguousarray(z)
    assert f(zz.ctypes.data, 3, 3, cdf[0] - 1e-9) == 0
    assert f(zz.ctypes.data, 3, 3, cdf[0] + 1e-9) == 1
    assert f(zz.ctypes.data, 3, 3, cdf[1] + 1e-9) == 2
    assert f(zz.ctypes.data, 3, 3, 1.5) == 2  # never reached: last class
    assert f(zz.ctypes.data, 3, 4, 0.0) == 1  # arg-max
    ties = np.ascontiguousarray([1.0, 3.0, 3.0])
    assert f(ties.ctypes.data, 3, 4, 0.0) == 1  # lowest index on ties


def test_calibration_scales_are_powers_of_two(net_files):
    net = O.Net(net_files["stp4_res"])
    st = synth.stp_walks(4, synth.throughput_seeds(64), lengths=200)
    sc = net.calibrate(st)
    _, amax = net.forward(st, mode=0, want_act_max=True)
    assert sc.shape == (net.n_act,)
    for a, m in zip(sc, amax):
        e = math.log2(a)
        assert e == int(e)
        assert m / a <= 448.0 and m / a > 224.0


def test_network_shapes(net_files):
    for name, spec in synth.NETS.items():
        net = O.Net(net_files[name])
        assert net.dims == spec["dims"] and net.n_res == spec["n_res"] and net.n_out == spec["n_out"]
        assert net.n_in == spec["n_in"]


def _md_net_one_output(path, n, shift):
    """The closed-form network with only its second output, shifted: y = 2 MD - 2 + shift."""
    ts = [np.asarray(t, dtype=np.float64) for t in nets.md_net_tensors(n)]
    ts[-2] = ts[-2][:, 1:2]
    ts[-1] = np.asarray(ts[-1]).reshape(-1)[1:2] + shift
    synth.write_weights_arrays(path, 0 if n == 3 else 1, n ** 4, [2, 3], 1, 1, 0, ts)


@pytest.mark.parametrize("n", [3, 4])
def test_ensemble_forward_closed_form(n, tmp_path):
    """Minimum and sum over members with known outputs 2 MD - 2 + shift."""
    shifts = [0.0, 3.0, -1.5]
    paths = []
    for i, sh in enumerate(shifts):
        paths.append(str(tmp_path / f"m{i}.hbw"))
        _md_net_one_output(paths[-1], n, sh)
    members = [O.Net(p) for p in paths]
    st = synth.stp_walks(n, range(200), lengths=41)
    md = O.manhattan(n - 3, st).astype(np.float64)
    np.testing.assert_array_equal(O.ensemble_forward(members[:1], st, O.ENS_MIN), 2 * md - 2)
    np.testing.assert_array_equal(O.ensemble_forward(members, st, O.ENS_MIN), 2 * md - 2 - 1.5)
    np.testing.assert_array_equal(O.ensemble_forward(members, st, O.ENS_SUM), 3 * (2 * md - 2) + 1.5)


def test_combined_regression_rule():
    md = np.array([5, 5, 5, 9, 9, 0])
    y = np.array([2.7, -1.0, np.nan, 12.7, 3.0, 0.999999])
    np.testing.assert_array_equal(O.h_regression(y, md, combine=3), [7, 5, 5, 21, 12, 0])
    np.testing.assert_array_equal(O.h_regression(y, md, combine=2), [5, 5, 5, 12, 9, 0])
    np.testing.assert_array_equal(O.h_regression(y, md, combine=1), [2, 0, 5, 9, 3, 0])
    np.testing.assert_array_equal(O.h_regression(np.array([12.7]), None, offset=2.2), [10])
    np.testing.assert_array_equal(O.h_regression(np.array([2.5, 3.5]), None, mode=1), [2, 4])
    # the written-out rule agrees with the C rule on a sweep (classic = min)
    f = O.lib().orc_h_regression
    f.argtypes = [O.C.c_double, O.C.c_int, O.C.c_double, O.C.c_int]
    rng = np.random.default_rng(3)
    ys = np.concatenate([rng.uniform(-5, 60, 500), np.arange(-3, 50) + 0.0, np.arange(-3, 50) + 0.5])
    cl = rng.integers(0, 50, ys.size)
    for mode in (0, 1):
        ref = [f(float(a), mode, 0.7, int(c)) for a, c in zip(ys, cl)]
        np.testing.assert_array_equal(O.h_regression(ys, cl, combine=1, offset=0.7, mode=mode), ref)


def test_classifier_rule_is_undefined_on_nan_or_infinite_logits():
    """A NaN or +infinite logit leaves softmax and arg-max undefined: the rule
    returns -1 and the batch rule falls back to the classic value (or 0);
    a -infinite logit is an ordinary class of probability zero."""
    f = O.lib().orc_h_classifier
    f.argtypes = [O.C.c_void_p, O.C.c_int, O.C.c_int, O.C.c_double]
    for bad in (np.nan, np.inf):
        z = np.ascontiguousarray([0.0, bad, 1.0])
        assert f(z.ctypes.data, 3, 3, 0.99) == -1 and f(z.ctypes.data, 3, 4, 0.0) == -1
    z = np.ascontiguousarray([-np.inf, 0.0, 0.0])
    assert f(z.ctypes.data, 3, 4, 0.0) == 1 and f(z.ctypes.data, 3, 3, 0.4) == 1
