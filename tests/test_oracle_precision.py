"""Pins of the oracle's reduced-precision forward pass (orc_net_forward modes 1
and 2) against what the number formats and the network definition fix.

* An independent float64 forward written here with numpy: layer 1 as a dense
  one-hot product, bfloat16 through torch's CPU float32 -> bfloat16 cast, OCP
  e4m3 from the format's definition (3 mantissa bits, exponent floor at 2^-6,
  ties to even via numpy's rint, saturation at 448).  It is compared element
  by element with the oracle on seeded nets of the 15-puzzle and cube shapes.
* Hand-built nets whose BF16 and FP8 outputs are derived by hand below: every
  activation and weight is placed on a value, or a tie, of the format, the FP8
  column maxima are 448 times a power of two, and the activation scales are
  not 1, so a dropped activation rounding, a weight scale taken along K instead
  of N, or an inverted activation scale changes the output.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth


# ------------------------------------------------------------ formats
def bf16(x):
    """float64 -> float32 (round to nearest even) -> bfloat16 (torch's CPU cast)."""
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32)
    return torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()


def e4m3(x):
    """OCP e4m3 rounding from the format's definition: a magnitude a (clamped at
    448) in binade [2^e, 2^(e+1)) has spacing 2^(e-3), with e no lower than -6
    (the subnormal spacing 2^-9); rint rounds halves to even, which for this
    format is the even code."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), 448.0)
    _, ex = np.frexp(np.where(a > 0, a, 1.0))  # a = m 2^ex with m in [0.5, 1)
    step = np.ldexp(1.0, np.maximum(ex - 1, -6) - 3)
    r = np.rint(a / step) * step
    return np.where(np.isnan(x), np.nan, np.copysign(r, x))


def test_independent_e4m3_matches_torch():
    rng = np.random.default_rng(8)
    x = (rng.uniform(-448, 448, 40000) * 10 ** rng.uniform(-4, 0, 40000)).astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(e4m3(x), ref)
    assert e4m3(np.array([1.0625, 1.1875, 136.0, 124.0, 600.0]))[:].tolist() == [1.0, 1.25, 128.0, 128.0, 448.0]


# ------------------------------------------------------------ reference forward
def read_hbw(path):
    with open(path, "rb") as f:
        raw = f.read()
    u = np.frombuffer(raw, dtype="<u4")
    domain, n_in, nd = int(u[2]), int(u[3]), int(u[4])
    dims = [int(v) for v in u[5:5 + nd]]
    n_res, n_out, head_kind = (int(v) for v in u[5 + nd:8 + nd])
    off = 4 * (8 + nd)
    ts = []
    for _, r, c in synth.net_tensor_shapes(n_in, dims, n_res, n_out):
        ts.append(np.frombuffer(raw, dtype="<f4", count=r * c, offset=off).astype(np.float64).reshape(r, c))
        off += 4 * r * c
    return dict(domain=domain, n_in=n_in, dims=dims, n_res=n_res, n_out=n_out, head_kind=head_kind, T=ts)


def onehot(states, S):
    n, P = states.shape
    x = np.zeros((n, P * S))
    x[np.arange(n)[:, None], np.arange(P)[None, :] * S + states.astype(np.int64)] = 1.0
    return x


def ref_forward(net, states, mode, act_scale=None):
    """Float64 forward with the operand rounding of mode 0 (none), 1 (bf16
    weights and stored activations) or 2 (fp8 matrix layers: e4m3 weights with
    a float32 scale max_k |W[k, n]| / 448 per output column n, e4m3 activations
    under a per-tensor scale; layer-1 and head weights in bf16)."""
    T = net["T"]
    S = net["n_in"] // states.shape[1]
    nd, nr = len(net["dims"]), net["n_res"]
    heads = len(T) - 2

    def weight(t):
        w = T[t]
        if mode == 0:
            return w
        if mode == 1 or t == 0 or t == heads:
            return bf16(w)
        s = (np.abs(w).max(axis=0) / 448.0).astype(np.float32).astype(np.float64)  # per output column
        safe = np.where(s > 0, s, 1.0)
        q = e4m3((w / safe).astype(np.float32).astype(np.float64))
        return np.where(s > 0, q * s, 0.0)

    acts = []

    def store(v):
        a = len(acts)
        acts.append(v.max() if v.size else 0.0)
        if mode == 1:
            return bf16(v)
        if mode == 2:
            return e4m3(v / act_scale[a]) * act_scale[a]
        return v

    x = store(np.maximum(onehot(states, S) @ weight(0) + T[1][0], 0.0))
    t = 2
    for _ in range(1, nd):
        x = store(np.maximum(x @ weight(t) + T[t + 1][0], 0.0))
        t += 2
    for _ in range(nr):
        u = store(np.maximum(x @ weight(t) + T[t + 1][0], 0.0))
        x = store(np.maximum(x + u @ weight(t + 2) + T[t + 3][0], 0.0))
        t += 4
    return x @ weight(t) + T[t + 1][0], np.array(acts)


def ref_calibrate(net, states):
    """Smallest power of two a with max activation / a <= 448, per tensor."""
    _, mx = ref_forward(net, states, 0)
    out = []
    for m in mx:
        if not m > 0:
            out.append(1.0)
            continue
        e = int(np.ceil(np.log2(m / 448.0)))
        while 448.0 * 2.0 ** e < m:
            e += 1
        while 448.0 * 2.0 ** (e - 1) >= m:
            e -= 1
        out.append(2.0 ** e)
    return np.array(out)


def _cube_states(n, base):
    mv = synth.rc_walk_moves_array(synth.throughput_seeds(n, base), length_base=20, length_span=11)
    return O.apply_moves(2, mv)


def _states(name, n, base):
    if name == "rc_cls":
        return _cube_states(n, base)
    return synth.stp_walks(4, synth.throughput_seeds(n, base), lengths=200)


@pytest.mark.parametrize("name,mode", [("stp4_res", 1), ("stp4_res", 2), ("rc_cls", 1), ("rc_cls", 2)])
def test_reduced_precision_forward_matches_independent_reference(net_files, name, mode):
    """Catches: a stored activation left unrounded, a rounding on the wrong
    tensor (biases, layer 1's float32 sum, the residual sum before ReLU), an
    fp8 scale along the wrong axis or inverted, a head kept in fp8."""
    path = net_files[name]
    net = read_hbw(path)
    onet = O.Net(path)
    st = _states(name, 24, 5151)
    scales = None
    if mode == 2:
        calib = _states(name, 96, 6161)
        scales = ref_calibrate(net, calib)
        np.testing.assert_array_equal(onet.calibrate(calib), scales)
    y_ref, _ = ref_forward(net, st, mode, scales)
    y = onet.forward(st, mode=mode, act_scale=scales)
    np.testing.assert_allclose(y, y_ref, rtol=1e-11, atol=1e-11 * np.abs(y_ref).max())
    # and the rounding matters at this size: the unrounded forward is farther away
    y0 = onet.forward(st)
    assert np.abs(y0 - y_ref).max() > 1e3 * 1e-11 * np.abs(y_ref).max()


# ------------------------------------------------------------ hand-built nets
def _write(path, b1, W2, b2, Wa, ba, Wb, bb, wo, bo):
    """8-puzzle-domain net 81 -> 3 -> 3 -> one residual block -> 1, layer-1
    weights zero (so x1 = ReLU(b1) for every state)."""
    ts = [np.zeros((81, 3)), np.array(b1), np.array(W2), np.array(b2), np.array(Wa), np.array(ba),
          np.array(Wb), np.array(bb), np.array(wo).reshape(3, 1), np.array([bo])]
    synth.write_weights_arrays(path, 0, 81, [3, 3], 1, 1, 0, ts)


def test_fp8_forward_closed_form(tmp_path):
    """Worked by hand, with activation scales (2^-7, 2^-5, 2^-6, 2^-4):
    x1 = (1.125, 3, 1.0625): /2^-7 = (144, 384, 136) -> (144, 384, 128 (tie to
      the even code)) -> x1q = (1.125, 3, 1).  (Scale inverted: 1.125 * 2^-7 is
      a subnormal 4.5 * 2^-9 -> 4 * 2^-9, giving 1.0 for the first element.)
    W2 columns: col 0 (448, 1.0625, 0): scale 1, codes (448, 1 (tie), 0);
      col 1 (3.5, -0.1484375, 0.5): scale 2^-7, W/s = (448, -19 -> -20 (tie to
      even), 64) -> (3.5, -0.15625, 0.5); col 2 all zero (scale 0).
      (Rows instead of columns: row 1's scale 1.0625/448 keeps 1.0625.)
    z2 = (504 + 3 - 503, 3.9375 - 0.46875 + 0.5 - 0.09375, 0.75) = (4, 3.875, 0.75);
      /2^-5 = (128, 124, 24) -> (128, 128 (tie across the binade: even), 24)
      -> x2q = (4, 4, 0.75).
    t = ReLU(0.875 x2q) = (3.5, 3.5, 0.65625) (W_a = 0.875 I: scale 2^-9, exact);
      /2^-6 = (224, 224, 42) -> (224, 224, 40 (tie to even)) -> tq = (3.5, 3.5, 0.625).
    x3 = ReLU(x2q + 0.4375 tq) = (5.53125, 5.53125, 1.0234375);
      /2^-4 = (88.5, 88.5, 16.375) -> (88, 88, 16) -> (5.5, 5.5, 1).
    y = (1, 2, 4) . x3q + 0.125 = 5.5 + 11 + 4 + 0.125 = 20.625."""
    path = str(tmp_path / "fp8.hbw")
    _write(path, [1.125, 3.0, 1.0625],
           [[448.0, 3.5, 0.0], [1.0625, -0.1484375, 0.0], [0.0, 0.5, 0.0]], [-503.0, -0.09375, 0.75],
           np.eye(3) * 0.875, [0.0, 0.0, 0.0], np.eye(3) * 0.4375, [0.0, 0.0, 0.0], [1.0, 2.0, 4.0], 0.125)
    net = O.Net(path)
    st = synth.stp_walks(3, range(5), lengths=12)
    scales = [2.0 ** -7, 2.0 ** -5, 2.0 ** -6, 2.0 ** -4]
    y = net.forward(st, mode=2, act_scale=scales)[:, 0]
    np.testing.assert_array_equal(y, 20.625)
    # unrounded, the same net gives another value (all terms are dyadic: exact in float64)
    x1 = np.array([1.125, 3.0, 1.0625])
    W2 = np.array([[448.0, 3.5, 0.0], [1.0625, -0.1484375, 0.0], [0.0, 0.5, 0.0]])
    x2 = np.maximum(x1 @ W2 + [-503.0, -0.09375, 0.75], 0)
    x3 = np.maximum(x2 + 0.4375 * np.maximum(0.875 * x2, 0), 0)
    np.testing.assert_array_equal(net.forward(st, mode=0)[:, 0], x3 @ [1.0, 2.0, 4.0] + 0.125)
    assert x3 @ [1.0, 2.0, 4.0] + 0.125 != 20.625


def test_bf16_forward_closed_form(tmp_path):
    """Worked by hand (bfloat16 spacing at 1 is 2^-7, at 2 it is 2^-6):
    x1 = (1 + 2^-8, 1 + 3 2^-8, 1 + 2^-8 + 2^-20) -> (1 (tie to even),
      1 + 2^-6 (tie to even), 1 + 2^-7 (above the tie)).
    W2 = diag(1 + 2^-8, 1, 1) -> identity (tie to even); b2 = (2^-8, 0, 2^-8):
      z2 = (1 + 2^-8, 1 + 2^-6, 1 + 2^-7 + 2^-8) -> (1, 1 + 2^-6, 1 + 2^-6).
    t = ReLU(x2 + (0, 2^-8, 0)) = (1, 1 + 2^-6 + 2^-8, 1 + 2^-6) -> (1, 1 + 2^-6, 1 + 2^-6).
    x3 = ReLU(x2 + t + (2^-7, 0, 0)) = (2 + 2^-7, 2 + 2^-5, 2 + 2^-5) -> (2, 2 + 2^-5, 2 + 2^-5).
    head (1, 2, 1 + 2^-8) -> (1, 2, 1): y = 2 + 4.0625 + 2.03125 = 8.09375."""
    path = str(tmp_path / "bf16.hbw")
    e8 = 2.0 ** -8
    _write(path, [1 + e8, 1 + 3 * e8, 1 + e8 + 2.0 ** -20],
           np.diag([1 + e8, 1.0, 1.0]), [e8, 0.0, e8],
           np.eye(3), [0.0, e8, 0.0], np.eye(3), [2.0 ** -7, 0.0, 0.0], [1.0, 2.0, 1 + e8], 0.0)
    net = O.Net(path)
    st = synth.stp_walks(3, range(5), lengths=12)
    np.testing.assert_array_equal(net.forward(st, mode=1)[:, 0], 8.09375)
    assert net.forward(st, mode=0)[0, 0] != 8.09375


# ------------------------------------------------ one layer at a time
@pytest.mark.parametrize("name", ["stp4_res", "rc_cls"])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_layer_by_layer_composes_to_the_forward_pass(net_files, name, mode):
    """orc_net_layer (used for the library's layer-by-layer parity) applied
    layer after layer, with ReLU and the storage rounding between layers (bf16
    and e4m3 here from the format definitions above), gives the oracle's
    forward pass; its sum of |terms| bounds |z|.  A layer that took the wrong
    tensor, skipped the residual input or the bias fails this."""
    net = O.Net(net_files[name])
    dom = 2 if name == "rc_cls" else 1
    if dom == 2:
        mv = synth.rc_walk_moves_array(synth.throughput_seeds(6, 31), length_base=20, length_span=11)
        st = O.apply_moves(2, mv)
    else:
        st = synth.stp_walks(4, synth.throughput_seeds(6, 31), lengths=200)
    scales = net.calibrate(st) if mode == 2 else np.ones(net.n_act)
    acts = {}
    for a in range(net.n_act):
        if a == 0:
            z, A = net.layer(0, states=st, mode=mode)
        else:
            r = acts[a - 2] if net.is_residual_output(a) else None
            z, A = net.layer(a, x_in=acts[a - 1], r_in=r, mode=mode)
        assert np.all(A >= np.abs(z) * (1 - 1e-12))
        v = np.maximum(z, 0.0)
        acts[a] = v if mode == 0 else bf16(v) if mode == 1 else e4m3(v / scales[a]) * scales[a]
    y, _ = net.layer(net.n_act, x_in=acts[net.n_act - 1], mode=mode)
    ref = net.forward(st, mode=mode, act_scale=scales if mode == 2 else None)
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-9)
    with pytest.raises(ValueError):
        net.layer(net.n_act + 1, x_in=acts[0])
