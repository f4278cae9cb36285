"""Pins of the oracle's training arithmetic: the chain-rule gradient against
central finite differences of the loss (every parameter tensor), Adam against
its closed form, and descent of the loss under Adam."""
import numpy as np
import pytest

import oracle as O
import synth


def _small_net(path, dom, dims, n_res, seed):
    rng = np.random.default_rng(seed)
    P, S = {0: (9, 9), 1: (16, 16)}[dom]
    ts = []
    for name, r, c in synth.net_tensor_shapes(P * S, dims, n_res, 1):
        if name.startswith("b") or name.endswith("_b"):
            ts.append(rng.standard_normal(c) * 0.3 + (8.0 if name == "bout" else 0.0))
        else:
            ts.append(rng.standard_normal((r, c)) * np.sqrt(2.0 / (P if name == "W0" else r)))
    synth.write_weights_arrays(path, dom, P * S, dims, n_res, 1, 0, ts)
    return O.Net(path)


@pytest.mark.parametrize("asym", [False, True])
def test_gradient_matches_central_differences(tmp_path, asym):
    net = _small_net(str(tmp_path / "n.hbw"), 1, [12, 10], 2, 1)
    st = synth.stp_walks(4, range(16), lengths=30)
    labels = np.arange(16, dtype=np.float64) * 1.5 + 2.0
    loss, g, _ = net.loss_grad(st, labels, asym=asym, alpha=4.0)
    w0 = net.params()
    shapes = synth.net_tensor_shapes(256, [12, 10], 2, 1)
    rng = np.random.default_rng(7)
    off = 0
    h = 1e-6
    for name, r, c in shapes:
        size = r * c
        # layer 1 only receives gradient on the rows that the states select
        candidates = np.nonzero(g[off:off + size])[0] if name == "W0" else np.arange(size)
        for idx in rng.choice(candidates, size=min(6, len(candidates)), replace=False):
            wp = w0.copy(); wp[off + idx] += h
            wm = w0.copy(); wm[off + idx] -= h
            net.set_params(wp); lp, _, _ = net.loss_grad(st, labels, asym, 4.0)
            net.set_params(wm); lm, _, _ = net.loss_grad(st, labels, asym, 4.0)
            fd = (lp - lm) / (2 * h)
            an = g[off + idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, idx, fd, an)
        off += size
    net.set_params(w0)


def test_loss_matches_forward():
    import tempfile, os
    d = tempfile.mkdtemp()
    net = _small_net(os.path.join(d, "n.hbw"), 0, [16, 16], 1, 3)
    st = synth.stp3_instances(40)
    labels = np.linspace(0, 30, 40)
    loss, _, y = net.loss_grad(st, labels)
    np.testing.assert_allclose(y, net.forward(st)[:, 0], rtol=1e-12, atol=1e-12)
    assert abs(loss - np.mean((y - labels) ** 2)) <= 1e-10 * max(1.0, loss)
    lossa, _, _ = net.loss_grad(st, labels, asym=True, alpha=4.0)
    w = np.where(y > labels, 4.0, 1.0)
    assert abs(lossa - np.mean(w * (y - labels) ** 2)) <= 1e-10 * max(1.0, lossa)


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    w = np.array([1.0, 1.0, 1.0, 1.0])
    m = np.zeros(4); v = np.zeros(4)
    O.adam_step(w, g, m, v, 1, lr=0.1)
    # first step: m_hat = g, v_hat = g^2, update = lr * g / (|g| + eps)
    expect = 1.0 - 0.1 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(w, expect, rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
    # second step with the same gradient keeps m_hat = g
    O.adam_step(w, g, m, v, 2, lr=0.1)
    np.testing.assert_allclose(w, 1.0 - 0.2 * g / (np.abs(g) + 1e-8), rtol=1e-9)


def test_adam_descends_on_8puzzle_distances(tmp_path):
    net = _small_net(str(tmp_path / "n.hbw"), 0, [32, 32], 1, 5)
    d, _ = O.bfs8()
    st = O.all8()[::97]
    labels = d[[O.lib().orc_perm9_rank(np.ascontiguousarray(s).ctypes.data) for s in st]].astype(np.float64)
    w = net.params()
    m = np.zeros_like(w); v = np.zeros_like(w)
    first, _, _ = net.loss_grad(st, labels)
    for t in range(1, 61):
        loss, g, _ = net.loss_grad(st, labels)
        O.adam_step(w, g, m, v, t, lr=3e-3)
        net.set_params(w)
    last, _, _ = net.loss_grad(st, labels)
    assert last < 0.5 * first
