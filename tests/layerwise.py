"""Layer-by-layer ("teacher-forced") parity of the GPU forward pass.

For every stored activation tensor the library's value is read back
(hb_model_activation) and compared with the oracle's double-precision layer
applied to the library's own stored input of that layer.  Any float32
evaluation order of a layer with K inputs (the MFMA accumulation, the
epilogue's scale, bias and residual adds) is within

    E = gamma(K + 4) * A,  gamma(n) = n u / (1 - n u),  u = 2^-24,

of the exact value z, where A is the sum of |terms| (inputs times weights,
bias, residual): the standard bound for recursive summation (Higham, Accuracy
and Stability of Numerical Algorithms, 2nd ed., eq. 3.5), whatever the order.
ReLU and the storage rounding Q (bfloat16 round to nearest even, or e4m3
with the tensor's scale) are monotone, so every stored value must lie in
[Q(relu(z - E)), Q(relu(z + E))]; where that interval holds one value the
library must store exactly Q(relu(z)).  A "flip" is an element where the
library stored the other neighbour of a rounding boundary that lies within E
of z.  A row with no flip in any layer follows the oracle's quantised forward
pass (same operand rounding, double accumulation) exactly, so its output must
match the oracle's to the head's own float32 bound; only rows with a flip may
drift, and the tests check those against the oracle's rounding envelope.
"""
import numpy as np
import torch

import oracle as O

U = 2.0 ** -24
_E4M3 = None


def gamma(n):
    return n * U / (1 - n * U)


def _e4m3_table():
    global _E4M3
    if _E4M3 is None:
        _E4M3 = np.array([O.e4m3_decode(c) for c in range(256)], dtype=np.float64)
    return _E4M3


def _read(m, d_packed, a, n, width, prec):
    dt = {0: torch.float32, 1: torch.int16, 2: torch.uint8}[prec]
    d = torch.zeros((n, width), dtype=dt, device="cuda")
    m.activation(d_packed, a, d)
    return d.cpu().numpy()


def _decode(raw, prec, scale):
    if prec == 0:
        return raw.astype(np.float64)
    if prec == 1:
        return (raw.view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return _e4m3_table()[raw] * scale


def _quantise(v, prec, scale):
    if prec == 1:
        return O.bf16_round(v)
    return O.e4m3_round(v / scale) * scale


def teacher_forced(m, net, states, d_packed, prec, scales=None):
    """Walk the GPU forward pass layer by layer against the oracle.

    `net` is an oracle network, or the list of an ensemble's member networks
    (the library keeps the members' activations side by side, each padded to
    128 columns).  Asserts the per-element interval condition for every
    stored activation and returns a dict: `flip_rows` (rows with at least one
    flip), `stats` (per activation: elements, elements whose interval holds
    two values, flips), `y_tf` (the oracle's head on the GPU's last
    activation, n x n_out per member: a list for an ensemble) and `e_head`
    (its float32 error bound, same shape)."""
    nets = net if isinstance(net, (list, tuple)) else [net]
    n = states.shape[0]
    n_act = nets[0].n_act
    scales = np.ones(n_act) if scales is None else np.asarray(scales, dtype=np.float64)
    flip_rows = np.zeros(n, dtype=bool)
    stats = []
    stored = [dict() for _ in nets]
    for a in range(n_act):
        raw = None
        tot, two, nflip = 0, 0, 0
        for i, nt in enumerate(nets):
            if a == 0:
                z, A = nt.layer(0, states=states, mode=prec)
                K = 8 + {0: 9, 1: 16, 2: 54}[nt.domain]
            else:
                r = stored[i][a - 2] if nt.is_residual_output(a) else None
                z, A = nt.layer(a, x_in=stored[i][a - 1], r_in=r, mode=prec)
                K = stored[i][a - 1].shape[1]
            N = z.shape[1]
            npad = -(-N // 128) * 128
            if raw is None:
                raw = _read(m, d_packed, a, n, npad * len(nets), prec)
            g_all = _decode(raw[:, i * npad:(i + 1) * npad], prec, scales[a])
            assert np.all(g_all[:, N:] == 0), f"activation {a}, member {i}: padded columns are not zero"
            g = g_all[:, :N]
            E = gamma(K + 4) * A
            if prec == 0:
                v = np.maximum(z, 0.0)
                bad = np.abs(g - v) > E + U * np.abs(v)
                assert not bad.any(), (a, i, np.argwhere(bad)[:5], np.abs(g - v)[bad][:5], E[bad][:5])
            else:
                lo = _quantise(np.maximum(z - E, 0.0), prec, scales[a])
                hi = _quantise(np.maximum(z + E, 0.0), prec, scales[a])
                mid = _quantise(np.maximum(z, 0.0), prec, scales[a])
                bad = (g < lo) | (g > hi)
                assert not bad.any(), (a, i, np.argwhere(bad)[:5], g[bad][:5], lo[bad][:5], hi[bad][:5])
                flips = g != mid
                flip_rows |= flips.any(axis=1)
                two += int((lo != hi).sum())
                nflip += int(flips.sum())
            tot += g.size
            stored[i][a] = g
        stats.append((a, tot, two, nflip))
    y_tf, e_head = [], []
    for i, nt in enumerate(nets):
        zh, Ah = nt.layer(n_act, x_in=stored[i][n_act - 1], mode=prec)
        y_tf.append(zh)
        e_head.append(gamma(stored[i][n_act - 1].shape[1] + 4) * Ah + U * np.abs(zh))
    if not isinstance(net, (list, tuple)):
        y_tf, e_head = y_tf[0], e_head[0]
    return dict(flip_rows=flip_rows, stats=stats, y_tf=y_tf, e_head=e_head)
