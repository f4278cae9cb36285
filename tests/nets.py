"""Hand-designed networks with closed-form outputs (test helpers)."""
import numpy as np

import synth


def md_net_tensors(n):
    """n x n sliding tile.  Layer 1 gathers, for tile t at cell p, its Manhattan
    contribution into unit 0 and nothing into unit 1 (bias 1), so x = (MD, 1).
    Dense layer: z = (MD, 5, 2 MD - 1).  Residual block: t = (0, 0, MD),
    x' = ReLU(x + t Wb + bb) = (3, 0, 2 MD - 1) for MD >= 1.
    Head: y = (3 + 0.5, (2 MD - 1) - 1) = (3.5, 2 MD - 2)."""
    P = n * n
    W0 = np.zeros((P * P, 2))
    for p in range(P):
        for t in range(1, P):
            W0[p * P + t, 0] = abs(p // n - t // n) + abs(p % n - t % n)
    b0 = np.array([0.0, 1.0])
    W1 = np.array([[1.0, 0.0, 2.0], [0.0, 5.0, -1.0]])
    b1 = np.zeros(3)
    Wa = np.zeros((3, 3)); Wa[0, 2] = 1.0
    ba = np.zeros(3)
    Wb = np.zeros((3, 3)); Wb[2, 0] = -1.0
    bb = np.array([3.0, -7.0, 0.0])
    Wo = np.array([[1.0, 0.0], [4.0, 0.0], [0.0, 1.0]])
    bo = np.array([0.5, -1.0])
    return [W0, b0, W1, b1, Wa, ba, Wb, bb, Wo, bo]


def write_md_net(path, n):
    dom = 0 if n == 3 else 1
    synth.write_weights_arrays(path, dom, n * n * n * n, [2, 3], 1, 2, 0, md_net_tensors(n))


def cube_misplaced_net_tensors(scale):
    """Cube regression net with y = scale x (number of non-centre stickers not
    showing their face's colour).  Sticker p sits on face p // 9 (centre
    9f + 4), whose colour is f.  Layer 1 gathers scale for each sticker whose
    colour differs from its face into unit 0; one identity dense layer; the
    head reads unit 0.  With a power-of-two scale every value is exact in
    float32.  A half turn or quarter turn moves 20 stickers, so the value
    changes by at most 20 x scale per move."""
    W0 = np.zeros((54 * 6, 2))
    for p in range(54):
        if p % 9 == 4:
            continue
        for c in range(6):
            if c != p // 9:
                W0[p * 6 + c, 0] = scale
    b0 = np.zeros(2)
    W1 = np.eye(2)
    b1 = np.zeros(2)
    Wo = np.array([[1.0], [0.0]])
    bo = np.zeros(1)
    return [W0, b0, W1, b1, Wo, bo]


def write_cube_misplaced_net(path, scale):
    synth.write_weights_arrays(path, 2, 324, [2, 2], 0, 1, 0, cube_misplaced_net_tensors(scale))
