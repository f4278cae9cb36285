"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds random-number generation and input construction only: it
contains none of the heuristic-evaluation or search arithmetic.  It produces

* splitmix64 streams (Steele, Lea & Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014), scalar and vectorised over numpy uint64;
* sliding-tile start states from random walks away from the goal (the paper
  builds its Rubik's cube instances from random walks, Experimental Setup; the
  sliding-tile instances here are walks too because the benchmark instance set
  the paper uses is not available);
* Rubik's cube random-walk *move sequences* (each side applies them with its own
  cube model);
* seeded weight files for the three network shapes;
* uneven batch-size lists.

Conventions (restated here because they define the inputs, not the method):

* Sliding tile, n x n: byte p of a state is the tile at cell p (row-major),
  tile 0 is the blank; the goal has tile p at cell p.  A move moves the blank:
  0 = up, 1 = left, 2 = right, 3 = down; the inverse of move a is 3 - a.
* Rubik's cube: move m turns face m // 3 (U, D, L, R, F, B) by
  (clockwise, counter-clockwise, half turn)[m % 3].
"""
from __future__ import annotations

import math
import struct

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


# ---------------------------------------------------------------- splitmix64
def splitmix64(state: int):
    """Scalar splitmix64: returns (new_state, output)."""
    state = (state + GOLDEN) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return state, z ^ (z >> 31)


class Stream:
    """A splitmix64 stream seeded with an integer."""

    def __init__(self, seed: int):
        self.s = seed & MASK64

    def next(self) -> int:
        self.s, z = splitmix64(self.s)
        return z

    def uniform(self) -> float:
        """Uniform double in [0, 1) from the top 53 bits."""
        return (self.next() >> 11) * (1.0 / (1 << 53))


def _sm64_vec(state: np.ndarray):
    """Vectorised splitmix64 over a uint64 array (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        state = state + np.uint64(GOLDEN)
        z = state
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return state, z


# ------------------------------------------------------------- sliding tile
def stp_goal(n: int) -> np.ndarray:
    return np.arange(n * n, dtype=np.uint8)


def stp_walks(n: int, seeds, lengths=None, length_base=None, length_span=None) -> np.ndarray:
    """Random walks from the goal, one splitmix64 stream per walk.

    seeds: iterable of stream seeds (one per walk).
    Either `lengths` (one per walk) or (length_base, length_span): then the
    first draw r of each stream sets the length to length_base + r % length_span.
    Each step lists the blank moves that stay on the board and do not undo the
    previous move, in move order, and takes entry r % k of that list.
    Returns uint8 [count, n*n].
    """
    seeds = np.asarray(list(seeds), dtype=np.uint64)
    cnt = seeds.shape[0]
    st = seeds.copy()
    if lengths is None:
        st, r = _sm64_vec(st)
        lengths = (np.uint64(length_base) + r % np.uint64(length_span)).astype(np.int64)
    lengths = np.asarray(lengths, dtype=np.int64)
    if lengths.ndim == 0:
        lengths = np.full(cnt, int(lengths), dtype=np.int64)
    states = np.tile(stp_goal(n), (cnt, 1))
    blank = np.zeros(cnt, dtype=np.int64)
    prev = np.full(cnt, -1, dtype=np.int64)
    rows = np.arange(cnt)
    dcell = np.array([-n, -1, 1, n], dtype=np.int64)
    for step in range(int(lengths.max(initial=0))):
        active = step < lengths
        br, bc = blank // n, blank % n
        ok = np.stack([br > 0, bc > 0, bc < n - 1, br < n - 1], axis=1)
        ok &= ~(np.arange(4)[None, :] == (3 - prev)[:, None])
        k = ok.sum(axis=1).astype(np.uint64)
        st2, r = _sm64_vec(st)
        st = np.where(active, st2, st)
        pick = (r % k).astype(np.int64)
        # index of the pick-th allowed move
        csum = np.cumsum(ok, axis=1) - 1
        move = np.argmax((csum == pick[:, None]) & ok, axis=1)
        dst = blank + dcell[move]
        a = rows[active]
        tile = states[a, dst[active]]
        states[a, blank[active]] = tile
        states[a, dst[active]] = 0
        blank = np.where(active, dst, blank)
        prev = np.where(active, move, prev)
    return states


def stp_walk_moves(n: int, seeds, lengths=None, length_base=None, length_span=None) -> np.ndarray:
    """The moves of the walks stp_walks takes (same streams, same draws), as
    int8 [count, max length] blank moves (0 up, 1 left, 2 right, 3 down), each
    row ended by -1 where the walk is shorter.  Only the blank's cell is
    tracked, so this is fast for millions of walks; applying the rows to the
    goal gives stp_walks' states.
    """
    seeds = np.asarray(list(seeds) if not isinstance(seeds, np.ndarray) else seeds, dtype=np.uint64)
    cnt = seeds.shape[0]
    st = seeds.copy()
    if lengths is None:
        st, r = _sm64_vec(st)
        lengths = (np.uint64(length_base) + r % np.uint64(length_span)).astype(np.int64)
    lengths = np.asarray(lengths, dtype=np.int64)
    if lengths.ndim == 0:
        lengths = np.full(cnt, int(lengths), dtype=np.int64)
    L = int(lengths.max(initial=0))
    # allowed[cell, prev + 1] lists the moves that stay on the board and do not
    # undo prev, in move order; kcount holds their number
    allowed = np.zeros((n * n, 5, 4), dtype=np.int8)
    kcount = np.zeros((n * n, 5), dtype=np.uint64)
    for cell in range(n * n):
        br, bc = divmod(cell, n)
        on = [br > 0, bc > 0, bc < n - 1, br < n - 1]
        for prev in range(-1, 4):
            ms = [m for m in range(4) if on[m] and m != 3 - prev]
            allowed[cell, prev + 1, :len(ms)] = ms
            kcount[cell, prev + 1] = len(ms)
    allowed_f = allowed.reshape(-1, 4)
    kcount_f = kcount.reshape(-1)
    dcell = np.array([-n, -1, 1, n], dtype=np.int16)
    out = np.full((cnt, max(L, 1)), -1, dtype=np.int8)
    # blocks of walks small enough to stay in cache; a finished walk's stream,
    # blank and previous move are never read again, so they are not masked
    for c0 in range(0, cnt, 1 << 16):
        c1 = min(cnt, c0 + (1 << 16))
        sc = st[c0:c1].copy()
        lc = lengths[c0:c1]
        key = np.zeros(c1 - c0, dtype=np.int64)  # blank * 5 + prev + 1
        blank = np.zeros(c1 - c0, dtype=np.int64)
        for step in range(int(lc.max(initial=0))):
            sc, r = _sm64_vec(sc)
            pick = (r % kcount_f[key]).astype(np.int64)
            move = allowed_f[key, pick]
            out[c0:c1, step] = np.where(step < lc, move, -1)
            blank += dcell[move]
            key = blank * 5 + move + 1
    return out


def _walk_moves_job(args):
    n, seeds, length_base, length_span = args
    return stp_walk_moves(n, seeds, length_base=length_base, length_span=length_span)


def stp_walk_moves_parallel(n: int, seeds, length_base: int, length_span: int, workers: int) -> np.ndarray:
    """stp_walk_moves split over `workers` fresh processes (spawned, so a
    parent that has initialised a GPU is not forked); same rows."""
    import multiprocessing as mp
    seeds = np.asarray(seeds, dtype=np.uint64)
    if workers <= 1 or len(seeds) < 65536:
        return stp_walk_moves(n, seeds, length_base=length_base, length_span=length_span)
    chunks = np.array_split(seeds, workers * 2)
    with mp.get_context("spawn").Pool(workers) as pool:
        parts = pool.map(_walk_moves_job, [(n, c, length_base, length_span) for c in chunks])
    out = np.full((len(seeds), max(p.shape[1] for p in parts)), -1, dtype=np.int8)
    r0 = 0
    for part in parts:
        out[r0:r0 + part.shape[0], :part.shape[1]] = part
        r0 += part.shape[0]
    return out


# --------------------------------------------------------------- Rubik's cube
def rc_walk_moves(seeds, lengths=None, length_base=None, length_span=None) -> list:
    """Random move sequences under canonical pruning, one stream per walk.

    After a turn of face F the next turn may not be of F, and may not be of the
    lower-indexed face of F's opposite pair when F is the higher one
    (pairs U/D, L/R, F/B).  Entry r % k of the allowed move list (ascending
    move index) is taken.  Returns a list of int lists.
    """
    out = []
    for seed in seeds:
        s = Stream(int(seed))
        if lengths is None:
            L = length_base + s.next() % length_span
        else:
            L = int(lengths[len(out)]) if hasattr(lengths, "__len__") else int(lengths)
        prev_face = -1
        seq = []
        for _ in range(L):
            allowed = [m for m in range(18)
                       if prev_face < 0 or (m // 3 != prev_face and
                                            not ((m // 3) % 2 == 0 and prev_face == m // 3 + 1))]
            m = allowed[s.next() % len(allowed)]
            seq.append(m)
            prev_face = m // 3
        out.append(seq)
    return out


def rc_walk_moves_array(seeds, lengths=None, length_base=None, length_span=None) -> np.ndarray:
    """Same as rc_walk_moves, vectorised; returns int8 [count, Lmax] padded with -1."""
    seeds = np.asarray(list(seeds), dtype=np.uint64)
    cnt = seeds.shape[0]
    st = seeds.copy()
    if lengths is None:
        st, r = _sm64_vec(st)
        lengths = (np.uint64(length_base) + r % np.uint64(length_span)).astype(np.int64)
    lengths = np.asarray(lengths, dtype=np.int64)
    if lengths.ndim == 0:
        lengths = np.full(cnt, int(lengths), dtype=np.int64)
    Lmax = int(lengths.max(initial=0))
    moves = np.full((cnt, Lmax), -1, dtype=np.int8)
    prev = np.full(cnt, -1, dtype=np.int64)
    face = np.arange(18) // 3
    for step in range(Lmax):
        active = step < lengths
        ok = (prev[:, None] < 0) | ((face[None, :] != prev[:, None]) &
                                    ~((face[None, :] % 2 == 0) & (prev[:, None] == face[None, :] + 1)))
        k = ok.sum(axis=1).astype(np.uint64)
        st2, r = _sm64_vec(st)
        st = np.where(active, st2, st)
        pick = (r % k).astype(np.int64)
        csum = np.cumsum(ok, axis=1) - 1
        m = np.argmax((csum == pick[:, None]) & ok, axis=1)
        moves[active, step] = m[active]
        prev = np.where(active, m // 3, prev)
    return moves


# ------------------------------------------------------------------ networks
# Network shapes of the three configurations (one-hot input P*S; hidden
# widths; residual blocks; outputs).  Domain ids: 0 = 3x3 tile, 1 = 4x4 tile,
# 2 = Rubik's cube.
NETS = {
    "stp3_small": dict(domain=0, n_in=81, dims=[128, 128], n_res=0, n_out=1, head_kind=0),
    "stp4_res": dict(domain=1, n_in=256, dims=[1000, 1000], n_res=2, n_out=1, head_kind=0),
    "rc_cls": dict(domain=2, n_in=324, dims=[2000, 1000], n_res=4, n_out=21, head_kind=1),
}

HBW_MAGIC = 0x31574248  # "HBW1" little-endian


def net_tensor_shapes(n_in, dims, n_res, n_out):
    """(name, rows, cols) of every tensor in file order; W stored [in][out]."""
    shapes = []
    prev = n_in
    for i, d in enumerate(dims):
        shapes.append((f"W{i}", prev, d))
        shapes.append((f"b{i}", 1, d))
        prev = d
    for r in range(n_res):
        shapes.append((f"R{r}a_W", prev, prev))
        shapes.append((f"R{r}a_b", 1, prev))
        shapes.append((f"R{r}b_W", prev, prev))
        shapes.append((f"R{r}b_b", 1, prev))
    shapes.append(("Wout", prev, n_out))
    shapes.append(("bout", 1, n_out))
    return shapes


def widened(net: str, width: int) -> dict:
    """The architecture of `net` with every hidden layer `width` wide (same depth):
    the model-size sweep varies the width only."""
    spec = dict(NETS[net])
    spec["dims"] = [width] * len(spec["dims"])
    return spec


def make_weights(net: str, seed: int, head_bias=0.0, scale=1.0, spec=None):
    """Seeded He-uniform weights U(+-sqrt(6/fan_in)) drawn in double precision
    and rounded to float32; hidden biases zero; output bias `head_bias`.
    Tensor t uses the splitmix64 stream seeded (seed << 20) + t.  `spec`
    overrides the architecture of `net` (see widened)."""
    spec = NETS[net] if spec is None else spec
    tensors = []
    for t, (name, rows, cols) in enumerate(net_tensor_shapes(spec["n_in"], spec["dims"],
                                                              spec["n_res"], spec["n_out"])):
        if name.startswith("b") or name.endswith("_b"):
            if name == "bout":
                hb = np.broadcast_to(np.asarray(head_bias, dtype=np.float64), (cols,))
                arr = hb.astype(np.float32).reshape(1, cols)
            else:
                arr = np.zeros((1, cols), dtype=np.float32)
        else:
            fan_in = spec["n_in"] if name == "W0" else rows
            # the first layer sees a one-hot vector with P ones; He-uniform on P keeps
            # the pre-activation scale of a dense input of the same norm
            if name == "W0":
                fan_in = {0: 9, 1: 16, 2: 54}[spec["domain"]]
            a = math.sqrt(6.0 / fan_in) * scale
            st = (np.uint64(((seed << 20) + t) & MASK64) +
                  np.arange(rows * cols, dtype=np.uint64) * np.uint64(GOLDEN))
            _, r = _sm64_vec(st)
            u = (r >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
            arr = ((2.0 * u - 1.0) * a).astype(np.float32).reshape(rows, cols)
        tensors.append((name, arr))
    return spec, tensors


def write_weights(path: str, net: str, seed: int, head_bias=0.0, scale=1.0, spec=None) -> dict:
    """Write the binary weight file.

    Layout (little-endian): u32 magic "HBW1", u32 version=1, u32 domain,
    u32 n_in, u32 n_dense, u32 dims[n_dense], u32 n_res, u32 n_out,
    u32 head_kind (0 regression, 1 classifier), then float32 tensors in the
    order of net_tensor_shapes: W [in][out] row-major, then b [out].
    """
    spec, tensors = make_weights(net, seed, head_bias, scale, spec)
    with open(path, "wb") as f:
        hdr = [HBW_MAGIC, 1, spec["domain"], spec["n_in"], len(spec["dims"])] + list(spec["dims"]) + \
              [spec["n_res"], spec["n_out"], spec["head_kind"]]
        f.write(struct.pack("<%dI" % len(hdr), *hdr))
        for _, arr in tensors:
            f.write(np.ascontiguousarray(arr, dtype="<f4").tobytes())
    return spec


# ------------------------------------------------------------- batch sizes
def uneven_batch_sizes(seed: int, count: int, lo=1, hi=16384) -> list:
    """Seeded log-uniform sizes on [lo, hi] followed by a fixed edge-case list."""
    s = Stream(seed)
    out = []
    for _ in range(count):
        u = s.uniform()
        out.append(int(min(hi, max(lo, math.floor(math.exp(math.log(lo) + u * (math.log(hi + 1) - math.log(lo))))))))
    return out + [1, 2, 3, 63, 64, 65, 1000, 4000, 8000, 16383, 16384]


# ---------------------------------------------------------- instance sets
def config_seeds(config: int, count: int = 100):
    """Instance i of configuration c uses stream seed 1000*c + i."""
    return [1000 * config + i for i in range(count)]


def stp3_instances(count=100):
    """8-puzzle starts: walks of 30 + r % 31 moves (30..60)."""
    return stp_walks(3, config_seeds(1, count), length_base=30, length_span=31)


def stp4_instances(count=100, length=200):
    return stp_walks(4, config_seeds(2, count), lengths=length)


def rc_instance_moves(count=100):
    """Rubik's cube starts: walks of 14 + r % 5 moves (14..18)."""
    return rc_walk_moves(config_seeds(3, count), length_base=14, length_span=5)


def throughput_seeds(count: int, base: int = 9009):
    return [(base << 32) + i for i in range(count)]


def write_weights_arrays(path: str, domain: int, n_in: int, dims, n_res: int, n_out: int, head_kind: int,
                         tensors) -> None:
    """Write a weight file from explicit float32 arrays (file order of
    net_tensor_shapes).  Used to build hand-designed networks whose outputs are
    known in closed form."""
    shapes = net_tensor_shapes(n_in, list(dims), n_res, n_out)
    assert len(shapes) == len(tensors)
    with open(path, "wb") as f:
        hdr = [HBW_MAGIC, 1, domain, n_in, len(dims)] + list(dims) + [n_res, n_out, head_kind]
        f.write(struct.pack("<%dI" % len(hdr), *hdr))
        for (name, r, c), arr in zip(shapes, tensors):
            a = np.asarray(arr, dtype="<f4").reshape(r, c)
            f.write(np.ascontiguousarray(a).tobytes())
