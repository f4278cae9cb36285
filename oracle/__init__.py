"""Python access to the plain-C double-precision oracle.

TEST INFRASTRUCTURE ONLY.  The oracle is a slow, obviously-correct CPU model of
the batched neural-heuristic search (domains, network forward pass, output
rules, reduced-precision emulation, serial IDA* and Budgeted Tree Search,
training gradients).  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the library never does.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

STP3, STP4, RUBIK = 0, 1, 2
STATE_LEN = {STP3: 9, STP4: 16, RUBIK: 54}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b  # noqa: F401
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


class HSpec(C.Structure):
    _fields_ = [("kind", C.c_int), ("table8", C.POINTER(C.c_int32)), ("pdb_k", C.c_int),
                ("pdb", C.POINTER(C.c_uint8)), ("apdb_groups", C.c_int), ("apdb_tiles", C.POINTER(C.c_int32)),
                ("apdb_tables", C.POINTER(C.c_uint8))]


class Iter(C.Structure):
    _fields_ = [("bound", C.c_int32), ("expanded", C.c_int64), ("generated", C.c_int64),
                ("complete", C.c_int32), ("found", C.c_int32), ("limit", C.c_int64)]


class IterReal(C.Structure):
    _fields_ = [("bound", C.c_double), ("expanded", C.c_int64), ("generated", C.c_int64),
                ("complete", C.c_int32), ("found", C.c_int32), ("limit", C.c_int64)]


def _declare(L):
    vp = C.c_void_p
    L.orc_apply_seq_batch.argtypes = [C.c_int, vp, C.c_int64, C.c_int, vp]
    L.orc_apply.argtypes = [C.c_int, vp, C.c_int, vp]
    L.orc_manhattan_batch.argtypes = [C.c_int, vp, C.c_int64, vp]
    L.orc_bfs8.argtypes = [vp]
    L.orc_bfs8.restype = C.c_int64
    L.orc_all8.argtypes = [vp]
    L.orc_all8.restype = C.c_int64
    L.orc_perm9_rank.argtypes = [vp]
    L.orc_perm9_rank.restype = C.c_int64
    L.orc_corner_pdb.argtypes = [C.c_int, vp]
    L.orc_corner_pdb.restype = C.c_int64
    L.orc_corner_k_size.argtypes = [C.c_int]
    L.orc_corner_k_size.restype = C.c_int64
    L.orc_corner_k_index_batch.argtypes = [vp, C.c_int64, C.c_int, vp]
    L.orc_apdb_group.argtypes = [C.c_int, vp, vp]
    L.orc_apdb_h_batch.argtypes = [vp, C.c_int64, C.c_int, vp, vp, vp]
    L.orc_apdb_group_lookup.argtypes = [C.c_int, vp, vp, vp, C.c_int64, vp]
    L.orc_bf16_round_array.argtypes = [vp, C.c_int64, vp]
    L.orc_e4m3_round_array.argtypes = [vp, C.c_int64, vp]
    L.orc_e4m3_decode.argtypes = [C.c_int]
    L.orc_e4m3_decode.restype = C.c_double
    L.orc_e4m3_encode.argtypes = [C.c_double]
    L.orc_e4m3_encode.restype = C.c_int
    L.orc_net_load.argtypes = [C.c_char_p]
    L.orc_net_load.restype = vp
    L.orc_net_free.argtypes = [vp]
    L.orc_net_info.argtypes = [vp, vp]
    L.orc_net_n_act.argtypes = [vp]
    L.orc_net_forward.argtypes = [vp, vp, C.c_int64, C.c_int, vp, vp, vp]
    L.orc_net_calibrate.argtypes = [vp, vp, C.c_int64, vp]
    L.orc_net_fp8_col_scales.argtypes = [vp, C.c_int, vp]
    L.orc_net_layer_width.argtypes = [vp, C.c_int]
    L.orc_net_layer1.argtypes = [vp, vp, C.c_int64, C.c_int, vp, vp]
    L.orc_net_layer.argtypes = [vp, C.c_int, vp, vp, C.c_int64, C.c_int, vp, vp]
    L.orc_h_batch.argtypes = [vp, vp, C.c_int64, C.c_int, C.c_double, C.c_double, vp, vp]
    L.orc_ida.argtypes = [C.c_int, vp, C.POINTER(HSpec), C.c_int, C.c_int, C.c_int64,
                          C.POINTER(Iter), C.POINTER(C.c_int), C.POINTER(C.c_int32), vp, C.POINTER(C.c_int)]
    L.orc_bts.argtypes = [C.c_int, vp, C.POINTER(HSpec), C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int,
                          C.c_int64, C.POINTER(Iter), C.POINTER(C.c_int), C.POINTER(C.c_int32), vp,
                          C.POINTER(C.c_int)]
    L.orc_ida_real.argtypes = [vp, vp, C.c_int, C.c_int, C.c_int64, C.POINTER(IterReal), C.POINTER(C.c_int),
                               C.POINTER(C.c_int32), vp, C.POINTER(C.c_int)]
    L.orc_bts_real.argtypes = [vp, vp, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64,
                               C.POINTER(IterReal), C.POINTER(C.c_int), C.POINTER(C.c_int32), vp, C.POINTER(C.c_int)]
    L.orc_ida_real_net.argtypes = [vp, C.c_double, vp, C.c_int, C.c_int, C.c_int64, C.POINTER(IterReal),
                                   C.POINTER(C.c_int), C.POINTER(C.c_int32), vp, C.POINTER(C.c_int)]
    L.orc_bts_real_net.argtypes = [vp, C.c_double, vp, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64,
                                   C.POINTER(IterReal), C.POINTER(C.c_int), C.POINTER(C.c_int32), vp,
                                   C.POINTER(C.c_int)]
    L.orc_train_grad.argtypes = [vp, vp, C.c_int64, vp, C.c_int, C.c_double, vp, vp]
    L.orc_train_grad.restype = C.c_double
    L.orc_adam_step.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_double, C.c_double, C.c_double,
                                C.c_double, C.c_int]
    L.orc_net_param_count.argtypes = [vp]
    L.orc_net_get_params.argtypes = [vp, vp]
    L.orc_net_set_params.argtypes = [vp, vp]


# ----------------------------------------------------------------- domains
def goal(domain):
    if domain == RUBIK:
        return np.repeat(np.arange(6, dtype=np.uint8), 9)
    n = 3 if domain == STP3 else 4
    return np.arange(n * n, dtype=np.uint8)


def apply(domain, state, move):
    s = np.ascontiguousarray(state, dtype=np.uint8)
    out = np.zeros_like(s)
    ok = lib().orc_apply(domain, s.ctypes.data, int(move), out.ctypes.data)
    return out if ok else None


def apply_moves(domain, moves):
    """moves: int array [count, L] padded with -1 (applied to the goal)."""
    m = np.ascontiguousarray(moves, dtype=np.int8)
    if m.ndim == 1:
        m = m[None, :]
    out = np.zeros((m.shape[0], STATE_LEN[domain]), dtype=np.uint8)
    ok = lib().orc_apply_seq_batch(domain, m.ctypes.data, m.shape[0], m.shape[1], out.ctypes.data)
    if not ok:
        raise ValueError("invalid move sequence")
    return out


def manhattan(domain, states):
    s = np.ascontiguousarray(states, dtype=np.uint8).reshape(-1, STATE_LEN[domain])
    out = np.zeros(s.shape[0], dtype=np.int32)
    lib().orc_manhattan_batch(domain, s.ctypes.data, s.shape[0], out.ctypes.data)
    return out


def bfs8():
    d = np.zeros(362880, dtype=np.int8)
    n = lib().orc_bfs8(d.ctypes.data)
    return d, n


def all8():
    out = np.zeros((181440, 9), dtype=np.uint8)
    n = lib().orc_all8(out.ctypes.data)
    return out[:n]


def perm9_rank(states):
    s = np.ascontiguousarray(states, dtype=np.uint8).reshape(-1, 9)
    return np.array([lib().orc_perm9_rank(s[i].ctypes.data) for i in range(s.shape[0])], dtype=np.int64)


def corner_pdb(k):
    size = lib().orc_corner_k_size(k)
    t = np.zeros(size, dtype=np.uint8)
    reached = lib().orc_corner_pdb(k, t.ctypes.data)
    return t, reached


def apdb(groups):
    """Additive 15-puzzle PDB (groups of at most 4 tiles): (tiles [G][4] with -1
    padding, tables [G][65536]) for apdb_h and the searches."""
    G = len(groups)
    tiles = np.full((G, 4), -1, dtype=np.int32)
    tables = np.full((G, 65536), 255, dtype=np.uint8)
    for g, ts in enumerate(groups):
        ts = sorted(int(t) for t in ts)
        if not 1 <= len(ts) <= 4:
            raise ValueError("groups of 1 to 4 tiles")
        tiles[g, :len(ts)] = ts
        t = np.zeros(16 ** len(ts), dtype=np.uint8)
        if not lib().orc_apdb_group(len(ts), tiles[g].ctypes.data, t.ctypes.data):
            raise ValueError("bad group")
        tables[g, :t.size] = t
    return tiles, tables


def apdb_group_table(group):
    """One group's table (1 to 6 tiles), indexed by sum of cell * 16^i over
    the group's tiles in ascending order: (tiles, table)."""
    ts = np.array(sorted(int(t) for t in group), dtype=np.int32)
    if not 1 <= ts.size <= 6:
        raise ValueError("groups of 1 to 6 tiles")
    t = np.zeros(16 ** ts.size, dtype=np.uint8)
    if not lib().orc_apdb_group(ts.size, ts.ctypes.data, t.ctypes.data):
        raise ValueError("bad group or out of memory")
    return ts, t


def apdb_group_lookup(group_table, states):
    ts, t = group_table
    s = np.ascontiguousarray(states, dtype=np.uint8).reshape(-1, 16)
    out = np.zeros(s.shape[0], dtype=np.int32)
    lib().orc_apdb_group_lookup(ts.size, ts.ctypes.data, t.ctypes.data, s.ctypes.data, s.shape[0], out.ctypes.data)
    return out


def apdb_h(states, spec):
    tiles, tables = spec
    s = np.ascontiguousarray(states, dtype=np.uint8).reshape(-1, 16)
    out = np.zeros(s.shape[0], dtype=np.int32)
    lib().orc_apdb_h_batch(s.ctypes.data, s.shape[0], tiles.shape[0], tiles.ctypes.data, tables.ctypes.data,
                           out.ctypes.data)
    return out


def corner_index(states, k):
    s = np.ascontiguousarray(states, dtype=np.uint8).reshape(-1, 54)
    out = np.zeros(s.shape[0], dtype=np.int64)
    if not lib().orc_corner_k_index_batch(s.ctypes.data, s.shape[0], k, out.ctypes.data):
        raise ValueError("not a valid cube state")
    return out


# ------------------------------------------------------------- rounding
def bf16_round(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().orc_bf16_round_array(x.ctypes.data, x.size, out.ctypes.data)
    return out


def e4m3_round(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().orc_e4m3_round_array(x.ctypes.data, x.size, out.ctypes.data)
    return out


def e4m3_decode(code):
    return lib().orc_e4m3_decode(int(code))


def e4m3_encode(x):
    return lib().orc_e4m3_encode(float(x))


# ---------------------------------------------------------------- network
class Net:
    """Double-precision network loaded from a weight file."""

    def __init__(self, path):
        self._h = lib().orc_net_load(path.encode())
        if not self._h:
            raise ValueError(f"cannot load weights {path}")
        info = np.zeros(16, dtype=np.int32)
        lib().orc_net_info(self._h, info.ctypes.data)
        self.domain, self.n_in, self.n_dense, self.n_res, self.n_out, self.head_kind, self.nt = map(int, info[:7])
        self.dims = [int(v) for v in info[7:7 + self.n_dense]]
        self.n_act = lib().orc_net_n_act(self._h)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_net_free(self._h)
            self._h = None

    def forward(self, states, mode=0, act_scale=None, want_act_max=False):
        s = np.ascontiguousarray(states, dtype=np.uint8).reshape(-1, STATE_LEN[self.domain])
        y = np.zeros((s.shape[0], self.n_out), dtype=np.float64)
        sc = None if act_scale is None else np.ascontiguousarray(act_scale, dtype=np.float64)
        am = np.zeros(self.n_act, dtype=np.float64) if want_act_max else None
        lib().orc_net_forward(self._h, s.ctypes.data, s.shape[0], mode,
                              None if sc is None else sc.ctypes.data, y.ctypes.data,
                              None if am is None else am.ctypes.data)
        return (y, am) if want_act_max else y

    def calibrate(self, states):
        s = np.ascontiguousarray(states, dtype=np.uint8).reshape(-1, STATE_LEN[self.domain])
        out = np.zeros(self.n_act, dtype=np.float64)
        lib().orc_net_calibrate(self._h, s.ctypes.data, s.shape[0], out.ctypes.data)
        return out

    def is_residual_output(self, a):
        """True for the activation a residual block's second layer writes."""
        return self.n_dense <= a < self.n_act and (a - self.n_dense) % 2 == 1

    def layer(self, a, x_in=None, r_in=None, states=None, mode=0):
        """One layer in double precision from given (dequantised) inputs:
        returns (z, A), the pre-activation and the sum of |terms| (inputs times
        weights, bias, residual) that bounds any float32 evaluation's error.
        a = 0 gathers layer 1 from `states`; 1..n_act-1 are the matrix layers
        (r_in: the block input for a residual block's second layer); a = n_act
        is the head."""
        N = lib().orc_net_layer_width(self._h, a)
        if N == 0:
            raise ValueError(f"no layer for activation index {a}")
        if a == 0:
            s = np.ascontiguousarray(states, dtype=np.uint8).reshape(-1, STATE_LEN[self.domain])
            n = s.shape[0]
            z = np.zeros((n, N)); A = np.zeros((n, N))
            lib().orc_net_layer1(self._h, s.ctypes.data, n, mode, z.ctypes.data, A.ctypes.data)
            return z, A
        x = np.ascontiguousarray(x_in, dtype=np.float64)
        n = x.shape[0]
        if self.is_residual_output(a) != (r_in is not None):
            raise ValueError("r_in is required exactly for a residual block's second layer")
        r = None if r_in is None else np.ascontiguousarray(r_in, dtype=np.float64)
        z = np.zeros((n, N)); A = np.zeros((n, N))
        lib().orc_net_layer(self._h, a, x.ctypes.data, None if r is None else r.ctypes.data, n, mode,
                            z.ctypes.data, A.ctypes.data)
        return z, A

    def fp8_col_scales(self, tensor_index):
        cols = None
        # tensor shapes follow the file order; column count from dims
        out = np.zeros(4096, dtype=np.float32)
        lib().orc_net_fp8_col_scales(self._h, tensor_index, out.ctypes.data)
        return out if cols is None else out[:cols]

    # ------------------------------------------------------------ training
    def n_params(self):
        return lib().orc_net_param_count(self._h)

    def params(self):
        out = np.zeros(self.n_params(), dtype=np.float64)
        lib().orc_net_get_params(self._h, out.ctypes.data)
        return out

    def set_params(self, flat):
        f = np.ascontiguousarray(flat, dtype=np.float64)
        assert f.size == self.n_params()
        lib().orc_net_set_params(self._h, f.ctypes.data)

    def loss_grad(self, states, labels, asym=False, alpha=1.0):
        """(loss, flat gradient in file order, y) of the squared-error loss."""
        s = np.ascontiguousarray(states, dtype=np.uint8).reshape(-1, STATE_LEN[self.domain])
        t = np.ascontiguousarray(labels, dtype=np.float64)
        g = np.zeros(self.n_params(), dtype=np.float64)
        y = np.zeros(s.shape[0], dtype=np.float64)
        loss = lib().orc_train_grad(self._h, s.ctypes.data, s.shape[0], t.ctypes.data, int(asym), alpha,
                                    g.ctypes.data, y.ctypes.data)
        return loss, g, y

    def h(self, y, mode=0, q=0.99, offset=0.0, classic=None):
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1, self.n_out)
        out = np.zeros(y.shape[0], dtype=np.int32)
        cl = None if classic is None else np.ascontiguousarray(classic, dtype=np.int32)
        lib().orc_h_batch(self._h, y.ctypes.data, y.shape[0], mode, q, offset,
                          None if cl is None else cl.ctypes.data, out.ctypes.data)
        return out


# ----------------------------------------------------------------- ensembles
ENS_MIN, ENS_SUM = 0, 1


def ensemble_forward(nets, states, rule, mode=0, act_scales=None):
    """Output of an ensemble of one-output regression networks: the minimum of
    the members' outputs (the related work's admissibility device) or their sum
    in member order (learned residuals added together, as in the experiments'
    sliding-tile heuristic).  act_scales: one FP8 scale vector per member."""
    ys = [net.forward(states, mode=mode, act_scale=None if act_scales is None else act_scales[i])[:, 0]
          for i, net in enumerate(nets)]
    out = ys[0].copy()
    for y in ys[1:]:
        out = np.minimum(out, y) if rule == ENS_MIN else out + y
    return out


def h_regression(y, md=None, combine=0, offset=0.0, mode=0):
    """Regression output rule, written out: v = floor(y - offset) (mode 1:
    round half to even), clamped at 0 and at 1e9; then with Manhattan distance md:
    combine 1 min(v, md), 2 max(v, md), 3 md + v.  A non-finite y gives md (0
    without it)."""
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros(y.shape[0], dtype=np.int64)
    for i, yi in enumerate(y):
        c = None if md is None or combine == 0 else int(md[i])
        if not np.isfinite(yi):
            out[i] = c if c is not None else 0
            continue
        t = yi - offset
        r = np.floor(t)
        if mode == 1:
            frac = t - r
            if frac > 0.5 or (frac == 0.5 and r % 2 != 0):
                r += 1
        v = int(min(max(r, 0.0), 1e9))
        if c is not None:
            v = min(v, c) if combine == 1 else max(v, c) if combine == 2 else c + min(v, int(1e9) - c)
        out[i] = v
    return out


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays."""
    for a in (w, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam_step(w.ctypes.data, g.ctypes.data, m.ctypes.data, v.ctypes.data, w.size, lr, b1, b2, eps, t)


# ----------------------------------------------------------------- search
H_ZERO, H_MD, H_TABLE8, H_PDB, H_APDB = 0, 1, 2, 3, 4


def _hspec(kind, table8=None, pdb=None, pdb_k=0, apdb=None):
    hs = HSpec()
    hs.kind = kind
    keep = []
    if apdb is not None:
        tiles, tables = apdb
        keep += [tiles, tables]
        hs.apdb_groups = tiles.shape[0]
        hs.apdb_tiles = _p(tiles, C.c_int32)
        hs.apdb_tables = _p(tables, C.c_uint8)
    if table8 is not None:
        t = np.ascontiguousarray(table8, dtype=np.int32)
        keep.append(t)
        hs.table8 = _p(t, C.c_int32)
    if pdb is not None:
        keep.append(pdb)
        hs.pdb = _p(pdb, C.c_uint8)
        hs.pdb_k = pdb_k
    return hs, keep


def _iters(arr, n):
    return [dict(bound=arr[i].bound, expanded=arr[i].expanded, generated=arr[i].generated,
                 complete=arr[i].complete, found=arr[i].found, limit=arr[i].limit) for i in range(n)]


def ida(domain, start, hkind=H_MD, table8=None, pdb=None, pdb_k=0, complete_final=False,
        max_iters=200, node_limit=-1, apdb=None):
    hs, keep = _hspec(hkind, table8, pdb, pdb_k, apdb)
    s = np.ascontiguousarray(start, dtype=np.uint8)
    arr = (Iter * max_iters)()
    n = C.c_int(0)
    cost = C.c_int32(-1)
    path = np.zeros(512, dtype=np.int8)
    plen = C.c_int(0)
    rc = lib().orc_ida(domain, s.ctypes.data, C.byref(hs), int(complete_final), max_iters, node_limit,
                       arr, C.byref(n), C.byref(cost), path.ctypes.data, C.byref(plen))
    del keep
    return dict(status=rc, cost=cost.value, path=path[:plen.value].tolist() if rc == 1 else [],
                iters=_iters(arr, n.value))


def bts(domain, start, hkind=H_MD, table8=None, pdb=None, pdb_k=0, b0=10000, c1=2, c2=8, plus_one=True,
        max_iters=400, max_total=-1, apdb=None):
    hs, keep = _hspec(hkind, table8, pdb, pdb_k, apdb)
    s = np.ascontiguousarray(start, dtype=np.uint8)
    arr = (Iter * max_iters)()
    n = C.c_int(0)
    cost = C.c_int32(-1)
    path = np.zeros(512, dtype=np.int8)
    plen = C.c_int(0)
    rc = lib().orc_bts(domain, s.ctypes.data, C.byref(hs), b0, c1, c2, int(plus_one), max_iters, max_total,
                       arr, C.byref(n), C.byref(cost), path.ctypes.data, C.byref(plen))
    del keep
    return dict(status=rc, cost=cost.value, path=path[:plen.value].tolist() if rc == 1 else [],
                iters=_iters(arr, n.value))


# ------------------------------------------------ real-valued heuristics
def _iters_real(arr, n):
    return [dict(bound=a.bound, expanded=a.expanded, generated=a.generated, complete=a.complete,
                 found=a.found, limit=a.limit) for a in arr[:n]]


def ida_real(start, table8f, complete_final=False, max_iters=5000, node_limit=-1):
    """Serial IDA* on the 8-puzzle with real-valued h (float32 table by rank)."""
    t = np.ascontiguousarray(table8f, dtype=np.float32)
    s = np.ascontiguousarray(start, dtype=np.uint8)
    arr = (IterReal * max_iters)()
    n, cost, plen = C.c_int(0), C.c_int32(-1), C.c_int(0)
    path = np.zeros(512, dtype=np.int8)
    rc = lib().orc_ida_real(s.ctypes.data, t.ctypes.data, int(complete_final), max_iters, node_limit, arr,
                            C.byref(n), C.byref(cost), path.ctypes.data, C.byref(plen))
    return dict(status=rc, cost=cost.value, path=path[:plen.value].tolist() if rc == 1 else [],
                iters=_iters_real(arr, n.value))


def ida_real_net(net, start, offset=0.0, complete_final=False, max_iters=5000, node_limit=-1):
    """Serial IDA* on the network's domain with h = max(0, y - offset), y the
    oracle's double-precision output per node."""
    s = np.ascontiguousarray(start, dtype=np.uint8)
    arr = (IterReal * max_iters)()
    n, cost, plen = C.c_int(0), C.c_int32(-1), C.c_int(0)
    path = np.zeros(512, dtype=np.int8)
    rc = lib().orc_ida_real_net(net._h, offset, s.ctypes.data, int(complete_final), max_iters, node_limit, arr,
                                C.byref(n), C.byref(cost), path.ctypes.data, C.byref(plen))
    return dict(status=rc, cost=cost.value, path=path[:plen.value].tolist() if rc == 1 else [],
                iters=_iters_real(arr, n.value))


def bts_real_net(net, start, offset=0.0, b0=10000, c1=2, c2=8, plus_one=True, max_iters=2000, max_total=-1):
    """Serial BTS on the network's domain with h = max(0, y - offset)."""
    s = np.ascontiguousarray(start, dtype=np.uint8)
    arr = (IterReal * max_iters)()
    n, cost, plen = C.c_int(0), C.c_int32(-1), C.c_int(0)
    path = np.zeros(512, dtype=np.int8)
    rc = lib().orc_bts_real_net(net._h, offset, s.ctypes.data, b0, c1, c2, int(plus_one), max_iters, max_total, arr,
                                C.byref(n), C.byref(cost), path.ctypes.data, C.byref(plen))
    return dict(status=rc, cost=cost.value, path=path[:plen.value].tolist() if rc == 1 else [],
                iters=_iters_real(arr, n.value))


def bts_real(start, table8f, b0=10000, c1=2, c2=8, plus_one=True, max_iters=2000, max_total=-1):
    """Serial BTS on the 8-puzzle with real-valued h (float32 table by rank)."""
    t = np.ascontiguousarray(table8f, dtype=np.float32)
    s = np.ascontiguousarray(start, dtype=np.uint8)
    arr = (IterReal * max_iters)()
    n, cost, plen = C.c_int(0), C.c_int32(-1), C.c_int(0)
    path = np.zeros(512, dtype=np.int8)
    rc = lib().orc_bts_real(s.ctypes.data, t.ctypes.data, b0, c1, c2, int(plus_one), max_iters, max_total, arr,
                            C.byref(n), C.byref(cost), path.ctypes.data, C.byref(plen))
    return dict(status=rc, cost=cost.value, path=path[:plen.value].tolist() if rc == 1 else [],
                iters=_iters_real(arr, n.value))
