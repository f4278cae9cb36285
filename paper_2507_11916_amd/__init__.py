"""Python binding of libhb (include/hb.h): argument marshalling only.

Every computation runs in the library: HIP kernels on the GPU for the network,
C++ for the search runtime.  PyTorch provides device memory and streams: device
buffers are torch tensors whose data_ptr() is handed to the C ABI together with
the current HIP stream.  The binding fails loudly if the built library is
missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libhb.so")
_lib = None

HB_OK, HB_E_INVAL, HB_E_NOMEM, HB_E_DEVICE, HB_E_UNSUPPORTED, HB_E_BUDGET, HB_E_NOSOLUTION = 0, -1, -2, -3, -4, -5, -6
HB_STP3, HB_STP4, HB_RUBIK3 = 0, 1, 2
HB_FP32, HB_BF16, HB_FP8_E4M3 = 0, 1, 2
HB_OUT_REG_FLOOR, HB_OUT_REG_ROUND, HB_OUT_REG_REAL, HB_OUT_CLS_QUANTILE, HB_OUT_CLS_ARGMAX = 0, 1, 2, 3, 4
HB_IDA, HB_BTS = 0, 1
HB_H_NN, HB_H_MIN_NN_CLASSIC, HB_H_FIXED_TREE, HB_H_CLASSIC, HB_H_CLASSIC_BATCHED, HB_H_NN_REAL = 0, 1, 2, 3, 4, 5
HB_CLASSIC_ZERO, HB_CLASSIC_MD, HB_CLASSIC_PDB = 0, 1, 2
HB_ENSEMBLE_MIN, HB_ENSEMBLE_SUM = 0, 1


class HBError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hb status {status}: {msg}")
        self.status = status


class ModelOpts(C.Structure):
    _fields_ = [("prec", C.c_int), ("device", C.c_int), ("out", C.c_int), ("q", C.c_float),
                ("offset", C.c_float), ("combine_md", C.c_int), ("max_batch", C.c_int)]


class TuneEntry(C.Structure):
    _fields_ = [("batch", C.c_int32), ("tile", C.c_int32), ("us", C.c_double), ("evals_per_s", C.c_double)]


class ModelInfo(C.Structure):
    _fields_ = [("domain", C.c_int), ("n_in", C.c_int), ("n_dense", C.c_int), ("n_res", C.c_int),
                ("n_out", C.c_int), ("head_kind", C.c_int), ("n_act", C.c_int), ("prec", C.c_int),
                ("dims", C.c_int * 8), ("weight_bytes", C.c_int64), ("flops_per_eval", C.c_double)]


class TrainOpts(C.Structure):
    _fields_ = [("prec", C.c_int), ("device", C.c_int), ("max_batch", C.c_int), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float), ("asym", C.c_int),
                ("alpha", C.c_float)]


class Heuristic(C.Structure):
    _fields_ = [("model", C.c_void_p), ("combine", C.c_int), ("classic", C.c_int), ("pdb", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("batch_size", C.c_int), ("work_num", C.c_int), ("d_init", C.c_int), ("timeout_us", C.c_int),
                ("n_slabs", C.c_int), ("flush_when_idle", C.c_int), ("node_limit", C.c_int64),
                ("time_limit_s", C.c_double), ("bts_b0", C.c_int64), ("bts_c1", C.c_int), ("bts_c2", C.c_int),
                ("bts_root_plus_one", C.c_int), ("dedup_frontier", C.c_int), ("complete_final_iter", C.c_int),
                ("start_bound", C.c_int32), ("max_iters", C.c_int), ("use_graphs", C.c_int),
                ("gpu_depth", C.c_int)]


class Iter(C.Structure):
    _fields_ = [("bound", C.c_int32), ("limit", C.c_int64), ("expanded", C.c_int64), ("generated", C.c_int64),
                ("complete", C.c_int32), ("found", C.c_int32), ("bound_real", C.c_double),
                ("batches", C.c_int64), ("evals", C.c_int64)]


class Result(C.Structure):
    _fields_ = [("cost", C.c_int32), ("path_len", C.c_int32), ("path", C.POINTER(C.c_int8)),
                ("n_iter", C.c_int32), ("iters", C.POINTER(Iter)), ("evals", C.c_int64), ("batches", C.c_int64),
                ("mean_batch", C.c_double), ("wall_s", C.c_double), ("gpu_busy_s", C.c_double),
                ("expanded", C.c_int64), ("generated", C.c_int64), ("frontier", C.c_int32),
                ("peak_nodes", C.c_int64)]


def lib():
    """Load libhb.so (built by __graft_entry__.build() / paper_2507_11916_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2507_11916_amd/build.py")
        # torch ships its own HIP runtime with the same soname; loading torch
        # first makes libhb bind to that one, so device pointers and streams
        # from torch and from the library live in a single runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i64 = C.c_void_p, C.c_int64
        sigs = {
            "hb_last_error": ([], C.c_char_p),
            "hb_state_bytes": ([C.c_int], C.c_int),
            "hb_packed_bytes": ([C.c_int], C.c_int),
            "hb_encode": ([C.c_int, vp, i64, vp], C.c_int),
            "hb_decode": ([C.c_int, vp, i64, vp], C.c_int),
            "hb_apply_moves": ([C.c_int, vp, i64, C.c_int32, vp], C.c_int),
            "hb_manhattan": ([C.c_int, vp, i64, vp], C.c_int),
            "hb_pdb_build_corner": ([C.c_int, C.c_int, C.POINTER(vp)], C.c_int),
            "hb_pdb_lookup": ([vp, vp, i64, vp], C.c_int),
            "hb_pdb_value_counts": ([vp, vp, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
            "hb_pdb_build_stp_additive": ([vp, C.c_int, C.POINTER(vp)], C.c_int),
            "hb_pdb_free": ([vp], None),
            "hb_model_load": ([C.c_char_p, C.POINTER(ModelOpts), C.POINTER(vp)], C.c_int),
            "hb_model_load_ensemble": ([C.POINTER(C.c_char_p), C.c_int, C.c_int, C.POINTER(ModelOpts), C.POINTER(vp)],
                                       C.c_int),
            "hb_model_free": ([vp], None),
            "hb_model_get_info": ([vp, C.POINTER(ModelInfo)], C.c_int),
            "hb_model_calibrate": ([vp, vp, i64], C.c_int),
            "hb_model_get_act_scales": ([vp, vp, C.c_int], C.c_int),
            "hb_model_set_act_scales": ([vp, vp, C.c_int], C.c_int),
            "hb_eval_batch": ([vp, vp, i64, vp, vp, vp], C.c_int),
            "hb_eval_batch_dev_n": ([vp, vp, vp, i64, vp, vp, vp], C.c_int),
            "hb_eval_batch_noalloc": ([vp, vp, i64, vp, vp, vp], C.c_int),
            "hb_model_activation": ([vp, vp, i64, C.c_int, vp, i64, vp], C.c_int),
            "hb_model_set_tile": ([vp, C.c_int], C.c_int),
            "hb_model_tune": ([vp, vp, i64, vp, C.c_int], C.c_int),
            "hb_model_autotune": ([vp, vp, i64, C.POINTER(TuneEntry), C.c_int, C.POINTER(C.c_int),
                                   C.POINTER(C.c_int32)], C.c_int),
            "hb_model_tile_for": ([vp, i64, C.POINTER(C.c_int)], C.c_int),
            "hb_model_save_tuning": ([vp, C.c_char_p], C.c_int),
            "hb_model_load_tuning": ([vp, C.c_char_p], C.c_int),
            "hb_model_profile": ([vp, C.c_int], C.c_int),
            "hb_model_profile_read": ([vp, vp], C.c_int),
            "hb_trainer_create": ([C.c_char_p, C.POINTER(TrainOpts), C.POINTER(vp)], C.c_int),
            "hb_trainer_free": ([vp], None),
            "hb_trainer_n_params": ([vp], i64),
            "hb_train_step": ([vp, vp, vp, i64, vp, vp], C.c_int),
            "hb_train_grad": ([vp, vp, vp, i64, vp, vp], C.c_int),
            "hb_trainer_get_params": ([vp, vp], C.c_int),
            "hb_trainer_save": ([vp, C.c_char_p], C.c_int),
            "cbdfs_params_default": ([C.POINTER(Params)], None),
            "cbdfs_solve": ([C.c_int, vp, C.POINTER(Heuristic), C.c_int, C.c_int, C.POINTER(Params),
                             C.POINTER(Result)], C.c_int),
            "cbdfs_result_free": ([C.POINTER(Result)], None),
        }
        for name, (args, res) in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(st):
    if st != HB_OK:
        raise HBError(st, lib().hb_last_error().decode())
    return st


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _stream(stream=None):
    import torch
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


# ----------------------------------------------------------------- host side
def state_bytes(domain):
    return lib().hb_state_bytes(domain)


def packed_bytes(domain):
    return lib().hb_packed_bytes(domain)


def hb_encode(domain, states):
    s = np.ascontiguousarray(states, dtype=np.uint8).reshape(-1, state_bytes(domain))
    out = np.zeros((s.shape[0], packed_bytes(domain)), dtype=np.uint8)
    _check(lib().hb_encode(domain, _np_ptr(s), s.shape[0], _np_ptr(out)))
    return out


def hb_decode(domain, packed):
    p = np.ascontiguousarray(packed, dtype=np.uint8).reshape(-1, packed_bytes(domain))
    out = np.zeros((p.shape[0], state_bytes(domain)), dtype=np.uint8)
    _check(lib().hb_decode(domain, _np_ptr(p), p.shape[0], _np_ptr(out)))
    return out


def hb_apply_moves(domain, moves):
    m = np.ascontiguousarray(moves, dtype=np.int8)
    if m.ndim == 1:
        m = m[None, :]
    out = np.zeros((m.shape[0], state_bytes(domain)), dtype=np.uint8)
    _check(lib().hb_apply_moves(domain, _np_ptr(m), m.shape[0], m.shape[1], _np_ptr(out)))
    return out


def hb_manhattan(domain, states):
    s = np.ascontiguousarray(states, dtype=np.uint8).reshape(-1, state_bytes(domain))
    out = np.zeros(s.shape[0], dtype=np.int32)
    _check(lib().hb_manhattan(domain, _np_ptr(s), s.shape[0], _np_ptr(out)))
    return out


class Pdb:
    """Pattern database built by the library (host memory): the cube's k-corner
    PDB, or (groups=...) an additive 15-puzzle PDB."""

    def __init__(self, k=None, threads=0, groups=None):
        """k: corners of a cube PDB; groups: tile groups of an additive 15-puzzle
        PDB, e.g. [range(1, 8), range(8, 16)] for the 7-8 split."""
        h = C.c_void_p()
        if groups is not None:
            g = np.full(16, -1, dtype=np.int32)
            for i, tiles in enumerate(groups):
                for t in tiles:
                    g[int(t)] = i
            _check(lib().hb_pdb_build_stp_additive(_np_ptr(g), threads, C.byref(h)))
        else:
            _check(lib().hb_pdb_build_corner(k, threads, C.byref(h)))
        self.handle = h
        self._free = lib().hb_pdb_free
        self.k = k
        self.groups = groups

    def lookup(self, states):
        s = np.ascontiguousarray(states, dtype=np.uint8).reshape(-1, 16 if self.groups is not None else 54)
        out = np.zeros(s.shape[0], dtype=np.int32)
        _check(lib().hb_pdb_lookup(self.handle, _np_ptr(s), s.shape[0], _np_ptr(out)))
        return out

    def value_counts(self, n=32):
        """(counts of the entries holding each value 0..n-1, largest value)."""
        counts = np.zeros(n, dtype=np.int64)
        vmax = C.c_int32(0)
        _check(lib().hb_pdb_value_counts(self.handle, _np_ptr(counts), n, C.byref(vmax)))
        return counts, vmax.value

    def close(self):
        # the free function is bound at creation: at interpreter exit the
        # module's globals may already be gone when __del__ runs
        if getattr(self, "handle", None):
            self._free(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


# ----------------------------------------------------------------- model
class Model:
    """A network resident on one GPU (hb_model)."""

    def __init__(self, path, prec=HB_FP32, out=HB_OUT_REG_FLOOR, q=0.99, offset=0.0, combine_md=False,
                 max_batch=16384, device=0, ensemble_rule=HB_ENSEMBLE_MIN):
        """path: a weight file, or a list of 1-4 weight files of one architecture
        (an ensemble combined by ensemble_rule).  combine_md: 0/False none, 1/True
        min, 2 max, 3 plus (Manhattan distance)."""
        o = ModelOpts(prec, device, out, q, offset, int(combine_md), max_batch)
        h = C.c_void_p()
        if isinstance(path, (list, tuple)):
            arr = (C.c_char_p * len(path))(*[os.fsencode(p) for p in path])
            _check(lib().hb_model_load_ensemble(arr, len(path), ensemble_rule, C.byref(o), C.byref(h)))
        else:
            _check(lib().hb_model_load(os.fsencode(path), C.byref(o), C.byref(h)))
        self.handle = h
        self._free = lib().hb_model_free
        self.opts = o
        info = ModelInfo()
        _check(lib().hb_model_get_info(h, C.byref(info)))
        self.info = info
        self.domain = info.domain
        self.n_out = info.n_out
        self.n_act = info.n_act

    def close(self):
        # the free function is bound at creation: at interpreter exit the
        # module's globals may already be gone when __del__ runs
        if getattr(self, "handle", None):
            self._free(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    @property
    def flops_per_eval(self):
        return self.info.flops_per_eval

    def calibrate(self, d_packed):
        _check(lib().hb_model_calibrate(self.handle, C.c_void_p(d_packed.data_ptr()), d_packed.shape[0]))

    def act_scales(self):
        out = np.zeros(self.n_act, dtype=np.float32)
        _check(lib().hb_model_get_act_scales(self.handle, _np_ptr(out), self.n_act))
        return out

    def set_act_scales(self, scales):
        s = np.ascontiguousarray(scales, dtype=np.float32)
        _check(lib().hb_model_set_act_scales(self.handle, _np_ptr(s), s.shape[0]))

    def eval_batch(self, d_packed, d_h, d_raw=None, n=None, stream=None):
        """hb_eval_batch on torch device tensors (uint8 packed, int32 h, float32 raw)."""
        n = d_packed.shape[0] if n is None else n
        _check(lib().hb_eval_batch(self.handle, C.c_void_p(d_packed.data_ptr()), n,
                                   C.c_void_p(d_h.data_ptr()),
                                   None if d_raw is None else C.c_void_p(d_raw.data_ptr()), _stream(stream)))

    def activation(self, d_packed, act, d_out, n=None, stream=None):
        """hb_model_activation: stored activation tensor `act` of the forward pass
        into d_out (a 2-D device tensor of the operand type's element size)."""
        n = d_packed.shape[0] if n is None else n
        _check(lib().hb_model_activation(self.handle, C.c_void_p(d_packed.data_ptr()), n, act,
                                         C.c_void_p(d_out.data_ptr()), d_out.stride(0), _stream(stream)))

    def eval_batch_noalloc(self, d_packed, d_h, d_raw=None, n=None, stream=None):
        """hb_eval_batch_noalloc: as eval_batch, with the library's fixed device array as workspace."""
        n = d_packed.shape[0] if n is None else n
        _check(lib().hb_eval_batch_noalloc(self.handle, C.c_void_p(d_packed.data_ptr()), n,
                                           C.c_void_p(d_h.data_ptr()),
                                           None if d_raw is None else C.c_void_p(d_raw.data_ptr()),
                                           _stream(stream)))

    def eval_batch_dev_n(self, d_packed, d_n, max_n, d_h, d_raw=None, stream=None):
        _check(lib().hb_eval_batch_dev_n(self.handle, C.c_void_p(d_packed.data_ptr()),
                                         C.c_void_p(d_n.data_ptr()), max_n, C.c_void_p(d_h.data_ptr()),
                                         None if d_raw is None else C.c_void_p(d_raw.data_ptr()),
                                         _stream(stream)))

    def set_tile(self, tile_id):
        _check(lib().hb_model_set_tile(self.handle, tile_id))

    def tune(self, d_packed, n=None):
        """Tile timings [(tile id, us)] at one batch size; keeps the fastest for its bucket."""
        n = d_packed.shape[0] if n is None else n
        rep = np.zeros(32, dtype=np.float64)
        _check(lib().hb_model_tune(self.handle, C.c_void_p(d_packed.data_ptr()), n, _np_ptr(rep), 32))
        return [(int(rep[2 * i]), float(rep[2 * i + 1])) for i in range(16) if rep[2 * i + 1] > 0]

    def autotune(self, d_packed, n=None):
        """Bucket table [{batch, tile, us, evals_per_s}] and the recommended batch size."""
        n = d_packed.shape[0] if n is None else n
        table = (TuneEntry * 64)()
        rows, rec = C.c_int(0), C.c_int32(0)
        _check(lib().hb_model_autotune(self.handle, C.c_void_p(d_packed.data_ptr()), n, table, 64,
                                       C.byref(rows), C.byref(rec)))
        return [{"batch": e.batch, "tile": e.tile, "us": e.us, "evals_per_s": e.evals_per_s}
                for e in table[:rows.value]], rec.value

    def tile_for(self, n):
        t = C.c_int(0)
        _check(lib().hb_model_tile_for(self.handle, n, C.byref(t)))
        return t.value

    def save_tuning(self, path):
        _check(lib().hb_model_save_tuning(self.handle, os.fsencode(path)))

    def load_tuning(self, path):
        _check(lib().hb_model_load_tuning(self.handle, os.fsencode(path)))


# --------------------------------------------------------------- training
class Trainer:
    """On-GPU training of a sliding-tile regression network (hb_trainer)."""

    def __init__(self, path, prec=HB_BF16, max_batch=8192, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 asym=False, alpha=4.0, device=0):
        o = TrainOpts(prec, device, max_batch, lr, beta1, beta2, eps, int(asym), alpha)
        h = C.c_void_p()
        _check(lib().hb_trainer_create(path.encode(), C.byref(o), C.byref(h)))
        self.handle = h
        self._free = lib().hb_trainer_free
        self.n_params = lib().hb_trainer_n_params(h)

    def close(self):
        # the free function is bound at creation: at interpreter exit the
        # module's globals may already be gone when __del__ runs
        if getattr(self, "handle", None):
            self._free(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    def step(self, d_packed, d_labels, n=None, want_loss=True, stream=None):
        n = d_packed.shape[0] if n is None else n
        loss = C.c_float(0.0)
        _check(lib().hb_train_step(self.handle, C.c_void_p(d_packed.data_ptr()), C.c_void_p(d_labels.data_ptr()), n,
                                   C.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None

    def grad(self, d_packed, d_labels, d_grads, n=None):
        n = d_packed.shape[0] if n is None else n
        loss = C.c_float(0.0)
        _check(lib().hb_train_grad(self.handle, C.c_void_p(d_packed.data_ptr()), C.c_void_p(d_labels.data_ptr()), n,
                                   C.c_void_p(d_grads.data_ptr()), C.byref(loss)))
        return loss.value

    def params(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().hb_trainer_get_params(self.handle, _np_ptr(out)))
        return out

    def save(self, path):
        _check(lib().hb_trainer_save(self.handle, path.encode()))


# ----------------------------------------------------------------- search
def default_params(**kw):
    p = Params()
    lib().cbdfs_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def cbdfs_solve(domain, start, model=None, combine=HB_H_NN, classic=HB_CLASSIC_MD, pdb=None, algo=HB_IDA,
                threads=8, params=None, raise_on_error=True):
    """Run Batch IDA* / Batch BTS; returns a dict of the result fields."""
    s = np.ascontiguousarray(start, dtype=np.uint8)
    h = Heuristic(model.handle if model is not None else None, combine, classic,
                  pdb.handle if pdb is not None else None)
    p = params if params is not None else default_params()
    r = Result()
    st = lib().cbdfs_solve(domain, _np_ptr(s), C.byref(h), algo, threads, C.byref(p), C.byref(r))
    if st not in (HB_OK, HB_E_BUDGET, HB_E_NOSOLUTION) and raise_on_error:
        raise HBError(st, lib().hb_last_error().decode())
    out = dict(status=st, cost=r.cost, path=[r.path[i] for i in range(r.path_len)] if r.path else [],
               iters=[dict(bound=r.iters[i].bound, limit=r.iters[i].limit, expanded=r.iters[i].expanded,
                           generated=r.iters[i].generated, complete=r.iters[i].complete, found=r.iters[i].found,
                           bound_real=r.iters[i].bound_real, batches=r.iters[i].batches,
                           evals=r.iters[i].evals)
                      for i in range(r.n_iter)],
               evals=r.evals, batches=r.batches, mean_batch=r.mean_batch, wall_s=r.wall_s,
               gpu_busy_s=r.gpu_busy_s, expanded=r.expanded, generated=r.generated, frontier=r.frontier,
               peak_nodes=r.peak_nodes,
               error=lib().hb_last_error().decode() if st != HB_OK else "")
    lib().cbdfs_result_free(C.byref(r))
    return out
