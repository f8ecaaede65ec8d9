"""Python binding of libtrs (include/trs.h): argument marshalling only.

Every step of the rewriting runs in the HIP library; this module converts
numpy arrays to pointers, passes PyTorch's device memory and stream to the
library, and turns status codes into exceptions.  The functions carry the C
names (``trs_create``, ``trs_load_rules``, ``trs_load_terms``,
``trs_normalize``, ``trs_read_nf`` ...); :class:`Context` wraps them.

The library must have been built (``python -m paper_2009_07174_amd.build``);
importing this module without it raises ``ImportError`` -- there is no other
implementation to fall back to.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtrs.so")

TRS_OK, TRS_E_ARG, TRS_E_STATE, TRS_E_RULE, TRS_E_TERM = 0, -1, -2, -3, -4
TRS_E_POOL, TRS_E_ROUNDS, TRS_E_HIP, TRS_E_LIMIT, TRS_E_INTERNAL = -5, -6, -7, -8, -9
TRS_MODE_PLAIN, TRS_MODE_FRONTIER, TRS_MODE_LEARNED = 0, 1, 2


class trs_config(ctypes.Structure):
    _fields_ = [("pool_slots", ctypes.c_int64), ("maxarity", ctypes.c_int32),
                ("device", ctypes.c_int32), ("hip_stream", ctypes.c_void_p),
                ("dev_mem", ctypes.c_void_p), ("dev_bytes", ctypes.c_int64)]


class trs_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("block", ctypes.c_int32),
                ("nodes_per_thread", ctypes.c_int32), ("rounds_per_poll", ctypes.c_int32),
                ("max_rounds", ctypes.c_int64), ("threshold", ctypes.c_float),
                ("persistent", ctypes.c_int32), ("trace", ctypes.c_int32),
                ("trace_cap", ctypes.c_int64), ("label_horizon", ctypes.c_int32),
                ("sweep_every", ctypes.c_int32), ("max_grid", ctypes.c_int32),
                ("pf_depth", ctypes.c_int32), ("nf_walk", ctypes.c_int32),
                ("cont_passes", ctypes.c_int32), ("nf_walk_wide", ctypes.c_int32),
                ("cont_passes_wide", ctypes.c_int32), ("place_fresh", ctypes.c_int32)]


class trs_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "rounds", "rule_apps", "node_visits", "active_visits", "allocs", "frees",
        "peak_slots", "gc_rounds", "mlp_evals", "full_sweeps", "launches", "ready_visits",
        "nf_set", "rc_atomics", "memo_blocked", "mlp_kept", "trace_records", "nf_walked",
        "last_progress_round")] + [
        ("device_ms", ctypes.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class trs_membench_result(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "stream_read_gbps", "gather4_hbm_gops", "gather4_llc_gops", "gather1_llc_gops",
        "atomic_random_gops", "load_latency_far_ns", "load_latency_near_ns",
        "atomic_latency_ns", "empty_kernel_us")] + [
        ("copy_gbps", ctypes.c_double), ("copy_bytes", ctypes.c_int64),
        ("clock_mhz", ctypes.c_double),
        ("l2_bytes", ctypes.c_int64), ("cu_count", ctypes.c_int32), ("pad", ctypes.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_ if n != "pad"}


class trs_train_opts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("val_frac", ctypes.c_float)]


class trs_train_result(ctypes.Structure):
    _fields_ = [("epochs_run", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("train_loss", ctypes.c_float * 64), ("val_loss", ctypes.c_float * 64),
                ("device_ms", ctypes.c_double)]

    def as_dict(self):
        k = self.epochs_run
        return {"epochs_run": k, "train_loss": list(self.train_loss[:k]),
                "val_loss": list(self.val_loss[:k]), "device_ms": self.device_ms}


class trs_tune_result(ctypes.Structure):
    _fields_ = [("trials", ctypes.c_int32), ("best_block", ctypes.c_int32),
                ("best_npt", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("block", ctypes.c_int32 * 16),
                ("npt", ctypes.c_int32 * 16), ("ms", ctypes.c_double * 16),
                ("best_grid", ctypes.c_int32), ("pad2", ctypes.c_int32),
                ("grid", ctypes.c_int32 * 16)]

    def as_dict(self):
        k = self.trials
        return {"trials": k, "best_block": self.best_block, "best_npt": self.best_npt,
                "best_grid": self.best_grid, "best_ms": self.best_ms,
                "table": [(self.block[i], self.npt[i], self.grid[i], self.ms[i])
                          for i in range(k)]}


class trs_pool_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("free0", ctypes.c_int64), ("free1", ctypes.c_int64),
                ("maxarity", ctypes.c_int32), ("n_terms", ctypes.c_int32)]


TRS_MLP_EMB, TRS_MLP_DIN, TRS_MLP_H, TRS_MLP_MAX_SYM = 16, 24, 32, 256

EXPORTS = ["trs_create", "trs_destroy", "trs_load_rules", "trs_load_terms", "trs_normalize",
           "trs_read_nf", "trs_rule_counts", "trs_default_opts", "trs_device_bytes",
           "trs_membench", "trs_status_str", "trs_last_error", "trs_mlp_param_count",
           "trs_mlp_eval", "trs_mlp_train", "trs_mlp_table", "trs_set_predictor",
           "trs_read_trace", "trs_autotune", "trs_mlp_eval_noalloc", "trs_read_pool"]


def _load_lib():
    # PyTorch brings its own HIP runtime; importing it first makes that the
    # one the library binds to, so that both share devices, memory and
    # streams in one process
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2009_07174_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    i32p, i64p = P(ctypes.c_int32), P(ctypes.c_int64)
    lib.trs_create.argtypes = [P(vp), P(trs_config)]
    lib.trs_create.restype = ctypes.c_int32
    lib.trs_destroy.argtypes = [vp]
    lib.trs_destroy.restype = None
    lib.trs_load_rules.argtypes = [vp, ctypes.c_int32, i32p, ctypes.c_int32, i32p, i32p,
                                   ctypes.c_int64]
    lib.trs_load_rules.restype = ctypes.c_int32
    lib.trs_load_terms.argtypes = [vp, ctypes.c_int32, i64p, i32p, ctypes.c_int64]
    lib.trs_load_terms.restype = ctypes.c_int32
    lib.trs_normalize.argtypes = [vp, P(trs_opts), P(trs_stats)]
    lib.trs_normalize.restype = ctypes.c_int32
    lib.trs_read_nf.argtypes = [vp, ctypes.c_int32, i32p, ctypes.c_int64, i64p]
    lib.trs_read_nf.restype = ctypes.c_int32
    lib.trs_rule_counts.argtypes = [vp, i64p, ctypes.c_int32]
    lib.trs_rule_counts.restype = ctypes.c_int32
    lib.trs_read_pool.argtypes = [vp, P(trs_pool_info), i32p, i32p, P(ctypes.c_uint8), i32p,
                                  i32p, i32p, i32p]
    lib.trs_read_pool.restype = ctypes.c_int32
    lib.trs_default_opts.argtypes = [P(trs_opts)]
    lib.trs_default_opts.restype = None
    lib.trs_device_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32]
    lib.trs_device_bytes.restype = ctypes.c_int64
    lib.trs_membench.argtypes = [ctypes.c_int32, P(trs_membench_result)]
    lib.trs_membench.restype = ctypes.c_int32
    lib.trs_status_str.argtypes = [ctypes.c_int32]
    lib.trs_status_str.restype = ctypes.c_char_p
    lib.trs_last_error.argtypes = [vp]
    lib.trs_last_error.restype = ctypes.c_char_p
    u16p, u32p, u64p, f32p = (P(ctypes.c_uint16), P(ctypes.c_uint32), P(ctypes.c_uint64),
                              P(ctypes.c_float))
    lib.trs_mlp_param_count.argtypes = [ctypes.c_int32]
    lib.trs_mlp_param_count.restype = ctypes.c_int64
    lib.trs_mlp_eval.argtypes = [ctypes.c_int32, ctypes.c_int32, u16p, ctypes.c_int64, u64p,
                                 P(ctypes.c_double), f32p, f32p]
    lib.trs_mlp_eval.restype = ctypes.c_int32
    lib.trs_mlp_eval_noalloc.argtypes = lib.trs_mlp_eval.argtypes
    lib.trs_mlp_eval_noalloc.restype = ctypes.c_int32
    lib.trs_mlp_train.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, u64p,
                                  P(trs_train_opts), u16p, u16p, P(trs_train_result)]
    lib.trs_mlp_train.restype = ctypes.c_int32
    lib.trs_mlp_table.argtypes = [ctypes.c_int32, ctypes.c_int32, i32p, u16p, ctypes.c_float,
                                  f32p, u32p]
    lib.trs_mlp_table.restype = ctypes.c_int32
    lib.trs_set_predictor.argtypes = [vp, u16p, ctypes.c_int64]
    lib.trs_set_predictor.restype = ctypes.c_int32
    lib.trs_read_trace.argtypes = [vp, u64p, ctypes.c_int64, i64p]
    lib.trs_read_trace.restype = ctypes.c_int32
    lib.trs_autotune.argtypes = [vp, P(trs_opts), P(trs_opts), P(trs_tune_result)]
    lib.trs_autotune.restype = ctypes.c_int32
    return lib


_lib = _load_lib()


class TRSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_lib.trs_status_str(code).decode()} ({code}): {msg}")
        self.code = code


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _i64(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


# ----------------------------------------------------------- C-named calls

def trs_create(cfg: trs_config):
    h = ctypes.c_void_p()
    st = _lib.trs_create(ctypes.byref(h), ctypes.byref(cfg))
    if st != TRS_OK:
        raise TRSError(st, "trs_create")
    return h


def trs_destroy(h):
    _lib.trs_destroy(h)


def _check(h, st):
    if st != TRS_OK:
        raise TRSError(st, _lib.trs_last_error(h).decode())


def trs_load_rules(h, arity, rule_off, rule_code):
    a, ap = _i32(arity)
    o, op = _i32(rule_off)
    c, cp = _i32(rule_code)
    _check(h, _lib.trs_load_rules(h, len(a), ap, len(o) - 1, op, cp, len(c)))


def trs_load_terms(h, term_off, term_code):
    o, op = _i64(term_off)
    c, cp = _i32(term_code)
    _check(h, _lib.trs_load_terms(h, len(o) - 1, op, cp, len(c)))


def trs_default_opts() -> trs_opts:
    o = trs_opts()
    _lib.trs_default_opts(ctypes.byref(o))
    return o


def trs_normalize(h, opts: trs_opts) -> dict:
    st = trs_stats()
    _check(h, _lib.trs_normalize(h, ctypes.byref(opts), ctypes.byref(st)))
    return st.as_dict()


def trs_read_nf(h, term_id: int) -> np.ndarray:
    n = ctypes.c_int64(0)
    _check(h, _lib.trs_read_nf(h, term_id, None, 0, ctypes.byref(n)))
    out = np.empty(n.value, dtype=np.int32)
    _check(h, _lib.trs_read_nf(h, term_id, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               len(out), ctypes.byref(n)))
    return out


def trs_rule_counts(h, n_rules: int) -> np.ndarray:
    out = np.zeros(max(n_rules, 1), dtype=np.int64)
    _check(h, _lib.trs_rule_counts(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   len(out)))
    return out[:n_rules]


def trs_read_pool(h) -> dict:
    """The node pool after the last normalisation (hss, args as an n x A
    array, state, rc, the two free stacks' entries, the term roots)."""
    info = trs_pool_info()
    nul = ctypes.POINTER(ctypes.c_int32)()
    _check(h, _lib.trs_read_pool(h, ctypes.byref(info), nul, nul,
                                 ctypes.POINTER(ctypes.c_uint8)(), nul, nul, nul, nul))
    n, A = int(info.n), int(info.maxarity)
    hss = np.zeros(max(n, 1), np.int32)
    args = np.zeros(max(n * A, 1), np.int32)
    state = np.zeros(max(n, 1), np.uint8)
    rc = np.zeros(max(n, 1), np.int32)
    f0 = np.zeros(max(int(info.free0), 1), np.int32)
    f1 = np.zeros(max(int(info.free1), 1), np.int32)
    roots = np.zeros(max(int(info.n_terms), 1), np.int32)
    ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))  # noqa: E731
    _check(h, _lib.trs_read_pool(h, ctypes.byref(info), ip(hss), ip(args),
                                 state.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ip(rc),
                                 ip(f0), ip(f1), ip(roots)))
    return {"n": n, "maxarity": A, "hss": hss[:n], "args": args[:n * A].reshape(n, A),
            "state": state[:n], "rc": rc[:n], "free0": f0[:int(info.free0)],
            "free1": f1[:int(info.free1)], "roots": roots[:int(info.n_terms)]}


def trs_membench(device: int = 0) -> dict:
    r = trs_membench_result()
    st = _lib.trs_membench(device, ctypes.byref(r))
    if st != TRS_OK:
        raise TRSError(st, "trs_membench")
    return r.as_dict()


def trs_device_bytes(pool_slots: int, maxarity: int) -> int:
    return int(_lib.trs_device_bytes(pool_slots, maxarity))


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _u16(a):
    return np.ascontiguousarray(a, dtype=np.uint16)


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def trs_mlp_param_count(n_sym: int) -> int:
    return int(_lib.trs_mlp_param_count(n_sym))


def trs_mlp_eval(n_sym: int, params_bf16, records, grads: bool = True, probs: bool = False,
                 device: int = 0):
    """(mean loss, gradients or None, probabilities or None) on the device."""
    w, r = _u16(params_bf16), _u64(records)
    P = trs_mlp_param_count(n_sym)
    loss = ctypes.c_double(0.0)
    g = np.zeros(P, np.float32) if grads else None
    p = np.zeros(len(r), np.float32) if probs else None
    st = _lib.trs_mlp_eval(device, n_sym, _ptr(w, ctypes.c_uint16), len(r),
                           _ptr(r, ctypes.c_uint64), ctypes.byref(loss),
                           _ptr(g, ctypes.c_float) if grads else None,
                           _ptr(p, ctypes.c_float) if probs else None)
    if st != TRS_OK:
        raise TRSError(st, "trs_mlp_eval")
    return loss.value, g, p


TRS_MLP_NOALLOC_MAX_RECORDS = 65536


def trs_mlp_eval_noalloc(n_sym: int, params_bf16, records, grads: bool = True,
                         probs: bool = False, device: int = 0):
    """trs_mlp_eval computed in the library's static device buffer (the C
    call allocates no device memory): (mean loss, gradients or None,
    probabilities or None)."""
    w, r = _u16(params_bf16), _u64(records)
    P = trs_mlp_param_count(n_sym)
    loss = ctypes.c_double(0.0)
    g = np.zeros(max(P, 0), np.float32) if grads else None
    p = np.zeros(len(r), np.float32) if probs else None
    st = _lib.trs_mlp_eval_noalloc(device, n_sym, _ptr(w, ctypes.c_uint16), len(r),
                                   _ptr(r, ctypes.c_uint64), ctypes.byref(loss),
                                   _ptr(g, ctypes.c_float) if grads else None,
                                   _ptr(p, ctypes.c_float) if probs else None)
    if st != TRS_OK:
        raise TRSError(st, "trs_mlp_eval_noalloc")
    return loss.value, g, p


def trs_mlp_train(n_sym: int, records, init_bf16, epochs: int = 4, batch: int = 4096,
                  lr: float = 3e-3, val_frac: float = 0.1, device: int = 0):
    """(trained bfloat16 parameters, result dict)."""
    r, w0 = _u64(records), _u16(init_bf16)
    out = np.zeros(trs_mlp_param_count(n_sym), np.uint16)
    o = trs_train_opts(epochs=epochs, batch=batch, lr=lr, val_frac=val_frac)
    res = trs_train_result()
    st = _lib.trs_mlp_train(device, n_sym, len(r), _ptr(r, ctypes.c_uint64), ctypes.byref(o),
                            _ptr(w0, ctypes.c_uint16), _ptr(out, ctypes.c_uint16),
                            ctypes.byref(res))
    if st != TRS_OK:
        raise TRSError(st, "trs_mlp_train")
    return out, res.as_dict()


def trs_mlp_table(arity, params_bf16, threshold: float, device: int = 0):
    """(probabilities [n_sym, 32, 16], keep-bit words) evaluated on the device."""
    a, ap = _i32(arity)
    w = _u16(params_bf16)
    n_sym = len(a)
    probs = np.zeros(n_sym * 512, np.float32)
    words = np.zeros(n_sym * 16, np.uint32)
    st = _lib.trs_mlp_table(device, n_sym, ap, _ptr(w, ctypes.c_uint16), threshold,
                            _ptr(probs, ctypes.c_float), _ptr(words, ctypes.c_uint32))
    if st != TRS_OK:
        raise TRSError(st, "trs_mlp_table")
    return probs.reshape(n_sym, 32, 16), words


def trs_set_predictor(h, params_bf16):
    w = _u16(params_bf16)
    _check(h, _lib.trs_set_predictor(h, _ptr(w, ctypes.c_uint16), len(w)))


def trs_autotune(h, base: trs_opts):
    """(best trs_opts, result dict)."""
    best = trs_opts()
    res = trs_tune_result()
    _check(h, _lib.trs_autotune(h, ctypes.byref(base), ctypes.byref(best), ctypes.byref(res)))
    return best, res.as_dict()


def trs_read_trace(h) -> np.ndarray:
    n = ctypes.c_int64(0)
    _check(h, _lib.trs_read_trace(h, None, 0, ctypes.byref(n)))
    out = np.zeros(n.value, np.uint64)
    _check(h, _lib.trs_read_trace(h, _ptr(out, ctypes.c_uint64), len(out), ctypes.byref(n)))
    return out[:n.value]


# ----------------------------------------------------------- convenience

@dataclass
class Options:
    mode: int = TRS_MODE_PLAIN
    block: int = 0
    nodes_per_thread: int = 0
    rounds_per_poll: int = 0
    max_rounds: int = 0
    threshold: float = 0.1
    persistent: int = 0
    trace: int = 0
    trace_cap: int = 0
    label_horizon: int = 0
    sweep_every: int = 0
    max_grid: int = 0
    pf_depth: int = 0
    nf_walk: int = 0
    cont_passes: int = 0
    nf_walk_wide: int = 0
    cont_passes_wide: int = 0
    place_fresh: int = 0

    def to_c(self) -> trs_opts:
        o = trs_default_opts()
        for k in ("mode", "block", "nodes_per_thread", "rounds_per_poll", "max_rounds",
                  "threshold", "persistent", "trace", "trace_cap", "label_horizon",
                  "sweep_every", "max_grid", "pf_depth", "nf_walk", "cont_passes",
                  "nf_walk_wide", "cont_passes_wide", "place_fresh"):
            setattr(o, k, getattr(self, k))
        return o


class Context:
    """One rewriting context.  With ``torch_memory=True`` (and a GPU present)
    the device block is a PyTorch allocation and the work is issued on
    PyTorch's current stream; otherwise the library allocates and creates its
    own stream."""

    def __init__(self, pool_slots: int, maxarity: int = 0, device: int = 0,
                 torch_memory: bool = True, stream=None):
        # the C context is created by load_rules, once the argument stride
        # (maxarity, or the highest arity of the system) is known
        self.pool_slots, self.maxarity, self.device = pool_slots, maxarity, device
        self.torch_memory, self.stream = torch_memory, stream
        self.h = None
        self._keep = None
        self.stream_handle = None
        self.n_rules = 0

    def _create(self, A: int):
        self.close()
        cfg = trs_config(pool_slots=self.pool_slots, maxarity=A, device=self.device)
        if self.torch_memory:
            import torch
            if torch.cuda.is_available():
                nbytes = trs_device_bytes(self.pool_slots, A)
                if nbytes < 0:
                    raise TRSError(TRS_E_ARG, "bad pool size or maxarity")
                dev = torch.device("cuda", self.device)
                self._keep = torch.empty(nbytes, dtype=torch.uint8, device=dev)
                s = self.stream if self.stream is not None else torch.cuda.current_stream(dev)
                self._stream = s
                self.stream_handle = s.cuda_stream
                cfg.dev_mem = self._keep.data_ptr()
                cfg.dev_bytes = nbytes
                cfg.hip_stream = self.stream_handle
        self.h = trs_create(cfg)

    def close(self):
        if getattr(self, "h", None):
            trs_destroy(self.h)
            self.h = None
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def load_rules(self, arity, rule_off, rule_code):
        arity = np.asarray(arity)
        A = self.maxarity or max(1, int(arity.max()) if len(arity) else 1)
        self._create(A)
        trs_load_rules(self.h, arity, rule_off, rule_code)
        self.n_rules = len(rule_off) - 1

    def load_trs(self, trs):
        self.load_rules(*trs.encode_rules())

    def load_terms(self, term_off, term_code):
        trs_load_terms(self.h, term_off, term_code)

    def load_term_list(self, terms):
        off = np.zeros(len(terms) + 1, dtype=np.int64)
        off[1:] = np.cumsum([len(t) for t in terms])
        code = np.concatenate(terms) if terms else np.zeros(0, np.int32)
        self.load_terms(off, code)

    def normalize(self, opts: Options | None = None, **kw) -> dict:
        o = opts or Options(**kw)
        return trs_normalize(self.h, o.to_c())

    def read_nf(self, term_id: int) -> np.ndarray:
        return trs_read_nf(self.h, term_id)

    def rule_counts(self) -> np.ndarray:
        return trs_rule_counts(self.h, self.n_rules)

    def read_pool(self) -> dict:
        return trs_read_pool(self.h)

    def set_predictor(self, params_bf16):
        trs_set_predictor(self.h, params_bf16)

    def read_trace(self) -> np.ndarray:
        return trs_read_trace(self.h)

    def autotune(self, opts: Options | None = None, **kw):
        """(Options with the tuned block / nodes_per_thread, result dict)."""
        o = opts or Options(**kw)
        best, res = trs_autotune(self.h, o.to_c())
        out = Options(**{k: getattr(o, k) for k in o.__dataclass_fields__})
        out.block, out.nodes_per_thread = best.block, best.nodes_per_thread
        out.max_grid = best.max_grid
        return out, res
