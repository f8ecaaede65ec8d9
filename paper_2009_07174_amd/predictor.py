"""The frontier predictor of learned mode: training data, training, storage.

* Training data are trace records logged on the device by plain-mode runs
  (``trs_opts.trace``): for a sampled node found blocked in round r, its head
  symbol, arity, which arguments are normal forms, and how long ago it last
  changed; the label says whether it fired or became a normal form in the
  next round (the label horizon, 1 by default).  In learned mode a node the
  predictor drops sleeps until the argument it waits on notifies it (or a
  periodic sweep finds it).
* Training runs on the device (``trs_mlp_train``: the library's forward,
  backward and Adam kernels).
* Parameters are stored as ``.npz`` (uint16 bfloat16 bit patterns plus the
  symbol names they were trained for; loaded with ``allow_pickle=False``).

All training workloads are encoded in the batch system's symbol numbering,
so one predictor serves every configuration built on that system.
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from . import trs as T

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "data", "frontier_batch.npz")


def bf16_bits(x) -> np.ndarray:
    """float values -> bfloat16 bit patterns (round to nearest, ties to even)."""
    f = np.ascontiguousarray(np.asarray(x, np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def init_params(n_sym: int, seed: int = 0) -> np.ndarray:
    """Seeded initial parameters (scaled normal weights, zero biases) in the
    C-ABI order E, W1, b1, W2, b2, w3, b3."""
    rng = np.random.default_rng(seed)
    E, D, H = T.TRS_MLP_EMB, T.TRS_MLP_DIN, T.TRS_MLP_H
    parts = [rng.normal(0, 0.5, n_sym * E), rng.normal(0, np.sqrt(2.0 / D), H * D),
             np.zeros(H), rng.normal(0, np.sqrt(2.0 / H), H * H), np.zeros(H),
             rng.normal(0, np.sqrt(1.0 / H), H), np.zeros(1)]
    out = bf16_bits(np.concatenate(parts))
    assert len(out) == T.trs_mlp_param_count(n_sym)
    return out


def collect(trs, terms, pool_slots: int, target: int, cap: int = 1 << 24,
            seed_rate: int | None = None, log=print):
    """Trace records of a plain-mode run of ``terms``: a first run without
    tracing counts the blocked node-rounds, the sampling rate is set so that
    about ``target`` records are kept."""
    ctx = T.Context(pool_slots)
    try:
        ctx.load_trs(trs)
        ctx.load_term_list(list(terms))
        rate = seed_rate
        if rate is None:
            st = ctx.normalize(mode=T.TRS_MODE_PLAIN)
            blocked = max(1, st["active_visits"] - st["ready_visits"])
            rate = int(min(65536, max(1, round(65536.0 * target / blocked))))
        st = ctx.normalize(mode=T.TRS_MODE_PLAIN, trace=rate, trace_cap=cap)
        rec = ctx.read_trace()
    finally:
        ctx.close()
    log(f"[predictor] {len(rec)} records (rate {rate}/65536, rounds {st['rounds']}, "
        f"positive {float(np.mean((rec >> np.uint64(32)) & np.uint64(1))) if len(rec) else 0:.3f})")
    return rec


def training_sets(scale: str = "full"):
    """(name, trs, terms, pool_slots, share) of the default training mix:
    the three workload kinds of configurations 1-3, in the batch system."""
    from trs_workloads import generators as G
    from trs_workloads import systems
    trs = systems.batch()
    if scale == "full":
        # configurations 1 (n = 25) and 2 whole; of configuration 3 the first
        # 512 of its 4096 terms (same recipe and seeds), so that the plain
        # trace run, which tests every blocked node every round, stays short
        g_n, sort_len, n_batch = 25, 4096, 512
    else:
        g_n, sort_len, n_batch = 12, 64, 48
    vals = np.random.default_rng(G.BASE_SEED + 2).integers(0, 64, size=sort_len)
    batch = G.cfg3(n_batch, 1 << 26, "full" if scale == "full" else "mini")
    return [
        ("g", trs, [G.g_term(trs, g_n)], 1 << 24, 1 / 3),
        ("sort", trs, [G.sort_term(trs, vals)], 1 << 25, 1 / 3),
        ("batch", trs, batch.terms, 1 << 26, 1 / 3),
    ]


def train(n_sym: int, records, epochs: int = 3, batch: int = 4096, lr: float = 3e-3,
          val_frac: float = 0.1, seed: int = 0, init=None, log=print):
    """Shuffle (seeded) and train on the device; returns (params, result)."""
    rec = np.asarray(records, np.uint64)
    rec = rec[np.random.default_rng(seed).permutation(len(rec))]
    w0 = init_params(n_sym, seed) if init is None else init
    params, res = T.trs_mlp_train(n_sym, rec, w0, epochs=epochs, batch=batch, lr=lr,
                                  val_frac=val_frac)
    log(f"[predictor] trained on {len(rec)} records: train loss {res['train_loss']}, "
        f"val loss {res['val_loss']}, {res['device_ms']:.0f} ms")
    return params, res


def save(path: str, params, symbols, meta: dict):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=np.asarray(params, np.uint16), symbols=np.asarray(symbols),
             meta=np.asarray(json.dumps(meta)))


def load(path: str, symbols=None) -> np.ndarray:
    """Parameters from ``path``; with ``symbols`` given, checks that they
    were trained for that symbol numbering."""
    z = np.load(path, allow_pickle=False)
    if symbols is not None and list(z["symbols"]) != list(symbols):
        raise ValueError(f"{path}: trained for another symbol set")
    return np.asarray(z["params"], np.uint16)


def build_default(out: str = DEFAULT_WEIGHTS, n_records: int = 10_000_000,
                  scale: str = "full", epochs: int = 3, log=print):
    """Collect about n_records trace records from the default mix and train."""
    t0 = time.time()
    recs = []
    sets = training_sets(scale)
    for name, trs, terms, pool, share in sets:
        log(f"[predictor] tracing {name}: {len(terms)} terms")
        recs.append(collect(trs, terms, pool, int(n_records * share), cap=int(n_records),
                            log=log))
    rec = np.concatenate(recs)
    trs = sets[0][1]
    params, res = train(len(trs.symbols), rec, epochs=epochs, log=log)
    meta = {"records": int(len(rec)), "train": res, "scale": scale,
            "sources": [s[0] for s in sets], "seconds": time.time() - t0}
    save(out, params, trs.symbols, meta)
    log(f"[predictor] wrote {out}")
    return params, meta


if __name__ == "__main__":
    out = sys.argv[1] if len(sys.argv) > 1 else DEFAULT_WEIGHTS
    n = int(float(sys.argv[2])) if len(sys.argv) > 2 else 10_000_000
    build_default(out, n)
