"""CPU reference of the frontier predictor -- TEST INFRASTRUCTURE ONLY.

Only tests/ (and the benchmark's CPU leg) use this module.  It computes, in
float64, the forward pass, the binary cross-entropy loss and its gradients
for the small network the library trains on the GPU, so that the GPU
gradients can be checked element by element.  The reference is itself pinned
by central finite differences and by closed-form special cases in
tests/test_mlp_ref.py.

Network (the learned part of the workload configuration; the paper has no
learned component):

    x  = [E[sym] (16), arity/8, c_0..c_4, bucket(age)/15, 0]       (24)
    h1 = relu(W1 x + b1)                                           (32)
    h2 = relu(W2 h1 + b2)                                          (32)
    z  = w3 . h2 + b3 ;  p = sigmoid(z)
    loss = mean over the batch of  softplus(z) - y z   (= BCE(p, y))

c_j = 1 when argument j is a normal form or j >= arity.  age is the number of
rounds since the node last changed; bucket(0) = 0 and bucket(a) =
min(15, floor(log2 a) + 1) for a >= 1, so the input space is finite:
(symbol, 5 bits, 16 buckets).

Trace record (one uint64 per sampled node-round): symbol in bits 0-15, arity
in bits 16-19, c_0..c_4 in bits 20-24, age bucket in bits 25-28, label in
bit 32 (1 when the node fired or became a normal form within the label
horizon, a number of rounds).
Weights are stored in bfloat16; the reference takes them already rounded
(float64 values exactly representable in bfloat16) so that it evaluates the
same function as the GPU, whose arithmetic accumulates in float32.
"""

from __future__ import annotations

import numpy as np

EMB = 16
D_IN = 24
H = 32
MAX_ARGS = 5


def param_shapes(n_sym: int) -> dict:
    return {"E": (n_sym, EMB), "W1": (H, D_IN), "b1": (H,), "W2": (H, H), "b2": (H,),
            "w3": (H,), "b3": (1,)}


PARAM_ORDER = ["E", "W1", "b1", "W2", "b2", "w3", "b3"]


def n_params(n_sym: int) -> int:
    return sum(int(np.prod(s)) for s in param_shapes(n_sym).values())


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[k], np.float64).ravel() for k in PARAM_ORDER])


def unflatten(vec, n_sym: int) -> dict:
    out, off = {}, 0
    for k in PARAM_ORDER:
        shp = param_shapes(n_sym)[k]
        size = int(np.prod(shp))
        out[k] = np.asarray(vec[off:off + size], np.float64).reshape(shp)
        off += size
    return out


def bf16_round(a) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned
    as float64."""
    f = np.ascontiguousarray(np.asarray(a, np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def age_bucket(age) -> np.ndarray:
    """bucket(0) = 0, bucket(a) = min(15, floor(log2 a) + 1)."""
    a = np.asarray(age, np.int64)
    out = np.zeros(a.shape, np.int64)
    pos = a > 0
    out[pos] = np.minimum(15, np.floor(np.log2(a[pos])).astype(np.int64) + 1)
    return out


def decode_records(rec):
    """(sym, arity, bits, bucket, label) arrays from uint64 trace records."""
    r = np.asarray(rec, np.uint64)
    f = lambda sh, m: ((r >> np.uint64(sh)) & np.uint64(m)).astype(np.int64)
    return f(0, 0xFFFF), f(16, 0xF), f(20, 0x1F), f(25, 0xF), f(32, 1)


def encode_records(sym, arity, bits, bucket, label) -> np.ndarray:
    u = lambda a: np.asarray(a, np.uint64)
    return (u(sym) | (u(arity) << np.uint64(16)) | (u(bits) << np.uint64(20)) |
            (u(bucket) << np.uint64(25)) | (u(label) << np.uint64(32)))


def features(n_sym_emb: np.ndarray, sym, arity, bits, bucket) -> np.ndarray:
    """Input matrix (n x 24) from per-record fields (bits: c_0..c_4 as a
    5-bit mask, bucket: age bucket 0..15)."""
    sym = np.asarray(sym, np.int64)
    n = len(sym)
    x = np.zeros((n, D_IN), np.float64)
    x[:, :EMB] = n_sym_emb[sym]
    x[:, EMB] = np.asarray(arity, np.float64) / 8.0
    bits = np.asarray(bits, np.int64)
    for j in range(MAX_ARGS):
        x[:, EMB + 1 + j] = (bits >> j) & 1
    x[:, EMB + 1 + MAX_ARGS] = np.asarray(bucket, np.float64) / 15.0
    return x


def forward_backward(params: dict, sym, arity, bits, bucket, label):
    """Loss (mean BCE), probabilities and gradients of the loss with respect
    to every parameter, all in float64."""
    E, W1, b1, W2, b2, w3, b3 = (params[k] for k in PARAM_ORDER)
    y = np.asarray(label, np.float64)
    n = len(y)
    x = features(E, sym, arity, bits, bucket)
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    z = h2 @ w3 + b3[0]
    p = 1.0 / (1.0 + np.exp(-z))
    loss = np.mean(np.logaddexp(0.0, z) - y * z)
    dz = (p - y) / n                      # d loss / d z
    g = {}
    g["w3"] = h2.T @ dz
    g["b3"] = np.array([dz.sum()])
    dh2 = np.outer(dz, w3) * (z2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ W2) * (z1 > 0)
    g["W1"] = dh1.T @ x
    g["b1"] = dh1.sum(axis=0)
    dx = dh1 @ W1
    gE = np.zeros_like(E)
    np.add.at(gE, np.asarray(sym, np.int64), dx[:, :EMB])
    g["E"] = gE
    return loss, p, g


def loss_only(params: dict, sym, arity, bits, bucket, label) -> float:
    return forward_backward(params, sym, arity, bits, bucket, label)[0]


def decision_table(params: dict, n_sym: int, arity_of, threshold: float) -> np.ndarray:
    """Probability for every input the predictor can see, indexed
    [sym, bits, bucket] (shape n_sym x 32 x 16); arity_of[sym] is the
    symbol's arity.  A node is kept when p >= threshold."""
    sym, bits, bucket = np.meshgrid(np.arange(n_sym), np.arange(32), np.arange(16), indexing="ij")
    sym, bits, bucket = sym.ravel(), bits.ravel(), bucket.ravel()
    ar = np.asarray(arity_of, np.int64)[sym]
    p = forward_backward(params, sym, ar, bits, bucket, np.zeros(len(sym)))[1]
    return p.reshape(n_sym, 32, 16)


def init_params(n_sym: int, seed: int) -> dict:
    """Seeded initialisation (scaled normal), rounded to bfloat16."""
    rng = np.random.default_rng(seed)
    shp = param_shapes(n_sym)
    p = {
        "E": rng.normal(0, 0.5, shp["E"]),
        "W1": rng.normal(0, np.sqrt(2.0 / D_IN), shp["W1"]),
        "b1": np.zeros(shp["b1"]),
        "W2": rng.normal(0, np.sqrt(2.0 / H), shp["W2"]),
        "b2": np.zeros(shp["b2"]),
        "w3": rng.normal(0, np.sqrt(1.0 / H), shp["w3"]),
        "b3": np.zeros(shp["b3"]),
    }
    return {k: bf16_round(v) for k, v in p.items()}
