"""Weights of the learned correction-tier gate.

The network (three hidden layers of 64 ReLU units, four ordinal outputs)
runs inside the library (``csbq_gate_*``); this module only initialises,
stores and loads its weights.  Layout (float32, ``GATE_NW`` values):
W1[16][64] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64][4] b4[4].
"""
from __future__ import annotations

import os

import numpy as np

from . import GATE_NF, GATE_NO, GATE_NW, TABLE_DIR

H = 64
DEFAULT_WEIGHTS = os.path.join(TABLE_DIR, "gate_mlp.npz")            # mixed precision, quad_tol 1e-7
FP64_WEIGHTS = os.path.join(TABLE_DIR, "gate_mlp_fp64.npz")          # FP64, quad_tol 1e-12
SHAPES = (("W1", (GATE_NF, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
          ("W4", (H, GATE_NO)), ("b4", (GATE_NO,)))


def unpack(w):
    """Named views of a flat weight vector."""
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = w[o:o + n].reshape(shp)
        o += n
    assert o == GATE_NW
    return out


def init_weights(seed=0):
    """He-normal weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in SHAPES:
        if name.startswith("W"):
            parts.append(rng.normal(0.0, np.sqrt(2.0 / shp[0]), shp).astype(np.float32).ravel())
        else:
            parts.append(np.zeros(shp, np.float32).ravel())
    w = np.concatenate(parts)
    assert w.size == GATE_NW
    return w


def save_weights(path, w, **meta):
    np.savez(path, weights=np.asarray(w, np.float32), **{k: np.asarray(v) for k, v in meta.items()})


def load_weights(path=DEFAULT_WEIGHTS):
    """(weights, metadata dict) from an .npz written by save_weights."""
    with np.load(path, allow_pickle=False) as z:
        w = z["weights"].astype(np.float32)
        meta = {k: z[k] for k in z.files if k != "weights"}
    if w.size != GATE_NW:
        raise ValueError(f"{path}: {w.size} weights, expected {GATE_NW}")
    return w, meta
