#!/usr/bin/env python3
"""Train the learned correction-tier gate and write its weights.

Training data are made by the method itself on the GPU: random batches of
pipe-with-spheres geometries of uneven size (panels U{20..60}, spheres
U{10..120}, radii U(0.1, 0.25), gaps 10**U(-3,-1); seeds disjoint from every
evaluation workload), evaluated with the criterion gate in mixed precision at
quad_tol 1e-7 (or in FP64 at the tolerance given).  For every candidate pair
the library computes the correction with each tier and labels the pair with
the cheapest tier that agrees with the special quadrature to label_tol of the
largest |u| (csbq_gate_dataset).  The network is trained with Adam on the
weighted ordinal cross-entropy (misses, i.e. a predicted tier below the
label, weighted 4x).

    python paper_2310_00889_amd/tables/train_gate.py --out paper_2310_00889_amd/tables/gate_mlp.npz
    python paper_2310_00889_amd/tables/train_gate.py --precision fp64 --quad-tol 1e-12 --label-tol 1e-13 \
        --out paper_2310_00889_amd/tables/gate_mlp_fp64.npz
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def log(msg):
    print(msg, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "gate_mlp.npz"))
    ap.add_argument("--batches", type=int, default=3)
    ap.add_argument("--geoms", type=int, default=6)
    ap.add_argument("--cap", type=int, default=700_000)
    ap.add_argument("--epochs", type=int, default=24)
    ap.add_argument("--quad-tol", type=float, default=1e-7)
    ap.add_argument("--label-tol", type=float, default=1e-8)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    a = ap.parse_args()
    import torch
    import synth
    import paper_2310_00889_amd as pk
    from paper_2310_00889_amd import gate

    torch.zeros(1, device="cuda")
    ev = pk.Evaluator(quad_tol=a.quad_tol, precision=a.precision)
    feats, labs, crits = [], [], []
    for b in range(a.batches):
        t0 = time.time()
        scs = synth.config4(seed=5100 + 37 * b, n_geom=a.geoms, max_spheres=120, max_panels=60)
        bs = synth.merge_scenes(scs)
        ev.set_geometry(bs)
        f, l, c = ev.gate_dataset(bs.sigma, None, bs.tgt_node, label_tol=a.label_tol, cap=a.cap)
        feats.append(f)
        labs.append(l)
        crits.append(c)
        log(f"batch {b}: {bs.n_nodes} nodes, {len(l)} pairs, labels {np.bincount(l, minlength=5).tolist()}, "
            f"criterion {np.bincount(c, minlength=5).tolist()}, {time.time() - t0:.1f} s")
    F = np.concatenate(feats)
    L = np.concatenate(labs)
    Cr = np.concatenate(crits)
    posw = np.array([4.0, 4.0, 4.0, 4.0], np.float32)
    w0 = gate.init_weights(seed=1)
    t0 = time.time()
    w, losses = ev.gate_train(F, L, posw, w0, epochs=a.epochs, batch=4096, lr=2e-3, seed=2)
    log(f"trained {a.epochs} epochs in {time.time() - t0:.1f} s; loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    ev.gate_load(w, 0.05)
    tier, esc, _ = ev.gate_infer(F)
    conf = np.zeros((5, 5), np.int64)
    np.add.at(conf, (L, tier), 1)
    miss = float(np.mean(tier < L))
    miss_kept = float(np.mean((tier < L) & (esc == 0)))
    log(f"confusion (label x predicted):\n{conf}")
    log(f"below label: {miss:.4f} of pairs; below label and not escalated: {miss_kept:.5f}; "
        f"escalated {float(np.mean(esc)):.3f}")
    gate.save_weights(a.out, w, losses=losses, posw=posw, quad_tol=a.quad_tol, label_tol=a.label_tol,
                      precision=a.precision,
                      n_train=len(L), label_counts=np.bincount(L, minlength=5),
                      criterion_counts=np.bincount(Cr, minlength=5), confusion=conf, miss=miss,
                      miss_kept=miss_kept, tau_esc=0.05)
    log(f"wrote {a.out}")


if __name__ == "__main__":
    main()
