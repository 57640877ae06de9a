#!/usr/bin/env python3
"""Benchmark: Stokes single- and double-layer potentials at all surface nodes of
the pipe-with-spheres workload (torus-arc pipe of 100 panels, 200 spheres of
radius 0.2; 153,600 nodes = sources = on-surface targets), FP64, quadrature
tolerance 1e-12.

One step = one full evaluation (near-pair search, gate, corrections, smooth
sum, reduction) with geometry, density and targets already resident in HBM.
Prints one JSON line.  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "layer-potential target evals/sec at rel.err 1e-10 (FP64) and 1e-6 (mixed+MLP)"
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector peak
FP32_PEAK_TFLOPS = 157.3         # MI355X FP32 vector peak (the mixed-precision smooth sum)
# Algorithmic count of the smooth sum: 48 flops (FMA = 2, 1/sqrt = 1) for S and
# D of one pair of surface nodes, over every (node, node) pair -- the work the
# method's Nystrom sum defines, whatever rules the implementation sums.
ALG_FLOPS_PER_PAIR = 48
FAR_FLOPS_PER_PAIR = 44          # the implementation's own count per summed pair (its 1/2 powers taken out)
# special quadrature flops: per theta-rule node 82 + 9 per density Fourier mode
# (synthesis; a mirror pair of nodes shares one recurrence, 18 flops per pair
# and mode), per s-node 800 (interpolation weights, centerline data, frame,
# local coordinates) + 192 per mode (6 coefficients x 16-point interpolation)
THETA_FLOPS, THETA_MODE_FLOPS = 82, 9
SNODE_FLOPS, SNODE_MODE_FLOPS = 800, 192


WORKLOADS = {
    "pipe100-spheres200": "pipe100-spheres200: torus-arc pipe (R=5, r=1, arc pi, 100 panels) + 200 spheres r=0.2, "
                          "16x32 nodes per element, 153,600 sources = on-surface targets",
    "batch64-full": "batch64-full: 64 independent torus-arc pipes, panels U{20..200} + spheres U{10..500} "
                    "r U(0.1,0.25), 16x32 nodes per element, 11,493,888 on-surface targets",
}


def measured_traffic(kernel, precision):
    """HBM bytes per launch of `kernel` from the committed memory-counter
    record, or None when there is none or the kernels have changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_pipe100_spheres200_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, "paper_2310_00889_amd", "csrc", "csbq_kernels.hip"), "rb") as f:
        sha = hashlib.sha1(f.read()).hexdigest()
    return rec["traffic_bytes"] if rec.get("kernels_sha1") == sha else None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, n_sample, seconds):
    import numpy as np
    import oracle
    rng = np.random.default_rng(12345)
    nwall = sc.bodies[0].n_panels * sc.ns * sc.nt
    idx = np.concatenate([rng.choice(nwall, n_sample // 3, replace=False),
                          nwall + rng.choice(sc.n_nodes - nwall, n_sample - n_sample // 3, replace=False)])
    threads = oracle.num_threads()
    t0 = time.time()
    done = 0
    chunk = max(threads, 8)
    while done < len(idx) and time.time() - t0 < seconds:
        sel = idx[done:done + chunk]
        oracle.evaluate(sc, None, None, sc.tgt_node[sel])
        done += len(sel)
    dt = time.time() - t0
    return dict(value=done / dt, unit="target evals/s", cores=threads, kind="oracle",
                sample=f"{done} on-surface targets of the same workload (1/3 wall, 2/3 particle), {dt:.1f} s",
                cpu_model=cpu_model(), nproc=os.cpu_count())


def run_mode(sc, sig, tn, precision, gate, quad_tol, steps, warmup, ref=None):
    """One evaluation mode on the resident workload: timing, phases and, given
    the reference outputs, the largest deviation per output and target class
    relative to that class's largest reference value."""
    import torch
    import paper_2310_00889_amd as pk
    ev = pk.Evaluator(quad_tol=quad_tol, precision=precision, gate=gate)
    if gate == "mlp":
        from paper_2310_00889_amd import gate as gmod
        w, meta = gmod.load_weights(gmod.FP64_WEIGHTS if precision == "fp64" else gmod.DEFAULT_WEIGHTS)
        ev.gate_load(w, float(meta["tau_esc"]))
    ev.set_geometry(sc)
    T = int(tn.shape[0])
    usl = torch.empty((T, 3), dtype=torch.float64, device="cuda")
    udl = torch.empty((T, 3), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        ev.eval(sig, None, tn, usl, udl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ev.eval(sig, None, tn, usl, udl)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ev.stats()
    out = dict(precision=precision, gate=gate, quad_tol=quad_tol, value=T * steps / dt,
               ms_per_step=1e3 * dt / steps, steps=steps, phases_ms=st.get("ms"), flags=ev.flags(),
               pairs={k: st.get(k) for k in ("candidates", "pairs_up1", "pairs_up2", "pairs_up3", "pairs_full",
                                             "gate_escalated")})
    if ref is not None:
        cls = torch.from_numpy(sc.tgt_class).cuda()
        errs = {}
        for name, u, r in (("S", usl, ref[0]), ("D", udl, ref[1])):
            for c in sorted(set(sc.tgt_class.tolist())):
                m = cls == c
                errs[f"{name}_{sc.class_names[c]}"] = float((u[m] - r[m]).abs().max() / r[m].abs().max())
        out["rel_err_vs_fp64_1e-12"] = errs
    ev.close()
    return out


def run_matrix(sc, sig, tn, quad_tol, steps, ref):
    """Plan with the special-quadrature pairs' correction matrices (built once)
    and time applies of the density: ms per apply, the build time, the
    matrices' size and the apply kernel's bandwidth (it reads every matrix once)."""
    import torch
    import paper_2310_00889_amd as pk
    ev = pk.Evaluator(quad_tol=quad_tol)
    ev.set_geometry(sc)
    T = int(tn.shape[0])
    usl = torch.empty((T, 3), dtype=torch.float64, device="cuda")
    udl = torch.empty((T, 3), dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    ev.plan(sig, None, tn, usl, udl, matrix=True)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    st = ev.stats()
    ev.apply(sig, usl, udl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ev.apply(sig, usl, udl)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    errs = {name: float((u - r).abs().max() / r.abs().max()) for name, u, r in (("S", usl, ref[0]), ("D", udl, ref[1]))}
    mb = st["plan"]["matrix_bytes"]
    out = dict(ms_per_apply=1e3 * dt, value=T / dt, unit="target evals/s", plan_s=plan_s,
               build_ms=st["plan"]["build_ms"], matrix_bytes=mb, pairs_full=st.get("pairs_full"),
               rel_err_vs_eval=errs)
    ev.close()
    return out


def run_slender(steps, n_panels=64, eps=1e-3):
    """Every node of a slender torus (R = 1, cross-section radius eps,
    n_panels elements; aspect 2 pi / (n_panels eps) per element) as an
    on-surface target, FP64 at quad_tol 1e-12, with the whole-element singular
    s-rules and with the general rule (dyadic panels and the log rule): ms per
    evaluation, the special quadrature's share and s-node count, and the
    largest difference between the two."""
    import numpy as np
    import torch
    import paper_2310_00889_amd as pk
    import synth
    sc = synth.Scene([synth.torus_body(n_panels, 1.0, eps)])
    rng = np.random.default_rng(17)
    sig = torch.from_numpy(rng.standard_normal((sc.n_nodes, 3))).cuda()
    tn = torch.arange(sc.n_nodes, dtype=torch.int64, device="cuda")
    T = sc.n_nodes
    out = dict(workload=f"torus R=1, eps={eps:g}, {n_panels} elements (aspect {2 * np.pi / (n_panels * eps):.0f}), "
                        f"{T} on-surface targets, FP64, quad_tol 1e-12")
    res = {}
    for srule in ("whole", "general"):
        ev = pk.Evaluator(quad_tol=1e-12, srule=srule)
        ev.set_geometry(sc)
        usl = torch.empty((T, 3), dtype=torch.float64, device="cuda")
        udl = torch.empty((T, 3), dtype=torch.float64, device="cuda")
        ev.eval(sig, None, tn, usl, udl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ev.eval(sig, None, tn, usl, udl)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        st = ev.stats()
        res[srule] = (usl.clone(), udl.clone())
        out[srule] = dict(ms_per_eval=1e3 * dt, value=T / dt, special_quadrature_ms=st["ms"]["corr_full"],
                          s_nodes=st.get("s_nodes"), pairs_whole_rule=st.get("pairs_whole_rule"),
                          pairs_full=st.get("pairs_full"), flags=ev.flags())
        ev.close()
    out["rel_diff"] = {name: float((res["whole"][k] - res["general"][k]).abs().max() / res["general"][k].abs().max())
                       for k, name in ((0, "S"), (1, "D"))}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--workload", default="pipe100-spheres200", choices=["pipe100-spheres200", "batch64-full"],
                    help="batch64-full: 64 independent pipe geometries, panels U{20..200}, spheres U{10..500} "
                         "(11.5M targets; building it takes minutes of host time)")
    ap.add_argument("--gate", default=None, choices=["criterion", "mlp"],
                    help="correction-tier gate (default: criterion for fp64, the trained network for mixed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--copy-check", action="store_true",
                    help="first copy 1 GiB device to device (a known-size reference for memory counters)")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the three evaluation modes at quad_tol 1e-7 timed after the headline run")
    ap.add_argument("--mode-steps", type=int, default=5)
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not supported"}))
        sys.exit(2)
    import numpy as np
    import torch
    import synth
    import paper_2310_00889_amd as pk

    log("bench: building workload")
    if a.workload == "batch64-full":
        scenes = synth.config4(progress=lambda g, s: log(f"bench: geometry {g + 1}/64, {s.n_nodes} nodes"))
        sc = synth.merge_scenes(scenes)
        base_sc = scenes[0]   # the CPU baseline samples one geometry (the oracle knows no batches)
    else:
        sc = synth.config2()
        base_sc = sc
    quad_tol = 1e-12 if a.precision == "fp64" else 1e-7   # under the 1e-10 / 1e-6 parity gates
    gate = a.gate or ("criterion" if a.precision == "fp64" else "mlp")
    ev = pk.Evaluator(quad_tol=quad_tol, precision=a.precision, gate=gate)
    if gate == "mlp":
        from paper_2310_00889_amd import gate as gmod
        w, meta = gmod.load_weights(gmod.FP64_WEIGHTS if a.precision == "fp64" else gmod.DEFAULT_WEIGHTS)
        ev.gate_load(w, float(meta["tau_esc"]))
    ev.set_geometry(sc)
    sig = torch.from_numpy(sc.sigma).cuda()
    tn = torch.from_numpy(sc.tgt_node).cuda()
    T = int(tn.shape[0])
    usl = torch.empty((T, 3), dtype=torch.float64, device="cuda")
    udl = torch.empty((T, 3), dtype=torch.float64, device="cuda")
    if a.copy_check:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(f"bench: {T} targets, {ev.n_nodes} sources; warmup {a.warmup}")
    for _ in range(a.warmup):
        ev.eval(sig, None, tn, usl, udl)
    torch.cuda.synchronize()
    log(f"bench: timing {a.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        ev.eval(sig, None, tn, usl, udl)
        log(f"bench: step {k + 1}/{a.steps} enqueued")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # per-phase times of the last timed step (HIP events on the library's stream)
    counts = ev.stats()
    phases = counts["ms"]
    value = T * a.steps / dt
    # roofline of the dominant kernel, timed with HIP events on the library's stream
    dom = max(("far", "corr_full"), key=lambda k: phases.get(k, 0.0))
    nsrc = counts.get("sources_base", ev.n_nodes)
    far_pairs = float(counts.get("far_pairs") or float(T) * nsrc)   # a batch pairs targets with their group only
    if dom == "far":
        flops = FAR_FLOPS_PER_PAIR * far_pairs
    else:
        flops = (THETA_FLOPS * float(counts.get("theta_nodes", 0)) + THETA_MODE_FLOPS * float(counts.get("theta_modes", 0))
                 + SNODE_FLOPS * float(counts.get("s_nodes", 0)) + SNODE_MODE_FLOPS * float(counts.get("s_modes", 0)))
    achieved = flops / (phases[dom] * 1e-3) / 1e12
    far_kernel = "k_far" if a.precision == "fp64" else "k_far_mx"
    far_peak = FP64_PEAK_TFLOPS if a.precision == "fp64" else FP32_PEAK_TFLOPS
    peak = far_peak if dom == "far" else FP64_PEAK_TFLOPS
    roof = dict(kernel=far_kernel if dom == "far" else "k_corr_full", bound="alu", achieved=achieved,
                peak=peak, unit="TFLOP/s", frac=achieved / peak,
                traffic=measured_traffic(far_kernel if dom == "far" else "k_corr_full", a.precision)
                if a.workload == "pipe100-spheres200" else None)   # the counters were taken on that workload
    far_ach = FAR_FLOPS_PER_PAIR * far_pairs / (phases["far"] * 1e-3) / 1e12
    # the smooth sum's algorithmic rate: 48 flops per pair of surface nodes of
    # one geometry (the implementation sums other pairs: a block of targets
    # sums a body closed at its poles with its 32 x 32 far-field rule near it,
    # farther away with a coarser tensor rule, down to 16 x 16)
    node_pairs = float(T) * float(ev.n_nodes) if a.workload == "pipe100-spheres200" else None
    if node_pairs is not None and dom == "far":
        alg = ALG_FLOPS_PER_PAIR * node_pairs / (phases["far"] * 1e-3) / 1e12
        roof_alg = dict(kernel=far_kernel, bound="alu", achieved=alg, peak=far_peak, unit="TFLOP/s",
                        frac=alg / far_peak, traffic=roof["traffic"],
                        flops=f"{ALG_FLOPS_PER_PAIR} per pair of surface nodes x {T} targets x {ev.n_nodes} nodes")
        roof_impl = dict(roof, flops=f"{FAR_FLOPS_PER_PAIR} per summed pair x {int(far_pairs)} pairs "
                                     "(spheres: 32 x 32 near, coarser tensor rules by distance)")
        roof = roof_alg
    else:
        roof_impl = None
    out = {
        "metric": METRIC, "value": value, "unit": "target evals/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * dt / a.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if a.precision == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[a.workload],
                   "quad_tol": quad_tol, "precision": a.precision, "gate": gate, "targets": T, "sources": ev.n_nodes},
        "roofline": roof,
        "roofline_impl": roof_impl,
        "far_roofline": dict(kernel=far_kernel, bound="alu", achieved=far_ach,
                             peak=far_peak, unit="TFLOP/s", frac=far_ach / far_peak),
        "phases_ms": phases,
        "pairs": {k: counts.get(k) for k in ("far_pairs", "candidates", "pairs_up1", "pairs_up2", "pairs_up3",
                                              "pairs_full", "theta_nodes", "theta_modes", "s_nodes", "s_modes",
                                              "sources_base")},
    }
    out["flags"] = ev.flags()
    if not a.no_modes and a.workload == "pipe100-spheres200" and a.precision == "fp64":
        # the same workload at quad_tol 1e-7 (under the 1e-6 bar) in three
        # modes, each checked against the headline FP64 result (quad_tol
        # 1e-12, itself within 1e-10 of the oracle)
        ref = (usl.clone(), udl.clone())
        usl_ref, udl_ref = ref
        ev.close()
        modes = {}
        for prec, gt in (("fp64", "criterion"), ("mixed", "criterion"), ("mixed", "mlp")):
            log(f"bench: mode {prec}+{gt} at quad_tol 1e-7")
            modes[f"{prec}+{gt}@1e-7"] = run_mode(sc, sig, tn, prec, gt, 1e-7, a.mode_steps, 2, ref)
        out["modes_at_1e-7"] = modes
        # FP64 at the headline tolerance with the network trained for it
        # (labels at 1e-13), against the headline result on every target
        log("bench: mode fp64+mlp at quad_tol 1e-12")
        out["fp64_mlp_at_1e-12"] = run_mode(sc, sig, tn, "fp64", "mlp", 1e-12, a.mode_steps, 2, ref)
    if not a.no_modes and a.workload == "pipe100-spheres200" and a.precision == "fp64":
        # the setup/evaluation split with stored correction matrices (the
        # special-quadrature pairs' E): build time once, then timed applies of
        # the same density, checked against the headline result
        log("bench: matrix plan")
        out["matrix_apply"] = run_matrix(sc, sig, tn, 1e-12, a.mode_steps, (usl_ref, udl_ref))
    if not a.no_modes and a.workload == "pipe100-spheres200" and a.precision == "fp64":
        # slender elements: whole-element singular s-rules against the
        # general rule on a slender torus's on-surface targets
        log("bench: slender torus, whole-element and general s-rules")
        out["slender_torus"] = run_slender(a.mode_steps)
    if not a.no_cpu_baseline:
        log("bench: timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(base_sc, 240, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
