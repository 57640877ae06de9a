"""Host-side logic that runs without a GPU: batch assembly, the learned gate's
weight files and constants, the measured-traffic record, the benchmark's
one-GPU check, and a clean failure when no device is present."""
import json
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_merge_scenes_offsets_groups_and_targets():
    a = synth.small_pipe_scene(n_panels=3, n_spheres=1)
    b = synth.small_pipe_scene(seed=7100, n_panels=4, n_spheres=2)
    m = synth.merge_scenes([a, b])
    assert m.n_nodes == a.n_nodes + b.n_nodes
    assert list(m.body_group) == [0] * len(a.bodies) + [1] * len(b.bodies)
    assert list(m.group_node_offsets) == [0, a.n_nodes, a.n_nodes + b.n_nodes]
    assert list(m.group_target_offsets) == [0, a.n_nodes, a.n_nodes + b.n_nodes]
    # targets default to all nodes, renumbered into the merged node list
    assert np.array_equal(m.tgt_node, np.arange(m.n_nodes))
    assert np.array_equal(m.sigma[:a.n_nodes], a.sigma) and np.array_equal(m.sigma[a.n_nodes:], b.sigma)
    f = m.flat()
    assert f["n_bodies"] == len(a.bodies) + len(b.bodies)
    assert f["xc"].shape[0] == (a.n_panels + b.n_panels) * synth.NS


def test_gate_constants_match_header():
    import paper_2310_00889_amd as pk
    from paper_2310_00889_amd import gate
    h = open(os.path.join(ROOT, "include", "csbq.h")).read()
    consts = dict(re.findall(r"#define CSBQ_GATE_(\w+) (\d+)", h))
    assert int(consts["NF"]) == pk.GATE_NF and int(consts["NO"]) == pk.GATE_NO and int(consts["NW"]) == pk.GATE_NW
    n = sum(int(np.prod(s)) for _, s in gate.SHAPES)
    assert n == pk.GATE_NW


def test_gate_weights_roundtrip(tmp_path):
    from paper_2310_00889_amd import gate
    w = gate.init_weights(seed=4)
    p = tmp_path / "w.npz"
    gate.save_weights(p, w, tau_esc=0.05, note="test")
    w2, meta = gate.load_weights(p)
    assert np.array_equal(w, w2) and float(meta["tau_esc"]) == 0.05
    parts = gate.unpack(w2)
    assert parts["W2"].shape == (64, 64) and parts["b4"].shape == (4,)
    # He initialisation: biases zero, weight scale sqrt(2 / fan_in)
    assert np.all(parts["b1"] == 0) and abs(parts["W2"].std() - np.sqrt(2 / 64)) < 0.02
    with pytest.raises(ValueError):
        gate.save_weights(p, w[:-1])
        gate.load_weights(p)


def test_shipped_gate_weights():
    from paper_2310_00889_amd import gate
    if not os.path.exists(gate.DEFAULT_WEIGHTS):
        pytest.skip("no trained weights shipped")
    w, meta = gate.load_weights()
    assert np.isfinite(w).all()
    assert 0 < float(meta["tau_esc"]) < 1
    assert float(meta["quad_tol"]) == 1e-7
    conf = np.asarray(meta["confusion"])
    assert conf.shape == (5, 5) and conf.sum() == int(meta["n_train"])


def test_traffic_records_are_complete():
    import glob
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*_pipe100_spheres200_*.json")))
    assert paths
    for path in paths:
        rec = json.load(open(path))
        for k in ("kernel", "precision", "fetch_kib", "write_kib", "fetch_factor", "write_factor", "traffic_bytes",
                  "kernels_sha1", "commands"):
            assert k in rec, (path, k)
        assert os.path.basename(path) == f"traffic_{rec['kernel']}_pipe100_spheres200_{rec['precision']}.json"
        expect = rec["fetch_kib"] * 1024 / rec["fetch_factor"] + rec["write_kib"] * 1024 / rec["write_factor"]
        assert abs(expect - rec["traffic_bytes"]) < 1e-6 * expect


def test_bench_refuses_more_than_one_gpu():
    """The benchmark is a one-GPU measurement: --gpus N with N != 1 exits
    with status 2 and a JSON error line before touching any device."""
    import subprocess
    import sys
    for n in ("2", "8"):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", n], capture_output=True,
                           text=True, timeout=120, cwd=ROOT)
        assert r.returncode == 2, (n, r.returncode, r.stderr[-500:])
        line = json.loads(r.stdout.strip().splitlines()[-1])
        assert "one GPU" in line["error"]


def test_binding_checks_sizes_and_types_before_the_c_abi():
    """The C ABI takes bare pointers, so the binding refuses any array whose
    size or element type does not match the geometry and the targets."""
    import paper_2310_00889_amd as pk
    ev = pk.Evaluator.__new__(pk.Evaluator)   # no device needed for the checks
    ev.n_nodes = 10
    sig = np.zeros((10, 3))
    tn = np.arange(4, dtype=np.int64)
    assert ev._check_shapes(sig, None, tn, None, None, None) == 4
    assert ev._check_shapes(sig, np.zeros((5, 3)), None, np.zeros(5, np.int32), np.zeros((5, 3)), None) == 5
    bad = [(np.zeros((9, 3)), None, tn, None, None, None),                  # density of 9 nodes
           (sig.astype(np.float32), None, tn, None, None, None),            # float32 density
           (sig, np.zeros((5, 3)), tn, None, None, None),                   # x and tgt_node disagree on T
           (sig, None, tn.astype(np.int32), None, None, None),              # int32 node ids
           (sig, None, tn, np.zeros(4, np.int64), None, None),              # int64 groups
           (sig, None, tn, None, np.zeros((3, 3)), None),                   # short output
           (sig, None, None, None, None, None)]                             # no targets
    for args in bad:
        with pytest.raises(pk.CsbqError):
            ev._check_shapes(*args)


def test_create_without_device_fails_cleanly():
    import torch
    import paper_2310_00889_amd as pk
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    if not os.path.exists(pk.LIB_PATH):
        pytest.skip("libcsbq.so not built")
    with pytest.raises(pk.CsbqError):
        pk.Evaluator(stream=0)
