"""The allocation-free smooth sum (csbq_smooth_sum_noalloc) against the
allocating entry point csbq_smooth_sum, through the C ABI, on two calls in a
row, the second with a smaller input: within 1e-12 of the largest value of
each output (the same sum split into other source chunks)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

BAR = 1e-12


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


def _targets(sc, n_free, seed):
    """All surface nodes plus free targets 0.01 .. 0.5 off random nodes."""
    rng = np.random.default_rng(seed)
    k = rng.choice(sc.n_nodes, n_free, replace=False)
    return k, rng.uniform(0.01, 0.5, n_free) * np.where(rng.random(n_free) < 0.5, 1, -1)


@pytest.fixture(scope="module")
def ev():
    import torch
    import paper_2310_00889_amd as pk
    torch.zeros(1, device="cuda")
    e = pk.Evaluator(quad_tol=1e-12)
    yield e
    e.close()


def _compare(ev, sc, tn_host, x_host):
    import torch
    ev.set_geometry(sc)
    sig = torch.from_numpy(sc.sigma).cuda()
    tn = torch.from_numpy(tn_host).cuda()
    x = torch.from_numpy(x_host).cuda()
    us_a, ud_a = ev.smooth_sum_noalloc(sig, x, tn)
    fa = ev.flags()
    us_b, ud_b = ev.smooth_sum(sig, x, tn)
    torch.cuda.synchronize()
    es, ed = _rel(us_a, us_b), _rel(ud_a, ud_b)
    print(f"noalloc vs smooth_sum, {len(tn_host)} targets, {sc.n_nodes} nodes: u_S {es:.2e} u_D {ed:.2e}", flush=True)
    assert fa == 0
    assert es < BAR and ed < BAR
    assert torch.isfinite(us_a).all() and torch.isfinite(ud_a).all()


def test_noalloc_matches_smooth_sum_twice(ev):
    import oracle
    # first call: 6 pipe panels + 3 spheres, every node plus 500 free targets
    sc = synth.small_pipe_scene(n_panels=6, n_spheres=3)
    y, n, _ = oracle.nodes(sc)
    k, d = _targets(sc, 500, 7)
    tn = np.concatenate([np.arange(sc.n_nodes, dtype=np.int64), -np.ones(500, np.int64)])
    x = np.concatenate([np.zeros((sc.n_nodes, 3)), y[k] + d[:, None] * n[k]])
    _compare(ev, sc, tn, x)
    # second call, smaller: 2 panels + 1 sphere, 300 nodes and 37 free targets
    sc2 = synth.small_pipe_scene(n_panels=2, n_spheres=1)
    y2, n2, _ = oracle.nodes(sc2)
    k2, d2 = _targets(sc2, 37, 8)
    sel = np.random.default_rng(9).choice(sc2.n_nodes, 300, replace=False).astype(np.int64)
    tn2 = np.concatenate([sel, -np.ones(37, np.int64)])
    x2 = np.concatenate([np.zeros((300, 3)), y2[k2] + d2[:, None] * n2[k2]])
    _compare(ev, sc2, tn2, x2)


def test_noalloc_limits_and_flags(ev):
    import torch
    import paper_2310_00889_amd as pk
    sc = synth.small_pipe_scene(n_panels=2, n_spheres=1)
    ev.set_geometry(sc)
    sig = torch.from_numpy(sc.sigma).cuda()
    # more targets than the scratch holds: refused before any work
    big = torch.zeros((262145, 3), dtype=torch.float64, device="cuda") + 3.0
    with pytest.raises(pk.CsbqError, match="ELIMIT"):
        ev.smooth_sum_noalloc(sig, big, None)
    # an out-of-range node id is reported through the flag word
    bad = torch.tensor([0, sc.n_nodes + 5], dtype=torch.int64, device="cuda")
    ev.smooth_sum_noalloc(sig, None, bad)
    assert ev.flags() & pk.FLAG_NODE_RANGE
    good = torch.tensor([0, 9], dtype=torch.int64, device="cuda")
    us, ud = ev.smooth_sum_noalloc(sig, None, good)
    assert ev.flags() == 0
    torch.cuda.synchronize()
    assert torch.isfinite(us).all()
    # a batch of geometries is refused
    merged = synth.merge_scenes([sc, synth.small_pipe_scene(n_panels=1, n_spheres=1)])
    ev.set_geometry(merged)
    with pytest.raises(pk.CsbqError, match="EINVAL"):
        ev.smooth_sum_noalloc(torch.from_numpy(merged.sigma).cuda(), None, good)
