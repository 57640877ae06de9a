"""Batched geometries (several independent scenes in one context): one
evaluation over the batch equals every scene evaluated alone, and the oracle
per scene; free targets carry their group; unordered groups are rejected."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GATE = 1e-10


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def evs():
    import torch
    import paper_2310_00889_amd as pk
    torch.zeros(1, device="cuda")
    a, b = pk.Evaluator(quad_tol=1e-12), pk.Evaluator(quad_tol=1e-12)
    yield a, b
    a.close()
    b.close()


def _scenes():
    return [synth.small_pipe_scene(seed=7000 + 100 * k, n_panels=3 + k, n_spheres=1 + k % 3) for k in range(4)]


def test_batch_equals_separate_and_oracle(evs):
    ev, ev1 = evs
    scs = _scenes()
    b = synth.merge_scenes(scs)
    ev.set_geometry(b)
    us, ud = ev.eval(b.sigma, None, b.tgt_node)
    rng = np.random.default_rng(11)
    for g, sc in enumerate(scs):
        sl = slice(int(b.group_target_offsets[g]), int(b.group_target_offsets[g + 1]))
        ev1.set_geometry(sc)
        tn = np.arange(sc.n_nodes, dtype=np.int64)
        u1, d1 = ev1.eval(sc.sigma, None, tn)
        print(f"group {g}: batch vs alone S {_rel(us[sl], u1):.2e} D {_rel(ud[sl], d1):.2e}", flush=True)
        assert _rel(us[sl], u1) < 1e-12 and _rel(ud[sl], d1) < 1e-12
        k = rng.choice(sc.n_nodes, 12, replace=False)
        uo, do = oracle.evaluate(sc, None, None, tn[k])
        print(f"group {g}: vs oracle S {_rel(us[sl][k], uo):.2e} D {_rel(ud[sl][k], do):.2e}", flush=True)
        assert _rel(us[sl][k], uo) < GATE and _rel(ud[sl][k], do) < GATE


def test_batch_free_targets_with_groups(evs):
    ev, ev1 = evs
    scs = _scenes()
    b = synth.merge_scenes(scs)
    ev.set_geometry(b)
    rng = np.random.default_rng(12)
    xs, gs, per = [], [], []
    for g, sc in enumerate(scs):
        y, n, _ = oracle.nodes(sc)
        k = rng.choice(sc.n_nodes, 40, replace=False)
        d = 10.0 ** rng.uniform(-3, -0.5, 40) * np.where(rng.random(40) < 0.5, 1, -1)
        x = y[k] + d[:, None] * n[k]
        xs.append(x)
        gs.append(np.full(40, g, np.int32))
        per.append(x)
    x = np.concatenate(xs)
    grp = np.concatenate(gs)
    us, ud = ev.eval(b.sigma, x, None, tgt_group=grp)
    for g, sc in enumerate(scs):
        ev1.set_geometry(sc)
        u1, d1 = ev1.eval(sc.sigma, per[g], None)
        sl = slice(40 * g, 40 * (g + 1))
        assert _rel(us[sl], u1) < 1e-12 and _rel(ud[sl], d1) < 1e-12, g
    import paper_2310_00889_amd as pk
    with pytest.raises(pk.CsbqError):
        ev.eval(b.sigma, x, None, tgt_group=grp[::-1].copy())
    with pytest.raises(pk.CsbqError):
        ev.eval(b.sigma, x, None, tgt_group=np.full(len(x), len(scs), np.int32))


def test_batch_64_geometries_sampled(evs):
    """64 uneven pipe geometries (panels U{20..30}, spheres U{10..30}) in one
    batch, all nodes as targets; two sampled targets per geometry against the
    oracle."""
    import torch
    ev, _ = evs
    scs = synth.config4(max_spheres=30, max_panels=30)
    b = synth.merge_scenes(scs)
    ev.set_geometry(b)
    sig = torch.from_numpy(b.sigma).cuda()
    tn = torch.from_numpy(b.tgt_node).cuda()
    us, ud = ev.eval(sig, None, tn)
    torch.cuda.synchronize()
    us, ud = us.cpu().numpy(), ud.cpu().numpy()
    st = ev.stats()
    print("batch64 stats", st, flush=True)
    assert np.isfinite(us).all() and np.isfinite(ud).all()
    rng = np.random.default_rng(13)
    worst = [0.0, 0.0]
    for g, sc in enumerate(scs):
        k = rng.choice(sc.n_nodes, 2, replace=False)
        uo, do = oracle.evaluate(sc, None, None, k.astype(np.int64))
        t = int(b.group_target_offsets[g]) + k
        scale_s = np.abs(uo).max()
        scale_d = np.abs(do).max()
        worst[0] = max(worst[0], np.abs(us[t] - uo).max() / scale_s)
        worst[1] = max(worst[1], np.abs(ud[t] - do).max() / scale_d)
    print("batch64 worst vs oracle", worst, flush=True)
    assert worst[0] < GATE and worst[1] < GATE


def test_batch_plan_apply_per_geometry(evs):
    """The setup/apply split on a batch: plan on 16 uneven geometries (all
    nodes), then apply a second density; each geometry's part against the
    oracle (sampled) and against the batch's own eager evaluation of that
    density (rounding only)."""
    import torch
    ev, ev1 = evs
    scs = synth.config4(seed=4100, n_geom=16, max_spheres=20, max_panels=24)
    b = synth.merge_scenes(scs)
    ev.set_geometry(b)
    sig = torch.from_numpy(b.sigma).cuda()
    tn = torch.from_numpy(b.tgt_node).cuda()
    ev.plan(sig, None, tn, full_band=True)   # rules for any density's band
    sig2 = 0.5 * b.sigma + np.roll(b.sigma, 1, axis=1)
    us, ud = ev.apply(torch.from_numpy(sig2).cuda())
    torch.cuda.synchronize()
    us, ud = us.cpu().numpy(), ud.cpu().numpy()
    ev1.set_geometry(b)
    ue, de = ev1.eval(sig2, None, b.tgt_node)
    assert _rel(us, ue) < 1e-12 and _rel(ud, de) < 1e-12
    rng = np.random.default_rng(14)
    for g, sc in enumerate(scs):
        off = int(b.group_target_offsets[g])
        k = rng.choice(sc.n_nodes, 3, replace=False)
        s2 = sig2[off: off + sc.n_nodes]   # targets are every node, in geometry order
        uo, do = oracle.evaluate(sc, s2, None, k.astype(np.int64))
        es, ed = _rel(us[off + k], uo), _rel(ud[off + k], do)
        assert es < GATE and ed < GATE, (g, es, ed)


def test_batch_mixed_precision_sampled(evs):
    """A batch in mixed precision (FP32 smooth sum with the FP64 near part,
    quad_tol 1e-7) against the oracle, 3 sampled targets per geometry: 1e-6."""
    import torch
    import paper_2310_00889_amd as pk
    scs = synth.config4(seed=4200, n_geom=16, max_spheres=20, max_panels=24)
    b = synth.merge_scenes(scs)
    ev = pk.Evaluator(quad_tol=1e-7, precision="mixed")
    try:
        ev.set_geometry(b)
        us, ud = ev.eval(torch.from_numpy(b.sigma).cuda(), None, torch.from_numpy(b.tgt_node).cuda())
        torch.cuda.synchronize()
        us, ud = us.cpu().numpy(), ud.cpu().numpy()
    finally:
        ev.close()
    rng = np.random.default_rng(15)
    worst = [0.0, 0.0]
    for g, sc in enumerate(scs):
        off = int(b.group_target_offsets[g])
        k = rng.choice(sc.n_nodes, 3, replace=False)
        uo, do = oracle.evaluate(sc, None, None, k.astype(np.int64))
        worst[0] = max(worst[0], _rel(us[off + k], uo))
        worst[1] = max(worst[1], _rel(ud[off + k], do))
    print("mixed batch worst vs oracle", worst, flush=True)
    assert worst[0] < 1e-6 and worst[1] < 1e-6


def test_config4_full_range_geometry_sampled(evs):
    """One geometry at the top of config 4's ranges (200 pipe panels, 500
    spheres, radii U(0.1, 0.25), gaps 10^U(-3,-1)), in a batch with a small
    one: 24 sampled targets (stratified: wall, spheres, nearest-contact
    sphere nodes) against the oracle, 1e-10."""
    import torch
    ev, _ = evs
    rng = np.random.default_rng(4300)
    M = 500
    radii = rng.uniform(0.1, 0.25, M)
    gaps = 10.0 ** rng.uniform(-3, -1, M)
    vs = np.sum(4 / 3 * np.pi * radii ** 3)
    lam = max(1.0, (vs / (0.136 * np.pi * 5.0 * np.pi)) ** (1 / 3))
    big = synth.pipe_scene(4301, M, lam, n_panels=200, radii=radii, gaps=gaps)
    small = synth.small_pipe_scene(seed=7300, n_panels=3, n_spheres=1)
    b = synth.merge_scenes([big, small])
    ev.set_geometry(b)
    us, ud = ev.eval(torch.from_numpy(b.sigma).cuda(), None, torch.from_numpy(b.tgt_node).cuda())
    torch.cuda.synchronize()
    assert ev.flags() == 0
    us, ud = us.cpu().numpy()[: big.n_nodes], ud.cpu().numpy()[: big.n_nodes]
    nwall = 200 * 512
    y, _, _ = oracle.nodes(big)
    sph = np.arange(nwall, big.n_nodes)
    # sphere nodes nearest another sphere's surface
    cen, rad = big.sphere_centers, big.sphere_radii
    owner = (sph - nwall) // 512
    dmin = np.full(len(sph), np.inf)
    for j in range(len(cen)):
        dj = np.linalg.norm(y[sph] - cen[j], axis=1) - rad[j]
        dj[owner == j] = np.inf
        dmin = np.minimum(dmin, dj)
    pick = np.concatenate([rng.choice(nwall, 8, replace=False), rng.choice(sph, 8, replace=False),
                           sph[np.argsort(dmin)[:8]]]).astype(np.int64)
    uo, do = oracle.evaluate(big, None, None, pick)
    es, ed = _rel(us[pick], uo), _rel(ud[pick], do)
    print("config-4 full-range geometry vs oracle", es, ed, flush=True)
    assert es < GATE and ed < GATE
