"""GPU path vs the CPU oracle (element by element on the same seeded inputs).

Bar: every output within 1e-10 of the oracle relative to the largest oracle
value of that output (u_S or u_D) and target class; geometry and the plain
smooth sum within 1e-12 (1e-10 for the fat-pipe normals and weights, whose
second centerline derivatives carry ~1e-11 rounding in both evaluators)."""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GATE = 1e-10


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def ev():
    import torch
    import paper_2310_00889_amd as pk
    torch.zeros(1, device="cuda")           # initialise the device through torch first
    e = pk.Evaluator(quad_tol=1e-12)
    yield e
    e.close()


def _no_flags(ev):
    """The last evaluation raised no accuracy warning (s-rule limit, theta
    bracket clamp) or input flag."""
    f = ev.flags()
    assert f == 0, f"evaluation flags {f}"


def _argmax_report(u, uo, what, tn=None, x=None):
    """Print where the largest deviation sits: target index, node id and
    element (on-surface) or position (free target)."""
    k = int(np.unravel_index(np.argmax(np.abs(u - uo)), u.shape)[0])
    where = f"node {int(tn[k])} element {int(tn[k]) // 512}" if tn is not None and tn[k] >= 0 else \
        (f"x {np.round(x[k], 6).tolist()}" if x is not None else "")
    print(f"{what}: worst target {k} {where} |du| {np.abs(u[k] - uo[k]).max():.2e}", flush=True)


def _check_classes(u, uo, cls, what, tn=None, x=None):
    _argmax_report(u, uo, what, tn, x)
    for c in np.unique(cls):
        m = cls == c
        err = np.abs(u[m] - uo[m]).max() / np.abs(uo[m]).max()
        print(f"{what} class {c}: {err:.2e}", flush=True)
        assert err < GATE, (what, c, err)


def test_native_library_is_loaded(ev):
    import paper_2310_00889_amd as pk
    with open("/proc/self/maps") as f:
        maps = f.read()
    assert os.path.realpath(pk.LIB_PATH) in maps


def test_smoke_in_a_fresh_process():
    """The smoke entry point in a process where nothing has imported torch
    before the package loads its library (the HIP runtime must be torch's)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", "import __graft_entry__ as g; g.smoke()"], cwd=root,
                       capture_output=True, text=True, timeout=300)
    print(r.stdout[-400:], r.stderr[-400:], flush=True)
    assert r.returncode == 0


def test_nodes_match_oracle(ev):
    for sc, tol in ((synth.config1(4), 1e-13), (synth.small_pipe_scene(), 1e-10)):
        ev.set_geometry(sc)
        y, n, w = ev.nodes()
        yo, no, wo = oracle.nodes(sc)
        assert _rel(y, yo) < 1e-13
        assert np.abs(n - no).max() < tol
        assert _rel(w, wo) < tol


def test_smooth_sum_matches_oracle(ev):
    sc = synth.small_pipe_scene(n_panels=6, n_spheres=3)
    ev.set_geometry(sc)
    rng = np.random.default_rng(1)
    # free targets away from the surfaces: a well-conditioned sum
    y, n, _ = oracle.nodes(sc)
    k = rng.choice(sc.n_nodes, 200, replace=False)
    x = y[k] + rng.uniform(0.05, 1.0, 200)[:, None] * n[k] * np.where(rng.random(200) < 0.5, 1, -1)[:, None]
    us, ud = ev.smooth_sum(sc.sigma, x, None)
    uso, udo = oracle.smooth_sum(sc, None, x, -np.ones(200, np.int64))
    assert _rel(us, uso) < 1e-12 and _rel(ud, udo) < 1e-12
    # on-surface targets sum 1/r (and (r.n)/r^3) over neighbours ~1e-3 away
    # near a sphere's poles: terms up to ~1e3 times the sum, and a change of
    # a node position by dy changes a term by up to ~dy/r of itself (the D
    # term's (r.n) factor, ~r^2 on a smooth surface, by ~dy/r^2).  The two
    # sums run over two evaluations of the geometry (nodes, normals, weights
    # that differ by the amounts measured here, each bounded by
    # test_nodes_match_oracle), so each target's difference is bounded by the
    # rounding of the sums (64 eps of the sum of |term|) plus the first-order
    # change those differences can make, from the oracle's change bounds
    # (per unit displacement of the target and of every node; per unit
    # change of every normal), with a factor 2 of margin
    ys, ns_, ws = ev.nodes()
    dy = np.abs(ys - y).max()
    dn = np.abs(ns_ - n).max()
    _, _, wo = oracle.nodes(sc)
    dw = (np.abs(ws - wo) / np.abs(wo)).max()
    tn = rng.choice(sc.n_nodes, 300, replace=False)
    us, ud = ev.smooth_sum(sc.sigma, None, tn)
    uso, udo = oracle.smooth_sum(sc, None, None, tn)
    mag = oracle.smooth_sum_magnitude(sc, None, None, tn)
    eps = 64 * np.finfo(np.float64).eps
    bar_s = 2 * ((eps + dw) * mag[:, 0] + 2 * dy * mag[:, 2])
    bar_d = 2 * ((eps + dw) * mag[:, 1] + 2 * dy * mag[:, 3] + dn * mag[:, 4])
    ks = (np.abs(us - uso).max(1) / bar_s).max()
    kd = (np.abs(ud - udo).max(1) / bar_d).max()
    print(f"on-surface smooth sum: node differences y {dy:.1e} n {dn:.1e} w {dw:.1e}; largest difference / "
          f"bound: S {ks:.2e}, D {kd:.2e}; relative to the largest value: S {_rel(us, uso):.2e}, "
          f"D {_rel(ud, udo):.2e}", flush=True)
    assert ks < 1 and kd < 1


def test_sphere_config1_off_surface(ev):
    sc = synth.config1()
    ev.set_geometry(sc)
    us, ud = ev.eval(sc.sigma, sc.x, sc.tgt_node)
    _no_flags(ev)
    uso, udo = oracle.evaluate(sc)
    _check_classes(us, uso, sc.tgt_class, "S", x=sc.x)
    _check_classes(ud, udo, sc.tgt_class, "D", x=sc.x)


def test_sphere_on_surface(ev):
    sc = synth.config1(4)
    ev.set_geometry(sc)
    tn = np.arange(0, sc.n_nodes, 3)
    us, ud = ev.eval(sc.sigma, None, tn)
    _no_flags(ev)
    uso, udo = oracle.evaluate(sc, None, None, tn)
    _argmax_report(ud, udo, "D", tn)
    assert _rel(us, uso) < GATE, _rel(us, uso)
    assert _rel(ud, udo) < GATE, _rel(ud, udo)


def test_constant_density_on_unit_sphere_closed_forms(ev):
    """Degenerate band (a constant density, Ms = Mt = 0) against closed forms
    rather than the oracle: on the unit sphere S[c] = 2c/3 inside and on the
    surface (the translating sphere), and D[c] = c inside, c/2 on the surface,
    0 outside (the stresslet identity of the kernel as printed)."""
    sc = synth.config1(400)
    c = np.array([0.3, -1.1, 0.7])
    sc.sigma = np.tile(c, (sc.n_nodes, 1))
    ev.set_geometry(sc)
    us, ud = ev.eval(sc.sigma, sc.x, None)
    inside = sc.tgt_class == 0
    scale = np.abs(c).max()
    err_si = np.abs(us[inside] - 2 * c / 3).max() / scale
    err_di = np.abs(ud[inside] - c).max() / scale
    err_do = np.abs(ud[~inside]).max() / scale
    tn = np.arange(0, sc.n_nodes, 5)
    us_on, ud_on = ev.eval(sc.sigma, None, tn)
    err_son = np.abs(us_on - 2 * c / 3).max() / scale
    err_don = np.abs(ud_on - c / 2).max() / scale
    print("constant density", err_si, err_di, err_do, err_son, err_don, ev.stats().get("pairs_full"), flush=True)
    assert max(err_si, err_di, err_do, err_son, err_don) < GATE


def test_small_pipe_on_and_off_surface(ev):
    sc = synth.small_pipe_scene(n_panels=6, n_spheres=3)
    ev.set_geometry(sc)
    rng = np.random.default_rng(2)
    tn = rng.choice(sc.n_nodes, 300, replace=False)
    us, ud = ev.eval(sc.sigma, None, tn)
    _no_flags(ev)
    uso, udo = oracle.evaluate(sc, None, None, tn)
    print("on-surface", _rel(us, uso), _rel(ud, udo), ev.stats(), flush=True)
    _argmax_report(ud, udo, "D on-surface", tn)
    assert _rel(us, uso) < GATE and _rel(ud, udo) < GATE
    y, n, _ = oracle.nodes(sc)
    k = rng.choice(sc.n_nodes, 300, replace=False)
    d = 10.0 ** rng.uniform(-3, -0.3, 300) * np.where(rng.random(300) < 0.5, 1, -1)
    xs = y[k] + d[:, None] * n[k]
    us, ud = ev.eval(sc.sigma, xs, None)
    _no_flags(ev)
    uso, udo = oracle.evaluate(sc, None, xs, -np.ones(300, np.int64))
    print("off-surface", _rel(us, uso), _rel(ud, udo), ev.stats(), flush=True)
    _argmax_report(ud, udo, "D off-surface", None, xs)
    assert _rel(us, uso) < GATE and _rel(ud, udo) < GATE


def _config2_strata(sc):
    """Stratified on-surface targets of the 200-sphere pipe: sphere nodes
    nearest the poles (first and last GL circle), sphere nodes near contact
    (within 0.05 of another surface), wall nodes on the rims (first and last
    GL circle of the end panels) and the wall nodes nearest a sphere."""
    rng = np.random.default_rng(31)
    nwall = sc.bodies[0].n_panels * 512
    node = np.arange(sc.n_nodes)
    i_s = (node % 512) // 32
    sph = node >= nwall
    poles = node[sph & ((i_s == 0) | (i_s == 15))]
    lab = synth.label_near_contact(synth.config2(), dist=0.05).tgt_class
    contact = node[lab == 2]
    panel = node // 512
    rims = node[(~sph) & (((panel == 0) & (i_s == 0)) | ((panel == sc.bodies[0].n_panels - 1) & (i_s == 15)))]
    y = synth.analytic_node_positions(sc)[:nwall]
    dmin = np.full(nwall, np.inf)
    for c, r in zip(sc.sphere_centers, sc.sphere_radii):
        dmin = np.minimum(dmin, np.linalg.norm(y - c[None, :], axis=1) - r)
    wall_near = np.argsort(dmin)[:200]
    pick = [rng.choice(a, 6, replace=False) for a in (poles, contact, rims, wall_near)]
    return np.concatenate(pick)


def test_config2_full_size_sampled(ev):
    """Full config-2 evaluation (153,600 on-surface targets) in the launch
    configuration the benchmark times; 24 random targets and 24 stratified
    ones (sphere poles, near-contact sphere nodes, pipe rims, wall nodes
    nearest a sphere) against the oracle."""
    import torch
    sc = synth.config2()
    ev.set_geometry(sc)
    sig = torch.from_numpy(sc.sigma).cuda()
    tn = torch.from_numpy(sc.tgt_node).cuda()
    us, ud = ev.eval(sig, None, tn)
    torch.cuda.synchronize()
    _no_flags(ev)
    us, ud = us.cpu().numpy(), ud.cpu().numpy()
    assert np.isfinite(us).all() and np.isfinite(ud).all()
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(51200, 8, replace=False), 51200 + rng.choice(102400, 16, replace=False),
                          _config2_strata(sc)])
    uso, udo = oracle.evaluate(sc, None, None, sc.tgt_node[idx])
    _check_classes(us[idx], uso, sc.tgt_class[idx], "S", sc.tgt_node[idx])
    _check_classes(ud[idx], udo, sc.tgt_class[idx], "D", sc.tgt_node[idx])


def test_full_band_density(ev):
    """A density of nodal noise: every Fourier mode up to the Nyquist mode 16
    and every Legendre degree up to 15 on every element, on and off the
    surface, against the oracle (1e-10)."""
    sc = synth.small_pipe_scene(n_panels=6, n_spheres=3)
    sc.sigma = np.random.default_rng(41).standard_normal((sc.n_nodes, 3))
    ev.set_geometry(sc)
    rng = np.random.default_rng(42)
    tn = rng.choice(sc.n_nodes, 150, replace=False)
    us, ud = ev.eval(sc.sigma, None, tn)
    _no_flags(ev)
    st = ev.stats()
    uso, udo = oracle.evaluate(sc, None, None, tn)
    print("full band on-surface", _rel(us, uso), _rel(ud, udo), st, flush=True)
    _argmax_report(ud, udo, "D full band on-surface", tn)
    assert _rel(us, uso) < GATE and _rel(ud, udo) < GATE
    y, n, _ = oracle.nodes(sc)
    k = rng.choice(sc.n_nodes, 150, replace=False)
    d = 10.0 ** rng.uniform(-3, -0.3, 150) * np.where(rng.random(150) < 0.5, 1, -1)
    xs = y[k] + d[:, None] * n[k]
    us, ud = ev.eval(sc.sigma, xs, None)
    _no_flags(ev)
    uso, udo = oracle.evaluate(sc, None, xs, -np.ones(150, np.int64))
    print("full band off-surface", _rel(us, uso), _rel(ud, udo), flush=True)
    _argmax_report(ud, udo, "D full band off-surface", None, xs)
    assert _rel(us, uso) < GATE and _rel(ud, udo) < GATE


def test_free_targets_very_near_surface(ev):
    """Free targets 1e-6 and 1e-7 off the surface, inside and outside, above
    random (off-node) points of the pipe panels and the spheres, against the
    oracle (which forms such pairs in long double): 1e-10."""
    sc = synth.small_pipe_scene(n_panels=6, n_spheres=3)
    ev.set_geometry(sc)
    rng = np.random.default_rng(43)
    xs = []
    for e in range(sc.n_panels):
        b, p = (0, e) if e < 6 else (e - 5, 0)
        sb = sc.bodies[b].s_break
        s = rng.uniform(sb[p] + 0.05 * (sb[p + 1] - sb[p]), sb[p + 1] - 0.05 * (sb[p + 1] - sb[p]), 4)
        t = rng.uniform(0, 2 * np.pi, 4)
        yp, npt, _, _ = oracle.surface_point(sc, e, s, t)
        d = np.array([1e-6, -1e-6, 1e-7, -1e-7])
        xs.append(yp + d[:, None] * npt)
    xs = np.concatenate(xs)
    us, ud = ev.eval(sc.sigma, xs, None)
    _no_flags(ev)
    uso, udo = oracle.evaluate(sc, None, xs, -np.ones(len(xs), np.int64))
    print("very near", _rel(us, uso), _rel(ud, udo), ev.stats(), flush=True)
    _argmax_report(ud, udo, "D very near", None, xs)
    assert _rel(us, uso) < GATE and _rel(ud, udo) < GATE


def test_out_of_range_device_node_raises(ev):
    """A device-resident tgt_node beyond the node count fails the call with
    CsbqError (checked on the device before the call's first wait), and the
    context stays usable."""
    import torch
    import paper_2310_00889_amd as pk
    sc = synth.small_pipe_scene(n_panels=2, n_spheres=1)
    ev.set_geometry(sc)
    sig = torch.from_numpy(sc.sigma).cuda()
    bad = torch.tensor([0, sc.n_nodes + 3, 5], dtype=torch.int64, device="cuda")
    with pytest.raises(pk.CsbqError, match="out of range"):
        ev.eval(sig, None, bad)
    assert ev.flags() & pk.FLAG_NODE_RANGE
    good = torch.tensor([0, 7, 5], dtype=torch.int64, device="cuda")
    us, ud = ev.eval(sig, None, good)
    torch.cuda.synchronize()
    _no_flags(ev)
    assert torch.isfinite(us).all() and torch.isfinite(ud).all()


def test_determinism_and_device_host_agree(ev):
    import torch
    sc = synth.small_pipe_scene(n_panels=4, n_spheres=2)
    ev.set_geometry(sc)
    tn = np.arange(0, sc.n_nodes, 5)
    a1, b1 = ev.eval(sc.sigma, None, tn)
    a2, b2 = ev.eval(sc.sigma, None, tn)
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)
    ad, bd = ev.eval(torch.from_numpy(sc.sigma).cuda(), None, torch.from_numpy(tn).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(ad.cpu().numpy(), a1) and np.array_equal(bd.cpu().numpy(), b1)


def test_empty_and_invalid_inputs(ev):
    import paper_2310_00889_amd as pk
    sc = synth.small_pipe_scene(n_panels=2, n_spheres=1)
    ev.set_geometry(sc)
    us, ud = ev.eval(sc.sigma, np.zeros((0, 3)), None)
    assert us.shape == (0, 3)
    bad = sc.sigma.copy()
    bad[5, 1] = np.nan
    with pytest.raises(pk.CsbqError):
        ev.eval(bad, np.ones((2, 3)), None)
    with pytest.raises(pk.CsbqError):
        ev.eval(sc.sigma, None, np.array([sc.n_nodes + 3]))
    # the context stays usable after an error
    us, ud = ev.eval(sc.sigma, None, np.array([0, 1]))
    assert np.isfinite(us).all()


def test_asymmetric_theta_rule_table_is_refused(tmp_path):
    """The special quadrature evaluates every theta-rule in mirror pairs, so a
    table whose rule is not symmetric must be refused when a context loads it
    (here one node of the first rule moved)."""
    import struct
    import paper_2310_00889_amd as pk
    raw = bytearray(open(os.path.join(pk.TABLE_DIR, "rules.bin"), "rb").read())
    m = struct.unpack_from("<i", raw, 28)[0]            # header: magic, version, NB, l0, tol
    th0 = struct.unpack_from("<d", raw, 32)[0]
    struct.pack_into("<d", raw, 32, th0 * (1 + 1e-9))
    assert m > 0
    (tmp_path / "rules.bin").write_bytes(bytes(raw))
    with pytest.raises(pk.CsbqError, match="ETABLE"):
        pk.Evaluator(table_dir=str(tmp_path))


MIXED_GATE = 1e-6


@pytest.fixture(scope="module")
def ev_mixed():
    import torch
    import paper_2310_00889_amd as pk
    torch.zeros(1, device="cuda")
    e = pk.Evaluator(quad_tol=1e-7, precision="mixed")
    yield e
    e.close()


def test_mixed_small_pipe(ev_mixed):
    """Mixed precision (FP32 far field, FP64 near corrections) at quad_tol 1e-7:
    every output within 1e-6 of the FP64 oracle, on and off the surface."""
    sc = synth.small_pipe_scene(n_panels=6, n_spheres=3)
    ev_mixed.set_geometry(sc)
    rng = np.random.default_rng(4)
    tn = rng.choice(sc.n_nodes, 200, replace=False)
    us, ud = ev_mixed.eval(sc.sigma, None, tn)
    _no_flags(ev_mixed)
    uso, udo = oracle.evaluate(sc, None, None, tn)
    print("mixed on-surface", _rel(us, uso), _rel(ud, udo), flush=True)
    assert _rel(us, uso) < MIXED_GATE and _rel(ud, udo) < MIXED_GATE
    y, n, _ = oracle.nodes(sc)
    k = rng.choice(sc.n_nodes, 200, replace=False)
    d = 10.0 ** rng.uniform(-3, -0.3, 200) * np.where(rng.random(200) < 0.5, 1, -1)
    xs = y[k] + d[:, None] * n[k]
    us, ud = ev_mixed.eval(sc.sigma, xs, None)
    _no_flags(ev_mixed)
    uso, udo = oracle.evaluate(sc, None, xs, -np.ones(200, np.int64))
    print("mixed off-surface", _rel(us, uso), _rel(ud, udo), flush=True)
    assert _rel(us, uso) < MIXED_GATE and _rel(ud, udo) < MIXED_GATE


def test_mixed_config3_full_size_sampled(ev_mixed):
    """Config 3 (1000 spheres in the scaled pipe, 563,200 on-surface targets) in
    mixed precision, full size; 12 sampled targets per class (wall, particle,
    near-contact particle) against the oracle, 1e-6 per class."""
    import torch
    sc = synth.config3()
    ev_mixed.set_geometry(sc)
    sig = torch.from_numpy(sc.sigma).cuda()
    tn = torch.from_numpy(sc.tgt_node).cuda()
    us, ud = ev_mixed.eval(sig, None, tn)
    torch.cuda.synchronize()
    _no_flags(ev_mixed)
    us, ud = us.cpu().numpy(), ud.cpu().numpy()
    assert np.isfinite(us).all() and np.isfinite(ud).all()
    print("config3 mixed stats", ev_mixed.stats(), flush=True)
    rng = np.random.default_rng(6)
    idx = np.concatenate([rng.choice(np.where(sc.tgt_class == c)[0], 12, replace=False) for c in (0, 1, 2)])
    uso, udo = oracle.evaluate(sc, None, None, sc.tgt_node[idx])
    for u, uo, what in ((us[idx], uso, "S"), (ud[idx], udo, "D")):
        for c in (0, 1, 2):
            m = sc.tgt_class[idx] == c
            err = np.abs(u[m] - uo[m]).max() / np.abs(uo[m]).max()
            print(f"mixed {what} class {c}: {err:.2e}", flush=True)
            assert err < MIXED_GATE, (what, c, err)


def test_criterion_never_below_method_labels(ev):
    """The error-estimate criterion against the method itself: on the
    200-sphere pipe (every 8th node as a target, 1.5M candidate pairs) every
    pair's tier is at least its label, the cheapest tier whose correction
    agrees with the special quadrature to 1e-13 of the largest |u|."""
    sc = synth.config2()
    ev.set_geometry(sc)
    tn = sc.tgt_node[::8].copy()
    f, lab, crit = ev.gate_dataset(sc.sigma, None, tn, label_tol=1e-13, cap=3_000_000)
    print("labels", np.bincount(lab, minlength=5), "criterion", np.bincount(crit, minlength=5), flush=True)
    assert len(lab) > 1_000_000
    assert int(np.sum(lab > crit)) == 0
