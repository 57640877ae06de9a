"""Coarser far-field rules of the smooth sum: for a block of targets, each
element is summed with the coarsest tensor rule whose distances, by the
criterion's estimates, let it meet quad_tol beyond them (a sphere: 24, 20
or its own 16 Gauss-Legendre points in s; a wall panel: 16, 12 or 8; times
32, 24 or 16 angles), else with its base rule (Section 3.2.1's smooth rule,
with the error estimates of Section 3.3).  Checked against the oracle and
against the same evaluation with the base rules everywhere
(far_rule="base")."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GATE = 1e-10


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _lattice_scene(seed=11, n=3, spacing=2.5, radius=0.3):
    """n^3 spheres on a cubic lattice, randomly oriented, each carrying a
    constant density vector (Legendre and Fourier bands 0: at quad_tol 1e-12
    the 24-, 20- and 16-point rules in s suffice from about 5, 6 and 10
    radii, 16 angles from about 5)."""
    rng = np.random.default_rng(seed)
    bodies, sig = [], []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                q, r = np.linalg.qr(rng.standard_normal((3, 3)))
                q = q * np.sign(np.diag(r))[None, :]
                c = spacing * np.array([i, j, k], float) + 0.1 * rng.standard_normal(3)
                bodies.append(synth.sphere_body(c, radius, q[:, 0], q[:, 1]))
                sig.append(np.tile(rng.standard_normal(3), (synth.NS * synth.NT, 1)))
    sigma = np.concatenate(sig)
    nn = sigma.shape[0]
    return synth.Scene(bodies, synth.NS, synth.NT, sigma, np.zeros((nn, 3)), np.arange(nn, dtype=np.int64),
                       np.zeros(nn, np.int32), ("particle",), "sphere-lattice")


@pytest.fixture(scope="module")
def evs():
    import torch
    import paper_2310_00889_amd as pk
    torch.zeros(1, device="cuda")
    a = pk.Evaluator(quad_tol=1e-12)
    b = pk.Evaluator(quad_tol=1e-12, far_rule="base")
    yield a, b
    a.close()
    b.close()


def test_far_rule_option_reported(evs):
    ev, base = evs
    sc = _lattice_scene(n=2)
    for e in (ev, base):
        e.set_geometry(sc)
        e.eval(sc.sigma, None, sc.tgt_node[:64])
    assert ev.stats()["far_split"] == 1 and base.stats()["far_split"] == 0


def test_coarser_rules_on_separated_spheres_fp64(evs):
    """27 spheres, constant densities, quad_tol 1e-12: coarser rules replace
    the 32 x 32 rule for far blocks (fewer pairs summed), every output stays
    within 1e-10 of the oracle on and off the surfaces (off them the double
    layer vanishes), and within 1e-11 of the evaluation with the 32 x 32 rule
    everywhere."""
    ev, base = evs
    sc = _lattice_scene()
    ev.set_geometry(sc)
    base.set_geometry(sc)
    tn = sc.tgt_node
    us, ud = ev.eval(sc.sigma, None, tn)
    st = ev.stats()
    ub, db = base.eval(sc.sigma, None, tn)
    sb = base.stats()
    print("far pairs", st["far_pairs"], "of", st["far_pairs_base"], "; base", sb["far_pairs"], flush=True)
    assert st["far_pairs_base"] == sb["far_pairs"] == sb["far_pairs_base"]
    assert st["far_pairs"] < 0.9 * st["far_pairs_base"]
    assert ev.flags() == 0
    print("coarser rules vs 32 x 32 rule:", _rel(us, ub), _rel(ud, db), flush=True)
    assert _rel(us, ub) < 1e-11 and _rel(ud, db) < 1e-11
    rng = np.random.default_rng(3)
    k = rng.choice(sc.n_nodes, 80, replace=False)
    uso, udo = oracle.evaluate(sc, None, None, tn[k])
    print("on-surface vs oracle:", _rel(us[k], uso), _rel(ud[k], udo), flush=True)
    assert _rel(us[k], uso) < GATE and _rel(ud[k], udo) < GATE
    # free targets between the spheres (lattice cell centres) and near them
    y, n, _ = oracle.nodes(sc)
    c = 2.5 * (rng.integers(0, 2, (20, 3)) + 0.5)
    j = rng.choice(sc.n_nodes, 20, replace=False)
    x = np.concatenate([c, y[j] + 10.0 ** rng.uniform(-3, -1, 20)[:, None] * n[j]])
    uf, df = ev.eval(sc.sigma, x, None)
    assert ev.flags() == 0
    ufo, dfo = oracle.evaluate(sc, None, x, -np.ones(len(x), np.int64))
    # the double layer of a constant density vanishes outside its closed
    # surface: judge it against the density scale (both sides are ~1e-15)
    smax = np.abs(sc.sigma).max()
    print("free targets vs oracle:", _rel(uf, ufo), np.abs(df - dfo).max() / smax, "|u_D|", np.abs(df).max(),
          flush=True)
    assert _rel(uf, ufo) < GATE and np.abs(df - dfo).max() < GATE * smax and np.abs(df).max() < GATE * smax


def test_coarser_rules_on_a_pipe_wall_fp64(evs):
    """A 60-panel torus-arc pipe with a constant density (bands 0), FP64
    quad_tol 1e-12: the wall panels' coarser rules (12 or 8 points in s, 24 or
    16 angles) replace their own nodes far from the targets; every node within
    1e-11 of the evaluation with the base rules, 60 on-surface and 20 interior
    targets within 1e-10 of the oracle."""
    ev, base = evs
    b = synth.pipe_body(n_panels=60)
    nn = b.n_panels * synth.NS * synth.NT
    rng = np.random.default_rng(21)
    sigma = np.tile(rng.standard_normal(3), (nn, 1))
    sc = synth.Scene([b], synth.NS, synth.NT, sigma, np.zeros((nn, 3)), np.arange(nn, dtype=np.int64),
                     np.zeros(nn, np.int32), ("wall",), "pipe60")
    ev.set_geometry(sc)
    base.set_geometry(sc)
    us, ud = ev.eval(sc.sigma, None, sc.tgt_node)
    st = ev.stats()
    ub, db = base.eval(sc.sigma, None, sc.tgt_node)
    print("far pairs", st["far_pairs"], "of", st["far_pairs_base"], flush=True)
    assert st["far_pairs"] < 0.8 * st["far_pairs_base"]
    assert ev.flags() == 0
    print("coarser rules vs base rules:", _rel(us, ub), _rel(ud, db), flush=True)
    assert _rel(us, ub) < 1e-11 and _rel(ud, db) < 1e-11
    k = rng.choice(nn, 60, replace=False)
    uso, udo = oracle.evaluate(sc, None, None, sc.tgt_node[k])
    print("on-surface vs oracle:", _rel(us[k], uso), _rel(ud[k], udo), flush=True)
    assert _rel(us[k], uso) < GATE and _rel(ud[k], udo) < GATE
    phi = rng.uniform(0.05, np.pi - 0.05, 20)
    off = rng.uniform(-0.6, 0.6, (20, 2))
    x = np.stack([(5.0 + off[:, 0]) * np.cos(phi), (5.0 + off[:, 0]) * np.sin(phi), off[:, 1]], axis=1)
    uf, df = ev.eval(sc.sigma, x, None)
    assert ev.flags() == 0
    ufo, dfo = oracle.evaluate(sc, None, x, -np.ones(len(x), np.int64))
    print("interior targets vs oracle:", _rel(uf, ufo), _rel(df, dfo), flush=True)
    assert _rel(uf, ufo) < GATE and _rel(df, dfo) < GATE


def test_coarser_rules_under_a_plan(evs):
    """A frozen plan replays the rule choice of its evaluation: apply()
    with a density of the same band equals a fresh evaluation bit for bit
    (8 spheres 5 apart: small enough that both contexts keep the default
    smooth-sum shape, far enough apart for the coarser rules)."""
    ev, _ = evs
    import paper_2310_00889_amd as pk
    sc = _lattice_scene(seed=12, n=2, spacing=5.0)
    ev.set_geometry(sc)
    tn = sc.tgt_node
    ev.plan(sc.sigma, None, tn)
    sig2 = -0.75 * sc.sigma[:, [2, 0, 1]]
    us, ud = ev.apply(sig2)
    ref = pk.Evaluator(quad_tol=1e-12)
    try:
        ref.set_geometry(sc)
        ur, dr = ref.eval(sig2, None, tn)
        st = ref.stats()
        assert st["far_pairs"] < st["far_pairs_base"]
    finally:
        ref.close()
    assert np.array_equal(us, ur) and np.array_equal(ud, dr)


def test_coarser_rules_config3_fp64_at_1e7():
    """The 1000-sphere pipe (563,200 on-surface targets) in FP64 at quad_tol
    1e-7: coarser rules take over most sphere pairs of the smooth sum; the
    result stays within 1e-6 of the evaluation with the 32 x 32 rule and, on
    12 sampled targets per class, of the oracle."""
    import torch
    import paper_2310_00889_amd as pk
    sc = synth.config3()
    sig = torch.from_numpy(sc.sigma).cuda()
    tn = torch.from_numpy(sc.tgt_node).cuda()
    out = {}
    for rule in ("auto", "base"):
        ev = pk.Evaluator(quad_tol=1e-7, far_rule=rule)
        try:
            ev.set_geometry(sc)
            us, ud = ev.eval(sig, None, tn)
            torch.cuda.synchronize()
            assert ev.flags() == 0
            st = ev.stats()
            print(rule, "far pairs", st["far_pairs"], "of", st["far_pairs_base"], "ms", st["ms"], flush=True)
            out[rule] = (us.cpu().numpy(), ud.cpu().numpy(), st)
        finally:
            ev.close()
    us, ud, st = out["auto"]
    ub, db, _ = out["base"]
    assert st["far_pairs"] < 0.8 * st["far_pairs_base"]
    print("coarser rules vs 32 x 32 rule:", _rel(us, ub), _rel(ud, db), flush=True)
    assert _rel(us, ub) < 1e-6 and _rel(ud, db) < 1e-6
    rng = np.random.default_rng(8)
    idx = np.concatenate([rng.choice(np.where(sc.tgt_class == c)[0], 12, replace=False) for c in (0, 1, 2)])
    uso, udo = oracle.evaluate(sc, None, None, sc.tgt_node[idx])
    for u, uo, what in ((us[idx], uso, "S"), (ud[idx], udo, "D")):
        for c in (0, 1, 2):
            m = sc.tgt_class[idx] == c
            err = np.abs(u[m] - uo[m]).max() / np.abs(uo[m]).max()
            print(f"FP64 1e-7 {what} class {c}: {err:.2e}", flush=True)
            assert err < 1e-6, (what, c, err)
