"""The correction-matrix form of the special quadrature (Section 3.2.1: the
corrected Nystrom rule's matrix E, built once in a setup and applied per
density; Section 3.4's setup/evaluation split), through the C ABI:
csbq_plan_ex with CSBQ_PLAN_MATRIX, then csbq_apply of other densities,
against the density route of the same plan (rounding only) and the CPU
oracle (1e-10)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GATE = 1e-10


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def evs():
    import torch
    import paper_2310_00889_amd as pk
    torch.zeros(1, device="cuda")
    a = pk.Evaluator(quad_tol=1e-12)
    b = pk.Evaluator(quad_tol=1e-12)
    yield a, b
    a.close()
    b.close()


def _targets(sc, rng, n):
    y, nrm, _ = oracle.nodes(sc)
    tn = np.concatenate([rng.choice(sc.n_nodes, n, replace=False), -np.ones(n, np.int64)]).astype(np.int64)
    k = rng.choice(sc.n_nodes, n, replace=False)
    d = 10.0 ** rng.uniform(-3, -0.3, n) * np.where(rng.random(n) < 0.5, 1, -1)
    x = np.concatenate([np.zeros((n, 3)), y[k] + d[:, None] * nrm[k]])
    return tn, x


@pytest.mark.parametrize("full_band", [False, True])
def test_matrix_apply_matches_density_route_and_oracle(evs, full_band):
    em, ed = evs
    sc = synth.small_pipe_scene(n_panels=6, n_spheres=3)
    rng = np.random.default_rng(21)
    tn, x = _targets(sc, rng, 120)
    for ev in evs:
        ev.set_geometry(sc)
    em.plan(sc.sigma, x, tn, matrix=True, full_band=full_band)
    ed.plan(sc.sigma, x, tn, matrix=False, full_band=full_band)
    st = em.stats()
    print("matrix plan", st["plan"], st["pairs_full"], flush=True)
    assert st["plan"]["matrix"] and st["plan"]["matrix_bytes"] == st["pairs_full"] * 12 * 512 * 8
    # a second density of the same band (full band: nodal noise)
    # (band-limited plan: components of the planning density mixed, which keeps
    # every element's band limits)
    sig2 = rng.standard_normal((sc.n_nodes, 3)) if full_band else 0.3 * sc.sigma + np.roll(sc.sigma, 1, axis=1)
    us_m, ud_m = em.apply(sig2)
    us_d, ud_d = ed.apply(sig2)
    uso, udo = oracle.evaluate(sc, sig2, x, tn)
    eo_s, eo_d = _rel(us_m, uso), _rel(ud_m, udo)
    print("matrix vs oracle", full_band, eo_s, eo_d, flush=True)
    assert eo_s < GATE and eo_d < GATE
    # the same terms summed in another order: near a surface the special rule
    # and the subtracted far-field rule cancel to ~1e-3 of their terms, so the
    # two routes agree to ~1e-13 .. 1e-12 of the result
    es, edd = _rel(us_m, us_d), _rel(ud_m, ud_d)
    print("matrix vs density route", full_band, es, edd, flush=True)
    assert es < 1e-11 and edd < 1e-11
    us_2, ud_2 = em.apply(sig2)
    assert np.array_equal(us_2, us_m) and np.array_equal(ud_2, ud_m)
