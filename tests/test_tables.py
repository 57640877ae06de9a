"""The precomputed quadrature tables (theta-rules per distance bracket and the
log-singular rule), checked against independent references on the CPU."""
import os
import sys

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2310_00889_amd", "tables"))
import gen_rules  # noqa: E402

TDIR = os.path.join(ROOT, "paper_2310_00889_amd", "tables")
TAB = gen_rules.read_tables(os.path.join(TDIR, "rules.bin"))
# the tables built to 1e-13 (rules.bin) and to 1e-8 (rules_t8.bin, loaded by
# contexts with quad_tol >= 1e-8)
TABLES = {"rules.bin": TAB, "rules_t8.bin": gen_rules.read_tables(os.path.join(TDIR, "rules_t8.bin"))}


@pytest.mark.parametrize("name", sorted(TABLES))
def test_table_header_and_sizes(name):
    tab = TABLES[name]
    assert tab["l0"] == 20 and len(tab["rules"]) == 40
    for th, om in tab["rules"]:
        assert 40 <= len(th) <= 256 and np.all(np.abs(th) <= np.pi)
        assert np.allclose(th, -th[::-1]) and np.allclose(om, om[::-1])   # mirrored rule


@pytest.mark.parametrize("name", sorted(TABLES))
def test_theta_rules_are_mirror_symmetric(name):
    """The special quadrature evaluates each theta-rule in pairs (phi, -phi)
    sharing one weight, and the library refuses a table where that fails."""
    for th, w in TABLES[name]["rules"]:
        m = len(th)
        assert m % 2 == 0
        assert np.array_equal(th[: m // 2], -th[::-1][: m // 2]) and np.all(th[m // 2:] > 0)
        assert np.array_equal(w[: m // 2], w[::-1][: m // 2])


def test_log_rule_moments():
    x, w = TAB["log_rule"]
    assert x.min() > 1e-7 and x.max() < 1
    for k in range(16):
        assert abs(np.dot(w, x ** k) - 1 / (k + 1)) < 1e-14
        assert abs(np.dot(w, x ** k * np.log(x)) + 1 / (k + 1) ** 2) < 1e-14


def _ring_potential_reference(d, z, l, comp):
    """Composite GL on [-pi, pi] with panels refined toward t = 0 (independent
    of the rule's own discretisation: different panels and order)."""
    a = max(np.hypot(d, z), 1e-14)
    br = [0.0]
    h = a / 16
    while h < np.pi:
        br.append(h)
        h *= 1.5
    br.append(np.pi)
    br = np.array(br)
    xg, wg = leggauss(50)
    xs = (0.5 * (br[1:] + br[:-1])[:, None] + 0.5 * (br[1:] - br[:-1])[:, None] * xg).ravel()
    ws = (0.5 * (br[1:] - br[:-1])[:, None] * wg).ravel()
    xs = np.concatenate([-xs[::-1], xs])
    ws = np.concatenate([ws[::-1], ws])
    ev, od = gen_rules._components(xs, d, z)
    f = (ev + od)[comp]
    return np.sum(ws * f * np.cos(l * xs)), np.sum(ws * np.abs(f))


@pytest.mark.parametrize("name,b", [(n, b) for n in sorted(TABLES) for b in (1, 2, 5, 9, 14, 20, 27, 33)])
def test_theta_rule_integrates_kernel_modes(name, b):
    """Each rule integrates the kernel components times modes to ten times its
    construction tolerance (1e-13), relative to the integral of |f|."""
    th, om = TABLES[name]["rules"][b - 1]
    bar = 10 * TABLES[name]["tol"]
    rng = np.random.default_rng(b)
    alpha = 2.0 ** (-b)
    worst = 0.0
    for _ in range(12):
        r = alpha * (1 + rng.random())
        phi = 2 * np.pi * rng.random()
        d, z = r * np.cos(phi), r * np.sin(phi)
        for comp in rng.choice(17, 4, replace=False):
            l = int(rng.integers(0, 21))
            ref, scale = _ring_potential_reference(d, z, l, comp)
            ev, od = gen_rules._components(th, d, z)
            got = np.sum(om * (ev + od)[comp] * np.cos(l * th))
            worst = max(worst, abs(got - ref) / scale)
    assert worst < bar, worst
