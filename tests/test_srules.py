"""The whole-element singular s-rules (Section 3.2.4, second part; built per
Appendix B by tables/gen_srules.py), checked on the CPU against integrals
computed independently of the generator:
* cylinder rules: the element integral of the mode-l modal Green's function
  of 1/R on a straight cylinder, times P_0 or P_1, with the integral over
  the element done in closed form (asinh and square roots) and the integral
  over the angle by scipy's adaptive quadrature;
* sphere rules: single layers of the spherical harmonics of degree 0 and 1
  (4 pi a Y_l / (2l + 1) on the surface) and the double layer of a constant
  (half the solid angle, 2 pi), with the angular integrals by scipy's
  adaptive quadrature on the interpolated sphere."""
import math
import os
import sys

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss
from scipy.integrate import quad

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2310_00889_amd", "tables"))
import gen_srules  # noqa: E402

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
TDIR = os.path.join(ROOT, "paper_2310_00889_amd", "tables")
# the rules built to 1e-12 (srules.bin) and to 1e-8 (srules_t8.bin, loaded by
# contexts with quad_tol >= 1e-8); each is held to its own bar
TABLES = {name: gen_srules.read_srules(os.path.join(TDIR, name)) for name in ("srules.bin", "srules_t8.bin")}
TAB = TABLES["srules.bin"]


def _bar(tab):
    return max(1e-12, 10 * tab["tol"])
XG = leggauss(16)[0]


@pytest.mark.parametrize("name", sorted(TABLES))
def test_header_and_node_sets(name):
    tab = TABLES[name]
    assert tab["ns"] == 16 and tab["b_lo"] == 2 and tab["b_lo"] + tab["nb"] - 1 == 30
    assert tab["l0"] >= 16 and tab["np"] >= 16
    assert tab["sphere"] is not None and len(tab["sphere"]) == 16
    for (b, i), (d, w) in list(tab["rules"].items()) + [((1, i), r) for i, r in tab["sphere"].items()]:
        assert 32 <= len(d) <= 160
        x = XG[i] + d
        assert np.all(np.diff(d) > 0) and np.all(d != 0) and np.all((x > -1) & (x < 1))
        # nodes on both sides of the target, crowding toward it on the
        # bracket's scale 1/beta
        assert d.min() < 0 < d.max() or i in (0, 15)
        assert np.abs(d).min() < 1.0 / 2.0 ** b
        # weights of both signs are allowed (Appendix B gives no positivity);
        # their magnitudes sum to at most ~12 (2 for a positive rule), which
        # bounds the rounding amplification
        assert np.all(np.isfinite(w)) and np.abs(w).sum() < 16.0


def _mode_1r(dz, l):
    """int_0^{2 pi} cos(l t) / sqrt(2 - 2 cos t + dz^2) dt (adaptive, split at
    the peak's width)."""
    f = lambda t: math.cos(l * t) / math.sqrt(4 * math.sin(0.5 * t) ** 2 + dz * dz)
    c = min(abs(dz), 1.0)
    return 2 * (quad(f, 0, c, epsabs=0, epsrel=2e-14, limit=200)[0] +
                quad(f, c, math.pi, epsabs=0, epsrel=2e-14, limit=400)[0])


def _element_integral(A, xi, l, p):
    """int_{-1}^{1} P_p(v) G_l(A (xi - v) / 2) dv for p = 0, 1, by exchanging
    the order: closed form in v, adaptive quadrature in the angle (the
    inner integral grows like log(1/t) at t = 0, handled by splitting)."""
    k = 0.5 * A
    u1, u2 = 1.0 - xi, 1.0 + xi

    def inner(t):
        a = 2.0 * math.sin(0.5 * t)
        i0 = (math.asinh(k * u1 / a) + math.asinh(k * u2 / a)) / k
        if p == 0:
            return math.cos(l * t) * i0
        i1 = (math.sqrt(a * a + k * k * u1 * u1) - math.sqrt(a * a + k * k * u2 * u2)) / (k * k)
        return math.cos(l * t) * (xi * i0 + i1)

    pts = [min(1e-12 * 10 ** j, 0.5) for j in range(0, 12, 2)]
    br = [0.0] + sorted(set(pts)) + [math.pi]
    return 2 * sum(quad(inner, a, b, epsabs=0, epsrel=2e-14, limit=400)[0] for a, b in zip(br[:-1], br[1:]))


CASES = [(2, 7, 0.37), (5, 0, 0.81), (9, 15, 0.05), (13, 4, 0.5), (20, 11, 0.93), (30, 8, 0.21)]


@pytest.mark.parametrize("name,b,i,frac", [(n,) + c for n in sorted(TABLES) for c in CASES])
def test_rule_integrates_modal_greens_function(name, b, i, frac):
    """Error relative to the mode-0 integral of |P_p| / R (the family's
    scale): at most 1e-12 (the 1e-8 table: 1e-7) for modes 0, 3 and 16,
    polynomials P_0 and P_1, at an aspect inside the bracket that the
    generator did not sample."""
    tab = TABLES[name]
    bar = _bar(tab)
    d, w = tab["rules"][(b, i)]
    A = 2.0 ** b * (1.0 + frac)
    xi = XG[i]
    scale = _element_integral(A, xi, 0, 0)
    for l in (0, 3, 16):
        g = np.array([_mode_1r(-0.5 * A * dm, l) for dm in d])
        for p in (0, 1):
            got = np.sum(w * g * ((xi + d) if p else 1.0))
            ref = _element_integral(A, xi, l, p)
            assert abs(got - ref) < bar * scale, (b, i, l, p, got, ref, scale)


def _sphere_geometry(v):
    """The unit sphere element as both evaluators see it: the degree-15
    interpolants of sin(pi t), cos(pi t) at the 16 GL nodes, t = (v + 1)/2:
    E, z and their v-derivatives."""
    from numpy.polynomial import legendre as L
    t = 0.5 * np.pi * (XG + 1.0)
    cE, cz = L.legfit(XG, np.sin(t), 15), L.legfit(XG, np.cos(t), 15)
    return (L.legval(v, cE), L.legval(v, cz), L.legval(v, L.legder(cE)), L.legval(v, L.legder(cz)))


def _differences(i, v):
    """E0 - E and z0 - z at v from the samples' differences to the i-th node's
    (p(v) - p(x_i) = sum_j (p_j - p_i) l_j(v), the Lagrange basis from the
    offsets v - x_j): they keep their relative accuracy next to the target,
    where the double layer's r.n is a difference of second order."""
    t = 0.5 * np.pi * (XG + 1.0)
    lam = np.array([1.0 / np.prod([XG[j] - XG[k] for k in range(16) if k != j]) for j in range(16)])
    dv = (v - XG[i]) - (XG - XG[i])
    q = lam / dv
    q /= q.sum()
    return -np.dot(q, np.sin(t) - np.sin(t[i])), -np.dot(q, np.cos(t) - np.cos(t[i]))


def _sphere_angle_integral(v, i, kind):
    """Integral over the circle at v of J / R (kind "S") or J (r.n) / R^3
    (kind "D"), target at the i-th GL node, angle 0."""
    E0, _, _, _ = _sphere_geometry(XG[i])
    dE, Z = _differences(i, v)
    E = E0 - dE
    _, _, Ep, zp = _sphere_geometry(v)
    sp = math.hypot(Ep, zp)

    def f(t):
        h2 = 2.0 * math.sin(0.5 * t) ** 2
        X = dE + E * h2
        Y = -E * math.sin(t)
        R2 = X * X + Y * Y + Z * Z
        if kind == "S":
            return E * sp / math.sqrt(R2)
        rn = (zp * (dE - E0 * h2) - Z * Ep) / sp
        return E * sp * rn / R2 ** 1.5
    c = min(1.0, math.hypot(dE, Z) / E)
    return 2 * (quad(f, 0, c, epsabs=0, epsrel=2e-14, limit=200)[0] +
                quad(f, c, math.pi, epsabs=0, epsrel=2e-14, limit=200)[0])


@pytest.mark.parametrize("name,i", [(n, i) for n in sorted(TABLES) for i in (0, 3, 7, 12, 15)])
def test_sphere_rule_closed_forms(name, i):
    """On the unit sphere, for the target at the i-th GL node: the single
    layer of 1 is 4 pi, that of cos(polar angle) is (4 pi / 3) cos(polar
    angle at the target), the double layer of 1 has magnitude 2 pi.  The
    interpolated sphere departs from the sphere by ~1e-11, hence the 1e-9
    (the 1e-8 table: 1e-7)."""
    tab = TABLES[name]
    bar = max(1e-9, _bar(tab))
    d, w = tab["sphere"][i]
    v = XG[i] + d
    gS = np.array([_sphere_angle_integral(x, i, "S") for x in v])
    gD = np.array([_sphere_angle_integral(x, i, "D") for x in v])
    assert abs(np.sum(w * gS) - 4 * np.pi) < bar * 4 * np.pi
    t0 = 0.5 * np.pi * (XG[i] + 1.0)
    ct = np.cos(0.5 * np.pi * (v + 1.0))
    assert abs(np.sum(w * gS * ct) - 4 * np.pi / 3 * math.cos(t0)) < bar * 4 * np.pi
    assert abs(abs(np.sum(w * gD)) - 2 * np.pi) < bar * 2 * np.pi
