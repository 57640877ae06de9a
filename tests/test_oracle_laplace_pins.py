"""Pins of the oracle's Laplace layer potentials (Section 4.1: G(r) =
1/(4 pi |r|), double layer dG/dn_y = (r.n)/(4 pi |r|^3), r = x - y, n the
outward normal) against closed forms:

* Gauss's law: D[1] = -1 inside a closed surface, -1/2 on it, 0 outside;
* the single layer of a constant on a sphere of radius a: a inside and on,
  a^2/|x| outside;
* the single layer of a spherical harmonic of degree l on the unit sphere:
  Y_l r^l/(2l+1) inside, Y_l/(2l+1) on, Y_l/((2l+1) r^(l+1)) outside;
* Green's representation of a harmonic function (the paper's validation,
  Section 5.1, Eq. e:greens-rep: torus R = 1, eps = 0.25, unit charge at
  (1, 2, 3)): S[du/dn] - D[u] = u inside, u/2 on, 0 outside;
at distances down to 1e-7 from the surface; every adaptive cell must meet
its tolerance before the depth cap.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _ev(sc, sig, x=None, tgt_node=None):
    if x is not None and tgt_node is None:
        tgt_node = -np.ones(len(x), np.int64)
    us, ud, deep = oracle.evaluate_laplace(sc, sig, x, tgt_node, return_deep=True)
    assert deep == 0, f"{deep} adaptive cells accepted at the depth cap"
    return us, ud


def _dirs(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("d", (1e-1, 1e-3, 1e-5, 1e-7))
def test_gauss_law_and_constant_single_layer_on_sphere(d):
    a = 0.7
    sc = synth.Scene([synth.sphere_body([0.2, -0.1, 0.3], a, [0.0, 0.6, 0.8], [1.0, 0.0, 0.0])])
    c0 = np.array([0.2, -0.1, 0.3])
    rng = np.random.default_rng(int(-math.log10(d)))
    v = _dirs(rng, 4)
    xin, xout = c0 + v * a * (1 - d), c0 + v * a * (1 + d)
    one = np.ones(sc.n_nodes)
    sin_, din = _ev(sc, one, xin)
    sout, dout = _ev(sc, one, xout)
    assert np.abs(din + 1).max() < 1e-12
    assert np.abs(dout).max() < 1e-12
    assert np.abs(sin_ - a).max() < 1e-12 * a
    assert np.abs(sout - a * a / np.linalg.norm(xout - c0, axis=1)).max() < 1e-12 * a
    nodes = rng.choice(sc.n_nodes, 5, replace=False)
    son, don = _ev(sc, one, None, nodes)
    assert np.abs(don + 0.5).max() < 1e-12
    assert np.abs(son - a).max() < 1e-12 * a


def _y_l(l, v):
    """A real spherical harmonic of degree l: the zonal Legendre P_l about an
    oblique axis (unnormalised)."""
    from numpy.polynomial import legendre as npleg
    ax = np.array([0.36, 0.48, 0.8])
    return npleg.legval(v @ ax, np.eye(l + 1)[l])


@pytest.mark.parametrize("l,bar", ((1, 1e-12), (2, 1e-11)))
def test_single_layer_of_spherical_harmonics(l, bar):
    """(The density is the polynomial-times-trigonometric interpolant of the
    nodal values of Y_l, within ~1e-12 of Y_l for l = 2 at 16 Gauss-Legendre
    nodes in polar angle; hence that case's bar.)"""
    sc = synth.config1(4)
    y, _, _ = oracle.nodes(sc)
    sig = _y_l(l, y)
    rng = np.random.default_rng(40 + l)
    v = _dirs(rng, 4)
    for r in (0.5, 1 - 1e-4):
        us, _ = _ev(sc, sig, v * r)
        assert np.abs(us - _y_l(l, v) * r ** l / (2 * l + 1)).max() < bar
    for r in (1 + 1e-4, 2.0):
        us, _ = _ev(sc, sig, v * r)
        assert np.abs(us - _y_l(l, v) / ((2 * l + 1) * r ** (l + 1))).max() < bar
    nodes = rng.choice(sc.n_nodes, 5, replace=False)
    us, _ = _ev(sc, sig, None, nodes)
    assert np.abs(us - _y_l(l, y[nodes]) / (2 * l + 1)).max() < bar


@pytest.mark.parametrize("d", (1e-2, 1e-4, 1e-7))
def test_greens_representation_torus(d):
    """Section 5.1's test geometry and charge, checked inside, on and outside."""
    sc = synth.Scene([synth.torus_body(8, 1.0, 0.25)])
    y, n, _ = oracle.nodes(sc)
    x0 = np.array([1.0, 2.0, 3.0])
    r = y - x0
    rn = np.linalg.norm(r, axis=1)
    u = 1 / (4 * math.pi * rn)
    dudn = -np.sum(r * n, 1) / (4 * math.pi * rn ** 3)
    rng = np.random.default_rng(60 + int(-math.log10(d)))
    k = rng.choice(sc.n_nodes, 3, replace=False)
    xin, xout = y[k] - d * n[k], y[k] + d * n[k]
    ref = lambda x: 1 / (4 * math.pi * np.linalg.norm(x - x0, axis=1))
    scale = np.abs(u).max()
    s1, _ = _ev(sc, dudn, xin)
    _, d1 = _ev(sc, u, xin)
    assert np.abs(s1 - d1 - ref(xin)).max() < 1e-12 * scale
    s1, _ = _ev(sc, dudn, xout)
    _, d1 = _ev(sc, u, xout)
    assert np.abs(s1 - d1).max() < 1e-12 * scale
    nodes = rng.choice(sc.n_nodes, 4, replace=False)
    s1, _ = _ev(sc, dudn, None, nodes)
    _, d1 = _ev(sc, u, None, nodes)
    assert np.abs(s1 - d1 - 0.5 * u[nodes]).max() < 1e-12 * scale


def test_kernel_switch_restores_stokes():
    """The Laplace setting is confined to its call: a Stokes evaluation
    afterwards gives the Stokes double layer of a constant (c inside)."""
    sc = synth.config1(4)
    _ev(sc, np.ones(sc.n_nodes), np.array([[0.1, 0.2, 0.3]]))
    c = np.array([0.3, -0.4, 0.5])
    _, ud = oracle.evaluate(sc, np.tile(c, (sc.n_nodes, 1)), np.array([[0.1, 0.2, 0.3]]), np.array([-1]))
    assert np.abs(ud[0] - c).max() < 1e-12
