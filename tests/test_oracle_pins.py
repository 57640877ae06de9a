"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against a closed form, an identity, a library
routine or an independent brute-force computation, chosen so that a dropped
term, a wrong sign or a transposed operand in the oracle fails one of them.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle
import synth


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# ---------------------------------------------------------------- quadrature
def test_gauss_legendre_matches_library_and_is_exact():
    for n in (1, 2, 5, 16, 20, 32):
        x, w = oracle.gauss_legendre(n)
        xr, wr = npleg.leggauss(n)
        assert np.abs(x - xr).max() < 2e-15 and np.abs(w - wr).max() < 2e-15
        for k in range(2 * n):
            exact = 0.0 if k % 2 else 2.0 / (k + 1)
            assert abs(np.dot(w, x ** k) - exact) < 1e-14


# ---------------------------------------------------------------- geometry
def test_sphere_surface_nodes_normals_area():
    sc = synth.config1(4)
    y, n, w = oracle.nodes(sc)
    assert np.abs(np.linalg.norm(y, axis=1) - 1).max() < 1e-14
    assert np.abs(n - y).max() < 1e-13          # outward unit normal of a unit sphere
    assert abs(w.sum() - 4 * np.pi) < 1e-13      # sphere area


def test_torus_surface_area_and_shape():
    b = synth.torus_body(8, 1.0, 0.25)
    sc = synth.Scene([b])
    y, n, w = oracle.nodes(sc)
    rho = np.hypot(y[:, 0], y[:, 1])
    assert np.abs(np.hypot(rho - 1.0, y[:, 2]) - 0.25).max() < 1e-13
    assert abs(w.sum() - 4 * np.pi ** 2 * 0.25) < 1e-12
    # normal points away from the centerline
    cen = np.stack([y[:, 0] / rho, y[:, 1] / rho, 0 * rho], 1)
    assert (np.sum(n * (y - cen), 1) > 0).all()


def test_interpolation_reproduces_polynomial_density_and_trig_modes():
    sc = synth.small_pipe_scene(n_panels=2, n_spheres=0)
    rng = np.random.default_rng(3)
    s_nodes = synth.panel_gl_points(sc.bodies[0].s_break, 16)
    th = 2 * np.pi * np.arange(32) / 32
    c = rng.standard_normal((16, 3))
    a = rng.standard_normal((3, 3))
    def f(s, t):   # degree-15 polynomial in s times modes 0, 5, 16 (Nyquist) in t
        P = npleg.legval(2 * s - 1, c)
        return (P.T * (1 + a[0] * np.cos(5 * t)[..., None] + a[1] * np.sin(5 * t)[..., None] +
                       a[2] * np.cos(16 * t)[..., None]).T).T
    S = np.repeat(s_nodes.reshape(-1), 32)
    T = np.tile(th, s_nodes.size)
    sig = np.stack([npleg.legval(2 * S - 1, c[:, d]) * (1 + a[0, d] * np.cos(5 * T) + a[1, d] * np.sin(5 * T)
                                                      + a[2, d] * np.cos(16 * T)) for d in range(3)], 1)
    sc.sigma = sig
    sp = rng.uniform(0, 0.5, 40)
    tp = rng.uniform(0, 2 * np.pi, 40)
    _, _, _, sg = oracle.surface_point(sc, 0, sp, tp, sig)
    ref = np.stack([npleg.legval(2 * sp - 1, c[:, d]) * (1 + a[0, d] * np.cos(5 * tp) + a[1, d] * np.sin(5 * tp)
                                                       + a[2, d] * np.cos(16 * tp)) for d in range(3)], 1)
    assert _rel(sg, ref) < 1e-13


# ---------------------------------------------------------------- identities
def _sphere_targets(rng, n, rmin, rmax):
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v * rng.uniform(rmin, rmax, n)[:, None]


def test_stresslet_identity_sphere_inside_on_outside():
    sc = synth.config1(4)
    rng = np.random.default_rng(11)
    c = rng.standard_normal(3)
    sig = np.tile(c, (sc.n_nodes, 1))
    xin = _sphere_targets(rng, 6, 0.0, 0.999)
    xout = _sphere_targets(rng, 6, 1.001, 3.0)
    nodes = rng.choice(sc.n_nodes, 6, replace=False)
    _, din = oracle.evaluate(sc, sig, xin, -np.ones(6, np.int64))
    _, dout = oracle.evaluate(sc, sig, xout, -np.ones(6, np.int64))
    _, don = oracle.evaluate(sc, sig, None, nodes)
    assert np.abs(din - c).max() < 1e-12
    assert np.abs(dout).max() < 1e-12
    assert np.abs(don - 0.5 * c).max() < 1e-12


def test_stresslet_identity_closed_torus():
    b = synth.torus_body(6, 1.0, 0.25)
    sc = synth.Scene([b])
    rng = np.random.default_rng(12)
    c = rng.standard_normal(3)
    sig = np.tile(c, (sc.n_nodes, 1))
    xin = np.array([[1.0, 0.0, 0.1], [0.0, -1.1, -0.05], [-0.9, 0.2, 0.0]])
    xout = np.array([[0.0, 0.0, 0.0], [1.3, 0.0, 0.0], [0.5, 0.5, 0.5]])
    nodes = rng.choice(sc.n_nodes, 4, replace=False)
    _, din = oracle.evaluate(sc, sig, xin, -np.ones(3, np.int64))
    _, dout = oracle.evaluate(sc, sig, xout, -np.ones(3, np.int64))
    _, don = oracle.evaluate(sc, sig, None, nodes)
    assert np.abs(din - c).max() < 1e-12
    assert np.abs(dout).max() < 1e-12
    assert np.abs(don - 0.5 * c).max() < 1e-12


def test_double_layer_of_rigid_rotation():
    sc = synth.config1(4)
    y, _, _ = oracle.nodes(sc)
    rng = np.random.default_rng(13)
    bvec = rng.standard_normal(3)
    c0 = np.array([0.1, -0.2, 0.3])
    sig = np.cross(bvec, y - c0)
    xin = _sphere_targets(rng, 5, 0.0, 0.99)
    xout = _sphere_targets(rng, 5, 1.01, 2.0)
    nodes = rng.choice(sc.n_nodes, 5, replace=False)
    _, din = oracle.evaluate(sc, sig, xin, -np.ones(5, np.int64))
    _, dout = oracle.evaluate(sc, sig, xout, -np.ones(5, np.int64))
    _, don = oracle.evaluate(sc, sig, None, nodes)
    assert np.abs(din - np.cross(bvec, xin - c0)).max() < 1e-12
    assert np.abs(dout).max() < 1e-12
    assert np.abs(don - 0.5 * np.cross(bvec, y[nodes] - c0)).max() < 1e-12


def test_translating_sphere_single_layer():
    sc = synth.config1(4)
    rng = np.random.default_rng(14)
    U = rng.standard_normal(3)
    sig = np.tile(1.5 * U, (sc.n_nodes, 1))       # traction 3U/(2a), a = 1
    xin = _sphere_targets(rng, 4, 0.0, 0.999)
    xout = _sphere_targets(rng, 6, 1.001, 4.0)
    nodes = rng.choice(sc.n_nodes, 4, replace=False)
    sin_, _ = oracle.evaluate(sc, sig, xin, -np.ones(4, np.int64))
    son, _ = oracle.evaluate(sc, sig, None, nodes)
    sout, _ = oracle.evaluate(sc, sig, xout, -np.ones(6, np.int64))
    r = np.linalg.norm(xout, axis=1)[:, None]
    ur = np.sum(xout * U, 1)[:, None]
    ext = 0.75 * (U / r + ur * xout / r ** 3) + 0.25 * (U / r ** 3 - 3 * ur * xout / r ** 5)
    assert np.abs(sin_ - U).max() < 1e-12
    assert np.abs(son - U).max() < 1e-12
    assert np.abs(sout - ext).max() < 1e-12


def test_rotating_sphere_single_layer():
    sc = synth.config1(4)
    y, _, _ = oracle.nodes(sc)
    rng = np.random.default_rng(15)
    Om = rng.standard_normal(3)
    sig = 3.0 * np.cross(Om, y)                   # traction (3/a) Omega x (y - c)
    xin = _sphere_targets(rng, 4, 0.0, 0.99)
    xout = _sphere_targets(rng, 4, 1.01, 3.0)
    nodes = rng.choice(sc.n_nodes, 4, replace=False)
    sin_, _ = oracle.evaluate(sc, sig, xin, -np.ones(4, np.int64))
    son, _ = oracle.evaluate(sc, sig, None, nodes)
    sout, _ = oracle.evaluate(sc, sig, xout, -np.ones(4, np.int64))
    r = np.linalg.norm(xout, axis=1)[:, None]
    assert np.abs(sin_ - np.cross(Om, xin)).max() < 1e-12
    assert np.abs(son - np.cross(Om, y[nodes])).max() < 1e-12
    assert np.abs(sout - np.cross(Om, xout) / r ** 3).max() < 1e-12


def _stokeslet(r, f):
    rn = np.linalg.norm(r, axis=-1)[..., None]
    return (f / rn + r * np.sum(r * f, -1)[..., None] / rn ** 3) / (8 * np.pi)


def test_greens_representation_closed_torus():
    """Stokeslet flow from a point outside the body: S[t] + D[u] = u inside,
    u/2 on the surface and 0 in the fluid (the Stokes analogue of the paper's
    Green's-identity validation on a torus, R = 1, eps = 0.25, source (1,2,3))."""
    b = synth.torus_body(8, 1.0, 0.25)
    sc = synth.Scene([b])
    y, n, _ = oracle.nodes(sc)
    x0 = np.array([1.0, 2.0, 3.0])
    f = np.array([0.3, -0.7, 1.1])
    r = y - x0
    rn = np.linalg.norm(r, axis=1)[:, None]
    traction = -(3 / (4 * np.pi)) * r * np.sum(r * f, 1)[:, None] * np.sum(r * n, 1)[:, None] / rn ** 5
    uy = _stokeslet(r, f)
    xin = np.array([[1.0, 0.1, 0.05], [0.0, -1.1, 0.0], [-0.95, 0.0, -0.1]])
    xout = np.array([[0.0, 0.0, 0.0], [2.0, 0.5, 0.3]])
    nodes = np.array([0, 77, 1000, 3333])
    for xs, tn, fac in ((xin, None, 1.0), (xout, None, 0.0), (None, nodes, 0.5)):
        a1, _ = oracle.evaluate(sc, traction, xs, tn if tn is not None else -np.ones(len(xs), np.int64))
        _, b2 = oracle.evaluate(sc, uy, xs, tn if tn is not None else -np.ones(len(xs), np.int64))
        xt = y[nodes] if xs is None else xs
        assert np.abs(a1 + b2 - fac * _stokeslet(xt - x0, f)).max() < 1e-12


# ---------------------------------------------------------------- brute force
def _numpy_panel_potential(sc, x, nsq=96, ntq=2048):
    """Independent brute-force tensor rule on one torus-arc pipe panel
    (e1 = z, constant radius) written with numpy's Legendre routines."""
    b = sc.bodies[0]
    a, c = b.s_break[0], b.s_break[1]
    xg, wg = npleg.leggauss(16)
    # discrete Legendre transform at the GL nodes (exact interpolation)
    T = npleg.legvander(xg, 15) * wg[:, None] * (np.arange(16) + 0.5)[None, :]

    def legcoef(f):
        return T.T @ f

    X = b.xc[0]
    cx = legcoef(X)
    ce = legcoef(b.eps[0])
    sq, wq = npleg.leggauss(nsq)
    ds = 2.0 / (c - a)
    Xs = npleg.legval(sq, cx).T
    X1 = npleg.legval(sq, npleg.legder(cx)).T * ds
    X2 = npleg.legval(sq, npleg.legder(cx, 2)).T * ds ** 2
    E = npleg.legval(sq, ce)
    E1 = npleg.legval(sq, npleg.legder(ce)) * ds
    sp = np.linalg.norm(X1, axis=1)[:, None]
    t = X1 / sp
    tp = (X2 - np.sum(X2 * t, 1)[:, None] * t) / sp
    z = np.array([0.0, 0.0, 1.0])
    e1 = np.tile(z, (nsq, 1))
    e2 = np.cross(t, e1)
    e2p = np.cross(tp, e1)
    th = 2 * np.pi * np.arange(ntq) / ntq
    ct, st = np.cos(th)[None, :, None], np.sin(th)[None, :, None]
    Y = Xs[:, None, :] + E[:, None, None] * (e1[:, None, :] * ct + e2[:, None, :] * st)
    Ys = X1[:, None, :] + E1[:, None, None] * (e1[:, None, :] * ct + e2[:, None, :] * st) + \
        E[:, None, None] * (e2p[:, None, :] * st)
    Yt = E[:, None, None] * (-e1[:, None, :] * st + e2[:, None, :] * ct)
    Jn = np.cross(Yt, Ys)
    J = np.linalg.norm(Jn, axis=-1)
    nrm = Jn / J[..., None]
    # density interpolant: Legendre in s at each node angle, then FFT trig interpolation
    sig = sc.sigma.reshape(16, 32, 3)
    cs = legcoef(sig.reshape(16, -1))
    sq_vals = npleg.legval(sq, cs).T.reshape(nsq, 32, 3)
    F = np.fft.rfft(sq_vals, axis=1)
    F[:, 16, :] *= 0.5  # Nyquist split symmetrically: real part of the one-sided sum
    Fz = np.zeros((nsq, ntq // 2 + 1, 3), dtype=complex)
    Fz[:, :17, :] = F
    Fz[:, 16, :] *= 1.0
    sig_q = np.fft.irfft(Fz, n=ntq, axis=1) * (ntq / 32)
    # Nyquist: cos(16 t) coefficient must be F16/32 (not doubled); irfft doubles interior bins
    W = J * (wq / ds)[:, None] * (2 * np.pi / ntq)
    r = x[None, None, :] - Y
    rr = np.sqrt(np.sum(r * r, -1))
    rs = np.sum(r * sig_q, -1)
    rn = np.sum(r * nrm, -1)
    uS = np.sum(W[..., None] * (sig_q / rr[..., None] + r * (rs / rr ** 3)[..., None]), (0, 1)) / (8 * np.pi)
    uD = -3 / (4 * np.pi) * np.sum(W[..., None] * r * (rn * rs / rr ** 5)[..., None], (0, 1))
    return uS, uD


def test_adaptive_oracle_matches_brute_force_on_curved_panel():
    sc = synth.small_pipe_scene(n_panels=1, n_spheres=0, arc=0.1)
    rng = np.random.default_rng(16)
    sc.sigma = rng.standard_normal((sc.n_nodes, 3)) * 0 + synth.wall_density(sc.bodies[0], 16, 32, rng)
    # targets 0.25 .. 0.6 away from the wall, inside and outside
    y, n, _ = oracle.nodes(sc)
    pick = rng.choice(sc.n_nodes, 6, replace=False)
    d = rng.uniform(0.25, 0.6, 6) * np.where(np.arange(6) % 2, 1, -1)
    xs = y[pick] + d[:, None] * n[pick]
    us, ud = oracle.evaluate(sc, None, xs, -np.ones(6, np.int64), force_adaptive=True)
    # the brute force forms x_c'' by differentiating a Legendre series twice,
    # which carries ~1e-12 relative rounding; a dropped term or a wrong sign
    # shows up at the 1e-3 level
    for k in range(6):
        bs, bd = _numpy_panel_potential(sc, xs[k])
        assert np.abs(us[k] - bs).max() < 5e-12 * max(1, np.abs(bs).max())
        assert np.abs(ud[k] - bd).max() < 5e-12 * max(1, np.abs(bd).max())


def test_far_test_agrees_with_adaptive_and_smooth_sum():
    sc = synth.small_pipe_scene(n_panels=3, n_spheres=1)
    rng = np.random.default_rng(17)
    xs = np.array([[30.0, 5.0, 1.0], [-20.0, 12.0, -9.0]])
    a1, b1 = oracle.evaluate(sc, None, xs, -np.ones(2, np.int64))
    a2, b2 = oracle.evaluate(sc, None, xs, -np.ones(2, np.int64), force_adaptive=True)
    a3, b3 = oracle.smooth_sum(sc, None, xs, -np.ones(2, np.int64))
    # far values are ~1e-3 of the near-field scale the adaptive tolerance is set on
    for p, q in ((a1, a2), (b1, b2), (a1, a3), (b1, b3)):
        assert _rel(p, q) < 1e-12


# ---------------------------------------------------------------- invariances
def test_rigid_motion_and_scaling_invariance():
    sc = synth.small_pipe_scene(n_panels=2, n_spheres=1, arc=0.3)
    rng = np.random.default_rng(18)
    y, n, _ = oracle.nodes(sc)
    xs = y[rng.choice(sc.n_nodes, 3, replace=False)] + 0.05 * rng.standard_normal((3, 3))
    us, ud = oracle.evaluate(sc, None, xs, -np.ones(3, np.int64))
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    shift = np.array([0.3, -1.0, 2.0])
    lam = 1.7
    rot = synth.Scene([synth.Body(b.s_break, lam * (b.xc @ q.T) + shift, lam * b.eps, b.e1 @ q.T, b.normal_sign)
                       for b in sc.bodies], sc.ns, sc.nt, sc.sigma @ q.T)
    us2, ud2 = oracle.evaluate(rot, None, lam * (xs @ q.T) + shift, -np.ones(3, np.int64))
    assert np.abs(us2 - lam * (us @ q.T)).max() < 1e-12 * np.abs(us).max() * lam
    assert np.abs(ud2 - ud @ q.T).max() < 1e-12 * np.abs(ud).max()
