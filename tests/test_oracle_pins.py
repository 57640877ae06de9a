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


def _ev(scene, sigma, x=None, tgt_node=None, **kw):
    """oracle.evaluate that also requires every adaptive cell to have met its
    tolerance before the depth cap."""
    if x is not None and tgt_node is None:
        tgt_node = -np.ones(len(x), np.int64)
    us, ud, deep = oracle.evaluate(scene, sigma, x, tgt_node, return_deep=True, **kw)
    assert deep == 0, f"{deep} adaptive cells accepted at the depth cap"
    return us, ud


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
    _, din = _ev(sc, sig, xin, -np.ones(6, np.int64))
    _, dout = _ev(sc, sig, xout, -np.ones(6, np.int64))
    _, don = _ev(sc, sig, None, nodes)
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
    _, din = _ev(sc, sig, xin, -np.ones(3, np.int64))
    _, dout = _ev(sc, sig, xout, -np.ones(3, np.int64))
    _, don = _ev(sc, sig, None, nodes)
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
    _, din = _ev(sc, sig, xin, -np.ones(5, np.int64))
    _, dout = _ev(sc, sig, xout, -np.ones(5, np.int64))
    _, don = _ev(sc, sig, None, nodes)
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
    sin_, _ = _ev(sc, sig, xin, -np.ones(4, np.int64))
    son, _ = _ev(sc, sig, None, nodes)
    sout, _ = _ev(sc, sig, xout, -np.ones(6, np.int64))
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
    sin_, _ = _ev(sc, sig, xin, -np.ones(4, np.int64))
    son, _ = _ev(sc, sig, None, nodes)
    sout, _ = _ev(sc, sig, xout, -np.ones(4, np.int64))
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
        a1, _ = _ev(sc, traction, xs, tn if tn is not None else -np.ones(len(xs), np.int64))
        _, b2 = _ev(sc, uy, xs, tn if tn is not None else -np.ones(len(xs), np.int64))
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
    us, ud = _ev(sc, None, xs, -np.ones(6, np.int64), force_adaptive=True)
    # the brute force forms x_c'' by differentiating a Legendre series twice,
    # which carries ~1e-12 relative rounding; a dropped term or a wrong sign
    # shows up at the 1e-3 level
    for k in range(6):
        bs, bd = _numpy_panel_potential(sc, xs[k])
        assert np.abs(us[k] - bs).max() < 5e-12 * max(1, np.abs(bs).max())
        assert np.abs(ud[k] - bd).max() < 5e-12 * max(1, np.abs(bd).max())


def _sphere_scene(center, radius, seed):
    b = synth.sphere_body(center, radius, [0.3, 0.5, 0.8], [1.0, 0.0, 0.0])
    sc = synth.Scene([b])
    sc.sigma = np.random.default_rng(seed).standard_normal((sc.n_nodes, 3))
    return sc


@pytest.mark.parametrize("radius", [1.0, 0.2])
def test_far_route_just_beyond_threshold_on_sphere(radius):
    """The oracle's far route (a plain 48 x 32 tensor rule) against adaptive
    integration just beyond the far test's threshold, on a sphere as one
    element (a body closed at its poles, the hardest case for a plain rule:
    the integrand is a high-degree polynomial in s).  They agree to 2e-14 of
    the largest value.  Two plausible weakenings are caught: the panel's own
    16-point rule as the far rule (6e-12 .. 3e-11 off) and a far test moved
    in to 2 % of its distance (2e-9 off)."""
    sc = _sphere_scene([0.3, -0.1, 0.2], radius, 5)
    y, _, _ = oracle.nodes(sc)
    cen = y.mean(0)
    v = np.random.default_rng(7).standard_normal((6, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    # threshold: 40 surface extents along s (pi * radius for a sphere in polar
    # angle) beyond the bounding ball (about 1.05 radius)
    xs = cen + v * (1.05 * radius + 1.02 * 40 * np.pi * radius)
    ref = _ev(sc, None, xs, force_adaptive=True, rel_tol=1e-18)
    far = _ev(sc, None, xs)
    assert max(_rel(far[0], ref[0]), _rel(far[1], ref[1])) < 2e-14
    weak = _ev(sc, None, xs, -np.ones(6, np.int64), far_ns_mult=1)
    assert max(_rel(weak[0], ref[0]), _rel(weak[1], ref[1])) > 1e-12
    xn = cen + v * 4.0 * radius
    refn = _ev(sc, None, xn, force_adaptive=True, rel_tol=1e-18)
    weak = _ev(sc, None, xn, -np.ones(6, np.int64), far_scale=0.02)
    assert max(_rel(weak[0], refn[0]), _rel(weak[1], refn[1])) > 1e-13


def test_far_route_just_beyond_threshold_on_pipe_panel():
    """Same on one fat pipe panel, whose threshold is 8 radii."""
    sc = synth.small_pipe_scene(n_panels=1, n_spheres=0)
    y, _, _ = oracle.nodes(sc)
    cen = y.mean(0)
    rad = np.linalg.norm(y - cen, axis=1).max()
    v = np.random.default_rng(8).standard_normal((6, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    xs = cen + v * (1.1 * rad + 8.1)
    ref = _ev(sc, None, xs, force_adaptive=True, rel_tol=1e-18)
    far = _ev(sc, None, xs)
    assert max(_rel(far[0], ref[0]), _rel(far[1], ref[1])) < 2e-14


def test_far_test_agrees_with_adaptive_and_smooth_sum():
    sc = synth.small_pipe_scene(n_panels=3, n_spheres=1)
    rng = np.random.default_rng(17)
    xs = np.array([[30.0, 5.0, 1.0], [-20.0, 12.0, -9.0]])
    a1, b1 = _ev(sc, None, xs, -np.ones(2, np.int64))
    a2, b2 = _ev(sc, None, xs, -np.ones(2, np.int64), force_adaptive=True)
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
    us, ud = _ev(sc, None, xs, -np.ones(3, np.int64))
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    shift = np.array([0.3, -1.0, 2.0])
    lam = 1.7
    rot = synth.Scene([synth.Body(b.s_break, lam * (b.xc @ q.T) + shift, lam * b.eps, b.e1 @ q.T, b.normal_sign)
                       for b in sc.bodies], sc.ns, sc.nt, sc.sigma @ q.T)
    us2, ud2 = _ev(rot, None, lam * (xs @ q.T) + shift, -np.ones(3, np.int64))
    assert np.abs(us2 - lam * (us @ q.T)).max() < 1e-12 * np.abs(us).max() * lam
    assert np.abs(ud2 - ud @ q.T).max() < 1e-12 * np.abs(ud).max()


# ---------------------------------------------------------------- near the surface
# The closed forms hold at any distance; these pins put targets 1e-3, 1e-5 and
# 1e-7 from the surface, inside and outside, where the integrands are nearly
# singular (the double layer jumps by the density across the surface).
NEAR = (1e-3, 1e-5, 1e-7)


@pytest.mark.parametrize("d", NEAR)
def test_sphere_closed_forms_near_surface(d):
    """P1 stresslet identity, P2 rigid rotation in the double layer, P3
    translating and P4 rotating sphere in the single layer, on the unit
    sphere at distance d inside and outside."""
    sc = synth.config1(4)
    y, _, _ = oracle.nodes(sc)
    rng = np.random.default_rng(int(-np.log10(d)))
    v = rng.standard_normal((4, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    xin, xout = v * (1 - d), v * (1 + d)
    c = rng.standard_normal(3)
    sig = np.tile(c, (sc.n_nodes, 1))
    _, din = _ev(sc, sig, xin)
    _, dout = _ev(sc, sig, xout)
    assert np.abs(din - c).max() < 1e-12 * np.abs(c).max()
    assert np.abs(dout).max() < 1e-12 * np.abs(c).max()
    b = rng.standard_normal(3)
    c0 = np.array([0.1, -0.2, 0.3])
    _, din = _ev(sc, np.cross(b, y - c0), xin)
    _, dout = _ev(sc, np.cross(b, y - c0), xout)
    assert np.abs(din - np.cross(b, xin - c0)).max() < 1e-12 * np.abs(b).max()
    assert np.abs(dout).max() < 1e-12 * np.abs(b).max()
    U = rng.standard_normal(3)
    sin_, _ = _ev(sc, np.tile(1.5 * U, (sc.n_nodes, 1)), xin)
    sout, _ = _ev(sc, np.tile(1.5 * U, (sc.n_nodes, 1)), xout)
    r = np.linalg.norm(xout, axis=1)[:, None]
    ur = np.sum(xout * U, 1)[:, None]
    ext = 0.75 * (U / r + ur * xout / r ** 3) + 0.25 * (U / r ** 3 - 3 * ur * xout / r ** 5)
    assert np.abs(sin_ - U).max() < 1e-12 * np.abs(U).max()
    assert np.abs(sout - ext).max() < 1e-12 * np.abs(U).max()
    Om = rng.standard_normal(3)
    sin_, _ = _ev(sc, 3.0 * np.cross(Om, y), xin)
    sout, _ = _ev(sc, 3.0 * np.cross(Om, y), xout)
    assert np.abs(sin_ - np.cross(Om, xin)).max() < 1e-12 * np.abs(Om).max()
    assert np.abs(sout - np.cross(Om, xout) / r ** 3).max() < 1e-12 * np.abs(Om).max()


@pytest.mark.parametrize("d", NEAR)
def test_closed_torus_identities_near_surface(d):
    """P1 stresslet identity and P5 Stokes Green's representation (stokeslet
    at (1, 2, 3), torus R = 1, eps = 0.25 as in the paper's Green's-identity
    validation) with targets d off surface nodes along the normal, inside and
    outside; the targets sit over GL nodes anywhere on the 8 panels."""
    b = synth.torus_body(8, 1.0, 0.25)
    sc = synth.Scene([b])
    y, n, _ = oracle.nodes(sc)
    rng = np.random.default_rng(20 + int(-np.log10(d)))
    k = rng.choice(sc.n_nodes, 3, replace=False)
    xin, xout = y[k] - d * n[k], y[k] + d * n[k]
    c = rng.standard_normal(3)
    sig = np.tile(c, (sc.n_nodes, 1))
    _, din = _ev(sc, sig, xin)
    _, dout = _ev(sc, sig, xout)
    assert np.abs(din - c).max() < 1e-12 * np.abs(c).max()
    assert np.abs(dout).max() < 1e-12 * np.abs(c).max()
    x0 = np.array([1.0, 2.0, 3.0])
    f = np.array([0.3, -0.7, 1.1])
    r = y - x0
    rn = np.linalg.norm(r, axis=1)[:, None]
    traction = -(3 / (4 * np.pi)) * r * np.sum(r * f, 1)[:, None] * np.sum(r * n, 1)[:, None] / rn ** 5
    uy = _stokeslet(r, f)
    scale = np.abs(_stokeslet(xin - x0, f)).max()
    a1, _ = _ev(sc, traction, xin)
    _, b2 = _ev(sc, uy, xin)
    assert np.abs(a1 + b2 - _stokeslet(xin - x0, f)).max() < 1e-12 * scale
    a1, _ = _ev(sc, traction, xout)
    _, b2 = _ev(sc, uy, xout)
    assert np.abs(a1 + b2).max() < 1e-12 * scale


def test_double_layer_jump_resolved_at_1e_7():
    """Across the unit sphere's surface at 1e-7 on either side the double
    layer of a constant density jumps by exactly that constant (c inside, 0
    outside): both near-singular integrals are resolved to 1e-12 (the oracle
    forms pairs inside an element's bounding ball in long double; in double
    the jump carries ~5e-10 of rounding at this distance)."""
    sc = synth.config1(4)
    c = np.array([0.7, -0.2, 0.4])
    sig = np.tile(c, (sc.n_nodes, 1))
    v = np.array([[0.6, 0.0, 0.8]])
    _, din = _ev(sc, sig, v * (1 - 1e-7))
    _, dout = _ev(sc, sig, v * (1 + 1e-7))
    assert np.abs((din - dout) - c).max() < 1e-12


def test_smooth_sum_scales_bound_the_sum_and_its_change():
    """The smooth sum's scales (the sums of |term| and the first-order change
    per unit displacement) are bounds: they dominate the sums themselves, and
    moving a target by delta changes the sums by at most delta times the
    change bound, while the bound is not loose by orders of magnitude (a
    dropped 1/r^3 term or a wrong power would break one side)."""
    sc = synth.small_pipe_scene(n_panels=4, n_spheres=2)
    y, n, _ = oracle.nodes(sc)
    rng = np.random.default_rng(5)
    k = rng.choice(sc.n_nodes, 40, replace=False)
    d = 10.0 ** rng.uniform(-3, -1, 40)[:, None]
    x = y[k] + d * n[k] * np.where(rng.random(40) < 0.5, 1, -1)[:, None]
    free = -np.ones(40, np.int64)
    us, ud = oracle.smooth_sum(sc, None, x, free)
    mag = oracle.smooth_sum_magnitude(sc, None, x, free)
    assert np.all(np.abs(us).max(1) <= mag[:, 0]) and np.all(np.abs(ud).max(1) <= mag[:, 1])
    delta = 1e-9
    e = rng.standard_normal((40, 3))
    e /= np.linalg.norm(e, axis=1)[:, None]
    us2, ud2 = oracle.smooth_sum(sc, None, x + delta * e, free)
    ch_s = np.abs(us2 - us).max(1)
    ch_d = np.abs(ud2 - ud).max(1)
    rnd = 1e-15
    assert np.all(ch_s <= 1.001 * delta * mag[:, 2] + rnd * mag[:, 0])
    assert np.all(ch_d <= 1.001 * delta * mag[:, 3] + rnd * mag[:, 1])
    assert (ch_s / (delta * mag[:, 2])).max() > 1e-2
    assert (ch_d / (delta * mag[:, 3])).max() > 1e-2
    # on-surface targets exclude only their own node: the scales are finite
    tn = rng.choice(sc.n_nodes, 20, replace=False)
    m2 = oracle.smooth_sum_magnitude(sc, None, None, tn)
    assert np.all(np.isfinite(m2)) and np.all(m2 > 0)
