"""Seeded synthetic workloads for the Stokes layer-potential evaluator.

This module only *describes* inputs: body centerlines sampled at the
Gauss-Legendre nodes of each panel, nodal densities and target lists.  It
holds none of the quadrature method's arithmetic (no surface expansion, no
kernels, no interpolation) and is shared by the CPU oracle, the tests and the
benchmark.

Discretisation convention (the paper's Section 3.1, surface discretisation):
a body is a centerline x_c(s), s in [0,1], with cross-section radius eps(s)
and an orientation vector e1(s) orthogonal to the centerline.  The interval is
cut into panels; each panel carries the values of x_c, eps, e1 at its ``ns``
Gauss-Legendre nodes (ascending in s).  Surface nodes are the tensor product of
those s-nodes with ``nt`` uniform angles theta_j = 2 pi j / nt, j = 0..nt-1,
numbered body-major, then panel, then s-node, then angle.

Workload recipe (seed = 1000 * config + stream; stream 0 = geometry,
1 = densities, 2 = targets):

* config 1: unit sphere as one element, SH density of degree <= 8, 2000 targets
  at distance 10**U(-3,0) from the surface, half inside and half outside.
* config 2: torus-arc pipe (centerline radius 5, radius 1, arc pi, 100 panels)
  with 200 spheres of radius 0.2 placed by random sequential addition
  (gap >= 0.02 to each other and to the wall); targets = all surface nodes.
* config 3: the config-2 pipe scaled by (1000/200)**(1/3) holding 1000 spheres.
* config 4: 64 independent pipe geometries of uneven size.
* config 5: 2000 spheres in the pipe scaled by 10**(1/3).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy.special import lpmv

NS = 16
NT = 32


@dataclasses.dataclass
class Body:
    s_break: np.ndarray      # (P+1,) panel end points in [0,1]
    xc: np.ndarray           # (P, ns, 3) centerline at panel GL nodes
    eps: np.ndarray          # (P, ns) cross-section radius
    e1: np.ndarray           # (P, ns, 3) orientation vector (orthogonal to centerline)
    normal_sign: int = 1
    kind: str = "body"       # "sphere", "pipe", "torus" (labels only)

    @property
    def n_panels(self) -> int:
        return int(self.xc.shape[0])


@dataclasses.dataclass
class Scene:
    bodies: List[Body]
    ns: int = NS
    nt: int = NT
    sigma: Optional[np.ndarray] = None      # (N, 3) nodal density
    x: Optional[np.ndarray] = None          # (T, 3) targets (ignored where tgt_node >= 0)
    tgt_node: Optional[np.ndarray] = None   # (T,) int64 node id or -1
    tgt_class: Optional[np.ndarray] = None  # (T,) int class label
    class_names: tuple = ()
    name: str = ""

    @property
    def n_panels(self) -> int:
        return sum(b.n_panels for b in self.bodies)

    @property
    def n_nodes(self) -> int:
        return self.n_panels * self.ns * self.nt

    def body_node_offsets(self) -> np.ndarray:
        off = [0]
        for b in self.bodies:
            off.append(off[-1] + b.n_panels * self.ns * self.nt)
        return np.asarray(off, dtype=np.int64)

    def flat(self) -> dict:
        """Concatenated C-contiguous arrays (body-major) for the C interfaces."""
        return dict(
            n_bodies=len(self.bodies),
            n_panels=np.ascontiguousarray([b.n_panels for b in self.bodies], dtype=np.int32),
            normal_sign=np.ascontiguousarray([b.normal_sign for b in self.bodies], dtype=np.int32),
            s_break=np.ascontiguousarray(np.concatenate([b.s_break for b in self.bodies]), dtype=np.float64),
            xc=np.ascontiguousarray(np.concatenate([b.xc.reshape(-1, 3) for b in self.bodies]), dtype=np.float64),
            eps=np.ascontiguousarray(np.concatenate([b.eps.reshape(-1) for b in self.bodies]), dtype=np.float64),
            e1=np.ascontiguousarray(np.concatenate([b.e1.reshape(-1, 3) for b in self.bodies]), dtype=np.float64),
        )

    def subset_targets(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return dataclasses.replace(
            self, x=self.x[idx].copy(), tgt_node=self.tgt_node[idx].copy(),
            tgt_class=None if self.tgt_class is None else self.tgt_class[idx].copy())


# --------------------------------------------------------------------------
# centerline samplers
# --------------------------------------------------------------------------

def panel_gl_points(s_break: np.ndarray, ns: int) -> np.ndarray:
    """(P, ns) GL nodes (ascending) of each panel [s_break[k], s_break[k+1]]."""
    xg, _ = leggauss(ns)
    a = s_break[:-1, None]
    b = s_break[1:, None]
    return 0.5 * (a + b) + 0.5 * (b - a) * xg[None, :]


def sphere_body(center, radius, axis, e1, ns=NS) -> Body:
    """Sphere as one element: x_c(s) = c + a cos(pi s) axis, eps = a sin(pi s)."""
    center = np.asarray(center, float)
    axis = np.asarray(axis, float)
    axis = axis / np.linalg.norm(axis)
    e1 = np.asarray(e1, float)
    e1 = e1 - np.dot(e1, axis) * axis
    e1 = e1 / np.linalg.norm(e1)
    sb = np.array([0.0, 1.0])
    s = panel_gl_points(sb, ns)[0]
    xc = center[None, :] + radius * np.cos(np.pi * s)[:, None] * axis[None, :]
    eps = radius * np.sin(np.pi * s)
    e1s = np.repeat(e1[None, :], ns, axis=0)
    return Body(sb, xc[None], eps[None], e1s[None], 1, "sphere")


def pipe_body(n_panels=100, R=5.0, radius=1.0, arc=math.pi, ns=NS) -> Body:
    """Torus-arc tube: x_c(s) = R (cos(arc s), sin(arc s), 0), eps = radius, e1 = z."""
    sb = np.linspace(0.0, 1.0, n_panels + 1)
    s = panel_gl_points(sb, ns)
    xc = np.stack([R * np.cos(arc * s), R * np.sin(arc * s), np.zeros_like(s)], axis=-1)
    eps = np.full_like(s, radius)
    e1 = np.zeros_like(xc)
    e1[..., 2] = 1.0
    return Body(sb, xc, eps, e1, 1, "pipe")


def torus_body(n_panels=8, R=1.0, radius=0.25, ns=NS) -> Body:
    """Closed torus loop (used by closed-surface identities)."""
    b = pipe_body(n_panels, R, radius, 2 * math.pi, ns)
    b.kind = "torus"
    return b


def straight_tube_body(n_panels=4, length=2.0, radius=1e-2, ns=NS) -> Body:
    """Open straight tube along z: x_c(s) = (0, 0, length s), constant radius,
    e1 = x (every panel a straight cylinder of constant radius)."""
    sb = np.linspace(0.0, 1.0, n_panels + 1)
    s = panel_gl_points(sb, ns)
    xc = np.stack([np.zeros_like(s), np.zeros_like(s), length * s], axis=-1)
    eps = np.full_like(s, radius)
    e1 = np.zeros_like(xc)
    e1[..., 0] = 1.0
    return Body(sb, xc, eps, e1, 1, "tube")


def wavy_ring_body(n_panels=8, R=1.0, radius=1e-2, taper=0.3, ns=NS) -> Body:
    """Closed slender loop that is neither planar nor of constant radius:
    x_c(s) = (R + 0.1 R cos 3u) (cos u, sin u, 0) + 0.15 R sin 2u z, u = 2 pi s,
    eps = radius (1 + taper cos 4u), e1 = z (re-orthonormalised by the
    evaluators against the tangent)."""
    sb = np.linspace(0.0, 1.0, n_panels + 1)
    u = 2 * math.pi * panel_gl_points(sb, ns)
    rr = R * (1.0 + 0.1 * np.cos(3 * u))
    xc = np.stack([rr * np.cos(u), rr * np.sin(u), 0.15 * R * np.sin(2 * u)], axis=-1)
    eps = radius * (1.0 + taper * np.cos(4 * u))
    e1 = np.zeros_like(xc)
    e1[..., 2] = 1.0
    return Body(sb, xc, eps, e1, 1, "ring")


# --------------------------------------------------------------------------
# densities
# --------------------------------------------------------------------------

def _real_sh(l, m, polar, azim):
    am = abs(m)
    norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
    p = lpmv(am, l, np.cos(polar))
    if m == 0:
        return norm * p
    if m > 0:
        return math.sqrt(2.0) * norm * p * np.cos(am * azim)
    return math.sqrt(2.0) * norm * p * np.sin(am * azim)


def sh_density(ns, nt, rng, lmax=8) -> np.ndarray:
    """(ns*nt, 3) density on a sphere element: each component a real SH series
    of degree <= lmax with N(0,1) coefficients, evaluated at the node angles
    (polar = pi s_i, azimuth = -theta_j)."""
    s = panel_gl_points(np.array([0.0, 1.0]), ns)[0]
    th = 2 * np.pi * np.arange(nt) / nt
    polar = np.repeat(np.pi * s, nt)
    azim = np.tile(-th, ns)
    out = np.zeros((ns * nt, 3))
    for c in range(3):
        for l in range(lmax + 1):
            for m in range(-l, l + 1):
                out[:, c] += rng.standard_normal() * _real_sh(l, m, polar, azim)
    return out


def wall_density(body: Body, ns, nt, rng, kmax=12, mmax=8) -> np.ndarray:
    """(P*ns*nt, 3) smooth wall density: Fourier modes in s (k <= kmax) and
    theta (m <= mmax) with N(0,1)/((1+k)(1+m)) coefficients."""
    s = panel_gl_points(body.s_break, ns).reshape(-1)
    th = 2 * np.pi * np.arange(nt) / nt
    S = np.repeat(s, nt)
    T = np.tile(th, s.size)
    out = np.zeros((S.size, 3))
    for c in range(3):
        for k in range(kmax + 1):
            fs = [np.cos(2 * np.pi * k * S)] + ([np.sin(2 * np.pi * k * S)] if k > 0 else [])
            for m in range(mmax + 1):
                ft = [np.cos(m * T)] + ([np.sin(m * T)] if m > 0 else [])
                for a in fs:
                    for b in ft:
                        out[:, c] += rng.standard_normal() / ((1 + k) * (1 + m)) * a * b
    return out


# --------------------------------------------------------------------------
# geometry builders
# --------------------------------------------------------------------------

def _random_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def place_spheres(rng, m, radius, pipe_R, pipe_r, arc, gap, max_tries=2_000_000):
    """Random sequential addition of m spheres (radius, or array of radii) inside
    a torus-arc tube, keeping `gap` to each other, to the wall and to the open
    ends.  Centres are uniform in the tube volume."""
    radii = np.broadcast_to(np.asarray(radius, float), (m,)).copy()
    centers = np.zeros((m, 3))
    placed = 0
    tries = 0
    gaps = np.broadcast_to(np.asarray(gap, float), (m,))
    while placed < m:
        tries += 1
        if tries > max_tries:
            raise RuntimeError(f"RSA failed after {max_tries} tries ({placed}/{m} placed)")
        a = radii[placed]
        g = gaps[placed]
        rmax = pipe_r - a - g
        if rmax <= 0:
            raise ValueError("sphere does not fit in the pipe")
        r = rmax * math.sqrt(rng.random())
        psi = 2 * math.pi * rng.random()
        if rng.random() > (pipe_R + r * math.cos(psi)) / (pipe_R + rmax):
            continue
        loc = pipe_R + r * math.cos(psi)
        margin = (a + g) / (pipe_R - rmax)
        phi = margin + (arc - 2 * margin) * rng.random()
        c = np.array([loc * math.cos(phi), loc * math.sin(phi), r * math.sin(psi)])
        if placed:
            d = np.linalg.norm(centers[:placed] - c[None, :], axis=1)
            if np.any(d < radii[:placed] + a + np.maximum(gaps[:placed], g)):
                continue
        centers[placed] = c
        placed += 1
    return centers, radii


def pipe_scene(seed_base, n_spheres, scale=1.0, n_panels=100, radius=0.2, gap=0.02,
               ns=NS, nt=NT, radii=None, gaps=None) -> Scene:
    rng_g = np.random.default_rng(seed_base + 0)
    pipe = pipe_body(n_panels, 5.0 * scale, 1.0 * scale, math.pi, ns)
    rad = radius if radii is None else radii
    gp = gap if gaps is None else gaps
    centers, rads = place_spheres(rng_g, n_spheres, rad, 5.0 * scale, 1.0 * scale, math.pi, gp)
    bodies = [pipe]
    for i in range(n_spheres):
        rot = _random_rotation(rng_g)
        bodies.append(sphere_body(centers[i], rads[i], rot[:, 2], rot[:, 0], ns))
    rng_d = np.random.default_rng(seed_base + 1)
    sig = [wall_density(pipe, ns, nt, rng_d)]
    for _ in range(n_spheres):
        sig.append(sh_density(ns, nt, rng_d))
    sc = Scene(bodies, ns, nt, np.ascontiguousarray(np.concatenate(sig)))
    sc.sphere_centers = centers
    sc.sphere_radii = rads
    sc.pipe_scale = scale
    n = sc.n_nodes
    sc.x = np.zeros((n, 3))
    sc.tgt_node = np.arange(n, dtype=np.int64)
    nwall = pipe.n_panels * ns * nt
    cls = np.zeros(n, dtype=np.int32)
    cls[nwall:] = 1
    sc.tgt_class = cls
    sc.class_names = ("wall", "particle", "near-contact")
    return sc


def analytic_node_positions(sc: Scene) -> np.ndarray:
    """Node positions from the generating analytic shapes (used only to label
    target classes; the evaluators expand the surface themselves)."""
    out = []
    th = 2 * np.pi * np.arange(sc.nt) / sc.nt
    for b in sc.bodies:
        s = panel_gl_points(b.s_break, sc.ns)
        xc = b.xc
        t = np.zeros_like(xc)
        # tangent direction from the analytic shapes used here
        if b.kind == "sphere":
            ax = (xc[0, -1] - xc[0, 0])
            ax = ax / np.linalg.norm(ax)
            t[:] = ax
        else:
            R = np.linalg.norm(xc[..., :2], axis=-1)
            t[..., 0] = -xc[..., 1] / R
            t[..., 1] = xc[..., 0] / R
        e1 = b.e1 - np.sum(b.e1 * t, -1, keepdims=True) * t
        e1 /= np.linalg.norm(e1, axis=-1, keepdims=True)
        e2 = np.cross(t, e1)
        y = (xc[..., None, :] + b.eps[..., None, None] *
             (e1[..., None, :] * np.cos(th)[:, None] + e2[..., None, :] * np.sin(th)[:, None]))
        out.append(y.reshape(-1, 3))
    return np.concatenate(out)


def label_near_contact(sc: Scene, dist=0.1):
    """Particle nodes within `dist` of another surface get class 2."""
    y = analytic_node_positions(sc)
    cls = sc.tgt_class.copy()
    nwall = sc.bodies[0].n_panels * sc.ns * sc.nt
    per = sc.ns * sc.nt
    centers = sc.sphere_centers
    radii = sc.sphere_radii
    R = 5.0 * sc.pipe_scale
    r_pipe = 1.0 * sc.pipe_scale
    for i in range(len(centers)):
        yi = y[nwall + i * per: nwall + (i + 1) * per]
        # wall distance (torus tube)
        rho = np.linalg.norm(yi[:, :2], axis=1)
        dw = r_pipe - np.sqrt((rho - R) ** 2 + yi[:, 2] ** 2)
        near = dw < dist
        dc = np.linalg.norm(centers - centers[i][None, :], axis=1) - radii - radii[i]
        for j in np.nonzero(dc < dist + 1e-12)[0]:
            if j == i:
                continue
            near |= np.linalg.norm(yi - centers[j][None, :], axis=1) - radii[j] < dist
        sub = cls[nwall + i * per: nwall + (i + 1) * per]
        sub[near] = 2
    sc.tgt_class = cls
    return sc


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def config1(n_targets=2000, seed=1000) -> Scene:
    b = sphere_body([0, 0, 0], 1.0, [0, 0, 1], [1, 0, 0])
    sig = sh_density(NS, NT, np.random.default_rng(seed + 1))
    rng = np.random.default_rng(seed + 2)
    v = rng.standard_normal((n_targets, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    d = 10.0 ** rng.uniform(-3, 0, n_targets)
    half = n_targets // 2
    r = np.concatenate([1 - d[:half], 1 + d[half:]])
    x = v * r[:, None]
    cls = np.concatenate([np.zeros(half, np.int32), np.ones(n_targets - half, np.int32)])
    return Scene([b], NS, NT, sig, x, -np.ones(n_targets, np.int64), cls,
                 ("inside", "outside"), "sphere-512")


def config2(seed=2000) -> Scene:
    sc = pipe_scene(seed, 200, 1.0)
    sc.name = "pipe100-spheres200"
    return sc


def config3(seed=3000, label=True) -> Scene:
    sc = pipe_scene(seed, 1000, (1000 / 200) ** (1 / 3))
    sc.name = "pipe100x1.71-spheres1000"
    if label:
        label_near_contact(sc)
    return sc


def config4(seed=4000, n_geom=64, max_spheres=500, max_panels=200, progress=None):
    """List of independent scenes: panels U{20..200}, spheres U{10..500},
    radii U(0.1,0.25), gaps 10**U(-3,-1); pipe scaled so RSA stays at <= 13.6 %.
    progress(g, scene) is called after each geometry (the full size takes
    minutes of host time)."""
    rng = np.random.default_rng(seed)
    scenes = []
    for g in range(n_geom):
        P = int(rng.integers(20, max_panels + 1))
        M = int(rng.integers(10, max_spheres + 1))
        radii = rng.uniform(0.1, 0.25, M)
        gaps = 10.0 ** rng.uniform(-3, -1, M)
        vs = np.sum(4 / 3 * np.pi * radii ** 3)
        vpipe = np.pi * 1.0 ** 2 * 5.0 * np.pi
        lam = max(1.0, (vs / (0.136 * vpipe)) ** (1 / 3))
        sc = pipe_scene(seed + 17 * (g + 1), M, lam, n_panels=P, radii=radii, gaps=gaps)
        sc.name = f"batch{g}-P{P}-M{M}"
        scenes.append(sc)
        if progress is not None:
            progress(g, sc)
    return scenes


def config5(seed=5000) -> Scene:
    sc = pipe_scene(seed, 2000, 10 ** (1 / 3))
    sc.name = "pipe100x2.15-spheres2000"
    return sc


def small_pipe_scene(seed=7000, n_panels=6, n_spheres=3, arc=0.6) -> Scene:
    """A few-panel pipe section with spheres: small enough for element-wise
    oracle parity while spanning several tiles and a ragged tail."""
    rng_g = np.random.default_rng(seed)
    pipe = pipe_body(n_panels, 5.0, 1.0, arc)
    centers, rads = place_spheres(rng_g, n_spheres, 0.2, 5.0, 1.0, arc, 0.02)
    bodies = [pipe]
    for i in range(n_spheres):
        rot = _random_rotation(rng_g)
        bodies.append(sphere_body(centers[i], rads[i], rot[:, 2], rot[:, 0]))
    rng_d = np.random.default_rng(seed + 1)
    sig = [wall_density(pipe, NS, NT, rng_d)] + [sh_density(NS, NT, rng_d) for _ in range(n_spheres)]
    sc = Scene(bodies, NS, NT, np.ascontiguousarray(np.concatenate(sig)))
    sc.sphere_centers = centers
    sc.sphere_radii = rads
    sc.pipe_scale = 1.0
    sc.name = f"pipe{n_panels}-spheres{n_spheres}"
    return sc


def merge_scenes(scenes) -> Scene:
    """Several independent scenes as one batch: bodies concatenated in order,
    ``body_group[b]`` = index of the scene body b comes from (bodies of
    different groups do not interact), densities and targets concatenated
    (node ids shifted to the merged numbering).  ``group_node_offsets`` and
    ``group_target_offsets`` give each scene's slice of nodes and targets."""
    bodies, groups, sig, xs, tns, cls = [], [], [], [], [], []
    noff, toff = [0], [0]
    for g, sc in enumerate(scenes):
        bodies.extend(sc.bodies)
        groups.extend([g] * len(sc.bodies))
        sig.append(sc.sigma)
        tn = sc.tgt_node if sc.tgt_node is not None else np.arange(sc.n_nodes, dtype=np.int64)  # default: all nodes
        T = len(tn)
        xs.append(sc.x if sc.x is not None else np.zeros((T, 3)))
        tns.append(np.where(tn >= 0, tn + noff[-1], -1))
        cls.append(sc.tgt_class if sc.tgt_class is not None else np.zeros(T, np.int64))
        noff.append(noff[-1] + sc.n_nodes)
        toff.append(toff[-1] + T)
    out = Scene(bodies, scenes[0].ns, scenes[0].nt, np.ascontiguousarray(np.concatenate(sig)),
                np.ascontiguousarray(np.concatenate(xs)), np.ascontiguousarray(np.concatenate(tns)).astype(np.int64),
                np.concatenate(cls), scenes[0].class_names, "batch%d" % len(scenes))
    out.body_group = np.asarray(groups, dtype=np.int32)
    out.group_node_offsets = np.asarray(noff, dtype=np.int64)
    out.group_target_offsets = np.asarray(toff, dtype=np.int64)
    return out
