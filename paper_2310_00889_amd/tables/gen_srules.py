"""Offline generator of the whole-element singular s-rules.

Section 3.2.4 (second part) and Appendix B: for an on-surface target at the
i-th Gauss-Legendre node of an element, one generalised Chebyshev rule in s
covers the whole element, in place of dyadic panels refined toward the target
plus log-singular panels on its two sides.  A rule is built per target index
i (0..NS-1) and per aspect bracket [beta, 2 beta), beta = 2^b, from the
integrands of straight circular cylinders whose length-to-radius ratio A
samples the bracket (21 ratios, both ends included).

Integrand family, on the element variable v in [-1, 1] with the target at
v_i = x_i (the GL node), on a straight cylinder of unit radius and length A
(so a v-distance dv is an axial distance dz = A dv / 2), target at angle 0:
    r = (1 - cos t, -sin t, dz),  R^2 = 2 (1 - cos t) + dz^2,  r.n = cos t - 1
  * modal Green's functions of the kernel components, over the full circle:
      even in t (times cos l t): 1/R, r_a r_b / R^3 for ab = xx, yy, zz, xz,
                                  (r.n) r_a r_b / R^5 for ab = xx, yy, zz, xz;
      odd in t (times sin l t):  r_a r_b / R^3 and (r.n) r_a r_b / R^5 for
                                  ab = xy, yz;
    l = 0..L0 (L0 = 18: the density's band 16 plus two modes for the
    angular variation of a curved element's Jacobian); every Stokes and
    Laplace single- and double-layer component is a combination of these;
  * each times the Legendre polynomials P_p(v), p < NP (NP = 20: the
    density's degree 15 plus the smooth variation of a curved element's
    geometry along s).

Construction (Appendix B):
  * reference rule: composite Gauss-Legendre panels refined dyadically toward
    the target from both sides, down to 1/(4 beta L0) in v (where every mode
    is in its logarithmic regime), and the generalised Chebyshev log rule
    (p(u) log u + q(u)) on the two innermost panels.  Nodes are kept as
    offsets d = v - x_i so that nodes 1e-16 from the target keep their
    relative accuracy;
  * the integrand samples times sqrt(w m), m(d) = sqrt(beta^-2 + d^2) (the
    inner product weight that makes an L2 truncation bound the error relative
    to the integral of |f| for integrands peaked on the 1/beta scale);
  * every integrand is scaled by the norm of the same polynomial times the
    mode-0 1/R function at that ratio, the largest of the family (|every
    component| <= 1/R), so the truncation at tol is relative to the size of
    the element's potential, and integrands that are tiny (high modes of
    small components) do not enter at their own rounding level;
  * truncated SVD basis (compressed block by block), column-pivoted QR of its
    transpose for the nodes, the transposed-Vandermonde solve for the weights.

Sphere family.  A sphere given as one element in its polar-angle
parametrisation (x_c = c + a cos(pi t) axis, eps = a sin(pi t), t = (v+1)/2,
constant e1; both evaluators use the degree-15 interpolant of these samples)
is one shape up to a similarity, so its on-surface s-integrands are exactly
the modal Green's functions of that one surface of revolution times its
Jacobian times the density's polynomials: one rule per target index, built
from that family with the same construction (the closed ends need no special
treatment: the surface is smooth there).  The same routine evaluates both
families: for a surface of revolution with radius E(v) and axial position
z(v), target at (E0, 0, z0) and r = x0 - y(v, t),
    X = (E0 - E) + 2 E sin^2(t/2),  Y = -E sin t,  Z = z0 - z,
    r.n = (z' ((E0 - E) - 2 E0 sin^2(t/2)) - Z E') / sqrt(z'^2 + E'^2),
    J = E sqrt(z'^2 + E'^2),
with E0 - E and z0 - z formed from sample differences (barycentric form)
so that they keep their relative accuracy next to the target.

Output: ``srules.bin`` next to this file, little-endian:
  header  char[8] "CSBQSRL2", int32 version, int32 NS, int32 b_lo, int32 nb,
          int32 n_sphere (0 or 1), int32 L0, int32 NP, double tol
  per bracket b = b_lo .. b_lo + nb - 1, per target index i = 0..NS-1, then
  (n_sphere = 1) per target index of the sphere:
          int32 m, m doubles d (node offsets from x_i, ascending), m doubles w
          (weights for the integral over v in [-1, 1])
"""
from __future__ import annotations

import argparse
import os
import struct
import time

import numpy as np
from numpy.polynomial.legendre import leggauss, legvander

from gen_rules import build_log_rule, cheb_rule, compress

HERE = os.path.dirname(os.path.abspath(__file__))
NS = 16
L0 = 18
NP = 20
N_ASPECT = 20


def fine_rule(i, beta, log_rule, p=16, depth=4.0):
    """Offsets d and weights of the reference rule on [-1 - x_i, 1 - x_i]:
    GL-p panels [h/2, h] on each side, h halving from the side's length down
    to 1/(depth beta L0), then the log rule on [0, h]."""
    xi = leggauss(NS)[0][i]
    xg, wg = leggauss(p)
    lx, lw = log_rule
    hmin = 1.0 / (depth * beta * L0)
    ds, ws = [], []
    for side in (-1.0, 1.0):
        h = (1.0 + xi) if side < 0 else (1.0 - xi)
        while h > hmin:
            ds.append(side * (0.75 * h + 0.25 * h * xg))
            ws.append(0.25 * h * wg)
            h *= 0.5
        ds.append(side * h * lx)
        ws.append(h * lw)
    d = np.concatenate(ds)
    w = np.concatenate(ws)
    o = np.argsort(d)
    return xi, d[o], w[o]


def theta_rule(dz_min, p=20):
    """Composite GL on [0, pi]: eight panels on [pi/8, pi], then dyadic panels
    toward 0 down to dz_min/8 (the modal integrand's peak at t = 0 has width
    ~dz)."""
    br = list(np.linspace(np.pi / 8, np.pi, 8))
    h = np.pi / 8
    while h > dz_min / 8:
        h *= 0.5
        br.insert(0, h)
    br.insert(0, 0.0)
    br = np.array(br)
    xg, wg = leggauss(p)
    a, b = br[:-1, None], br[1:, None]
    return (0.5 * (a + b) + 0.5 * (b - a) * xg).ravel(), (0.5 * (b - a) * wg).ravel()


def modal_functions(dz, l0=L0):
    """The straight cylinder's modal Green's functions (unit radius) at
    axial offsets dz: (len(dz), 13 (l0 + 1)), component-major (9 even
    components x modes 0..l0, then 4 odd components x modes 0..l0; an odd
    component's mode-0 column is zero)."""
    dz = np.asarray(dz, dtype=np.float64)
    one = np.ones_like(dz)
    return revolution_functions(np.zeros_like(dz), one, -dz, np.zeros_like(dz), one, 1.0, l0)


def revolution_functions(dE, E, dz, Ep, zp, E0, l0=L0):
    """Modal Green's functions, times the Jacobian E sqrt(z'^2 + E'^2), of a
    surface of revolution for the target (E0, 0, z0): circles of radius E at
    axial offsets z - z0 = dz from the target, dE = E0 - E, with derivatives
    Ep = E', zp = z' in the element variable.  Layout of modal_functions."""
    out = np.zeros((len(E), 13 * (l0 + 1)))
    Z = -np.asarray(dz, dtype=np.float64)
    sp = np.sqrt(zp * zp + Ep * Ep)
    J = E * sp
    dist = np.sqrt(dE * dE + Z * Z) / E   # distance to the circle's nearest point over its radius
    lev = np.ceil(np.log2(np.pi / np.maximum(dist, 1e-300))).clip(0, 200).astype(int)
    ll = np.arange(l0 + 1)
    for L in np.unique(lev):
        idx = np.nonzero(lev == L)[0]
        t, w = theta_rule(dist[idx].min())
        h2 = (2.0 * np.sin(0.5 * t) ** 2)[None, :]
        st = np.sin(t)[None, :]
        Ei = E[idx][:, None]
        X = dE[idx][:, None] + Ei * h2
        Y = -Ei * st
        Zi = Z[idx][:, None]
        R2 = X * X + Y * Y + Zi * Zi
        i1 = J[idx][:, None] / np.sqrt(R2)
        i3 = i1 / R2
        i5 = i3 / R2
        rn = (zp[idx][:, None] * (dE[idx][:, None] - E0 * h2) - Zi * Ep[idx][:, None]) / sp[idx][:, None]
        even = [i1, X * X * i3, Y * Y * i3, Zi * Zi * i3, X * Zi * i3,
                rn * X * X * i5, rn * Y * Y * i5, rn * Zi * Zi * i5, rn * X * Zi * i5]
        odd = [X * Y * i3, Y * Zi * i3, rn * X * Y * i5, rn * Y * Zi * i5]
        C = 2.0 * np.cos(np.outer(t, ll)) * w[:, None]   # full circle: twice [0, pi]
        S = 2.0 * np.sin(np.outer(t, ll)) * w[:, None]
        out[idx] = np.concatenate([f @ C for f in even] + [f @ S for f in odd], 1)
    return out


def _bary(i, d):
    """Lagrange basis of the NS GL nodes at x_i + d (rows), from the offsets
    (x_i + d) - x_j = d - (x_j - x_i), exact at d = 0 (row = unit vector)."""
    x, _ = leggauss(NS)
    lam = np.array([1.0 / np.prod([x[j] - x[k] for k in range(NS) if k != j]) for j in range(NS)])
    off = d[:, None] - (x[None, :] - x[i])
    with np.errstate(divide="ignore"):
        q = lam[None, :] / off
    q = q / q.sum(1, keepdims=True)
    return q


def sphere_geometry(i, d):
    """Unit sphere element, polar-angle parametrisation, interpolated at the
    NS GL nodes: E0 - E, E, z - z0, E', z' at the offsets d from node i."""
    x, _ = leggauss(NS)
    tt = np.pi * 0.5 * (x + 1.0)
    Es, zs = np.sin(tt), np.cos(tt)
    B = _bary(i, d)
    dE = (B * (Es[i] - Es)[None, :]).sum(1)          # E0 - E
    dz = (B * (zs - zs[i])[None, :]).sum(1)          # z - z0
    cE = np.polynomial.legendre.legfit(x, Es, NS - 1)
    cz = np.polynomial.legendre.legfit(x, zs, NS - 1)
    v = x[i] + d
    Ep = np.polynomial.legendre.legval(v, np.polynomial.legendre.legder(cE))
    zp = np.polynomial.legendre.legval(v, np.polynomial.legendre.legder(cz))
    return dE, Es[i] - dE, dz, Ep, zp, Es[i]


def sphere_scale(i):
    """v-distance over which the sphere's circles near the target stay within
    one radius: E0 / |dx/dv| at the target."""
    x, _ = leggauss(NS)
    t = np.pi * 0.5 * (x[i] + 1.0)
    return np.sin(t) / (0.5 * np.pi)


def _rule_from_family(d, w, m, xi, families, tol):
    """App. B on the reference rule (d, w) with inner-product weight m: each
    family member's integrand G (columns) times P_p, scaled by the norm of
    |G[:, 0] P_p| (the largest member), compressed, nodes and weights."""
    sw = np.sqrt(w * m)
    Pv = legvander(xi + d, NP - 1)
    blocks = []
    for G in families:
        cols = []
        for p in range(NP):
            ref = np.linalg.norm(np.abs(G[:, 0] * Pv[:, p]) * sw)
            cols.append(G * (Pv[:, p] * sw / ref)[:, None])
        blocks.append(np.concatenate(cols, 1))
    U = compress(blocks, tol)
    return cheb_rule(d, w, U, m)


def build_rule(b, i, tol, log_rule):
    """Nodes (offsets from x_i) and weights of the rule for bracket
    [2^b, 2^(b+1)) and target index i."""
    beta = 2.0 ** b
    xi, d, w = fine_rule(i, beta, log_rule)
    m = np.sqrt(beta ** -2 + d * d)
    fams = (modal_functions(-0.5 * beta * (1.0 + k / N_ASPECT) * d) for k in range(N_ASPECT + 1))
    return _rule_from_family(d, w, m, xi, fams, tol)


def build_sphere_rule(i, tol, log_rule):
    """Nodes and weights of the sphere element's rule for target index i:
    the reference rule is refined toward the target down to 1/(4 L0) of the
    scale E0/|dx/dv| (at most 1/(4 beta L0) with beta = 1/scale)."""
    sc = sphere_scale(i)
    xi, d, w = fine_rule(i, 1.0 / sc, log_rule)
    m = np.sqrt(sc * sc + d * d)
    dE, E, dz, Ep, zp, E0 = sphere_geometry(i, d)
    G = revolution_functions(dE, E, dz, Ep, zp, E0)
    return _rule_from_family(d, w, m, xi, [G], tol)


def check_sphere_rule(i, dr, wr, log_rule):
    """Largest error over every family function (every polynomial degree)
    against a finer reference rule, relative to the integral of |P_p| times
    the mode-0 1/R function."""
    sc = sphere_scale(i)
    xi, d, w = fine_rule(i, 1.0 / sc, log_rule, p=24, depth=16.0)
    G = revolution_functions(*sphere_geometry(i, d))
    Gq = revolution_functions(*sphere_geometry(i, dr))
    Pv = legvander(xi + d, NP - 1)
    Pq = legvander(xi + dr, NP - 1)
    worst = 0.0
    for p in range(NP):
        ref = (w * Pv[:, p]) @ G
        got = (wr * Pq[:, p]) @ Gq
        scale = np.sum(w * np.abs(G[:, 0] * Pv[:, p]))
        worst = max(worst, np.abs(got - ref).max() / scale)
    return worst


def check_rule(b, i, dr, wr, log_rule, n_aspect=12, seed=0):
    """Largest error over random ratios in the bracket and every family
    function (a random polynomial degree each), against a finer reference
    rule (log panels 4x deeper, GL-24 panels), relative to the integral of the
    polynomial's magnitude times the mode-0 1/R function."""
    beta = 2.0 ** b
    rng = np.random.default_rng(seed + 1000 * b + i)
    xi, d, w = fine_rule(i, beta, log_rule, p=24, depth=16.0)
    Pv = legvander(xi + d, NP - 1)
    Pq = legvander(xi + dr, NP - 1)
    worst = 0.0
    for _ in range(n_aspect):
        A = beta * (1.0 + rng.random())
        G = modal_functions(-0.5 * A * d)
        Gq = modal_functions(-0.5 * A * dr)
        for c in range(G.shape[1]):
            p = int(rng.integers(0, NP))
            ref = np.sum(w * G[:, c] * Pv[:, p])
            got = np.sum(wr * Gq[:, c] * Pq[:, p])
            scale = np.sum(w * np.abs(G[:, 0] * Pv[:, p]))
            worst = max(worst, abs(got - ref) / scale)
    return worst


def write_srules(path, b_lo, nb, tol, rules, sphere=None):
    with open(path, "wb") as f:
        f.write(b"CSBQSRL2")
        f.write(struct.pack("<iiiiiiid", 2, NS, b_lo, nb, 1 if sphere else 0, L0, NP, tol))
        sets = [rules[(b, i)] for b in range(b_lo, b_lo + nb) for i in range(NS)]
        if sphere:
            sets += [sphere[i] for i in range(NS)]
        for dr, wr in sets:
            f.write(struct.pack("<i", len(dr)))
            f.write(np.asarray(dr, "<f8").tobytes())
            f.write(np.asarray(wr, "<f8").tobytes())


def read_srules(path):
    with open(path, "rb") as f:
        magic = f.read(8)
        if magic == b"CSBQSRL1":
            ver, ns, b_lo, nb, l0, npoly, tol = struct.unpack("<iiiiiid", f.read(32))
            nsph = 0
        else:
            assert magic == b"CSBQSRL2"
            ver, ns, b_lo, nb, nsph, l0, npoly, tol = struct.unpack("<iiiiiiid", f.read(36))

        def one():
            (m,) = struct.unpack("<i", f.read(4))
            return np.frombuffer(f.read(8 * m), "<f8"), np.frombuffer(f.read(8 * m), "<f8")

        rules = {(b, i): one() for b in range(b_lo, b_lo + nb) for i in range(ns)}
        sphere = {i: one() for i in range(ns)} if nsph else None
    return dict(version=ver, ns=ns, b_lo=b_lo, nb=nb, l0=l0, np=npoly, tol=tol, rules=rules, sphere=sphere)


def _one(args):
    b, i, tol, check = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        t0 = time.time()
        lr = build_log_rule()
        if b is None:
            dr, wr = build_sphere_rule(i, tol, lr)
            err = check_sphere_rule(i, dr, wr, lr) if check else float("nan")
        else:
            dr, wr = build_rule(b, i, tol, lr)
            err = check_rule(b, i, dr, wr, lr) if check else float("nan")
    return b, i, dr, wr, err, time.time() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--b-lo", type=int, default=2)
    ap.add_argument("--b-hi", type=int, default=30)
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--out", default=os.path.join(HERE, "srules.bin"))
    ap.add_argument("--check", action="store_true")
    ap.add_argument("--sphere-only", action="store_true",
                    help="keep the cylinder rules of --out, (re)build the sphere rules")
    a = ap.parse_args()
    from multiprocessing import Pool
    rules = {}
    b_lo, nb = a.b_lo, a.b_hi - a.b_lo + 1
    if a.sphere_only:
        old = read_srules(a.out)
        rules, b_lo, nb = old["rules"], old["b_lo"], old["nb"]
        work = []
    else:
        work = [(b, i, a.tol, a.check) for b in range(a.b_hi, a.b_lo - 1, -1) for i in range(NS)]
    work += [(None, i, a.tol, a.check) for i in range(NS)]
    sphere = {}
    with Pool(max(1, a.jobs)) as pool:
        for b, i, dr, wr, err, dt in pool.imap_unordered(_one, work):
            name = "sphere" if b is None else f"bracket 2^{b:<3d}"
            print(f"{name} i {i:2d}: m0 = {len(dr):3d}  sum|w| = {np.abs(wr).sum():.3f}  "
                  f"({dt:.1f}s)  check err {err:.2e}", flush=True)
            if b is None:
                sphere[i] = (dr, wr)
            else:
                rules[(b, i)] = (dr, wr)
    write_srules(a.out, b_lo, nb, a.tol, rules, sphere)
    print("wrote", a.out)


if __name__ == "__main__":
    main()
