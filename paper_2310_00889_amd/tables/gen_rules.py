"""Offline generator of the precomputed quadrature tables the GPU library loads.

* theta-rules (Section 3.2.2, "fast evaluation of angular integrals"): for each
  distance bracket alpha in [2^-b, 2^-b+1), b = 1..NB, a generalised Chebyshev
  rule on the unit source circle that integrates the kernel components times
  Fourier modes e^{i l t}, l <= l0, for every target of the annulus of radii
  alpha..2 alpha around the circle point t = 0 (the annulus lies in the plane
  orthogonal to the circle there).  Kernel components: 1/R and r_a r_b/R^3
  (single layer), r_a r_b r_c/R^5 (double layer, any normal), R = |r|.
  With the target at angle 0 every component is even or odd in t, so the rule
  is built on [0, pi] for the even products (even components x cos(l t), odd
  components x sin(l t)) and mirrored: the odd products then integrate to zero
  exactly, as they must.
* log rule (Section 3.2.4, general singular s-quadrature): a generalised
  Chebyshev rule on [0,1] for p(u) log u + q(u), p, q polynomials.

Construction (Appendix B): a composite Gauss-Legendre discretisation refined
dyadically toward the singular point; the matrix A of integrand samples times
sqrt(weights); an orthonormal basis of its column space truncated at the
tolerance (SVD, compressed block by block); column-pivoted QR of U^T selects
the nodes; the weights solve the transposed-Vandermonde system sum_j u_i(y_j)
w_j = int u_i.  Double precision is used throughout (adequate above 1e-13 per
the appendix's remark for tolerances above 1e-10, verified by the tests).

Output: ``rules.bin`` next to this file, little-endian:
  header  char[8] "CSBQRUL1", int32 version, int32 NB, int32 l0, double tol
  per bracket b=1..NB: int32 m, then m doubles theta, m doubles weight
  log rule: int32 m, m doubles nodes (in (0,1)), m doubles weights
"""
from __future__ import annotations

import argparse
import os
import struct
import time

import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy.linalg import qr, solve, svd

HERE = os.path.dirname(os.path.abspath(__file__))


def composite_gl(breaks, p):
    xg, wg = leggauss(p)
    xs, ws = [], []
    for a, b in zip(breaks[:-1], breaks[1:]):
        xs.append(0.5 * (a + b) + 0.5 * (b - a) * xg)
        ws.append(0.5 * (b - a) * wg)
    return np.concatenate(xs), np.concatenate(ws)


def theta_breaks(alpha_lo, refine=1):
    """Panels on [0, pi]: uniform pi/16 panels on [pi/8, pi], then dyadic toward 0
    down to alpha_lo/8."""
    br = list(np.linspace(np.pi / 8, np.pi, 15 * refine))
    h = np.pi / 8
    while h > alpha_lo / 8:
        h /= 2
        br.insert(0, h)
    br.insert(0, 0.0)
    return np.array(sorted(set(br)))


def _components(t, d, z):
    """Even and odd kernel components at angles t (array) for the target
    (1 + d, 0, z); r = target - (cos t, sin t, 0).  X = d + 2 sin^2(t/2) avoids
    the cancellation of (1 + d) - cos t when d and t are small."""
    s = np.sin(t)
    h = np.sin(0.5 * t)
    X = d + 2 * h * h
    Y = -s
    R2 = X * X + Y * Y + z * z
    R = np.sqrt(R2)
    i1 = 1 / R
    i3 = i1 / R2
    i5 = i3 / R2
    even = [i1, X * X * i3, Y * Y * i3, i3, X * i3,
            X ** 3 * i5, X * Y * Y * i5, X * X * i5, Y * Y * i5, X * i5, i5]
    odd = [X * Y * i3, Y * i3, X * X * Y * i5, Y ** 3 * i5, X * Y * i5, Y * i5]
    return even, odd


def theta_functions(t, d, z, l0):
    even, odd = _components(t, d, z)
    cols = []
    for l in range(l0 + 1):
        cl = np.cos(l * t)
        for f in even:
            cols.append(f * cl)
        if l:
            sl = np.sin(l * t)
            for f in odd:
                cols.append(f * sl)
    return np.stack(cols, 1)


def annulus_targets(alpha_lo, nr=12, nphi=24):
    """Polar grid on the half annulus alpha_lo..2 alpha_lo (z >= 0)."""
    r = alpha_lo * (1 + (np.arange(nr) + 0.5) / nr)
    r = np.concatenate([[alpha_lo], r, [2 * alpha_lo]])
    phi = np.pi * np.arange(nphi + 1) / nphi
    R, P = np.meshgrid(r, phi, indexing="ij")
    return (R * np.cos(P)).ravel(), (R * np.sin(P)).ravel()


def compress(blocks, tol):
    """Orthonormal basis of the span of the (already sqrt(w)-scaled,
    column-normalised) blocks, truncated at singular value tol."""
    basis = None
    for B in blocks:
        M = B if basis is None else np.concatenate([basis, B], 1)
        U, S, _ = svd(M, full_matrices=False, lapack_driver="gesdd")
        k = int(np.sum(S > tol))
        basis = U[:, :k] * S[:k]
    U, S, _ = svd(basis, full_matrices=False)
    k = int(np.sum(S > tol))
    return U[:, :k]


def cheb_rule(x, w, U, m=None):
    """Nodes by pivoted QR of U^T, weights from int u_i = sum_j u_i(y_j) w_j.
    U holds u_i(x_k) sqrt(w_k m_k): the basis is orthonormal for the inner
    product with weight m (default 1); the rule integrates with weight 1."""
    if m is None:
        m = np.ones_like(w)
    n = U.shape[1]
    _, _, piv = qr(U.T, pivoting=True, mode="economic")
    sel = np.sort(piv[:n])
    b = U.T @ np.sqrt(w / m)
    V = U[sel, :]                      # u_i(y_j) sqrt(w_j m_j)
    v = solve(V.T, b)
    return x[sel], v * np.sqrt(w[sel] * m[sel])


def build_theta_rule(b, l0, tol, p=40, batch=24):
    """Rule for bracket b.  The inner product used for the compression carries
    the weight m(t) = sqrt(alpha^2 + t^2) (the Jacobian of t = alpha sinh v), so
    that a truncation at tol bounds the error relative to int |f| even for
    integrands peaked on the alpha scale."""
    alpha = 2.0 ** (-b)
    x, w = composite_gl(theta_breaks(alpha), p)
    m = np.sqrt(alpha * alpha + x * x)
    sw = np.sqrt(w * m)
    dd, z = annulus_targets(alpha)
    blocks = []
    cur = []
    for k in range(len(dd)):
        A = theta_functions(x, dd[k], z[k], l0) * sw[:, None]
        A /= np.linalg.norm(A, axis=0, keepdims=True)
        cur.append(A)
        if len(cur) == batch:
            blocks.append(np.concatenate(cur, 1))
            cur = []
    if cur:
        blocks.append(np.concatenate(cur, 1))
    U = compress(blocks, tol)
    th, om = cheb_rule(x, w, U, m)
    # mirror to the full circle
    return np.concatenate([-th[::-1], th]), np.concatenate([om[::-1], om])


def check_theta_rule(b, th, om, l0, n_test=60, seed=0):
    """Max error relative to int |f| over random targets and products."""
    rng = np.random.default_rng(seed + b)
    alpha = 2.0 ** (-b)
    x, w = composite_gl(theta_breaks(alpha, refine=2), 48)
    worst = 0.0
    for _ in range(n_test):
        r = alpha * (1 + rng.random())
        phi = 2 * np.pi * rng.random()
        dd, z = r * np.cos(phi), r * np.sin(phi)
        ev, od = _components(x, dd, z)
        evq, odq = _components(th, dd, z)
        for _ in range(4):
            l = int(rng.integers(0, l0 + 1))
            ph = rng.random() * 2 * np.pi
            k = int(rng.integers(0, len(ev) + len(od)))
            fx = (ev + od)[k]
            fq = (evq + odq)[k]
            # full-circle integral of component * cos(l t + ph): the even part
            # pairs with cos(l t), the odd part with sin(l t)
            if k < len(ev):
                ref = 2 * np.sum(w * fx * np.cos(l * x)) * np.cos(ph)
            else:
                ref = -2 * np.sum(w * fx * np.sin(l * x)) * np.sin(ph)
            got = np.sum(om * fq * np.cos(l * th + ph))
            scale = 2 * np.sum(w * np.abs(fx))
            worst = max(worst, abs(got - ref) / scale)
    return worst


def log_functions(u, K):
    """Legendre polynomials P_k(2u-1) and P_k(2u-1) log u, k < K."""
    P = np.polynomial.legendre.legvander(2 * u - 1, K - 1)
    return np.concatenate([P, P * np.log(u)[:, None]], 1)


def build_log_rule(K=16, tol=1e-15, p=30, lowest=1e-12):
    """Rule for P_k(2u-1) and P_k(2u-1) log u, k < K, on [0,1]; the dyadic
    panels stop at `lowest`, which keeps every node above ~5e-6 (K = 16) with
    all weights positive and moments exact to ~1e-15."""
    br = [1.0]
    h = 1.0
    while h > lowest:
        h /= 2
        br.insert(0, h)
    br.insert(0, 0.0)
    x, w = composite_gl(np.array(br), p)
    A = log_functions(x, K) * np.sqrt(w)[:, None]
    A /= np.linalg.norm(A, axis=0, keepdims=True)
    U = compress([A], tol)
    return cheb_rule(x, w, U)


def write_tables(path, rules, l0, tol, log_rule):
    with open(path, "wb") as f:
        f.write(b"CSBQRUL1")
        f.write(struct.pack("<iiid", 1, len(rules), l0, tol))
        for th, om in rules:
            f.write(struct.pack("<i", len(th)))
            f.write(np.asarray(th, "<f8").tobytes())
            f.write(np.asarray(om, "<f8").tobytes())
        f.write(struct.pack("<i", len(log_rule[0])))
        f.write(np.asarray(log_rule[0], "<f8").tobytes())
        f.write(np.asarray(log_rule[1], "<f8").tobytes())


def read_tables(path):
    with open(path, "rb") as f:
        assert f.read(8) == b"CSBQRUL1"
        ver, nb, l0, tol = struct.unpack("<iiid", f.read(20))
        rules = []
        for _ in range(nb):
            (m,) = struct.unpack("<i", f.read(4))
            th = np.frombuffer(f.read(8 * m), "<f8")
            om = np.frombuffer(f.read(8 * m), "<f8")
            rules.append((th, om))
        (m,) = struct.unpack("<i", f.read(4))
        xl = np.frombuffer(f.read(8 * m), "<f8")
        wl = np.frombuffer(f.read(8 * m), "<f8")
    return dict(version=ver, l0=l0, tol=tol, rules=rules, log_rule=(xl, wl))


def _one(args):
    b, l0, tol, check = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):   # one BLAS thread per worker process
        t0 = time.time()
        th, om = build_theta_rule(b, l0, tol)
        err = check_theta_rule(b, th, om, l0) if check else float("nan")
    return b, th, om, err, time.time() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nb", type=int, default=40)
    ap.add_argument("--l0", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-13)
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--out", default=os.path.join(HERE, "rules.bin"))
    ap.add_argument("--check", action="store_true")
    ap.add_argument("--log-only", action="store_true", help="keep the theta-rules of --out, rebuild the log rule")
    a = ap.parse_args()
    if a.log_only:
        old = read_tables(a.out)
        lr = build_log_rule()
        write_tables(a.out, old["rules"], old["l0"], old["tol"], lr)
        print(f"log rule: m = {len(lr[0])}; wrote {a.out}")
        return
    from multiprocessing import Pool
    work = [(b, a.l0, a.tol, a.check) for b in range(1, a.nb + 1)]
    res = {}
    with Pool(max(1, a.jobs)) as pool:
        for b, th, om, err, dt in pool.imap_unordered(_one, work):
            print(f"bracket {b:2d}: m0 = {len(th):3d}  ({dt:.1f}s)  check err {err:.2e}", flush=True)
            res[b] = (th, om)
    rules = [res[b] for b in range(1, a.nb + 1)]
    lr = build_log_rule()
    print(f"log rule: m = {len(lr[0])}", flush=True)
    write_tables(a.out, rules, a.l0, a.tol, lr)
    print("wrote", a.out)


if __name__ == "__main__":
    main()
