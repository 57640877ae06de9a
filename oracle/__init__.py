"""ctypes front end of the CPU oracle (``csbq_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may use this package; the GPU library never does.  It shares
no code with the GPU path.  See the header of ``csbq_oracle.c`` for what is
computed and how.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csbq_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE arithmetic, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        lp = C.POINTER(C.c_int64)
        geo = [C.c_int, ip, ip, dp, dp, dp, dp, C.c_int, C.c_int]
        lib.oracle_nodes.argtypes = geo + [dp, dp, dp]
        lib.oracle_smooth_sum.argtypes = geo + [dp, C.c_int64, dp, lp, dp, dp, C.c_int]
        lib.oracle_eval.argtypes = geo + [dp, C.c_int64, dp, lp, dp, dp, C.c_double, C.c_int, C.c_int, C.c_double,
                                          C.c_int, lp]
        lib.oracle_surface_point.argtypes = geo + [dp, C.c_int, C.c_int, dp, dp, dp, dp, dp, dp]
        lib.oracle_gauss_legendre.argtypes = [C.c_int, dp, dp]
        lib.oracle_num_threads.restype = C.c_int
        lib.oracle_smooth_sum_magnitude.argtypes = geo + [dp, C.c_int64, dp, lp, dp, C.c_int]
        lib.oracle_set_kernel.argtypes = [C.c_int]
        lib.oracle_set_kernel.restype = C.c_int
        _lib = lib
    return _lib


def _p(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


def _geo_args(scene):
    f = scene.flat()
    keep = [f["n_panels"], f["normal_sign"], f["s_break"], f["xc"], f["eps"], f["e1"]]
    args = [f["n_bodies"], _p(f["n_panels"], C.c_int), _p(f["normal_sign"], C.c_int), _p(f["s_break"]),
            _p(f["xc"]), _p(f["eps"]), _p(f["e1"]), scene.ns, scene.nt]
    return args, keep


def gauss_legendre(n: int):
    lib = _load()
    x = np.zeros(n)
    w = np.zeros(n)
    lib.oracle_gauss_legendre(n, _p(x), _p(w))
    return x, w


def nodes(scene):
    """(y, normal, weight) of every surface node, as the oracle computes them."""
    lib = _load()
    args, keep = _geo_args(scene)
    n = scene.n_nodes
    y = np.zeros((n, 3))
    nr = np.zeros((n, 3))
    w = np.zeros(n)
    rc = lib.oracle_nodes(*args, _p(y), _p(nr), _p(w))
    if rc:
        raise ValueError(f"oracle_nodes failed ({rc})")
    return y, nr, w


def _targets(scene, x, tgt_node):
    if x is None and tgt_node is None:
        x, tgt_node = scene.x, scene.tgt_node
    if x is None:
        x = np.zeros((len(tgt_node), 3))
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    tn = np.ascontiguousarray(tgt_node if tgt_node is not None else -np.ones(len(x)), dtype=np.int64)
    if tn.shape != (len(x),):
        raise ValueError("tgt_node must have one entry per target")
    return x, tn


def smooth_sum(scene, sigma=None, x=None, tgt_node=None, threads=0):
    """Plain tensor-rule sum over all nodes (self term zero)."""
    lib = _load()
    args, keep = _geo_args(scene)
    sig = np.ascontiguousarray(scene.sigma if sigma is None else sigma, dtype=np.float64)
    x, tn = _targets(scene, x, tgt_node)
    usl = np.zeros((len(tn), 3))
    udl = np.zeros((len(tn), 3))
    rc = lib.oracle_smooth_sum(*args, _p(sig), len(tn), _p(x), _p(tn, C.c_int64), _p(usl), _p(udl), threads)
    if rc:
        raise ValueError(f"oracle_smooth_sum failed ({rc})")
    return usl, udl


def evaluate(scene, sigma=None, x=None, tgt_node=None, rel_tol=1e-15, force_adaptive=False, threads=0,
             far_scale=0.0, far_ns_mult=0, return_deep=False):
    """Single- and double-layer velocities (u_S, u_D), each (T, 3).

    Test knobs that weaken the far route (so that pins can show they catch
    it): far_scale scales the far test's distance, far_ns_mult replaces the
    far rule's Gauss-Legendre points per panel node.  With return_deep the
    number of adaptive cells accepted at the depth cap is returned as a third
    value."""
    lib = _load()
    args, keep = _geo_args(scene)
    sig = np.ascontiguousarray(scene.sigma if sigma is None else sigma, dtype=np.float64)
    if sig.shape != (scene.n_nodes, 3):
        raise ValueError("sigma must be (n_nodes, 3)")
    x, tn = _targets(scene, x, tgt_node)
    usl = np.zeros((len(tn), 3))
    udl = np.zeros((len(tn), 3))
    deep = np.zeros(1, np.int64)
    rc = lib.oracle_eval(*args, _p(sig), len(tn), _p(x), _p(tn, C.c_int64), _p(usl), _p(udl), float(rel_tol),
                         int(bool(force_adaptive)), int(threads), float(far_scale), int(far_ns_mult),
                         _p(deep, C.c_int64))
    if rc:
        raise ValueError(f"oracle_eval failed ({rc})")
    if return_deep:
        return usl, udl, int(deep[0])
    return usl, udl


def smooth_sum_magnitude(scene, sigma=None, x=None, tgt_node=None, threads=0):
    """Per target (T, 5): the sums of |term| of the plain tensor rule's
    single- and double-layer terms (the scale of the sums' rounding), the
    first-order change of the S and D sums per unit displacement of the
    target and of every node, and of the D sum per unit change of every
    normal (bounds, not estimates)."""
    lib = _load()
    args, keep = _geo_args(scene)
    sig = np.ascontiguousarray(scene.sigma if sigma is None else sigma, dtype=np.float64)
    x, tn = _targets(scene, x, tgt_node)
    mag = np.zeros((len(tn), 5))
    rc = lib.oracle_smooth_sum_magnitude(*args, _p(sig), len(tn), _p(x), _p(tn, C.c_int64), _p(mag), threads)
    if rc:
        raise ValueError(f"oracle_smooth_sum_magnitude failed ({rc})")
    return mag


def evaluate_laplace(scene, sigma, x=None, tgt_node=None, rel_tol=1e-15, force_adaptive=False, threads=0,
                     return_deep=False):
    """Laplace single and double layers (Section 4.1) of a scalar density
    sigma (n_nodes,): (u_S, u_D), each (T,), with u_S = int G sigma,
    u_D = int dG/dn_y sigma, G = 1/(4 pi |x - y|)."""
    lib = _load()
    sig = np.zeros((scene.n_nodes, 3))
    sig[:, 0] = np.asarray(sigma, dtype=np.float64).reshape(scene.n_nodes)
    lib.oracle_set_kernel(1)
    try:
        r = evaluate(scene, sig, x, tgt_node, rel_tol, force_adaptive, threads, return_deep=return_deep)
    finally:
        lib.oracle_set_kernel(0)
    if return_deep:
        return r[0][:, 0].copy(), r[1][:, 0].copy(), r[2]
    return r[0][:, 0].copy(), r[1][:, 0].copy()


def smooth_sum_laplace(scene, sigma, x=None, tgt_node=None, threads=0):
    """Plain tensor-rule Laplace sums (self term zero): (u_S, u_D), each (T,)."""
    lib = _load()
    sig = np.zeros((scene.n_nodes, 3))
    sig[:, 0] = np.asarray(sigma, dtype=np.float64).reshape(scene.n_nodes)
    lib.oracle_set_kernel(1)
    try:
        us, ud = smooth_sum(scene, sig, x, tgt_node, threads)
    finally:
        lib.oracle_set_kernel(0)
    return us[:, 0].copy(), ud[:, 0].copy()


def surface_point(scene, elem, s, t, sigma=None):
    """Interpolated (y, normal, J, sigma) at parameter points of one element."""
    lib = _load()
    args, keep = _geo_args(scene)
    sig = np.ascontiguousarray(scene.sigma if sigma is not None or scene.sigma is not None else
                               np.zeros((scene.n_nodes, 3)), dtype=np.float64)
    if sigma is not None:
        sig = np.ascontiguousarray(sigma, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64).ravel()
    t = np.ascontiguousarray(t, dtype=np.float64).ravel()
    n = len(s)
    y = np.zeros((n, 3))
    nr = np.zeros((n, 3))
    J = np.zeros(n)
    sg = np.zeros((n, 3))
    rc = lib.oracle_surface_point(*args, _p(sig), int(elem), n, _p(s), _p(t), _p(y), _p(nr), _p(J), _p(sg))
    if rc:
        raise ValueError(f"oracle_surface_point failed ({rc})")
    return y, nr, J, sg


def num_threads() -> int:
    return int(_load().oracle_num_threads())
