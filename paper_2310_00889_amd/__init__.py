"""MI355X (gfx950) Stokes single/double-layer potential evaluator.

Thin ctypes binding over ``libcsbq.so`` (C ABI in ``include/csbq.h``): the
binding only marshals arguments; every step of the evaluation runs in the
library's HIP kernels.  There is no CPU fallback: if the library is missing or
the device is absent, construction raises.

Arrays may be numpy arrays (host memory; calls are synchronous) or torch CUDA
tensors (device memory; work is enqueued on the context's stream, which by
default is torch's current stream).
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsbq.so")
TABLE_DIR = os.path.join(HERE, "tables")

CSBQ_HOST, CSBQ_DEVICE = 0, 1
CSBQ_FP64, CSBQ_MIXED = 0, 1
CSBQ_GATE_CRITERION, CSBQ_GATE_MLP = 0, 1
CSBQ_KERNEL_STOKES, CSBQ_KERNEL_LAPLACE = 0, 1
CSBQ_SRULE_AUTO, CSBQ_SRULE_WHOLE, CSBQ_SRULE_GENERAL = 0, 1, 2
CSBQ_FAR_AUTO, CSBQ_FAR_BASE = 0, 1
GATE_NF, GATE_NO, GATE_NW = 16, 4, 9668
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ETABLE", -5: "ESTATE", -6: "ELIMIT"}
# bits of an evaluation's flag word (csbq_flag)
FLAG_NODE_RANGE, FLAG_SRULE_LIMIT, FLAG_THETA_CLAMP = 1, 2, 4
FLAG_GROUP_RANGE, FLAG_GROUP_ORDER, FLAG_BAND = 8, 16, 32


class CsbqError(RuntimeError):
    pass


class _Options(C.Structure):
    _fields_ = [("quad_tol", C.c_double), ("precision", C.c_int32), ("gate", C.c_int32), ("device", C.c_int32),
                ("stream", C.c_void_p), ("table_dir", C.c_char_p), ("kernel", C.c_int32), ("srule", C.c_int32),
                ("far_rule", C.c_int32)]


class _SolveOptions(C.Structure):
    _fields_ = [("eta", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32), ("restart", C.c_int32)]


class _SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("rel_residual", C.c_double)]


def slender_eta(eps):
    """The slender combined-field weight 1 / (2 eps log(1/eps)) (Section 4.1);
    positive for eps < 1."""
    import math
    if not 0 < eps < 1:
        raise ValueError("the slender weight needs 0 < eps < 1")
    return 1.0 / (2.0 * eps * math.log(1.0 / eps))


_lib = None


def load_library():
    """Load libcsbq.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2310_00889_amd.build` "
                          "(there is no CPU fallback)")
    # PyTorch carries its own HIP runtime.  Loading it first makes libcsbq's
    # HIP dependency resolve to that same runtime (one runtime per process
    # shares the device, streams and pointers with torch); loaded the other way
    # round, the second runtime finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    vp, dp, ip, lp = C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p
    lib.csbq_default_options.argtypes = [C.POINTER(_Options)]
    lib.csbq_create.argtypes = [C.POINTER(_Options), C.POINTER(C.c_void_p)]
    lib.csbq_destroy.argtypes = [vp]
    lib.csbq_last_error.argtypes = [vp]
    lib.csbq_last_error.restype = C.c_char_p
    lib.csbq_set_geometry.argtypes = [vp, C.c_int32, ip, ip, dp, dp, dp, dp, C.c_int32, C.c_int32, C.c_int]
    lib.csbq_set_geometry_batch.argtypes = [vp, C.c_int32, ip, ip, ip, dp, dp, dp, dp, C.c_int32, C.c_int32, C.c_int]
    lib.csbq_num_nodes.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.csbq_get_nodes.argtypes = [vp, dp, dp, dp, C.c_int]
    lib.csbq_eval.argtypes = [vp, dp, C.c_int64, dp, lp, dp, dp, C.c_int]
    lib.csbq_eval_batch.argtypes = [vp, dp, C.c_int64, dp, lp, ip, dp, dp, C.c_int]
    lib.csbq_smooth_sum.argtypes = [vp, dp, C.c_int64, dp, lp, dp, dp, C.c_int]
    lib.csbq_smooth_sum_noalloc.argtypes = [vp, dp, C.c_int64, dp, lp, dp, dp]
    lib.csbq_stats.argtypes = [vp, C.c_char_p, C.c_int64]
    lib.csbq_plan.argtypes = [vp, dp, C.c_int64, dp, lp, ip, dp, dp, C.c_int]
    lib.csbq_plan_ex.argtypes = [vp, dp, C.c_int64, dp, lp, ip, C.c_int32, dp, dp, C.c_int]
    lib.csbq_apply.argtypes = [vp, dp, dp, dp, C.c_int]
    lib.csbq_gate_load.argtypes = [vp, dp, C.c_float]
    lib.csbq_gate_infer.argtypes = [vp, dp, C.c_int64, dp, dp, dp]
    lib.csbq_gate_grad.argtypes = [vp, dp, dp, dp, C.c_int64, dp, dp, dp]
    lib.csbq_gate_train.argtypes = [vp, dp, dp, C.c_int64, dp, C.c_int, C.c_int, C.c_float, C.c_uint64, dp, dp]
    lib.csbq_gate_dataset.argtypes = [vp, dp, C.c_int64, dp, lp, C.c_double, C.c_int64, dp, dp, dp,
                                      C.POINTER(C.c_int64)]
    lib.csbq_synchronize.argtypes = [vp]
    lib.csbq_default_solve_options.argtypes = [C.POINTER(_SolveOptions)]
    lib.csbq_solve_dirichlet.argtypes = [vp, C.POINTER(_SolveOptions), dp, dp, C.POINTER(_SolveInfo), C.c_int]
    lib.csbq_solve_mobility.argtypes = [vp, C.POINTER(_SolveOptions), dp, dp, dp, dp, dp, dp, dp,
                                        C.POINTER(_SolveInfo), C.c_int]
    lib.csbq_eval_flags.argtypes = [vp, C.POINTER(C.c_int32)]
    _lib = lib
    return lib


def _is_torch_cuda(a):
    return a is not None and type(a).__module__.startswith("torch") and getattr(a, "is_cuda", False)


def _ptr(a):
    if a is None:
        return None
    if _is_torch_cuda(a):
        return C.c_void_p(a.data_ptr())
    return C.c_void_p(a.ctypes.data)


class Evaluator:
    """One library context: geometry, quadrature tables, device buffers."""

    nc = 3   # density / output components per node / target (1 for the Laplace layers)

    def __init__(self, quad_tol=1e-12, precision="fp64", device=0, stream=None, table_dir=None, gate="criterion",
                 kernel="stokes", srule="auto", far_rule="auto"):
        """kernel: "stokes" (densities and outputs of three components per
        node / target) or "laplace" (one).  srule: the own element's s-rule
        for on-surface targets: "auto" (the whole-element singular rules on
        the shapes they were built from: straight constant-radius cylinders,
        spheres as one element; the general rule elsewhere), "whole" (also
        the cylinder rules on every other open element with a tabulated
        aspect) or "general" (dyadic panels and the log-singular rule
        everywhere).  far_rule: "auto" (for each block of targets, the
        coarsest Gauss x trapezoid rule of every element that meets quad_tol
        there by the criterion's estimates, else the element's base rule) or
        "base" (the base rules: own nodes, 32 x 32 for spheres)."""
        lib = load_library()
        opt = _Options()
        lib.csbq_default_options(C.byref(opt))
        if kernel not in ("stokes", "laplace"):
            raise CsbqError(f"unknown kernel {kernel!r}")
        srules = {"auto": CSBQ_SRULE_AUTO, "whole": CSBQ_SRULE_WHOLE, "general": CSBQ_SRULE_GENERAL}
        if srule not in srules:
            raise CsbqError(f"unknown s-rule {srule!r}")
        opt.srule = srules[srule]
        far_rules = {"auto": CSBQ_FAR_AUTO, "base": CSBQ_FAR_BASE}
        if far_rule not in far_rules:
            raise CsbqError(f"unknown far-field rule {far_rule!r}")
        opt.far_rule = far_rules[far_rule]
        opt.kernel = CSBQ_KERNEL_LAPLACE if kernel == "laplace" else CSBQ_KERNEL_STOKES
        self.nc = 1 if kernel == "laplace" else 3
        opt.quad_tol = float(quad_tol)
        opt.precision = CSBQ_MIXED if precision == "mixed" else CSBQ_FP64
        opt.gate = CSBQ_GATE_MLP if gate == "mlp" else CSBQ_GATE_CRITERION
        opt.device = int(device)
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream(device).cuda_stream
            except Exception:
                stream = None
        opt.stream = stream
        self._tdir = (table_dir or TABLE_DIR).encode()
        opt.table_dir = self._tdir
        h = C.c_void_p()
        rc = lib.csbq_create(C.byref(opt), C.byref(h))
        if rc != 0:
            raise CsbqError(f"csbq_create failed: {_STATUS.get(rc, rc)}")
        self._h = h
        self._lib = lib
        self.n_nodes = 0
        self._keep = []

    def close(self):
        if getattr(self, "_h", None):
            self._lib.csbq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != 0:
            msg = self._lib.csbq_last_error(self._h).decode(errors="replace")
            raise CsbqError(f"{what} failed ({_STATUS.get(rc, rc)}): {msg}")

    def set_geometry(self, scene):
        """Geometry from a scene (see ``synth.Scene``) or a dict of flat arrays.
        A scene with ``body_group`` (see ``synth.merge_scenes``) is a batch of
        independent geometries."""
        f = scene.flat() if hasattr(scene, "flat") else scene
        bg = getattr(scene, "body_group", None) if hasattr(scene, "flat") else f.get("body_group")
        ns = getattr(scene, "ns", 16)
        nt = getattr(scene, "nt", 32)
        arrs = dict(n_panels=np.ascontiguousarray(f["n_panels"], np.int32),
                    normal_sign=np.ascontiguousarray(f["normal_sign"], np.int32),
                    s_break=np.ascontiguousarray(f["s_break"], np.float64),
                    xc=np.ascontiguousarray(f["xc"], np.float64),
                    eps=np.ascontiguousarray(f["eps"], np.float64),
                    e1=np.ascontiguousarray(f["e1"], np.float64))
        bga = None if bg is None else np.ascontiguousarray(bg, np.int32)
        rc = self._lib.csbq_set_geometry_batch(self._h, int(f["n_bodies"]), _ptr(bga), _ptr(arrs["n_panels"]),
                                               _ptr(arrs["normal_sign"]), _ptr(arrs["s_break"]), _ptr(arrs["xc"]),
                                               _ptr(arrs["eps"]), _ptr(arrs["e1"]), ns, nt, CSBQ_HOST)
        self._check(rc, "csbq_set_geometry_batch")
        self._plan_T = None   # the library drops its plan with the geometry
        self._n_bodies = int(f["n_bodies"])
        n = C.c_int64()
        self._check(self._lib.csbq_num_nodes(self._h, C.byref(n)), "csbq_num_nodes")
        self.n_nodes = n.value

    def nodes(self):
        y = np.zeros((self.n_nodes, 3))
        nr = np.zeros((self.n_nodes, 3))
        w = np.zeros(self.n_nodes)
        self._check(self._lib.csbq_get_nodes(self._h, _ptr(y), _ptr(nr), _ptr(w), CSBQ_HOST), "csbq_get_nodes")
        return y, nr, w

    def _check_shapes(self, sigma, x, tgt_node, tgt_group, out_sl, out_dl):
        """The C ABI takes bare pointers: every size and element type is checked
        here, so that no call reads or writes past an array."""
        def _dt(a):
            return str(a.dtype).replace("torch.", "")

        def need(a, what, n, dtype):
            if a is None:
                return
            if int(np.prod(a.shape)) != n or _dt(a) != dtype:
                raise CsbqError(f"{what}: expected {n} {dtype} values, got shape {tuple(a.shape)} of {_dt(a)}")

        if tgt_node is None and x is None:
            raise CsbqError("targets: give x, tgt_node or both")
        T = int(tgt_node.shape[0] if tgt_node is not None else x.shape[0])
        need(sigma, "sigma", self.nc * self.n_nodes, "float64")
        need(x, "x", 3 * T, "float64")
        need(tgt_node, "tgt_node", T, "int64")
        need(tgt_group, "tgt_group", T, "int32")
        need(out_sl, "out_sl", self.nc * T, "float64")
        need(out_dl, "out_dl", self.nc * T, "float64")
        return T

    def _oshape(self, T):
        return (T, 3) if self.nc == 3 else (T,)

    def _call(self, fn, name, sigma, x, tgt_node, out_sl, out_dl, tgt_group=None, batch=False):
        dev = _is_torch_cuda(sigma)
        if dev:
            import torch
            T = int(tgt_node.shape[0] if tgt_node is not None else x.shape[0])
            if out_sl is None:
                out_sl = torch.empty(self._oshape(T), dtype=torch.float64, device=sigma.device)
            if out_dl is None:
                out_dl = torch.empty(self._oshape(T), dtype=torch.float64, device=sigma.device)
            for a in (sigma, x, tgt_node, tgt_group, out_sl, out_dl):
                if a is not None and not (_is_torch_cuda(a) and a.is_contiguous()):
                    raise CsbqError("device calls need contiguous CUDA tensors throughout")
            self._last_T = self._check_shapes(sigma, x, tgt_node, tgt_group, out_sl, out_dl)
            if batch:
                rc = fn(self._h, _ptr(sigma), T, _ptr(x), _ptr(tgt_node), _ptr(tgt_group), _ptr(out_sl),
                        _ptr(out_dl), CSBQ_DEVICE)
            else:
                rc = fn(self._h, _ptr(sigma), T, _ptr(x), _ptr(tgt_node), _ptr(out_sl), _ptr(out_dl), CSBQ_DEVICE)
            self._check(rc, name)
            return out_sl, out_dl
        sigma = np.ascontiguousarray(sigma, np.float64)
        if x is not None:
            x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
        if tgt_node is not None:
            tgt_node = np.ascontiguousarray(tgt_node, np.int64).reshape(-1)
        if tgt_group is not None:
            tgt_group = np.ascontiguousarray(tgt_group, np.int32).reshape(-1)
        T = self._check_shapes(sigma, x, tgt_node, tgt_group, None, None)
        self._last_T = T
        usl = np.zeros(self._oshape(T))
        udl = np.zeros(self._oshape(T))
        if batch:
            rc = fn(self._h, _ptr(sigma), T, _ptr(x), _ptr(tgt_node), _ptr(tgt_group), _ptr(usl), _ptr(udl),
                    CSBQ_HOST)
        else:
            rc = fn(self._h, _ptr(sigma), T, _ptr(x), _ptr(tgt_node), _ptr(usl), _ptr(udl), CSBQ_HOST)
        self._check(rc, name)
        return usl, udl

    def eval(self, sigma, x=None, tgt_node=None, out_sl=None, out_dl=None, tgt_group=None):
        """(u_S, u_D) at the targets: the full evaluation.  ``tgt_group`` names
        the geometry of each free target of a batch (targets ordered by group)."""
        if tgt_group is not None:
            return self._call(self._lib.csbq_eval_batch, "csbq_eval_batch", sigma, x, tgt_node, out_sl, out_dl,
                              tgt_group, batch=True)
        return self._call(self._lib.csbq_eval, "csbq_eval", sigma, x, tgt_node, out_sl, out_dl)

    def smooth_sum(self, sigma, x=None, tgt_node=None, out_sl=None, out_dl=None):
        """(u_S, u_D) of the plain smooth Nystrom sum (no corrections)."""
        return self._call(self._lib.csbq_smooth_sum, "csbq_smooth_sum", sigma, x, tgt_node, out_sl, out_dl)

    def smooth_sum_noalloc(self, sigma, x=None, tgt_node=None, out_sl=None, out_dl=None):
        """The smooth sum through the allocation-free entry point: device
        tensors only (outputs are allocated here, by torch, when not given);
        the call only enqueues work (flags via flags())."""
        import torch
        T = int(tgt_node.shape[0] if tgt_node is not None else x.shape[0])
        if out_sl is None:
            out_sl = torch.empty(self._oshape(T), dtype=torch.float64, device=sigma.device)
        if out_dl is None:
            out_dl = torch.empty(self._oshape(T), dtype=torch.float64, device=sigma.device)
        for a in (sigma, x, tgt_node, out_sl, out_dl):
            if a is not None and not (_is_torch_cuda(a) and a.is_contiguous()):
                raise CsbqError("smooth_sum_noalloc takes contiguous CUDA tensors only")
        self._check_shapes(sigma, x, tgt_node, None, out_sl, out_dl)
        self._check(self._lib.csbq_smooth_sum_noalloc(self._h, _ptr(sigma), T, _ptr(x), _ptr(tgt_node), _ptr(out_sl),
                                                      _ptr(out_dl)), "csbq_smooth_sum_noalloc")
        return out_sl, out_dl

    # ---- setup / apply split
    def plan(self, sigma, x=None, tgt_node=None, out_sl=None, out_dl=None, tgt_group=None, matrix=False,
             full_band=False):
        """Evaluate and freeze the plan (pairs, tiers, rules, smooth-sum blocks)
        for later apply() calls on the same targets.  matrix: store the
        special-quadrature pairs' correction matrices (CSBQ_PLAN_MATRIX);
        full_band: rules for any density's band (CSBQ_PLAN_FULL_BAND)."""
        self._plan_T = None
        flags = (1 if matrix else 0) | (2 if full_band else 0)
        fn = lambda h, sg, T, xx, tn, tg, us, ud, mem: self._lib.csbq_plan_ex(h, sg, T, xx, tn, tg, flags, us, ud, mem)
        out = self._call(fn, "csbq_plan_ex", sigma, x, tgt_node, out_sl, out_dl, tgt_group, batch=True)
        self._plan_T = self._last_T   # apply() writes the plan's targets, whatever is evaluated in between
        return out

    def apply(self, sigma, out_sl=None, out_dl=None):
        """(u_S, u_D) of a new density under the frozen plan (graph replay)."""
        if getattr(self, "_plan_T", None) is None:
            raise CsbqError("apply: no plan (call plan() first)")
        plan_targets = np.zeros(self._plan_T, np.int64)   # stands for the plan's targets in the size checks
        if _is_torch_cuda(sigma):
            for a in (sigma, out_sl, out_dl):
                if a is not None and not (_is_torch_cuda(a) and a.is_contiguous()):
                    raise CsbqError("device calls need contiguous CUDA tensors throughout")
            self._check_shapes(sigma, None, plan_targets, None, out_sl, out_dl)
            import torch
            T = self._plan_T
            if out_sl is None:
                out_sl = torch.empty(self._oshape(T), dtype=torch.float64, device=sigma.device)
            if out_dl is None:
                out_dl = torch.empty(self._oshape(T), dtype=torch.float64, device=sigma.device)
            self._check(self._lib.csbq_apply(self._h, _ptr(sigma), _ptr(out_sl), _ptr(out_dl), CSBQ_DEVICE),
                        "csbq_apply")
            return out_sl, out_dl
        sigma = np.ascontiguousarray(sigma, np.float64)
        self._check_shapes(sigma, None, plan_targets, None, None, None)
        usl = np.zeros(self._oshape(self._plan_T))
        udl = np.zeros(self._oshape(self._plan_T))
        self._check(self._lib.csbq_apply(self._h, _ptr(sigma), _ptr(usl), _ptr(udl), CSBQ_HOST), "csbq_apply")
        return usl, udl

    # ---- boundary-integral solves (Section 4)
    def _solve_opts(self, eta, tol, max_iter, restart):
        o = _SolveOptions()
        self._lib.csbq_default_solve_options(C.byref(o))
        o.eta, o.tol, o.max_iter, o.restart = float(eta), float(tol), int(max_iter), int(restart)
        return o

    def solve_dirichlet(self, u0, eta, tol=1e-10, max_iter=200, restart=60):
        """Density sigma of the slender combined-field Dirichlet problem
        K sigma = u0 (K = I/2 + D_4 + eta S, D_4 = -u_dl's double layer) at
        the surface nodes; returns (sigma, iterations, relative residual).
        The exterior velocity is eta u_S - u_D of eval(sigma, ...)."""
        o = self._solve_opts(eta, tol, max_iter, restart)
        info = _SolveInfo()
        if _is_torch_cuda(u0):
            import torch
            if not u0.is_contiguous() or u0.dtype != torch.float64 or u0.numel() != self.nc * self.n_nodes:
                raise CsbqError(f"u0: expected {self.nc * self.n_nodes} contiguous float64 values")
            sig = torch.empty_like(u0)
            self._check(self._lib.csbq_solve_dirichlet(self._h, C.byref(o), _ptr(u0), _ptr(sig), C.byref(info),
                                                       CSBQ_DEVICE), "csbq_solve_dirichlet")
        else:
            u = np.ascontiguousarray(u0, np.float64)
            if u.size != self.nc * self.n_nodes:
                raise CsbqError(f"u0: expected {self.nc * self.n_nodes} values, got {u.size}")
            sig = np.zeros(self._oshape(self.n_nodes))
            self._check(self._lib.csbq_solve_dirichlet(self._h, C.byref(o), _ptr(u), _ptr(sig), C.byref(info),
                                                       CSBQ_HOST), "csbq_solve_dirichlet")
        return sig, int(info.iterations), float(info.rel_residual)

    def solve_mobility(self, force, torque, eta, u_slip=None, tol=1e-10, max_iter=200, restart=60):
        """Rigid bodies under given forces and torques (n_bodies x 3 each) and
        an optional slip velocity: the slender mobility combined-field
        equation.  Returns a dict with the representation's density sigma
        ((I - L) sigma), the completion density nu, the rigid motions (V, Omega)
        per body about the centroids, the centroids, iterations and residual."""
        B = int(np.asarray(force).reshape(-1, 3).shape[0])
        f = np.ascontiguousarray(force, np.float64).reshape(-1, 3)
        t = np.ascontiguousarray(torque, np.float64).reshape(-1, 3)
        if f.shape != t.shape:
            raise CsbqError("force and torque need one row per body")
        o = self._solve_opts(eta, tol, max_iter, restart)
        info = _SolveInfo()
        rigid = np.zeros((B, 6))
        cen = np.zeros((B, 3))
        us = None if u_slip is None else np.ascontiguousarray(u_slip, np.float64)
        if us is not None and us.size != 3 * self.n_nodes:
            raise CsbqError(f"u_slip: expected {3 * self.n_nodes} values, got {us.size}")
        if B != getattr(self, "_n_bodies", B):
            raise CsbqError(f"force and torque: {B} rows for {self._n_bodies} bodies")
        sig = np.zeros((self.n_nodes, 3))
        nu = np.zeros((self.n_nodes, 3))
        self._check(self._lib.csbq_solve_mobility(self._h, C.byref(o), _ptr(f), _ptr(t), _ptr(us), _ptr(sig), _ptr(nu),
                                                  _ptr(rigid), _ptr(cen), C.byref(info), CSBQ_HOST),
                    "csbq_solve_mobility")
        return dict(sigma=sig, nu=nu, velocity=rigid[:, :3].copy(), omega=rigid[:, 3:].copy(), centers=cen,
                    iterations=int(info.iterations), rel_residual=float(info.rel_residual))

    # ---- learned gate
    def gate_load(self, weights, tau_esc=0.05):
        w = np.ascontiguousarray(weights, np.float32).reshape(GATE_NW)
        self._check(self._lib.csbq_gate_load(self._h, _ptr(w), float(tau_esc)), "csbq_gate_load")

    def gate_infer(self, feat):
        f = np.ascontiguousarray(feat, np.float32).reshape(-1, GATE_NF)
        n = f.shape[0]
        tier = np.zeros(n, np.int8)
        esc = np.zeros(n, np.uint8)
        lg = np.zeros((n, GATE_NO), np.float32)
        self._check(self._lib.csbq_gate_infer(self._h, _ptr(f), n, _ptr(tier), _ptr(esc), _ptr(lg)),
                    "csbq_gate_infer")
        return tier, esc, lg

    def gate_grad(self, weights, feat, label, posw):
        w = np.ascontiguousarray(weights, np.float32).reshape(GATE_NW)
        f = np.ascontiguousarray(feat, np.float32).reshape(-1, GATE_NF)
        lab = np.ascontiguousarray(label, np.int8).reshape(-1)
        if lab.shape[0] != f.shape[0]:
            raise CsbqError(f"gate_grad: {f.shape[0]} feature rows but {lab.shape[0]} labels")
        pw = np.ascontiguousarray(posw, np.float32).reshape(GATE_NO)
        g = np.zeros(GATE_NW, np.float32)
        loss = np.zeros(1, np.float32)
        self._check(self._lib.csbq_gate_grad(self._h, _ptr(w), _ptr(f), _ptr(lab), f.shape[0], _ptr(pw), _ptr(g),
                                             _ptr(loss)), "csbq_gate_grad")
        return g, float(loss[0])

    def gate_train(self, feat, label, posw, weights, epochs=10, batch=4096, lr=1e-3, seed=0):
        w = np.array(weights, np.float32).reshape(GATE_NW).copy()
        f = np.ascontiguousarray(feat, np.float32).reshape(-1, GATE_NF)
        lab = np.ascontiguousarray(label, np.int8).reshape(-1)
        if lab.shape[0] != f.shape[0]:
            raise CsbqError(f"gate_train: {f.shape[0]} feature rows but {lab.shape[0]} labels")
        pw = np.ascontiguousarray(posw, np.float32).reshape(GATE_NO)
        losses = np.zeros(epochs, np.float32)
        self._check(self._lib.csbq_gate_train(self._h, _ptr(f), _ptr(lab), f.shape[0], _ptr(pw), int(epochs),
                                              int(batch), float(lr), int(seed), _ptr(w), _ptr(losses)),
                    "csbq_gate_train")
        return w, losses

    def gate_dataset(self, sigma, x=None, tgt_node=None, label_tol=1e-8, cap=1 << 20):
        sigma = np.ascontiguousarray(sigma, np.float64)
        if x is not None:
            x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
        if tgt_node is not None:
            tgt_node = np.ascontiguousarray(tgt_node, np.int64).reshape(-1)
        T = self._check_shapes(sigma, x, tgt_node, None, None, None)
        feat = np.zeros((cap, GATE_NF), np.float32)
        lab = np.zeros(cap, np.int8)
        crit = np.zeros(cap, np.int8)
        n = C.c_int64()
        self._check(self._lib.csbq_gate_dataset(self._h, _ptr(sigma), T, _ptr(x), _ptr(tgt_node), float(label_tol),
                                                int(cap), _ptr(feat), _ptr(lab), _ptr(crit), C.byref(n)),
                    "csbq_gate_dataset")
        k = n.value
        return feat[:k].copy(), lab[:k].copy(), crit[:k].copy()

    def synchronize(self):
        self._check(self._lib.csbq_synchronize(self._h), "csbq_synchronize")

    def flags(self):
        """Flag word of the last evaluation (FLAG_* bits; waits for the
        stream after a device-mode call)."""
        f = C.c_int32()
        self._check(self._lib.csbq_eval_flags(self._h, C.byref(f)), "csbq_eval_flags")
        return int(f.value)

    def stats(self):
        buf = C.create_string_buffer(4096)
        self._check(self._lib.csbq_stats(self._h, buf, 4096), "csbq_stats")
        return json.loads(buf.value.decode())
