"""ctypes binding of libvtx (include/vtx.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of libvtx.so.  PyTorch supplies device memory and the current
stream.  The binding raises if the library was not built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("VTX_LIB", os.path.join(HERE, "libvtx.so"))

OK, E_ARG, E_TOPOLOGY, E_CAPACITY, E_HIP, E_NONFINITE = 0, -1, -2, -3, -4, -5
CONVERGED, NOT_CONVERGED, CG_NEG_CURVATURE, CG_MAXITER = 0, 1, 2, 3
F32, F64, MIXED = 0, 1, 2
THETA_LAMBDA, THETA_P0 = 0, 1
GRAD_ADJOINT, GRAD_EP_CENTRED, GRAD_EP_FORWARD, GRAD_ADJOINT_MINRES = 0, 1, 2, 3
_METHODS = {"adjoint": GRAD_ADJOINT, "adjoint_minres": GRAD_ADJOINT_MINRES,
            "ep": GRAD_EP_CENTRED, "ep_centred": GRAD_EP_CENTRED, "ep_forward": GRAD_EP_FORWARD}
SCHED_AUTO, SCHED_PERSISTENT, SCHED_GRID, SCHED_SPLIT = -1, 0, 1, 2

_MODE_NAMES = {"f32": F32, "f64": F64, "mixed": MIXED}


class VtxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libvtx error {code}: {msg}")
        self.code = code


class _Params(C.Structure):
    _fields_ = [("KA", C.c_void_p), ("A0", C.c_void_p), ("KP", C.c_void_p), ("P0", C.c_void_p),
                ("lam", C.c_void_p), ("KA_s", C.c_double), ("A0_s", C.c_double),
                ("KP_s", C.c_double), ("P0_s", C.c_double), ("lam_s", C.c_double)]


class _RelaxOpts(C.Structure):
    _fields_ = [("eta", C.c_double), ("tol", C.c_double), ("patience", C.c_int64),
                ("max_iter", C.c_int64), ("t1_enable", C.c_int32), ("l_min", C.c_double),
                ("l_new", C.c_double), ("beta", C.c_double), ("X_target", C.c_void_p),
                ("g_lin", C.c_void_p), ("chunk", C.c_int32)]


class _RelaxResult(C.Structure):
    _fields_ = [("iters", C.c_int64), ("n_t1", C.c_int64), ("n_stretch", C.c_int64),
                ("max_f", C.c_double), ("energy", C.c_double), ("status", C.c_int32)]

    def as_dict(self):
        return dict(iters=self.iters, n_t1=self.n_t1, n_stretch=self.n_stretch,
                    max_f=self.max_f, energy=self.energy, status=self.status)


class _GradOpts(C.Structure):
    _fields_ = [("method", C.c_int32), ("theta", C.c_int32), ("cg_tol", C.c_double),
                ("cg_max_iter", C.c_int64), ("beta", C.c_double), ("ep_relax", _RelaxOpts)]


class _GradResult(C.Structure):
    _fields_ = [("cg_iters", C.c_int64), ("cg_rel_res", C.c_double), ("status", C.c_int32),
                ("ep_plus", _RelaxResult), ("ep_minus", _RelaxResult)]


_lib = None


def lib():
    """Load libvtx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2604_06896_amd/build.py "
                               "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        P = C.POINTER
        L.vtx_last_error.restype = C.c_char_p
        L.vtx_tissue_create.argtypes = [vp, i64, i64, i64, d, d, P(vp)]
        L.vtx_tissue_destroy.argtypes = [vp]
        L.vtx_tissue_sizes.argtypes = [vp, P(i64), P(i64), P(i64), P(i64)]
        L.vtx_tissue_tile_stats.argtypes = [vp, P(i64)]
        L.vtx_tissue_get_topology.argtypes = [vp, vp]
        L.vtx_tissue_set_topology.argtypes = [vp, vp]
        L.vtx_energy_forces.argtypes = [vp, i32, vp, P(_Params), vp, vp, vp, vp]
        L.vtx_energy_forces_noalloc.argtypes = [vp, i32, vp, P(_Params), vp, vp, vp, vp]
        L.vtx_cell_coeffs.argtypes = [vp, i32, vp, P(_Params), vp, vp]
        L.vtx_vertex_forces.argtypes = [vp, i32, vp, P(_Params), vp, vp, vp, vp]
        L.vtx_cell_geometry.argtypes = [vp, i32, vp, vp, vp, vp]
        L.vtx_edge_lengths.argtypes = [vp, i32, vp, vp, vp]
        L.vtx_relax.argtypes = [vp, i32, vp, P(_Params), P(_RelaxOpts), P(_RelaxResult), vp]
        L.vtx_t1.argtypes = [vp, i32, vp, P(_Params), d, d, P(i64), P(i64), vp]
        L.vtx_hvp.argtypes = [vp, i32, vp, P(_Params), vp, vp, vp]
        L.vtx_param_grad.argtypes = [vp, i32, vp, P(_Params), vp, vp, P(_GradOpts), vp,
                                     P(_GradResult), vp]
        L.vtx_v2v.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.vtx_param_sens.argtypes = [vp, i32, vp, P(_Params), vp, vp, P(_GradOpts), vp, vp,
                                     P(_GradResult), vp]
        if hasattr(L, "vtx_batch_create"):
            L.vtx_batch_autotune.argtypes = [vp, i32, P(vp), P(_Params), P(_RelaxOpts), i32,
                                             P(i32), P(i32), P(d), vp]
            L.vtx_batch_create.argtypes = [P(vp), i32, P(vp)]
            L.vtx_batch_destroy.argtypes = [vp]
            L.vtx_batch_relax.argtypes = [vp, i32, P(vp), P(_Params), P(_RelaxOpts), i32, i32,
                                          P(_RelaxResult), vp]
            L.vtx_batch_param_grad.argtypes = [vp, i32, P(vp), P(_Params), P(vp), P(vp),
                                               P(_GradOpts), P(vp), i32, P(_GradResult), vp]
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise VtxError(rc, lib().vtx_last_error().decode())


def _mode(mode):
    if isinstance(mode, str):
        return _MODE_NAMES[mode]
    return int(mode)


def pos_dtype(mode):
    return torch.float32 if _mode(mode) == F32 else torch.float64


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


@dataclasses.dataclass
class Params:
    """Mechanical parameters: each field a scalar or a device tensor with the
    element type of X (per cell: KA, A0, KP, P0; per edge: lam)."""
    KA: object = 1.0
    A0: object = 1.0
    KP: object = 1.0
    P0: object = 3.8
    lam: object = 0.0

    def to_c(self, dtype, device):
        keep = []

        def conv(v):
            if isinstance(v, torch.Tensor):
                t = v.to(device=device, dtype=dtype).contiguous()
                keep.append(t)
                return C.c_void_p(t.data_ptr()), 0.0
            if isinstance(v, np.ndarray) and v.ndim > 0:
                t = torch.as_tensor(v, dtype=dtype, device=device).contiguous()
                keep.append(t)
                return C.c_void_p(t.data_ptr()), 0.0
            return None, float(v)

        f = [conv(getattr(self, k)) for k in ("KA", "A0", "KP", "P0", "lam")]
        p = _Params(f[0][0], f[1][0], f[2][0], f[3][0], f[4][0], f[0][1], f[1][1], f[2][1],
                    f[3][1], f[4][1])
        return p, keep

    @classmethod
    def from_numpy(cls, p, device="cuda", dtype=torch.float64):
        def t(a):
            return torch.as_tensor(np.asarray(a), dtype=dtype, device=device)
        return cls(t(p.KA), t(p.A0), t(p.KP), t(p.P0), t(p.lam))


def relax_opts(eta=1e-2, tol=1e-6, patience=1, max_iter=100000, t1_enable=False, l_min=0.01,
               l_new=None, beta=0.0, X_target=None, g_lin=None, chunk=0):
    if l_new is None:
        l_new = 2.0 * l_min
    return _RelaxOpts(float(eta), float(tol), int(patience), int(max_iter), int(bool(t1_enable)),
                      float(l_min), float(l_new), float(beta), _ptr(X_target), _ptr(g_lin),
                      int(chunk))


class Tissue:
    """Handle of a periodic tissue on the current GPU (library-owned topology
    and workspaces)."""

    def __init__(self, he, n_vert, Lx, Ly, n_cell=None):
        he = np.ascontiguousarray(he, dtype=np.int32)
        if n_cell is None:
            n_cell = int(he[:, 5].max()) + 1
        h = C.c_void_p()
        _check(lib().vtx_tissue_create(he.ctypes.data_as(C.c_void_p), he.shape[0], int(n_vert),
                                       int(n_cell), float(Lx), float(Ly), C.byref(h)))
        self._h = h
        self.n_vert, self.n_cell, self.n_he = int(n_vert), int(n_cell), int(he.shape[0])
        self.n_edge = self.n_he // 2
        self.Lx, self.Ly = float(Lx), float(Ly)

    @classmethod
    def from_tissue(cls, t):
        return cls(t.he, t.n_vert, t.Lx, t.Ly)

    def close(self):
        if getattr(self, "_h", None):
            lib().vtx_tissue_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def tile_stats(self):
        """Layout of the fused evaluation's tile tables: tiles, cells listed,
        halo vertices, corner references, tiles on the global path."""
        out = (C.c_int64 * 5)()
        _check(lib().vtx_tissue_tile_stats(self._h, out))
        return dict(zip(("tiles", "cells", "halo", "corners", "global_tiles"), list(out)))

    # -------------------------------------------------------- topology
    def topology(self):
        out = np.empty((self.n_he, 8), np.int32)
        _check(lib().vtx_tissue_get_topology(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_topology(self, he):
        he = np.ascontiguousarray(he, dtype=np.int32)
        _check(lib().vtx_tissue_set_topology(self._h, he.ctypes.data_as(C.c_void_p)))

    # -------------------------------------------------------- evaluation
    def _xcheck(self, X, mode):
        m = _mode(mode)
        if X.dtype != pos_dtype(m) or not X.is_cuda or not X.is_contiguous() or \
                tuple(X.shape) != (self.n_vert, 2):
            raise ValueError(f"X must be a contiguous CUDA tensor [{self.n_vert},2] of "
                             f"{pos_dtype(m)}")
        return m

    def energy_forces(self, X, params, mode="f64", want_energy=True, want_forces=True,
                      want_maxf=False):
        m = self._xcheck(X, mode)
        p, keep = params.to_c(X.dtype, X.device)
        E = torch.empty((), dtype=torch.float64, device=X.device) if want_energy else None
        F = torch.empty_like(X) if want_forces else None
        mf = torch.empty((), dtype=torch.float64, device=X.device) if want_maxf else None
        _check(lib().vtx_energy_forces(self._h, m, _ptr(X), C.byref(p), _ptr(E), _ptr(F),
                                       _ptr(mf), _stream()))
        return E, F, mf

    def energy_forces_into(self, X, c_params, E, F, maxf=None, mode="f32"):
        """Low-overhead variant for timing loops: parameters already marshalled."""
        _check(lib().vtx_energy_forces(self._h, _mode(mode), _ptr(X), C.byref(c_params), _ptr(E),
                                       _ptr(F), _ptr(maxf), _stream()))

    def cell_coeffs(self, X, params, mode="f64"):
        """Per-cell (cA, cP) = (2K_A(A-A0), 2K_P(P-P0))."""
        m = self._xcheck(X, mode)
        p, keep = params.to_c(X.dtype, X.device)
        dt = torch.float64 if m == F64 else torch.float32
        out = torch.empty((self.n_cell, 2), dtype=dt, device=X.device)
        _check(lib().vtx_cell_coeffs(self._h, m, _ptr(X), C.byref(p), _ptr(out), _stream()))
        return out

    def vertex_forces(self, X, params, coeffs, mode="f64", want_maxf=False):
        m = self._xcheck(X, mode)
        p, keep = params.to_c(X.dtype, X.device)
        F = torch.empty_like(X)
        mf = torch.empty((), dtype=torch.float64, device=X.device) if want_maxf else None
        _check(lib().vtx_vertex_forces(self._h, m, _ptr(X), C.byref(p), _ptr(coeffs), _ptr(F),
                                       _ptr(mf), _stream()))
        return F, mf

    def vertex_forces_into(self, X, c_params, coeffs, F, mode="f32"):
        _check(lib().vtx_vertex_forces(self._h, _mode(mode), _ptr(X), C.byref(c_params),
                                       _ptr(coeffs), _ptr(F), None, _stream()))

    def cell_geometry(self, X, mode="f64"):
        m = self._xcheck(X, mode)
        A = torch.empty(self.n_cell, dtype=torch.float64, device=X.device)
        P = torch.empty_like(A)
        _check(lib().vtx_cell_geometry(self._h, m, _ptr(X), _ptr(A), _ptr(P), _stream()))
        return A, P

    def edge_lengths(self, X, mode="f64"):
        m = self._xcheck(X, mode)
        out = torch.empty(self.n_edge, dtype=torch.float64, device=X.device)
        _check(lib().vtx_edge_lengths(self._h, m, _ptr(X), _ptr(out), _stream()))
        return out

    def relax(self, X, params, mode="f64", **opts):
        """Relax X in place; returns the result dict."""
        m = self._xcheck(X, mode)
        p, keep = params.to_c(X.dtype, X.device)
        o = relax_opts(**opts)
        r = _RelaxResult()
        _check(lib().vtx_relax(self._h, m, _ptr(X), C.byref(p), C.byref(o), C.byref(r),
                               _stream()))
        return r.as_dict()

    def t1(self, X, params, l_min, l_new=None, mode="f64"):
        m = self._xcheck(X, mode)
        if l_new is None:
            l_new = 2.0 * l_min
        p, keep = params.to_c(X.dtype, X.device)
        a, b = C.c_int64(0), C.c_int64(0)
        _check(lib().vtx_t1(self._h, m, _ptr(X), C.byref(p), float(l_min), float(l_new),
                            C.byref(a), C.byref(b), _stream()))
        return a.value, b.value

    def hvp(self, X, params, v, mode="f64"):
        m = self._xcheck(X, mode)
        p, keep = params.to_c(X.dtype, X.device)
        v = v.to(dtype=torch.float64).contiguous()
        Hv = torch.empty_like(v)
        _check(lib().vtx_hvp(self._h, m, _ptr(X), C.byref(p), _ptr(v), _ptr(Hv), _stream()))
        return Hv

    def v2v(self, X, X_target, mode="f64"):
        m = self._xcheck(X, mode)
        Cst = torch.empty((), dtype=torch.float64, device=X.device)
        g = torch.empty((self.n_vert, 2), dtype=torch.float64, device=X.device)
        _check(lib().vtx_v2v(self._h, m, _ptr(X), _ptr(X_target), _ptr(Cst), _ptr(g), _stream()))
        return Cst, g

    def param_grad(self, X_star, params, dC_dX=None, X_target=None, method="adjoint",
                   theta="lambda", mode="f64", cg_tol=1e-8, cg_max_iter=100000, beta=1e-3,
                   ep_relax=None):
        m = self._xcheck(X_star, mode)
        p, keep = params.to_c(X_star.dtype, X_star.device)
        th = THETA_LAMBDA if theta == "lambda" else THETA_P0
        meth = _METHODS[method]
        n = self.n_edge if th == THETA_LAMBDA else self.n_cell
        out = torch.empty(n, dtype=torch.float64, device=X_star.device)
        if dC_dX is not None:
            dC_dX = dC_dX.to(dtype=torch.float64).contiguous()
            keep.append(dC_dX)
        ro = relax_opts(**(ep_relax or {}))
        o = _GradOpts(meth, th, float(cg_tol), int(cg_max_iter), float(beta), ro)
        r = _GradResult()
        _check(lib().vtx_param_grad(self._h, m, _ptr(X_star), C.byref(p), _ptr(dC_dX),
                                    _ptr(X_target), C.byref(o), _ptr(out), C.byref(r), _stream()))
        info = dict(cg_iters=r.cg_iters, cg_rel_res=r.cg_rel_res, status=r.status,
                    ep_plus=r.ep_plus.as_dict(), ep_minus=r.ep_minus.as_dict())
        return out, info

    def param_sens(self, X_star, params, d, dC_dX, theta="lambda", mode="f64", cg_tol=1e-8,
                   cg_max_iter=100000, want_dX=False, solver="cg"):
        """Forward implicit differentiation along the parameter direction d:
        returns (dC_dX . dX*/dtheta . d  as a 0-d device tensor,
        dX*/dtheta . d or None, info)."""
        m = self._xcheck(X_star, mode)
        p, keep = params.to_c(X_star.dtype, X_star.device)
        th = THETA_LAMBDA if theta == "lambda" else THETA_P0
        d = d.to(device=X_star.device, dtype=torch.float64).contiguous()
        dC_dX = dC_dX.to(device=X_star.device, dtype=torch.float64).contiguous()
        if d.numel() != (self.n_edge if th == THETA_LAMBDA else self.n_cell):
            raise ValueError("d has the wrong length for theta")
        out = torch.empty((), dtype=torch.float64, device=X_star.device)
        w = torch.empty((self.n_vert, 2), dtype=torch.float64, device=X_star.device) \
            if want_dX else None
        meth = GRAD_ADJOINT_MINRES if solver == "minres" else GRAD_ADJOINT
        o = _GradOpts(meth, th, float(cg_tol), int(cg_max_iter), 0.0, relax_opts())
        r = _GradResult()
        _check(lib().vtx_param_sens(self._h, m, _ptr(X_star), C.byref(p), _ptr(d), _ptr(dC_dX),
                                    C.byref(o), _ptr(out), _ptr(w), C.byref(r), _stream()))
        return out, w, dict(cg_iters=r.cg_iters, cg_rel_res=r.cg_rel_res, status=r.status)


class Batch:
    """Group of tissues relaxed together in one persistent launch."""

    def __init__(self, tissues):
        self.tissues = list(tissues)
        arr = (C.c_void_p * len(self.tissues))(*[t.handle for t in self.tissues])
        h = C.c_void_p()
        _check(lib().vtx_batch_create(arr, len(self.tissues), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().vtx_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _marshal(self, Xs, params_list, m):
        n = len(self.tissues)
        assert len(Xs) == n and len(params_list) == n
        keep = []
        cps = (_Params * n)()
        for k, (X, pr) in enumerate(zip(Xs, params_list)):
            if X.dtype != pos_dtype(m) or not X.is_contiguous():
                raise ValueError("bad X dtype/layout")
            cp, kp = pr.to_c(X.dtype, X.device)
            keep.append(kp)
            cps[k] = cp
        xs = (C.c_void_p * n)(*[X.data_ptr() for X in Xs])
        return xs, cps, keep

    def relax(self, Xs, params_list, mode="mixed", schedule=SCHED_PERSISTENT, block_threads=0,
              **opts):
        """schedule: SCHED_PERSISTENT (one workgroup of `block_threads` per
        tissue: 256, 512 or 1024, or 0 to let the library choose, which takes
        the LDS-resident kernel when every tissue fits it), SCHED_GRID (each
        tissue in turn on the whole GPU), SCHED_SPLIT (T1 off: each tissue
        over `block_threads` = 1, 2, 4 or 8 cooperating workgroups, 0
        chooses) or SCHED_AUTO (timed trials pick one)."""
        m = _mode(mode)
        xs, cps, keep = self._marshal(Xs, params_list, m)
        o = relax_opts(**opts)
        res = (_RelaxResult * len(self.tissues))()
        _check(lib().vtx_batch_relax(self._h, m, xs, cps, C.byref(o), int(schedule),
                                     int(block_threads), res, _stream()))
        return [r.as_dict() for r in res]

    def autotune(self, Xs, params_list, mode="mixed", trial_iters=200, **opts):
        """(schedule, block_threads, projected trial times in ms for persistent
        256/512/1024, grid and split 2/4/8 (-1: not tried, T1 on)); Xs are
        not modified."""
        m = _mode(mode)
        xs, cps, keep = self._marshal(Xs, params_list, m)
        o = relax_opts(**opts)
        sch, bt = C.c_int32(), C.c_int32()
        ms = (C.c_double * 7)()
        _check(lib().vtx_batch_autotune(self._h, m, xs, cps, C.byref(o), int(trial_iters),
                                        C.byref(sch), C.byref(bt), ms, _stream()))
        return sch.value, bt.value, list(ms)

    def param_grad(self, Xs, params_list, dC_dX=None, X_target=None, method="adjoint",
                   theta="lambda", mode="f64", cg_tol=1e-8, cg_max_iter=100000, beta=1e-3,
                   ep_relax=None, block_threads=0):
        """Hypergradients of every tissue in one batched launch sequence
        (one workgroup of `block_threads` per tissue: 256, 512 or 1024, or 0
        to let the library choose; for CG on tissues of up to 1024 cells it
        takes 512 threads, which keep each solve's topology and vectors in
        LDS and registers; -K splits each tissue over K = 1, 2, 4 or 8
        cooperating workgroups: FP64 CG, or the nudged relaxations of EP)."""
        m = _mode(mode)
        n = len(self.tissues)
        keep = []
        cps = (_Params * n)()
        for k, (X, pr) in enumerate(zip(Xs, params_list)):
            if X.dtype != pos_dtype(m) or not X.is_contiguous():
                raise ValueError("bad X dtype/layout")
            cp, kp = pr.to_c(X.dtype, X.device)
            keep.append(kp)
            cps[k] = cp
        th = THETA_LAMBDA if theta == "lambda" else THETA_P0
        outs = [torch.empty(t.n_edge if th == THETA_LAMBDA else t.n_cell, dtype=torch.float64,
                            device=X.device) for t, X in zip(self.tissues, Xs)]
        xs = (C.c_void_p * n)(*[X.data_ptr() for X in Xs])
        gs = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        db = None
        if dC_dX is not None:
            dC_dX = [d.to(dtype=torch.float64).contiguous() for d in dC_dX]
            keep.append(dC_dX)
            db = (C.c_void_p * n)(*[d.data_ptr() for d in dC_dX])
        xt = None
        if X_target is not None:
            xt = (C.c_void_p * n)(*[x.data_ptr() for x in X_target])
        meth = _METHODS[method]
        ro = relax_opts(**(ep_relax or {}))
        o = _GradOpts(meth, th, float(cg_tol), int(cg_max_iter), float(beta), ro)
        res = (_GradResult * n)()
        _check(lib().vtx_batch_param_grad(self._h, m, xs, cps, db, xt, C.byref(o), gs,
                                          int(block_threads), res, _stream()))
        infos = [dict(cg_iters=r.cg_iters, cg_rel_res=r.cg_rel_res, status=r.status,
                      ep_plus=r.ep_plus.as_dict(), ep_minus=r.ep_minus.as_dict()) for r in res]
        return outs, infos
