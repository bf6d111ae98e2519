"""CPU FP64 oracle of the periodic vertex model -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over vtx_oracle.c plus the two hypergradient estimators
composed from its primitives:

  * adjoint implicit differentiation: grad_theta C = d_theta C
    - (d2E/dX dtheta)^T H^-1 grad_X C (Methods, "Implicit differentiation
    (ID)"); H^-1 is applied by conjugate gradients on the zero-mean
    subspace;
  * centred equilibrium propagation: (1/beta) [dE/dtheta(X*_{+beta/2})
    - dE/dtheta(X*_{-beta/2})] with E + (+-beta/2) C relaxed from X*
    (Methods, "Equilibrium propagation (EP)").

Only tests, the smoke check and the CPU baseline of the benchmark import
this package; the library under paper_2604_06896_amd never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vtx_oracle.c")
_LIB = os.path.join(_HERE, "libvtx_oracle.so")

RELAX_CONVERGED = 0
RELAX_NOT_CONVERGED = 1
CG_CONVERGED = 0
CG_NEG_CURVATURE = 2
CG_MAXITER = 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Mesh(C.Structure):
    _fields_ = [("he", C.POINTER(C.c_int32)), ("n_he", C.c_int64), ("n_vert", C.c_int64),
                ("n_cell", C.c_int64), ("Lx", C.c_double), ("Ly", C.c_double)]


class _Par(C.Structure):
    _fields_ = [("KA", C.POINTER(C.c_double)), ("A0", C.POINTER(C.c_double)),
                ("KP", C.POINTER(C.c_double)), ("P0", C.POINTER(C.c_double)),
                ("lam", C.POINTER(C.c_double))]


class _RelaxOpts(C.Structure):
    _fields_ = [("eta", C.c_double), ("tol", C.c_double), ("patience", C.c_int64),
                ("max_iter", C.c_int64), ("t1_enable", C.c_int32), ("l_min", C.c_double),
                ("l_new", C.c_double), ("beta", C.c_double),
                ("X_target", C.POINTER(C.c_double)), ("g_lin", C.POINTER(C.c_double))]


class _RelaxOut(C.Structure):
    _fields_ = [("iters", C.c_int64), ("n_t1", C.c_int64), ("n_stretch", C.c_int64),
                ("max_f", C.c_double), ("energy", C.c_double), ("status", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER
        dp = P(C.c_double)
        mp = P(_Mesh)
        pp = P(_Par)
        L.ora_edge_index.restype = C.c_int64
        L.ora_edge_index.argtypes = [mp, P(C.c_int64), P(C.c_int64)]
        L.ora_edge_lengths.argtypes = [mp, dp, dp]
        L.ora_cells.argtypes = [mp, dp, dp, dp, P(C.c_int32)]
        L.ora_energy.restype = C.c_double
        L.ora_energy.argtypes = [mp, dp, pp]
        L.ora_energy_forces.restype = C.c_double
        L.ora_energy_forces.argtypes = [mp, dp, pp, dp]
        L.ora_hvp.argtypes = [mp, dp, pp, dp, dp]
        L.ora_mixed_lambda.argtypes = [mp, dp, dp, dp]
        L.ora_mixed_p0.argtypes = [mp, dp, pp, dp, dp]
        L.ora_v2v.restype = C.c_double
        L.ora_v2v.argtypes = [mp, dp, dp, dp]
        L.ora_t1_admissible.restype = C.c_int
        L.ora_t1_admissible.argtypes = [mp, C.c_int64]
        L.ora_t1_topology.argtypes = [mp, C.c_int64]
        L.ora_t1_pass.restype = C.c_int
        L.ora_t1_pass.argtypes = [mp, dp, pp, C.c_double, C.c_double, P(C.c_int64), P(C.c_int64)]
        L.ora_relax.restype = C.c_int
        L.ora_relax.argtypes = [mp, dp, pp, P(_RelaxOpts), P(_RelaxOut)]
        L.ora_cg.restype = C.c_int
        L.ora_cg.argtypes = [mp, dp, pp, dp, C.c_double, C.c_int64, dp, P(C.c_int64), dp]
        L.ora_minres.restype = C.c_int
        L.ora_minres.argtypes = [mp, dp, pp, dp, C.c_double, C.c_int64, dp, P(C.c_int64), dp]
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Mesh:
    """Topology (mutable int32 half-edge table) plus the periodic box."""

    def __init__(self, he, n_vert, Lx, Ly, n_cell=None):
        self.he = np.ascontiguousarray(he, dtype=np.int32).copy()
        self.n_vert = int(n_vert)
        self.n_cell = int(self.he[:, 5].max()) + 1 if n_cell is None else int(n_cell)
        self.Lx, self.Ly = float(Lx), float(Ly)

    @classmethod
    def from_tissue(cls, t):
        return cls(t.he, t.n_vert, t.Lx, t.Ly)

    @property
    def n_he(self):
        return int(self.he.shape[0])

    @property
    def n_edge(self):
        return self.n_he // 2

    def _c(self):
        return _Mesh(self.he.ctypes.data_as(C.POINTER(C.c_int32)), self.n_he, self.n_vert,
                     self.n_cell, self.Lx, self.Ly)

    def copy(self):
        return Mesh(self.he, self.n_vert, self.Lx, self.Ly, self.n_cell)


class _ParHold:
    def __init__(self, mesh, params):
        nc, ne = mesh.n_cell, mesh.n_edge
        self.KA = _f64(np.broadcast_to(params.KA, (nc,)))
        self.A0 = _f64(np.broadcast_to(params.A0, (nc,)))
        self.KP = _f64(np.broadcast_to(params.KP, (nc,)))
        self.P0 = _f64(np.broadcast_to(params.P0, (nc,)))
        self.lam = _f64(np.broadcast_to(params.lam, (ne,)))
        self.c = _Par(_dptr(self.KA), _dptr(self.A0), _dptr(self.KP), _dptr(self.P0),
                      _dptr(self.lam))


def edge_index(mesh):
    eoh = np.empty(mesh.n_he, np.int64)
    hoe = np.empty(mesh.n_edge, np.int64)
    m = mesh._c()
    lib().ora_edge_index(C.byref(m), eoh.ctypes.data_as(C.POINTER(C.c_int64)),
                         hoe.ctypes.data_as(C.POINTER(C.c_int64)))
    return eoh, hoe


def edge_lengths(mesh, X):
    X = _f64(X)
    out = np.empty(mesh.n_edge)
    m = mesh._c()
    lib().ora_edge_lengths(C.byref(m), _dptr(X), _dptr(out))
    return out


def cells(mesh, X):
    X = _f64(X)
    A = np.empty(mesh.n_cell)
    P = np.empty(mesh.n_cell)
    n = np.empty(mesh.n_cell, np.int32)
    m = mesh._c()
    lib().ora_cells(C.byref(m), _dptr(X), _dptr(A), _dptr(P), n.ctypes.data_as(C.POINTER(C.c_int32)))
    return A, P, n


def energy(mesh, X, params):
    X = _f64(X)
    ph = _ParHold(mesh, params)
    m = mesh._c()
    return lib().ora_energy(C.byref(m), _dptr(X), C.byref(ph.c))


def energy_forces(mesh, X, params):
    X = _f64(X)
    F = np.empty_like(X)
    ph = _ParHold(mesh, params)
    m = mesh._c()
    E = lib().ora_energy_forces(C.byref(m), _dptr(X), C.byref(ph.c), _dptr(F))
    return E, F


def hvp(mesh, X, params, v):
    X = _f64(X)
    v = _f64(v)
    out = np.empty_like(X)
    ph = _ParHold(mesh, params)
    m = mesh._c()
    lib().ora_hvp(C.byref(m), _dptr(X), C.byref(ph.c), _dptr(v), _dptr(out))
    return out


def mixed_lambda(mesh, X, mu):
    X, mu = _f64(X), _f64(mu)
    out = np.empty(mesh.n_edge)
    m = mesh._c()
    lib().ora_mixed_lambda(C.byref(m), _dptr(X), _dptr(mu), _dptr(out))
    return out


def mixed_p0(mesh, X, params, mu):
    X, mu = _f64(X), _f64(mu)
    out = np.empty(mesh.n_cell)
    ph = _ParHold(mesh, params)
    m = mesh._c()
    lib().ora_mixed_p0(C.byref(m), _dptr(X), C.byref(ph.c), _dptr(mu), _dptr(out))
    return out


def v2v(mesh, X, Xt):
    X, Xt = _f64(X), _f64(Xt)
    g = np.empty_like(X)
    m = mesh._c()
    c = lib().ora_v2v(C.byref(m), _dptr(X), _dptr(Xt), _dptr(g))
    return c, g


def t1_admissible(mesh, h):
    m = mesh._c()
    return bool(lib().ora_t1_admissible(C.byref(m), int(h)))


def t1_topology(mesh, h):
    """Apply the neighbour-exchange topology patch to edge of half-edge h
    (in place on mesh.he)."""
    m = mesh._c()
    lib().ora_t1_topology(C.byref(m), int(h))


def t1_pass(mesh, X, params, l_min, l_new):
    """One sequential T1 pass; mutates mesh.he and X in place."""
    assert X.dtype == np.float64 and X.flags.c_contiguous
    ph = _ParHold(mesh, params)
    a = C.c_int64(0)
    b = C.c_int64(0)
    m = mesh._c()
    lib().ora_t1_pass(C.byref(m), _dptr(X), C.byref(ph.c), float(l_min), float(l_new),
                      C.byref(a), C.byref(b))
    return a.value, b.value


def relax(mesh, X, params, eta=1e-2, tol=1e-6, patience=1, max_iter=100000,
          t1_enable=False, l_min=0.01, l_new=None, beta=0.0, X_target=None, g_lin=None):
    """Gradient-descent relaxation; mutates mesh.he (T1) and X in place.
    Returns a dict with iters, n_t1, n_stretch, max_f, energy, status."""
    assert X.dtype == np.float64 and X.flags.c_contiguous
    if l_new is None:
        l_new = 2.0 * l_min
    ph = _ParHold(mesh, params)
    Xt = None if X_target is None else _f64(X_target)
    gl = None if g_lin is None else _f64(g_lin)
    o = _RelaxOpts(float(eta), float(tol), int(patience), int(max_iter), int(bool(t1_enable)),
                   float(l_min), float(l_new), float(beta), _dptr(Xt), _dptr(gl))
    out = _RelaxOut()
    m = mesh._c()
    lib().ora_relax(C.byref(m), _dptr(X), C.byref(ph.c), C.byref(o), C.byref(out))
    return dict(iters=out.iters, n_t1=out.n_t1, n_stretch=out.n_stretch, max_f=out.max_f,
                energy=out.energy, status=out.status)


def cg(mesh, X, params, b, tol=1e-8, maxit=100000):
    X, b = _f64(X), _f64(b)
    mu = np.empty_like(X)
    it = C.c_int64(0)
    rr = C.c_double(0.0)
    ph = _ParHold(mesh, params)
    m = mesh._c()
    st = lib().ora_cg(C.byref(m), _dptr(X), C.byref(ph.c), _dptr(b), float(tol), int(maxit),
                      _dptr(mu), C.byref(it), C.byref(rr))
    return mu, dict(status=st, iters=it.value, rel_res=rr.value)


def minres(mesh, X, params, b, tol=1e-8, maxit=100000):
    X, b = _f64(X), _f64(b)
    x = np.empty_like(X)
    it = C.c_int64(0)
    rr = C.c_double(0.0)
    ph = _ParHold(mesh, params)
    m = mesh._c()
    st = lib().ora_minres(C.byref(m), _dptr(X), C.byref(ph.c), _dptr(b), float(tol), int(maxit),
                          _dptr(x), C.byref(it), C.byref(rr))
    return x, dict(status=st, iters=it.value, rel_res=rr.value)


def adjoint_grad(mesh, X, params, dC_dX, theta="lambda", tol=1e-8, maxit=100000,
                 dC_dtheta=None, solver="cg"):
    """grad_theta C = d_theta C - M^T mu,  H mu = grad_X C  (Methods, ID)."""
    mu, info = (cg if solver == "cg" else minres)(mesh, X, params, dC_dX, tol, maxit)
    if theta == "lambda":
        g = -mixed_lambda(mesh, X, mu)
    elif theta == "P0":
        g = -mixed_p0(mesh, X, params, mu)
    else:
        raise ValueError(theta)
    if dC_dtheta is not None:
        g = g + dC_dtheta
    return g, info


def ep_grad(mesh, X_star, params, X_target, beta, theta="lambda", **relax_kw):
    """Centred EP: relax E +- (beta/2) C from X*, then difference dE/dtheta.
    dE/dlambda_e = l_e;  dE/dP0_c = -2 K_P (P_c - P0_c)."""
    mp = mesh.copy()
    mm = mesh.copy()
    Xp = _f64(X_star).copy()
    Xm = _f64(X_star).copy()
    rp = relax(mp, Xp, params, beta=+0.5 * beta, X_target=X_target, **relax_kw)
    rm = relax(mm, Xm, params, beta=-0.5 * beta, X_target=X_target, **relax_kw)
    if theta == "lambda":
        g = (edge_lengths(mp, Xp) - edge_lengths(mm, Xm)) / beta
    elif theta == "P0":
        KP = np.broadcast_to(params.KP, (mesh.n_cell,))
        _, Pp, _ = cells(mp, Xp)
        _, Pm, _ = cells(mm, Xm)
        g = -2.0 * KP * (Pp - Pm) / beta
    else:
        raise ValueError(theta)
    return g, dict(plus=rp, minus=rm, X_plus=Xp, X_minus=Xm)


def ep_grad_forward(mesh, X_star, params, X_target, beta, theta="lambda", **relax_kw):
    """First-order EP (Methods, EP): relax E + beta C from X*, then
    (dE/dtheta(X_beta) - dE/dtheta(X*)) / beta; bias O(beta)."""
    mp = mesh.copy()
    Xp = _f64(X_star).copy()
    rp = relax(mp, Xp, params, beta=beta, X_target=X_target, **relax_kw)
    if theta == "lambda":
        g = (edge_lengths(mp, Xp) - edge_lengths(mesh, X_star)) / beta
    elif theta == "P0":
        KP = np.broadcast_to(params.KP, (mesh.n_cell,))
        _, Pp, _ = cells(mp, Xp)
        _, P0, _ = cells(mesh, X_star)
        g = -2.0 * KP * (Pp - P0) / beta
    else:
        raise ValueError(theta)
    return g, dict(plus=rp, X_plus=Xp)


def sens_derivative(mesh, X, params, d, dC_dX, theta="lambda", tol=1e-8, maxit=100000,
                    solver="cg"):
    """Forward implicit differentiation along a parameter direction d
    (Methods, ID): H w = -(d2E/dX dtheta) d, then dC/dtheta . d = grad_X C . w.
    The right-hand side is a force of modified parameters: for theta =
    lambda the force of tensions d alone (K_A = K_P = 0); for theta = P0
    minus the force of perimeter coefficients 2 K_P d (K_A = 0, lambda = 0,
    P0 = P(X) - d, so that 2 K_P (P - P0) = 2 K_P d)."""
    nc, ne = mesh.n_cell, mesh.n_edge
    d = np.asarray(d, dtype=np.float64)
    q = params.copy()
    q.KA = np.zeros(nc)
    q.A0 = np.broadcast_to(params.A0, (nc,)).copy()
    if theta == "lambda":
        q.KP = np.zeros(nc)
        q.P0 = np.broadcast_to(params.P0, (nc,)).copy()
        q.lam = d.copy()
        _, rhs = energy_forces(mesh, X, q)
    elif theta == "P0":
        _, P, _ = cells(mesh, X)
        q.KP = np.broadcast_to(params.KP, (nc,)).copy()
        q.P0 = P - d
        q.lam = np.zeros(ne)
        _, F = energy_forces(mesh, X, q)
        rhs = -F
    else:
        raise ValueError(theta)
    w, info = (cg if solver == "cg" else minres)(mesh, X, params, rhs, tol, maxit)
    return float(np.sum(_f64(dC_dX) * w)), w, info
