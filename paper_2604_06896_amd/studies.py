"""Workflows built on the hot path.

rigidity_sweep: forward simulations across the target shape factor p0
(Results, the solid-to-fluid rigidity transition used for tissue
fluidisation inference): for each p0, a batch of random periodic Voronoi
tissues of n_cell cells (L = sqrt(n_cell), K_A = A0 = K_P = 1, no line
tension) is relaxed with T1 exchanges in one persistent launch; a tissue
whose relaxed energy per cell is below `e_tol` counts as a zero-energy
(fluid) state, and a logistic curve 1 / (1 + exp(-(p0 - p_c) / w)) is fitted
to the fractions.

bilevel_fit: the outer loop of the bilevel problem (Methods, "Bilevel
optimization"): theta_{k+1} = ADAM(theta_k, grad_theta C, lr), with X*(theta)
from the inner relaxation and grad_theta C from the library's hypergradient
(adjoint ID, Sen-ID is not used here, or EP) through the autograd op.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import tissue_gen as g
from . import vtx as V
from .autograd import equilibrium


def _logistic(x, pc, w):
    from scipy.special import expit
    return expit((np.asarray(x, dtype=np.float64) - pc) / w)


def fit_logistic(p0, frac):
    """Least-squares logistic fit (p_c, w) to fractions in [0, 1], with p_c
    inside the sampled range and the width between 1e-3 and the range (a
    step between two grid points then fits at the smallest width instead
    of running off to zero)."""
    from scipy.optimize import least_squares
    p0 = np.asarray(p0, dtype=np.float64)
    frac = np.asarray(frac, dtype=np.float64)
    lo, hi = float(p0.min()), float(p0.max())
    span = max(hi - lo, 1e-3)
    k = int(np.argmin(np.abs(frac - 0.5)))
    r = least_squares(lambda q: _logistic(p0, q[0], q[1]) - frac,
                      x0=(min(max(p0[k], lo), hi), min(0.02, span)),
                      bounds=([lo, 1e-3], [hi, span]), method="trf")
    if not r.success:
        return float("nan"), float("nan")
    return float(r.x[0]), float(r.x[1])


def rigidity_sweep(p0_grid=None, n_per_p0=100, n_cell=100, seed=601, e_tol=1e-6,
                   eta=1e-2, tol=1e-6, max_iter=300000, l_min=0.01, mode="mixed",
                   block_threads=0, log=print):
    if p0_grid is None:
        p0_grid = np.round(np.linspace(3.6, 4.1, 11), 4)
    rng = np.random.default_rng(seed)
    L = float(np.sqrt(n_cell))
    dt = V.pos_dtype(mode)
    out = {"p0": [], "fraction_zero_energy": [], "energy_per_cell_median": [],
           "converged": [], "batch_s": [], "energy_per_cell": []}
    for p0 in p0_grid:
        ts = [g.random_tissue(n_cell, L, rng=rng) for _ in range(n_per_p0)]
        Ts = [V.Tissue.from_tissue(t) for t in ts]
        Xs = [torch.as_tensor(t.X, dtype=dt, device="cuda") for t in ts]
        P = V.Params(KA=1.0, A0=1.0, KP=1.0, P0=float(p0), lam=0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = V.Batch(Ts).relax(Xs, [P] * n_per_p0, mode=mode, block_threads=block_threads,
                                eta=eta, tol=tol, max_iter=max_iter, t1_enable=True, l_min=l_min)
        torch.cuda.synchronize()
        dtb = time.perf_counter() - t0
        e = np.array([r["energy"] for r in res]) / n_cell
        frac = float((e < e_tol).mean())
        conv = int(sum(r["status"] == 0 for r in res))
        log(f"rigidity sweep: p0 = {p0:.3f}: zero-energy fraction {frac:.2f}, "
            f"median E/N {np.median(e):.2e}, {conv}/{n_per_p0} converged, {dtb:.2f}s")
        out["p0"].append(float(p0))
        out["fraction_zero_energy"].append(frac)
        out["energy_per_cell_median"].append(float(np.median(e)))
        out["converged"].append(conv)
        out["batch_s"].append(dtb)
        out["energy_per_cell"].append([float(x) for x in e])
    pc, w = fit_logistic(out["p0"], out["fraction_zero_energy"])
    out["fit_p_c"], out["fit_width"] = pc, w
    log(f"rigidity sweep: logistic fit p_c = {pc:.4f}, width {w:.4f}")
    return out


def bilevel_fit(n_cell=20, seed=701, epochs=300, lr=1e-3, p0_mean=3.75, p0_sd=0.05,
                method="adjoint", inner=None, grad=None, log=print):
    """Recover per-cell shape factors theta = p0 from a target equilibrium.

    Ground truth and the initial guess are drawn from the same prior
    N(p0_mean, p0_sd^2) (the prior's parameters are a choice: the paper does
    not state them).  Inner relaxation: gradient descent with the given
    options (defaults: the paper's benchmark settings, eta 1e-2, at most 1e3
    iterations, tolerance 1e-3, patience 10, T1 below 5e-3), warm-started at
    the previous equilibrium.  Outer cost: v2v to the target vertices.
    Returns per-epoch cost, mean relative L1 error and Pearson correlation,
    and theta before the first and after every epoch."""
    rng = np.random.default_rng(seed)
    t = g.random_tissue(n_cell, float(np.sqrt(n_cell)), rng=rng)
    theta_star = rng.normal(p0_mean, p0_sd, n_cell)
    theta0 = rng.normal(p0_mean, p0_sd, n_cell)
    inner = dict(eta=1e-2, tol=1e-3, patience=10, max_iter=1000, t1_enable=True,
                 l_min=5e-3) | (inner or {})
    grad = dict(method=method, cg_tol=1e-8) | (grad or {})
    if method != "adjoint":
        grad.pop("cg_tol", None)
    dev = "cuda"
    base = V.Params(KA=1.0, A0=1.0, KP=1.0, P0=3.75, lam=0.0)
    # target: relax the Voronoi tissue under theta*
    Tt = V.Tissue.from_tissue(t)
    Xt = torch.as_tensor(t.X, dtype=torch.float64, device=dev)
    Tt.relax(Xt, V.Params(P0=torch.as_tensor(theta_star, device=dev), lam=0.0), mode="f64",
             **inner)
    # prediction: the same tissue relaxed under theta0, then the outer loop
    T = V.Tissue.from_tissue(t)
    X = torch.as_tensor(t.X, dtype=torch.float64, device=dev)
    T.relax(X, V.Params(P0=torch.as_tensor(theta0, device=dev), lam=0.0), mode="f64", **inner)
    theta = torch.tensor(theta0, dtype=torch.float64, device=dev, requires_grad=True)
    opt = torch.optim.Adam([theta], lr=lr)
    nv = t.n_vert
    Lbox = torch.tensor([t.Lx, t.Ly], dtype=torch.float64, device=dev)
    ts = torch.as_tensor(theta_star, dtype=torch.float64, device=dev)
    hist = {"cost": [], "rel_l1": [], "pearson": [], "theta": [theta0.copy()]}
    for k in range(epochs):
        opt.zero_grad()
        Xs = equilibrium(theta, X, T, base, which="P0", mode="f64", relax=inner, grad=grad)
        d = Xs - Xt
        d = d - Lbox * torch.floor(d / Lbox + 0.5)       # minimum image
        cost = (d * d).sum() / (2 * nv)
        cost.backward()
        opt.step()
        X = Xs.detach()
        with torch.no_grad():
            rel = float(((theta - ts).abs() / ts.abs()).mean())
            th = theta - theta.mean()
            tt = ts - ts.mean()
            r = float((th * tt).sum() / (th.norm() * tt.norm()))
        hist["cost"].append(cost.item())
        hist["rel_l1"].append(rel)
        hist["pearson"].append(r)
        hist["theta"].append(theta.detach().cpu().numpy().copy())
        if log and (k % max(1, epochs // 10) == 0 or k == epochs - 1):
            log(f"bilevel fit [{method}] epoch {k}: cost {cost.item():.3e}, "
                f"rel L1 {rel:.4f}, Pearson {r:.3f}")
    return hist
