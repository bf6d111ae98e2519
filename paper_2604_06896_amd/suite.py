"""Secondary measurements (used by bench.py).

single_100 / single_10k: the single-tissue relaxations of the 100-cell
(FP64, P0 = 3.8, no line tension) and 10^4-cell (MIXED, heterogeneous P0
and lambda, T1 at 0.01) workloads to max |F| < 1e-6.

batched_relax: the 512-tissue workload (N ~ U{64..4096}, one P0 ~ U[3.6,3.9]
per tissue, lambda ~ U[0,0.2]) relaxed with T1 (l_min 0.01) towards
max |F| < 1e-6 in one persistent launch, against the single-tissue path
(captured graph chunks) on a stratified sample of the same tissues, all of
whose solves are timed.

param_gradients: tissues of 1000 cells, P0 = 3.75, hidden tensions lambda*
and initial tensions theta0 ~ U[0.05,0.15]; targets and predictions are
relaxed with T1 (batched); dC/dtheta of the v2v cost at the predictions by
the adjoint (CG tol 1e-8, FP64; also by MINRES), by centred and first-order
EP (beta = 1e-3), batched (one launch sequence for all tissues) against the
single-tissue calls, and by forward (sensitivity) ID along 8 random
directions on a sample of tissues.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import tissue_gen as g
from . import vtx as V


def _sync():
    torch.cuda.synchronize()


def single_100(log=print):
    """100 cells, FP64, K_A = A0 = K_P = 1, P0 = 3.8, lambda = 0, GD step
    1e-2 to max |F| < 1e-6: with T1 at 0.01, and without T1 for 2e5 steps
    (the tissue's edges collapse and GD keeps oscillating)."""
    t, p = g.workload_single_100()
    P = V.Params(KA=1.0, A0=1.0, KP=1.0, P0=3.8, lam=0.0)
    out = {}
    for name, t1, cap in (("with_t1", True, 2000000), ("without_t1", False, 200000)):
        T = V.Tissue.from_tissue(t)
        X = torch.as_tensor(t.X, dtype=torch.float64, device="cuda")
        _sync()
        t0 = time.perf_counter()
        r = T.relax(X, P, mode="f64", eta=1e-2, tol=1e-6, max_iter=cap, t1_enable=t1,
                    l_min=0.01)
        _sync()
        dt = time.perf_counter() - t0
        out[name] = dict(r, s=dt, steps_per_s=r["iters"] / dt, max_iter=cap)
        log(f"100 cells {name}: status {r['status']}, {r['iters']} steps, T1 {r['n_t1']}, "
            f"max|F| {r['max_f']:.2e}, {dt:.2f}s")
        if t1:
            # the same relaxation as a batch of one: the whole loop in one
            # workgroup (LDS-resident kernel) instead of three launches a step
            T2 = V.Tissue.from_tissue(t)
            X2 = torch.as_tensor(t.X, dtype=torch.float64, device="cuda")
            B = V.Batch([T2])
            _sync()
            t0 = time.perf_counter()
            rb = B.relax([X2], [P], mode="f64", eta=1e-2, tol=1e-6, max_iter=cap,
                         t1_enable=True, l_min=0.01)[0]
            _sync()
            db = time.perf_counter() - t0
            same = bool(torch.equal(X, X2)) and np.array_equal(T.topology(), T2.topology())
            out["with_t1_batch_of_one"] = dict(rb, s=db, steps_per_s=rb["iters"] / db,
                                               same_iterates_as_single=same)
            log(f"100 cells with_t1 as a batch of one: status {rb['status']}, {rb['iters']} "
                f"steps, T1 {rb['n_t1']}, {db:.2f}s, same positions and topology: {same}")
    return out


def single_10k(log=print, max_iter=1000000):
    """10^4 cells, MIXED (FP64 positions, FP32 force arithmetic), P0 ~
    U[3.6, 3.9] per cell, lambda ~ N(0.1, 0.02^2) clipped at 0, T1 below
    0.01, GD step 3e-3 to max |F| < 1e-6."""
    t, p = g.workload_single_10k()
    T = V.Tissue.from_tissue(t)
    X = torch.as_tensor(t.X, dtype=torch.float64, device="cuda")
    _sync()
    t0 = time.perf_counter()
    r = T.relax(X, V.Params.from_numpy(p), mode="mixed", eta=3e-3, tol=1e-6, max_iter=max_iter,
                t1_enable=True, l_min=0.01)
    _sync()
    dt = time.perf_counter() - t0
    log(f"1e4 cells: status {r['status']}, {r['iters']} steps, T1 {r['n_t1']}, stretches "
        f"{r['n_stretch']}, max|F| {r['max_f']:.2e}, {dt:.2f}s")
    return dict(r, s=dt, steps_per_s=r["iters"] / dt, max_iter=max_iter)


def _stratified(work, k):
    """Indices of k tissues spread over the size range and the P0 range:
    sorted by size, one tissue per size stratum, alternating the lower and
    upper P0 half of the stratum."""
    sizes = np.array([t.n_cell for t, _ in work])
    p0 = np.array([float(p.P0[0]) for _, p in work])
    order = np.argsort(sizes, kind="stable")
    picks = []
    for j, chunk in enumerate(np.array_split(order, k)):
        chunk = chunk[np.argsort(p0[chunk], kind="stable")]
        half = chunk[len(chunk) // 2:] if j % 2 else chunk[:len(chunk) // 2]
        picks.append(int(half[len(half) // 2]))
    return picks


def batch_sample(k, seed=401, n_tissue=512):
    """k stratified tissues of the 512-tissue workload (see _stratified)."""
    work = g.workload_batch(seed=seed, n_tissue=n_tissue)
    return [work[i] for i in _stratified(work, k)]


def batched_relax(n_tissue=512, n_max=4096, max_iter=200000, plain_sample=16, seed=401,
                  mode="mixed", eta=3e-3, block_threads=256, t1=True, log=print):
    work = g.workload_batch(seed=seed, n_tissue=n_tissue, n_max=n_max)
    dt = V.pos_dtype(mode)
    Ts = [V.Tissue.from_tissue(t) for t, _ in work]
    Ps = [V.Params(KA=1.0, A0=1.0, KP=1.0, P0=float(p.P0[0]),
                   lam=torch.as_tensor(p.lam, dtype=dt, device="cuda")) for _, p in work]
    opts = dict(eta=eta, tol=1e-6, max_iter=max_iter, t1_enable=t1, l_min=0.01)
    Xs = [torch.as_tensor(t.X, dtype=dt, device="cuda") for t, _ in work]
    B = V.Batch(Ts)
    _sync()
    t0 = time.perf_counter()
    res = B.relax(Xs, Ps, mode=mode, block_threads=block_threads, **opts)
    _sync()
    tb = time.perf_counter() - t0
    iters = np.array([r["iters"] for r in res])
    nv = np.array([t.n_vert for t, _ in work])
    conv = np.array([r["status"] == 0 for r in res])
    n_t1 = np.array([r["n_t1"] for r in res])
    n_st = np.array([r["n_stretch"] for r in res])
    log(f"batched relax: {n_tissue} tissues in {tb:.2f}s, {conv.sum()} converged, "
        f"iterations median {int(np.median(iters))} max {iters.max()}, "
        f"T1 total {n_t1.sum()}, stretches total {n_st.sum()} (max {n_st.max()})")
    p0 = np.array([float(p.P0[0]) for _, p in work])
    bins = {}
    for lo, hi in ((3.6, 3.7), (3.7, 3.8), (3.8, 3.9)):
        sel = (p0 >= lo) & (p0 < hi if hi < 3.9 else p0 <= hi)
        bins[f"P0 {lo}-{hi}"] = {"tissues": int(sel.sum()), "converged": int(conv[sel].sum()),
                                 "iters_median": int(np.median(iters[sel])) if sel.any() else 0}
    log("batched relax by P0: " + ", ".join(f"{k}: {v['converged']}/{v['tissues']}"
                                            for k, v in bins.items()))
    # plain path on a stratified sample (same options, fresh handles and
    # positions), every solve timed in full
    sample = np.array(_stratified(work, plain_sample), dtype=np.int64) if plain_sample else \
        np.zeros(0, np.int64)
    tp = 0.0
    same = True
    for i in sample:
        t, p = work[i]
        T = V.Tissue.from_tissue(t)
        X = torch.as_tensor(t.X, dtype=dt, device="cuda")
        _sync()
        t0 = time.perf_counter()
        r = T.relax(X, Ps[i], mode=mode, **opts)
        _sync()
        tp += time.perf_counter() - t0
        same &= (r["iters"], r["n_t1"], r["status"]) == (res[i]["iters"], res[i]["n_t1"],
                                                         res[i]["status"])
    vi_all = float((nv * iters).sum())
    n_s = len(sample)
    conv_s = int(conv[sample].sum()) if n_s else 0
    plain_tps = n_s / tp if tp > 0 else float("nan")
    log(f"plain relax: stratified sample of {n_s} tissues solved in {tp:.2f}s "
        f"({plain_tps:.3f} tissues/s, {conv_s} converged) against {n_tissue / tb:.2f} "
        f"tissues/s batched")
    return {"tissues": n_tissue, "mode": mode, "max_iter": max_iter, "tol": 1e-6,
            "converged": int(conv.sum()), "converged_by_P0": bins,
            "iters_median": int(np.median(iters)),
            "iters_max": int(iters.max()), "batched_s": tb,
            "batched_tissues_per_s": n_tissue / tb,
            "batched_converged_tissues_per_s": int(conv.sum()) / tb,
            "batched_vertex_iters_per_s": vi_all / tb,
            "plain_sample": n_s, "plain_sample_cells": [int(nv[i] // 2) for i in sample],
            "plain_sample_s": tp, "plain_tissues_per_s": plain_tps,
            "plain_sample_converged": conv_s,
            "speedup_tissues_per_s": (n_tissue / tb) / plain_tps if n_s else None,
            "plain_matches_batched_on_sample": bool(same),
            "note": "tissues that reach max_iter are counted at the cap; the plain sample is "
                    "run to the same cap and gives the same iterates"}


def param_gradients(n_tissue=64, n_cell=1000, seed=501, relax_max_iter=2000000, plain_sample=8,
                    log=print):
    work = g.workload_inverse(seed=seed, n_tissue=n_tissue, n_cell=n_cell)
    Ts_t = [V.Tissue.from_tissue(t) for t, _, _ in work]
    Ts = [V.Tissue.from_tissue(t) for t, _, _ in work]
    dev = "cuda"

    def prm(p):
        return V.Params(KA=1.0, A0=1.0, KP=1.0, P0=3.75,
                        lam=torch.as_tensor(p.lam, dtype=torch.float64, device=dev))
    ropts = dict(eta=3e-3, tol=1e-6, max_iter=relax_max_iter, t1_enable=True, l_min=0.01)
    Xt = [torch.as_tensor(t.X, dtype=torch.float64, device=dev) for t, _, _ in work]
    Xs = [torch.as_tensor(t.X, dtype=torch.float64, device=dev) for t, _, _ in work]
    Pt = [prm(ps) for _, ps, _ in work]
    Pi = [prm(pi) for _, _, pi in work]
    _sync()
    t0 = time.perf_counter()
    # targets and predictions are independent: one batch of 2n tissues
    r2 = V.Batch(Ts_t + Ts).relax(Xt + Xs, Pt + Pi, mode="f64", **ropts)
    rt, rs = r2[:n_tissue], r2[n_tissue:]
    _sync()
    t_setup = time.perf_counter() - t0
    conv = sum(r["status"] == 0 for r in rs) + sum(r["status"] == 0 for r in rt)
    log(f"inverse workload: {2 * n_tissue} relaxations in {t_setup:.1f}s, {conv} converged")
    b = [T.v2v(X, Y)[1] for T, X, Y in zip(Ts, Xs, Xt)]
    B = V.Batch(Ts)
    out = {"tissues": n_tissue, "n_cell": n_cell, "params_per_tissue": Ts[0].n_edge,
           "setup_relax_s": t_setup, "relaxations_converged": int(conv)}
    # adjoint, batched
    _sync()
    t0 = time.perf_counter()
    gb, ib = B.param_grad(Xs, Pi, dC_dX=b, cg_tol=1e-8, cg_max_iter=100000)
    _sync()
    tb = time.perf_counter() - t0
    # adjoint, plain
    t0 = time.perf_counter()
    gp = []
    for T, X, P_, bb in zip(Ts, Xs, Pi, b):
        gg, _ = T.param_grad(X, P_, dC_dX=bb, cg_tol=1e-8, cg_max_iter=100000)
        gp.append(gg)
    _sync()
    tp = time.perf_counter() - t0
    diff = max(float((x - y).abs().max() / y.abs().max()) for x, y in zip(gb, gp))
    cg = [i["cg_iters"] for i in ib]
    st = [i["status"] for i in ib]
    log(f"adjoint: batched {tb * 1e3:.1f} ms, plain {tp * 1e3:.1f} ms, CG iters median "
        f"{int(np.median(cg))}, statuses {sorted(set(st))}, max rel diff {diff:.2e}")
    out["adjoint"] = {"batched_s": tb, "plain_s": tp,
                      "batched_grads_per_s": n_tissue / tb, "plain_grads_per_s": n_tissue / tp,
                      "speedup": tp / tb, "cg_iters_median": int(np.median(cg)),
                      "cg_iters_max": int(max(cg)),
                      "converged": int(sum(s == 0 for s in st)),
                      "batched_vs_plain_max_rel_diff": diff}
    # adjoint by MINRES (the paper's solver), batched
    _sync()
    t0 = time.perf_counter()
    gm, im = B.param_grad(Xs, Pi, dC_dX=b, cg_tol=1e-8, cg_max_iter=100000,
                          method="adjoint_minres")
    _sync()
    tm = time.perf_counter() - t0
    dm = max(float((x - y).abs().max() / y.abs().max()) for x, y in zip(gm, gb))
    mi = [i["cg_iters"] for i in im]
    log(f"adjoint (MINRES): batched {tm * 1e3:.1f} ms, iterations median {int(np.median(mi))}, "
        f"vs CG max rel diff {dm:.2e}")
    out["adjoint_minres"] = {"batched_s": tm, "batched_grads_per_s": n_tissue / tm,
                             "iters_median": int(np.median(mi)),
                             "converged": int(sum(i["status"] == 0 for i in im)),
                             "vs_cg_max_rel_diff": dm}
    # EP, batched and plain (beta = 1e-3, FP64 nudged relaxations)
    ep = dict(eta=3e-3, tol=1e-10, max_iter=relax_max_iter)
    _sync()
    t0 = time.perf_counter()
    ge, ie = B.param_grad(Xs, Pi, X_target=Xt, method="ep", beta=1e-3, ep_relax=ep)
    _sync()
    te = time.perf_counter() - t0
    n_plain = max(1, min(plain_sample, n_tissue))
    t0 = time.perf_counter()
    for T, X, P_, Y in list(zip(Ts, Xs, Pi, Xt))[:n_plain]:
        T.param_grad(X, P_, X_target=Y, method="ep", beta=1e-3, ep_relax=ep)
    _sync()
    tep = (time.perf_counter() - t0) * n_tissue / n_plain
    rel = [float((x - y).abs().max() / y.abs().max()) for x, y in zip(ge, gb)]
    log(f"EP: batched {te:.2f}s, plain {tep:.2f}s (extrapolated from {n_plain}), "
        f"EP vs adjoint max rel diff median {np.median(rel):.2e}")
    out["ep"] = {"beta": 1e-3, "batched_s": te, "plain_s_extrapolated": tep,
                 "plain_sample": n_plain, "batched_grads_per_s": n_tissue / te,
                 "speedup": tep / te, "vs_adjoint_rel_diff_median": float(np.median(rel))}
    # first-order EP, batched (one nudged relaxation per tissue)
    _sync()
    t0 = time.perf_counter()
    gf, _ = B.param_grad(Xs, Pi, X_target=Xt, method="ep_forward", beta=1e-3, ep_relax=ep)
    _sync()
    tf = time.perf_counter() - t0
    # (its accuracy is checked below at a tightly relaxed X*: here X* is
    # relaxed to 1e-6 only, and the one-sided estimate also sees X* move
    # towards the 1e-10 equilibrium of the nudged relaxation, divided by beta)
    log(f"first-order EP: batched {tf:.2f}s")
    out["ep_forward"] = {"beta": 1e-3, "batched_s": tf, "batched_grads_per_s": n_tissue / tf}
    out["finite_differences"] = finite_differences(Ts[:2], [w[0] for w in work[:2]], Xs[:2],
                                                   Pi[:2], Xt[:2], log=log)
    # forward (sensitivity) ID: one CG solve per parameter direction, 8 random
    # unit directions on a sample of tissues, checked against adjoint . d
    rng = np.random.default_rng(seed + 7)
    n_s = max(1, min(plain_sample, n_tissue))
    errs, n_solve = [], 0
    _sync()
    t0 = time.perf_counter()
    for T, X, P_, bb, ga in list(zip(Ts, Xs, Pi, b, gb))[:n_s]:
        for _ in range(8):
            d = torch.as_tensor(rng.normal(size=T.n_edge), dtype=torch.float64, device=dev)
            d /= d.norm()
            sv, _, info = T.param_sens(X, P_, d, bb, cg_tol=1e-8)
            ref = float(ga @ d)
            errs.append(abs(sv.item() - ref) / max(abs(ref), 1e-300))
            n_solve += 1
    _sync()
    ts = time.perf_counter() - t0
    log(f"sensitivity ID: {n_solve} directional solves in {ts * 1e3:.1f} ms "
        f"({ts / n_solve * 1e3:.2f} ms each), vs adjoint . d max rel diff {max(errs):.2e}")
    out["sensitivity"] = {"directions": n_solve, "s": ts, "ms_per_direction": ts / n_solve * 1e3,
                          "directions_per_full_gradient": Ts[0].n_edge,
                          "vs_adjoint_max_rel_diff": max(errs)}
    return out


def finite_differences(Ts, ts, Xs, Ps, Xts, n_dir=8, h=1e-3, beta=1e-3, tol=1e-11, seed=512,
                       relax_max_iter=3000000, log=print):
    """Central differences of the relaxed v2v cost C(X*(lambda)) along
    n_dir random unit directions d per tissue, at steps 2h, h and h/2,
    against adjoint . d, centred EP . d and first-order EP . d at the same
    state.  Every relaxation runs without T1 to max |F| < tol (FP64) from
    X* relaxed to the same tolerance; the FD relaxations of all tissues,
    directions and steps form one batch.

    A centred difference at step s carries two errors: truncation, a s^2,
    and the part of the displacement that gradient descent leaves
    unrelaxed when it stops at max |F| < tol (along the softest modes, of
    about tol / mu_min each), which does not shrink with s and so enters
    the difference as c / s.  (GD in FP64 cannot go below tol ~ 1e-11 on
    these tissues: a step eta |F| = 3e-15 is below the spacing of doubles
    near the box side.)  The three steps determine g + a s^2 + c / s
    exactly; g is the FD estimate, and a h^2 and c / h say which error
    dominated at h.  The EP estimates are limited by the same tolerance,
    an error of about tol / (beta |grad C|) relative to the gradient."""
    rng = np.random.default_rng(seed)
    dev = "cuda"
    B = V.Batch(Ts)
    X0s = [X.clone() for X in Xs]
    t0 = time.perf_counter()
    r0 = B.relax(X0s, Ps, mode="f64", eta=3e-3, tol=tol, max_iter=relax_max_iter,
                 t1_enable=False)
    log(f"finite differences: X* relaxed to {tol:g} ({[r['iters'] for r in r0]} steps, "
        f"{time.perf_counter() - t0:.1f}s)")
    bs = [T.v2v(X0, Xt)[1] for T, X0, Xt in zip(Ts, X0s, Xts)]
    ga, ia = B.param_grad(X0s, Ps, dC_dX=bs, cg_tol=1e-12)
    ep_t = dict(eta=3e-3, tol=tol, max_iter=relax_max_iter)
    t0 = time.perf_counter()
    ge, ie = B.param_grad(X0s, Ps, X_target=Xts, method="ep", beta=beta, ep_relax=ep_t)
    log(f"finite differences: centred EP {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    gf, if_ = B.param_grad(X0s, Ps, X_target=Xts, method="ep_forward", beta=beta, ep_relax=ep_t)
    log(f"finite differences: first-order EP {time.perf_counter() - t0:.1f}s")
    grads = list(zip(ga, ge, gf))
    ep_status = [{"x_star": r0[i]["status"], "adjoint_cg": ia[i]["status"],
                  "ep_plus": ie[i]["ep_plus"]["status"], "ep_minus": ie[i]["ep_minus"]["status"],
                  "ep_forward": if_[i]["ep_plus"]["status"],
                  "ep_iters": [ie[i]["ep_plus"]["iters"], ie[i]["ep_minus"]["iters"],
                               if_[i]["ep_plus"]["iters"]]} for i in range(len(Ts))]
    steps = (2.0 * h, h, 0.5 * h)
    dirs = []
    Tfd, Xfd, Pfd = [], [], []
    for T, t, X0, P in zip(Ts, ts, X0s, Ps):
        he = T.topology()
        ds = []
        for _ in range(n_dir):
            d = torch.as_tensor(rng.normal(size=T.n_edge), dtype=torch.float64, device=dev)
            d /= d.norm()
            ds.append(d)
            for hh in steps:
                for sgn in (1.0, -1.0):
                    Tfd.append(V.Tissue(he, T.n_vert, t.Lx, t.Ly))
                    Xfd.append(X0.clone())
                    Pfd.append(V.Params(KA=1.0, A0=1.0, KP=1.0, P0=3.75,
                                        lam=P.lam + sgn * hh * d))
        dirs.append(ds)
    _sync()
    t0 = time.perf_counter()
    rfd = V.Batch(Tfd).relax(Xfd, Pfd, mode="f64", eta=3e-3, tol=tol, max_iter=relax_max_iter,
                             t1_enable=False)
    _sync()
    tfd = time.perf_counter() - t0
    per_t = 2 * len(steps) * n_dir
    Cs = [T.v2v(X, Xts[k // per_t])[0].item() for k, (T, X) in enumerate(zip(Tfd, Xfd))]
    # FD(s) = g + a s^2 + c / s through the three steps
    A = np.array([[1.0, s_ * s_, 1.0 / s_] for s_ in steps])
    rows = []
    for i in range(len(Ts)):
        ga, ge, gf = grads[i]
        for j, d in enumerate(dirs[i]):
            k = 2 * len(steps) * (n_dir * i + j)
            fd = [(Cs[k + 2 * q] - Cs[k + 2 * q + 1]) / (2.0 * s_) for q, s_ in enumerate(steps)]
            gx, ax, cx = np.linalg.solve(A, np.array(fd))
            rows.append({"fd_2h": fd[0], "fd_h": fd[1], "fd_h2": fd[2], "fd_extrapolated": gx,
                         "truncation_at_h": ax * h * h, "tolerance_term_at_h": cx / h,
                         "adjoint": float(ga @ d), "ep": float(ge @ d),
                         "ep_forward": float(gf @ d)})
    ref = np.array([r["fd_extrapolated"] for r in rows])
    scale = np.abs(ref).max()

    def err(key, against=ref):
        v = np.array([r[key] for r in rows])
        return float(np.abs(v - against).max() / scale)

    adj = np.array([r["adjoint"] for r in rows])
    res = {"tissues": len(Ts), "directions_per_tissue": n_dir, "steps": list(steps),
           "beta": beta, "relax_tol": tol,
           "fd_relaxations_converged": int(sum(r["status"] == 0 for r in rfd)),
           "fd_relaxations": len(rfd), "batched_relax_s": tfd,
           "error_basis": "max over directions of |x - FD extrapolated| / max |FD extrapolated|",
           "adjoint_vs_fd_extrapolated": err("adjoint"),
           "adjoint_vs_fd_h": err("fd_h", adj), "adjoint_vs_fd_h2": err("fd_h2", adj),
           "adjoint_vs_fd_2h": err("fd_2h", adj),
           "truncation_term_at_h": float(np.abs([r["truncation_at_h"] for r in rows]).max() / scale),
           "tolerance_term_at_h": float(np.abs([r["tolerance_term_at_h"] for r in rows]).max()
                                        / scale),
           "ep_vs_fd_extrapolated": err("ep"), "ep_forward_vs_fd_extrapolated": err("ep_forward"),
           "ep_vs_adjoint": err("ep", adj), "ep_forward_vs_adjoint": err("ep_forward", adj),
           "statuses": ep_status, "per_direction": rows}
    log(f"finite differences ({len(Ts)} tissues x {n_dir} directions, steps {steps}): error "
        f"terms at h: truncation {res['truncation_term_at_h']:.1e}, relaxation tolerance "
        f"{res['tolerance_term_at_h']:.1e}; adjoint against the extrapolated FD "
        f"{res['adjoint_vs_fd_extrapolated']:.2e} (against FD(h) alone "
        f"{res['adjoint_vs_fd_h']:.2e}); centred EP {res['ep_vs_fd_extrapolated']:.2e}, "
        f"first-order EP {res['ep_forward_vs_fd_extrapolated']:.2e} "
        f"({res['fd_relaxations_converged']}/{len(rfd)} relaxations converged in {tfd:.1f}s; "
        f"statuses {ep_status})")
    return res


def _inverse_equilibria(n_tissue, n_cell, seed, relax_max_iter):
    """The inverse workload's targets and predictions relaxed (batched,
    FP64, T1, to 1e-6): tissues, predicted equilibria, targets, parameters."""
    work = g.workload_inverse(seed=seed, n_tissue=n_tissue, n_cell=n_cell)
    Ts_t = [V.Tissue.from_tissue(t) for t, _, _ in work]
    Ts = [V.Tissue.from_tissue(t) for t, _, _ in work]

    def prm(p):
        return V.Params(KA=1.0, A0=1.0, KP=1.0, P0=3.75,
                        lam=torch.as_tensor(p.lam, dtype=torch.float64, device="cuda"))
    ropts = dict(eta=3e-3, tol=1e-6, max_iter=relax_max_iter, t1_enable=True, l_min=0.01)
    Xt = [torch.as_tensor(t.X, dtype=torch.float64, device="cuda") for t, _, _ in work]
    Xs = [torch.as_tensor(t.X, dtype=torch.float64, device="cuda") for t, _, _ in work]
    V.Batch(Ts_t).relax(Xt, [prm(ps) for _, ps, _ in work], mode="f64", **ropts)
    Pi = [prm(pi) for _, _, pi in work]
    V.Batch(Ts).relax(Xs, Pi, mode="f64", **ropts)
    return Ts, Xs, Xt, Pi


def batched_adjoint_once(n_tissue=64, n_cell=1000, seed=501, relax_max_iter=2000000,
                         log=print):
    """The inverse workload's batched adjoint on its own: targets and
    predictions relaxed (batched, FP64, T1), then one batched adjoint
    launch (CG to 1e-8).  A short program for kernel counters."""
    Ts, Xs, Xt, Pi = _inverse_equilibria(n_tissue, n_cell, seed, relax_max_iter)
    b = [T.v2v(X, Y)[1] for T, X, Y in zip(Ts, Xs, Xt)]
    _sync()
    t0 = time.perf_counter()
    _, info = V.Batch(Ts).param_grad(Xs, Pi, dC_dX=b, cg_tol=1e-8, cg_max_iter=100000)
    _sync()
    dt = time.perf_counter() - t0
    it = [i["cg_iters"] for i in info]
    log(f"batched adjoint: {n_tissue} tissues in {dt * 1e3:.2f} ms, CG steps median "
        f"{int(np.median(it))} max {max(it)}")
    return dt


def batched_ep_once(n_tissue=64, n_cell=1000, seed=501, relax_max_iter=2000000,
                    ep_steps=20000, log=print):
    """The inverse workload's set-up relaxations, then one batched centred EP
    (beta = 1e-3, v2v nudge to the targets) whose nudged relaxations run a
    fixed number of steps.  A short program for kernel counters."""
    Ts, Xs, Xt, Pi = _inverse_equilibria(n_tissue, n_cell, seed, relax_max_iter)
    _sync()
    t0 = time.perf_counter()
    V.Batch(Ts).param_grad(Xs, Pi, X_target=Xt, method="ep", beta=1e-3,
                           ep_relax=dict(eta=3e-3, tol=0.0, max_iter=ep_steps))
    _sync()
    dt = time.perf_counter() - t0
    log(f"batched centred EP: {n_tissue} tissues, {ep_steps} nudged steps each sign, "
        f"{dt:.2f} s")
    return dt


if __name__ == "__main__":
    # short programs for kernel counters: the batched adjoint or a
    # fixed-length batched centred EP of the inverse workload, or the
    # 512-tissue batched relaxation capped at 2e4 iterations
    import sys
    if sys.argv[1:] == ["adjoint"]:
        batched_adjoint_once()
    elif sys.argv[1:] == ["ep"]:
        batched_ep_once()
    elif sys.argv[1:] == ["relax"]:
        batched_relax(max_iter=20000, plain_sample=0, block_threads=1024)
    else:
        raise SystemExit("usage: python -m paper_2604_06896_amd.suite adjoint|ep|relax")
