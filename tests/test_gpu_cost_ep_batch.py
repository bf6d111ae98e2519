"""Parity of the v2v cost, the nudged relaxations and the batched schedules
with the FP64 CPU oracle, at the sizes and launch configurations the
benchmark uses.

  * v2v cost and gradient (Methods, "Geometric vertex-to-vertex (v2v)
    cost"), minimum image, on a tissue whose targets straddle the box;
  * the linear-nudge energy of a relaxation in FP32;
  * batched centred and first-order EP (Methods, "Equilibrium propagation
    (EP)") on a 1000-cell tissue of the inverse workload in the
    LDS-resident batch kernel (four vertices per thread), against the
    single-tissue path and the oracle;
  * the 512-tissue batched relaxation in the benchmark's mode (MIXED, 1024
    threads per tissue, T1) against the single-tissue path;
  * the bilevel ADAM loop (Methods, "Bilevel optimization framework")
    against the same loop driven by oracle relaxations and oracle adjoint
    gradients.
"""
import os
import sys

import numpy as np
import pytest
import torch

from paper_2604_06896_amd import tissue_gen as g

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def vtx():
    from paper_2604_06896_amd import vtx as V
    V.lib()
    assert torch.cuda.is_available()
    return V


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


# ------------------------------------------------------------------ v2v

@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_v2v_matches_oracle_across_the_box(vtx, oracle, errlog, mode):
    """Targets are the positions moved by N(0, 0.05) and wrapped into the
    box, and a third of the positions are shifted by a whole box length, so
    raw differences near +-L occur for many vertices; the cost is
    1/(2 n_vert) sum |min_image(x - x_t)|^2 and the gradient
    min_image(x - x_t) / n_vert."""
    rng = np.random.default_rng(17)
    t = g.random_tissue(1000, np.sqrt(1000.0), rng=rng)
    L = np.array([t.Lx, t.Ly])
    Xt = np.mod(t.X + rng.normal(0, 0.05, t.X.shape), L)
    X = t.X + L * rng.integers(-1, 2, t.X.shape) * (rng.random((t.n_vert, 1)) < 1 / 3)
    raw = np.abs(X - Xt)
    assert (raw > L / 2).sum() > 100          # the minimum image matters
    dt = vtx.pos_dtype(mode)
    Xd, Xtd = _dev(X, dt), _dev(Xt, dt)
    # the oracle sees exactly the GPU's inputs
    Xh, Xth = Xd.double().cpu().numpy(), Xtd.double().cpu().numpy()
    co, go = oracle.v2v(oracle.Mesh.from_tissue(t), Xh, Xth)
    T = vtx.Tissue.from_tissue(t)
    C, grad = T.v2v(Xd, Xtd, mode=mode)
    grad = grad.cpu().numpy()
    errlog(f"v2v cost {mode}, 1000 cells across the box (relative)", abs(C.item() / co - 1))
    errlog(f"v2v gradient {mode}, 1000 cells across the box (max |d| / max)",
           np.abs(grad - go).max() / np.abs(go).max())
    assert C.item() == pytest.approx(co, rel=1e-12)
    assert np.abs(grad - go).max() <= 1e-12 * np.abs(go).max()
    # the closed form at a pure translation by (a, b): C = (a^2 + b^2) / 2
    C2, g2 = T.v2v(_dev(X + np.array([0.3, -0.2]), dt), Xd, mode=mode)
    assert C2.item() == pytest.approx(0.5 * (0.3 ** 2 + 0.2 ** 2), rel=1e-6 if mode == "f32"
                                      else 1e-12)


# -------------------------------------------------- linear-nudge energy

@pytest.mark.parametrize("mode", ["f32", "mixed", "f64"])
def test_linear_nudge_energy(vtx, oracle, errlog, mode):
    """A relaxation nudged by the linear cost g . X reports E + beta g . X at
    the positions it returns; g is double for every precision, the positions
    are the mode's own type."""
    rng = np.random.default_rng(19)
    t = g.random_tissue(300, np.sqrt(300.0), rng=rng)
    p = g.uniform_params(t, P0=3.7)
    p.lam = rng.uniform(0.05, 0.15, t.n_edge)
    gl = rng.normal(0, 1e-2, t.X.shape)
    dt = vtx.pos_dtype(mode)
    T = vtx.Tissue.from_tissue(t)
    X = _dev(t.X, dt)
    beta = 0.1
    r = T.relax(X, vtx.Params.from_numpy(p, dtype=dt), mode=mode, eta=3e-3, tol=0.0,
                max_iter=50, beta=beta, g_lin=_dev(gl))
    assert r["iters"] == 50
    Xh = X.double().cpu().numpy()
    Eo = oracle.energy(oracle.Mesh.from_tissue(t), Xh, p)
    ref = Eo + beta * float((gl * Xh).sum())
    rel = abs(r["energy"] - ref) / (abs(Eo) + abs(beta * float((gl * Xh).sum())))
    errlog(f"linear-nudge relaxation energy {mode} (relative)", rel)
    # MIXED sums the line-tension energy from FP32 lengths, FP32 also the
    # cell terms; FP64 is exact to rounding
    assert rel < {"f32": 2e-6, "mixed": 1e-8, "f64": 1e-12}[mode]


# --------------------------------------------- batched EP at 1000 cells

def _inverse_equilibrium():
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_inverse_equilibrium as mk
    return mk.load()


@pytest.fixture(scope="module")
def inverse_x_star(oracle):
    """The first 1000-cell tissue of the inverse workload relaxed by the
    oracle (max |F| < 1e-6, T1 on; stored in tests/golden by a script that
    calls only the oracle), checked here to be that equilibrium."""
    t, X, pi = _inverse_equilibrium()
    m = oracle.Mesh.from_tissue(t)
    _, F = oracle.energy_forces(m, X, pi)
    assert np.abs(F).max() < 1e-6
    return t, m, X, pi


@pytest.mark.parametrize("method", ["ep", "ep_forward"])
def test_batched_ep_1000_cells_lds_kernel(vtx, oracle, errlog, inverse_x_star, method):
    """EP at beta = 1e-3 (the inverse workload's) from the oracle's X*: each
    nudged relaxation runs a fixed 3000 FP64 steps on both sides (the
    tolerance is not reached in that time; status NOT_CONVERGED on both),
    so the estimator's whole procedure is compared step for step.  The batch
    (library choice: the LDS-resident kernel, 512 threads, four vertices per
    thread) against the single-tissue path and the oracle."""
    t, m, X, pi = inverse_x_star
    beta, iters = 1e-3, 3000
    rng = np.random.default_rng(29)
    Xt = X + rng.normal(0, 0.05, X.shape)
    ep = dict(eta=3e-3, tol=1e-14, max_iter=iters)
    if method == "ep":
        go, info_o = oracle.ep_grad(m, X, pi, Xt, beta, patience=1, **ep)
    else:
        go, info_o = oracle.ep_grad_forward(m, X, pi, Xt, beta, patience=1, **ep)
    assert info_o["plus"]["iters"] == iters and info_o["plus"]["status"] == 1
    P = vtx.Params.from_numpy(pi)
    T1 = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
    gs, info_s = T1.param_grad(_dev(X), P, X_target=_dev(Xt), method=method, beta=beta,
                               ep_relax=ep)
    T2 = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
    outs, infos = vtx.Batch([T2]).param_grad([_dev(X)], [P], X_target=[_dev(Xt)],
                                             method=method, beta=beta, ep_relax=ep)
    gb, info_b = outs[0].cpu().numpy(), infos[0]
    gs = gs.cpu().numpy()
    assert info_b["ep_plus"]["iters"] == iters and info_b["status"] == 1
    assert info_b["ep_plus"]["status"] == info_s["ep_plus"]["status"] == 1
    scale = np.abs(go).max()
    d_bs = np.abs(gb - gs).max() / scale
    d_bo = np.abs(gb - go).max() / scale
    errlog(f"batched {method} (LDS kernel, 1000 cells, 2x{iters} steps) vs single path "
           "(max |dg| / max |g|)", d_bs)
    errlog(f"batched {method} (LDS kernel, 1000 cells, 2x{iters} steps) vs oracle "
           "(max |dg| / max |g|)", d_bo)
    # the nudge mean is summed in a different order by the grid path and the
    # persistent kernel, so bit-for-bit equality is not guaranteed (measured:
    # equal on this tissue)
    assert d_bs < 1e-8
    assert d_bo < 1e-6
    assert info_b["ep_plus"]["energy"] == pytest.approx(info_o["plus"]["energy"], rel=1e-11)


# ----------------------------------- 512-tissue workload, benchmark mode

def test_batched_relax_bench_mode_matches_single(vtx, errlog):
    """The 512-tissue workload in the benchmark's launch configuration
    (MIXED, one 1024-thread workgroup per tissue, T1 at 0.01, step 3e-3),
    capped at 2e4 iterations: the smallest, a median and the largest tissue
    equal the single-tissue path, topology bit-exact.  (The oracle is FP64;
    MIXED rounds the force arithmetic to FP32, so this mode is held to the
    single path here and the FP64 batch to the oracle elsewhere.)"""
    work = g.workload_batch()
    sizes = np.array([t.n_cell for t, _ in work])
    picks = [int(sizes.argmin()), int(np.argsort(sizes)[len(sizes) // 2]), int(sizes.argmax())]
    opts = dict(eta=3e-3, tol=1e-6, max_iter=20000, t1_enable=True, l_min=0.01)
    Ts = [vtx.Tissue.from_tissue(t) for t, _ in work]
    Xs = [_dev(t.X) for t, _ in work]
    Ps = [vtx.Params.from_numpy(p) for _, p in work]
    res = vtx.Batch(Ts).relax(Xs, Ps, mode="mixed", block_threads=1024, **opts)
    for i in picks:
        t, p = work[i]
        T = vtx.Tissue.from_tissue(t)
        X = _dev(t.X)
        rs = T.relax(X, Ps[i], mode="mixed", **opts)
        r = res[i]
        print(t.n_cell, "single", rs, "batch", r)
        assert (r["iters"], r["n_t1"], r["n_stretch"], r["status"]) == (
            rs["iters"], rs["n_t1"], rs["n_stretch"], rs["status"])
        assert r["iters"] == 20000 or r["status"] == 0
        np.testing.assert_array_equal(Ts[i].topology(), T.topology())
        d = float((Xs[i] - X).abs().max())
        errlog(f"batched vs single relaxation, 512-tissue workload in its benchmark mode "
               f"(MIXED, 1024 threads), {t.n_cell}-cell tissue, 2e4 steps: positions (max abs)",
               d)
        assert d == 0.0
        assert r["energy"] == pytest.approx(rs["energy"], rel=1e-7)


# ----------------------------------------------- bilevel loop vs oracle

def _adam_reference(theta0, grads_fn, epochs, lr, b1=0.9, b2=0.999, eps=1e-8):
    """ADAM (Kingma and Ba, 2015) with bias correction, written out."""
    th = theta0.copy()
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    out = [th.copy()]
    for k in range(1, epochs + 1):
        gr = grads_fn(th)
        m = b1 * m + (1 - b1) * gr
        v = b2 * v + (1 - b2) * gr * gr
        mh = m / (1 - b1 ** k)
        vh = v / (1 - b2 ** k)
        th = th - lr * mh / (np.sqrt(vh) + eps)
        out.append(th.copy())
    return out


def test_bilevel_fit_matches_oracle_loop(vtx, oracle, errlog):
    """Five epochs of the bilevel p0 fit (N = 20, the paper's benchmark
    settings: inner GD 1e-2, <= 1e3 iterations, tol 1e-3, patience 10, T1
    below 5e-3; outer ADAM lr 1e-3; v2v cost; adjoint CG to 1e-8) equal the
    same loop run on the oracle: oracle relaxations (warm-started, T1
    mutating the oracle's topology), oracle v2v gradient, oracle adjoint."""
    from paper_2604_06896_amd import studies
    epochs = 5
    hist = studies.bilevel_fit(epochs=epochs, method="adjoint", log=None)
    rng = np.random.default_rng(701)
    t = g.random_tissue(20, float(np.sqrt(20)), rng=rng)
    theta_star = rng.normal(3.75, 0.05, 20)
    theta0 = rng.normal(3.75, 0.05, 20)
    inner = dict(eta=1e-2, tol=1e-3, patience=10, max_iter=1000, t1_enable=True, l_min=5e-3)

    def prm(th):
        p = g.uniform_params(t, P0=3.75)
        p.P0 = np.asarray(th, dtype=np.float64).copy()
        return p

    mt = oracle.Mesh.from_tissue(t)
    Xt = t.X.copy()
    oracle.relax(mt, Xt, prm(theta_star), **inner)
    m = oracle.Mesh.from_tissue(t)
    X = t.X.copy()
    oracle.relax(m, X, prm(theta0), **inner)

    def grads(th):
        oracle.relax(m, X, prm(th), **inner)
        _, gX = oracle.v2v(m, X, Xt)
        gth, _ = oracle.adjoint_grad(m, X, prm(th), gX, theta="P0", tol=1e-8)
        return gth

    ref = _adam_reference(theta0, grads, epochs, 1e-3)
    assert len(hist["theta"]) == epochs + 1
    worst = max(float(np.abs(a - b).max()) for a, b in zip(hist["theta"], ref))
    errlog("bilevel p0 fit, 5 ADAM epochs: theta against the oracle-driven loop (max abs)",
           worst)
    assert worst <= 1e-8
    assert float(np.abs(ref[-1] - ref[0]).max()) > 1e-3     # theta did move
