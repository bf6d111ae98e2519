"""Parity of the HIP library (through its C ABI) with the FP64 CPU oracle.

Tolerances: forces within 1e-5 of max |F| (relative, the requirement for the
FP32 path; the FP64 path is held to 1e-10), energies within the rounding of
each precision, topology after T1 bit-exact, relaxed positions within 1e-4
of the mean edge length."""
import numpy as np
import pytest
import torch

from paper_2604_06896_amd import tissue_gen as g

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vtx():
    from paper_2604_06896_amd import vtx as V
    V.lib()
    assert torch.cuda.is_available()
    return V


def _rand_params(t, rng):
    p = g.uniform_params(t)
    p.KA = rng.uniform(0.5, 1.5, t.n_cell)
    p.A0 = rng.uniform(0.8, 1.2, t.n_cell)
    p.KP = rng.uniform(0.5, 1.5, t.n_cell)
    p.P0 = rng.uniform(3.5, 4.0, t.n_cell)
    p.lam = rng.uniform(0.0, 0.2, t.n_edge)
    return p


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _force_err(F, Fo):
    return np.abs(F - Fo).max() / np.abs(Fo).max()


# ----------------------------------------------------------- energy / forces

@pytest.mark.parametrize("n_cell,seed", [(100, 101), (1000, 5), (37, 9)])
def test_energy_forces_f64(vtx, oracle, errlog, n_cell, seed):
    rng = np.random.default_rng(seed)
    t = g.random_tissue(n_cell, np.sqrt(n_cell), rng=rng)
    p = _rand_params(t, rng)
    X = t.X + rng.normal(0, 0.02, t.X.shape)
    Eo, Fo = oracle.energy_forces(oracle.Mesh.from_tissue(t), X, p)
    T = vtx.Tissue.from_tissue(t)
    E, F, mf = T.energy_forces(_dev(X), vtx.Params.from_numpy(p), mode="f64", want_maxf=True)
    F = F.cpu().numpy()
    errlog(f"forces f64, {n_cell} cells (max |dF| / max |F|)", _force_err(F, Fo))
    errlog(f"energy f64, {n_cell} cells (relative)", abs(E.item() / Eo - 1))
    assert _force_err(F, Fo) < 1e-10
    assert E.item() == pytest.approx(Eo, rel=1e-12)
    assert mf.item() == pytest.approx(np.abs(Fo).max(), rel=1e-10)


@pytest.mark.parametrize("mode", ["f32", "mixed"])
def test_energy_forces_reduced_precision(vtx, oracle, errlog, mode):
    t, p = g.workload_single_10k()
    dt = torch.float32 if mode == "f32" else torch.float64
    Xd = _dev(t.X, dt)
    Xin = Xd.double().cpu().numpy()       # the oracle sees exactly the GPU's input
    Eo, Fo = oracle.energy_forces(oracle.Mesh.from_tissue(t), Xin, p)
    T = vtx.Tissue.from_tissue(t)
    E, F, _ = T.energy_forces(Xd, vtx.Params.from_numpy(p, dtype=dt), mode=mode)
    err = _force_err(F.double().cpu().numpy(), Fo)
    print(f"{mode}: max |dF| / max |F| = {err:.3e}, E rel err = {abs(E.item() / Eo - 1):.3e}")
    errlog(f"forces {mode}, 1e4 cells (max |dF| / max |F|)", err)
    errlog(f"energy {mode}, 1e4 cells (relative)", abs(E.item() / Eo - 1))
    assert err < 1e-5
    assert E.item() == pytest.approx(Eo, rel=1e-6)


def test_forces_scalar_params_and_hex_lattice(vtx, oracle):
    s = 0.62
    t = g.hex_lattice(6, 8, s)
    T = vtx.Tissue.from_tissue(t)
    prm = vtx.Params(KA=1.3, A0=0.9, KP=0.7, P0=3.5, lam=0.2)
    E, F, _ = T.energy_forces(_dev(t.X), prm, mode="f64")
    Ah, Ph = 1.5 * np.sqrt(3.0) * s * s, 6 * s
    N = t.n_cell
    assert E.item() == pytest.approx(N * (1.3 * (Ah - 0.9) ** 2 + 0.7 * (Ph - 3.5) ** 2)
                                     + 3 * N * 0.2 * s, rel=1e-12)
    assert F.abs().max().item() < 1e-12


def test_forces_deterministic(vtx):
    t, p = g.workload_single_10k()
    T = vtx.Tissue.from_tissue(t)
    Xd = _dev(t.X, torch.float32)
    P = vtx.Params.from_numpy(p, dtype=torch.float32)
    E1, F1, _ = T.energy_forces(Xd, P, mode="f32")
    E2, F2, _ = T.energy_forces(Xd, P, mode="f32")
    assert torch.equal(F1, F2) and E1.item() == E2.item()


def test_force_kernel_full_size_1m_cells(vtx, oracle, errlog):
    """The 10^6-cell workload in the launch configuration the benchmark times
    (FP32 positions); all 4e6 force components against the oracle."""
    t, p = g.workload_force_1m()
    T = vtx.Tissue.from_tissue(t)
    Xd = _dev(t.X, torch.float32)
    P = vtx.Params(KA=1.0, A0=1.0, KP=1.0, P0=3.75,
                   lam=torch.as_tensor(p.lam, dtype=torch.float32, device="cuda"))
    E, F, _ = T.energy_forces(Xd, P, mode="f32")
    pin = g.uniform_params(t, P0=3.75)
    pin.lam = torch.as_tensor(p.lam, dtype=torch.float32).double().numpy()
    Eo, Fo = oracle.energy_forces(oracle.Mesh.from_tissue(t), Xd.double().cpu().numpy(), pin)
    err = _force_err(F.double().cpu().numpy(), Fo)
    print(f"1e6 cells f32: max |dF| / max |F| = {err:.3e}")
    errlog("forces f32, 1e6 cells (max |dF| / max |F|)", err)
    errlog("energy f32, 1e6 cells (relative)", abs(E.item() / Eo - 1))
    assert err < 1e-5
    assert E.item() == pytest.approx(Eo, rel=1e-6)


def test_geometry_and_lengths(vtx, oracle):
    rng = np.random.default_rng(2)
    t = g.random_tissue(200, np.sqrt(200.0), rng=rng)
    T = vtx.Tissue.from_tissue(t)
    A, P = T.cell_geometry(_dev(t.X))
    Ao, Po, _ = oracle.cells(oracle.Mesh.from_tissue(t), t.X)
    np.testing.assert_allclose(A.cpu().numpy(), Ao, rtol=1e-12)
    np.testing.assert_allclose(P.cpu().numpy(), Po, rtol=1e-12)
    L = T.edge_lengths(_dev(t.X))
    np.testing.assert_allclose(L.cpu().numpy(), oracle.edge_lengths(oracle.Mesh.from_tissue(t), t.X),
                               rtol=1e-12)


def _many_sided_tissue():
    """A seed inside a ring of 16 seeds (a 16-sided cell) among 260 random
    seeds: 12 cells have more than 8 sides, one more than 12."""
    rng = np.random.default_rng(3)
    L = 20.0
    c = np.array([L / 2, L / 2])
    ang = np.linspace(0, 2 * np.pi, 16, endpoint=False) + 0.05
    ring = c + np.stack([np.cos(ang), np.sin(ang)], 1)
    far = []
    while len(far) < 260:
        q = rng.uniform(0, L, 2)
        if np.linalg.norm(q - c) > 2.6:
            far.append(q)
    t = g.periodic_voronoi(np.vstack([c[None], ring, np.array(far)]), L, L)
    return t, _rand_params(t, rng)


def test_cells_with_many_sides(vtx, oracle):
    """Corner loops past the prefetched slots (8 in the cell pass and the
    HVP, 12 in the T1 row geometry): forces, geometry, HVP and a T1 pass
    around the 16-sided cell as the oracle's."""
    t, p = _many_sided_tissue()
    ns = np.bincount(t.he[:, 5])
    assert ns.max() == 16 and (ns > 8).sum() >= 10
    m = oracle.Mesh.from_tissue(t)
    T = vtx.Tissue.from_tissue(t)
    P = vtx.Params.from_numpy(p)
    Eo, Fo = oracle.energy_forces(m, t.X, p)
    E, F, _ = T.energy_forces(_dev(t.X), P, mode="f64")
    assert _force_err(F.cpu().numpy(), Fo) < 1e-10 and E.item() == pytest.approx(Eo, rel=1e-12)
    E32, F32, _ = T.energy_forces(_dev(t.X, torch.float32), vtx.Params.from_numpy(
        p, dtype=torch.float32), mode="f32")
    Fo32 = oracle.energy_forces(m, _dev(t.X, torch.float32).double().cpu().numpy(), p)[1]
    assert _force_err(F32.double().cpu().numpy(), Fo32) < 1e-5
    A, Pc = T.cell_geometry(_dev(t.X))
    Ao, Po, _ = oracle.cells(m, t.X)
    np.testing.assert_allclose(A.cpu().numpy(), Ao, rtol=1e-12)
    np.testing.assert_allclose(Pc.cpu().numpy(), Po, rtol=1e-12)
    v = np.random.default_rng(4).normal(size=t.X.shape)
    Hv = T.hvp(_dev(t.X), P, _dev(v)).cpu().numpy()
    Hvo = oracle.hvp(m, t.X, p, v)
    assert np.abs(Hv - Hvo).max() < 1e-10 * np.abs(Hvo).max()
    # a T1 pass whose threshold makes half the 16-sided cell's edges short
    big = int(np.argmax(ns))
    ell = oracle.edge_lengths(m, t.X)
    eoh, _ = oracle.edge_index(m)
    l_min = float(np.median(ell[eoh[t.he[:, 5] == big]]))
    X = t.X.copy()
    n_sw, n_st = oracle.t1_pass(m, X, p, l_min, 1.2 * l_min)
    assert n_sw + n_st > 0
    Xd = _dev(t.X)
    assert tuple(T.t1(Xd, P, l_min, 1.2 * l_min, mode="f64")) == (n_sw, n_st)
    np.testing.assert_array_equal(T.topology(), m.he)
    assert np.abs(Xd.cpu().numpy() - X).max() < 1e-12


def test_batched_lds_paths_with_many_sided_cells(vtx, small_equilibria):
    """The LDS-resident relaxation (no T1) and the register-resident batched
    CG walk corner rows past their prefetched slots too: a batch of the
    16-sided-cell tissue and a random one, run for a fixed number of
    relaxation steps and then differentiated with 512 threads, equals the
    single-tissue calls (the many-sided tissue is not at equilibrium, so its
    CG may stop at negative curvature: the same step either way)."""
    t0, p0 = _many_sided_tissue()
    t1, m1, X1, p1, _ = small_equilibria[0]  # an equilibrium (with T1) of the oracle
    t1 = g.Tissue(m1.he.copy(), X1.copy(), t1.Lx, t1.Ly)
    cases = [(t0, p0, 4000), (t1, p1, 1000)]
    singles = []
    for t, p, iters in cases:
        T = vtx.Tissue.from_tissue(t)
        X = _dev(t.X)
        P = vtx.Params.from_numpy(p)
        r = T.relax(X, P, mode="f64", eta=3e-3, tol=1e-9, max_iter=iters, t1_enable=False)
        b = _dev(np.random.default_rng(9).normal(size=t.X.shape))
        gs, info = T.param_grad(X, P, dC_dX=b, cg_tol=1e-10)
        singles.append((r, X.cpu().numpy(), b, gs.cpu().numpy(), info))
    assert singles[1][0]["status"] == 0 and singles[1][4]["status"] == 0
    Ts = [vtx.Tissue.from_tissue(t) for t, _, _ in cases]
    Ps = [vtx.Params.from_numpy(p) for _, p, _ in cases]
    Xs = []
    for (t, p, iters), T, P, (rs, Xref, _, _, _) in zip(cases, Ts, Ps, singles):
        X = _dev(t.X)
        r = vtx.Batch([T]).relax([X], [P], mode="f64", block_threads=512, eta=3e-3, tol=1e-9,
                                 max_iter=iters, t1_enable=False)[0]
        assert (r["status"], r["iters"]) == (rs["status"], rs["iters"])
        assert np.abs(X.cpu().numpy() - Xref).max() < 1e-9
        Xs.append(X)
    outs, infos = vtx.Batch(Ts).param_grad(Xs, Ps, dC_dX=[s[2] for s in singles],
                                           cg_tol=1e-10, block_threads=512)
    for (_, _, _, gref, iref), gb, inf in zip(singles, outs, infos):
        # the workgroup CG and the grid CG add their dot products in
        # different orders, so the step at which the residual crosses 1e-10
        # may differ by one
        assert inf["status"] == iref["status"]
        assert abs(inf["cg_iters"] - iref["cg_iters"]) <= 1, (inf, iref)
        assert np.abs(gb.cpu().numpy() - gref).max() < 1e-8 * np.abs(gref).max()


# ----------------------------------------------------------------------- T1

@pytest.mark.parametrize("mode", ["f64", "mixed"])
def test_t1_pass_bit_exact_topology(vtx, oracle, errlog, mode):
    t, p = g.workload_single_10k(n_cell=2000, seed=211)
    m = oracle.Mesh.from_tissue(t)
    X = t.X.copy()
    n_sw, n_st = oracle.t1_pass(m, X, p, 0.01, 0.02)
    assert n_sw > 0 and n_st > 0
    T = vtx.Tissue.from_tissue(t)
    Xd = _dev(t.X)
    # an evaluation before the pass: the pass must see (and later replace)
    # state left by earlier calls on the handle
    T.energy_forces(Xd, vtx.Params.from_numpy(p), mode="f64")
    a, b = T.t1(Xd, vtx.Params.from_numpy(p), 0.01, 0.02, mode=mode)
    assert (a, b) == (n_sw, n_st)
    errlog(f"T1 pass {mode}, 2000 cells: half-edge entries differing", (T.topology() != m.he).sum())
    errlog(f"T1 pass {mode}, 2000 cells: positions (max abs)", np.abs(Xd.cpu().numpy() - X).max())
    np.testing.assert_array_equal(T.topology(), m.he)
    assert np.abs(Xd.cpu().numpy() - X).max() < 1e-12
    # the staged layouts follow: forces after the pass match the oracle
    E, F, _ = T.energy_forces(Xd, vtx.Params.from_numpy(p), mode="f64")
    Eo, Fo = oracle.energy_forces(m, X, p)
    assert _force_err(F.cpu().numpy(), Fo) < 1e-10
    assert E.item() == pytest.approx(Eo, rel=1e-12)


def test_evaluation_after_topology_replaced(vtx, oracle):
    """set_topology to a T1-edited table: the next evaluation uses it."""
    t, p = g.workload_single_10k(n_cell=1500, seed=212)
    m = oracle.Mesh.from_tissue(t)
    X = t.X.copy()
    n_sw, _ = oracle.t1_pass(m, X, p, 0.01, 0.02)
    assert n_sw > 0
    T = vtx.Tissue.from_tissue(t)
    P = vtx.Params.from_numpy(p)
    T.energy_forces(_dev(t.X), P, mode="f64")
    T.set_topology(m.he)
    E, F, _ = T.energy_forces(_dev(X), P, mode="f64")
    Eo, Fo = oracle.energy_forces(m, X, p)
    assert _force_err(F.cpu().numpy(), Fo) < 1e-10
    assert E.item() == pytest.approx(Eo, rel=1e-12)


# ---------------------------------------------------------------- relaxation

def test_relax_fixed_iterations_f64(vtx, oracle):
    """100-cell tissue, P0 = 3.8, no line tension, no T1.  Without T1 this
    tissue never reaches an equilibrium (edges collapse and GD chatters), and
    the trajectory is chaotic after ~100 steps (a 1e-15 perturbation grows
    to 1e-8 by step 100 in the oracle itself), so 50 steps are compared."""
    t, p = g.workload_single_100()
    m = oracle.Mesh.from_tissue(t)
    X = t.X.copy()
    ro = oracle.relax(m, X, p, eta=1e-2, tol=0.0, patience=1, max_iter=50)
    T = vtx.Tissue.from_tissue(t)
    Xd = _dev(t.X)
    r = T.relax(Xd, vtx.Params(P0=3.8, lam=0.0), mode="f64", eta=1e-2, tol=0.0, max_iter=50,
                chunk=16)
    assert r["iters"] == ro["iters"] == 50 and r["status"] == 1
    assert np.abs(Xd.cpu().numpy() - X).max() < 1e-9
    assert r["max_f"] == pytest.approx(ro["max_f"], rel=1e-8)
    assert r["energy"] == pytest.approx(ro["energy"], rel=1e-12)


def test_relax_with_t1_to_equilibrium_f64(vtx, oracle, errlog):
    """100-cell tissue with T1 (l_min 0.01) relaxed to max |F| < 1e-6."""
    t, p = g.workload_single_100()
    m = oracle.Mesh.from_tissue(t)
    X = t.X.copy()
    ro = oracle.relax(m, X, p, eta=1e-2, tol=1e-6, patience=1, max_iter=200000,
                      t1_enable=True, l_min=0.01)
    assert ro["status"] == 0
    T = vtx.Tissue.from_tissue(t)
    Xd = _dev(t.X)
    r = T.relax(Xd, vtx.Params(P0=3.8, lam=0.0), mode="f64", eta=1e-2, tol=1e-6,
                max_iter=200000, t1_enable=True, l_min=0.01)
    print("gpu", r, "oracle", ro)
    assert r["status"] == 0
    assert (r["n_t1"], r["n_stretch"]) == (ro["n_t1"], ro["n_stretch"])
    np.testing.assert_array_equal(T.topology(), m.he)
    ell = oracle.edge_lengths(m, X).mean()
    d = Xd.cpu().numpy() - X
    d -= t.Lx * np.round(d / t.Lx)
    errlog("relaxed equilibrium f64, 100 cells with T1 (max |dX| / mean edge)", np.abs(d).max() / ell)
    assert np.abs(d).max() < 1e-4 * ell
    # the oracle confirms the returned state is an equilibrium
    _, Fo = oracle.energy_forces(m, Xd.cpu().numpy(), p)
    assert np.abs(Fo).max() < 1e-6


def test_relax_patience_and_stretch_length_f64(vtx, oracle):
    """Patience 10 (the paper's benchmark setting) and a T1 length of
    3 l_min instead of the default 2 l_min: iteration and event counts,
    topology and positions as the oracle's."""
    t, p = g.workload_single_100()
    m = oracle.Mesh.from_tissue(t)
    X = t.X.copy()
    opts = dict(eta=1e-2, tol=1e-6, max_iter=200000, t1_enable=True, l_min=0.01, l_new=0.03)
    ro = oracle.relax(m, X, p, patience=10, **opts)
    assert ro["status"] == 0 and ro["n_t1"] + ro["n_stretch"] > 0
    T = vtx.Tissue.from_tissue(t)
    Xd = _dev(t.X)
    r = T.relax(Xd, vtx.Params(P0=3.8, lam=0.0), mode="f64", patience=10, **opts)
    assert (r["status"], r["iters"], r["n_t1"], r["n_stretch"]) == \
        (ro["status"], ro["iters"], ro["n_t1"], ro["n_stretch"])
    np.testing.assert_array_equal(T.topology(), m.he)
    d = Xd.cpu().numpy() - X
    d -= t.Lx * np.round(d / t.Lx)
    assert np.abs(d).max() < 1e-4 * oracle.edge_lengths(m, X).mean()


def test_relax_10k_cells_full_size(vtx, oracle, errlog):
    """The 10^4-cell workload (P0 ~ U[3.6, 3.9] per cell, lambda ~ N(0.1,
    0.02^2), T1 below 0.01) at full size: the first 300 iterations in FP64
    against the oracle (every T1 event of the initial passes, bit-exact
    topology), then 2e4 MIXED iterations checked by properties: a valid
    3-valent periodic tiling with the box area, and the reported energy
    equal to the oracle's at the returned state."""
    t, p = g.workload_single_10k()
    P = vtx.Params.from_numpy(p)
    m = oracle.Mesh.from_tissue(t)
    X = t.X.copy()
    ro = oracle.relax(m, X, p, eta=3e-3, tol=0.0, patience=1, max_iter=300, t1_enable=True,
                      l_min=0.01)
    T = vtx.Tissue.from_tissue(t)
    Xd = _dev(t.X)
    r = T.relax(Xd, P, mode="f64", eta=3e-3, tol=0.0, max_iter=300, t1_enable=True, l_min=0.01)
    print("10k cells, 300 f64 iterations:", r, ro)
    assert ro["n_t1"] + ro["n_stretch"] > 100
    assert (r["iters"], r["n_t1"], r["n_stretch"]) == (ro["iters"], ro["n_t1"], ro["n_stretch"])
    np.testing.assert_array_equal(T.topology(), m.he)
    errlog("1e4 cells, 300 f64 steps with T1: positions (max abs)", np.abs(Xd.cpu().numpy() - X).max())
    assert np.abs(Xd.cpu().numpy() - X).max() < 1e-9
    # MIXED, longer
    T2 = vtx.Tissue.from_tissue(t)
    Xm = _dev(t.X)
    r2 = T2.relax(Xm, P, mode="mixed", eta=3e-3, tol=0.0, max_iter=20000, t1_enable=True,
                  l_min=0.01)
    he = T2.topology()
    m2 = oracle.Mesh(he, t.n_vert, t.Lx, t.Ly)
    Xh = Xm.cpu().numpy()
    A, Pc, ns = oracle.cells(m2, Xh)
    assert ns.sum() == he.shape[0] and np.bincount(he[:, 3], minlength=t.n_vert).min() == 3
    assert np.bincount(he[:, 3], minlength=t.n_vert).max() == 3 and ns.min() >= 3
    assert A.sum() == pytest.approx(t.Lx * t.Ly, rel=1e-12) and A.min() > 0
    Eo, Fo = oracle.energy_forces(m2, Xh, p)
    print("10k cells, 2e4 mixed iterations:", r2, "oracle E", Eo, "max|F|", np.abs(Fo).max())
    # the reported energy is that of the returned state (its line term summed
    # from FP32 lengths in MIXED mode)
    errlog("1e4 cells, 2e4 mixed steps: reported energy vs FP64 energy of the state (relative)",
           abs(r2["energy"] / Eo - 1))
    assert r2["energy"] == pytest.approx(Eo, rel=1e-7)


def test_relax_mixed_precision_reaches_tolerance(vtx, oracle, errlog):
    """10^3-cell tissue, FP32 force arithmetic on FP64 positions, T1 on."""
    t, p = g.workload_single_10k(n_cell=1000, seed=221)
    T = vtx.Tissue.from_tissue(t)
    Xd = _dev(t.X)
    r = T.relax(Xd, vtx.Params.from_numpy(p), mode="mixed", eta=3e-3, tol=1e-6,
                max_iter=2000000, t1_enable=True, l_min=0.01)
    print("mixed relax", r)
    assert r["status"] == 0
    m = oracle.Mesh(T.topology(), t.n_vert, t.Lx, t.Ly)
    _, Fo = oracle.energy_forces(m, Xd.cpu().numpy(), p)
    errlog("mixed relaxation to 1e-6, 1000 cells: FP64 max |F| of the returned state",
           np.abs(Fo).max())
    assert np.abs(Fo).max() < 2e-6          # FP64 forces of the FP32-relaxed state


# ------------------------------------------------------------------- adjoint

@pytest.fixture(scope="module")
def equilibrium(oracle):
    rng = np.random.default_rng(11)
    t = g.random_tissue(20, np.sqrt(20.0), rng=rng)
    p = g.uniform_params(t, P0=3.75)
    p.lam = rng.uniform(0.05, 0.15, t.n_edge)
    m = oracle.Mesh.from_tissue(t)
    X = t.X.copy()
    r = oracle.relax(m, X, p, eta=3e-3, tol=1e-11, patience=1, max_iter=400000,
                     t1_enable=True, l_min=0.01)
    assert r["status"] == 0
    Xt = X + rng.normal(0, 0.05, X.shape)
    return t, m, X, p, Xt


def test_hvp_f64(vtx, oracle, errlog, equilibrium):
    t, m, X, p, Xt = equilibrium
    rng = np.random.default_rng(3)
    v = rng.normal(size=X.shape)
    T = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
    Hv = T.hvp(_dev(X), vtx.Params.from_numpy(p), _dev(v)).cpu().numpy()
    Hvo = oracle.hvp(m, X, p, v)
    errlog("HVP f64 (max |d| / max)", np.abs(Hv - Hvo).max() / np.abs(Hvo).max())
    assert np.abs(Hv - Hvo).max() < 1e-10 * np.abs(Hvo).max()


@pytest.mark.parametrize("theta", ["lambda", "P0"])
def test_adjoint_gradient_f64(vtx, oracle, errlog, equilibrium, theta):
    t, m, X, p, Xt = equilibrium
    _, b = oracle.v2v(m, X, Xt)
    go, info_o = oracle.adjoint_grad(m, X, p, b, theta=theta, tol=1e-10)
    T = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
    gg, info = T.param_grad(_dev(X), vtx.Params.from_numpy(p), dC_dX=_dev(b), theta=theta,
                            cg_tol=1e-10)
    assert info["status"] == 0
    assert abs(info["cg_iters"] - info_o["iters"]) <= 2
    errlog(f"adjoint CG f64, theta={theta} (max |dg| / max |g|)",
           np.abs(gg.cpu().numpy() - go).max() / np.abs(go).max())
    assert np.abs(gg.cpu().numpy() - go).max() < 1e-7 * np.abs(go).max()


@pytest.mark.parametrize("theta", ["lambda", "P0"])
def test_adjoint_minres_f64(vtx, oracle, errlog, equilibrium, theta):
    t, m, X, p, Xt = equilibrium
    _, b = oracle.v2v(m, X, Xt)
    go, info_o = oracle.adjoint_grad(m, X, p, b, theta=theta, tol=1e-10, solver="minres")
    T = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
    gg, info = T.param_grad(_dev(X), vtx.Params.from_numpy(p), dC_dX=_dev(b), theta=theta,
                            method="adjoint_minres", cg_tol=1e-10)
    assert info["status"] == 0 and info_o["status"] == 0
    assert abs(info["cg_iters"] - info_o["iters"]) <= 2
    assert info["cg_rel_res"] <= 1e-10
    errlog(f"adjoint MINRES f64, theta={theta} (max |dg| / max |g|)",
           np.abs(gg.cpu().numpy() - go).max() / np.abs(go).max())
    assert np.abs(gg.cpu().numpy() - go).max() < 1e-7 * np.abs(go).max()


@pytest.mark.parametrize("seed", [11, 12])
def test_minres_sensitivity_at_indefinite_state(vtx, oracle, seed):
    """At an unrelaxed Voronoi state (H strongly indefinite) CG stops on
    negative curvature on both sides; MINRES matches the oracle's MINRES."""
    rng = np.random.default_rng(seed)
    t = g.random_tissue(20, np.sqrt(20.0), rng=rng)
    p = g.uniform_params(t, P0=3.75)
    p.lam = rng.uniform(0.05, 0.15, t.n_edge)
    m = oracle.Mesh.from_tissue(t)
    b = rng.normal(size=t.X.shape)
    d = rng.normal(size=t.n_edge)
    so, wo, io = oracle.sens_derivative(m, t.X, p, d, b, tol=1e-11, solver="minres")
    assert io["status"] == 0
    T = vtx.Tissue.from_tissue(t)
    P = vtx.Params.from_numpy(p)
    s, w, info = T.param_sens(_dev(t.X), P, _dev(d), _dev(b), cg_tol=1e-11, want_dX=True,
                              solver="minres")
    # Lanczos loses orthogonality over ~200 steps on this system, so the
    # summation order (the GPU's fixed tree against the oracle's loop) moves
    # the stopping step by a few percent
    assert info["status"] == 0 and abs(info["cg_iters"] - io["iters"]) <= 0.1 * io["iters"]
    assert s.item() == pytest.approx(so, rel=1e-7)
    assert np.abs(w.cpu().numpy() - wo).max() < 1e-7 * np.abs(wo).max()
    _, _, info_cg = T.param_sens(_dev(t.X), P, _dev(d), _dev(b), cg_tol=1e-11)
    assert info_cg["status"] == vtx.CG_NEG_CURVATURE


def test_ep_gradient_f64(vtx, oracle, errlog, equilibrium):
    t, m, X, p, Xt = equilibrium
    beta = 0.04
    go, _ = oracle.ep_grad(m, X, p, Xt, beta, eta=3e-3, tol=1e-12, patience=1, max_iter=400000)
    T = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
    gg, info = T.param_grad(_dev(X), vtx.Params.from_numpy(p), X_target=_dev(Xt),
                            method="ep", beta=beta,
                            ep_relax=dict(eta=3e-3, tol=1e-12, max_iter=400000))
    assert info["status"] == 0
    errlog("centred EP f64 vs the oracle's EP (max |dg| / max |g|)",
           np.abs(gg.cpu().numpy() - go).max() / np.abs(go).max())
    assert np.abs(gg.cpu().numpy() - go).max() < 1e-6 * np.abs(go).max()


@pytest.mark.parametrize("theta", ["lambda", "P0"])
@pytest.mark.parametrize("mode", ["f64", "mixed"])
def test_sensitivity_f64(vtx, oracle, errlog, equilibrium, theta, mode):
    """Forward ID along a random direction: value and dX*/dtheta . d against
    the oracle, and against the library's own adjoint gradient . d."""
    t, m, X, p, Xt = equilibrium
    _, b = oracle.v2v(m, X, Xt)
    rng = np.random.default_rng(23)
    d = rng.normal(size=m.n_edge if theta == "lambda" else m.n_cell)
    so, wo, info_o = oracle.sens_derivative(m, X, p, d, b, theta=theta, tol=1e-10)
    T = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
    P = vtx.Params.from_numpy(p)
    # MIXED runs the HVP with FP32 force arithmetic: its CG floors near 1e-7
    # and meets spurious non-positive curvature below that, so it solves to 1e-5
    s, w, info = T.param_sens(_dev(X), P, _dev(d), _dev(b), theta=theta, mode=mode,
                              cg_tol=1e-10 if mode == "f64" else 1e-5, want_dX=True)
    assert info["status"] == 0
    tol = 1e-7 if mode == "f64" else 1e-3
    if mode == "f64":
        assert abs(info["cg_iters"] - info_o["iters"]) <= 2
    errlog(f"Sen-ID {mode}, theta={theta}: derivative (relative)", abs(s.item() / so - 1))
    errlog(f"Sen-ID {mode}, theta={theta}: dX*/dtheta.d (max |d| / max)",
           np.abs(w.cpu().numpy() - wo).max() / np.abs(wo).max())
    assert s.item() == pytest.approx(so, rel=tol)
    assert np.abs(w.cpu().numpy() - wo).max() < tol * np.abs(wo).max()
    gg, _ = T.param_grad(_dev(X), P, dC_dX=_dev(b), theta=theta, cg_tol=1e-10)
    assert s.item() == pytest.approx(float(gg.cpu().numpy() @ d), rel=10 * tol)


def test_ep_forward_gradient_f64(vtx, oracle, errlog, equilibrium):
    t, m, X, p, Xt = equilibrium
    beta = 0.04
    go, _ = oracle.ep_grad_forward(m, X, p, Xt, beta, eta=3e-3, tol=1e-12, patience=1,
                                   max_iter=400000)
    T = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
    gg, info = T.param_grad(_dev(X), vtx.Params.from_numpy(p), X_target=_dev(Xt),
                            method="ep_forward", beta=beta,
                            ep_relax=dict(eta=3e-3, tol=1e-12, max_iter=400000))
    assert info["status"] == 0 and info["ep_minus"]["iters"] == 0
    errlog("first-order EP f64 vs the oracle's (max |dg| / max |g|)",
           np.abs(gg.cpu().numpy() - go).max() / np.abs(go).max())
    assert np.abs(gg.cpu().numpy() - go).max() < 1e-6 * np.abs(go).max()


def test_inverse_workload_full_size_gradients(vtx, oracle, errlog):
    """One tissue of the 64 x 1000-cell inverse workload at full size: target
    and prediction relaxed on the GPU (FP64, T1), then the adjoint (CG, tol
    1e-8) and a Sen-ID directional derivative against the oracle's at the
    same state and topology."""
    t, ps, pi = g.workload_inverse(n_tissue=1)[0]
    opts = dict(eta=3e-3, tol=1e-6, max_iter=2000000, t1_enable=True, l_min=0.01)
    Tt = vtx.Tissue.from_tissue(t)
    Xt = _dev(t.X)
    assert Tt.relax(Xt, vtx.Params.from_numpy(ps), mode="f64", **opts)["status"] == 0
    T = vtx.Tissue.from_tissue(t)
    X = _dev(t.X)
    P = vtx.Params.from_numpy(pi)
    assert T.relax(X, P, mode="f64", **opts)["status"] == 0
    _, b = T.v2v(X, Xt)
    gg, info = T.param_grad(X, P, dC_dX=b, cg_tol=1e-8)
    m = oracle.Mesh(T.topology(), t.n_vert, t.Lx, t.Ly)
    Xh, bh = X.cpu().numpy(), b.cpu().numpy()
    go, info_o = oracle.adjoint_grad(m, Xh, pi, bh, tol=1e-8)
    print("1000 cells adjoint:", info, info_o)
    assert info["status"] == 0 and info_o["status"] == 0
    assert abs(info["cg_iters"] - info_o["iters"]) <= 0.05 * info_o["iters"]
    errlog("adjoint CG f64, 1000-cell inverse workload, tol 1e-8 (max |dg| / max |g|)",
           np.abs(gg.cpu().numpy() - go).max() / np.abs(go).max())
    assert np.abs(gg.cpu().numpy() - go).max() < 1e-6 * np.abs(go).max()
    rng = np.random.default_rng(5)
    d = rng.normal(size=t.n_edge)
    sv, _, _ = T.param_sens(X, P, _dev(d), b, cg_tol=1e-8)
    so, _, _ = oracle.sens_derivative(m, Xh, pi, d, bh, tol=1e-8)
    errlog("Sen-ID f64, 1000-cell inverse workload (relative)", abs(sv.item() / so - 1))
    assert sv.item() == pytest.approx(so, rel=1e-6)


# ------------------------------------------------------------------- batched

def test_batched_adjoint_full_size_64_tissues(vtx, oracle, errlog):
    """The inverse workload at full size (64 tissues of 1000 cells): targets
    and predictions relaxed in one batch each (FP64, T1), then the batched
    adjoint in the benchmark's configuration (the library's choice, the
    register-resident CG at 512 threads; CG to 1e-8); two sampled tissues
    against the oracle's adjoint at the same state and topology."""
    work = g.workload_inverse()
    assert len(work) == 64
    opts = dict(eta=3e-3, tol=1e-6, max_iter=2000000, t1_enable=True, l_min=0.01)
    Tt = [vtx.Tissue.from_tissue(t) for t, _, _ in work]
    T = [vtx.Tissue.from_tissue(t) for t, _, _ in work]
    Xt = [_dev(t.X) for t, _, _ in work]
    X = [_dev(t.X) for t, _, _ in work]
    P = [vtx.Params.from_numpy(pi) for _, _, pi in work]
    rt = vtx.Batch(Tt).relax(Xt, [vtx.Params.from_numpy(ps) for _, ps, _ in work], mode="f64",
                             **opts)
    r = vtx.Batch(T).relax(X, P, mode="f64", **opts)
    assert all(x["status"] == 0 for x in rt + r)
    b = [Ti.v2v(Xi, Yi)[1] for Ti, Xi, Yi in zip(T, X, Xt)]
    grads, infos = vtx.Batch(T).param_grad(X, P, dC_dX=b, cg_tol=1e-8)
    assert all(i["status"] == 0 for i in infos)
    for k in (0, 37):
        t, _, pi = work[k]
        m = oracle.Mesh(T[k].topology(), t.n_vert, t.Lx, t.Ly)
        go, info_o = oracle.adjoint_grad(m, X[k].cpu().numpy(), pi, b[k].cpu().numpy(), tol=1e-8)
        assert info_o["status"] == 0
        err = np.abs(grads[k].cpu().numpy() - go).max() / np.abs(go).max()
        errlog(f"batched adjoint f64, inverse workload at full size, tissue {k} (max |dg| / "
               "max |g|)", err)
        assert err < 1e-6


def test_batched_relax_full_size_512_tissues(vtx, oracle, errlog):
    """The 512-tissue workload at full size (64-4096 cells per tissue) in the
    benchmark's launch configuration (one persistent launch, a 1024-thread
    workgroup per tissue, T1 on), capped at 300 iterations and in FP64: the
    smallest, a median and the largest tissue of the batch equal the
    oracle's relaxation of the same tissue, topology bit-exact.  (The
    benchmark's MIXED run differs from FP64 by FP32 force rounding, which can
    move a T1 decision at the threshold, so it is compared at the force level
    elsewhere.)"""
    work = g.workload_batch()
    assert len(work) == 512
    sizes = np.array([t.n_cell for t, _ in work])
    picks = [int(sizes.argmin()), int(np.argsort(sizes)[len(sizes) // 2]), int(sizes.argmax())]
    opts = dict(eta=3e-3, tol=1e-6, max_iter=300, t1_enable=True, l_min=0.01)
    Ts = [vtx.Tissue.from_tissue(t) for t, _ in work]
    Xs = [_dev(t.X) for t, _ in work]
    Ps = [vtx.Params.from_numpy(p) for _, p in work]
    res = vtx.Batch(Ts).relax(Xs, Ps, mode="f64", block_threads=1024, **opts)
    assert all(r["iters"] == 300 or r["status"] == 0 for r in res)
    for i in picks:
        t, p = work[i]
        m = oracle.Mesh.from_tissue(t)
        X = t.X.copy()
        ro = oracle.relax(m, X, p, patience=1, **opts)
        r = res[i]
        assert (r["iters"], r["n_t1"], r["n_stretch"], r["status"]) == (
            ro["iters"], ro["n_t1"], ro["n_stretch"], ro["status"])
        np.testing.assert_array_equal(Ts[i].topology(), m.he)
        d = np.abs(Xs[i].cpu().numpy() - X).max()
        errlog(f"batched relaxation, 512-tissue workload, {t.n_cell}-cell tissue, 300 FP64 "
               "steps with T1: positions against the oracle (max abs)", d)
        assert d < 1e-9
        assert r["energy"] == pytest.approx(ro["energy"], rel=1e-10)


def _batch_case(rng, n, P0):
    t = g.random_tissue(n, np.sqrt(n), rng=rng)
    p = g.uniform_params(t, P0=P0)
    p.lam = rng.uniform(0.0, 0.2, t.n_edge)
    return t, p


@pytest.mark.parametrize("block_threads", [256, 512])
@pytest.mark.parametrize("mode", ["f64", "mixed", "f32"])
def test_batch_relax_matches_single(vtx, oracle, errlog, mode, block_threads):
    """Solid tissues (P0 < 3.8; some converge within the iteration cap, some
    do not yet) plus one fluid tissue (P0 = 3.86) that keeps cycling short
    edges and stops at max_iter: the persistent batch kernel reproduces the
    single-tissue path exactly in every case.  With 512 threads these
    tissues run in the LDS-resident kernel, T1 passes included."""
    rng = np.random.default_rng(41)
    cases = [_batch_case(rng, n, P0) for n, P0 in
             ((64, 3.65), (150, 3.70), (90, 3.63), (300, 3.72), (120, 3.86))]
    opts = dict(eta=3e-3, tol=1e-6, max_iter=60000, t1_enable=True, l_min=0.01)
    dt = vtx.pos_dtype(mode)
    single = []
    for t, p in cases:
        T = vtx.Tissue.from_tissue(t)
        Xd = _dev(t.X, dt)
        r = T.relax(Xd, vtx.Params.from_numpy(p, dtype=dt), mode=mode, **opts)
        single.append((r, Xd.cpu().numpy(), T.topology()))
    Ts = [vtx.Tissue.from_tissue(t) for t, _ in cases]
    Xs = [_dev(t.X, dt) for t, _ in cases]
    B = vtx.Batch(Ts)
    res = B.relax(Xs, [vtx.Params.from_numpy(p, dtype=dt) for _, p in cases], mode=mode,
                  block_threads=block_threads, **opts)
    for (rs, Xs_ref, he_ref), r, X, T in zip(single, res, Xs, Ts):
        print("single", rs, "batch", r)
        assert r["status"] == rs["status"]
        assert (r["iters"], r["n_t1"], r["n_stretch"]) == (rs["iters"], rs["n_t1"], rs["n_stretch"])
        np.testing.assert_array_equal(T.topology(), he_ref)
        errlog(f"batched vs single relaxation {mode}, {block_threads} threads, {T.n_cell} cells: "
               "positions (max abs)", np.abs(X.cpu().numpy() - Xs_ref).max())
        assert np.abs(X.cpu().numpy() - Xs_ref).max() < 1e-9
        # the single path sums the line energy from FP32 lengths in MIXED mode
        assert r["energy"] == pytest.approx(
            rs["energy"], rel={"f64": 1e-9, "mixed": 1e-7, "f32": 1e-6}[mode])
    # evaluations after the batched T1 passes use the new topologies (at
    # perturbed positions: equilibrium forces are pure cancellation)
    for (t, p), X, T in zip(cases, Xs, Ts):
        m = oracle.Mesh.from_tissue(t)
        m.he[:] = T.topology()
        Xh = X.double().cpu().numpy() + rng.normal(0, 0.02, t.X.shape)
        _, F, _ = T.energy_forces(_dev(Xh), vtx.Params.from_numpy(p), mode="f64")
        _, Fo = oracle.energy_forces(m, Xh, p)
        assert _force_err(F.cpu().numpy(), Fo) < 1e-10
    st = [r["status"] for r in res]
    if mode != "f32":  # FP32 positions need not resolve a 1e-6 force tolerance
        assert st[0] == 0 and st[2] == 0 and st[4] == 1


@pytest.mark.parametrize("mode", ["f64", "mixed", "f32"])
def test_batch_relax_without_t1_in_lds(vtx, errlog, mode):
    """Without T1 and with 512 threads, a batch of tissues of 64-1000 cells
    runs in the LDS-resident relaxation kernel and a batch that also holds a
    1100-cell tissue (more than two cells per thread) in the general one:
    both reproduce the single-tissue path."""
    rng = np.random.default_rng(43)
    cases = [_batch_case(rng, n, P0) for n, P0 in ((64, 3.65), (300, 3.70), (1000, 3.72))]
    big = _batch_case(rng, 1100, 3.70)
    opts = dict(eta=3e-3, tol=1e-6, max_iter=20000, t1_enable=False)
    dt = vtx.pos_dtype(mode)
    refs = {}
    for k, (t, p) in enumerate(cases + [big]):
        T = vtx.Tissue.from_tissue(t)
        Xd = _dev(t.X, dt)
        r = T.relax(Xd, vtx.Params.from_numpy(p, dtype=dt), mode=mode, **opts)
        refs[k] = (r, Xd.cpu().numpy())
    for batch in (cases, cases + [big]):
        Ts = [vtx.Tissue.from_tissue(t) for t, _ in batch]
        Xs = [_dev(t.X, dt) for t, _ in batch]
        res = vtx.Batch(Ts).relax(Xs, [vtx.Params.from_numpy(p, dtype=dt) for _, p in batch],
                                  mode=mode, block_threads=512, **opts)
        for k, (r, X) in enumerate(zip(res, Xs)):
            rs, Xref = refs[k]
            assert (r["status"], r["iters"]) == (rs["status"], rs["iters"])
            d = np.abs(X.cpu().numpy() - Xref).max()
            errlog(f"batched (LDS-resident when it fits) vs single relaxation without T1, {mode}, "
                   f"{Ts[k].n_cell} cells: positions (max abs)", d)
            assert d < 1e-9
            assert r["energy"] == pytest.approx(
                rs["energy"], rel={"f64": 1e-9, "mixed": 1e-7, "f32": 1e-6}[mode])


def test_split_passes_equal_full_evaluation(vtx, oracle):
    t, p = g.workload_single_10k(n_cell=3000, seed=5)
    T = vtx.Tissue.from_tissue(t)
    for mode, dt in (("f32", torch.float32), ("f64", torch.float64), ("mixed", torch.float64)):
        Xd = _dev(t.X, dt)
        P = vtx.Params.from_numpy(p, dtype=dt)
        _, F, _ = T.energy_forces(Xd, P, mode=mode)
        cf = T.cell_coeffs(Xd, P, mode=mode)
        F2, mf = T.vertex_forces(Xd, P, cf, mode=mode, want_maxf=True)
        assert torch.equal(F, F2)
        assert mf.item() == F.abs().max().item()
    # the coefficients are -pressure and tension: 2K_A(A-A0), 2K_P(P-P0)
    Xd = _dev(t.X)
    cf = T.cell_coeffs(Xd, vtx.Params.from_numpy(p), mode="f64").cpu().numpy()
    A, P_, _ = oracle.cells(oracle.Mesh.from_tissue(t), t.X)
    np.testing.assert_allclose(cf[:, 0], 2 * p.KA * (A - p.A0), rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(cf[:, 1], 2 * p.KP * (P_ - p.P0), rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("mode", ["f32", "mixed", "f64"])
def test_fused_evaluation_follows_topology(vtx, oracle, errlog, mode):
    """The fused evaluation (one launch per 256-vertex tile) keeps its tile
    tables in step with the topology: after T1 relaxations, single and
    batched, its forces equal the two-pass evaluation bit for bit, its
    energy equals the oracle's on the edited topology, and a graph captured
    before the topology changed replays to the eager result."""
    dt = vtx.pos_dtype(mode)
    t, p = g.workload_single_10k(n_cell=2000, seed=213)
    T = vtx.Tissue.from_tissue(t)
    P = vtx.Params.from_numpy(p, dtype=dt)
    cp, keep = P.to_c(dt, torch.device("cuda"))
    Xd = _dev(t.X, dt)
    E = torch.empty((), dtype=torch.float64, device="cuda")
    F = torch.empty_like(Xd)
    mf = torch.empty((), dtype=torch.float64, device="cuda")
    T.energy_forces_into(Xd, cp, E, F, mf, mode=mode)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        T.energy_forces_into(Xd, cp, E, F, mf, mode=mode)
    torch.cuda.current_stream().wait_stream(s)
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        T.energy_forces_into(Xd, cp, E, F, mf, mode=mode)
    r = T.relax(Xd, P, mode=mode, eta=3e-3, tol=1e-6, max_iter=3000, t1_enable=True, l_min=0.01)
    assert r["n_t1"] > 0, r

    def check(Ti, Xi, Pi, ti_p):
        E1, F1, m1 = Ti.energy_forces(Xi, Pi, mode=mode, want_maxf=True)
        cf = Ti.cell_coeffs(Xi, Pi, mode=mode)
        F2, _ = Ti.vertex_forces(Xi, Pi, cf, mode=mode, want_maxf=True)
        assert torch.equal(F1, F2)
        assert m1.item() == F1.abs().max().item()
        m = oracle.Mesh(Ti.topology(), Ti.n_vert, Ti.Lx, Ti.Ly)
        Eo, _ = oracle.energy_forces(m, Xi.double().cpu().numpy(), ti_p)
        return E1, F1, abs(E1.item() - Eo) / abs(Eo)

    E1, F1, rel = check(T, Xd, P, p)
    errlog(f"fused evaluation {mode} after T1 relaxation: energy against the oracle "
           "(relative)", rel)
    assert rel < {"f32": 1e-5, "mixed": 1e-6, "f64": 1e-12}[mode]
    gr.replay()
    torch.cuda.synchronize()
    assert torch.equal(F, F1) and E.item() == E1.item() and mf.item() == F1.abs().max().item()
    # batched relaxation with T1, three tissues (one of them ragged: 301 cells)
    rng = np.random.default_rng(214)
    cases = [_batch_case(rng, n, P0) for n, P0 in ((301, 3.70), (700, 3.65), (1000, 3.72))]
    Ts = [vtx.Tissue.from_tissue(tc) for tc, _ in cases]
    Xs = [_dev(tc.X, dt) for tc, _ in cases]
    Ps = [vtx.Params.from_numpy(pc, dtype=dt) for _, pc in cases]
    res = vtx.Batch(Ts).relax(Xs, Ps, mode=mode, eta=3e-3, tol=1e-6, max_iter=3000,
                              t1_enable=True, l_min=0.01)
    assert sum(r["n_t1"] for r in res) > 0
    for Ti, Xi, Pi, (_, pc) in zip(Ts, Xs, Ps, cases):
        _, _, rel = check(Ti, Xi, Pi, pc)
        assert rel < {"f32": 1e-5, "mixed": 1e-6, "f64": 1e-12}[mode]


@pytest.mark.parametrize("mode", ["f32", "mixed", "f64"])
def test_fused_evaluation_global_path_tiles(vtx, oracle, errlog, mode):
    """Tiles whose halo or corner rows overflow their fixed slots take the
    fused kernel's global-memory path.  Shuffled vertex ids scatter each
    tile over the box, which sends every tile there; shuffling only the
    second half mixes both kinds in one launch.  The forces equal the two
    passes bit for bit and the energy and forces the oracle's."""
    dt = vtx.pos_dtype(mode)
    t, p = g.workload_single_10k(n_cell=3000, seed=215)
    rng = np.random.default_rng(216)
    nv = t.n_vert
    for part in ("all", "half"):
        perm = np.arange(nv)
        if part == "all":
            perm = rng.permutation(nv)
        else:
            perm[nv // 2:] = nv // 2 + rng.permutation(nv - nv // 2)
        he = t.he.copy()
        he[:, g.HE_SRC] = perm[t.he[:, g.HE_SRC]]
        he[:, g.HE_TGT] = perm[t.he[:, g.HE_TGT]]
        X = np.empty_like(t.X)
        X[perm] = t.X
        T = vtx.Tissue(he, nv, t.Lx, t.Ly)
        ts = T.tile_stats()
        print(part, ts)
        assert ts["global_tiles"] > 0
        assert part == "all" or ts["global_tiles"] < ts["tiles"]
        Xd = _dev(X, dt)
        P = vtx.Params.from_numpy(p, dtype=dt)
        E, F, mf = T.energy_forces(Xd, P, mode=mode, want_maxf=True)
        cf = T.cell_coeffs(Xd, P, mode=mode)
        F2, _ = T.vertex_forces(Xd, P, cf, mode=mode, want_maxf=True)
        assert torch.equal(F, F2)
        assert mf.item() == F.abs().max().item()
        m = oracle.Mesh(he, nv, t.Lx, t.Ly)
        Eo, Fo = oracle.energy_forces(m, Xd.double().cpu().numpy(), p)
        rel = abs(E.item() - Eo) / abs(Eo)
        ferr = _force_err(F.double().cpu().numpy(), Fo)
        errlog(f"fused evaluation {mode}, global-path tiles ({part} shuffled): energy "
               "against the oracle (relative)", rel)
        errlog(f"fused evaluation {mode}, global-path tiles ({part} shuffled): forces "
               "(max |dF| / max |F|)", ferr)
        assert rel < {"f32": 1e-5, "mixed": 1e-6, "f64": 1e-12}[mode]
        assert ferr < {"f32": 1e-5, "mixed": 1e-5, "f64": 1e-10}[mode]


def test_batch_schedules_agree(vtx):
    """The persistent schedule (256 and 1024 threads per tissue), the grid
    schedule and the autotuned choice give the same relaxations."""
    rng = np.random.default_rng(43)
    cases = [_batch_case(rng, n, P0) for n, P0 in ((64, 3.65), (200, 3.70), (120, 3.68))]
    opts = dict(eta=3e-3, tol=1e-6, max_iter=20000, t1_enable=True, l_min=0.01)
    runs = []
    for sched, bt in ((vtx.SCHED_PERSISTENT, 256), (vtx.SCHED_PERSISTENT, 1024),
                      (vtx.SCHED_GRID, 256), (vtx.SCHED_AUTO, 256)):
        Ts = [vtx.Tissue.from_tissue(t) for t, _ in cases]
        Xs = [_dev(t.X) for t, _ in cases]
        B = vtx.Batch(Ts)
        ps = [vtx.Params.from_numpy(p) for _, p in cases]
        if sched == vtx.SCHED_AUTO:
            X0 = [X.clone() for X in Xs]
            sch, bt_best, ms = B.autotune(Xs, ps, mode="mixed", trial_iters=100, **opts)
            print("autotune", sch, bt_best, ms)
            assert sch in (vtx.SCHED_PERSISTENT, vtx.SCHED_GRID)
            assert bt_best in ((256, 512, 1024) if sch == vtx.SCHED_PERSISTENT else (0,))
            assert all(m > 0 for m in ms[:4]) and ms[4:] == [-1.0] * 3   # T1 on: no split
            assert all(torch.equal(a, b) for a, b in zip(X0, Xs))  # trials leave X alone
        res = B.relax(Xs, ps, mode="mixed", schedule=sched, block_threads=bt, **opts)
        runs.append((res, [X.cpu().numpy() for X in Xs], [T.topology() for T in Ts]))
    ref = runs[0]
    for res, Xh, he in runs[1:]:
        for r0, r, x0, x, h0, h in zip(ref[0], res, ref[1], Xh, ref[2], he):
            assert (r["status"], r["iters"], r["n_t1"], r["n_stretch"]) == \
                (r0["status"], r0["iters"], r0["n_t1"], r0["n_stretch"])
            np.testing.assert_array_equal(h, h0)
            assert np.abs(x - x0).max() < 1e-9
            assert r["energy"] == pytest.approx(r0["energy"], rel=1e-7)


@pytest.mark.parametrize("mode", ["f64", "mixed", "f32"])
def test_batch_relax_split_schedule(vtx, errlog, mode):
    """The split schedule (T1 off; each tissue over K cooperating
    workgroups) reproduces the single-tissue relaxation bit for bit for
    K = 1, 2, 4, 8 and the library's choice, on tissues of 64 to 2600 cells
    (with K = 1 the tissues of more than 1024 vertices fall back to the
    persistent kernel); the autotuner then also times it."""
    rng = np.random.default_rng(47)
    cases = [_batch_case(rng, n, P0) for n, P0 in
             ((64, 3.65), (300, 3.70), (1000, 3.72), (2600, 3.68))]
    opts = dict(eta=3e-3, tol=1e-6, max_iter=8000, t1_enable=False)
    dt = vtx.pos_dtype(mode)
    refs = []
    for t, p in cases:
        T = vtx.Tissue.from_tissue(t)
        Xd = _dev(t.X, dt)
        r = T.relax(Xd, vtx.Params.from_numpy(p, dtype=dt), mode=mode, **opts)
        refs.append((r, Xd.cpu().numpy()))
    Ps = [vtx.Params.from_numpy(p, dtype=dt) for _, p in cases]
    for K in (1, 2, 4, 8, 0):
        Ts = [vtx.Tissue.from_tissue(t) for t, _ in cases]
        Xs = [_dev(t.X, dt) for t, _ in cases]
        res = vtx.Batch(Ts).relax(Xs, Ps, mode=mode, schedule=vtx.SCHED_SPLIT,
                                  block_threads=K, **opts)
        for (rs, Xref), r, X, (t, _) in zip(refs, res, Xs, cases):
            assert (r["status"], r["iters"]) == (rs["status"], rs["iters"]), (K, t.n_cell, r, rs)
            d = np.abs(X.cpu().numpy() - Xref).max()
            errlog(f"split relaxation {mode}, K={K}, {t.n_cell} cells: positions against the "
                   "single path (max abs)", d)
            assert d == 0.0
            assert r["energy"] == pytest.approx(
                rs["energy"], rel={"f64": 1e-10, "mixed": 1e-7, "f32": 1e-6}[mode])
    Ts = [vtx.Tissue.from_tissue(t) for t, _ in cases]
    Xs = [_dev(t.X, dt) for t, _ in cases]
    sch, bt, ms = vtx.Batch(Ts).autotune(Xs, Ps, mode=mode, trial_iters=100, **opts)
    print("autotune without T1", sch, bt, ms)
    assert all(m > 0 for m in ms)
    assert sch != vtx.SCHED_SPLIT or bt in (2, 4, 8)
    with pytest.raises(vtx.VtxError):
        vtx.Batch(Ts).relax(Xs, Ps, mode=mode, schedule=vtx.SCHED_SPLIT, block_threads=4,
                            eta=3e-3, tol=1e-6, max_iter=10, t1_enable=True, l_min=0.01)


# --------------------------------------------------- batched hypergradients

@pytest.fixture(scope="module")
def small_equilibria(oracle):
    out = []
    for seed in (11, 12, 13):
        rng = np.random.default_rng(seed)
        t = g.random_tissue(20, np.sqrt(20.0), rng=rng)
        p = g.uniform_params(t, P0=3.75)
        p.lam = rng.uniform(0.05, 0.15, t.n_edge)
        m = oracle.Mesh.from_tissue(t)
        X = t.X.copy()
        r = oracle.relax(m, X, p, eta=3e-3, tol=1e-11, patience=1, max_iter=400000,
                         t1_enable=True, l_min=0.01)
        assert r["status"] == 0
        Xt = X + rng.normal(0, 0.05, X.shape)
        out.append((t, m, X, p, Xt))
    return out


@pytest.mark.parametrize("block_threads", [1024, 512])
@pytest.mark.parametrize("solver", ["cg", "minres"])
@pytest.mark.parametrize("theta", ["lambda", "P0"])
def test_batch_adjoint_matches_single_and_oracle(vtx, oracle, errlog, small_equilibria, theta,
                                                 solver, block_threads):
    """Workgroups of 512 threads solve these tissues with CG in the
    register-resident form, 1024-thread ones in the general loop."""
    method = "adjoint" if solver == "cg" else "adjoint_minres"
    Ts, Xs, Ps, bs, refs = [], [], [], [], []
    for t, m, X, p, Xt in small_equilibria:
        T = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
        _, b = oracle.v2v(m, X, Xt)
        go, _ = oracle.adjoint_grad(m, X, p, b, theta=theta, tol=1e-10, solver=solver)
        gs, _ = T.param_grad(_dev(X), vtx.Params.from_numpy(p), dC_dX=_dev(b), theta=theta,
                             cg_tol=1e-10, method=method)
        Ts.append(T); Xs.append(_dev(X)); Ps.append(vtx.Params.from_numpy(p)); bs.append(_dev(b))
        refs.append((go, gs.cpu().numpy()))
    B = vtx.Batch(Ts)
    outs, infos = B.param_grad(Xs, Ps, dC_dX=bs, theta=theta, cg_tol=1e-10, method=method,
                               block_threads=block_threads)
    worst = 0.0
    for (go, gsingle), gb, inf in zip(refs, outs, infos):
        assert inf["status"] == 0
        gb = gb.cpu().numpy()
        worst = max(worst, np.abs(gb - go).max() / np.abs(go).max())
        assert np.abs(gb - gsingle).max() < 1e-9 * np.abs(go).max()
        assert np.abs(gb - go).max() < 1e-7 * np.abs(go).max()
    errlog(f"batched adjoint {solver} f64, theta={theta}, {block_threads} threads "
           "(max |dg| / max |g|, worst tissue)", worst)


@pytest.mark.parametrize("block_threads", [1024, 512])
@pytest.mark.parametrize("mode", ["mixed", "f32"])
def test_batch_adjoint_reduced_precision(vtx, errlog, small_equilibria, mode, block_threads):
    """The batched adjoint in MIXED and FP32 (FP32 Hessian products, FP64
    dots), in the general loop (1024 threads) and the register-resident form
    (512), equals the single-tissue solve in the same precision, and stays
    within that precision of the FP64 gradient."""
    dt = vtx.pos_dtype(mode)
    Ts, Xs, Ps, bs, singles, refs = [], [], [], [], [], []
    for t, m, X, p, Xt in small_equilibria:
        T = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
        b = _dev(np.random.default_rng(7).normal(size=X.shape))
        g64, _ = T.param_grad(_dev(X), vtx.Params.from_numpy(p), dC_dX=b, cg_tol=1e-10)
        P = vtx.Params.from_numpy(p, dtype=dt)
        gs, info = T.param_grad(_dev(X, dt), P, dC_dX=b, mode=mode, cg_tol=1e-5)
        assert info["status"] == 0, info
        Ts.append(T); Xs.append(_dev(X, dt)); Ps.append(P); bs.append(b)
        singles.append((gs.cpu().numpy(), info)); refs.append(g64.cpu().numpy())
    outs, infos = vtx.Batch(Ts).param_grad(Xs, Ps, dC_dX=bs, mode=mode, cg_tol=1e-5,
                                           block_threads=block_threads)
    worst = 0.0
    for (gs, info), g64, gb, inf in zip(singles, refs, outs, infos):
        assert inf["status"] == 0, inf
        gb = gb.cpu().numpy()
        assert np.abs(gb - gs).max() < 1e-4 * np.abs(gs).max()
        worst = max(worst, np.abs(gb - g64).max() / np.abs(g64).max())
        assert np.abs(gb - g64).max() < 1e-3 * np.abs(g64).max()
    errlog(f"batched adjoint {mode}, {block_threads} threads, CG to 1e-5: against the FP64 "
           "gradient (max |dg| / max |g|, worst tissue)", worst)


@pytest.mark.parametrize("block_threads", [1024, 512, 256])
def test_batch_adjoint_lds_and_global_paths(vtx, block_threads):
    """One batch holding tissues whose Hessian-product arrays fit in the
    workgroup's LDS (120 and 1088 cells) and one that does not (2600 cells in
    FP64: positions, vector and two cell-coefficient pairs take ~250 KB): all
    equal the single-tissue solve.  With 512 or 256 threads the 120-cell
    tissue takes the register-resident CG and the 1088-cell one (more cells
    than two per thread) the general loop in LDS."""
    rng = np.random.default_rng(61)
    s = np.sqrt(2.0 / (3.0 * np.sqrt(3.0)))  # unit-area hexagons
    Ts, Xs, Ps, bs, singles = [], [], [], [], []
    for nx, ny in [(12, 10), (34, 32), (52, 50)]:
        t = g.hex_lattice(nx, ny, s)
        need = 32 * t.n_vert + 32 * t.n_cell  # FP64 bytes of the four arrays
        assert need < 150 * 1024 if nx < 52 else need > 160 * 1024
        # the regular tiling with uniform tension is an equilibrium by
        # symmetry, and a stable one below the hexagon's shape index 3.72
        p = g.uniform_params(t, P0=3.7)
        p.lam = np.full(t.n_edge, 0.1)
        T = vtx.Tissue.from_tissue(t)
        P = vtx.Params.from_numpy(p)
        X = _dev(t.X)
        _, _, maxf = T.energy_forces(X, P, mode="f64", want_maxf=True)
        assert float(maxf) < 1e-9
        b = T.v2v(X, X + _dev(rng.normal(0, 0.05, t.X.shape)))[1]
        gs, info = T.param_grad(X, P, dC_dX=b, cg_tol=1e-10)
        assert info["status"] == 0, info
        Ts.append(T); Xs.append(X); Ps.append(P); bs.append(b); singles.append(gs.cpu().numpy())
    outs, infos = vtx.Batch(Ts).param_grad(Xs, Ps, dC_dX=bs, cg_tol=1e-10,
                                           block_threads=block_threads)
    for gsingle, gb, inf in zip(singles, outs, infos):
        assert inf["status"] == 0, inf
        assert np.abs(gb.cpu().numpy() - gsingle).max() < 1e-7 * np.abs(gsingle).max()
    if block_threads == 1024:
        # the library's own choice gives the same gradients
        outs0, infos0 = vtx.Batch(Ts).param_grad(Xs, Ps, dC_dX=bs, cg_tol=1e-10, block_threads=0)
        for a, b_, inf in zip(outs0, outs, infos0):
            assert inf["status"] == 0, inf
            assert float((a - b_).abs().max()) < 1e-7 * float(b_.abs().max())
        with pytest.raises(vtx.VtxError) as err:
            vtx.Batch(Ts).param_grad(Xs, Ps, dC_dX=bs, cg_tol=1e-10, block_threads=128)
        assert err.value.code == -1


def test_side_count_cell_order_on_ragged_tissues(vtx, oracle, errlog):
    """The LDS-resident relaxation and the register-resident CG give each
    thread one cell from each end of the cells sorted by side count.  On
    random tissues of odd cell counts (runs of unequal length; 3- to
    11-sided cells): the batched relaxation with T1 equals the
    single-tissue loop bit for bit (positions, topology, step and T1
    counts), and the batched adjoint at its end points equals the
    single-tissue (grid kernel) solve and, on the two smallest, the
    oracle."""
    rng = np.random.default_rng(71)
    cases = []
    for n in (9, 21, 333):
        t = g.random_tissue(n, np.sqrt(n), rng=rng)
        p = g.uniform_params(t, P0=3.7)
        p.lam = rng.uniform(0.05, 0.15, t.n_edge)
        cases.append((t, p))
    opts = dict(eta=3e-3, tol=1e-9, max_iter=400000, t1_enable=True, l_min=0.01)
    Ps = [vtx.Params.from_numpy(p) for _, p in cases]
    Ts, Xs, rs = [], [], []
    for (t, _), P in zip(cases, Ps):
        T = vtx.Tissue.from_tissue(t)
        X = _dev(t.X)
        rs.append(T.relax(X, P, mode="f64", **opts))
        Ts.append(T); Xs.append(X)
    Tb = [vtx.Tissue.from_tissue(t) for t, _ in cases]
    Xb = [_dev(t.X) for t, _ in cases]
    res = vtx.Batch(Tb).relax(Xb, Ps, mode="f64", block_threads=512, **opts)
    for T, X, r, Tq, Xq, rb in zip(Ts, Xs, rs, Tb, Xb, res):
        assert r["status"] == 0, r
        assert (rb["status"], rb["iters"], rb["n_t1"]) == (r["status"], r["iters"], r["n_t1"])
        assert torch.equal(X, Xq)
        assert np.array_equal(T.topology(), Tq.topology())
    bs = [_dev(rng.normal(0, 1e-3, tuple(X.shape))) for X in Xs]
    singles = []
    for T, X, P, b in zip(Ts, Xs, Ps, bs):
        gs, info = T.param_grad(X, P, dC_dX=b, cg_tol=1e-10)
        assert info["status"] == 0, info
        singles.append(gs.cpu().numpy())
    outs, infos = vtx.Batch(Tb).param_grad(Xb, Ps, dC_dX=bs, cg_tol=1e-10, block_threads=512)
    worst = 0.0
    for k, (gs, gb, inf) in enumerate(zip(singles, outs, infos)):
        assert inf["status"] == 0, inf
        gb = gb.cpu().numpy()
        worst = max(worst, np.abs(gb - gs).max() / np.abs(gs).max())
        if k < 2:
            t, p = cases[k]
            m = oracle.Mesh(Tb[k].topology(), t.n_vert, t.Lx, t.Ly)
            go, _ = oracle.adjoint_grad(m, Xb[k].cpu().numpy(), p, bs[k].cpu().numpy(),
                                        tol=1e-10)
            assert np.abs(gb - go).max() < 1e-7 * np.abs(go).max()
    errlog("batched register-resident CG vs single (grid) solve, odd cell counts "
           "(max |dg| / max |g|, worst tissue)", worst)
    assert worst < 1e-9


@pytest.mark.parametrize("parts", [-1, -2, -4, -8])
@pytest.mark.parametrize("theta", ["lambda", "P0"])
def test_batch_adjoint_multiblock(vtx, oracle, errlog, small_equilibria, theta, parts):
    """Each tissue split over 1, 2, 4 or 8 workgroups (block_threads = -K):
    the gradients and CG iteration counts equal the single-tissue solve's
    and the oracle's to the solve's tolerance."""
    Ts, Xs, Ps, bs, refs = [], [], [], [], []
    for t, m, X, p, Xt in small_equilibria:
        T = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
        _, b = oracle.v2v(m, X, Xt)
        go, info_o = oracle.adjoint_grad(m, X, p, b, theta=theta, tol=1e-10)
        gs, info_s = T.param_grad(_dev(X), vtx.Params.from_numpy(p), dC_dX=_dev(b), theta=theta,
                                  cg_tol=1e-10)
        Ts.append(T); Xs.append(_dev(X)); Ps.append(vtx.Params.from_numpy(p)); bs.append(_dev(b))
        refs.append((go, info_o, gs.cpu().numpy(), info_s))
    outs, infos = vtx.Batch(Ts).param_grad(Xs, Ps, dC_dX=bs, theta=theta, cg_tol=1e-10,
                                           block_threads=parts)
    worst = 0.0
    for (go, info_o, gs, info_s), gb, inf in zip(refs, outs, infos):
        assert inf["status"] == 0, inf
        assert abs(inf["cg_iters"] - info_o["iters"]) <= 2
        gb = gb.cpu().numpy()
        worst = max(worst, np.abs(gb - go).max() / np.abs(go).max())
        assert np.abs(gb - gs).max() < 1e-8 * np.abs(gs).max()
        assert np.abs(gb - go).max() < 1e-7 * np.abs(go).max()
    errlog(f"batched adjoint, each tissue over {-parts} workgroups, theta={theta} "
           "(max |dg| / max |g|, worst tissue)", worst)


def test_batch_adjoint_multiblock_sizes_and_fallback(vtx):
    """Hexagonal-lattice tissues of 120, 1088 and 2600 cells in one batch,
    split over 8 workgroups (the largest part owns 650 vertices) and over 1
    (the 2600-cell tissue does not fit one workgroup's share and goes to the
    one-workgroup kernel): both equal the single-tissue solves."""
    rng = np.random.default_rng(62)
    s = np.sqrt(2.0 / (3.0 * np.sqrt(3.0)))
    Ts, Xs, Ps, bs, singles = [], [], [], [], []
    for nx, ny in [(12, 10), (34, 32), (52, 50)]:
        t = g.hex_lattice(nx, ny, s)
        p = g.uniform_params(t, P0=3.7)
        p.lam = np.full(t.n_edge, 0.1)
        T = vtx.Tissue.from_tissue(t)
        P = vtx.Params.from_numpy(p)
        X = _dev(t.X)
        b = T.v2v(X, X + _dev(rng.normal(0, 0.05, t.X.shape)))[1]
        gs, info = T.param_grad(X, P, dC_dX=b, cg_tol=1e-10)
        assert info["status"] == 0, info
        Ts.append(T); Xs.append(X); Ps.append(P); bs.append(b); singles.append(gs.cpu().numpy())
    for parts in (-8, -1):
        outs, infos = vtx.Batch(Ts).param_grad(Xs, Ps, dC_dX=bs, cg_tol=1e-10,
                                               block_threads=parts)
        for gsingle, gb, inf in zip(singles, outs, infos):
            assert inf["status"] == 0, (parts, inf)
            assert np.abs(gb.cpu().numpy() - gsingle).max() < 1e-7 * np.abs(gsingle).max()
    with pytest.raises(vtx.VtxError):
        vtx.Batch(Ts).param_grad(Xs, Ps, dC_dX=bs, cg_tol=1e-10, block_threads=-4,
                                 method="adjoint_minres")


@pytest.mark.parametrize("block_threads", [0, -2, -4])
@pytest.mark.parametrize("method", ["ep", "ep_forward"])
def test_batch_ep_matches_single(vtx, oracle, small_equilibria, method, block_threads):
    """Batched EP (the library's choice of relaxation kernel, or the nudged
    relaxations split over 2 or 4 workgroups per tissue) against the
    single-tissue path."""
    beta = 0.04
    ep = dict(eta=3e-3, tol=1e-12, max_iter=400000)
    Ts, Xs, Ps, Xts, refs = [], [], [], [], []
    for t, m, X, p, Xt in small_equilibria:
        T = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
        gs, _ = T.param_grad(_dev(X), vtx.Params.from_numpy(p), X_target=_dev(Xt), method=method,
                             beta=beta, ep_relax=ep)
        Ts.append(T); Xs.append(_dev(X)); Ps.append(vtx.Params.from_numpy(p)); Xts.append(_dev(Xt))
        refs.append(gs.cpu().numpy())
    B = vtx.Batch(Ts)
    outs, infos = B.param_grad(Xs, Ps, X_target=Xts, method=method, beta=beta, ep_relax=ep,
                               block_threads=block_threads)
    for gsingle, gb, inf in zip(refs, outs, infos):
        assert inf["status"] == 0
        assert inf["ep_plus"]["iters"] > 1
        assert np.abs(gb.cpu().numpy() - gsingle).max() < 1e-9 * np.abs(gsingle).max()


@pytest.mark.parametrize("method", ["ep", "ep_forward"])
def test_ep_status_reports_a_failed_relaxation(vtx, small_equilibria, method):
    """A nudged relaxation that overflows (step 1e30) is reported as
    VTX_E_NONFINITE, the error code of the single and of the batched call
    (which names the first failed tissue), for centred and first-order EP."""
    t, m, X, p, Xt = small_equilibria[0]
    ep = dict(eta=1e30, tol=1e-12, max_iter=1000)
    T = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
    P = vtx.Params.from_numpy(p)
    with pytest.raises(vtx.VtxError) as err:
        T.param_grad(_dev(X), P, X_target=_dev(Xt), method=method, beta=0.04, ep_relax=ep)
    assert err.value.code == -5
    T2 = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
    with pytest.raises(vtx.VtxError) as err:
        vtx.Batch([T, T2]).param_grad([_dev(X), _dev(X)], [P, P], X_target=[_dev(Xt), _dev(Xt)],
                                      method=method, beta=0.04, ep_relax=ep)
    assert err.value.code == -5 and "tissue 0" in str(err.value)


# ------------------------------------------------------------- autograd

@pytest.mark.parametrize("method", ["adjoint", "ep"])
def test_autograd_equilibrium_gradient(vtx, oracle, small_equilibria, method):
    from paper_2604_06896_amd.autograd import equilibrium
    t, m, X, p, Xt = small_equilibria[0]
    T = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
    theta = torch.as_tensor(p.lam, dtype=torch.float64, device="cuda").requires_grad_(True)
    prm = vtx.Params(KA=1.0, A0=1.0, KP=1.0, P0=3.75)
    grad_kw = dict(cg_tol=1e-11) if method == "adjoint" else \
        dict(method="ep", beta=1e-2, ep_relax=dict(eta=3e-3, tol=1e-13, max_iter=400000))
    Xs = equilibrium(theta, _dev(X), T, prm, which="lambda", mode="f64",
                     relax=dict(eta=3e-3, tol=1e-11, max_iter=400000), grad=grad_kw)
    Xt_d = _dev(Xt)
    loss = ((Xs - Xt_d) ** 2).sum() / (2 * t.n_vert)
    loss.backward()
    _, b = oracle.v2v(m, Xs.detach().cpu().numpy(), Xt)
    go, _ = oracle.adjoint_grad(m, Xs.detach().cpu().numpy(), p, b, tol=1e-11)
    err = np.abs(theta.grad.cpu().numpy() - go).max() / np.abs(go).max()
    print(method, "relative error vs oracle adjoint", err)
    assert err < (1e-7 if method == "adjoint" else 1e-3)


def test_gradient_matches_library_finite_differences(vtx, small_equilibria, errlog):
    """Central differences of the relaxed v2v cost, all on the GPU (FP64
    relaxations from X* without T1 to max |F| < 1e-12), along 8 random unit
    directions at h = 1e-3 and h/2: the two differ by their h^2 truncation
    (ratio 4), Richardson's (4 FD(h/2) - FD(h)) / 3 equals adjoint . d to
    1e-6, and centred EP (beta = 1e-3, nudged relaxations to 1e-12) equals
    it within its budget c beta^2 + tol / (beta |grad C|) (here 1e-4),
    first-order EP within its O(beta) bias (1e-2)."""
    t, m, X, p, Xt = small_equilibria[1]
    T = vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly)
    Xd, Xtd = _dev(X), _dev(Xt)
    P = vtx.Params.from_numpy(p)
    X0 = Xd.clone()
    assert T.relax(X0, P, mode="f64", eta=3e-3, tol=1e-12, max_iter=2000000)["status"] == 0
    _, b = T.v2v(X0, Xtd)
    gg, info = T.param_grad(X0, P, dC_dX=b, cg_tol=1e-13)
    ep = dict(eta=3e-3, tol=1e-12, max_iter=2000000)
    ge, ie = T.param_grad(X0, P, X_target=Xtd, method="ep", beta=1e-3, ep_relax=ep)
    gf, if_ = T.param_grad(X0, P, X_target=Xtd, method="ep_forward", beta=1e-3, ep_relax=ep)
    assert info["status"] == 0 and ie["status"] == 0 and if_["status"] == 0
    rng = np.random.default_rng(8)
    dirs, Ts, Xs, Ps = [], [], [], []
    for _ in range(8):
        d = rng.normal(size=t.n_edge)
        d /= np.linalg.norm(d)
        dirs.append(d)
        for h in (1e-3, 5e-4):
            for sgn in (1.0, -1.0):
                Ts.append(vtx.Tissue(m.he, t.n_vert, t.Lx, t.Ly))
                Xs.append(X0.clone())
                Ps.append(vtx.Params(P0=3.75, lam=_dev(p.lam + sgn * h * d)))
    res = vtx.Batch(Ts).relax(Xs, Ps, mode="f64", eta=3e-3, tol=1e-12, max_iter=2000000)
    assert all(r["status"] == 0 for r in res)
    Cs = [Ti.v2v(Xi, Xtd)[0].item() for Ti, Xi in zip(Ts, Xs)]
    worst = {"adjoint vs Richardson": 0.0, "adjoint vs FD(h/2)": 0.0, "centred EP": 0.0,
             "first-order EP": 0.0}
    for j, d in enumerate(dirs):
        fd_h = (Cs[4 * j] - Cs[4 * j + 1]) / 2e-3
        fd_h2 = (Cs[4 * j + 2] - Cs[4 * j + 3]) / 1e-3
        rich = (4 * fd_h2 - fd_h) / 3
        a = float(gg.cpu().numpy() @ d)
        # the truncation error shrinks four-fold with h (or is below the
        # relaxation noise)
        assert abs(fd_h - a) > 3 * abs(fd_h2 - a) or abs(fd_h - a) < 1e-6 * abs(a)
        for key, val, ref in (("adjoint vs Richardson", a, rich), ("adjoint vs FD(h/2)", a, fd_h2),
                              ("centred EP", float(ge.cpu().numpy() @ d), a),
                              ("first-order EP", float(gf.cpu().numpy() @ d), a)):
            worst[key] = max(worst[key], abs(val - ref) / abs(ref))
    for key, v in worst.items():
        errlog(f"finite differences, 20-cell tissue, 8 directions: {key} (relative)", v)
    assert worst["adjoint vs Richardson"] < 1e-6
    assert worst["adjoint vs FD(h/2)"] < 1e-5
    assert worst["centred EP"] < 1e-4
    assert worst["first-order EP"] < 1e-2
