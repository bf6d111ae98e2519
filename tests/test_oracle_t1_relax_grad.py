"""Pins of the oracle's T1 pass, relaxation and hypergradients (no GPU)."""
import numpy as np
import pytest

from paper_2604_06896_amd import tissue_gen as g


def check_topology(t_he, n_vert, n_cell):
    """Structural validity of a periodic 3-valent half-edge table."""
    he = t_he
    n = he.shape[0]
    ar = np.arange(n)
    assert np.all(he[he[:, 2], 2] == ar)               # twin is an involution
    assert np.all(he[:, 2] != ar)
    assert np.all(he[he[:, 1], 0] == ar)               # prev(next(h)) = h
    assert np.all(he[he[:, 1], 3] == he[:, 4])         # src(next(h)) = tgt(h)
    assert np.all(he[he[:, 2], 3] == he[:, 4])         # twin reverses
    assert np.all(he[he[:, 2], 6] == -he[:, 6])
    assert np.all(he[he[:, 2], 7] == -he[:, 7])
    assert np.all(he[he[:, 1], 5] == he[:, 5])         # next stays in the face
    assert np.all(np.bincount(he[:, 3], minlength=n_vert) == 3)   # 3-valent
    for c in range(n_cell):
        sel = he[:, 5] == c
        assert sel.sum() >= 3
        assert he[sel, 6].sum() == 0 and he[sel, 7].sum() == 0


def cells_of_vertex(he, v):
    return sorted(he[he[:, 3] == v, 5].tolist())


# ------------------------------------------------------------------- T1

def _hex_with_short_edge(e=0, s=0.62, ell=0.005):
    t = g.hex_lattice(4, 4, s)
    h = 2 * e
    i, j = t.he[h, 3], t.he[h, 4]
    o = t.he[h, 6:8] * np.array([t.Lx, t.Ly])
    d = t.X[j] + o - t.X[i]
    u = d / np.linalg.norm(d)
    mid = t.X[i] + 0.5 * d
    t.X[i] = mid - 0.5 * ell * u
    t.X[j] = mid + 0.5 * ell * u - o
    return t, h, mid, u


def _around(t, h):
    he = t.he
    tw = he[h, 2]
    C1, C2 = he[h, 5], he[tw, 5]
    C3 = he[he[he[h, 0], 2], 5]
    C4 = he[he[he[h, 1], 2], 5]
    return C1, C2, C3, C4


@pytest.mark.parametrize("favour", ["exchange", "stretch"])
def test_t1_on_hex_lattice(oracle, favour):
    t, h, mid, u = _hex_with_short_edge()
    C1, C2, C3, C4 = _around(t, h)
    p = g.uniform_params(t, P0=6 * 0.62, lam=0.0)
    lo, hi = 2.0, 5.0
    if favour == "exchange":       # losing cells want less perimeter, gaining more
        p.P0[[C1, C2]] = lo
        p.P0[[C3, C4]] = hi
    else:
        p.P0[[C1, C2]] = hi
        p.P0[[C3, C4]] = lo
    m = oracle.Mesh.from_tissue(t)
    X = t.X.copy()
    E_before = oracle.energy(m, X, p)
    n_sw, n_st = oracle.t1_pass(m, X, p, 0.01, 0.02)
    assert n_sw + n_st == 1
    check_topology(m.he, t.n_vert, t.n_cell)
    A, P, n = oracle.cells(m, X)
    assert A.sum() == pytest.approx(t.Lx * t.Ly, rel=1e-12)
    i, j = m.he[h, 3], m.he[h, 4]
    o = m.he[h, 6:8] * np.array([t.Lx, t.Ly])
    d = X[j] + o - X[i]
    assert np.linalg.norm(d) == pytest.approx(0.02, rel=1e-12)
    np.testing.assert_allclose(X[i] + 0.5 * d, mid, atol=1e-13)   # midpoint kept
    if favour == "exchange":
        assert (n_sw, n_st) == (1, 0)
        assert abs(np.dot(d, u)) < 1e-12                     # orthogonal edge
        assert n[C1] == 5 and n[C2] == 5 and n[C3] == 7 and n[C4] == 7
        assert cells_of_vertex(m.he, i) == sorted([C1, C3, C4])
        assert cells_of_vertex(m.he, j) == sorted([C2, C3, C4])
        # i was moved into C1: the new edge points from the C1 side to C2
        v = X[i] - mid
        assert u[0] * v[1] - u[1] * v[0] > 0
        assert sorted([m.he[h, 5], m.he[m.he[h, 2], 5]]) == sorted([C3, C4])
    else:
        assert (n_sw, n_st) == (0, 1)
        np.testing.assert_array_equal(m.he, t.he)            # topology unchanged
        np.testing.assert_allclose(d / 0.02, u, atol=1e-12)  # same orientation
    # the kept candidate has the lower total energy of the two
    alt_m = oracle.Mesh.from_tissue(t)
    alt_X = t.X.copy()
    if favour == "exchange":
        ui = u
        alt_X[i] = mid - 0.01 * ui
        alt_X[j] = mid + 0.01 * ui - (t.he[h, 6:8] * [t.Lx, t.Ly])
    else:
        oracle.t1_topology(alt_m, h)
        nrm = np.array([-u[1], u[0]])
        alt_X[i] = mid + 0.01 * nrm
        alt_X[j] = mid - 0.01 * nrm - (t.he[h, 6:8] * [t.Lx, t.Ly])
        check_topology(alt_m.he, t.n_vert, t.n_cell)
    assert oracle.energy(m, X, p) < oracle.energy(alt_m, alt_X, p)
    assert np.isfinite(E_before)


def test_t1_not_admissible_for_triangle(oracle):
    """After three exchanges that each take an edge from the same hexagon it
    is a triangle, and an exchange that would leave it a 2-gon is refused."""
    t = g.hex_lattice(4, 4, 0.62)
    m = oracle.Mesh.from_tissue(t)
    C1 = int(m.he[0, 5])
    for _ in range(3):
        hs = np.nonzero(m.he[:, 5] == C1)[0]
        h = next(int(x) for x in hs if oracle.t1_admissible(m, int(x)))
        oracle.t1_topology(m, h)
        check_topology(m.he, t.n_vert, t.n_cell)
    hs = np.nonzero(m.he[:, 5] == C1)[0]
    assert hs.size == 3
    assert not any(oracle.t1_admissible(m, int(x)) for x in hs)
    assert not any(oracle.t1_admissible(m, int(m.he[x, 2])) for x in hs)


def test_t1_pass_on_random_tissue_keeps_invariants(oracle):
    t, p = g.workload_single_100()
    m = oracle.Mesh.from_tissue(t)
    X = t.X.copy()
    r = oracle.relax(m, X, p, eta=1e-2, tol=1e-6, patience=1, max_iter=3000,
                     t1_enable=True, l_min=0.01)
    assert r["n_t1"] > 0
    check_topology(m.he, t.n_vert, t.n_cell)
    A, P, n = oracle.cells(m, X)
    assert np.all(A > 0)
    assert A.sum() == pytest.approx(t.Lx * t.Ly, rel=1e-10)
    assert n.sum() == 6 * t.n_cell


# ------------------------------------------------------------ relaxation

def test_tense_hex_lattice_relaxes_back(oracle):
    """A regular hexagonal lattice whose cells have their preferred area and
    a preferred perimeter below the hexagon's is a strict local minimum
    (positive tension on every edge, 3-fold symmetric vertices): a perturbed
    lattice returns to it, with E = N K_P (P_hex - P0)^2."""
    s = 0.62
    t = g.hex_lattice(4, 4, s)
    Ah, Ph = 1.5 * np.sqrt(3.0) * s * s, 6 * s
    p = g.uniform_params(t, A0=Ah, P0=Ph - 0.3, lam=0.0)
    m = oracle.Mesh.from_tissue(t)
    rng = np.random.default_rng(1)
    X = t.X + rng.normal(0, 0.02 * s, t.X.shape)
    c0 = X.sum(0)
    r = oracle.relax(m, X, p, eta=1e-2, tol=1e-10, patience=1, max_iter=200000)
    assert r["status"] == 0
    assert r["energy"] == pytest.approx(t.n_cell * 0.3 ** 2, rel=1e-12)
    np.testing.assert_allclose(X.sum(0), c0, rtol=1e-12)        # centroid kept
    disp = X - t.X
    disp -= disp.mean(0)
    assert np.abs(disp).max() < 1e-6 * s


def test_patience_and_max_iter(oracle):
    t = g.hex_lattice(4, 4, 0.62)
    p = g.uniform_params(t, P0=3.0, lam=0.1)
    m = oracle.Mesh.from_tissue(t)
    for pat in (1, 4):
        X = t.X.copy()
        r = oracle.relax(m, X, p, tol=1e-9, patience=pat, max_iter=100)
        assert r["status"] == 0 and r["iters"] == pat
    tr, pr = g.workload_single_100()
    mr = oracle.Mesh.from_tissue(tr)
    X = tr.X.copy()
    r = oracle.relax(mr, X, pr, tol=1e-6, patience=1, max_iter=50)
    assert r["status"] == 1 and r["iters"] == 50
    # GD steps descend the energy
    assert r["energy"] < oracle.energy(mr, tr.X, pr)


# ---------------------------------------------------------- hypergradient

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
    return m, X, p, Xt


def _fd_hessian(oracle, m, X, p, h=1e-5):
    n = X.size
    H = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        _, Fp = oracle.energy_forces(m, X + e.reshape(X.shape), p)
        _, Fm = oracle.energy_forces(m, X - e.reshape(X.shape), p)
        H[:, k] = -(Fp - Fm).ravel() / (2 * h)
    return 0.5 * (H + H.T)


def test_cg_matches_dense_pseudoinverse(oracle, equilibrium):
    m, X, p, Xt = equilibrium
    H = _fd_hessian(oracle, m, X, p)
    w = np.linalg.eigvalsh(H)
    assert abs(w[0]) < 1e-8 and abs(w[1]) < 1e-8 and w[2] > 1e-3   # 2 translations
    _, b = oracle.v2v(m, X, Xt)
    mu, info = oracle.cg(m, X, p, b, tol=1e-12)
    assert info["status"] == 0
    mu_ref = (np.linalg.pinv(H, rcond=1e-9) @ b.ravel()).reshape(X.shape)
    assert np.abs(mu - mu_ref).max() < 1e-6 * np.abs(mu_ref).max()


def _relaxed_cost(oracle, m, X0, p, Xt):
    mm = m.copy()
    X = X0.copy()
    r = oracle.relax(mm, X, p, eta=3e-3, tol=1e-12, patience=1, max_iter=400000)
    assert r["status"] == 0
    np.testing.assert_array_equal(mm.he, m.he)
    return oracle.v2v(mm, X, Xt)[0]


@pytest.mark.parametrize("theta", ["lambda", "P0"])
def test_adjoint_gradient_matches_finite_differences(oracle, equilibrium, theta):
    m, X, p, Xt = equilibrium
    _, b = oracle.v2v(m, X, Xt)
    gr, info = oracle.adjoint_grad(m, X, p, b, theta=theta, tol=1e-12)
    assert info["status"] == 0
    rng = np.random.default_rng(21)
    n = m.n_edge if theta == "lambda" else m.n_cell
    d = rng.normal(size=n)
    d /= np.linalg.norm(d)
    vals = []
    for hh in (1e-3, 5e-4):
        pp = p.copy()
        pm = p.copy()
        if theta == "lambda":
            pp.lam = p.lam + hh * d
            pm.lam = p.lam - hh * d
        else:
            pp.P0 = p.P0 + hh * d
            pm.P0 = p.P0 - hh * d
        Cp = _relaxed_cost(oracle, m, X, pp, Xt)
        Cm = _relaxed_cost(oracle, m, X, pm, Xt)
        vals.append((Cp - Cm) / (2 * hh))
    assert vals[0] == pytest.approx(vals[1], rel=1e-3)      # FD consistent in h
    assert gr @ d == pytest.approx(vals[1], rel=2e-3)


def test_centred_ep_converges_to_adjoint_at_second_order(oracle, equilibrium):
    m, X, p, Xt = equilibrium
    _, b = oracle.v2v(m, X, Xt)
    g_adj, _ = oracle.adjoint_grad(m, X, p, b, tol=1e-12)
    errs = []
    for beta in (1e-1, 4e-2):
        g_ep, info = oracle.ep_grad(m, X, p, Xt, beta, eta=3e-3, tol=1e-12,
                                    patience=1, max_iter=400000)
        assert info["plus"]["status"] == 0 and info["minus"]["status"] == 0
        errs.append(np.abs(g_ep - g_adj).max())
    # beta / 2.5: O(beta^2) shrinks the error 6.25x, O(beta) only 2.5x
    assert errs[1] < errs[0] / 4
    assert errs[1] < 1e-3 * np.abs(g_adj).max()


@pytest.mark.parametrize("theta", ["lambda", "P0"])
def test_sensitivity_matches_finite_differences_and_adjoint(oracle, equilibrium, theta):
    """Forward ID along d (one solve per direction) against central
    differences of the relaxed cost, and against the adjoint gradient . d
    (a different linear solve and a different mixed-derivative code path)."""
    m, X, p, Xt = equilibrium
    _, b = oracle.v2v(m, X, Xt)
    rng = np.random.default_rng(22)
    n = m.n_edge if theta == "lambda" else m.n_cell
    d = rng.normal(size=n)
    d /= np.linalg.norm(d)
    s, w, info = oracle.sens_derivative(m, X, p, d, b, theta=theta, tol=1e-12)
    assert info["status"] == 0
    assert abs(w.mean(axis=0)).max() < 1e-12          # solved on the zero-mean subspace
    gr, _ = oracle.adjoint_grad(m, X, p, b, theta=theta, tol=1e-12)
    assert s == pytest.approx(gr @ d, rel=1e-8)
    hh = 5e-4
    pp, pm = p.copy(), p.copy()
    if theta == "lambda":
        pp.lam, pm.lam = p.lam + hh * d, p.lam - hh * d
    else:
        pp.P0, pm.P0 = p.P0 + hh * d, p.P0 - hh * d
    fd = (_relaxed_cost(oracle, m, X, pp, Xt) - _relaxed_cost(oracle, m, X, pm, Xt)) / (2 * hh)
    assert s == pytest.approx(fd, rel=2e-3)
    # w is the directional derivative of the equilibrium itself
    Xp, Xm = X.copy(), X.copy()
    oracle.relax(m.copy(), Xp, pp, eta=3e-3, tol=1e-12, patience=1, max_iter=400000)
    oracle.relax(m.copy(), Xm, pm, eta=3e-3, tol=1e-12, patience=1, max_iter=400000)
    dX = (Xp - Xm) / (2 * hh)
    dX -= dX.mean(axis=0)
    assert np.abs(dX - w).max() < 5e-3 * np.abs(w).max()


def test_forward_ep_converges_to_adjoint_at_first_order(oracle, equilibrium):
    m, X, p, Xt = equilibrium
    _, b = oracle.v2v(m, X, Xt)
    g_adj, _ = oracle.adjoint_grad(m, X, p, b, tol=1e-12)
    errs = []
    for beta in (1e-1, 4e-2):
        g_ep, info = oracle.ep_grad_forward(m, X, p, Xt, beta, eta=3e-3, tol=1e-12,
                                            patience=1, max_iter=400000)
        assert info["plus"]["status"] == 0
        errs.append(np.abs(g_ep - g_adj).max())
    # beta / 2.5: an O(beta) bias shrinks about 2.5x (the centred one 6.25x)
    assert 1.8 < errs[0] / errs[1] < 3.5


def _exact_hessian(oracle, m, X, p):
    n = X.size
    return np.column_stack([oracle.hvp(m, X, p, np.eye(n)[k].reshape(X.shape)).ravel()
                            for k in range(n)])


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_minres_solves_indefinite_systems(oracle, seed):
    """At an unrelaxed Voronoi state H is strongly indefinite: CG stops on
    negative curvature, MINRES still returns the pseudo-inverse solution."""
    rng = np.random.default_rng(seed)
    t = g.random_tissue(20, np.sqrt(20.0), rng=rng)
    p = g.uniform_params(t, P0=3.75)
    p.lam = rng.uniform(0.05, 0.15, t.n_edge)
    m = oracle.Mesh.from_tissue(t)
    X = t.X.copy()
    H = _exact_hessian(oracle, m, X, p)
    ev = np.linalg.eigvalsh(0.5 * (H + H.T))
    assert ev[0] < -1.0                                  # indefinite
    b = rng.normal(size=X.shape)
    x, info = oracle.minres(m, X, p, b, tol=1e-13)
    assert info["status"] == 0 and info["rel_res"] < 1e-13
    ref = (np.linalg.pinv(H, rcond=1e-10) @ (b - b.mean(axis=0)).ravel()).reshape(X.shape)
    assert np.abs(x - ref).max() < 1e-9 * np.abs(ref).max()
    _, info_cg = oracle.cg(m, X, p, b, tol=1e-13)
    assert info_cg["status"] == 2                        # CG_NEG_CURVATURE


@pytest.mark.parametrize("theta", ["lambda", "P0"])
def test_minres_adjoint_equals_cg_adjoint_at_equilibrium(oracle, equilibrium, theta):
    m, X, p, Xt = equilibrium
    _, b = oracle.v2v(m, X, Xt)
    g_cg, i_cg = oracle.adjoint_grad(m, X, p, b, theta=theta, tol=1e-12)
    g_mr, i_mr = oracle.adjoint_grad(m, X, p, b, theta=theta, tol=1e-12, solver="minres")
    assert i_cg["status"] == 0 and i_mr["status"] == 0
    assert np.abs(g_mr - g_cg).max() < 1e-9 * np.abs(g_cg).max()
