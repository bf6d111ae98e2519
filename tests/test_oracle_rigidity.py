"""Oracle pins of the rigidity transition the sweep measures (Results, the
solid-to-fluid transition in the target shape factor, Fig. 3g left): under
the sweep's protocol (100-cell periodic Voronoi tissues, L = 10, K_A = A0 =
K_P = 1, no line tension, GD step 1e-2 with T1 below 0.01, max |F| < 1e-6)
a tissue at p0 = 3.85 relaxes to a mechanical equilibrium of positive energy
whose Hessian is positive definite apart from the two rigid translations (a
rigid, solid state), and tissues at p0 = 4.05 relax to zero energy.  Both
outcomes are the same whether the stretch candidate of a short edge puts its
vertices 2 l_min or 1.01 l_min apart, so the transition between them does not
come from that reading of the T1 rule."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2604_06896_amd import tissue_gen as g

SWEEP = dict(eta=1e-2, tol=1e-6, patience=1, t1_enable=True, l_min=0.01)
READINGS = {"stretch to 2 l_min": 0.02, "stretch to 1.01 l_min": 0.0101}


def _tissue(k):
    return g.random_tissue(100, 10.0, rng=np.random.default_rng(1000 + k))


def _relax(oracle, k, p0, l_new, max_iter):
    t = _tissue(k)
    m = oracle.Mesh.from_tissue(t)
    X = t.X.copy()
    r = oracle.relax(m, X, g.uniform_params(t, P0=p0), max_iter=max_iter, l_new=l_new, **SWEEP)
    return m, X, r


def test_solid_minimum_below_the_transition(oracle):
    runs = {}
    with ThreadPoolExecutor(2) as ex:       # the oracle releases the GIL in C
        futs = {name: ex.submit(_relax, oracle, 0, 3.85, l_new, 200000)
                for name, l_new in READINGS.items()}
        runs = {name: f.result() for name, f in futs.items()}
    energies = []
    for name, (m, X, r) in runs.items():
        assert r["status"] == oracle.RELAX_CONVERGED, (name, r)
        assert r["energy"] / 100 > 1e-4, (name, r)   # far above the zero-energy threshold
        energies.append(r["energy"])
    assert energies[1] == pytest.approx(energies[0], rel=1e-4)
    # the equilibrium is rigid: the Hessian (assembled column by column from
    # the oracle's Hessian-vector product) is positive definite on the
    # zero-mean subspace
    m, X, _ = runs["stretch to 2 l_min"]
    p = g.uniform_params(_tissue(0), P0=3.85)
    n = 2 * m.n_vert
    H = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        H[:, j] = oracle.hvp(m, X, p, e.reshape(-1, 2)).ravel()
    H = 0.5 * (H + H.T)
    t = np.zeros((n, 2))
    t[0::2, 0] = 1.0
    t[1::2, 1] = 1.0
    Q, _ = np.linalg.qr(t)
    P = np.eye(n) - Q @ Q.T
    w = np.linalg.eigvalsh(P @ H @ P)
    assert np.sum(np.abs(w) < 1e-9) == 2          # the two translations
    assert w[np.abs(w) >= 1e-9].min() > 1e-6


def test_zero_energy_above_the_transition(oracle):
    jobs = [(k, l_new) for k in range(3) for l_new in READINGS.values()]
    with ThreadPoolExecutor(6) as ex:
        res = list(ex.map(lambda a: _relax(oracle, a[0], 4.05, a[1], 200000)[2], jobs))
    for (k, l_new), r in zip(jobs, res):
        assert r["status"] == oracle.RELAX_CONVERGED, (k, l_new, r)
        assert r["energy"] / 100 < 1e-9, (k, l_new, r)
