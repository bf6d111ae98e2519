"""The workflows built on the path: the rigidity sweep (Results, the
solid-to-fluid transition in p0, Fig. 3g left) and the bilevel outer loop
(ADAM on the hypergradient)."""
import warnings

import numpy as np
import pytest

from paper_2604_06896_amd import tissue_gen as g

pytestmark = pytest.mark.gpu


def test_rigidity_sweep_fit_on_seven_points():
    """Seven p0 values, 8 tissues each (the benchmark's MIXED mode): the
    zero-energy fraction rises from 0 to 1 across the grid and the logistic
    fit is finite, inside the grid, and raises no warning."""
    from paper_2604_06896_amd import studies
    grid = [3.8, 3.85, 3.9, 3.95, 4.0, 4.05, 4.1]
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        r = studies.rigidity_sweep(p0_grid=grid, n_per_p0=8, log=print)
    f = r["fraction_zero_energy"]
    assert f[0] == 0.0 and f[-1] == 1.0
    assert all(a <= b + 0.25 for a, b in zip(f, f[1:]))      # rises, up to sampling noise
    assert np.isfinite(r["fit_p_c"]) and np.isfinite(r["fit_width"])
    assert grid[0] < r["fit_p_c"] < grid[-1] and r["fit_width"] > 0
    # solid side: positive-energy minima; fluid side: energy relaxed away
    assert r["energy_per_cell_median"][0] > 1e-4 > 1e-9 > r["energy_per_cell_median"][-1]


def test_rigidity_sweep_matches_oracle():
    """The sweep in FP64 on 4 tissues at a solid (3.75) and a fluid (4.05)
    p0: each tissue's relaxed energy and its zero-energy classification equal
    the oracle's relaxation of the same tissue (same protocol, 1e5 steps)."""
    import oracle as O
    from concurrent.futures import ThreadPoolExecutor

    from paper_2604_06896_amd import studies
    O.build(force=False)
    grid, n, cap = [3.75, 4.05], 4, 100000
    r = studies.rigidity_sweep(p0_grid=grid, n_per_p0=n, mode="f64", max_iter=cap, log=print)
    rng = np.random.default_rng(601)           # the sweep's default seed and draw order
    jobs = [(p0, g.random_tissue(100, 10.0, rng=rng)) for p0 in grid for _ in range(n)]

    def ora(job):
        p0, t = job
        m = O.Mesh.from_tissue(t)
        X = t.X.copy()
        return O.relax(m, X, g.uniform_params(t, P0=p0), eta=1e-2, tol=1e-6, patience=1,
                       max_iter=cap, t1_enable=True, l_min=0.01)["energy"] / 100

    with ThreadPoolExecutor(8) as ex:
        eo = list(ex.map(ora, jobs))
    eg = [e for row in r["energy_per_cell"] for e in row]
    for (p0, _), a, b in zip(jobs, eg, eo):
        print(p0, a, b)
        assert (a < 1e-6) == (b < 1e-6)
        assert a == pytest.approx(b, rel=1e-6, abs=1e-10)
    assert r["fraction_zero_energy"] == [0.0, 1.0]


@pytest.mark.parametrize("method", ["adjoint", "ep"])
def test_bilevel_fit_recovers_shape_factors(method):
    from paper_2604_06896_amd import studies
    grad = None if method == "adjoint" else \
        dict(beta=1e-2, ep_relax=dict(eta=1e-2, tol=1e-8, max_iter=100000))
    h = studies.bilevel_fit(epochs=60, method=method, grad=grad, log=print)
    assert h["cost"][-1] < 0.6 * h["cost"][0]
    assert h["pearson"][-1] > h["pearson"][0] + 0.2
    assert h["rel_l1"][-1] < h["rel_l1"][0]
