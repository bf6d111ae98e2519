"""The allocation-free evaluation entry point (vtx_energy_forces_noalloc)
through the C ABI: the same energy, forces and max |F| as
vtx_energy_forces, bit for bit, on two calls in a row with a smaller tissue
the second time, and a clear capacity error beyond its fixed scratch."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2604_06896_amd import tissue_gen as g

pytestmark = pytest.mark.gpu


def _call(V, fn, T, X, P, mode):
    cp, keep = P.to_c(X.dtype, X.device)
    E = torch.empty((), dtype=torch.float64, device=X.device)
    F = torch.empty_like(X)
    mf = torch.empty((), dtype=torch.float64, device=X.device)
    rc = fn(T.handle, V._mode(mode), V._ptr(X), C.byref(cp), V._ptr(E), V._ptr(F), V._ptr(mf),
            V._stream())
    return rc, E, F, mf


@pytest.mark.parametrize("mode", ["f32", "mixed", "f64"])
def test_noalloc_evaluation_equals_the_workspace_one(mode, oracle):
    from paper_2604_06896_amd import vtx as V
    L = V.lib()
    dt = V.pos_dtype(mode)
    cases = []
    for n, seed in ((20000, 3), (1000, 4)):       # the second call is smaller
        rng = np.random.default_rng(seed)
        t = g.random_tissue(n, np.sqrt(n), rng=rng)
        p = g.uniform_params(t, P0=3.75)
        p.lam = rng.uniform(0.05, 0.15, t.n_edge)
        cases.append((t, p))
    outs = []
    for t, p in cases:
        T = V.Tissue.from_tissue(t)
        X = torch.as_tensor(t.X, dtype=dt, device="cuda")
        P = V.Params.from_numpy(p, dtype=dt)
        rc, E, F, mf = _call(V, L.vtx_energy_forces_noalloc, T, X, P, mode)
        assert rc == 0, L.vtx_last_error().decode()
        outs.append((T, X, P, E.clone(), F.clone(), mf.clone()))
    for (t, p), (T, X, P, E, F, mf) in zip(cases, outs):
        rc, E0, F0, mf0 = _call(V, L.vtx_energy_forces, T, X, P, mode)
        assert rc == 0
        torch.cuda.synchronize()
        assert torch.equal(F, F0)
        assert E.item() == E0.item() and mf.item() == mf0.item()
        # and both against the oracle at the precision's bar
        Eo, Fo = oracle.energy_forces(oracle.Mesh.from_tissue(t), X.double().cpu().numpy(), p)
        err = np.abs(F.double().cpu().numpy() - Fo).max() / np.abs(Fo).max()
        assert err < (1e-10 if mode == "f64" else 1e-5)
        assert E.item() == pytest.approx(Eo, rel=1e-12 if mode == "f64" else 1e-6)


def test_noalloc_rejects_tissues_beyond_its_scratch():
    from paper_2604_06896_amd import vtx as V
    L = V.lib()
    t = g.random_tissue(140000, np.sqrt(140000.0), seed=9)
    T = V.Tissue.from_tissue(t)
    X = torch.as_tensor(t.X, dtype=torch.float32, device="cuda")
    rc, _, _, _ = _call(V, L.vtx_energy_forces_noalloc, T, X, V.Params(P0=3.75, lam=0.1), "f32")
    assert rc == V.E_CAPACITY
    assert "exceed" in L.vtx_last_error().decode()
