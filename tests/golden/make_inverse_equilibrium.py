"""Writes tests/golden/inverse_tissue0_equilibrium.txt with the CPU oracle only.

The tissue is the first of the inverse-problem workload (1000-cell periodic
Voronoi tissue, box sqrt(1000), P0 = 3.75, initial tensions theta0 ~
U[0.05, 0.15]; generator seed 501).  The oracle relaxes it by gradient
descent (Methods, "Simulation engine": step 3e-3, max |F| < 1e-6, patience 1)
with T1 exchanges below 0.01 (Methods, "T1 transitions"), which is how the
workload's predictions X* are made.  The file holds the relaxed positions
(exact, as hexadecimal floats) and the rows of the half-edge table that the
T1 exchanges changed.  Nothing here calls the HIP library.

    python tests/golden/make_inverse_equilibrium.py     (about 80 s)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "inverse_tissue0_equilibrium.txt")
OPTS = dict(eta=3e-3, tol=1e-6, patience=1, max_iter=2000000, t1_enable=True, l_min=0.01)


def main():
    import oracle as O
    from paper_2604_06896_amd import tissue_gen as g
    O.build(force=False)
    t, _, pi = g.workload_inverse(n_tissue=1)[0]
    m = O.Mesh.from_tissue(t)
    X = t.X.copy()
    r = O.relax(m, X, pi, **OPTS)
    assert r["status"] == O.RELAX_CONVERGED, r
    changed = np.nonzero((m.he != t.he).any(axis=1))[0]
    with open(OUT, "w") as f:
        f.write("# oracle equilibrium of the first 1000-cell tissue of the inverse workload\n")
        f.write("# written by tests/golden/make_inverse_equilibrium.py (oracle only)\n")
        f.write(f"# relax: {OPTS}\n")
        f.write(f"# result: iters {r['iters']} n_t1 {r['n_t1']} n_stretch {r['n_stretch']} "
                f"max_f {r['max_f']!r} energy {r['energy']!r}\n")
        f.write(f"n_vert {t.n_vert} n_cell {t.n_cell} n_he {t.n_he} changed_rows {len(changed)}\n")
        for x, y in X:
            f.write(f"{float(x).hex()} {float(y).hex()}\n")
        for h in changed:
            f.write(f"{h} " + " ".join(str(int(v)) for v in m.he[h]) + "\n")
    print(f"wrote {OUT}: {r}")


def load():
    """(tissue with the relaxed topology, X*, params theta0, relax result line)."""
    from paper_2604_06896_amd import tissue_gen as g
    t, _, pi = g.workload_inverse(n_tissue=1)[0]
    with open(OUT) as f:
        lines = [ln for ln in f if not ln.startswith("#")]
    head = lines[0].split()
    nv, nch = int(head[1]), int(head[7])
    assert nv == t.n_vert
    X = np.array([[float.fromhex(a) for a in ln.split()] for ln in lines[1:1 + nv]])
    he = t.he.copy()
    for ln in lines[1 + nv:1 + nv + nch]:
        v = [int(a) for a in ln.split()]
        he[v[0]] = v[1:]
    t2 = t.copy()
    t2.he = he
    t2.X = X
    return t2, X, pi


if __name__ == "__main__":
    main()
