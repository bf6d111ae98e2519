"""Seeded synthetic tissue generator (input data only).

This module builds the inputs that both the CPU oracle and the HIP path
consume: periodic Voronoi tilings in the half-edge table format of the
paper (Methods, "System state and data structure": an 8-column heTable of
prev, next, twin, source, target, face, x-offset, y-offset) plus the
parameter arrays of each workload.  It contains none of the method's
arithmetic (no area, perimeter, energy, force or gradient): only seed
sampling, the Delaunay/Voronoi construction of the initial mesh (Methods,
"Mesh initialization"), and bookkeeping of ids and periodic image offsets.

Conventions of the produced table
  * faces are traversed counter-clockwise (the cell lies left of each of
    its half-edges); every vertex is 3-valent;
  * the edge vector of half-edge h is
        X[tgt] + (ox * Lx, oy * Ly) - X[src];
  * twin half-edges are stored as adjacent pairs (2e, 2e+1), so edge e is
    half-edges 2e and 2e+1 (the library only assumes the general rule
    "edges are numbered by ascending lower half-edge id", which this
    satisfies);
  * cells and vertices are numbered along a Morton curve of their
    position, so that ids that are close are close in space.
"""
from __future__ import annotations

import dataclasses
import numpy as np

HE_PREV, HE_NEXT, HE_TWIN, HE_SRC, HE_TGT, HE_FACE, HE_OX, HE_OY = range(8)


@dataclasses.dataclass
class Tissue:
    he: np.ndarray        # int32 [n_he, 8]
    X: np.ndarray         # float64 [n_vert, 2], wrapped into the box
    Lx: float
    Ly: float
    seeds: np.ndarray | None = None

    @property
    def n_he(self) -> int:
        return int(self.he.shape[0])

    @property
    def n_vert(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_cell(self) -> int:
        return int(self.he[:, HE_FACE].max()) + 1 if self.n_he else 0

    @property
    def n_edge(self) -> int:
        return self.n_he // 2

    def copy(self) -> "Tissue":
        return Tissue(self.he.copy(), self.X.copy(), self.Lx, self.Ly,
                      None if self.seeds is None else self.seeds.copy())


def _spread_bits(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64)
    v = (v | (v << np.uint64(16))) & np.uint64(0x0000FFFF0000FFFF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF00FF00FF)
    v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F0F0F0F0F)
    v = (v | (v << np.uint64(2))) & np.uint64(0x3333333333333333)
    v = (v | (v << np.uint64(1))) & np.uint64(0x5555555555555555)
    return v


def morton_order(xy: np.ndarray, Lx: float, Ly: float, bits: int = 20) -> np.ndarray:
    """Permutation sorting points along a Morton (Z-order) curve."""
    n = 1 << bits
    qx = np.clip((xy[:, 0] / Lx * n).astype(np.int64), 0, n - 1)
    qy = np.clip((xy[:, 1] / Ly * n).astype(np.int64), 0, n - 1)
    key = _spread_bits(qx) | (_spread_bits(qy) << np.uint64(1))
    return np.argsort(key, kind="stable")


def _circumcenter(a, b, c):
    """Circumcentre of triangles given as [n,2] arrays (b, c relative to a)."""
    bx, by = b[:, 0] - a[:, 0], b[:, 1] - a[:, 1]
    cx, cy = c[:, 0] - a[:, 0], c[:, 1] - a[:, 1]
    d = 2.0 * (bx * cy - by * cx)
    b2 = bx * bx + by * by
    c2 = cx * cx + cy * cy
    ux = (cy * b2 - by * c2) / d
    uy = (bx * c2 - cx * b2) / d
    return np.stack([a[:, 0] + ux, a[:, 1] + uy], axis=1)


def periodic_voronoi(seeds: np.ndarray, Lx: float, Ly: float,
                     margin: float | None = None, sort: bool = True) -> Tissue:
    """Periodic Voronoi tessellation of `seeds` in the box [0,Lx) x [0,Ly).

    Follows the paper's mesh initialisation (Methods, "Mesh initialization"):
    the seeds are replicated into the eight neighbouring boxes, the
    tessellation is computed, and only the polygons of the primary seeds
    are kept; half-edges leaving the box get the image offset of their
    target.  For large inputs only the copies within `margin` of the box are
    kept (the polygons of primary seeds are unchanged as long as the margin
    exceeds the largest circumradius, which the counts check below
    verifies).
    """
    from scipy.spatial import Delaunay

    seeds = np.asarray(seeds, dtype=np.float64)
    N = seeds.shape[0]
    if sort:
        seeds = seeds[morton_order(seeds, Lx, Ly)]
    if margin is None:
        spacing = np.sqrt(Lx * Ly / N)
        margin = np.inf if N <= 20000 else 8.0 * spacing
    pts = [seeds]
    orig = [np.arange(N)]
    shx = [np.zeros(N, np.int64)]
    shy = [np.zeros(N, np.int64)]
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            if sx == 0 and sy == 0:
                continue
            p = seeds + np.array([sx * Lx, sy * Ly])
            keep = ((p[:, 0] > -margin) & (p[:, 0] < Lx + margin) &
                    (p[:, 1] > -margin) & (p[:, 1] < Ly + margin))
            idx = np.nonzero(keep)[0]
            pts.append(p[idx])
            orig.append(idx)
            shx.append(np.full(idx.size, sx, np.int64))
            shy.append(np.full(idx.size, sy, np.int64))
    P = np.concatenate(pts)
    orig = np.concatenate(orig)
    shx = np.concatenate(shx)
    shy = np.concatenate(shy)

    tri = Delaunay(P)
    indptr, indices = tri.vertex_neighbor_vertices
    # Delaunay neighbours of the primary seeds, sorted by angle (CCW).
    cnt = indptr[1:N + 1] - indptr[:N]
    owner = np.repeat(np.arange(N), cnt)
    nb = indices[indptr[0]:indptr[N]]
    ang = np.arctan2(P[nb, 1] - P[owner, 1], P[nb, 0] - P[owner, 0])
    order = np.lexsort((ang, owner))
    nb = nb[order]
    start = np.concatenate([[0], np.cumsum(cnt)])
    k_in = np.arange(nb.size) - start[owner]
    nxt_pos = start[owner] + (k_in + 1) % cnt[owner]
    q1 = nb                      # neighbour k
    q2 = nb[nxt_pos]             # neighbour k+1
    # Corner k of cell `owner` is the circumcentre of (owner, q1, q2).
    # Canonical key of that Voronoi vertex: the triple of (orig, shift)
    # made relative to its smallest member.
    mem_o = np.stack([owner, orig[q1], orig[q2]], axis=1)
    mem_x = np.stack([np.zeros_like(owner), shx[q1], shx[q2]], axis=1)
    mem_y = np.stack([np.zeros_like(owner), shy[q1], shy[q2]], axis=1)
    code = (mem_o * 25 + (mem_x + 2) * 5 + (mem_y + 2))
    # anchor: member with the smallest (orig, shx, shy)
    anchor = np.argmin(code, axis=1)
    r = np.arange(code.shape[0])
    ax = mem_x[r, anchor]
    ay = mem_y[r, anchor]
    rel_code = mem_o * 25 + (mem_x - ax[:, None] + 2) * 5 + (mem_y - ay[:, None] + 2)
    rel_code.sort(axis=1)
    keys, first, inv = np.unique(rel_code, axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    n_vert = keys.shape[0]
    # Canonical positions: circumcentre of the canonical triple computed in
    # the frame of its first member, wrapped into the box.
    ko = keys // 25
    kx = (keys // 5) % 5 - 2
    ky = keys % 5 - 2
    base = seeds[ko[:, 0]] + np.stack([kx[:, 0] * Lx, ky[:, 0] * Ly], 1)
    pb = seeds[ko[:, 1]] + np.stack([kx[:, 1] * Lx, ky[:, 1] * Ly], 1)
    pc = seeds[ko[:, 2]] + np.stack([kx[:, 2] * Lx, ky[:, 2] * Ly], 1)
    cc = _circumcenter(base, pb, pc)
    wx = np.floor(cc[:, 0] / Lx).astype(np.int64)
    wy = np.floor(cc[:, 1] / Ly).astype(np.int64)
    Xv = cc - np.stack([wx * Lx, wy * Ly], 1)
    # rounding can leave a coordinate at exactly the upper face
    over_x = Xv[:, 0] >= Lx
    over_y = Xv[:, 1] >= Ly
    wx = wx + over_x
    wy = wy + over_y
    Xv = cc - np.stack([wx * Lx, wy * Ly], 1)
    Xv[:, 0] = np.clip(Xv[:, 0], 0.0, np.nextafter(Lx, 0.0))
    Xv[:, 1] = np.clip(Xv[:, 1], 0.0, np.nextafter(Ly, 0.0))
    # Image of each corner as seen from its cell: anchor shift (relative to
    # the cell's own frame) plus the wrap of the canonical position.  The
    # canonical triple's first member is the anchor, whose shift relative to
    # the cell frame is (ax, ay) for this corner.
    # (The first member of the sorted relative triple is the anchor itself
    #  only when the anchor has the smallest code, which is how it was
    #  chosen, so the relative shift of member 0 is zero.)
    Wx = ax + wx[inv]
    Wy = ay + wy[inv]

    # Checks: 3 corners per vertex, V = 2F, E = 3F.
    per_vertex = np.bincount(inv, minlength=n_vert)
    if n_vert != 2 * N or not np.all(per_vertex == 3):
        raise RuntimeError(
            f"periodic Voronoi is not a 3-valent tiling (V={n_vert}, F={N}, "
            f"valence range {per_vertex.min()}..{per_vertex.max()}); "
            "increase the margin")

    # Vertex renumbering along a Morton curve of the wrapped positions.
    vperm = morton_order(Xv, Lx, Ly) if sort else np.arange(n_vert)
    vrank = np.empty(n_vert, np.int64)
    vrank[vperm] = np.arange(n_vert)
    Xv = Xv[vperm]
    vid = vrank[inv]

    # Half-edges, cell-major: half-edge k of cell c goes from corner k to
    # corner k+1 and is dual to the Delaunay edge (c, q2_k).
    n_c = N
    src = vid
    tgt = vid[nxt_pos]
    ox = Wx[nxt_pos] - Wx
    oy = Wy[nxt_pos] - Wy
    if np.abs(ox).max(initial=0) > 1 or np.abs(oy).max(initial=0) > 1:
        raise RuntimeError("an edge spans more than one periodic image")
    # twin: the half-edge of cell orig(q2) dual to the edge towards `owner`
    # seen with the opposite shift.
    nb_o = orig[q2]
    nb_x = shx[q2]
    nb_y = shy[q2]
    W = np.int64(N) * 64
    key_self = owner.astype(np.int64) * W + nb_o * 64 + (nb_x + 2) * 8 + (nb_y + 2)
    key_twin = nb_o.astype(np.int64) * W + owner * 64 + (-nb_x + 2) * 8 + (-nb_y + 2)
    srt = np.argsort(key_self)
    loc = np.clip(np.searchsorted(key_self[srt], key_twin), 0, key_self.size - 1)
    twin_cm = srt[loc]
    if not np.all(key_self[twin_cm] == key_twin):
        raise RuntimeError("twin lookup failed")
    if np.any(twin_cm < 0) or np.any(twin_cm[twin_cm] != np.arange(twin_cm.size)):
        raise RuntimeError("twin relation is not an involution")

    # Renumber half-edges so that twins are adjacent: edge e = (2e, 2e+1),
    # with the half-edge of the lower cell-major index first.
    n_he = src.size
    lo = np.minimum(np.arange(n_he), twin_cm)
    lo_is_self = np.arange(n_he) == lo
    edge_rank = np.empty(n_he, np.int64)
    reps = np.nonzero(lo_is_self)[0]           # ascending cell-major order
    edge_rank[reps] = np.arange(reps.size)
    new_id = np.empty(n_he, np.int64)
    new_id[reps] = 2 * np.arange(reps.size)
    new_id[twin_cm[reps]] = 2 * np.arange(reps.size) + 1
    prev_cm = start[owner] + (k_in - 1) % cnt[owner]
    nxt_cm = nxt_pos
    he = np.empty((n_he, 8), np.int64)
    he[new_id, HE_PREV] = new_id[prev_cm]
    he[new_id, HE_NEXT] = new_id[nxt_cm]
    he[new_id, HE_TWIN] = new_id[twin_cm]
    he[new_id, HE_SRC] = src
    he[new_id, HE_TGT] = tgt
    he[new_id, HE_FACE] = owner
    he[new_id, HE_OX] = ox
    he[new_id, HE_OY] = oy
    if sort:
        # Edges along the vertex order too (by their lower vertex id), so
        # that per-edge data of neighbouring vertices sits close together.
        n_e = n_he // 2
        emin = np.minimum(he[0::2, HE_SRC], he[0::2, HE_TGT])
        emax = np.maximum(he[0::2, HE_SRC], he[0::2, HE_TGT])
        eperm = np.lexsort((emax, emin))            # new edge k = old edge eperm[k]
        erank = np.empty(n_e, np.int64)
        erank[eperm] = np.arange(n_e)
        hmap = np.empty(n_he, np.int64)             # old half-edge id -> new
        hmap[0::2] = 2 * erank
        hmap[1::2] = 2 * erank + 1
        he2 = np.empty_like(he)
        he2[hmap] = he
        for col in (HE_PREV, HE_NEXT, HE_TWIN):
            he2[:, col] = hmap[he2[:, col]]
        he = he2
    return Tissue(he.astype(np.int32), Xv, float(Lx), float(Ly), seeds)


def random_tissue(n_cell: int, L: float | None = None, seed: int = 0,
                  rng: np.random.Generator | None = None) -> Tissue:
    """Periodic Voronoi of `n_cell` uniform-random seeds in a square box.

    The box side defaults to sqrt(n_cell) (unit mean cell area)."""
    if L is None:
        L = float(np.sqrt(n_cell))
    if rng is None:
        rng = np.random.default_rng(seed)
    seeds = rng.uniform(0.0, L, size=(n_cell, 2))
    return periodic_voronoi(seeds, L, L)


def hex_lattice(nx: int, ny: int, s: float, shift=(0.123, 0.071)) -> Tissue:
    """Regular hexagonal tiling (pointy-top hexagons of side s).

    Built as the periodic Voronoi tessellation of a triangular lattice of
    seeds: spacing sqrt(3)*s along rows, rows 1.5*s apart, odd rows offset by
    half a spacing.  The box is (nx*sqrt(3)*s) x (1.5*ny*s); ny must be even.
    """
    if ny % 2 or nx < 3 or ny < 4:
        raise ValueError("hex_lattice needs nx >= 3 and an even ny >= 4")
    a = np.sqrt(3.0) * s
    Lx, Ly = nx * a, 1.5 * ny * s
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    x = ii * a + (jj % 2) * (a / 2) + shift[0] * s
    y = jj * 1.5 * s + shift[1] * s
    seeds = np.stack([x.ravel() % Lx, y.ravel() % Ly], 1)
    return periodic_voronoi(seeds, Lx, Ly, sort=False)


# ---------------------------------------------------------------------------
# Workload recipes: tissues plus parameters, drawn from one RNG stream per
# workload (seeds first, then the parameters).
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Params:
    KA: np.ndarray   # [n_cell]
    A0: np.ndarray   # [n_cell]
    KP: np.ndarray   # [n_cell]
    P0: np.ndarray   # [n_cell]
    lam: np.ndarray  # [n_edge]

    def copy(self) -> "Params":
        return Params(self.KA.copy(), self.A0.copy(), self.KP.copy(),
                      self.P0.copy(), self.lam.copy())


def uniform_params(t: Tissue, KA=1.0, A0=1.0, KP=1.0, P0=3.8, lam=0.0) -> Params:
    c, e = t.n_cell, t.n_edge
    return Params(np.full(c, float(KA)), np.full(c, float(A0)), np.full(c, float(KP)),
                  np.full(c, float(P0)), np.full(e, float(lam)))


def workload_single_100(seed: int = 101):
    """100 cells, box side 10, K_A=A0=K_P=1, P0=3.8, no line tension."""
    rng = np.random.default_rng(seed)
    t = random_tissue(100, 10.0, rng=rng)
    return t, uniform_params(t, P0=3.8, lam=0.0)


def workload_single_10k(seed: int = 201, n_cell: int = 10000):
    """10^4 cells, box side 100, P0 ~ U[3.6,3.9] per cell,
    lambda ~ N(0.1, 0.02^2) clipped at 0 per edge."""
    rng = np.random.default_rng(seed)
    t = random_tissue(n_cell, float(np.sqrt(n_cell)), rng=rng)
    p = uniform_params(t)
    p.P0 = rng.uniform(3.6, 3.9, t.n_cell)
    p.lam = np.clip(rng.normal(0.1, 0.02, t.n_edge), 0.0, None)
    return t, p


def workload_force_1m(seed: int = 301, n_cell: int = 1000000):
    """10^6 cells, box side 1000, P0=3.75, lambda ~ U[0.05,0.15]."""
    rng = np.random.default_rng(seed)
    t = random_tissue(n_cell, float(np.sqrt(n_cell)), rng=rng)
    p = uniform_params(t, P0=3.75)
    p.lam = rng.uniform(0.05, 0.15, t.n_edge)
    return t, p


def workload_batch(seed: int = 401, n_tissue: int = 512, n_min: int = 64, n_max: int = 4096):
    """Independent tissues with N ~ U{n_min..n_max}, box side sqrt(N),
    one P0 ~ U[3.6,3.9] per tissue, lambda ~ U[0,0.2] per edge."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_min, n_max + 1, size=n_tissue)
    out = []
    for n in sizes:
        t = random_tissue(int(n), float(np.sqrt(n)), rng=rng)
        p = uniform_params(t, P0=float(rng.uniform(3.6, 3.9)))
        p.lam = rng.uniform(0.0, 0.2, t.n_edge)
        out.append((t, p))
    return out


def workload_inverse(seed: int = 501, n_tissue: int = 64, n_cell: int = 1000):
    """Tissues of n_cell cells (box sqrt(n_cell)), P0=3.75; hidden tensions
    lambda* and initial tensions theta0 both ~ U[0.05,0.15] (separate
    streams).  Returns [(tissue, params_star, params_init)]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_tissue):
        t = random_tissue(n_cell, float(np.sqrt(n_cell)), rng=rng)
        ps = uniform_params(t, P0=3.75)
        pi = uniform_params(t, P0=3.75)
        ps.lam = rng.uniform(0.05, 0.15, t.n_edge)
        pi.lam = rng.uniform(0.05, 0.15, t.n_edge)
        out.append((t, ps, pi))
    return out
