// Device functions shared by the grid kernels and the persistent batch
// kernel of libvtx.  Formulas follow VertAX (arXiv 2604.06896), Methods,
// "Vertex model formulation": E = sum_c K_A (A-A0)^2 + K_P (P-P0)^2 +
// sum_e lambda l, with the force derived per vertex from the three cells
// and three edges around it.
#pragma once

#include "vtx_internal.h"

namespace vtx {

// ---------------------------------------------------------------- cells
// Area and perimeter of one cell from its corner row.  Corner k is packed
// as vertex id + image (W_k) relative to corner 0; positions are taken
// relative to corner 0 (r_0 = 0) so the shoelace sum never sees absolute
// coordinates:  A = 1/2 sum_k r_{k-1} x r_k,  P = sum_k |r_k - r_{k-1}|.
// When `det` is set, edges shorter than sqrt(lmin2) whose source id is below
// the target id (one half-edge of each edge) are appended to `list` as the
// global index of their source corner.
template <typename PosT, typename M, typename CornerAt>
__device__ __forceinline__ void cell_geom(const DevTissue &t, const PosT *__restrict__ X,
                                          int n, CornerAt corner_at, int row_base, M &A, M &P,
                                          bool det, M lmin2, int32_t *list,
                                          unsigned int *count) {
    const PosT Lx = (PosT)t.Lx, Ly = (PosT)t.Ly;
    // The first U corners: ids, then all their positions in flight at once
    // (rows beyond U sides take the loop below).
    constexpr int U = 8;
    int32_t w[U];
    typename Vec2<PosT>::type q[U];
#pragma unroll
    for (int k = 0; k < U; ++k) w[k] = corner_at(k < n ? k : 0);
#pragma unroll
    for (int k = 0; k < U; ++k) q[k] = ld2(X, id_of(w[k]));
    const auto p0 = q[0];
    const int v0 = id_of(w[0]);
    M px = 0, py = 0, a = 0, per = 0;
    int vprev = v0;
    auto step = [&](int k, int32_t wk, typename Vec2<PosT>::type qk) {
        const int v = id_of(wk);
        const M rx = (M)pdiff<PosT>(qk.x, p0.x, ox_of(wk), Lx);
        const M ry = (M)pdiff<PosT>(qk.y, p0.y, oy_of(wk), Ly);
        const M dx = rx - px, dy = ry - py;
        const M l2 = dx * dx + dy * dy;
        a += px * ry - py * rx;
        per += sqrt(l2);
        if (det && l2 < lmin2 && vprev < v) {
            unsigned int s = atomicAdd(count, 1u);
            list[s] = row_base + k - 1;
        }
        px = rx;
        py = ry;
        vprev = v;
    };
#pragma unroll
    for (int k = 1; k < U; ++k)
        if (k < n) step(k, w[k], q[k]);
    for (int k = U; k < n; ++k) {
        const int32_t wk = corner_at(k);
        step(k, wk, ld2(X, id_of(wk)));
    }
    const M l2 = px * px + py * py;  // closing edge, corner n-1 -> corner 0
    per += sqrt(l2);
    if (det && l2 < lmin2 && vprev < v0) {
        unsigned int s = atomicAdd(count, 1u);
        list[s] = row_base + n - 1;
    }
    A = (M)0.5 * a;
    P = per;
}

// ---------------------------------------------------------------- vertex
// Force on vertex i from its star (outgoing half-edges h_k = i -> j_k,
// sector cell a_k = face(h_k), edge e_k).  With d_k = x_{j_k} - x_i,
// u_k = d_k / l_k and R(a) = (a_y, -a_x):
//   F_i = sum_k [ u_k (lambda_k + cP(a_k) + cP(a_{k-1}))
//                 - 1/2 R(d_k) (cA(a_k) - cA(a_{k-1})) ],
// cA = 2 K_A (A - A0), cP = 2 K_P (P - P0), indices mod 3.  This is
// -grad_i of the energy: the perimeter and line-tension terms pull along
// each edge, the area terms push across it by the pressure difference.
template <typename PosT, typename M>
struct Star {
    M dx[3], dy[3], ux[3], uy[3], l[3], inv[3];
    M cA[3], cP[3], lam[3];
    int nb[3];
};

template <typename PosT, typename M>
__device__ __forceinline__ void load_star(const DevTissue &t, const PosT *__restrict__ X,
                                          const DevParams<PosT> &p, const M *__restrict__ cap,
                                          int v, Star<PosT, M> &s, PosT &xi, PosT &yi) {
    const PosT Lx = (PosT)t.Lx, Ly = (PosT)t.Ly;
    const int nv = t.n_vert;
    // 1) the star (9 coalesced dword loads) and the own position
    int32_t w[3], c[3], e[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        w[k] = t.star_nb[k * nv + v];
        c[k] = t.star_cell[k * nv + v];
        e[k] = t.star_edge[k * nv + v];
    }
    const auto pi = ld2(X, v);
    // 2) every gather issued before any is used
    typename Vec2<PosT>::type q[3];
    typename Vec2<M>::type cc[3];
    PosT lam[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        q[k] = ld2(X, id_of(w[k]));
        cc[k] = ld2(cap, c[k]);
    }
    if (p.lam) {
#pragma unroll
        for (int k = 0; k < 3; ++k) lam[k] = p.lam[e[k]];
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) lam[k] = p.lam_s;
    }
    xi = pi.x;
    yi = pi.y;
    // 3) arithmetic
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        s.nb[k] = id_of(w[k]);
        s.dx[k] = (M)pdiff<PosT>(q[k].x, pi.x, ox_of(w[k]), Lx);
        s.dy[k] = (M)pdiff<PosT>(q[k].y, pi.y, oy_of(w[k]), Ly);
        s.cA[k] = cc[k].x;
        s.cP[k] = cc[k].y;
        s.lam[k] = (M)lam[k];
        const M l = sqrt(s.dx[k] * s.dx[k] + s.dy[k] * s.dy[k]);
        // a zero-length edge contributes its minimum-norm subgradient, 0
        const M inv = l > (M)0 ? (M)1 / l : (M)0;
        s.l[k] = l;
        s.inv[k] = inv;
        s.ux[k] = s.dx[k] * inv;
        s.uy[k] = s.dy[k] * inv;
    }
}

template <typename PosT, typename M>
__device__ __forceinline__ void star_force(const Star<PosT, M> &s, M &fx, M &fy) {
    fx = 0;
    fy = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int km = (k + 2) % 3;
        const M T = s.lam[k] + s.cP[k] + s.cP[km];
        const M dA = (M)0.5 * (s.cA[k] - s.cA[km]);
        fx += T * s.ux[k] - dA * s.dy[k];
        fy += T * s.uy[k] + dA * s.dx[k];
    }
}

// ---------------------------------------------------------- T1 helpers
// Exact (double) helpers used by the sequential T1 pass.  Positions of the
// two vertices of the edge under test can be overridden.
template <typename PosT>
struct PosOverride {
    int vi, vj;
    double xi, yi, xj, yj;
    __device__ __forceinline__ void get(const PosT *X, int v, double &x, double &y) const {
        if (v == vi) { x = xi; y = yi; }
        else if (v == vj) { x = xj; y = yj; }
        else { x = (double)X[2 * (int64_t)v]; y = (double)X[2 * (int64_t)v + 1]; }
    }
};

template <typename PosT>
__device__ __forceinline__ void he_vec(const DevTissue &t, const PosT *X, int h,
                                       const PosOverride<PosT> &ov, double &dx, double &dy) {
    const int32_t *r = t.he + 8 * (int64_t)h;
    double xs, ys, xg, yg;
    ov.get(X, r[HS], xs, ys);
    ov.get(X, r[HG], xg, yg);
    dx = pdiff<double>(xg, xs, r[HOX], t.Lx);
    dy = pdiff<double>(yg, ys, r[HOY], t.Ly);
}

template <typename PosT>
__device__ __forceinline__ void cell_walk(const DevTissue &t, const PosT *X, int h0,
                                          const PosOverride<PosT> &ov, double &A, double &P) {
    double rx = 0.0, ry = 0.0, a = 0.0, per = 0.0;
    int h = h0;
    int guard = 0;
    do {
        double dx, dy;
        he_vec<PosT>(t, X, h, ov, dx, dy);
        a += rx * dy - ry * dx;
        per += sqrt(dx * dx + dy * dy);
        rx += dx;
        ry += dy;
        h = t.he[8 * (int64_t)h + HN];
    } while (h != h0 && ++guard < 4096);
    A = 0.5 * a;
    P = per;
}

template <typename PosT>
__device__ __forceinline__ double cell_energy(const DevParams<PosT> &p, int c, double A,
                                              double P) {
    const double da = A - (double)p.a0(c), dp = P - (double)p.p0(c);
    return (double)p.ka(c) * da * da + (double)p.kp(c) * dp * dp;
}

__device__ __forceinline__ void star_refresh(const DevTissue &t, int v, int h0) {
    const int nv = t.n_vert;
    int h = h0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int32_t *r = t.he + 8 * (int64_t)h;
        t.star_he[k * nv + v] = h;
        t.star_nb[k * nv + v] = pack_id(r[HG], r[HOX], r[HOY]);
        t.star_cell[k * nv + v] = r[HF];
        t.star_edge[k * nv + v] = t.he_edge[h];
        h = t.he[8 * (int64_t)t.he[8 * (int64_t)h + HP] + HT];  // twin(prev(h))
    }
}

// Cell-term coefficients of one cell recomputed exactly after a T1 step.
template <typename PosT, typename M>
__device__ __forceinline__ void cell_refresh_cap(const DevTissue &t, const PosT *X,
                                                 const DevParams<PosT> &p, M *cap, int c,
                                                 int h0) {
    PosOverride<PosT> none{-1, -1, 0, 0, 0, 0};
    double A, P;
    cell_walk<PosT>(t, X, h0, none, A, P);
    cap[2 * (int64_t)c] = (M)(2.0 * (double)p.ka(c) * (A - (double)p.a0(c)));
    cap[2 * (int64_t)c + 1] = (M)(2.0 * (double)p.kp(c) * (P - (double)p.p0(c)));
}

// Half-edge records changed by one neighbour exchange, saved for undo.
struct T1Save {
    int32_t id[10];
    int32_t rec[10][8];
};

// Neighbour exchange of the edge of half-edge h (i -> j in C1, its twin
// j -> i in C2; C3 is the third cell at i, C4 the third cell at j).
// Afterwards h bounds C4 and its twin bounds C3, the edge to c (next of h
// in C1) moves from j to i and the edge to b (next of the twin in C2) from
// i to j; the moved half-edges change image offset by the offset of h so
// that every edge vector is kept.
__device__ __forceinline__ void t1_patch(const DevTissue &t, int h, T1Save *save) {
    int32_t *he = t.he;
    auto R = [&](int x) { return he + 8 * (int64_t)x; };
    const int tw = R(h)[HT];
    const int i = R(h)[HS], j = R(h)[HG];
    const int p1 = R(h)[HP], n1 = R(h)[HN];
    const int p2 = R(tw)[HP], n2 = R(tw)[HN];
    const int tp1 = R(p1)[HT], tn1 = R(n1)[HT];
    const int tp2 = R(p2)[HT], tn2 = R(n2)[HT];
    const int C3 = R(tp1)[HF], C4 = R(tn1)[HF];
    if (save) {
        const int ids[10] = {h, tw, p1, n1, p2, n2, tp1, tn1, tp2, tn2};
        for (int a = 0; a < 10; ++a) {
            save->id[a] = ids[a];
            for (int b = 0; b < 8; ++b) save->rec[a][b] = R(ids[a])[b];
        }
    }
    const int hox = R(h)[HOX], hoy = R(h)[HOY];
    // C1: a->i -> i->c
    R(p1)[HN] = n1;
    R(n1)[HP] = p1;
    R(n1)[HS] = i;
    R(tn1)[HG] = i;
    R(n1)[HOX] += hox;
    R(n1)[HOY] += hoy;
    R(tn1)[HOX] = -R(n1)[HOX];
    R(tn1)[HOY] = -R(n1)[HOY];
    // C2: d->j -> j->b
    R(p2)[HN] = n2;
    R(n2)[HP] = p2;
    R(n2)[HS] = j;
    R(tn2)[HG] = j;
    R(n2)[HOX] -= hox;
    R(n2)[HOY] -= hoy;
    R(tn2)[HOX] = -R(n2)[HOX];
    R(tn2)[HOY] = -R(n2)[HOY];
    // C4: c->i -> i->j -> j->d
    R(tn1)[HN] = h;
    R(h)[HP] = tn1;
    R(h)[HN] = tp2;
    R(tp2)[HP] = h;
    R(h)[HF] = C4;
    // C3: b->j -> j->i -> i->a
    R(tn2)[HN] = tw;
    R(tw)[HP] = tn2;
    R(tw)[HN] = tp1;
    R(tp1)[HP] = tw;
    R(tw)[HF] = C3;
}

__device__ __forceinline__ void t1_restore(const DevTissue &t, const T1Save &s) {
    for (int a = 0; a < 10; ++a)
        for (int b = 0; b < 8; ++b) t.he[8 * (int64_t)s.id[a] + b] = s.rec[a][b];
}

__device__ __forceinline__ int face_sides(const DevTissue &t, int h0) {
    int n = 0, h = h0;
    do {
        ++n;
        h = t.he[8 * (int64_t)h + HN];
    } while (h != h0 && n < 4096);
    return n;
}

// Result of one sequential T1 pass.
struct T1Counts {
    int64_t swaps, stretches;
    int changed;
    int overflow;
};

// Insert edge e into the small pending set `extra` (unsorted) if absent.
__device__ __forceinline__ bool extra_insert(int32_t *extra, int &n_extra, int e) {
    for (int a = 0; a < n_extra; ++a)
        if (extra[a] == e) return true;
    if (n_extra >= kT1Extra) return false;
    extra[n_extra++] = e;
    return true;
}

// Sequential T1 pass over the ascending candidate list `list[0..n)` (edge
// ids, sorted, may hold duplicates and INT_MAX padding), run by ONE thread.
// Each candidate is re-checked with the current positions; edges next to a
// processed edge that become short are visited in turn as well, so the
// result equals visiting every edge in ascending id order.
template <typename PosT, typename M>
__device__ T1Counts t1_sequential(const DevTissue &t, PosT *X, const DevParams<PosT> &p,
                                  M *cap, const int32_t *list, int n, int32_t *extra,
                                  double l_min, double l_new) {
    T1Counts out{0, 0, 0, 0};
    int pos = 0, n_extra = 0;
    int last = -1;
    const double hl = 0.5 * l_new;
    for (;;) {
        // next edge: min of list[pos] and the pending set
        int e = 0x7fffffff, ea = -1;
        while (pos < n && list[pos] <= last) ++pos;
        if (pos < n) e = list[pos];
        for (int a = 0; a < n_extra; ++a)
            if (extra[a] <= last) {
                extra[a] = extra[--n_extra];
                --a;
            }
        for (int a = 0; a < n_extra; ++a)
            if (extra[a] < e) { e = extra[a]; ea = a; }
        if (e == 0x7fffffff) break;
        if (ea >= 0) extra[ea] = extra[--n_extra];
        else ++pos;
        last = e;

        const int h = t.edge_he[e];
        const int32_t *rh = t.he + 8 * (int64_t)h;
        const int i = rh[HS], j = rh[HG];
        const int ohx = rh[HOX], ohy = rh[HOY];
        const double xi = (double)X[2 * (int64_t)i], yi = (double)X[2 * (int64_t)i + 1];
        const double xj = (double)X[2 * (int64_t)j], yj = (double)X[2 * (int64_t)j + 1];
        const double dx = pdiff<double>(xj, xi, ohx, t.Lx), dy = pdiff<double>(yj, yi, ohy, t.Ly);
        const double l = sqrt(dx * dx + dy * dy);
        if (!(l < l_min)) continue;
        double ux = 1.0, uy = 0.0;
        if (l > 0.0) { ux = dx / l; uy = dy / l; }
        const double mx = xi + 0.5 * dx, my = yi + 0.5 * dy;
        const double sx = ohx * t.Lx, sy = ohy * t.Ly;
        PosOverride<PosT> S{i, j, mx - hl * ux, my - hl * uy, mx + hl * ux - sx, my + hl * uy - sy};
        const double nx = -uy, ny = ux;
        PosOverride<PosT> T{i, j, mx + hl * nx, my + hl * ny, mx - hl * nx - sx, my - hl * ny - sy};

        const int tw = rh[HT];
        const int p1 = rh[HP], n1 = rh[HN];
        const int p2 = t.he[8 * (int64_t)tw + HP], n2 = t.he[8 * (int64_t)tw + HN];
        const int tp1 = t.he[8 * (int64_t)p1 + HT], tn1 = t.he[8 * (int64_t)n1 + HT];
        const int tp2 = t.he[8 * (int64_t)p2 + HT];
        const int C1 = rh[HF], C2 = t.he[8 * (int64_t)tw + HF];
        const int C3 = t.he[8 * (int64_t)tp1 + HF], C4 = t.he[8 * (int64_t)tn1 + HF];
        const bool distinct = C1 != C2 && C1 != C3 && C1 != C4 && C2 != C3 && C2 != C4 && C3 != C4;
        bool take_T = false;
        if (distinct && t.nsides[C1] > 3 && t.nsides[C2] > 3) {
            // local energies: the four cells around the edge and the five
            // edges ending at i or j (everything else is unchanged)
            const int cells[4] = {C1, C2, C3, C4};
            const int walk[4] = {p1, p2, tp1, tp2};  // half-edges in these cells before and after
            const int edges[5] = {h, p1, n1, p2, n2};
            double ES = 0.0, ET = 0.0;
            for (int a = 0; a < 4; ++a) {
                double A, P;
                cell_walk<PosT>(t, X, walk[a], S, A, P);
                ES += cell_energy<PosT>(p, cells[a], A, P);
            }
            for (int a = 0; a < 5; ++a) {
                double ex, ey;
                he_vec<PosT>(t, X, edges[a], S, ex, ey);
                ES += (double)p.lm(t.he_edge[edges[a]]) * sqrt(ex * ex + ey * ey);
            }
            T1Save sv;
            t1_patch(t, h, &sv);
            for (int a = 0; a < 4; ++a) {
                double A, P;
                cell_walk<PosT>(t, X, walk[a], T, A, P);
                ET += cell_energy<PosT>(p, cells[a], A, P);
            }
            for (int a = 0; a < 5; ++a) {
                double ex, ey;
                he_vec<PosT>(t, X, edges[a], T, ex, ey);
                ET += (double)p.lm(t.he_edge[edges[a]]) * sqrt(ex * ex + ey * ey);
            }
            take_T = ET < ES;
            if (!take_T) t1_restore(t, sv);
        }
        const PosOverride<PosT> &W = take_T ? T : S;
        X[2 * (int64_t)i] = (PosT)W.xi;
        X[2 * (int64_t)i + 1] = (PosT)W.yi;
        X[2 * (int64_t)j] = (PosT)W.xj;
        X[2 * (int64_t)j + 1] = (PosT)W.yj;
        if (take_T) {
            ++out.swaps;
            out.changed = 1;
            t.nsides[C1] -= 1;
            t.nsides[C2] -= 1;
            t.nsides[C3] += 1;
            t.nsides[C4] += 1;
            if (t.cell_he[C1] == h) t.cell_he[C1] = n1;
            if (t.cell_he[C2] == tw) t.cell_he[C2] = n2;
            // stars of i and j are rebuilt; c and b changed neighbour
            star_refresh(t, i, h);
            star_refresh(t, j, tw);
            star_refresh(t, t.he[8 * (int64_t)n1 + HG], tn1);   // c
            star_refresh(t, t.he[8 * (int64_t)n2 + HG], t.he[8 * (int64_t)n2 + HT]);  // b
        } else {
            ++out.stretches;
        }
        // cell terms of the four cells around the edge, exactly
        cell_refresh_cap<PosT, M>(t, X, p, cap, C1, p1);
        cell_refresh_cap<PosT, M>(t, X, p, cap, C2, p2);
        cell_refresh_cap<PosT, M>(t, X, p, cap, C3, tp1);
        cell_refresh_cap<PosT, M>(t, X, p, cap, C4, tp2);
        // the four other edges at i and j may have become short
        const int nbr[4] = {p1, n1, p2, n2};
        for (int a = 0; a < 4; ++a) {
            const int e2 = t.he_edge[nbr[a]];
            if (e2 <= e) continue;
            PosOverride<PosT> none{-1, -1, 0, 0, 0, 0};
            double ex, ey;
            he_vec<PosT>(t, X, nbr[a], none, ex, ey);
            if (sqrt(ex * ex + ey * ey) < l_min)
                if (!extra_insert(extra, n_extra, e2)) out.overflow = 1;
        }
    }
    return out;
}

// Block-wide bitonic sort (ascending) of `a[0..n)`, n a power of two.
__device__ __forceinline__ void block_bitonic(int32_t *a, int n) {
    for (int k = 2; k <= n; k <<= 1)
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const int ixj = i ^ jj;
                if (ixj > i) {
                    const bool asc = (i & k) == 0;
                    const int32_t x = a[i], y = a[ixj];
                    if ((x > y) == asc) {
                        a[i] = y;
                        a[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
}

// Rebuild the cell -> corner rows from the half-edge table (block-wide):
// row_ptr is the exclusive scan of nsides, each row is walked from
// cell_he[c] with the cumulative image of each corner.  Returns nonzero
// (in thread 0) if a cell spans more than one periodic image.
__device__ __forceinline__ int rebuild_rows_block(const DevTissue &t, int32_t *sh_scan) {
    __shared__ int32_t carry;
    __shared__ int bad;
    if (threadIdx.x == 0) { carry = 0; bad = 0; }
    __syncthreads();
    const int nc = t.n_cell;
    for (int base = 0; base < nc; base += blockDim.x) {
        const int c = base + threadIdx.x;
        const int v = c < nc ? t.nsides[c] : 0;
        sh_scan[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < (int)blockDim.x; off <<= 1) {
            int add = threadIdx.x >= (unsigned)off ? sh_scan[threadIdx.x - off] : 0;
            __syncthreads();
            sh_scan[threadIdx.x] += add;
            __syncthreads();
        }
        if (c < nc) t.row_ptr[c] = carry + sh_scan[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry += sh_scan[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) t.row_ptr[nc] = carry;
    __syncthreads();
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const int h0 = t.cell_he[c];
        int base = t.row_ptr[c];
        int wx = 0, wy = 0, h = h0, k = 0;
        do {
            const int32_t *r = t.he + 8 * (int64_t)h;
            if (wx < -1 || wx > 1 || wy < -1 || wy > 1) bad = 1;
            t.corner[base + k] = pack_id(r[HS], wx, wy);
            t.corner_he[base + k] = h;
            wx += r[HOX];
            wy += r[HOY];
            h = r[HN];
            ++k;
        } while (h != h0 && k < 4096);
    }
    __syncthreads();
    return bad;
}

// ------------------------------------------------------------------- HVP
// Directional derivatives of one cell's area and perimeter along v, in the
// precision of the positions:
//   dA = sum_k grad_k A . v_k,  grad_k A = 1/2 R(r_{k+1} - r_{k-1});
//   dP = sum_k u_k . (v_{k+1} - v_k)  (zero-length edges contribute 0).
// Stored as (G, B) = (2 K_A dA, 2 K_P dP).
template <typename PosT, typename M>
__device__ __forceinline__ void hvp_cell_one(const DevTissue &t, const PosT *__restrict__ X,
                                             const DevParams<PosT> &p,
                                             const double *__restrict__ v, M *__restrict__ aux,
                                             int c) {
    using C = PosT;
    const PosT Lx = (PosT)t.Lx, Ly = (PosT)t.Ly;
    const int rb = t.row_ptr[c], n = t.row_ptr[c + 1] - rb;
    const int32_t w0 = t.corner[rb];
    const auto p0 = ld2(X, id_of(w0));
    auto rel = [&](int k, C &rx, C &ry, C &vx, C &vy) {
        const int32_t w = t.corner[rb + k];
        const int vv = id_of(w);
        if (k == 0) {
            rx = 0;
            ry = 0;
        } else {
            const auto q = ld2(X, vv);
            rx = (C)pdiff<PosT>(q.x, p0.x, ox_of(w), Lx);
            ry = (C)pdiff<PosT>(q.y, p0.y, oy_of(w), Ly);
        }
        const auto vq = ld2(v, vv);
        vx = (C)vq.x;
        vy = (C)vq.y;
    };
    C rpx, rpy, vd0, vd1;
    rel(n - 1, rpx, rpy, vd0, vd1);
    C rcx, rcy, vcx, vcy;
    rel(0, rcx, rcy, vcx, vcy);
    C dA = 0, dP = 0;
    for (int k = 0; k < n; ++k) {
        const int kn = (k + 1 == n) ? 0 : k + 1;
        C rnx, rny, vnx, vny;
        rel(kn, rnx, rny, vnx, vny);
        const C gx = (C)0.5 * (rny - rpy), gy = (C)-0.5 * (rnx - rpx);
        dA += gx * vcx + gy * vcy;
        const C dx = rnx - rcx, dy = rny - rcy;
        const C l = sqrt(dx * dx + dy * dy);
        if (l > (C)0) dP += (dx * (vnx - vcx) + dy * (vny - vcy)) / l;
        rpx = rcx;
        rpy = rcy;
        rcx = rnx;
        rcy = rny;
        vcx = vnx;
        vcy = vny;
    }
    st2(aux, c, (M)((C)2 * (C)p.ka(c) * dA), (M)((C)2 * (C)p.kp(c) * dP));
}

// (H v)_i = sum_k [ T_k w_k - u_k (B_k + B_{k-1}) + 1/2 R(d_k)(G_k - G_{k-1})
//                   + 1/2 R(v_{j_k} - v_i)(cA_k - cA_{k-1}) ]
// with w_k = (I - u_k u_k^T)(v_i - v_{j_k}) / l_k, T_k the edge tension
// (lambda_k + cP_k + cP_{k-1}), G = 2K_A dA and B = 2K_P dP of the sector
// cells.  Writes (Hv)_i and returns v_i . (Hv)_i.
template <typename PosT, typename M>
__device__ __forceinline__ double hvp_vertex_one(const DevTissue &t, const PosT *__restrict__ X,
                                                 const DevParams<PosT> &p,
                                                 const M *__restrict__ cap,
                                                 const M *__restrict__ aux,
                                                 const double *__restrict__ v,
                                                 double *__restrict__ Hv, int i) {
    Star<PosT, M> s;
    PosT xi, yi;
    load_star<PosT, M>(t, X, p, cap, i, s, xi, yi);
    const auto vi = ld2(v, i);
    M G[3], B[3], vx[3], vy[3];
    const int nv = t.n_vert;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const auto g = ld2(aux, t.star_cell[k * nv + i]);
        G[k] = g.x;
        B[k] = g.y;
        const auto vj = ld2(v, s.nb[k]);
        vx[k] = (M)(vj.x - vi.x);  // v_{j_k} - v_i
        vy[k] = (M)(vj.y - vi.y);
    }
    M hx = 0, hy = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int km = (k + 2) % 3;
        const M T = s.lam[k] + s.cP[k] + s.cP[km];
        const M du = -(vx[k] * s.ux[k] + vy[k] * s.uy[k]);  // (v_i - v_j) . u
        const M wx = (-vx[k] - du * s.ux[k]) * s.inv[k];
        const M wy = (-vy[k] - du * s.uy[k]) * s.inv[k];
        const M Bs = B[k] + B[km];
        const M dG = (M)0.5 * (G[k] - G[km]);
        const M dC = (M)0.5 * (s.cA[k] - s.cA[km]);
        hx += T * wx - s.ux[k] * Bs + dG * s.dy[k] + dC * vy[k];
        hy += T * wy - s.uy[k] * Bs - dG * s.dx[k] - dC * vx[k];
    }
    st2(Hv, i, (double)hx, (double)hy);
    return vi.x * (double)hx + vi.y * (double)hy;
}

// ------------------------------------------------------------ contractions
// theta = lambda:  g_e = -(d2E/dX dlambda_e) . mu = -u_e . (mu_tgt - mu_src)
template <typename PosT>
__device__ __forceinline__ double contract_lambda_one(const DevTissue &t, const PosT *X,
                                                      const double *mu, int e) {
    const int32_t *r = t.he + 8 * (int64_t)t.edge_he[e];
    const int s = r[HS], q = r[HG];
    const double dx = pdiff<double>((double)X[2 * (int64_t)q], (double)X[2 * (int64_t)s], r[HOX], t.Lx);
    const double dy = pdiff<double>((double)X[2 * (int64_t)q + 1], (double)X[2 * (int64_t)s + 1], r[HOY], t.Ly);
    const double l = sqrt(dx * dx + dy * dy);
    return l > 0.0 ? -(dx * (mu[2 * (int64_t)q] - mu[2 * (int64_t)s]) +
                       dy * (mu[2 * (int64_t)q + 1] - mu[2 * (int64_t)s + 1])) / l
                   : 0.0;
}

// theta = P0:  g_c = -(d2E/dX dP0_c) . mu = 2 K_P grad P_c . mu
template <typename PosT>
__device__ __forceinline__ double contract_p0_one(const DevTissue &t, const PosT *X,
                                                  const DevParams<PosT> &p, const double *mu,
                                                  int c) {
    const int rb = t.row_ptr[c], n = t.row_ptr[c + 1] - rb;
    double dP = 0.0;
    for (int k = 0; k < n; ++k) {
        const int h = t.corner_he[rb + k];
        const int32_t *r = t.he + 8 * (int64_t)h;
        const int s = r[HS], q = r[HG];
        const double dx = pdiff<double>((double)X[2 * (int64_t)q], (double)X[2 * (int64_t)s], r[HOX], t.Lx);
        const double dy = pdiff<double>((double)X[2 * (int64_t)q + 1], (double)X[2 * (int64_t)s + 1], r[HOY], t.Ly);
        const double l = sqrt(dx * dx + dy * dy);
        if (l > 0.0)
            dP += (dx * (mu[2 * (int64_t)q] - mu[2 * (int64_t)s]) +
                   dy * (mu[2 * (int64_t)q + 1] - mu[2 * (int64_t)s + 1])) / l;
    }
    return 2.0 * (double)p.kp(c) * dP;
}

// Edge length in double from positions of any precision.
template <typename PosT>
__device__ __forceinline__ double edge_len_one(const DevTissue &t, const PosT *X, int e) {
    const int32_t *r = t.he + 8 * (int64_t)t.edge_he[e];
    const int s = r[HS], q = r[HG];
    const double dx = pdiff<double>((double)X[2 * (int64_t)q], (double)X[2 * (int64_t)s], r[HOX], t.Lx);
    const double dy = pdiff<double>((double)X[2 * (int64_t)q + 1], (double)X[2 * (int64_t)s + 1], r[HOY], t.Ly);
    return sqrt(dx * dx + dy * dy);
}

}  // namespace vtx
