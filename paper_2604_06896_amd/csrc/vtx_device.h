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
// global index of their source corner.  NOIMG: every corner is known to
// carry the zero image, and the periodic differences reduce to plain
// subtractions (the same values).
template <typename PosT, typename M, bool NOIMG = false, typename CornerAt>
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
        const M rx = (M)pdiff<PosT>(qk.x, p0.x, NOIMG ? 0 : ox_of(wk), Lx);
        const M ry = (M)pdiff<PosT>(qk.y, p0.y, NOIMG ? 0 : oy_of(wk), Ly);
        const M dx = rx - px, dy = ry - py;
        const M l2 = dx * dx + dy * dy;
        a += px * ry - py * rx;
        per += len_of(l2);
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
    per += len_of(l2);
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

// A star is loaded in three stages: (1) the star entries (two 16-byte and
// one 4-byte coalesced load) and the own position, (2) every gather they
// index, issued before any is used, (3) the arithmetic.
template <typename PosT, typename M>
struct StarLoad {
    int32_t w[3], c[3], e[3];
    typename Vec2<PosT>::type pi, q[3];
    typename Vec2<M>::type cc[3];
    PosT lam[3];
};

template <typename PosT, typename M>
__device__ __forceinline__ void star_ids(const DevTissue &t, const PosT *__restrict__ X, int v,
                                         StarLoad<PosT, M> &L) {
    const int nv = t.n_vert;
    const int4 a = reinterpret_cast<const int4 *>(t.star)[v];
    const int4 b = reinterpret_cast<const int4 *>(t.star + 4 * (int64_t)nv)[v];
    L.e[2] = t.star[8 * (int64_t)nv + v];
    L.w[0] = a.x;
    L.w[1] = a.y;
    L.w[2] = a.z;
    L.c[0] = a.w;
    L.c[1] = b.x;
    L.c[2] = b.y;
    L.e[0] = b.z;
    L.e[1] = b.w;
    L.pi = ld2(X, v);
}

template <typename PosT, typename M>
__device__ __forceinline__ void star_gather(const PosT *__restrict__ X, const DevParams<PosT> &p,
                                            const M *__restrict__ cap, StarLoad<PosT, M> &L) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        L.q[k] = ld2(X, id_of(L.w[k]));
        L.cc[k] = ld2(cap, L.c[k]);
    }
    if (p.lam) {
#pragma unroll
        for (int k = 0; k < 3; ++k) L.lam[k] = p.lam[L.e[k]];
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) L.lam[k] = p.lam_s;
    }
}

// NOIMG: the three neighbours are known to carry the zero image.  HVP: the
// inverse lengths of the Hessian-vector product (len_inv_hvp).
template <typename PosT, typename M, bool NOIMG = false, bool HVP = false>
__device__ __forceinline__ void star_math(const DevTissue &t, const StarLoad<PosT, M> &L,
                                          Star<PosT, M> &s, PosT &xi, PosT &yi) {
    const PosT Lx = (PosT)t.Lx, Ly = (PosT)t.Ly;
    xi = L.pi.x;
    yi = L.pi.y;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        s.nb[k] = id_of(L.w[k]);
        s.dx[k] = (M)pdiff<PosT>(L.q[k].x, L.pi.x, NOIMG ? 0 : ox_of(L.w[k]), Lx);
        s.dy[k] = (M)pdiff<PosT>(L.q[k].y, L.pi.y, NOIMG ? 0 : oy_of(L.w[k]), Ly);
        s.cA[k] = L.cc[k].x;
        s.cP[k] = L.cc[k].y;
        s.lam[k] = (M)L.lam[k];
        // a zero-length edge contributes its minimum-norm subgradient, 0
        M l, inv;
        if (HVP) len_inv_hvp(s.dx[k] * s.dx[k] + s.dy[k] * s.dy[k], l, inv);
        else len_inv(s.dx[k] * s.dx[k] + s.dy[k] * s.dy[k], l, inv);
        s.l[k] = l;
        s.inv[k] = inv;
        s.ux[k] = s.dx[k] * inv;
        s.uy[k] = s.dy[k] * inv;
    }
}

template <typename PosT, typename M>
__device__ __forceinline__ void load_star(const DevTissue &t, const PosT *__restrict__ X,
                                          const DevParams<PosT> &p, const M *__restrict__ cap,
                                          int v, Star<PosT, M> &s, PosT &xi, PosT &yi) {
    StarLoad<PosT, M> L;
    star_ids<PosT, M>(t, X, v, L);
    star_gather<PosT, M>(X, p, cap, L);
    star_math<PosT, M>(t, L, s, xi, yi);
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

__device__ __forceinline__ void star_refresh(const DevTissue &t, int v, int h0) {
    const int nv = t.n_vert;
    int h = h0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int32_t *r = t.he + 8 * (int64_t)h;
        t.star_he[k * nv + v] = h;
        t.star[star_nb_at(nv, k, v)] = pack_id(r[HG], r[HOX], r[HOY]);
        t.star[star_cell_at(nv, k, v)] = r[HF];
        t.star[star_edge_at(nv, k, v)] = t.he_edge[h];
        h = t.he[8 * (int64_t)t.he[8 * (int64_t)h + HP] + HT];  // twin(prev(h))
    }
}

// ------------------------------------------------------------------- T1
// One half-edge record loaded as two 16-byte vectors.
struct HeRec {
    int prev, next, twin, src, tgt, face, ox, oy;
};
__device__ __forceinline__ HeRec he_rec(const DevTissue &t, int h) {
    const int4 *r = reinterpret_cast<const int4 *>(t.he + 8 * (int64_t)h);
    const int4 a = r[0], b = r[1];
    return HeRec{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
}

// Area and perimeter (FP64) of cell c read from its corner row, with the
// two vertices of the edge under test at overridden positions and one
// optional edit of the corner sequence:
//   edit 1: drop vertex va;
//   edit 2: put vertex vb, at the image of va plus (sx, sy), right before va.
// Coordinates are unwrapped x + W L; the first corner is the origin.  The
// first kRowPre corners and their positions are loaded before any is used.
constexpr int kRowPre = 12;
template <typename PosT>
__device__ __noinline__ void row_geom(const DevTissue &t, const PosT *X, int c,
                                         const PosOverride<PosT> ov, int edit, int va, int vb,
                                         int sx, int sy, double &A, double &P) {
    const int rb = t.row_ptr[c], n = t.nsides[c];
    int32_t w[kRowPre];
    double qx[kRowPre], qy[kRowPre];
#pragma unroll
    for (int k = 0; k < kRowPre; ++k) w[k] = t.corner[rb + (k < n ? k : 0)];
#pragma unroll
    for (int k = 0; k < kRowPre; ++k) ov.get(X, id_of(w[k]), qx[k], qy[k]);
    double x0 = 0.0, y0 = 0.0, px = 0.0, py = 0.0, a = 0.0, per = 0.0;
    bool first = true;
    auto emit = [&](double x, double y, int wx, int wy) {
        const double rx = x + wx * t.Lx, ry = y + wy * t.Ly;
        if (first) {
            x0 = rx;
            y0 = ry;
            first = false;
            return;
        }
        const double ux = rx - x0, uy = ry - y0;
        const double dx = ux - px, dy = uy - py;
        a += px * uy - py * ux;
        per += sqrt(dx * dx + dy * dy);
        px = ux;
        py = uy;
    };
    auto corner = [&](int32_t wk, double x, double y) {
        const int v = id_of(wk);
        if (edit == 2 && v == va) {
            double bx, by;
            ov.get(X, vb, bx, by);
            emit(bx, by, ox_of(wk) + sx, oy_of(wk) + sy);
        }
        if (edit == 1 && v == va) return;
        emit(x, y, ox_of(wk), oy_of(wk));
    };
#pragma unroll
    for (int k = 0; k < kRowPre; ++k)
        if (k < n) corner(w[k], qx[k], qy[k]);
    for (int k = kRowPre; k < n; ++k) {
        const int32_t wk = t.corner[rb + k];
        double x, y;
        ov.get(X, id_of(wk), x, y);
        corner(wk, x, y);
    }
    const double dx = -px, dy = -py;  // closing edge back to the first corner
    per += sqrt(dx * dx + dy * dy);
    A = 0.5 * a;
    P = per;
}

template <typename PosT>
__device__ __forceinline__ double cell_energy(const DevParams<PosT> &p, int c, double A,
                                              double P) {
    const double da = A - (double)p.a0(c), dp = P - (double)p.p0(c);
    return (double)p.ka(c) * da * da + (double)p.kp(c) * dp * dp;
}

// Cell-term coefficients of one cell recomputed (FP64) after a T1 step.
template <typename PosT, typename M>
__device__ __forceinline__ void cell_refresh_cap(const DevTissue &t, const PosT *X,
                                                 const DevParams<PosT> &p, M *cap, int c) {
    PosOverride<PosT> none{-1, -1, 0, 0, 0, 0};
    double A, P;
    row_geom<PosT>(t, X, c, none, 0, -1, -1, 0, 0, A, P);
    cap[2 * (int64_t)c] = (M)(2.0 * (double)p.ka(c) * (A - (double)p.a0(c)));
    cap[2 * (int64_t)c + 1] = (M)(2.0 * (double)p.kp(c) * (P - (double)p.p0(c)));
}

// Length of the edge src -> tgt with image offset (ox, oy), overridden
// positions allowed.
template <typename PosT>
__device__ __forceinline__ double ov_len(const DevTissue &t, const PosT *X,
                                         const PosOverride<PosT> &ov, int s, int g, int ox,
                                         int oy) {
    double xs, ys, xg, yg;
    ov.get(X, s, xs, ys);
    ov.get(X, g, xg, yg);
    const double dx = xg + ox * t.Lx - xs, dy = yg + oy * t.Ly - ys;
    return sqrt(dx * dx + dy * dy);
}

// Neighbour exchange of the edge of half-edge h (i -> j in C1, its twin
// j -> i in C2; C3 is the third cell at i, C4 the third cell at j).
// Afterwards h bounds C4 and its twin bounds C3, the edge to c (next of h
// in C1) moves from j to i and the edge to b (next of the twin in C2) from
// i to j; the moved half-edges change image offset by the offset of h so
// that every edge vector is kept.
__device__ __forceinline__ void t1_patch(const DevTissue &t, int h) {
    int32_t *he = t.he;
    auto R = [&](int x) { return he + 8 * (int64_t)x; };
    const int tw = R(h)[HT];
    const int i = R(h)[HS], j = R(h)[HG];
    const int p1 = R(h)[HP], n1 = R(h)[HN];
    const int p2 = R(tw)[HP], n2 = R(tw)[HN];
    const int tp1 = R(p1)[HT], tn1 = R(n1)[HT];
    const int tp2 = R(p2)[HT], tn2 = R(n2)[HT];
    const int C3 = R(tp1)[HF], C4 = R(tn1)[HF];
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

// In-place edit of cell c's corner row after an exchange.
//   edit 1: drop vertex va; the corner before it now leaves by half-edge nh.
//   edit 2: insert vertex vb, leaving by half-edge nh, right before va, at
//           the image of va plus (sx, sy).
// Images are re-based so that the first corner has image 0.  A row without
// a spare slot is first moved to the free pool at the end of the corner
// arrays (*relocated is set; rows are compacted again after the pass).
// Returns false on an inconsistency or when the pool is exhausted.
__device__ __forceinline__ bool row_edit(const DevTissue &t, int c, int edit, int va, int vb,
                                         int nh, int sx, int sy, int *relocated) {
    int rb = t.row_ptr[c];
    const int n = t.nsides[c];
    if (edit == 2 && n + 1 > t.row_cap[c]) {
        const int nb = *t.pool_top;
        const int cap = n + 1 + kRowExtra;
        if (nb + cap > t.corner_cap) return false;
        for (int q = 0; q < n; ++q) {
            t.corner[nb + q] = t.corner[rb + q];
            t.corner_he[nb + q] = t.corner_he[rb + q];
        }
        *t.pool_top = nb + cap;
        t.row_ptr[c] = nb;
        t.row_cap[c] = cap;
        rb = nb;
        *relocated = 1;
    }
    int32_t *cw = t.corner + rb;
    int32_t *ch = t.corner_he + rb;
    int k = 0;
    while (k < n && id_of(cw[k]) != va) ++k;
    if (k == n) return false;
    if (edit == 1) {
        const int kp = (k + n - 1) % n;
        ch[kp] = nh;
        for (int q = k; q + 1 < n; ++q) {
            cw[q] = cw[q + 1];
            ch[q] = ch[q + 1];
        }
        t.nsides[c] = n - 1;
    } else {
        for (int q = n; q > k; --q) {
            cw[q] = cw[q - 1];
            ch[q] = ch[q - 1];
        }
        cw[k] = pack_id(vb, ox_of(cw[k + 1]) + sx, oy_of(cw[k + 1]) + sy);
        ch[k] = nh;
        t.nsides[c] = n + 1;
    }
    const int m = t.nsides[c];
    const int bx = ox_of(cw[0]), by = oy_of(cw[0]);
    if (bx || by)
        for (int q = 0; q < m; ++q) cw[q] = pack_id(id_of(cw[q]), ox_of(cw[q]) - bx, oy_of(cw[q]) - by);
    for (int q = 0; q < m; ++q)
        if (ox_of(cw[q]) < -1 || ox_of(cw[q]) > 1 || oy_of(cw[q]) < -1 || oy_of(cw[q]) > 1)
            return false;
    return true;
}

// Result of one sequential T1 pass.
struct T1Counts {
    int64_t swaps, stretches;
    int changed;    // topology changed
    int relocated;  // a row moved to the pool: compact all rows after the pass
    int overflow;   // 1: too many pending re-checks; 2: row edit failed
};

// Sequential T1 pass over the ascending candidate list `list[0..n)` (edge
// ids, sorted, may hold duplicates and INT_MAX padding), run by the 64
// lanes of ONE wave with wave-uniform control flow.  Each candidate is
// re-checked with the current positions; edges next to a processed edge
// that become short are visited in turn as well, so the result equals
// visiting every edge in ascending id order.  Both candidates are evaluated
// on the four cells around the edge (lanes 0-7: stretch on cells C1..C4,
// exchange on C1..C4, read from their corner rows with the exchange applied
// as row edits) and the five edges at its ends; everything else is common
// to both.  Lane 0 writes the result; the kept candidate's cell geometry
// gives the new cell coefficients.  Not inlined: it must not raise the
// register pressure of the loops around it.
template <typename PosT, typename M>
__device__ __noinline__ T1Counts t1_sequential(const DevTissue &t, PosT *X, const DevParams<PosT> &p,
                                               M *cap, const int32_t *list, int n, int32_t *extra,
                                               double l_min, double l_new) {
    const int lane = threadIdx.x & 63;
    T1Counts out{0, 0, 0, 0, 0};
    int pos = 0, n_extra = 0;
    int last = -1;
    const double hl = 0.5 * l_new;
    for (;;) {
        // next edge: min of list[pos] and the pending set.  Every lane keeps
        // the same bookkeeping (the LDS set is written by all lanes with the
        // same values), so no lane depends on another's writes.
        int e = 0x7fffffff;
        while (pos < n && list[pos] <= last) ++pos;
        if (pos < n) e = list[pos];
        for (int a = 0; a < n_extra; ++a)
            if (extra[a] < e) e = extra[a];
        if (e == 0x7fffffff) break;
        if (pos < n && list[pos] == e) ++pos;
        {   // drop e (and anything below it) from the pending set
            int m = 0;
            for (int a = 0; a < n_extra; ++a) {
                const int v = extra[a];
                if (v > e) extra[m++] = v;
            }
            n_extra = m;
        }
        last = e;

        const int h = t.edge_he[e];
        const HeRec rh = he_rec(t, h);
        const int i = rh.src, j = rh.tgt;
        const double xi = (double)X[2 * (int64_t)i], yi = (double)X[2 * (int64_t)i + 1];
        const double xj = (double)X[2 * (int64_t)j], yj = (double)X[2 * (int64_t)j + 1];
        const double dx = pdiff<double>(xj, xi, rh.ox, t.Lx), dy = pdiff<double>(yj, yi, rh.oy, t.Ly);
        const double l = sqrt(dx * dx + dy * dy);
        if (!(l < l_min)) continue;
        double ux = 1.0, uy = 0.0;
        if (l > 0.0) { ux = dx / l; uy = dy / l; }
        const double mx = xi + 0.5 * dx, my = yi + 0.5 * dy;
        const double sxL = rh.ox * t.Lx, syL = rh.oy * t.Ly;
        const PosOverride<PosT> S{i, j, mx - hl * ux, my - hl * uy, mx + hl * ux - sxL, my + hl * uy - syL};
        const double nx = -uy, ny = ux;
        const PosOverride<PosT> T{i, j, mx + hl * nx, my + hl * ny, mx - hl * nx - sxL, my - hl * ny - syL};

        const int tw = rh.twin, p1 = rh.prev, n1 = rh.next;
        const HeRec rt = he_rec(t, tw), rp1 = he_rec(t, p1), rn1 = he_rec(t, n1);
        const int p2 = rt.prev, n2 = rt.next;
        const HeRec rp2 = he_rec(t, p2), rn2 = he_rec(t, n2);
        const int tp1 = rp1.twin, tn1 = rn1.twin, tn2 = rn2.twin;
        const int C1 = rh.face, C2 = rt.face;
        const int C3 = he_rec(t, tp1).face, C4 = he_rec(t, tn1).face;
        const bool distinct = C1 != C2 && C1 != C3 && C1 != C4 && C2 != C3 && C2 != C4 && C3 != C4;
        const bool admissible = distinct && t.nsides[C1] > 3 && t.nsides[C2] > 3;

        // lanes 0..3: stretch geometry of C1..C4; lanes 4..7: exchange geometry
        const int q = lane & 3;
        const int cq = q == 0 ? C1 : q == 1 ? C2 : q == 2 ? C3 : C4;
        double A = 0.0, P = 0.0, Eq = 0.0;
        if (lane < 4 || (lane < 8 && admissible)) {
            // stretch: no row edit.  Exchange: C1 drops j, C2 drops i, C3
            // gains j before i, C4 gains i before j.  One call site for both.
            const bool ex = lane >= 4;
            const int ed = !ex ? 0 : (q < 2 ? 1 : 2);
            const int va = !ex ? -1 : ((q == 0 || q == 3) ? j : i);
            const int vb = !ex ? -1 : (q == 2 ? j : (q == 3 ? i : -1));
            const int sx = !ex ? 0 : (q == 2 ? rh.ox : (q == 3 ? -rh.ox : 0));
            const int sy = !ex ? 0 : (q == 2 ? rh.oy : (q == 3 ? -rh.oy : 0));
            row_geom<PosT>(t, X, cq, ex ? T : S, ed, va, vb, sx, sy, A, P);
            Eq = cell_energy<PosT>(p, cq, A, P);
        }
        bool take_T = false;
        if (admissible) {
            const double ES = ((__shfl(Eq, 0, 64) + __shfl(Eq, 1, 64)) + __shfl(Eq, 2, 64)) +
                              __shfl(Eq, 3, 64);
            const double ET0 = ((__shfl(Eq, 4, 64) + __shfl(Eq, 5, 64)) + __shfl(Eq, 6, 64)) +
                               __shfl(Eq, 7, 64);
            // edges i->c and j->b replace j->c and i->b in the exchange
            const double lh = (double)p.lm(e);
            const double lp1 = (double)p.lm(t.he_edge[p1]), ln1 = (double)p.lm(t.he_edge[n1]);
            const double lp2 = (double)p.lm(t.he_edge[p2]), ln2 = (double)p.lm(t.he_edge[n2]);
            const double ESe = lh * ov_len<PosT>(t, X, S, i, j, rh.ox, rh.oy) +
                               lp1 * ov_len<PosT>(t, X, S, rp1.src, i, rp1.ox, rp1.oy) +
                               ln1 * ov_len<PosT>(t, X, S, j, rn1.tgt, rn1.ox, rn1.oy) +
                               lp2 * ov_len<PosT>(t, X, S, rp2.src, j, rp2.ox, rp2.oy) +
                               ln2 * ov_len<PosT>(t, X, S, i, rn2.tgt, rn2.ox, rn2.oy);
            const double ETe = lh * ov_len<PosT>(t, X, T, i, j, rh.ox, rh.oy) +
                               lp1 * ov_len<PosT>(t, X, T, rp1.src, i, rp1.ox, rp1.oy) +
                               ln1 * ov_len<PosT>(t, X, T, i, rn1.tgt, rn1.ox + rh.ox, rn1.oy + rh.oy) +
                               lp2 * ov_len<PosT>(t, X, T, rp2.src, j, rp2.ox, rp2.oy) +
                               ln2 * ov_len<PosT>(t, X, T, j, rn2.tgt, rn2.ox - rh.ox, rn2.oy - rh.oy);
            take_T = ET0 + ETe < ES + ESe;
        }
        const PosOverride<PosT> W = take_T ? T : S;
        // the kept candidate's lanes write the new coefficients of C1..C4
        if ((take_T && lane >= 4 && lane < 8) || (!take_T && lane < 4)) {
            cap[2 * (int64_t)cq] = (M)(2.0 * (double)p.ka(cq) * (A - (double)p.a0(cq)));
            cap[2 * (int64_t)cq + 1] = (M)(2.0 * (double)p.kp(cq) * (P - (double)p.p0(cq)));
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
            X[2 * (int64_t)i] = (PosT)W.xi;
            X[2 * (int64_t)i + 1] = (PosT)W.yi;
            X[2 * (int64_t)j] = (PosT)W.xj;
            X[2 * (int64_t)j + 1] = (PosT)W.yj;
            if (take_T) {
                t1_patch(t, h);
                if (t.cell_he[C1] == h) t.cell_he[C1] = n1;
                if (t.cell_he[C2] == tw) t.cell_he[C2] = n2;
                // rows: C1 drops j (i now leaves by n1), C2 drops i (j leaves
                // by n2), C3 gains j (leaving by tw) before i, C4 gains i (by
                // h) before j
                bool ok = row_edit(t, C1, 1, j, -1, n1, 0, 0, &out.relocated);
                ok = row_edit(t, C2, 1, i, -1, n2, 0, 0, &out.relocated) && ok;
                ok = row_edit(t, C3, 2, i, j, tw, rh.ox, rh.oy, &out.relocated) && ok;
                ok = row_edit(t, C4, 2, j, i, h, -rh.ox, -rh.oy, &out.relocated) && ok;
                if (!ok) out.overflow = 2;
                // stars of i and j are rebuilt; c and b changed neighbour
                star_refresh(t, i, h);
                star_refresh(t, j, tw);
                star_refresh(t, rn1.tgt, tn1);   // c
                star_refresh(t, rn2.tgt, tn2);   // b
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        out.overflow = __shfl(out.overflow, 0, 64);
        out.relocated = __shfl(out.relocated, 0, 64);
        if (out.overflow == 2) return out;
        if (take_T) {
            ++out.swaps;
            out.changed = 1;
        } else {
            ++out.stretches;
        }
        // the four other edges at i and j may have become short: a->i, and
        // i->c, d->j, j->b after an exchange (j->c, i->b after a stretch)
        const int nbr[4] = {p1, n1, p2, n2};
        const int ns[4] = {rp1.src, take_T ? i : j, rp2.src, take_T ? j : i};
        const int ng[4] = {i, rn1.tgt, j, rn2.tgt};
        const int nox[4] = {rp1.ox, rn1.ox + (take_T ? rh.ox : 0), rp2.ox, rn2.ox - (take_T ? rh.ox : 0)};
        const int noy[4] = {rp1.oy, rn1.oy + (take_T ? rh.oy : 0), rp2.oy, rn2.oy - (take_T ? rh.oy : 0)};
        for (int a = 0; a < 4; ++a) {
            const int e2 = t.he_edge[nbr[a]];
            if (e2 <= e) continue;
            if (ov_len<PosT>(t, X, W, ns[a], ng[a], nox[a], noy[a]) < l_min) {
                bool present = false;
                for (int b = 0; b < n_extra; ++b) present |= extra[b] == e2;
                if (!present) {
                    if (n_extra >= kT1Extra) out.overflow = 1;
                    else extra[n_extra++] = e2;
                }
            }
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
        const int v = c < nc ? t.nsides[c] + kRowSlack : 0;
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
    if (threadIdx.x == 0) {
        t.row_ptr[nc] = carry;
        *t.pool_top = t.pool_start;
        if (carry > t.pool_start) bad = 1;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const int h0 = t.cell_he[c];
        int base = t.row_ptr[c];
        t.row_cap[c] = t.nsides[c] + kRowSlack;
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
// Stored as (G, B) = (2 K_A dA, 2 K_P dP).  `corner_at(k)` returns the
// packed corner k of the cell's row, which has n corners.
template <typename PosT, typename M, typename CornerAt>
__device__ __forceinline__ void hvp_cell_row(const DevTissue &t, const PosT *__restrict__ X,
                                             const double *__restrict__ v, int n,
                                             CornerAt corner_at, PosT ka, PosT kp,
                                             M *__restrict__ aux, int c) {
    using C = PosT;
    const PosT Lx = (PosT)t.Lx, Ly = (PosT)t.Ly;
    const int32_t w0 = corner_at(0);
    const auto p0 = ld2(X, id_of(w0));
    auto rel = [&](int k, C &rx, C &ry, C &vx, C &vy) {
        const int32_t w = corner_at(k);
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
        const C l2 = dx * dx + dy * dy;
        if (l2 > (C)0) dP += over_len_hvp(dx * (vnx - vcx) + dy * (vny - vcy), l2);
        rpx = rcx;
        rpy = rcy;
        rcx = rnx;
        rcy = rny;
        vcx = vnx;
        vcy = vny;
    }
    st2(aux, c, (M)((C)2 * (C)ka * dA), (M)((C)2 * (C)kp * dP));
}

template <typename PosT, typename M>
__device__ __forceinline__ void hvp_cell_one(const DevTissue &t, const PosT *__restrict__ X,
                                             const DevParams<PosT> &p,
                                             const double *__restrict__ v, M *__restrict__ aux,
                                             int c) {
    const int rb = t.row_ptr[c], n = t.nsides[c];
    hvp_cell_row<PosT, M>(
        t, X, v, n, [&](int k) { return t.corner[rb + k]; }, p.ka(c), p.kp(c), aux, c);
}

// (H v)_i = sum_k [ T_k w_k - u_k (B_k + B_{k-1}) + 1/2 R(d_k)(G_k - G_{k-1})
//                   + 1/2 R(v_{j_k} - v_i)(cA_k - cA_{k-1}) ]
// with w_k = (I - u_k u_k^T)(v_i - v_{j_k}) / l_k, T_k the edge tension
// (lambda_k + cP_k + cP_{k-1}), G = 2K_A dA and B = 2K_P dP of the sector
// cells.  From a star whose entries and gathers are in `L`: returns
// (Hv)_i in (hx, hy) and v_i . (Hv)_i.
template <typename PosT, typename M>
__device__ __forceinline__ double hvp_vertex_star(const DevTissue &t,
                                                  const StarLoad<PosT, M> &L,
                                                  const M *__restrict__ aux,
                                                  const double *__restrict__ v, int i,
                                                  double &hx_out, double &hy_out) {
    Star<PosT, M> s;
    PosT xi, yi;
    star_math<PosT, M, false, true>(t, L, s, xi, yi);
    const auto vi = ld2(v, i);
    M G[3], B[3], vx[3], vy[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const auto g = ld2(aux, L.c[k]);
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
    hx_out = (double)hx;
    hy_out = (double)hy;
    return vi.x * (double)hx + vi.y * (double)hy;
}

// Writes (Hv)_i and returns v_i . (Hv)_i.
template <typename PosT, typename M>
__device__ __forceinline__ double hvp_vertex_one(const DevTissue &t, const PosT *__restrict__ X,
                                                 const DevParams<PosT> &p,
                                                 const M *__restrict__ cap,
                                                 const M *__restrict__ aux,
                                                 const double *__restrict__ v,
                                                 double *__restrict__ Hv, int i) {
    StarLoad<PosT, M> L;
    star_ids<PosT, M>(t, X, i, L);
    star_gather<PosT, M>(X, p, cap, L);
    double hx, hy;
    const double d = hvp_vertex_star<PosT, M>(t, L, aux, v, i, hx, hy);
    st2(Hv, i, hx, hy);
    return d;
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
    const int rb = t.row_ptr[c], n = t.nsides[c];
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
