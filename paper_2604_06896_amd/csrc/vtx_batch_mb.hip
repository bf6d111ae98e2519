// Batched adjoint with each tissue split over several workgroups (Methods,
// "Implicit differentiation (ID)": H mu = P dC/dX solved by conjugate
// gradients, then the contraction with the mixed derivatives).
//
// A group of K workgroups solves one tissue.  Part p owns the vertices
// [p n/K, (p+1) n/K) (contiguous in the Morton order, so a compact patch)
// and recomputes the cells around them; the vertices of those cells that
// other parts own form its halo.  The Hessian-vector product at X* uses only
// quantities that stay fixed during the solve, so they are computed once
// per tissue: per cell corner the area gradient 1/2 R(r_{k+1} - r_{k-1}) and
// the unit vector of the edge leaving it (LDS), per owned vertex and star
// slot the edge vector, unit vector, tension / length and the pressure
// difference across the edge (registers).  A CG step is then
//   cell half (LDS) -> vertex half and q.Hq -> barrier (q.Hq of all parts)
//   -> x, r update and r.r -> barrier (r.r, and r of the halo)
//   -> q = r + beta q for owned and halo vertices,
// with two cross-workgroup barriers.  The sums over parts are taken in part
// order, so every part computes the same scalars and the result does not
// depend on timing.  The launch is cooperative (all workgroups resident),
// and every wait is bounded: a part that does not arrive within the limit
// turns into an error, never a hang.
#include "vtx_batch.h"

namespace vtx {

constexpr int kMbThreads = 512;
constexpr int kMbKV = 2;          // owned vertices per thread, at most
constexpr int kMbMaxParts = 8;
constexpr int kMbNoFit = 100;     // status of a tissue this kernel cannot hold

// Cross-workgroup state of one group.
struct MbGroup {
    unsigned int count;                      // arrivals; K more per barrier
    int err;                                 // a part gave up waiting
    int pad[2];
    double part[2][kMbMaxParts][4];          // per-part values, by barrier parity
};

// Barrier of the K workgroups of a group, carrying up to four doubles per
// part; returns false if the wait timed out (or another part's did).
// Stores made by any thread of the block before the call are visible to
// every part after it.
struct MbSync {
    MbGroup *g;
    int K, part;
    unsigned int round;
    uint64_t limit;   // wall-clock ticks
    // Values whose bit is set in `maxmask` are combined by max (NaN wins),
    // the others summed, in part order.
    __device__ bool arrive(const double *vals, int nval, double *sh_out, int *sh_flag,
                           unsigned maxmask = 0u) {
        ++round;
        const int par = round & 1;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 0; i < nval; ++i) g->part[par][part][i] = vals[i];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(&g->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned int target = (unsigned int)K * round;
            const uint64_t t0 = wall_clock64();
            int ok = 1;
            while (__hip_atomic_load(&g->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                   target) {
                if (__hip_atomic_load(&g->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                    wall_clock64() - t0 > limit) {
                    ok = 0;
                    __hip_atomic_store(&g->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            for (int i = 0; i < nval; ++i) {
                const bool mx = (maxmask >> i) & 1u;
                double s = 0.0;
                for (int q = 0; q < K; ++q)
                    s = mx ? nanmax(s, g->part[par][q][i]) : s + g->part[par][q][i];
                sh_out[i] = s;
            }
            *sh_flag = ok;
        }
        __syncthreads();
        return *sh_flag != 0;
    }
};

struct MbArgs {
    const GradItem *items;
    const int32_t *order;
    int n;            // tissues
    int K;            // parts per tissue
    int n_groups;
    GradOpts o;
    vtx_grad_result *res;
    MbGroup *groups;
    int lds_bytes;
    uint64_t wait_ticks;
};

// Bump allocator over the dynamic LDS (16-byte aligned pieces).
struct LdsBump {
    unsigned char *base;
    int64_t used, cap;
    __device__ void *take(int64_t bytes) {
        void *p = base + used;
        used += (bytes + 15) & ~(int64_t)15;
        return p;
    }
    __device__ bool ok() const { return used <= cap; }
};

// The part of a tissue one workgroup works on, built in LDS: the local
// cells (the sector cells of the owned vertices [v_lo, v_hi), numbered in
// ascending global id), their corner offsets, and the local vertex ids
// (owned vertices first, then the halo -- the other corners of the local
// cells -- in ascending global id).  Called by every thread of the block.
struct MbLocal {
    int32_t *vmap;    // [n_vert] global vertex -> local id (-1: not local)
    int32_t *cmap;    // [n_cell] global cell -> local id (-1: not local)
    int32_t *lcg;     // [n_lc] local cell -> global
    int32_t *cstart;  // [n_lc + 1] first corner of each local cell
    int32_t *halo;    // [n_halo] global id of halo vertex n_own + h
    int n_own, n_lc, n_corner, n_halo, n_lv;
    bool fits;        // the owned vertices and these arrays fit
};

__device__ MbLocal mb_partition(const DevTissue &t, int v_lo, int v_hi, LdsBump &lb,
                                int *s_scan, int *s_fail) {
    const int tid = threadIdx.x, bd = blockDim.x, nv = t.n_vert, nc = t.n_cell;
    MbLocal L{};
    L.n_own = v_hi - v_lo;
    if (tid == 0) *s_fail = L.n_own > kMbKV * bd;
    L.vmap = (int32_t *)lb.take(4 * (int64_t)nv);
    L.cmap = (int32_t *)lb.take(4 * (int64_t)nc);
    __syncthreads();
    if (lb.ok()) {
        for (int v = tid; v < nv; v += bd) L.vmap[v] = -1;
        for (int c = tid; c < nc; c += bd) L.cmap[c] = -1;
    }
    __syncthreads();
    const bool go = lb.ok() && !*s_fail;
    if (go)
        for (int v = v_lo + tid; v < v_hi; v += bd)
            for (int k = 0; k < 3; ++k) L.cmap[t.star[star_cell_at(nv, k, v)]] = 0;
    __syncthreads();
    if (go) {
        for (int base = 0; base < nc; base += bd) {
            const int c = base + tid;
            const int f = (c < nc && L.cmap[c] == 0) ? 1 : 0;
            int tot;
            const int e = block_exclusive_scan(f, s_scan, tot);
            if (f) L.cmap[c] = L.n_lc + e + 1;   // +1 keeps 0 free as the mark
            L.n_lc += tot;
        }
        L.lcg = (int32_t *)lb.take(4 * (int64_t)L.n_lc);
        if (lb.ok())
            for (int c = tid; c < nc; c += bd)
                if (L.cmap[c] > 0) {
                    L.cmap[c] -= 1;
                    L.lcg[L.cmap[c]] = c;
                }
    }
    __syncthreads();
    L.cstart = (int32_t *)lb.take(4 * ((int64_t)L.n_lc + 1));
    if (go && lb.ok()) {
        for (int l = tid; l < L.n_lc; l += bd) {
            const int c = L.lcg[l];
            const int rb = t.row_ptr[c], n = t.nsides[c];
            L.cstart[l] = n;
            for (int k = 0; k < n; ++k) {
                const int v = id_of(t.corner[rb + k]);
                if (v < v_lo || v >= v_hi) L.vmap[v] = -2;   // halo
            }
        }
    }
    __syncthreads();
    if (go && lb.ok()) {
        for (int base = 0; base < L.n_lc; base += bd) {
            const int l = base + tid;
            const int cnt = l < L.n_lc ? L.cstart[l] : 0;
            int tot;
            const int e = block_exclusive_scan(cnt, s_scan, tot);
            __syncthreads();
            if (l < L.n_lc) L.cstart[l] = L.n_corner + e;
            L.n_corner += tot;
            __syncthreads();
        }
        if (tid == 0) L.cstart[L.n_lc] = L.n_corner;
        for (int v = v_lo + tid; v < v_hi; v += bd) L.vmap[v] = v - v_lo;
        for (int base = 0; base < nv; base += bd) {
            const int v = base + tid;
            const int f = (v < nv && L.vmap[v] == -2) ? 1 : 0;
            int tot;
            const int e = block_exclusive_scan(f, s_scan, tot);
            if (f) L.vmap[v] = L.n_own + L.n_halo + e;
            L.n_halo += tot;
        }
    }
    L.n_lv = L.n_own + L.n_halo;
    L.halo = (int32_t *)lb.take(4 * (int64_t)L.n_halo);
    __syncthreads();
    L.fits = go && lb.ok();
    if (L.fits)
        for (int v = tid; v < nv; v += bd) {
            const int l = L.vmap[v];
            if (l >= L.n_own) L.halo[l - L.n_own] = v;
        }
    __syncthreads();
    return L;
}

__global__ __launch_bounds__(kMbThreads) void k_batch_cg_mb(MbArgs a) {
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    __shared__ double sh[16];
    __shared__ double s_out[4];
    __shared__ int s_flag;
    __shared__ int s_scan[16];
    __shared__ int s_fail;
    const int tid = threadIdx.x, bd = blockDim.x;
    const int grp = blockIdx.x % a.n_groups, part = blockIdx.x / a.n_groups;
    MbSync sync{a.groups + grp, a.K, part, 0u, a.wait_ticks};
    for (int slot = grp; slot < a.n; slot += a.n_groups) {
        const int idx = a.order[slot];
        const GradItem &G = a.items[idx];
        const DevTissue t = G.t;
        const DevParams<double> p = to_dev<double>(G.p);
        const double *X = (const double *)G.X;
        const int nv = t.n_vert, nc = t.n_cell;
        const int v_lo = (int)((int64_t)nv * part / a.K);
        const int v_hi = (int)((int64_t)nv * (part + 1) / a.K);
        const int n_own = v_hi - v_lo;
        LdsBump lb{lds_dyn, 0, a.lds_bytes};
        MbLocal L = mb_partition(t, v_lo, v_hi, lb, s_scan, &s_fail);
        const int n_lc = L.n_lc, n_corner = L.n_corner, n_halo = L.n_halo, n_lv = L.n_lv;
        int32_t *vmap = L.vmap, *cmap = L.cmap, *lcg = L.lcg, *cstart = L.cstart, *halo = L.halo;
        int32_t *cvert = (int32_t *)lb.take(4 * (int64_t)n_corner);
        double4 *cgeo = (double4 *)lb.take(32 * (int64_t)n_corner);
        double2 *qL = (double2 *)lb.take(16 * (int64_t)n_lv);
        double2 *auxL = (double2 *)lb.take(16 * (int64_t)n_lc);
        double2 *kkL = (double2 *)lb.take(16 * (int64_t)n_lc);
        double2 *capL = (double2 *)lb.take(16 * (int64_t)n_lc);
        __syncthreads();
        const bool fits = lb.ok() && L.fits;
        if (fits) {
            // per cell: corners (local ids), the constant geometry of the
            // Hessian-vector product, (2 K_A, 2 K_P) and (cA, cP) at X*
            for (int l = tid; l < n_lc; l += bd) {
                const int c = lcg[l];
                const int rb = t.row_ptr[c], n = t.nsides[c], off = cstart[l];
                const int32_t w0 = t.corner[rb];
                const double2 p0 = ld2(X, id_of(w0));
                auto rel = [&](int k, double &rx, double &ry) {
                    const int32_t w = t.corner[rb + k];
                    const double2 q = ld2(X, id_of(w));
                    rx = k == 0 ? 0.0 : pdiff<double>(q.x, p0.x, ox_of(w), t.Lx);
                    ry = k == 0 ? 0.0 : pdiff<double>(q.y, p0.y, oy_of(w), t.Ly);
                };
                double rpx, rpy, rcx, rcy, a2 = 0.0, per = 0.0;
                rel(n - 1, rpx, rpy);
                rel(0, rcx, rcy);
                for (int k = 0; k < n; ++k) {
                    const int kn = k + 1 == n ? 0 : k + 1;
                    double rnx, rny;
                    rel(kn, rnx, rny);
                    const double dx = rnx - rcx, dy = rny - rcy;
                    const double len = sqrt(dx * dx + dy * dy);
                    const double ux = len > 0.0 ? dx / len : 0.0, uy = len > 0.0 ? dy / len : 0.0;
                    cgeo[off + k] = double4{0.5 * (rny - rpy), -0.5 * (rnx - rpx), ux, uy};
                    cvert[off + k] = vmap[id_of(t.corner[rb + k])];
                    a2 += rcx * rny - rcy * rnx;
                    per += len;
                    rpx = rcx;
                    rpy = rcy;
                    rcx = rnx;
                    rcy = rny;
                }
                const double ka = p.ka(c), kp = p.kp(c);
                kkL[l] = double2{2.0 * ka, 2.0 * kp};
                capL[l] = double2{2.0 * ka * (0.5 * a2 - p.a0(c)), 2.0 * kp * (per - p.p0(c))};
            }
        }
        __syncthreads();
        // per owned vertex and star slot: local neighbour and cell ids and
        // the constant edge geometry
        int nbl[kMbKV][3], cll[kMbKV][3];
        double gux[kMbKV][3], guy[kMbKV][3], gdx[kMbKV][3], gdy[kMbKV][3], gti[kMbKV][3],
            gdc[kMbKV][3];
        double xs[kMbKV][2], rs[kMbKV][2], qs[kMbKV][2];
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int j = 0; j < kMbKV; ++j) {
            const int v = v_lo + tid + j * bd;
            xs[j][0] = xs[j][1] = rs[j][0] = rs[j][1] = qs[j][0] = qs[j][1] = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                nbl[j][k] = cll[j][k] = 0;
                gux[j][k] = guy[j][k] = gdx[j][k] = gdy[j][k] = gti[j][k] = gdc[j][k] = 0.0;
            }
            if (fits && v < v_hi) {
                const double2 pi = ld2(X, v);
                double cA[3], cP[3], lam[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int32_t w = t.star[star_nb_at(nv, k, v)];
                    const int c = t.star[star_cell_at(nv, k, v)];
                    const int e = t.star[star_edge_at(nv, k, v)];
                    nbl[j][k] = vmap[id_of(w)];
                    cll[j][k] = cmap[c];
                    const double2 q = ld2(X, id_of(w));
                    const double dx = pdiff<double>(q.x, pi.x, ox_of(w), t.Lx);
                    const double dy = pdiff<double>(q.y, pi.y, oy_of(w), t.Ly);
                    const double len = sqrt(dx * dx + dy * dy);
                    const double inv = len > 0.0 ? 1.0 / len : 0.0;
                    gdx[j][k] = dx;
                    gdy[j][k] = dy;
                    gux[j][k] = dx * inv;
                    guy[j][k] = dy * inv;
                    gti[j][k] = inv;
                    const double2 cc = capL[cll[j][k]];
                    cA[k] = cc.x;
                    cP[k] = cc.y;
                    lam[k] = p.lm(e);
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int km = (k + 2) % 3;
                    gti[j][k] *= lam[k] + cP[k] + cP[km];
                    gdc[j][k] = 0.5 * (cA[k] - cA[km]);
                }
                sx += G.b[2 * (int64_t)v];
                sy += G.b[2 * (int64_t)v + 1];
            }
        }
        // first barrier: whether every part holds its share, and the mean of b
        double vals[4] = {0.0, 0.0, 0.0, 0.0};
        vals[0] = block_allsum(sx, sh);
        vals[1] = block_allsum(sy, sh);
        vals[2] = fits ? 0.0 : 1.0;
        if (!sync.arrive(vals, 3, s_out, &s_flag)) break;
        if (s_out[2] != 0.0) {   // some part cannot hold this tissue: leave it to the host
            if (part == 0 && tid == 0) {
                vtx_grad_result gr{};
                gr.status = kMbNoFit;
                a.res[idx] = gr;
            }
            continue;
        }
        const double mbx = s_out[0] / (double)nv, mby = s_out[1] / (double)nv;
        // r = P b, q = r, x = 0 (owned in registers, q of owned and halo in LDS)
        double rr = 0.0;
#pragma unroll
        for (int j = 0; j < kMbKV; ++j) {
            const int v = v_lo + tid + j * bd;
            if (v < v_hi) {
                rs[j][0] = G.b[2 * (int64_t)v] - mbx;
                rs[j][1] = G.b[2 * (int64_t)v + 1] - mby;
                qs[j][0] = rs[j][0];
                qs[j][1] = rs[j][1];
                qL[v - v_lo] = double2{rs[j][0], rs[j][1]};
                rr += rs[j][0] * rs[j][0] + rs[j][1] * rs[j][1];
            }
        }
        for (int h = tid; h < n_halo; h += bd) {
            const int v = halo[h];
            qL[n_own + h] = double2{G.b[2 * (int64_t)v] - mbx, G.b[2 * (int64_t)v + 1] - mby};
        }
        vals[0] = block_allsum(rr, sh);
        if (!sync.arrive(vals, 1, s_out, &s_flag)) break;
        rr = s_out[0];
        const double rr0 = rr;
        int status = rr0 > 0.0 ? VTX_CG_MAXITER : VTX_CONVERGED;
        int64_t it = 0;
        double *rx = G.cg + 2 * (int64_t)nv;   // r of every vertex, for the halo exchange
        bool alive = true;
        while (status == VTX_CG_MAXITER && it < a.o.max_iter) {
            if (sqrt(rr) <= a.o.tol * sqrt(rr0)) {
                status = VTX_CONVERGED;
                break;
            }
            // cell half: (G, B) = (2 K_A dA[q], 2 K_P dP[q]) of the local cells
            for (int l = tid; l < n_lc; l += bd) {
                const int o0 = cstart[l], o1 = cstart[l + 1];
                double dA = 0.0, dP = 0.0;
                double2 qc = qL[cvert[o0]];
                for (int o = o0; o < o1; ++o) {
                    const double2 qn = qL[cvert[o + 1 < o1 ? o + 1 : o0]];
                    const double4 gg = cgeo[o];
                    dA += gg.x * qc.x + gg.y * qc.y;
                    dP += gg.z * (qn.x - qc.x) + gg.w * (qn.y - qc.y);
                    qc = qn;
                }
                const double2 kk = kkL[l];
                auxL[l] = double2{kk.x * dA, kk.y * dP};
            }
            __syncthreads();
            // vertex half and q . Hq
            double d = 0.0, hq[kMbKV][2];
#pragma unroll
            for (int j = 0; j < kMbKV; ++j) {
                hq[j][0] = hq[j][1] = 0.0;
                const int v = v_lo + tid + j * bd;
                if (v < v_hi) {
                    double hx = 0.0, hy = 0.0;
                    double Gs[3], Bs[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const double2 gb = auxL[cll[j][k]];
                        Gs[k] = gb.x;
                        Bs[k] = gb.y;
                    }
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const int km = (k + 2) % 3;
                        const double2 qj = qL[nbl[j][k]];
                        const double vx = qj.x - qs[j][0], vy = qj.y - qs[j][1];
                        const double du = -(vx * gux[j][k] + vy * guy[j][k]);
                        const double wx = -vx - du * gux[j][k], wy = -vy - du * guy[j][k];
                        const double Bsum = Bs[k] + Bs[km];
                        const double dG = 0.5 * (Gs[k] - Gs[km]);
                        hx += gti[j][k] * wx - gux[j][k] * Bsum + dG * gdy[j][k] + gdc[j][k] * vy;
                        hy += gti[j][k] * wy - guy[j][k] * Bsum - dG * gdx[j][k] - gdc[j][k] * vx;
                    }
                    hq[j][0] = hx;
                    hq[j][1] = hy;
                    d += qs[j][0] * hx + qs[j][1] * hy;
                }
            }
            vals[0] = block_allsum(d, sh);
            if (!sync.arrive(vals, 1, s_out, &s_flag)) {
                alive = false;
                break;
            }
            const double pAp = s_out[0];
            if (!(pAp > 0.0)) {
                status = VTX_CG_NEG_CURVATURE;
                break;
            }
            const double al = rr / pAp;
            double rn = 0.0;
#pragma unroll
            for (int j = 0; j < kMbKV; ++j) {
                const int v = v_lo + tid + j * bd;
                if (v < v_hi) {
                    xs[j][0] += al * qs[j][0];
                    xs[j][1] += al * qs[j][1];
                    rs[j][0] -= al * hq[j][0];
                    rs[j][1] -= al * hq[j][1];
                    rn += rs[j][0] * rs[j][0] + rs[j][1] * rs[j][1];
                    st2(rx, v, rs[j][0], rs[j][1]);
                }
            }
            vals[0] = block_allsum(rn, sh);
            if (!sync.arrive(vals, 1, s_out, &s_flag)) {
                alive = false;
                break;
            }
            rn = s_out[0];
            const double be = rn / rr;
            rr = rn;
            ++it;
#pragma unroll
            for (int j = 0; j < kMbKV; ++j) {
                const int v = v_lo + tid + j * bd;
                if (v < v_hi) {
                    qs[j][0] = rs[j][0] + be * qs[j][0];
                    qs[j][1] = rs[j][1] + be * qs[j][1];
                    qL[v - v_lo] = double2{qs[j][0], qs[j][1]};
                }
            }
            for (int h = tid; h < n_halo; h += bd) {
                const double2 rh = ld2((const double *)rx, halo[h]);
                const double2 qh = qL[n_own + h];
                qL[n_own + h] = double2{rh.x + be * qh.x, rh.y + be * qh.y};
            }
            __syncthreads();
        }
        if (!alive) break;
        if (status == VTX_CG_MAXITER && sqrt(rr) <= a.o.tol * sqrt(rr0)) status = VTX_CONVERGED;
        // project the solution to zero mean, publish it, contract
        sx = sy = 0.0;
#pragma unroll
        for (int j = 0; j < kMbKV; ++j)
            if (v_lo + tid + j * bd < v_hi) {
                sx += xs[j][0];
                sy += xs[j][1];
            }
        vals[0] = block_allsum(sx, sh);
        vals[1] = block_allsum(sy, sh);
        if (!sync.arrive(vals, 2, s_out, &s_flag)) break;
        const double mxx = s_out[0] / (double)nv, mxy = s_out[1] / (double)nv;
        double *x = G.cg;
#pragma unroll
        for (int j = 0; j < kMbKV; ++j) {
            const int v = v_lo + tid + j * bd;
            if (v < v_hi) st2(x, v, xs[j][0] - mxx, xs[j][1] - mxy);
        }
        vals[0] = 0.0;
        if (!sync.arrive(vals, 1, s_out, &s_flag)) break;
        if (a.o.theta == VTX_THETA_LAMBDA) {
            const int e0 = (int)((int64_t)t.n_edge * part / a.K);
            const int e1 = (int)((int64_t)t.n_edge * (part + 1) / a.K);
            for (int e = e0 + tid; e < e1; e += bd) G.g[e] = contract_lambda_one<double>(t, X, x, e);
        } else {
            const int c0 = (int)((int64_t)nc * part / a.K);
            const int c1 = (int)((int64_t)nc * (part + 1) / a.K);
            for (int c = c0 + tid; c < c1; c += bd) G.g[c] = contract_p0_one<double>(t, X, p, x, c);
        }
        if (part == 0 && tid == 0) {
            vtx_grad_result gr{};
            gr.cg_iters = it;
            gr.cg_rel_res = rr0 > 0.0 ? sqrt(rr / rr0) : 0.0;
            gr.status = status;
            a.res[idx] = gr;
        }
        // the next tissue rebuilds the LDS; the contraction reads only
        // global memory, so no part waits for another here
        __syncthreads();
    }
}

}  // namespace vtx

namespace vtx {

// ------------------------------------------------- relaxation, no T1
// Batched gradient descent (Methods, "Simulation engine"; with the EP nudge
// when the items carry one) with each tissue split over K workgroups as in
// k_batch_cg_mb.  Each part keeps the positions of its local vertices and the
// coefficients of its local cells in LDS and its stars in registers; an
// iteration is the cell pass over the local cells, the vertex pass with the
// step for the owned vertices, and one barrier that carries max |F| and the
// sums of the nudge gradient at the new positions (the next iteration's
// mean) while the new owned positions travel through the two global position
// buffers; then each part reads its halo.  The cell and vertex arithmetic
// are the functions of the other relaxation kernels, so the iterates equal
// theirs (the nudge mean is summed in another order).  Without T1 only.
struct MbRelaxArgs {
    const BatchItem *items;
    const int32_t *order;
    int n, K, n_groups;
    BatchOpts o;
    vtx_relax_result *res;
    MbGroup *groups;
    int lds_bytes;
    uint64_t wait_ticks;
};

template <typename PosT, typename M>
__global__ __launch_bounds__(kMbThreads) void k_batch_relax_mb(MbRelaxArgs a) {
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    __shared__ double sh[16];
    __shared__ double s_out[4];
    __shared__ int s_flag;
    __shared__ int s_scan[16];
    __shared__ int s_fail;
    const int tid = threadIdx.x, bd = blockDim.x;
    const int grp = blockIdx.x % a.n_groups, part = blockIdx.x / a.n_groups;
    MbSync sync{a.groups + grp, a.K, part, 0u, a.wait_ticks};
    for (int slot = grp; slot < a.n; slot += a.n_groups) {
        const int idx = a.order[slot];
        const BatchItem &B = a.items[idx];
        const DevTissue t = B.t;
        const DevParams<PosT> p = to_dev<PosT>(B.p);
        const int nv = t.n_vert;
        const int v_lo = (int)((int64_t)nv * part / a.K);
        const int v_hi = (int)((int64_t)nv * (part + 1) / a.K);
        LdsBump lb{lds_dyn, 0, a.lds_bytes};
        MbLocal L = mb_partition(t, v_lo, v_hi, lb, s_scan, &s_fail);
        const int n_own = L.n_own, n_lc = L.n_lc, n_halo = L.n_halo;
        int32_t *crow = (int32_t *)lb.take(4 * (int64_t)L.n_corner);
        PosT *posL = (PosT *)lb.take(2 * (int64_t)sizeof(PosT) * L.n_lv);
        M *capL = (M *)lb.take(2 * (int64_t)sizeof(M) * n_lc);
        PosT *cpar = (PosT *)lb.take(4 * (int64_t)sizeof(PosT) * n_lc);
        __syncthreads();
        const bool fits = lb.ok() && L.fits;
        PosT *buf[2] = {(PosT *)B.X, (PosT *)B.xbuf};
        if (fits) {
            // corner rows in local ids (image bits kept), cell parameters
            for (int l = tid; l < n_lc; l += bd) {
                const int c = L.lcg[l];
                const int rb = t.row_ptr[c], n = t.nsides[c], off = L.cstart[l];
                for (int k = 0; k < n; ++k) {
                    const int32_t w = t.corner[rb + k];
                    crow[off + k] = pack_id(L.vmap[id_of(w)], ox_of(w), oy_of(w));
                }
                cpar[4 * l] = p.ka(c);
                cpar[4 * l + 1] = p.a0(c);
                cpar[4 * l + 2] = p.kp(c);
                cpar[4 * l + 3] = p.p0(c);
            }
            for (int l = tid; l < L.n_lv; l += bd) {
                const int v = l < n_own ? v_lo + l : L.halo[l - n_own];
                posL[2 * l] = buf[0][2 * (int64_t)v];
                posL[2 * l + 1] = buf[0][2 * (int64_t)v + 1];
            }
        }
        // owned stars (local neighbour words, local cells, tensions) and
        // nudge targets in registers
        int32_t sw[kMbKV][3], sc[kMbKV][3];
        PosT sl[kMbKV][3];
        double nt[kMbKV][2];
        const double inv_n = 1.0 / (double)nv;
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int j = 0; j < kMbKV; ++j) {
            const int v = v_lo + tid + j * bd;
            nt[j][0] = nt[j][1] = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                sw[j][k] = sc[j][k] = 0;
                sl[j][k] = (PosT)0;
            }
            if (fits && v < v_hi) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int32_t w = t.star[star_nb_at(nv, k, v)];
                    sw[j][k] = pack_id(L.vmap[id_of(w)], ox_of(w), oy_of(w));
                    sc[j][k] = L.cmap[t.star[star_cell_at(nv, k, v)]];
                    sl[j][k] = p.lam ? p.lam[t.star[star_edge_at(nv, k, v)]] : p.lam_s;
                }
                if (B.beta != 0.0) {
                    if (B.Xt) {
                        const PosT *Xt = (const PosT *)B.Xt;
                        nt[j][0] = (double)Xt[2 * (int64_t)v];
                        nt[j][1] = (double)Xt[2 * (int64_t)v + 1];
                        sx += min_image((double)buf[0][2 * (int64_t)v] - nt[j][0], t.Lx) * inv_n;
                        sy += min_image((double)buf[0][2 * (int64_t)v + 1] - nt[j][1], t.Ly) * inv_n;
                    } else {
                        nt[j][0] = B.g_lin[2 * (int64_t)v];
                        nt[j][1] = B.g_lin[2 * (int64_t)v + 1];
                        sx += nt[j][0];
                        sy += nt[j][1];
                    }
                }
            }
        }
        double vals[4] = {block_allsum(sx, sh), block_allsum(sy, sh), fits ? 0.0 : 1.0, 0.0};
        if (!sync.arrive(vals, 3, s_out, &s_flag)) break;
        if (s_out[2] != 0.0) {   // some part cannot hold this tissue: leave it to the host
            if (part == 0 && tid == 0) {
                vtx_relax_result r{};
                r.status = kMbNoFit;
                a.res[idx] = r;
            }
            continue;
        }
        double mx = s_out[0] * inv_n, my = s_out[1] * inv_n;
        int64_t iter = 0, count = 0;
        double last_mf = 0.0;
        int status = VTX_NOT_CONVERGED, result_buf = 0, cur = 0;
        bool alive = true;
        for (;;) {
            // cell pass over the local cells
            for (int l = tid; l < n_lc; l += bd) {
                const int off = L.cstart[l], n = L.cstart[l + 1] - off;
                PosT A, P;
                cell_geom<PosT, PosT>(
                    t, posL, n, [&](int k) { return crow[off + k]; }, 0, A, P, false, (PosT)0,
                    nullptr, nullptr);
                st2(capL, l, (M)((PosT)2 * cpar[4 * l] * (A - cpar[4 * l + 1])),
                    (M)((PosT)2 * cpar[4 * l + 2] * (P - cpar[4 * l + 3])));
            }
            __syncthreads();
            // vertex pass with the step; new owned positions to the other buffer
            double mf = 0.0;
            PosT pn[kMbKV][2];
            sx = sy = 0.0;
#pragma unroll
            for (int j = 0; j < kMbKV; ++j) {
                const int v = v_lo + tid + j * bd;
                pn[j][0] = pn[j][1] = (PosT)0;
                if (v < v_hi) {
                    StarLoad<PosT, M> S;
                    S.pi = ld2(posL, v - v_lo);
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        S.w[k] = sw[j][k];
                        S.c[k] = sc[j][k];
                        S.lam[k] = sl[j][k];
                        S.q[k] = ld2(posL, id_of(S.w[k]));
                        S.cc[k] = ld2(capL, S.c[k]);
                    }
                    Star<PosT, M> st;
                    PosT xi, yi;
                    star_math<PosT, M>(t, S, st, xi, yi);
                    M fx, fy;
                    star_force<PosT, M>(st, fx, fy);
                    double gx = fx, gy = fy;
                    if (B.beta != 0.0) {
                        double cx, cy;
                        if (B.Xt) {
                            cx = min_image((double)xi - nt[j][0], t.Lx) * inv_n;
                            cy = min_image((double)yi - nt[j][1], t.Ly) * inv_n;
                        } else {
                            cx = nt[j][0];
                            cy = nt[j][1];
                        }
                        gx -= B.beta * (cx - mx);
                        gy -= B.beta * (cy - my);
                    }
                    mf = fmax(mf, fmax(fabs(gx), fabs(gy)));
                    if (!(gx == gx) || !(gy == gy)) mf = INFINITY;
                    pn[j][0] = (PosT)((double)xi + a.o.eta * gx);
                    pn[j][1] = (PosT)((double)yi + a.o.eta * gy);
                    st2(buf[cur ^ 1], v, pn[j][0], pn[j][1]);
                    if (B.beta != 0.0) {
                        if (B.Xt) {
                            sx += min_image((double)pn[j][0] - nt[j][0], t.Lx) * inv_n;
                            sy += min_image((double)pn[j][1] - nt[j][1], t.Ly) * inv_n;
                        } else {
                            sx += nt[j][0];
                            sy += nt[j][1];
                        }
                    }
                }
            }
            vals[0] = block_max(mf, sh);   // valid in thread 0, the one that publishes it
            vals[1] = block_allsum(sx, sh);
            vals[2] = block_allsum(sy, sh);
            if (!sync.arrive(vals, 3, s_out, &s_flag, 1u)) {
                alive = false;
                break;
            }
            const double m = s_out[0];
            ++iter;
            last_mf = m;
            bool done = false;
            if (!(m <= 1.7976931348623157e308)) {
                status = VTX_E_NONFINITE;
                result_buf = cur;
                done = true;
            } else {
                count = m < a.o.tol ? count + 1 : 0;
                if (count >= a.o.patience) {
                    status = VTX_CONVERGED;
                    result_buf = cur;
                    done = true;
                } else if (iter >= a.o.max_iter) {
                    status = VTX_NOT_CONVERGED;
                    result_buf = cur ^ 1;
                    done = true;
                }
            }
            if (done) break;
            // next iteration: owned from registers, halo from the buffer
#pragma unroll
            for (int j = 0; j < kMbKV; ++j) {
                const int v = v_lo + tid + j * bd;
                if (v < v_hi) {
                    posL[2 * (v - v_lo)] = pn[j][0];
                    posL[2 * (v - v_lo) + 1] = pn[j][1];
                }
            }
            const PosT *nb = buf[cur ^ 1];
            for (int h = tid; h < n_halo; h += bd) {
                const int v = L.halo[h];
                posL[2 * (n_own + h)] = nb[2 * (int64_t)v];
                posL[2 * (n_own + h) + 1] = nb[2 * (int64_t)v + 1];
            }
            mx = s_out[1] * inv_n;
            my = s_out[2] * inv_n;
            cur ^= 1;
            __syncthreads();
        }
        if (!alive) break;
        // the returned positions into the caller's buffer, then the energy
        // (+ beta C) there
        if (result_buf == 1)
            for (int v = v_lo + tid; v < v_hi; v += bd) {
                buf[0][2 * (int64_t)v] = buf[1][2 * (int64_t)v];
                buf[0][2 * (int64_t)v + 1] = buf[1][2 * (int64_t)v + 1];
            }
        vals[0] = 0.0;
        if (!sync.arrive(vals, 1, s_out, &s_flag)) break;
        const PosT *Xr = buf[0];
        double e = 0.0;
        const int c0 = (int)((int64_t)t.n_cell * part / a.K);
        const int c1 = (int)((int64_t)t.n_cell * (part + 1) / a.K);
        for (int c = c0 + tid; c < c1; c += bd) {
            const int rb = t.row_ptr[c], nn = t.nsides[c];
            PosT A, P;
            cell_geom<PosT, PosT>(
                t, Xr, nn, [&](int k) { return t.corner[rb + k]; }, rb, A, P, false, (PosT)0,
                nullptr, nullptr);
            const double da = (double)A - (double)p.a0(c), dp = (double)P - (double)p.p0(c);
            e += (double)p.ka(c) * da * da + (double)p.kp(c) * dp * dp;
        }
        const int e0 = (int)((int64_t)t.n_edge * part / a.K);
        const int e1 = (int)((int64_t)t.n_edge * (part + 1) / a.K);
        for (int k = e0 + tid; k < e1; k += bd) e += (double)p.lm(k) * edge_len_one<PosT>(t, Xr, k);
        if (B.beta != 0.0)
            for (int v = v_lo + tid; v < v_hi; v += bd) {
                if (B.Xt) {
                    const PosT *Xt = (const PosT *)B.Xt;
                    const double dx = min_image((double)Xr[2 * (int64_t)v] - (double)Xt[2 * (int64_t)v], t.Lx);
                    const double dy = min_image((double)Xr[2 * (int64_t)v + 1] - (double)Xt[2 * (int64_t)v + 1], t.Ly);
                    e += B.beta * (dx * dx + dy * dy) * 0.5 / (double)nv;
                } else {
                    e += B.beta * (B.g_lin[2 * (int64_t)v] * (double)Xr[2 * (int64_t)v] +
                                   B.g_lin[2 * (int64_t)v + 1] * (double)Xr[2 * (int64_t)v + 1]);
                }
            }
        vals[0] = block_allsum(e, sh);
        if (!sync.arrive(vals, 1, s_out, &s_flag)) break;
        if (part == 0 && tid == 0) {
            vtx_relax_result r{};
            r.iters = iter;
            r.max_f = last_mf;
            r.energy = s_out[0];
            r.status = status;
            a.res[idx] = r;
        }
        __syncthreads();
    }
}

}  // namespace vtx

// ------------------------------------------------------------------ host
namespace vtx {

int mb_no_fit_status() { return kMbNoFit; }
size_t mb_group_bytes() { return sizeof(MbGroup); }

// Largest cooperative grid of k_batch_cg_mb with the device's per-workgroup
// LDS as dynamic LDS; 0 if the device cannot launch it cooperatively.
hipError_t mb_capacity(int *max_blocks, int *lds_bytes) {
    *max_blocks = 0;
    *lds_bytes = 0;
    int dev = 0, coop = 0, cus = 0, lds_max = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess || !coop) return e;
    hipFuncAttributes fa{};
    e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&k_batch_cg_mb));
    if (e != hipSuccess) return e;
    const int lds = lds_max - (int)fa.sharedSizeBytes;
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch_cg_mb),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(&k_batch_cg_mb), kMbThreads, (size_t)lds);
    if (e != hipSuccess) return e;
    *max_blocks = per_cu * cus;
    *lds_bytes = lds;
    return hipSuccess;
}

// One cooperative launch: n tissues (items, order on the device), K parts
// each, n_groups groups (groups: n_groups zeroed MbGroup records).  Results
// go to res_d; tissues that do not fit report mb_no_fit_status().
hipError_t mb_launch(const GradItem *items, const int32_t *order, int n, const GradOpts &o,
                     int K, int n_groups, int lds_bytes, vtx_grad_result *res_d, void *groups,
                     hipStream_t s) {
    int dev = 0, rate_khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(groups, 0, sizeof(MbGroup) * (size_t)n_groups, s);
    if (e != hipSuccess) return e;
    MbArgs a{items, order, n, K, n_groups, o, res_d, (MbGroup *)groups, lds_bytes,
             (uint64_t)(rate_khz > 0 ? rate_khz : 100000) * 1000ull * 20ull};  // 20 s per wait
    void *args[] = {&a};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_batch_cg_mb),
                                      dim3(n_groups * K), dim3(kMbThreads), args,
                                      (unsigned)lds_bytes, s);
}


template <typename PosT, typename M>
static hipError_t mb_relax_capacity_t(int *max_blocks, int *lds_bytes) {
    *max_blocks = 0;
    *lds_bytes = 0;
    int dev = 0, coop = 0, cus = 0, lds_max = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess || !coop) return e;
    const void *f = reinterpret_cast<const void *>(&k_batch_relax_mb<PosT, M>);
    hipFuncAttributes fa{};
    e = hipFuncGetAttributes(&fa, f);
    if (e != hipSuccess) return e;
    const int lds = lds_max - (int)fa.sharedSizeBytes;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kMbThreads, (size_t)lds);
    if (e != hipSuccess) return e;
    *max_blocks = per_cu * cus;
    *lds_bytes = lds;
    return hipSuccess;
}

hipError_t mb_relax_capacity(int mode, int *max_blocks, int *lds_bytes) {
    if (mode == VTX_F32) return mb_relax_capacity_t<float, float>(max_blocks, lds_bytes);
    if (mode == VTX_F64) return mb_relax_capacity_t<double, double>(max_blocks, lds_bytes);
    return mb_relax_capacity_t<double, float>(max_blocks, lds_bytes);
}

hipError_t mb_relax_launch(int mode, const BatchItem *items, const int32_t *order, int n,
                           const BatchOpts &o, int K, int n_groups, int lds_bytes,
                           vtx_relax_result *res_d, void *groups, hipStream_t s) {
    int dev = 0, rate_khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(groups, 0, sizeof(MbGroup) * (size_t)n_groups, s);
    if (e != hipSuccess) return e;
    MbRelaxArgs a{items, order, n, K, n_groups, o, res_d, (MbGroup *)groups, lds_bytes,
                  (uint64_t)(rate_khz > 0 ? rate_khz : 100000) * 1000ull * 20ull};
    void *args[] = {&a};
    const void *f = mode == VTX_F32   ? reinterpret_cast<const void *>(&k_batch_relax_mb<float, float>)
                    : mode == VTX_F64 ? reinterpret_cast<const void *>(&k_batch_relax_mb<double, double>)
                                      : reinterpret_cast<const void *>(&k_batch_relax_mb<double, float>);
    return hipLaunchCooperativeKernel(f, dim3(n_groups * K), dim3(kMbThreads), args,
                                      (unsigned)lds_bytes, s);
}

}  // namespace vtx
