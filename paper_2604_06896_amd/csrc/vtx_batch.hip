// Batched relaxation of many independent periodic tissues in one persistent
// launch (VertAX, arXiv 2604.06896, Methods, "Simulation engine", applied
// per tissue).  One workgroup owns one tissue at a time and runs the whole
// loop -- cell pass, T1 pass, vertex pass with the gradient-descent step,
// convergence test -- with workgroup barriers only; tissues are taken from a
// device work queue in descending size so the largest start first.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include "vtx_batch.h"

using namespace vtx;

struct vtx_batch_s {
    std::vector<vtx_tissue> ts;
    std::vector<int32_t> order;  // tissue indices by descending size
    void *items;                 // device BatchItem[2n] (centred EP: both nudges)
    void *gitems;                // device GradItem[n]
    void **xm_list;              // device pointer list (EP minus states)
    int32_t *order_d;            // device [2n]: order, then order + n
    unsigned int *queue;
    vtx_relax_result *res_d;     // device [2n]
    vtx_grad_result *gres_d;
    void *mb_groups;             // device MbGroup[n] (multi-workgroup adjoint)
    int32_t *order2_d;           // device tissue list of a second launch
    hipStream_t cap_stream;
};

namespace vtx {

// Gradient of the nudge cost at vertex v (v2v, minimum image; or linear).
template <typename PosT>
__device__ __forceinline__ void nudge_grad(const BatchItem &B, const PosT *X, int v, double inv_n,
                                           double &cx, double &cy) {
    if (B.Xt) {
        const PosT *Xt = (const PosT *)B.Xt;
        cx = min_image((double)X[2 * (int64_t)v] - (double)Xt[2 * (int64_t)v], B.t.Lx) * inv_n;
        cy = min_image((double)X[2 * (int64_t)v + 1] - (double)Xt[2 * (int64_t)v + 1], B.t.Ly) * inv_n;
    } else {
        cx = B.g_lin[2 * (int64_t)v];
        cy = B.g_lin[2 * (int64_t)v + 1];
    }
}

__global__ void k_reset_queue(unsigned int *q) { *q = 0u; }

// LDS bytes the batched adjoint needs to hold, for one tissue, the arrays its
// Hessian-vector product gathers: positions, the vector multiplied, and the
// two per-cell coefficient pairs (cA, cP at X* and G, B of the vector).
template <typename PosT, typename M>
__host__ __device__ inline int64_t cg_lds_bytes(int64_t n_vert, int64_t n_cell) {
    auto a16 = [](int64_t b) { return (b + 15) & ~(int64_t)15; };
    return a16(2 * n_vert * (int64_t)sizeof(PosT)) + a16(2 * n_vert * 8) +
           2 * a16(2 * n_cell * (int64_t)sizeof(M));
}

// LDS bytes of the register-resident form of the batched CG: the arrays of
// cg_lds_bytes, then every cell's corner row (one int per half-edge).
template <typename PosT, typename M>
__host__ __device__ inline int64_t cg_fast_lds_bytes(int64_t n_vert, int64_t n_cell,
                                                     int64_t n_he) {
    return cg_lds_bytes<PosT, M>(n_vert, n_cell) + ((4 * n_he + 15) & ~(int64_t)15);
}

// Whether a tissue takes the register-resident CG with K cells and 2K
// vertices per thread: it has at most that many, and its arrays and rows fit
// in the LDS given.
template <typename PosT, typename M, int K>
__host__ __device__ inline bool cg_fast_fits(int64_t n_vert, int64_t n_cell, int64_t n_he,
                                             int block_threads, int64_t lds_bytes) {
    return n_cell <= K * (int64_t)block_threads && n_vert <= 2 * K * (int64_t)block_threads &&
           cg_fast_lds_bytes<PosT, M>(n_vert, n_cell, n_he) <= lds_bytes;
}

// Cells of a tissue handed to the threads of the register-resident CG by
// side count.  The cells, stably sorted by min(sides, 15), are cut into K
// runs of ceil(n_cell / K); slot k of thread i takes entry i of run k,
// counted from the front in even runs and from the back in odd ones.  The
// cells of one slot across a wave then have about the same number of
// corners (the wave walks them in step), and each thread's K cells about K
// times the mean, so the waves finish the cell phase together.  `tmp`
// holds n_cell ints.  cid[k] is the cell of the thread's slot k, -1 if the
// run has no entry i.
template <int K>
__device__ __forceinline__ void cells_by_sides(const DevTissue &t, int *tmp, int *s_scan,
                                               int (&cid)[K]) {
    constexpr int kBuckets = 16;
    const int tid = threadIdx.x, bd = blockDim.x, nc = t.n_cell;
    int b[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int c = tid + i * bd;
        b[i] = c < nc ? min(t.nsides[c], kBuckets - 1) : -1;
    }
    int base = 0;
    for (int bucket = 0; bucket < kBuckets; ++bucket) {
        int cnt = 0;
#pragma unroll
        for (int i = 0; i < K; ++i) cnt += b[i] == bucket ? 1 : 0;
        int tot;
        int at = base + block_exclusive_scan(cnt, s_scan, tot);
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (b[i] == bucket) tmp[at++] = tid + i * bd;
        base += tot;
    }
    __syncthreads();
    const int run = (nc + K - 1) / K;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int lo = i * run, len = min(run, nc - lo);
        cid[i] = tid < len ? tmp[lo + ((i & 1) ? len - 1 - tid : tid)] : -1;
    }
    __syncthreads();  // `tmp` is free again
}

// Conjugate gradients of one tissue in which thread i owns K cells (given
// by cells_by_sides) and vertices i + j B (j < 2K), B = blockDim.x.  What a
// step reads of the topology (the cells' corner rows, the vertices' star
// entries and tensions) is loaded once: the rows into LDS behind the arrays of
// cg_lds_bytes (already resident), the stars into registers; the solution
// and residual of the thread's own vertices stay in registers.  A step then
// waits only on LDS and the workgroup's reductions.  The arithmetic and the
// order of every sum are those of the general loop; on return the solution
// is in G.cg.
template <typename PosT, typename M, int K>
__device__ __forceinline__ int batch_cg_fast(const DevTissue &t, const DevParams<PosT> &p,
                                             const GradItem &G, unsigned char *lds,
                                             int64_t o_q, int64_t o_c, int64_t o_a,
                                             int64_t o_r, double mbx, double mby,
                                             const GradOpts &o, double *sh, int *s_scan,
                                             int64_t &it_out, double &rel_out) {
    constexpr int KV = 2 * K;
    const int tid = threadIdx.x, bd = blockDim.x, nv = t.n_vert;
    const PosT *Xl = (const PosT *)lds;
    double *ql = (double *)(lds + o_q);
    const M *capl = (const M *)(lds + o_c);
    M *auxl = (M *)(lds + o_a);
    int32_t *rowl = (int32_t *)(lds + o_r);
    int cid[K];
    // q is not set yet; its 2 n_vert doubles hold the n_cell <= n_vert ints
    // (three corners per vertex, at least three per cell)
    cells_by_sides<K>(t, reinterpret_cast<int *>(ql), s_scan, cid);
    int n[K], lrb[K];
    PosT ka[K], kp[K];
    int rows_base = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int c = cid[i];
        int rb = 0;
        n[i] = 0;
        ka[i] = kp[i] = 0;
        if (c >= 0) {
            rb = t.row_ptr[c];
            n[i] = t.nsides[c];
            ka[i] = p.ka(c);
            kp[i] = p.kp(c);
        }
        int tot;
        lrb[i] = rows_base + block_exclusive_scan(n[i], s_scan, tot);
        rows_base += tot;
        const int nk = min(n[i], t.n_he - lrb[i]);  // the rows hold n_he corners in all
        for (int k = 0; k < nk; ++k) rowl[lrb[i] + k] = t.corner[rb + k];
    }
    int32_t sw[KV][3], sc[KV][3];
    PosT sl[KV][3];
    double xs[KV][2], rs[KV][2];
    double rr = 0.0;
#pragma unroll
    for (int j = 0; j < KV; ++j) {
        const int v = tid + j * bd;
        if (v < nv) {
            const int4 a = reinterpret_cast<const int4 *>(t.star)[v];
            const int4 b = reinterpret_cast<const int4 *>(t.star + 4 * (int64_t)nv)[v];
            const int32_t e[3] = {b.z, b.w, t.star[8 * (int64_t)nv + v]};
            sw[j][0] = a.x;
            sw[j][1] = a.y;
            sw[j][2] = a.z;
            sc[j][0] = a.w;
            sc[j][1] = b.x;
            sc[j][2] = b.y;
#pragma unroll
            for (int k = 0; k < 3; ++k) sl[j][k] = p.lam ? p.lam[e[k]] : p.lam_s;
            // r = P b, q = r, x = 0
            const double r0 = G.b[2 * (int64_t)v] - mbx, r1 = G.b[2 * (int64_t)v + 1] - mby;
            rs[j][0] = r0;
            rs[j][1] = r1;
            ql[2 * v] = r0;
            ql[2 * v + 1] = r1;
            xs[j][0] = 0.0;
            xs[j][1] = 0.0;
            rr += r0 * r0 + r1 * r1;
        }
    }
    rr = block_allsum(rr, sh);  // its barriers also publish q and the rows
    const double rr0 = rr;
    int status = rr0 > 0.0 ? VTX_CG_MAXITER : VTX_CONVERGED;
    int64_t it = 0;
    while (status == VTX_CG_MAXITER && it < o.max_iter) {
        if (sqrt(rr) <= o.tol * sqrt(rr0)) {
            status = VTX_CONVERGED;
            break;
        }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int base = lrb[i];
            if (n[i] > 0)
                hvp_cell_row<PosT, M>(
                    t, Xl, ql, n[i], [&](int k) { return rowl[base + k]; }, ka[i], kp[i],
                    auxl, cid[i]);
        }
        __syncthreads();
        double d = 0.0, aq[KV][2];
#pragma unroll
        for (int j = 0; j < KV; ++j) {
            const int v = tid + j * bd;
            if (v < nv) {
                StarLoad<PosT, M> L;
                L.pi = ld2(Xl, v);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    L.w[k] = sw[j][k];
                    L.c[k] = sc[j][k];
                    L.lam[k] = sl[j][k];
                    L.q[k] = ld2(Xl, id_of(L.w[k]));
                    L.cc[k] = ld2(capl, L.c[k]);
                }
                d += hvp_vertex_star<PosT, M>(t, L, auxl, ql, v, aq[j][0], aq[j][1]);
            }
        }
        const double pAp = block_allsum(d, sh);
        if (!(pAp > 0.0)) {
            status = VTX_CG_NEG_CURVATURE;
            break;
        }
        const double al = rr / pAp;
        double rn = 0.0;
#pragma unroll
        for (int j = 0; j < KV; ++j) {
            const int v = tid + j * bd;
            if (v < nv) {
                xs[j][0] += al * ql[2 * v];
                xs[j][1] += al * ql[2 * v + 1];
                const double r0 = rs[j][0] - al * aq[j][0], r1 = rs[j][1] - al * aq[j][1];
                rs[j][0] = r0;
                rs[j][1] = r1;
                rn += r0 * r0 + r1 * r1;
            }
        }
        rn = block_allsum(rn, sh);
        const double be = rn / rr;
        rr = rn;
        ++it;
#pragma unroll
        for (int j = 0; j < KV; ++j) {
            const int v = tid + j * bd;
            if (v < nv) {
                ql[2 * v] = rs[j][0] + be * ql[2 * v];
                ql[2 * v + 1] = rs[j][1] + be * ql[2 * v + 1];
            }
        }
        __syncthreads();
    }
    if (status == VTX_CG_MAXITER && sqrt(rr) <= o.tol * sqrt(rr0)) status = VTX_CONVERGED;
    rel_out = rr0 > 0.0 ? sqrt(rr / rr0) : 0.0;
    it_out = it;
#pragma unroll
    for (int j = 0; j < KV; ++j) {
        const int v = tid + j * bd;
        if (v < nv) {
            G.cg[2 * (int64_t)v] = xs[j][0];
            G.cg[2 * (int64_t)v + 1] = xs[j][1];
        }
    }
    return status;
}

// Cells per thread of the register-resident CG for a kernel of up to MAXT
// threads (0: none).  Its state for two cells and four vertices per thread
// needs more registers than the 128 a 1024-thread workgroup allows, so only
// the 512-thread kernel (256 registers) has it.
template <int MAXT>
constexpr int kFastK = MAXT <= 512 ? 2 : 0;

// Batched adjoint: one workgroup per tissue runs conjugate gradients on
// H mu = P b (P removes the per-component mean) with FP64 dots, then the
// contraction with the mixed derivatives (Methods, "Implicit
// differentiation (ID)"); same steps as the grid path.  A tissue whose
// gathered arrays fit in the launch's dynamic LDS (`lds_bytes`) keeps them
// there for the whole solve: each step's gathers then wait on LDS instead
// of the L2.  The arithmetic is the same either way.
template <typename PosT, typename M, int MAXT>
__global__ __launch_bounds__(MAXT) void k_batch_cg(const GradItem *__restrict__ items,
                                                   const int32_t *__restrict__ order, int n,
                                                   unsigned int *queue, GradOpts o,
                                                   vtx_grad_result *res, int lds_bytes) {
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    __shared__ double sh[16];
    __shared__ int s_item;
    __shared__ int s_scan[16];
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int slot = s_item;
        __syncthreads();
        if (slot >= n) return;
        const int idx = order[slot];
        const GradItem &G = items[idx];
        const DevTissue t = G.t;
        const DevParams<PosT> p = to_dev<PosT>(G.p);
        const PosT *X = (const PosT *)G.X;
        const int nv = t.n_vert;
        const bool in_lds = cg_lds_bytes<PosT, M>(nv, t.n_cell) <= (int64_t)lds_bytes;
        const int64_t o_q = (2 * (int64_t)nv * (int64_t)sizeof(PosT) + 15) & ~(int64_t)15;
        const int64_t o_c = o_q + ((2 * (int64_t)nv * 8 + 15) & ~(int64_t)15);
        const int64_t o_a = o_c + ((2 * (int64_t)t.n_cell * (int64_t)sizeof(M) + 15) & ~(int64_t)15);
        // LDS layout: positions (Xh, read by the Hessian-vector product), the
        // vector it multiplies (q of CG, the Lanczos vector of MINRES), then
        // the cell coefficients (cap) and the HVP's per-cell terms (aux)
        const PosT *Xh = in_lds ? (const PosT *)lds_dyn : X;
        M *cap = in_lds ? (M *)(lds_dyn + o_c) : (M *)G.cap;
        M *aux = in_lds ? (M *)(lds_dyn + o_a) : (M *)G.aux;
        if (in_lds) {
            PosT *Xl = (PosT *)lds_dyn;
            for (int k = threadIdx.x; k < 2 * nv; k += blockDim.x) Xl[k] = X[k];
        }
        double *x = G.cg, *r = G.cg + 2 * (int64_t)nv,
               *q = in_lds ? (double *)(lds_dyn + o_q) : G.cg + 4 * (int64_t)nv,
               *Aq = G.cg + 6 * (int64_t)nv;
        // cell coefficients at X*
        for (int c = threadIdx.x; c < t.n_cell; c += blockDim.x) {
            const int rb = t.row_ptr[c], nn = t.nsides[c];
            PosT A, P;
            cell_geom<PosT, PosT>(
                t, X, nn, [&](int k) { return t.corner[rb + k]; }, rb, A, P, false, (PosT)0,
                nullptr, nullptr);
            st2(cap, c, (M)((PosT)2 * p.ka(c) * (A - p.a0(c))),
                (M)((PosT)2 * p.kp(c) * (P - p.p0(c))));
        }
        double sx = 0.0, sy = 0.0;
        for (int v = threadIdx.x; v < nv; v += blockDim.x) {
            sx += G.b[2 * (int64_t)v];
            sy += G.b[2 * (int64_t)v + 1];
        }
        const double mbx = block_allsum(sx, sh) / (double)nv;
        const double mby = block_allsum(sy, sh) / (double)nv;
        int status;
        int64_t it = 0;
        double rel_res;
        const int64_t o_r = o_a + ((2 * (int64_t)t.n_cell * (int64_t)sizeof(M) + 15) & ~(int64_t)15);
        if (kFastK<MAXT> > 0 && !o.minres && in_lds &&
            cg_fast_fits<PosT, M, kFastK<MAXT>>(nv, t.n_cell, t.n_he, (int)blockDim.x,
                                                 lds_bytes)) {
            status = batch_cg_fast<PosT, M, (kFastK<MAXT> > 0 ? kFastK<MAXT> : 1)>(
                t, p, G, lds_dyn, o_q, o_c, o_a, o_r, mbx, mby, o, sh, s_scan, it, rel_res);
        } else if (!o.minres) {
            // CG: r = P b, q = r, x = 0
            double rr = 0.0;
            for (int v = threadIdx.x; v < nv; v += blockDim.x) {
                const double r0 = G.b[2 * (int64_t)v] - mbx, r1 = G.b[2 * (int64_t)v + 1] - mby;
                r[2 * (int64_t)v] = r0;
                r[2 * (int64_t)v + 1] = r1;
                q[2 * (int64_t)v] = r0;
                q[2 * (int64_t)v + 1] = r1;
                x[2 * (int64_t)v] = 0.0;
                x[2 * (int64_t)v + 1] = 0.0;
                rr += r0 * r0 + r1 * r1;
            }
            rr = block_allsum(rr, sh);
            const double rr0 = rr;
            status = rr0 > 0.0 ? VTX_CG_MAXITER : VTX_CONVERGED;
            while (status == VTX_CG_MAXITER && it < o.max_iter) {
                if (sqrt(rr) <= o.tol * sqrt(rr0)) {
                    status = VTX_CONVERGED;
                    break;
                }
                for (int c = threadIdx.x; c < t.n_cell; c += blockDim.x)
                    hvp_cell_one<PosT, M>(t, Xh, p, q, aux, c);
                __syncthreads();
                double d = 0.0;
                for (int v = threadIdx.x; v < nv; v += blockDim.x)
                    d += hvp_vertex_one<PosT, M>(t, Xh, p, cap, aux, q, Aq, v);
                const double pAp = block_allsum(d, sh);
                if (!(pAp > 0.0)) {
                    status = VTX_CG_NEG_CURVATURE;
                    break;
                }
                const double al = rr / pAp;
                double rn = 0.0;
                for (int v = threadIdx.x; v < nv; v += blockDim.x) {
                    const int64_t k = 2 * (int64_t)v;
                    x[k] += al * q[k];
                    x[k + 1] += al * q[k + 1];
                    const double r0 = r[k] - al * Aq[k], r1 = r[k + 1] - al * Aq[k + 1];
                    r[k] = r0;
                    r[k + 1] = r1;
                    rn += r0 * r0 + r1 * r1;
                }
                rn = block_allsum(rn, sh);
                const double be = rn / rr;
                rr = rn;
                ++it;
                for (int v = threadIdx.x; v < nv; v += blockDim.x) {
                    const int64_t k = 2 * (int64_t)v;
                    q[k] = r[k] + be * q[k];
                    q[k + 1] = r[k + 1] + be * q[k + 1];
                }
                __syncthreads();
            }
            if (status == VTX_CG_MAXITER && sqrt(rr) <= o.tol * sqrt(rr0)) status = VTX_CONVERGED;
            rel_res = rr0 > 0.0 ? sqrt(rr / rr0) : 0.0;
        } else {
            // MINRES (the recurrences of k_mr_lanczos / k_mr_update): Lanczos
            // vectors mq (current), mqp (previous), mz (next); search
            // directions w1, w2; scalars are computed identically by every
            // thread from block-wide sums.
            double *mq = in_lds ? q : G.cg + 2 * (int64_t)nv, *mqp = G.cg + 4 * (int64_t)nv,
                   *mz = G.cg + 6 * (int64_t)nv, *w1 = G.cg + 8 * (int64_t)nv,
                   *w2 = G.cg + 10 * (int64_t)nv;
            double ss = 0.0;
            for (int v = threadIdx.x; v < nv; v += blockDim.x) {
                const double r0 = G.b[2 * (int64_t)v] - mbx, r1 = G.b[2 * (int64_t)v + 1] - mby;
                mq[2 * (int64_t)v] = r0;
                mq[2 * (int64_t)v + 1] = r1;
                ss += r0 * r0 + r1 * r1;
            }
            const double beta1 = sqrt(block_allsum(ss, sh));
            const double inv1 = beta1 > 0.0 ? 1.0 / beta1 : 0.0;
            for (int k = threadIdx.x; k < 2 * nv; k += blockDim.x) {
                mq[k] *= inv1;
                x[k] = mqp[k] = w1[k] = w2[k] = 0.0;
            }
            __syncthreads();
            double beta = 0.0, c1 = 1.0, s1 = 0.0, c2 = 1.0, s2 = 0.0, phibar = beta1;
            status = beta1 > 0.0 ? VTX_CG_MAXITER : VTX_CONVERGED;
            while (status == VTX_CG_MAXITER && it < o.max_iter) {
                for (int c = threadIdx.x; c < t.n_cell; c += blockDim.x)
                    hvp_cell_one<PosT, M>(t, Xh, p, mq, aux, c);
                __syncthreads();
                double d = 0.0;
                for (int v = threadIdx.x; v < nv; v += blockDim.x)
                    d += hvp_vertex_one<PosT, M>(t, Xh, p, cap, aux, mq, mz, v);
                const double alpha = block_allsum(d, sh);
                double zz = 0.0;
                for (int k = threadIdx.x; k < 2 * nv; k += blockDim.x) {
                    const double zk = mz[k] - (alpha * mq[k] + beta * mqp[k]);
                    mz[k] = zk;
                    zz += zk * zk;
                }
                const double beta_next = sqrt(block_allsum(zz, sh));
                const double eps = s2 * beta, dbar = c2 * beta;
                const double delta = c1 * dbar + s1 * alpha;
                const double gbar = -s1 * dbar + c1 * alpha;
                const double gamma = sqrt(gbar * gbar + beta_next * beta_next);
                ++it;
                if (!(gamma > 0.0)) {
                    status = fabs(phibar) <= o.tol * beta1 ? VTX_CONVERGED : VTX_CG_MAXITER;
                    break;
                }
                const double c = gbar / gamma, s = beta_next / gamma;
                const double tau = c * phibar;
                phibar = -s * phibar;
                for (int k = threadIdx.x; k < 2 * nv; k += blockDim.x) {
                    const double qk = mq[k];
                    const double w = (qk - delta * w1[k] - eps * w2[k]) / gamma;
                    x[k] += tau * w;
                    w2[k] = w1[k];
                    w1[k] = w;
                    mqp[k] = qk;
                    mq[k] = beta_next > 0.0 ? mz[k] / beta_next : 0.0;
                }
                __syncthreads();
                c2 = c1;
                s2 = s1;
                c1 = c;
                s1 = s;
                beta = beta_next;
                if (fabs(phibar) <= o.tol * beta1) status = VTX_CONVERGED;
                else if (!(beta_next > 0.0)) break;
            }
            rel_res = beta1 > 0.0 ? fabs(phibar) / beta1 : 0.0;
        }
        // project the solution to zero mean
        sx = 0.0;
        sy = 0.0;
        for (int v = threadIdx.x; v < nv; v += blockDim.x) {
            sx += x[2 * (int64_t)v];
            sy += x[2 * (int64_t)v + 1];
        }
        const double mxx = block_allsum(sx, sh) / (double)nv;
        const double mxy = block_allsum(sy, sh) / (double)nv;
        for (int v = threadIdx.x; v < nv; v += blockDim.x) {
            x[2 * (int64_t)v] -= mxx;
            x[2 * (int64_t)v + 1] -= mxy;
        }
        __syncthreads();
        if (o.theta == VTX_THETA_LAMBDA)
            for (int e = threadIdx.x; e < t.n_edge; e += blockDim.x)
                G.g[e] = contract_lambda_one<PosT>(t, X, x, e);
        else
            for (int c = threadIdx.x; c < t.n_cell; c += blockDim.x)
                G.g[c] = contract_p0_one<PosT>(t, X, p, x, c);
        if (threadIdx.x == 0) {
            vtx_grad_result gr{};
            gr.cg_iters = it;
            gr.cg_rel_res = rel_res;
            gr.status = status;
            res[idx] = gr;
        }
        __syncthreads();
    }
}

// EP estimate from two states, one workgroup per tissue: the states nudged
// by +beta/2 and -beta/2 (centred EP) or the state nudged by beta and X*
// itself (first-order EP); either way the difference of the parameter
// derivative of E divided by beta.
template <typename PosT>
__global__ __launch_bounds__(1024) void k_batch_ep(const GradItem *__restrict__ items, int n,
                                                   const void *const *Xm_list, double beta,
                                                   int theta) {
    for (int idx = blockIdx.x; idx < n; idx += gridDim.x) {
        const GradItem &G = items[idx];
        const DevTissue t = G.t;
        const PosT *Xp = (const PosT *)G.X;
        const PosT *Xm = (const PosT *)Xm_list[idx];
        if (theta == VTX_THETA_LAMBDA) {
            for (int e = threadIdx.x; e < t.n_edge; e += blockDim.x)
                G.g[e] = (edge_len_one<PosT>(t, Xp, e) - edge_len_one<PosT>(t, Xm, e)) / beta;
        } else {
            const DevParams<PosT> p = to_dev<PosT>(G.p);
            PosOverride<PosT> none{-1, -1, 0, 0, 0, 0};
            for (int c = threadIdx.x; c < t.n_cell; c += blockDim.x) {
                double a, pp, pm;
                cell_walk<PosT>(t, Xp, t.cell_he[c], none, a, pp);
                cell_walk<PosT>(t, Xm, t.cell_he[c], none, a, pm);
                G.g[c] = -2.0 * (double)p.kp(c) * (pp - pm) / beta;
            }
        }
    }
}

// Loop counters of one tissue's relaxation, kept in LDS by thread 0 so that
// no register holds them across the T1 call.
struct RelaxState {
    int64_t iter, count, n_t1, n_st;
    double last_mf;
    int status, result_buf, bad_t1, done, changed;
};

// One T1 pass of a batched tissue (block-wide): sort the candidate edges,
// run the sequential pass in one wave, compact the rows if one moved to the
// pool.  Called through the non-inlined wrappers below, which receive the
// tissue only by address: the pass needs many registers, and a caller that
// kept its own copies of the tissue and parameters live across the call
// would spill them inside the cell and vertex loops.
template <typename PosT, typename M>
__device__ __forceinline__ void t1_pass_body(const BatchItem *Bp, PosT *Xc, M *cap, int ncand,
                                             double l_min, double l_new, int32_t *sort_buf,
                                             int32_t *extra, int32_t *scan, RelaxState *st) {
    const BatchItem &B = *Bp;
    const DevTissue &t = B.t;
    const DevParams<PosT> p = to_dev<PosT>(B.p);
    int np2 = 1;
    while (np2 < ncand) np2 <<= 1;
    int32_t *arr = np2 <= kT1SortCap ? sort_buf : B.t1_list;
    for (int i = threadIdx.x; i < np2; i += blockDim.x)
        arr[i] = i < ncand ? t.he_edge[t.corner_he[B.t1_list[i]]] : INT_MAX;
    __syncthreads();
    block_bitonic(arr, np2);
    if (threadIdx.x < 64) {  // one wave runs the pass
        T1Counts r = t1_sequential<PosT, M>(t, Xc, p, cap, arr, ncand, extra, l_min, l_new);
        if (threadIdx.x == 0) {
            st->n_t1 += r.swaps;
            st->n_st += r.stretches;
            st->changed = r.relocated;
            if (r.overflow) st->bad_t1 = r.overflow;
        }
    }
    __syncthreads();
    if (st->changed) {
        const int bad = rebuild_rows_block(t, scan);
        if (threadIdx.x == 0 && bad) st->bad_t1 = 2;
    }
    __syncthreads();
}

template <typename PosT, typename M>
__device__ __noinline__ void batch_t1_pass(const BatchItem *Bp, PosT *Xc, int ncand,
                                           double l_min, double l_new, int32_t *sort_buf,
                                           int32_t *extra, int32_t *scan, RelaxState *st) {
    t1_pass_body<PosT, M>(Bp, Xc, (M *)Bp->cap, ncand, l_min, l_new, sort_buf, extra, scan, st);
}

// The same pass for a tissue whose positions and coefficients are in LDS.
template <typename PosT, typename M>
__device__ __noinline__ void batch_t1_pass_lds(const BatchItem *Bp, PosT *Xc, M *cap, int ncand,
                                               double l_min, double l_new, int32_t *sort_buf,
                                               int32_t *extra, int32_t *scan, RelaxState *st) {
    t1_pass_body<PosT, M>(Bp, Xc, cap, ncand, l_min, l_new, sort_buf, extra, scan, st);
}

// Energy (+ beta C) at the positions returned in B.X and the tissue's result
// record: the end of a batched relaxation.
template <typename PosT>
__device__ __forceinline__ void batch_relax_result(const BatchItem &B, const DevTissue &t,
                                                   const DevParams<PosT> &p,
                                                   const RelaxState &st, double *sh,
                                                   vtx_relax_result *res, int idx) {
    // energy at the returned positions
    double e = 0.0;
    const PosT *Xr = (const PosT *)B.X;
    for (int c = threadIdx.x; c < t.n_cell; c += blockDim.x) {
        const int rb = t.row_ptr[c], nn = t.nsides[c];
        PosT A, P;
        cell_geom<PosT, PosT>(
            t, Xr, nn, [&](int k) { return t.corner[rb + k]; }, rb, A, P, false, (PosT)0,
            nullptr, nullptr);
        const double da = (double)A - (double)p.a0(c), dp = (double)P - (double)p.p0(c);
        e += (double)p.ka(c) * da * da + (double)p.kp(c) * dp * dp;
    }
    for (int k = threadIdx.x; k < t.n_edge; k += blockDim.x) {
        const int32_t *r = t.he + 8 * (int64_t)t.edge_he[k];
        const double dx = pdiff<double>((double)Xr[2 * (int64_t)r[HG]], (double)Xr[2 * (int64_t)r[HS]], r[HOX], t.Lx);
        const double dy = pdiff<double>((double)Xr[2 * (int64_t)r[HG] + 1], (double)Xr[2 * (int64_t)r[HS] + 1], r[HOY], t.Ly);
        e += (double)p.lm(k) * sqrt(dx * dx + dy * dy);
    }
    if (B.beta != 0.0)
        for (int v = threadIdx.x; v < t.n_vert; v += blockDim.x) {
            if (B.Xt) {
                const PosT *Xt = (const PosT *)B.Xt;
                const double dx = min_image((double)Xr[2 * (int64_t)v] - (double)Xt[2 * (int64_t)v], t.Lx);
                const double dy = min_image((double)Xr[2 * (int64_t)v + 1] - (double)Xt[2 * (int64_t)v + 1], t.Ly);
                e += B.beta * (dx * dx + dy * dy) * 0.5 / (double)t.n_vert;
            } else {
                e += B.beta * (B.g_lin[2 * (int64_t)v] * (double)Xr[2 * (int64_t)v] +
                               B.g_lin[2 * (int64_t)v + 1] * (double)Xr[2 * (int64_t)v + 1]);
            }
        }
    const double E = block_sum(e, sh);
    if (threadIdx.x == 0) {
        vtx_relax_result r;
        r.iters = st.iter;
        r.n_t1 = st.n_t1;
        r.n_stretch = st.n_st;
        r.max_f = st.last_mf;
        r.energy = E;
        r.status = st.status;
        res[idx] = r;
    }
}

// LDS bytes of a batched relaxation without T1 held in LDS: both position
// buffers, the cell coefficients and the corner rows.
template <typename PosT, typename M>
__host__ __device__ inline int64_t relax_lds_bytes(int64_t n_vert, int64_t n_cell,
                                                   int64_t n_he) {
    auto a16 = [](int64_t b) { return (b + 15) & ~(int64_t)15; };
    return 2 * a16(2 * n_vert * (int64_t)sizeof(PosT)) + a16(2 * n_cell * (int64_t)sizeof(M)) +
           a16(4 * n_he);
}

// Cells (and twice as many vertices) per thread of k_batch_relax_lds.
constexpr int kRelaxLdsK = 2;
constexpr int kRelaxLdsThreads = 512;
static_assert(kRelaxLdsThreads <= 512, "block_allsum2 holds the sums of eight waves");

// Batched relaxation of tissues of at most two cells and four vertices per
// thread of a 512-thread workgroup whose two position buffers, cell
// coefficients and corner rows fit in LDS.  Thread i owns cells i + 512 k
// and vertices i + 512 j; their corner rows go to LDS and their star
// entries, tensions, cell parameters and nudge targets to registers, so an
// iteration reads only LDS.  With T1 (the T1 template flag) the cell pass
// also flags short edges, the pass runs on the LDS positions and
// coefficients, and the rows and stars are loaded again after it (a pass
// edits them in global memory).  The cell pass, the nudge mean, the vertex
// pass with the step and the convergence control are those of k_batch_relax
// (same arithmetic; the nudge mean is summed per thread in the same vertex
// order), and the state returned is copied back into the caller's buffer.
template <typename PosT, typename M, bool T1>
__global__ __launch_bounds__(kRelaxLdsThreads) void k_batch_relax_lds(
    const BatchItem *__restrict__ items, const int32_t *__restrict__ order, int n,
    unsigned int *queue, BatchOpts o, vtx_relax_result *res) {
    constexpr int K = kRelaxLdsK, KV = 2 * kRelaxLdsK;
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    __shared__ int32_t sort_buf[T1 ? kT1SortCap : 1];
    __shared__ int32_t extra[T1 ? kT1Extra : 1];
    __shared__ int32_t scan[T1 ? kRelaxLdsThreads : 1];
    __shared__ unsigned int s_cnt;
    __shared__ double sh[16];
    __shared__ int s_item;
    __shared__ int s_scan[16];
    __shared__ RelaxState st;
    auto a16 = [](int64_t b) { return (b + 15) & ~(int64_t)15; };
    const M lmin2 = (M)(o.l_min * o.l_min * (1.0 + 1e-4));
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int slot = s_item;
        __syncthreads();
        if (slot >= n) return;
        const int idx = order[slot];
        const BatchItem &B = items[idx];
        const DevTissue &t = B.t;
        const DevParams<PosT> p = to_dev<PosT>(B.p);
        const int tid = threadIdx.x, bd = blockDim.x, nv = t.n_vert, nc = t.n_cell;
        const int64_t xb = a16(2 * (int64_t)nv * (int64_t)sizeof(PosT));
        PosT *X0 = (PosT *)lds_dyn;
        PosT *X1 = (PosT *)(lds_dyn + xb);
        M *capl = (M *)(lds_dyn + 2 * xb);
        int32_t *rowl = (int32_t *)(lds_dyn + 2 * xb + a16(2 * (int64_t)nc * (int64_t)sizeof(M)));
        for (int k = tid; k < 2 * nv; k += bd) X0[k] = ((const PosT *)B.X)[k];
        // the thread's cells, by side count (kept across T1 passes, which
        // change a few cells' counts by one); X1 is free until the first step
        // and its 2 n_vert positions hold the n_cell <= n_vert ints
        int cid[K];
        cells_by_sides<K>(t, reinterpret_cast<int *>(X1), s_scan, cid);
        int cn[K], lrb[K], grb[K];
        PosT ka[K], a0[K], kp[K], p0[K];
        int32_t sw[KV][3], sc[KV][3];
        PosT sl[KV][3];
        // the topology a step reads: rows into LDS, stars and tensions into
        // registers (again after every T1 pass)
        auto load_topology = [&]() {
            int rows_base = 0;
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const int c = cid[i];
                grb[i] = 0;
                cn[i] = 0;
                if (c >= 0) {
                    grb[i] = t.row_ptr[c];
                    cn[i] = t.nsides[c];
                }
                int tot;
                lrb[i] = rows_base + block_exclusive_scan(cn[i], s_scan, tot);
                rows_base += tot;
                const int nk = min(cn[i], t.n_he - lrb[i]);  // the rows hold n_he corners
                for (int k = 0; k < nk; ++k) rowl[lrb[i] + k] = t.corner[grb[i] + k];
            }
#pragma unroll
            for (int j = 0; j < KV; ++j) {
                const int v = tid + j * bd;
                if (v < nv) {
                    const int4 a = reinterpret_cast<const int4 *>(t.star)[v];
                    const int4 b = reinterpret_cast<const int4 *>(t.star + 4 * (int64_t)nv)[v];
                    const int32_t e[3] = {b.z, b.w, t.star[8 * (int64_t)nv + v]};
                    sw[j][0] = a.x;
                    sw[j][1] = a.y;
                    sw[j][2] = a.z;
                    sc[j][0] = a.w;
                    sc[j][1] = b.x;
                    sc[j][2] = b.y;
#pragma unroll
                    for (int k = 0; k < 3; ++k) sl[j][k] = p.lam ? p.lam[e[k]] : p.lam_s;
                }
            }
        };
        load_topology();
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int c = cid[i];
            ka[i] = a0[i] = kp[i] = p0[i] = 0;
            if (c >= 0) {
                ka[i] = p.ka(c);
                a0[i] = p.a0(c);
                kp[i] = p.kp(c);
                p0[i] = p.p0(c);
            }
        }
        // a nudge (EP) never comes with T1: the T1 forms compile it out
        const bool nudged = !T1 && B.beta != 0.0;
        double nt[KV][2];  // nudge target (v2v) or linear cost gradient
#pragma unroll
        for (int j = 0; j < KV; ++j) {
            const int v = tid + j * bd;
            nt[j][0] = nt[j][1] = 0.0;
            if (v < nv && nudged) {
                if (B.Xt) {
                    const PosT *Xt = (const PosT *)B.Xt;
                    nt[j][0] = (double)Xt[2 * (int64_t)v];
                    nt[j][1] = (double)Xt[2 * (int64_t)v + 1];
                } else {
                    nt[j][0] = B.g_lin[2 * (int64_t)v];
                    nt[j][1] = B.g_lin[2 * (int64_t)v + 1];
                }
            }
        }
        if (tid == 0) st = RelaxState{0, 0, 0, 0, 0.0, VTX_NOT_CONVERGED, 0, 0, 0, 0};
        __syncthreads();
        const double inv_n = 1.0 / (double)nv;
        // gradient of the nudge cost at own vertex j (as nudge_grad)
        // (min_image returns d itself for |d| <= L/4: d/L rounds into
        // [-1/4, 1/4], so the floor is +0; such d skip its division)
        auto near_image = [](double d, double L) {
            return fabs(d) <= 0.25 * L ? d : min_image(d, L);
        };
        auto nudge = [&](int j, const PosT *Xc, int v, double &cx, double &cy) {
            if (B.Xt) {
                cx = near_image((double)Xc[2 * v] - nt[j][0], t.Lx) * inv_n;
                cy = near_image((double)Xc[2 * v + 1] - nt[j][1], t.Ly) * inv_n;
            } else {
                cx = nt[j][0];
                cy = nt[j][1];
            }
        };
        const PosT lmin2p = (PosT)lmin2;
        int cur = 0;
        for (;;) {
            PosT *Xc = cur ? X1 : X0;
            PosT *Xn = cur ? X0 : X1;
            if (T1) {
                if (tid == 0) s_cnt = 0u;
                __syncthreads();
            }
            // cell pass
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const int c = cid[i];
                const int base = lrb[i];
                if (c >= 0) {
                    PosT A, P;
                    cell_geom<PosT, PosT>(
                        t, Xc, cn[i], [&](int k) { return rowl[base + k]; }, grb[i], A, P,
                        T1 && o.t1_enable != 0, lmin2p, B.t1_list, &s_cnt);
                    st2(capl, c, (M)((PosT)2 * ka[i] * (A - a0[i])),
                        (M)((PosT)2 * kp[i] * (P - p0[i])));
                }
            }
            __syncthreads();
            if (T1) {
                const int ncand = (int)s_cnt;
                if (ncand > 0) {
                    const int64_t swaps0 = st.n_t1;
                    batch_t1_pass_lds<PosT, M>(&B, Xc, capl, ncand, o.l_min, o.l_new, sort_buf,
                                               extra, scan, &st);
                    // rows and stars change only with an exchange; a pass of
                    // stretches alone moves positions and rewrites cell
                    // coefficients, both in LDS already
                    if (st.n_t1 != swaps0) load_topology();
                    __syncthreads();
                }
            }
            // nudge gradient at the own vertices (kept for the vertex pass)
            // and its mean over the vertices
            double mx = 0.0, my = 0.0, ncx[KV], ncy[KV];
#pragma unroll
            for (int j = 0; j < KV; ++j) ncx[j] = ncy[j] = 0.0;
            if (nudged) {
                double sx = 0.0, sy = 0.0;
#pragma unroll
                for (int j = 0; j < KV; ++j) {
                    const int v = tid + j * bd;
                    if (v < nv) {
                        nudge(j, Xc, v, ncx[j], ncy[j]);
                        sx += ncx[j];
                        sy += ncy[j];
                    }
                }
                const double2 s2 = block_allsum2(sx, sy, sh);
                mx = s2.x * inv_n;
                my = s2.y * inv_n;
            }
            // vertex pass with the step
            double mf = 0.0;
#pragma unroll
            for (int j = 0; j < KV; ++j) {
                const int v = tid + j * bd;
                if (v < nv) {
                    StarLoad<PosT, M> L;
                    L.pi = ld2(Xc, v);
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        L.w[k] = sw[j][k];
                        L.c[k] = sc[j][k];
                        L.lam[k] = sl[j][k];
                        L.q[k] = ld2(Xc, id_of(L.w[k]));
                        L.cc[k] = ld2(capl, L.c[k]);
                    }
                    Star<PosT, M> s;
                    PosT xi, yi;
                    star_math<PosT, M>(t, L, s, xi, yi);
                    M fx, fy;
                    star_force<PosT, M>(s, fx, fy);
                    double gx = fx, gy = fy;
                    if (nudged) {
                        gx -= B.beta * (ncx[j] - mx);
                        gy -= B.beta * (ncy[j] - my);
                    }
                    mf = fmax(mf, fmax(fabs(gx), fabs(gy)));
                    if (!(gx == gx) || !(gy == gy)) mf = INFINITY;
                    st2(Xn, v, (PosT)((double)xi + o.eta * gx), (PosT)((double)yi + o.eta * gy));
                }
            }
            const double m = block_max(mf, sh);
            if (tid == 0) {
                st.iter += 1;
                st.last_mf = m;
                if (st.bad_t1) {
                    st.done = 1;
                    st.status = VTX_E_CAPACITY;
                    st.result_buf = cur;
                } else if (!(m <= 1.7976931348623157e308)) {
                    st.done = 1;
                    st.status = VTX_E_NONFINITE;
                    st.result_buf = cur;
                } else {
                    st.count = m < o.tol ? st.count + 1 : 0;
                    if (st.count >= o.patience) {
                        st.done = 1;
                        st.status = VTX_CONVERGED;
                        st.result_buf = cur;
                    } else if (st.iter >= o.max_iter) {
                        st.done = 1;
                        st.status = VTX_NOT_CONVERGED;
                        st.result_buf = cur ^ 1;
                    }
                }
            }
            __syncthreads();
            if (st.done) break;
            cur ^= 1;
        }
        const PosT *Xr = st.result_buf ? X1 : X0;
        for (int k = tid; k < 2 * nv; k += bd) ((PosT *)B.X)[k] = Xr[k];
        __syncthreads();
        batch_relax_result<PosT>(B, t, p, st, sh, res, idx);
        __syncthreads();
    }
}

// Persistent batched relaxation (Methods, "Simulation engine", per tissue):
// each workgroup takes tissues from a device queue (largest first) and runs
// the whole gradient-descent loop of one tissue with workgroup barriers
// only.  An iteration is the cell pass (coefficients, short-edge flags), the
// T1 pass if any edge was flagged, the mean of the nudge gradient (EP), the
// vertex pass with the step into the other position buffer, and the
// convergence control; the arithmetic and the order of every step equal
// those of the single-tissue kernels, so results are bit-identical to
// vtx_relax.  The returned state is copied back into the caller's buffer.
template <typename PosT, typename M>
__global__ __launch_bounds__(1024) void k_batch_relax(const BatchItem *__restrict__ items,
                                                      const int32_t *__restrict__ order, int n,
                                                      unsigned int *queue, BatchOpts o,
                                                      vtx_relax_result *res) {
    __shared__ int32_t sort_buf[kT1SortCap];
    __shared__ int32_t extra[kT1Extra];
    __shared__ int32_t scan[1024];
    __shared__ double sh[16];
    __shared__ unsigned int s_cnt;
    __shared__ int s_item;
    __shared__ RelaxState st;
    __shared__ double s_mean[2];
    const M lmin2 = (M)(o.l_min * o.l_min * (1.0 + 1e-4));
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int slot = s_item;
        __syncthreads();
        if (slot >= n) return;
        const int idx = order[slot];
        const BatchItem &B = items[idx];
        const DevTissue &t = B.t;
        const DevParams<PosT> p = to_dev<PosT>(B.p);
        M *cap = (M *)B.cap;
        int cur = 0;
        if (threadIdx.x == 0) st = RelaxState{0, 0, 0, 0, 0.0, VTX_NOT_CONVERGED, 0, 0, 0, 0};
        for (;;) {
            // buffer selector and threshold as wave-uniform values (scalar
            // registers), so they need no vector register across the T1 call
            const int cu = __builtin_amdgcn_readfirstlane(cur);
            PosT *Xc = (PosT *)(cu ? B.xbuf : B.X), *Xn = (PosT *)(cu ? B.X : B.xbuf);
            const PosT lmin2p = (PosT)first_lane_f64((double)(PosT)lmin2);
            if (threadIdx.x == 0) s_cnt = 0u;
            __syncthreads();
            // cell pass
            for (int c = threadIdx.x; c < t.n_cell; c += blockDim.x) {
                const int rb = t.row_ptr[c], nn = t.nsides[c];
                PosT A, P;  // in the position precision, as in the grid kernels
                cell_geom<PosT, PosT>(
                    t, Xc, nn, [&](int k) { return t.corner[rb + k]; }, rb, A, P,
                    o.t1_enable != 0, lmin2p, B.t1_list, &s_cnt);
                st2(cap, c, (M)((PosT)2 * p.ka(c) * (A - p.a0(c))),
                    (M)((PosT)2 * p.kp(c) * (P - p.p0(c))));
            }
            __syncthreads();
            // T1 pass
            const int ncand = (int)s_cnt;
            if (ncand > 0)
                batch_t1_pass<PosT, M>(&B, Xc, ncand, o.l_min, o.l_new, sort_buf, extra, scan,
                                       &st);
            // mean of the nudge gradient over the vertices
            const double inv_n = 1.0 / (double)t.n_vert;
            double mx = 0.0, my = 0.0;
            if (B.beta != 0.0) {
                double sx = 0.0, sy = 0.0;
                for (int v = threadIdx.x; v < t.n_vert; v += blockDim.x) {
                    double cx, cy;
                    nudge_grad<PosT>(B, Xc, v, inv_n, cx, cy);
                    sx += cx;
                    sy += cy;
                }
                const double bx = block_sum(sx, sh);
                const double by = block_sum(sy, sh);
                if (threadIdx.x == 0) {
                    s_mean[0] = bx * inv_n;
                    s_mean[1] = by * inv_n;
                }
                __syncthreads();
                mx = s_mean[0];
                my = s_mean[1];
            }
            // vertex pass with the step
            double mf = 0.0;
            for (int v = threadIdx.x; v < t.n_vert; v += blockDim.x) {
                Star<PosT, M> s;
                PosT xi, yi;
                load_star<PosT, M>(t, Xc, p, cap, v, s, xi, yi);
                M fx, fy;
                star_force<PosT, M>(s, fx, fy);
                double gx = fx, gy = fy;
                if (B.beta != 0.0) {
                    double cx, cy;
                    nudge_grad<PosT>(B, Xc, v, inv_n, cx, cy);
                    gx -= B.beta * (cx - mx);
                    gy -= B.beta * (cy - my);
                }
                mf = fmax(mf, fmax(fabs(gx), fabs(gy)));
                if (!(gx == gx) || !(gy == gy)) mf = INFINITY;
                st2(Xn, v, (PosT)((double)xi + o.eta * gx), (PosT)((double)yi + o.eta * gy));
            }
            const double m = block_max(mf, sh);
            if (threadIdx.x == 0) {
                st.iter += 1;
                st.last_mf = m;
                if (st.bad_t1) {
                    st.done = 1;
                    st.status = VTX_E_CAPACITY;
                    st.result_buf = cur;
                } else if (!(m <= 1.7976931348623157e308)) {
                    st.done = 1;
                    st.status = VTX_E_NONFINITE;
                    st.result_buf = cur;
                } else {
                    st.count = m < o.tol ? st.count + 1 : 0;
                    if (st.count >= o.patience) {
                        st.done = 1;
                        st.status = VTX_CONVERGED;
                        st.result_buf = cur;
                    } else if (st.iter >= o.max_iter) {
                        st.done = 1;
                        st.status = VTX_NOT_CONVERGED;
                        st.result_buf = cur ^ 1;
                    }
                }
            }
            __syncthreads();
            if (st.done) break;
            cur ^= 1;
        }
        const int rbuf = st.result_buf;
        if (rbuf == 1)
            for (int k = threadIdx.x; k < 2 * t.n_vert; k += blockDim.x)
                ((PosT *)B.X)[k] = ((PosT *)B.xbuf)[k];
        __syncthreads();
        batch_relax_result<PosT>(B, t, p, st, sh, res, idx);
        __syncthreads();
    }
}

}  // namespace vtx

namespace {

bool mode_ok(int m) { return m == VTX_F32 || m == VTX_F64 || m == VTX_MIXED; }

ParamsRaw raw_params(const vtx_params &q) {
    return ParamsRaw{q.KA, q.A0, q.KP, q.P0, q.lam, q.KA_s, q.A0_s, q.KP_s, q.P0_s, q.lam_s};
}

int hip_fail(hipError_t e) { return set_error(VTX_E_HIP, hipGetErrorString(e)); }

// Capture (queue reset + one persistent launch) as a graph and run it.
template <typename Launch>
int run_graph(vtx_batch b, hipStream_t s, Launch launch) {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e);
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(1), 0, b->cap_stream, b->queue);
    launch(b->cap_stream);
    e = hipStreamEndCapture(b->cap_stream, &g);
    if (e != hipSuccess) return hip_fail(e);
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(ge, s);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    return e == hipSuccess ? VTX_OK : hip_fail(e);
}

// Launch of the batched adjoint with the dynamic LDS the largest tissue that
// fits needs (tissues beyond the device's per-workgroup LDS keep their
// arrays in global memory).  Workgroups of up to 512 threads run the kernel
// that has the register-resident CG.
template <typename PosT, typename M, int MAXT>
int launch_batch_cg_t(vtx_batch b, const GradItem *gi, const int32_t *order, int n,
                      const GradOpts &go, int block_threads, hipStream_t s) {
    constexpr int K = kFastK<MAXT>;
    int dev = 0, lds_max = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return hip_fail(e);
    const int64_t budget = (int64_t)lds_max - 1024;  // the kernel's static LDS stays below
    int64_t need = 0;
    for (size_t i = 0; i < b->ts.size(); ++i) {
        const DevTissue &d = tissue_dev(b->ts[i]);
        int64_t nb = cg_lds_bytes<PosT, M>(d.n_vert, d.n_cell);
        if (K > 0 && !go.minres &&
            cg_fast_fits<PosT, M, (K > 0 ? K : 1)>(d.n_vert, d.n_cell, d.n_he, block_threads,
                                                   budget))
            nb = cg_fast_lds_bytes<PosT, M>(d.n_vert, d.n_cell, d.n_he);
        if (nb <= budget && nb > need) need = nb;
    }
    const int lds = (int)need;
    if (lds > 0) {
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch_cg<PosT, M, MAXT>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return hip_fail(e);
    }
    return run_graph(b, s, [&](hipStream_t cs) {
        hipLaunchKernelGGL((k_batch_cg<PosT, M, MAXT>), dim3(n), dim3(block_threads),
                           (size_t)lds, cs, gi, order, n, b->queue, go, b->gres_d, lds);
    });
}

// Workgroup size of the batched adjoint when the caller leaves it open: 512
// threads when every tissue takes the register-resident CG there (measured
// faster on 10^3-cell tissues: 11.9 against 15.5 ms for 64), else 1024.
template <typename PosT, typename M>
int auto_cg_threads(vtx_batch b, const GradOpts &go, int *out) {
    int dev = 0, lds_max = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return hip_fail(e);
    bool all = !go.minres;
    for (size_t i = 0; all && i < b->ts.size(); ++i) {
        const DevTissue &d = tissue_dev(b->ts[i]);
        all = cg_fast_fits<PosT, M, kFastK<512>>(d.n_vert, d.n_cell, d.n_he, 512,
                                                 (int64_t)lds_max - 1024);
    }
    *out = all ? 512 : 1024;
    return VTX_OK;
}

template <typename PosT, typename M>
int launch_batch_cg(vtx_batch b, const GradItem *gi, const int32_t *order, int n,
                    const GradOpts &go, int block_threads, hipStream_t s) {
    if (block_threads == 0) {
        const int rc = auto_cg_threads<PosT, M>(b, go, &block_threads);
        if (rc) return rc;
    }
    return block_threads <= 512
               ? launch_batch_cg_t<PosT, M, 512>(b, gi, order, n, go, block_threads, s)
               : launch_batch_cg_t<PosT, M, 1024>(b, gi, order, n, go, block_threads, s);
}

// Plan of the multi-workgroup adjoint (FP64 CG): K parts per tissue and the
// number of groups of the cooperative launch.  block_threads < 0 asks for
// K = -block_threads; 0 lets the library choose: the largest K (up to 8)
// that still gives every tissue its own group on the device at once, with
// at least 200 vertices per part, and enough parts that no part owns more
// than 1024 vertices.  *K = 0 when the plan does not apply.
int plan_mb(vtx_batch b, int block_threads, int *K, int *n_groups, int *lds) {
    *K = 0;
    int max_blocks = 0;
    hipError_t e = mb_capacity(&max_blocks, lds);
    if (e != hipSuccess) return hip_fail(e);
    const int n = (int)b->ts.size();
    int64_t nv_min = INT64_MAX, nv_max = 0;
    for (int i = 0; i < n; ++i) {
        nv_min = std::min(nv_min, tissue_size(b->ts[i]));
        nv_max = std::max(nv_max, tissue_size(b->ts[i]));
    }
    int k = 1;
    if (block_threads < 0) {
        k = -block_threads;
        if (max_blocks < k)
            return set_error(VTX_E_ARG, "the device cannot launch the multi-workgroup adjoint "
                                        "cooperatively");
    } else {
        while (k < 8 && (int64_t)n * 2 * k <= max_blocks && nv_min / (2 * k) >= 200) k *= 2;
        while (k < 8 && nv_max > 1024 * (int64_t)k && 2 * k <= max_blocks) k *= 2;
        if (k < 2) return VTX_OK;
    }
    int g = std::min(n, max_blocks / k);
    if (g >= 8) g -= g % 8;   // parts of a group then share an XCD (round-robin dispatch)
    *K = k;
    *n_groups = g;
    return VTX_OK;
}

// Dynamic LDS for k_batch_relax_lds if every tissue of the batch fits it
// (*lds > 0), else *lds = 0.
template <typename PosT, typename M, bool T1>
int relax_lds_plan(vtx_batch b, int *lds) {
    *lds = 0;
    int dev = 0, lds_max = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    hipFuncAttributes fa{};
    if (e == hipSuccess)
        e = hipFuncGetAttributes(&fa,
                                 reinterpret_cast<const void *>(&k_batch_relax_lds<PosT, M, T1>));
    if (e != hipSuccess) return hip_fail(e);
    const int64_t budget = (int64_t)lds_max - (int64_t)fa.sharedSizeBytes;
    int64_t need = 0;
    for (size_t i = 0; i < b->ts.size(); ++i) {
        const DevTissue &d = tissue_dev(b->ts[i]);
        const int64_t nb = relax_lds_bytes<PosT, M>(d.n_vert, d.n_cell, d.n_he);
        if (d.n_cell > (int64_t)kRelaxLdsK * kRelaxLdsThreads ||
            d.n_vert > 2 * (int64_t)kRelaxLdsK * kRelaxLdsThreads || nb > budget)
            return VTX_OK;
        need = nb > need ? nb : need;
    }
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch_relax_lds<PosT, M, T1>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
    if (e != hipSuccess) return hip_fail(e);
    *lds = (int)need;
    return VTX_OK;
}

// The split schedule: each tissue over K cooperating workgroups
// (k_batch_relax_mb, T1 off); tissues a part cannot hold are relaxed again
// by the general persistent kernel.  Results to b->res_d.
int relax_split(vtx_batch b, int mode, const BatchItem *it, const BatchOpts &bo, int n, int K,
                hipStream_t s) {
    int max_blocks = 0, lds = 0;
    hipError_t e = mb_relax_capacity(mode, &max_blocks, &lds);
    if (e != hipSuccess) return hip_fail(e);
    if (max_blocks < K)
        return set_error(VTX_E_ARG, "the device cannot launch the split schedule cooperatively");
    int g = std::min(n, max_blocks / K);
    if (g >= 8) g -= g % 8;   // parts of a group then share an XCD (round-robin dispatch)
    // a tissue whose result is never written keeps status -1 (an error)
    e = hipMemsetAsync(b->res_d, 0xff, sizeof(vtx_relax_result) * n, s);
    if (e == hipSuccess)
        e = mb_relax_launch(mode, it, b->order_d, n, bo, K, g, lds, b->res_d, b->mb_groups, s);
    std::vector<vtx_relax_result> r(n);
    if (e == hipSuccess)
        e = hipMemcpyAsync(r.data(), b->res_d, sizeof(vtx_relax_result) * n, hipMemcpyDeviceToHost,
                           s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    std::vector<int32_t> rest;
    for (int i = 0; i < n; ++i) {
        if (r[i].status == mb_no_fit_status()) rest.push_back(i);
        else if (r[i].status != VTX_CONVERGED && r[i].status != VTX_NOT_CONVERGED &&
                 r[i].status != VTX_E_NONFINITE)
            return set_error(VTX_E_HIP, "split relaxation: a wait between the workgroups of a "
                                        "tissue timed out");
    }
    if (rest.empty()) return VTX_OK;
    e = hipMemcpyAsync(b->order2_d, rest.data(), sizeof(int32_t) * rest.size(),
                       hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e);
    const int m = (int)rest.size();
    return run_graph(b, s, [&](hipStream_t cs) {
        if (mode == VTX_F32)
            hipLaunchKernelGGL((k_batch_relax<float, float>), dim3(m), dim3(1024), 0, cs, it,
                               b->order2_d, m, b->queue, bo, b->res_d);
        else if (mode == VTX_F64)
            hipLaunchKernelGGL((k_batch_relax<double, double>), dim3(m), dim3(1024), 0, cs, it,
                               b->order2_d, m, b->queue, bo, b->res_d);
        else
            hipLaunchKernelGGL((k_batch_relax<double, float>), dim3(m), dim3(1024), 0, cs, it,
                               b->order2_d, m, b->queue, bo, b->res_d);
    });
}

// The batch's items for positions X (nudge beta towards Xt, or along g_lin)
// into items[0, n).
int make_items(vtx_batch b, void *const *X, const vtx_params *p, const void *const *Xt,
               const double *const *g_lin, double beta, BatchItem *items) {
    const int n = (int)b->ts.size();
    for (int i = 0; i < n; ++i) {
        if (!X[i]) return set_error(VTX_E_ARG, "null X in batch");
        const Workspace &w = tissue_ws(b->ts[i]);
        BatchItem &it = items[i];
        it.t = tissue_dev(b->ts[i]);
        it.X = X[i];
        it.xbuf = w.xbuf;
        it.cap = w.cap;
        it.t1_list = w.t1_list;
        it.p = raw_params(p[i]);
        it.Xt = Xt ? Xt[i] : nullptr;
        it.g_lin = g_lin ? g_lin[i] : nullptr;
        it.beta = beta;
        if (beta != 0.0 && !it.Xt && !it.g_lin) return set_error(VTX_E_ARG, "nudge without a cost");
    }
    return VTX_OK;
}

// As vtx_relax: a failed tissue reports NOT_CONVERGED and the call returns
// the error of the first failed tissue, naming it.
int relax_statuses(vtx_relax_result *res, int n) {
    int err = VTX_OK, first = -1;
    for (int i = 0; i < n; ++i) {
        if (res[i].status == VTX_E_NONFINITE || res[i].status == VTX_E_CAPACITY) {
            if (first < 0) {
                first = i;
                err = res[i].status;
            }
            res[i].status = VTX_NOT_CONVERGED;
        }
    }
    if (first < 0) return VTX_OK;
    const std::string what = err == VTX_E_NONFINITE ? "non-finite forces" : "T1 pass overflow";
    const std::string msg = what + " in batched relaxation of tissue " + std::to_string(first);
    return set_error(err, msg.c_str());
}

int batch_relax_run(vtx_batch b, int mode, void *const *X, const vtx_params *p,
                    const vtx_relax_opts *o, const void *const *Xt, const double *const *g_lin,
                    double beta, int block_threads, vtx_relax_result *res, hipStream_t s,
                    int split_K = 0) {
    const int n = (int)b->ts.size();
    std::vector<BatchItem> items(n);
    int rc0 = make_items(b, X, p, Xt, g_lin, beta, items.data());
    if (rc0) return rc0;
    hipError_t e = hipMemcpyAsync(b->items, items.data(), sizeof(BatchItem) * n,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e);
    BatchOpts bo{o->eta, o->tol, o->l_min, o->l_new, o->patience, o->max_iter, o->t1_enable};
    const BatchItem *it = (const BatchItem *)b->items;
    // A batch whose every tissue fits k_batch_relax_lds runs there when the
    // caller asked for its workgroup size or left the choice open.
    int lds = 0;
    const bool t1 = o->t1_enable != 0;
    if (split_K > 0 && t1) return set_error(VTX_E_ARG, "the split schedule runs without T1");
    if (split_K > 0) {
        const int rc = relax_split(b, mode, it, bo, n, split_K, s);
        if (rc) return rc;
    } else if (block_threads == 0 || block_threads == kRelaxLdsThreads) {
        int rc;
        if (mode == VTX_F32)
            rc = t1 ? relax_lds_plan<float, float, true>(b, &lds)
                    : relax_lds_plan<float, float, false>(b, &lds);
        else if (mode == VTX_F64)
            rc = t1 ? relax_lds_plan<double, double, true>(b, &lds)
                    : relax_lds_plan<double, double, false>(b, &lds);
        else
            rc = t1 ? relax_lds_plan<double, float, true>(b, &lds)
                    : relax_lds_plan<double, float, false>(b, &lds);
        if (rc) return rc;
    }
    if (block_threads == 0) block_threads = 1024;
    auto launch_lds = [&](auto kern, hipStream_t cs) {
        hipLaunchKernelGGL(kern, dim3(n), dim3(kRelaxLdsThreads), (size_t)lds, cs, it, b->order_d,
                           n, b->queue, bo, b->res_d);
    };
    int rc = split_K > 0 ? VTX_OK : run_graph(b, s, [&](hipStream_t cs) {
        const dim3 grid(n), block(block_threads);
        if (lds > 0) {
            if (mode == VTX_F32)
                t1 ? launch_lds(k_batch_relax_lds<float, float, true>, cs)
                   : launch_lds(k_batch_relax_lds<float, float, false>, cs);
            else if (mode == VTX_F64)
                t1 ? launch_lds(k_batch_relax_lds<double, double, true>, cs)
                   : launch_lds(k_batch_relax_lds<double, double, false>, cs);
            else
                t1 ? launch_lds(k_batch_relax_lds<double, float, true>, cs)
                   : launch_lds(k_batch_relax_lds<double, float, false>, cs);
        } else if (mode == VTX_F32)
            hipLaunchKernelGGL((k_batch_relax<float, float>), grid, block, 0, cs, it, b->order_d,
                               n, b->queue, bo, b->res_d);
        else if (mode == VTX_F64)
            hipLaunchKernelGGL((k_batch_relax<double, double>), grid, block, 0, cs, it,
                               b->order_d, n, b->queue, bo, b->res_d);
        else
            hipLaunchKernelGGL((k_batch_relax<double, float>), grid, block, 0, cs, it, b->order_d,
                               n, b->queue, bo, b->res_d);
    });
    if (t1)
        for (int i = 0; i < n; ++i) {
            const int rt = tissue_topology_changed(b->ts[i], s);
            if (!rc) rc = rt;
        }
    if (rc) return rc;
    e = hipMemcpyAsync(res, b->res_d, sizeof(vtx_relax_result) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    return relax_statuses(res, n);
}

constexpr int kPlanDoesNotApply = 1;

// Centred EP's two nudged relaxations (+beta and -beta about X*, from Xp
// and Xm) as one launch of 2n items when every tissue takes the
// LDS-resident kernel: there the two items of a tissue share no global
// scratch (positions and coefficients live in LDS; no T1), so each runs
// exactly as it would alone and the 2n run side by side.  Returns
// kPlanDoesNotApply, having launched nothing, otherwise.
int batch_relax_pm(vtx_batch b, int mode, void *const *Xp, void *const *Xm, const vtx_params *p,
                   const vtx_relax_opts *o, const void *const *Xt, const double *const *g_lin,
                   double beta, int block_threads, vtx_relax_result *rp, vtx_relax_result *rm,
                   hipStream_t s) {
    if (o->t1_enable || (block_threads != 0 && block_threads != kRelaxLdsThreads))
        return kPlanDoesNotApply;
    int lds = 0, rc;
    if (mode == VTX_F32) rc = relax_lds_plan<float, float, false>(b, &lds);
    else if (mode == VTX_F64) rc = relax_lds_plan<double, double, false>(b, &lds);
    else rc = relax_lds_plan<double, float, false>(b, &lds);
    if (rc) return rc;
    if (lds == 0) return kPlanDoesNotApply;
    const int n = (int)b->ts.size();
    std::vector<BatchItem> items(2 * (size_t)n);
    if ((rc = make_items(b, Xp, p, Xt, g_lin, beta, items.data()))) return rc;
    if ((rc = make_items(b, Xm, p, Xt, g_lin, -beta, items.data() + n))) return rc;
    hipError_t e = hipMemcpyAsync(b->items, items.data(), sizeof(BatchItem) * 2 * n,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e);
    const BatchOpts bo{o->eta, o->tol, o->l_min, o->l_new, o->patience, o->max_iter, 0};
    const BatchItem *it = (const BatchItem *)b->items;
    auto launch = [&](auto kern, hipStream_t cs) {
        hipLaunchKernelGGL(kern, dim3(2 * n), dim3(kRelaxLdsThreads), (size_t)lds, cs, it,
                           b->order_d, 2 * n, b->queue, bo, b->res_d);
    };
    rc = run_graph(b, s, [&](hipStream_t cs) {
        if (mode == VTX_F32) launch(k_batch_relax_lds<float, float, false>, cs);
        else if (mode == VTX_F64) launch(k_batch_relax_lds<double, double, false>, cs);
        else launch(k_batch_relax_lds<double, float, false>, cs);
    });
    if (rc) return rc;
    std::vector<vtx_relax_result> r(2 * (size_t)n);
    e = hipMemcpyAsync(r.data(), b->res_d, sizeof(vtx_relax_result) * 2 * n,
                       hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    std::copy(r.begin(), r.begin() + n, rp);
    std::copy(r.begin() + n, r.end(), rm);
    if ((rc = relax_statuses(rp, n))) return rc;
    return relax_statuses(rm, n);
}

// Parts per tissue of the split schedule when the caller leaves it open:
// the largest K (up to 8) with at most 64 workgroups in all (a barrier of
// more concurrent workgroups costs several microseconds on this part:
// their device-scope fences serialise per XCD) and at least 200 vertices
// per part.
int split_parts(vtx_batch b) {
    const int n = (int)b->ts.size();
    int64_t nv_min = INT64_MAX;
    for (int i = 0; i < n; ++i) nv_min = std::min(nv_min, tissue_size(b->ts[i]));
    int k = 1;
    while (k < 8 && (int64_t)n * 2 * k <= 64 && nv_min / (2 * k) >= 200) k *= 2;
    return k;
}

int check_relax_opts(const vtx_relax_opts *o) {
    if (!(o->eta > 0) || !(o->tol >= 0) || o->patience < 1 || o->max_iter < 1)
        return set_error(VTX_E_ARG, "bad relax options");
    if (o->t1_enable && !(o->l_min > 0 && o->l_new > 0))
        return set_error(VTX_E_ARG, "T1 needs l_min > 0 and l_new > 0");
    return VTX_OK;
}

}  // namespace

extern "C" {

int vtx_batch_create(const vtx_tissue *ts, int32_t n, vtx_batch *out) {
    if (!ts || n <= 0 || !out) return set_error(VTX_E_ARG, "bad batch arguments");
    for (int i = 0; i < n; ++i)
        if (!ts[i]) return set_error(VTX_E_ARG, "null tissue in batch");
    vtx_batch b = new vtx_batch_s();
    b->ts.assign(ts, ts + n);
    b->order.resize(n);
    for (int i = 0; i < n; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) {
        return tissue_size(b->ts[a]) > tissue_size(b->ts[c]);
    });
    std::vector<int32_t> order2(2 * (size_t)n);  // order, then the same + n
    for (int i = 0; i < n; ++i) {
        order2[i] = b->order[i];
        order2[n + i] = b->order[i] + n;
    }
    hipError_t e = hipMalloc(&b->items, sizeof(BatchItem) * 2 * n);
    if (e == hipSuccess) e = hipMalloc(&b->gitems, sizeof(GradItem) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&b->xm_list, sizeof(void *) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&b->order_d, sizeof(int32_t) * 2 * n);
    if (e == hipSuccess) e = hipMalloc((void **)&b->queue, sizeof(unsigned int));
    if (e == hipSuccess) e = hipMalloc((void **)&b->res_d, sizeof(vtx_relax_result) * 2 * n);
    if (e == hipSuccess) e = hipMalloc((void **)&b->gres_d, sizeof(vtx_grad_result) * n);
    if (e == hipSuccess) e = hipMalloc(&b->mb_groups, mb_group_bytes() * n);
    if (e == hipSuccess) e = hipMalloc((void **)&b->order2_d, sizeof(int32_t) * n);
    if (e == hipSuccess)
        e = hipMemcpy(b->order_d, order2.data(), sizeof(int32_t) * 2 * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        vtx_batch_destroy(b);
        return hip_fail(e);
    }
    *out = b;
    return VTX_OK;
}

int vtx_batch_destroy(vtx_batch b) {
    if (!b) return set_error(VTX_E_ARG, "null batch");
    (void)hipDeviceSynchronize();
    void *ptrs[] = {b->items, b->gitems, b->xm_list, b->order_d, b->queue, b->res_d, b->gres_d,
                    b->mb_groups, b->order2_d};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return VTX_OK;
}

int vtx_batch_relax(vtx_batch b, int32_t mode, void *const *X, const vtx_params *p,
                    const vtx_relax_opts *o, int32_t schedule, int32_t block_threads,
                    vtx_relax_result *res, void *stream) {
    if (!b || !X || !p || !o || !res) return set_error(VTX_E_ARG, "null argument");
    if (!mode_ok(mode)) return set_error(VTX_E_ARG, "bad precision mode");
    if (o->beta != 0.0) return set_error(VTX_E_ARG, "batched relaxation takes no nudge");
    int rc = check_relax_opts(o);
    if (rc) return rc;
    const int n = (int)b->ts.size();
    for (int i = 0; i < n; ++i)
        if (!X[i]) return set_error(VTX_E_ARG, "null X in batch");
    if (schedule == VTX_SCHED_AUTO) {
        rc = vtx_batch_autotune(b, mode, X, p, o, 0, &schedule, &block_threads, nullptr, stream);
        if (rc) return rc;
    }
    if (schedule == VTX_SCHED_GRID) {
        for (int i = 0; i < n; ++i)
            if ((rc = vtx_relax(b->ts[i], mode, X[i], &p[i], o, &res[i], stream))) return rc;
        return VTX_OK;
    }
    if (schedule == VTX_SCHED_SPLIT) {
        if (o->t1_enable) return set_error(VTX_E_ARG, "the split schedule runs without T1");
        if (block_threads != 0 && block_threads != 1 && block_threads != 2 &&
            block_threads != 4 && block_threads != 8)
            return set_error(VTX_E_ARG, "split schedule: block_threads (parts) must be 0, 1, 2, "
                                        "4 or 8");
        const int K = block_threads ? block_threads : split_parts(b);
        return batch_relax_run(b, mode, X, p, o, nullptr, nullptr, 0.0, 0, res,
                               (hipStream_t)stream, K);
    }
    if (schedule != VTX_SCHED_PERSISTENT) return set_error(VTX_E_ARG, "unknown schedule");
    if (block_threads != 0 && block_threads != 256 && block_threads != 512 &&
        block_threads != 1024)
        return set_error(VTX_E_ARG, "block_threads must be 0, 256, 512 or 1024");
    return batch_relax_run(b, mode, X, p, o, nullptr, nullptr, 0.0, block_threads, res,
                           (hipStream_t)stream);
}

int vtx_batch_autotune(vtx_batch b, int32_t mode, void *const *X, const vtx_params *p,
                       const vtx_relax_opts *o, int32_t trial_iters, int32_t *schedule,
                       int32_t *block_threads, double *trial_ms, void *stream) {
    if (!b || !X || !p || !o || !schedule || !block_threads)
        return set_error(VTX_E_ARG, "null argument");
    if (!mode_ok(mode)) return set_error(VTX_E_ARG, "bad precision mode");
    const int n = (int)b->ts.size();
    hipStream_t s = (hipStream_t)stream;
    const int64_t iters = trial_iters > 0 ? trial_iters : 200;
    vtx_relax_opts to = *o;
    to.t1_enable = 0;
    to.tol = 0.0;
    to.patience = 1;
    to.max_iter = iters;
    to.beta = 0.0;
    to.X_target = nullptr;
    to.g_lin = nullptr;
    int rc = check_relax_opts(&to);
    if (rc) return rc;
    // trial copies of every tissue's positions
    const size_t elt = mode == VTX_F32 ? sizeof(float) : sizeof(double);
    std::vector<size_t> bytes(n);
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        if (!X[i]) return set_error(VTX_E_ARG, "null X in batch");
        bytes[i] = (size_t)tissue_size(b->ts[i]) * 2 * elt;
        total += (bytes[i] + 255) & ~(size_t)255;
    }
    char *buf = nullptr;
    hipError_t e = hipMalloc((void **)&buf, total);
    if (e != hipSuccess) return hip_fail(e);
    std::vector<void *> Xc(n);
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        Xc[i] = buf + off;
        off += (bytes[i] + 255) & ~(size_t)255;
    }
    std::vector<vtx_relax_result> res(n);
    auto reset = [&]() -> hipError_t {
        for (int i = 0; i < n; ++i) {
            const hipError_t ee = hipMemcpyAsync(Xc[i], X[i], bytes[i], hipMemcpyDeviceToDevice, s);
            if (ee != hipSuccess) return ee;
        }
        return hipStreamSynchronize(s);
    };
    auto now = []() { return std::chrono::steady_clock::now(); };
    double ms[4] = {0, 0, 0, 0};
    const int threads[3] = {256, 512, 1024};
    for (int k = 0; k < 3 && rc == VTX_OK; ++k) {
        if ((e = reset()) != hipSuccess) break;
        const auto t0 = now();
        rc = batch_relax_run(b, mode, Xc.data(), p, &to, nullptr, nullptr, 0.0, threads[k],
                             res.data(), s);
        ms[k] = std::chrono::duration<double, std::milli>(now() - t0).count();
    }
    if (rc == VTX_OK && e == hipSuccess) {
        // grid schedule: the two largest tissues, scaled to the batch
        const int m = n < 2 ? n : 2;
        double t = 0.0;
        for (int j = 0; j < m && rc == VTX_OK; ++j) {
            const int i = b->order[j];
            if ((e = reset()) != hipSuccess) break;
            const auto t0 = now();
            rc = vtx_relax(b->ts[i], mode, Xc[i], &p[i], &to, &res[i], stream);
            t += std::chrono::duration<double, std::milli>(now() - t0).count();
        }
        ms[3] = t / m * n;
    }
    // split schedule (T1 off only): 2, 4 and 8 workgroups per tissue
    double ms_split[3] = {-1.0, -1.0, -1.0};
    const int parts[3] = {2, 4, 8};
    int max_blocks = 0, lds_mb = 0;
    if (rc == VTX_OK && e == hipSuccess && !o->t1_enable)
        e = mb_relax_capacity(mode, &max_blocks, &lds_mb);
    for (int k = 0; k < 3 && rc == VTX_OK && e == hipSuccess && !o->t1_enable; ++k) {
        if (max_blocks < parts[k]) break;
        if ((e = reset()) != hipSuccess) break;
        const auto t0 = now();
        rc = batch_relax_run(b, mode, Xc.data(), p, &to, nullptr, nullptr, 0.0, 0, res.data(), s,
                             parts[k]);
        ms_split[k] = std::chrono::duration<double, std::milli>(now() - t0).count();
    }
    (void)hipFree(buf);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e);
    int best = 0;
    for (int k = 1; k < 4; ++k)
        if (ms[k] < ms[best]) best = k;
    *schedule = best == 3 ? VTX_SCHED_GRID : VTX_SCHED_PERSISTENT;
    *block_threads = best == 3 ? 0 : threads[best];
    double best_ms = ms[best];
    for (int k = 0; k < 3; ++k)
        if (ms_split[k] >= 0.0 && ms_split[k] < best_ms) {
            best_ms = ms_split[k];
            *schedule = VTX_SCHED_SPLIT;
            *block_threads = parts[k];
        }
    if (trial_ms) {
        for (int k = 0; k < 4; ++k) trial_ms[k] = ms[k];
        for (int k = 0; k < 3; ++k) trial_ms[4 + k] = ms_split[k];
    }
    return VTX_OK;
}

int vtx_batch_param_grad(vtx_batch b, int32_t mode, void *const *X_star, const vtx_params *p,
                         const double *const *dC_dX, const void *const *X_target,
                         const vtx_grad_opts *o, double *const *dC_dtheta, int32_t block_threads,
                         vtx_grad_result *res, void *stream) {
    if (!b || !X_star || !p || !o || !dC_dtheta || !res) return set_error(VTX_E_ARG, "null argument");
    if (!mode_ok(mode)) return set_error(VTX_E_ARG, "bad precision mode");
    if (o->theta != VTX_THETA_LAMBDA && o->theta != VTX_THETA_P0)
        return set_error(VTX_E_ARG, "unknown theta selector");
    if (block_threads != 0 && block_threads != 256 && block_threads != 512 &&
        block_threads != 1024 && block_threads != -1 && block_threads != -2 &&
        block_threads != -4 && block_threads != -8)
        return set_error(VTX_E_ARG, "block_threads must be 0, 256, 512, 1024 or -1, -2, -4, -8");
    if (block_threads < 0 && o->method == VTX_GRAD_ADJOINT_MINRES)
        return set_error(VTX_E_ARG, "the multi-workgroup schedule takes CG or EP");
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)b->ts.size();
    std::vector<GradItem> items(n);
    for (int i = 0; i < n; ++i) {
        if (!X_star[i] || !dC_dtheta[i]) return set_error(VTX_E_ARG, "null pointer in batch");
        const Workspace &w = tissue_ws(b->ts[i]);
        GradItem &g = items[i];
        g.t = tissue_dev(b->ts[i]);
        g.X = X_star[i];
        g.p = raw_params(p[i]);
        g.b = dC_dX ? dC_dX[i] : nullptr;
        g.cg = w.cg;
        g.cap = w.cap;
        g.aux = w.cell_aux;
        g.g = dC_dtheta[i];
    }
    hipError_t e;
    if (o->method == VTX_GRAD_ADJOINT || o->method == VTX_GRAD_ADJOINT_MINRES) {
        if (!dC_dX) return set_error(VTX_E_ARG, "the adjoint needs dC_dX");
        for (int i = 0; i < n; ++i)
            if (!dC_dX[i]) return set_error(VTX_E_ARG, "null dC_dX in batch");
        if (!(o->cg_tol > 0) || o->cg_max_iter < 1) return set_error(VTX_E_ARG, "bad CG options");
        e = hipMemcpyAsync(b->gitems, items.data(), sizeof(GradItem) * n, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e);
        GradOpts go{o->cg_tol, o->cg_max_iter, o->theta, o->method == VTX_GRAD_ADJOINT_MINRES};
        const GradItem *gi = (const GradItem *)b->gitems;
        int rc = VTX_OK;
        int K = 0, n_groups = 0, lds = 0;
        if (block_threads < 0 && (mode != VTX_F64 || go.minres))
            return set_error(VTX_E_ARG, "the multi-workgroup adjoint runs FP64 CG only");
        if (block_threads < 0 && (rc = plan_mb(b, block_threads, &K, &n_groups, &lds)))
            return rc;
        if (K > 0) {
            // a tissue whose result is never written keeps status -1 (an error)
            e = hipMemsetAsync(b->gres_d, 0xff, sizeof(vtx_grad_result) * n, s);
            if (e == hipSuccess)
                e = mb_launch(gi, b->order_d, n, go, K, n_groups, lds, b->gres_d, b->mb_groups,
                              s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(res, b->gres_d, sizeof(vtx_grad_result) * n,
                                   hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e);
            // tissues a part could not hold go to the one-workgroup kernel
            std::vector<int32_t> rest;
            for (int i = 0; i < n; ++i)
                if (res[i].status == mb_no_fit_status()) rest.push_back(i);
            if (rest.empty()) {
                for (int i = 0; i < n; ++i)
                    if (res[i].status < 0 || res[i].status > VTX_CG_MAXITER)
                        return set_error(VTX_E_HIP, "multi-workgroup adjoint: a wait between "
                                                    "the workgroups of a tissue timed out");
                return VTX_OK;
            }
            e = hipMemcpyAsync(b->order2_d, rest.data(), sizeof(int32_t) * rest.size(),
                               hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return hip_fail(e);
            rc = launch_batch_cg<double, double>(b, gi, b->order2_d, (int)rest.size(), go, 0, s);
        } else if (mode == VTX_F32)
            rc = launch_batch_cg<float, float>(b, gi, b->order_d, n, go, block_threads, s);
        else if (mode == VTX_F64)
            rc = launch_batch_cg<double, double>(b, gi, b->order_d, n, go, block_threads, s);
        else
            rc = launch_batch_cg<double, float>(b, gi, b->order_d, n, go, block_threads, s);
        if (rc) return rc;
        e = hipMemcpyAsync(res, b->gres_d, sizeof(vtx_grad_result) * n, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e == hipSuccess ? VTX_OK : hip_fail(e);
    }
    if (o->method != VTX_GRAD_EP_CENTRED && o->method != VTX_GRAD_EP_FORWARD)
        return set_error(VTX_E_ARG, "unknown method");
    const bool centred = o->method == VTX_GRAD_EP_CENTRED;
    if (!(o->beta != 0.0)) return set_error(VTX_E_ARG, "EP needs beta != 0");
    if (o->ep_relax.t1_enable) return set_error(VTX_E_ARG, "EP relaxations cannot use T1");
    int rc = check_relax_opts(&o->ep_relax);
    if (rc) return rc;
    if (!X_target && !dC_dX) return set_error(VTX_E_ARG, "EP needs X_target or dC_dX");
    const size_t esz = (mode == VTX_F32 ? sizeof(float) : sizeof(double));
    std::vector<void *> Xp(n), Xm(n);
    for (int i = 0; i < n; ++i) {
        const int64_t nv = tissue_dev(b->ts[i]).n_vert;
        char *base = (char *)tissue_ep_buf(b->ts[i]);
        Xp[i] = base;
        Xm[i] = base + 16 * (size_t)nv;
        e = hipMemcpyAsync(Xp[i], X_star[i], 2 * nv * esz, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(Xm[i], X_star[i], 2 * nv * esz, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e);
    }
    std::vector<vtx_relax_result> rp(n), rm(n);
    // block_threads < 0: the nudged relaxations split each tissue over
    // -block_threads workgroups
    const int split = block_threads < 0 ? -block_threads : 0;
    const int bt = block_threads < 0 ? 0 : block_threads;
    rc = kPlanDoesNotApply;
    if (centred && split == 0)  // both nudges in one launch where it applies
        rc = batch_relax_pm(b, mode, Xp.data(), Xm.data(), p, &o->ep_relax, X_target,
                            X_target ? nullptr : dC_dX, 0.5 * o->beta, bt, rp.data(), rm.data(), s);
    if (rc != kPlanDoesNotApply && rc != VTX_OK) return rc;
    if (rc == kPlanDoesNotApply) {
        // first-order EP: one relaxation nudged by beta; the other state stays X*
        rc = batch_relax_run(b, mode, Xp.data(), p, &o->ep_relax, X_target,
                             X_target ? nullptr : dC_dX, centred ? 0.5 * o->beta : o->beta, bt,
                             rp.data(), s, split);
        if (rc) return rc;
        if (centred) {
            rc = batch_relax_run(b, mode, Xm.data(), p, &o->ep_relax, X_target,
                                 X_target ? nullptr : dC_dX, -0.5 * o->beta, bt, rm.data(), s,
                                 split);
            if (rc) return rc;
        }
    }
    for (int i = 0; i < n; ++i) items[i].X = Xp[i];
    e = hipMemcpyAsync(b->gitems, items.data(), sizeof(GradItem) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->xm_list, Xm.data(), sizeof(void *) * n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e);
    const GradItem *gi = (const GradItem *)b->gitems;
    const dim3 grid(n), block(256);
    if (mode == VTX_F32)
        hipLaunchKernelGGL((k_batch_ep<float>), grid, block, 0, s, gi, n,
                           (const void *const *)b->xm_list, o->beta, o->theta);
    else
        hipLaunchKernelGGL((k_batch_ep<double>), grid, block, 0, s, gi, n,
                           (const void *const *)b->xm_list, o->beta, o->theta);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    for (int i = 0; i < n; ++i) {
        vtx_grad_result r{};
        r.ep_plus = rp[i];
        r.ep_minus = rm[i];
        r.status = combine_status(rp[i].status, rm[i].status);
        res[i] = r;
    }
    return VTX_OK;
}

}  // extern "C"
