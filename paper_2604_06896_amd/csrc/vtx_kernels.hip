// HIP kernels of libvtx for gfx950 (wave64) and their launchers.
//
// Hot path per energy/force evaluation (VertAX, arXiv 2604.06896, Methods,
// "Vertex model formulation"):
//   k_cell    one lane per cell: corner row read directly, shoelace
//             area and perimeter in a cell-local frame, cA = 2K_A(A-A0),
//             cP = 2K_P(P-P0), FP64 energy partial per block;
//   k_vertex  one lane per 3-valent vertex: gathers its 3 neighbours, 3 cells
//             and 3 edge tensions and forms F with no atomics; the max |F|
//             and energy are reduced per block and finished by the last
//             block or by k_finish (fixed order, deterministic).  In relaxation it also takes the
//             gradient-descent step and runs the convergence test on the
//             device (Methods, "Simulation engine").
//   k_t1      one workgroup: sequential T1 pass over the short edges flagged
//             by k_cell (Methods, "T1 transitions").
// Adjoint (Methods, "Implicit differentiation (ID)"): k_hvp_cell/k_hvp_vertex
// form H v with the same gathers, k_cg_* run conjugate gradients with FP64
// dots and device-side scalars, k_contract_* apply the mixed derivatives.
#include <climits>

#include "vtx_device.h"
#include "vtx_launch.h"

namespace vtx {

enum { F_ENERGY = 1, F_T1DET = 2, F_NUDGE_V2V = 4 };

// ------------------------------------------------------------------ cells
template <typename PosT, typename M>
__global__ __launch_bounds__(kBlock) void k_cell(DevTissue t, const PosT *__restrict__ X,
                                                 DevParams<PosT> p, M *__restrict__ cap,
                                                 double *__restrict__ epart, LoopCtl *ctl,
                                                 int32_t *t1_list, M lmin2, int flags,
                                                 const PosT *__restrict__ Xt,
                                                 double *__restrict__ npart) {
    if (ctl->done) return;
    __shared__ double sh[kBlock / 64];
    const int nc = t.n_cell;
    const int c = xcd_block() * kBlock + threadIdx.x;
    const bool det = (flags & F_T1DET) != 0;
    double e = 0.0;
    if (c < nc) {
        const int rb = t.row_ptr[c], n = t.nsides[c];
        // Area and perimeter in the precision of the positions: the
        // coefficients cA, cP come from differences (A - A0, P - P0) that
        // cancel, and in FP32 their rounding (~1e-6 on an edge tension) would
        // exceed a 1e-6 force tolerance.  The force gather stays in M.
        // (Staging the block's rows through LDS first measured slower: the
        // rows of consecutive cells are adjacent, so these reads share lines.)
        PosT A, P;
        cell_geom<PosT, PosT>(
            t, X, n, [&](int k) { return t.corner[rb + k]; }, rb, A, P, det, (PosT)lmin2,
            t1_list, &ctl->t1_count);
        const PosT ka = p.ka(c), kp = p.kp(c);
        const PosT da = A - p.a0(c), dp = P - p.p0(c);
        st2(cap, c, (M)((PosT)2 * ka * da), (M)((PosT)2 * kp * dp));
        if (flags & F_ENERGY)
            e = (double)ka * (double)da * (double)da + (double)kp * (double)dp * (double)dp;
    }
    if (flags & F_ENERGY) {
        const double s = block_sum(e, sh);
        if (threadIdx.x == 0) epart[blockIdx.x] = s;
    }
    // mean over vertices of the v2v displacement (minimum image), by the
    // first kRedBlocks blocks only (fewer device-scope arrivals)
    const int nred = min((int)gridDim.x, kRedBlocks);
    if ((flags & F_NUDGE_V2V) && (int)blockIdx.x < nred) {
        double sx = 0.0, sy = 0.0;
        for (int v = blockIdx.x * kBlock + threadIdx.x; v < t.n_vert; v += nred * kBlock) {
            sx += min_image((double)X[2 * (int64_t)v] - (double)Xt[2 * (int64_t)v], t.Lx);
            sy += min_image((double)X[2 * (int64_t)v + 1] - (double)Xt[2 * (int64_t)v + 1], t.Ly);
        }
        const double bx = block_sum(sx, sh);
        const double by = block_sum(sy, sh);
        __shared__ int s_last;
        if (threadIdx.x == 0) {
            npart[2 * blockIdx.x] = bx;
            npart[2 * blockIdx.x + 1] = by;
            s_last = last_of(&ctl->arrive2, (unsigned)nred);
        }
        __syncthreads();
        if (s_last) {
            const double ax = block_sum_array(npart, nred, 2, sh);
            const double ay = block_sum_array(npart + 1, nred, 2, sh);
            if (threadIdx.x == 0) {
                const double nv = (double)t.n_vert;
                ctl->nudge_mean[0] = ax / nv / nv;
                ctl->nudge_mean[1] = ay / nv / nv;
            }
        }
    }
}

// ----------------------------------------------------------------- vertex
// Each block stores its (energy, max |F|) partial.  Grids up to
// kLastBlockMax blocks finish the reduction in the last block to arrive;
// larger grids leave it to k_finish.  An arrival needs a device-scope
// release and acquire, which on this multi-XCD part write back and
// invalidate the XCD's L2 (tens of ns each, and they serialise): thousands
// of arrivals cost far more than one extra launch.
constexpr int kLastBlockMax = 128;

struct VertexArgs {
    LoopCtl *ctl;
    const double *epart_cell;  // per-block cell energies of the preceding k_cell
    int n_epart_cell;
    double2 *part;      // per-block (energy, max |F|)
    int finish;         // 1: the last block finishes here; 0: k_finish does
    double *E_out;
    double *maxf_out;
    double eta;
    int cur;
    int nudge;  // 0 none, 1 v2v, 2 linear
    double beta;
    const void *Xt;
    const void *g_lin;
};

__device__ __forceinline__ void relax_control(LoopCtl *ctl, double mf, int cur) {
    ctl->iter += 1;
    ctl->last_maxf = mf;
    if (!(mf <= 1.7976931348623157e308)) {  // NaN or infinity
        ctl->done = 1;
        ctl->status = VTX_E_NONFINITE;
        ctl->result_buf = cur;
        return;
    }
    if (mf < ctl->tol) ctl->count += 1;
    else ctl->count = 0;
    if (ctl->count >= ctl->patience) {
        ctl->done = 1;
        ctl->status = VTX_CONVERGED;
        ctl->result_buf = cur;
    } else if (ctl->iter >= ctl->max_iter) {
        ctl->done = 1;
        ctl->status = VTX_NOT_CONVERGED;
        ctl->result_buf = cur ^ 1;
    }
}

template <int MODE>
__device__ __forceinline__ void finish_reductions(const VertexArgs &a, int nblk, double *sh,
                                                  bool plain);

template <typename PosT, typename M, int MODE>  // MODE 0: evaluate, 1: relaxation step
__global__ __launch_bounds__(kBlock) void k_vertex(DevTissue t, const PosT *__restrict__ X,
                                                   PosT *__restrict__ out, DevParams<PosT> p,
                                                   const M *__restrict__ cap, VertexArgs a) {
    if (MODE == 1 && a.ctl->done) return;
    __shared__ double sh[2 * (kBlock / 64)];
    const int v = xcd_block() * kBlock + threadIdx.x;
    double el = 0.0, mf = 0.0;
    if (v < t.n_vert) {
        Star<PosT, M> s;
        PosT xi, yi;
        load_star<PosT, M>(t, X, p, cap, v, s, xi, yi);
        M fx, fy;
        star_force<PosT, M>(s, fx, fy);
        if (MODE == 0) {
            if (a.E_out)
                el = 0.5 * ((double)s.lam[0] * (double)s.l[0] + (double)s.lam[1] * (double)s.l[1] +
                            (double)s.lam[2] * (double)s.l[2]);
            if (out) st2(out, v, (PosT)fx, (PosT)fy);
            mf = fmax(fabs((double)fx), fabs((double)fy));
            if (!(fx == fx) || !(fy == fy)) mf = INFINITY;
        } else {
            double gx = fx, gy = fy;
            if (a.nudge == 1) {
                const PosT *Xt = (const PosT *)a.Xt;
                const double inv = 1.0 / (double)t.n_vert;
                const double cx = min_image((double)xi - (double)Xt[2 * (int64_t)v], t.Lx) * inv;
                const double cy = min_image((double)yi - (double)Xt[2 * (int64_t)v + 1], t.Ly) * inv;
                gx -= a.beta * (cx - a.ctl->nudge_mean[0]);
                gy -= a.beta * (cy - a.ctl->nudge_mean[1]);
            } else if (a.nudge == 2) {
                const double *g = (const double *)a.g_lin;
                gx -= a.beta * (g[2 * (int64_t)v] - a.ctl->nudge_mean[0]);
                gy -= a.beta * (g[2 * (int64_t)v + 1] - a.ctl->nudge_mean[1]);
            }
            mf = fmax(fabs(gx), fabs(gy));
            if (!(gx == gx) || !(gy == gy)) mf = INFINITY;
            st2(out, v, (PosT)((double)xi + a.eta * gx), (PosT)((double)yi + a.eta * gy));
        }
    }
    if (MODE == 1 || a.maxf_out || a.E_out) {
        // block b also takes the cell-pass energy partials b, b + grid, ...
        double ec = 0.0;
        if (MODE == 0 && a.E_out && threadIdx.x == 0)
            for (int j = blockIdx.x; j < a.n_epart_cell; j += gridDim.x) ec += a.epart_cell[j];
        double2 r = block_sum_max(el, mf, sh);
        __shared__ int s_last;
        if (threadIdx.x == 0) {
            r.x += ec;
            a.part[blockIdx.x] = r;
            s_last = a.finish ? last_block(&a.ctl->arrive) : 0;
        }
        __syncthreads();
        if (s_last) finish_reductions<MODE>(a, gridDim.x, sh, false);
    }
}

// Fixed-order reduction of the per-block (energy, max |F|) partials of one
// evaluation (or one relaxation step), then the result / the convergence
// control.  `plain`: the partials were written by an earlier kernel, so
// ordinary loads see them; otherwise (last block of the same kernel) they
// are read at device scope.  Each thread takes a fixed strided subset with
// eight loads in flight, so the order does not depend on which block runs it.
template <int MODE>
__device__ __forceinline__ void finish_reductions(const VertexArgs &a, int nblk, double *sh,
                                                  bool plain) {
    double e = 0.0, m = 0.0;
    for (int base = 0; base < nblk; base += 8 * (int)blockDim.x) {
        double2 x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = base + u * (int)blockDim.x + (int)threadIdx.x;
            x[u] = double2{0.0, 0.0};
            if (i < nblk) {
                if (plain) {
                    x[u] = a.part[i];
                } else {
                    const double *q = reinterpret_cast<const double *>(a.part + i);
                    x[u].x = ld_acquire(q);
                    x[u].y = ld_acquire(q + 1);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            e += x[u].x;
            m = nanmax(m, x[u].y);
        }
    }
    __syncthreads();  // `sh` may still be read by the block's own partial
    const double2 r = block_sum_max(e, m, sh);
    if (threadIdx.x == 0) {
        const double mfin = r.y != r.y ? INFINITY : r.y;
        if (MODE == 1) {
            relax_control(a.ctl, mfin, a.cur);
        } else {
            if (a.maxf_out) *a.maxf_out = mfin;
            if (a.E_out) *a.E_out = r.x;
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(1024) void k_finish(VertexArgs a, int nblk) {
    if (MODE == 1 && a.ctl->done) return;
    __shared__ double sh[2 * (1024 / 64)];
    finish_reductions<MODE>(a, nblk, sh, true);
}

// --------------------------------------------------------- fused evaluation
// Heads of runs of equal keys in keys[per * tid, per * (tid + 1)) (INT_MAX
// pads), compacted in order into out[0, cap); returns the number of
// distinct keys (valid in every thread; may exceed cap, then out holds the
// first cap).
template <int PER>
__device__ __forceinline__ int block_unique(const int32_t *keys, int32_t *out, int cap,
                                            int32_t *scan) {
    const int tid = threadIdx.x, nt = blockDim.x;
    int nh = 0;
    for (int j = 0; j < PER; ++j) {
        const int i = PER * tid + j;
        const int32_t x = keys[i];
        nh += (x != INT_MAX && (i == 0 || keys[i - 1] != x)) ? 1 : 0;
    }
    __syncthreads();
    scan[tid] = nh;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        const int add = tid >= off ? scan[tid - off] : 0;
        __syncthreads();
        scan[tid] += add;
        __syncthreads();
    }
    const int total = scan[nt - 1];
    int o = scan[tid] - nh;
    for (int j = 0; j < PER; ++j) {
        const int i = PER * tid + j;
        const int32_t x = keys[i];
        if (x != INT_MAX && (i == 0 || keys[i - 1] != x)) {
            if (o < cap) out[o] = x;
            ++o;
        }
    }
    __syncthreads();
    return total;
}

__device__ __forceinline__ int lower_bound_lds(const int32_t *a, int n, int32_t x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One block per vertex tile builds the tile's local mesh: its distinct
// cells (owner-tagged, ordered by side count), their corner rows and the tile's star
// neighbours as local references, and the halo of outside vertices they
// reach.  Tiles whose halo or rows overflow the fixed slots are marked for
// the global path.
__global__ __launch_bounds__(kTileV) void k_tile_build(DevTissue t, TileTables tt) {
    constexpr int NK = 4096;  // 3 kTileV neighbours + kCornerCap corners, padded
    static_assert(3 * kTileV + kCornerCap <= NK, "halo candidate buffer");
    __shared__ int32_t keys[NK];
    __shared__ int32_t uniq[kTileCap];  // distinct cells by id
    __shared__ int32_t ord[kTileCap];   // the same cells by side count (then id)
    __shared__ int32_t perm[kTileCap];  // position in ord of uniq[i]
    __shared__ int32_t oimg[kTileCap];  // ord[r] has a corner with a nonzero image
    __shared__ int32_t halo[kHaloCap];
    __shared__ int32_t scan[kTileV];
    const int tile = blockIdx.x, tid = threadIdx.x;
    const int nv = t.n_vert;
    const int lo = tile * kTileV;
    const int hi = min(nv, lo + kTileV);
    const int v = lo + tid;
    const bool live = v < nv;
    int32_t c[3] = {INT_MAX, INT_MAX, INT_MAX}, w[3] = {0, 0, 0};
    if (live) {
        const int4 a4 = reinterpret_cast<const int4 *>(t.star)[v];  // {nb_0, nb_1, nb_2, c_0}
        w[0] = a4.x;
        w[1] = a4.y;
        w[2] = a4.z;
        for (int k = 0; k < 3; ++k) c[k] = t.star[star_cell_at(nv, k, v)];
    }
    // (1) the distinct cells around the tile's vertices
    for (int k = 0; k < 3; ++k) keys[3 * tid + k] = c[k];
    keys[3 * kTileV + tid] = INT_MAX;
    __syncthreads();
    block_bitonic(keys, 4 * kTileV);
    const int nu = block_unique<4>(keys, uniq, kTileCap, scan);  // <= 3 kTileV
    // (1b) cells ordered by (crosses the box, side count), so that the lanes
    // of a wave walk rows of equal length and most waves need no images
    for (int i = tid; i < 4 * kTileV; i += kTileV) {
        int key = INT_MAX;
        if (i < nu) {
            const int cc = uniq[i];
            const int ns = t.nsides[cc], rb = t.row_ptr[cc];
            int img = 0;
            for (int k = 0; k < ns; ++k)
                img |= ((uint32_t)t.corner[rb + k] >> kIdBits) != kZeroImage ? 1 : 0;
            key = (((img << 10) | min(ns, 1023)) << 10) | i;
        }
        keys[i] = key;
    }
    __syncthreads();
    block_bitonic(keys, 4 * kTileV);
    for (int r = tid; r < nu; r += kTileV) {
        const int i = keys[r] & 1023;
        ord[r] = uniq[i];
        perm[i] = r;
        oimg[r] = (keys[r] >> 20) & 1;
    }
    __syncthreads();
    // (2) row starts: exclusive scan of the rows' lengths, cells 3 tid .. 3 tid + 2
    int len[3], cid[3];
    int sum = 0;
    for (int j = 0; j < 3; ++j) {
        const int i = 3 * tid + j;
        cid[j] = i < nu ? ord[i] : -1;
        len[j] = i < nu ? t.nsides[cid[j]] : 0;
        sum += len[j];
    }
    scan[tid] = sum;
    __syncthreads();
    for (int off = 1; off < kTileV; off <<= 1) {
        const int add = tid >= off ? scan[tid - off] : 0;
        __syncthreads();
        scan[tid] += add;
        __syncthreads();
    }
    const int ncorner = scan[kTileV - 1];
    int start[3];
    start[0] = scan[tid] - sum;
    start[1] = start[0] + len[0];
    start[2] = start[1] + len[1];
    bool fallback = ncorner > kCornerCap;
    // (3) the halo: neighbours and corners outside [lo, hi)
    int nh = 0;
    if (!fallback) {
        __syncthreads();
        for (int i = tid; i < NK; i += kTileV) keys[i] = INT_MAX;
        __syncthreads();
        for (int k = 0; k < 3; ++k) {
            const int id = id_of(w[k]);
            keys[3 * tid + k] = live && (id < lo || id >= hi) ? id : INT_MAX;
        }
        for (int j = 0; j < 3; ++j) {
            if (cid[j] < 0) continue;
            const int rb = t.row_ptr[cid[j]];
            for (int k = 0; k < len[j]; ++k) {
                const int id = id_of(t.corner[rb + k]);
                keys[3 * kTileV + start[j] + k] = id < lo || id >= hi ? id : INT_MAX;
            }
        }
        __syncthreads();
        block_bitonic(keys, NK);
        nh = block_unique<NK / kTileV>(keys, halo, kHaloCap, scan);
        fallback = nh > kHaloCap;
    }
    // (4) the tables
    int32_t *dst = tt.cells + (int64_t)tile * kTileCap;
    for (int j = 0; j < 3; ++j) {
        if (cid[j] < 0) continue;
        const int v0 = id_of(t.corner[t.row_ptr[cid[j]]]);
        uint32_t e = (uint32_t)cid[j] | (oimg[3 * tid + j] ? kCellImage : 0u);
        if (v0 / kTileV == tile) e |= kCellOwner;
        dst[3 * tid + j] = (int32_t)e;
    }
    auto local_of = [&](int32_t wk) -> int {
        const int id = id_of(wk);
        return id >= lo && id < hi ? id - lo : kTileV + lower_bound_lds(halo, nh, id);
    };
    if (!fallback) {
        for (int i = tid; i < nh; i += kTileV) tt.halo[(int64_t)tile * kHaloCap + i] = halo[i];
        uint16_t *cs = tt.cstart + (int64_t)tile * kCstartPad;
        uint16_t *co = tt.corners + (int64_t)tile * kCornerCap;
        for (int j = 0; j < 3; ++j) {
            if (cid[j] < 0) continue;
            cs[3 * tid + j] = (uint16_t)start[j];
            const int rb = t.row_ptr[cid[j]];
            for (int k = 0; k < len[j]; ++k) {
                const int32_t wk = t.corner[rb + k];
                co[start[j] + k] = (uint16_t)pack_local(local_of(wk), wk);
            }
        }
        if (tid == 0) cs[nu] = (uint16_t)ncorner;
    }
    if (tid == 0) tt.info[tile] = make_int4(nu, fallback ? 0 : nh, fallback ? 1 : 0, ncorner);
    if (live) {
        int lc = 0;
        for (int k = 0; k < 3; ++k) lc |= perm[lower_bound_lds(uniq, nu, c[k])] << (10 * k);
        uint32_t nb[3] = {0u, 0u, 0u};
        if (!fallback)
            for (int k = 0; k < 3; ++k) nb[k] = pack_local(local_of(w[k]), w[k]);
        uint32_t vimg = 0;
        for (int k = 0; k < 3; ++k) vimg |= ((uint32_t)w[k] >> kIdBits) != kZeroImage ? 1u : 0u;
        const int e0 = t.star[star_edge_at(nv, 0, v)];
        tt.fstar[v] = make_int4((int32_t)(nb[0] | (nb[1] << 16)), (int32_t)(nb[2] | (vimg << 16)),
                                lc, e0);
        tt.fe[v] = t.star[star_edge_at(nv, 1, v)];
        tt.fe[(int64_t)nv + v] = t.star[star_edge_at(nv, 2, v)];
    }
}

// Energy and forces in one launch.  Each block takes one vertex tile: it
// issues its vertices' edge-tension gathers, stages the positions of the
// tile and its halo, the tile's corner rows and row starts in LDS, computes
// (cA, cP) of the tile's cells there (cells on the tile border are computed
// by every tile around them; the owner adds the cell energy), then forms
// the forces from LDS.  The arithmetic is that of k_cell + k_vertex, so F is
// bit-identical to the two-pass evaluation.  Tiles marked for the global
// path read the star, the rows and the positions from global memory.
template <typename PosT, typename M>
__global__ __launch_bounds__(kTileV) void k_eval_fused(DevTissue t, const PosT *__restrict__ X,
                                                       PosT *__restrict__ out, DevParams<PosT> p,
                                                       TileTables tt, VertexArgs a) {
    using V2 = typename Vec2<PosT>::type;
    __shared__ V2 sh_x[kTileV + kHaloCap];
    __shared__ typename Vec2<M>::type sh_cap[kTileCap];
    __shared__ uint4 sh_corner[kCornerCap / 8];
    __shared__ uint16_t sh_cstart[kCstartPad];
    __shared__ double sh[2 * (kTileV / 64)];
    const int tid = threadIdx.x;
    const int tile = xcd_block();
    const int4 info = tt.info[tile];
    const int nc = info.x, nh = info.y, ncorner = info.w;
    const bool local = info.z == 0;
    const int nv = t.n_vert;
    const int v = tile * kTileV + tid;
    const bool live = v < nv;
    const PosT *Xl = reinterpret_cast<const PosT *>(sh_x);
    const uint16_t *crn = reinterpret_cast<const uint16_t *>(sh_corner);
    StarLoad<PosT, M> L;
    int lc = 0;
    uint32_t vimg = 0;
    if (live) {
        const int4 f = tt.fstar[v];
        lc = f.z;
        L.e[0] = f.w;
        L.e[1] = tt.fe[v];
        L.e[2] = tt.fe[(int64_t)nv + v];
        if (local) {
            L.w[0] = unpack_local((uint32_t)f.x & 0xffffu);
            L.w[1] = unpack_local((uint32_t)f.x >> 16);
            L.w[2] = unpack_local((uint32_t)f.y & 0xffffu);
            vimg = ((uint32_t)f.y >> 16) & 1u;
        } else {
            const int4 s4 = reinterpret_cast<const int4 *>(t.star)[v];
            L.w[0] = s4.x;
            L.w[1] = s4.y;
            L.w[2] = s4.z;
            L.pi = ld2(X, v);
#pragma unroll
            for (int k = 0; k < 3; ++k) L.q[k] = ld2(X, id_of(L.w[k]));
        }
        if (p.lam) {
#pragma unroll
            for (int k = 0; k < 3; ++k) L.lam[k] = p.lam[L.e[k]];
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) L.lam[k] = p.lam_s;
        }
    }
    // the thread's first cell (tiles rarely have more than kTileV cells)
    const int32_t *cl = tt.cells + (int64_t)tile * kTileCap;
    const int32_t x0 = tid < nc ? cl[tid] : 0;
    if (local) {
        if (live) sh_x[tid] = ld2(X, v);
        const int32_t *hl = tt.halo + (int64_t)tile * kHaloCap;
        for (int j = tid; j < nh; j += kTileV) sh_x[kTileV + j] = ld2(X, hl[j]);
        const uint4 *src = reinterpret_cast<const uint4 *>(tt.corners + (int64_t)tile * kCornerCap);
        for (int j = tid; j < (ncorner + 7) / 8; j += kTileV) sh_corner[j] = src[j];
        const uint16_t *cs = tt.cstart + (int64_t)tile * kCstartPad;
        for (int j = tid; j <= nc; j += kTileV) sh_cstart[j] = cs[j];
    }
    __syncthreads();
    double ec = 0.0;
    for (int i = tid; i < nc; i += kTileV) {
        const int32_t x = i == tid ? x0 : cl[i];
        const int c = (int)((uint32_t)x & kIdMask);
        PosT A, P;
        if (local) {
            const int rb = sh_cstart[i], n = (int)sh_cstart[i + 1] - rb;
            auto corner_at = [&](int k) { return unpack_local(crn[rb + k]); };
            // waves whose cells all lie inside the box take plain differences
            if (__builtin_amdgcn_ballot_w64(((uint32_t)x & kCellImage) != 0) != 0)
                cell_geom<PosT, PosT, false>(t, Xl, n, corner_at, 0, A, P, false, (PosT)0,
                                             (int32_t *)nullptr, (unsigned int *)nullptr);
            else
                cell_geom<PosT, PosT, true>(t, Xl, n, corner_at, 0, A, P, false, (PosT)0,
                                            (int32_t *)nullptr, (unsigned int *)nullptr);
        } else {
            const int rb = t.row_ptr[c], n = t.nsides[c];
            cell_geom<PosT, PosT>(
                t, X, n, [&](int k) { return t.corner[rb + k]; }, rb, A, P, false, (PosT)0,
                (int32_t *)nullptr, (unsigned int *)nullptr);
        }
        const PosT ka = p.ka(c), kp = p.kp(c);
        const PosT da = A - p.a0(c), dp = P - p.p0(c);
        typename Vec2<M>::type cc;
        cc.x = (M)((PosT)2 * ka * da);
        cc.y = (M)((PosT)2 * kp * dp);
        sh_cap[i] = cc;
        // the cell energy in the type of the positions (FP64 in the FP64
        // and MIXED modes, where this equals the two-pass kernel's sum)
        if (x < 0 && a.E_out) ec += (double)(ka * da * da + kp * dp * dp);
    }
    __syncthreads();
    double el = 0.0, mf = 0.0;
    if (live) {
        if (local) {
            L.pi = sh_x[tid];
#pragma unroll
            for (int k = 0; k < 3; ++k) L.q[k] = sh_x[id_of(L.w[k])];
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) L.cc[k] = sh_cap[(lc >> (10 * k)) & 1023];
        Star<PosT, M> s;
        PosT xi, yi;
        if (__builtin_amdgcn_ballot_w64(vimg != 0u || !local) != 0)
            star_math<PosT, M, false>(t, L, s, xi, yi);
        else
            star_math<PosT, M, true>(t, L, s, xi, yi);
        M fx, fy;
        star_force<PosT, M>(s, fx, fy);
        // half of each edge's line energy, summed in the arithmetic type
        if (a.E_out)
            el = 0.5 * (double)(s.lam[0] * s.l[0] + s.lam[1] * s.l[1] + s.lam[2] * s.l[2]);
        if (out) st2(out, v, (PosT)fx, (PosT)fy);
        mf = (double)fmax(fabs(fx), fabs(fy));
        if (!(fx == fx) || !(fy == fy)) mf = INFINITY;
    }
    if (a.maxf_out || a.E_out) {
        // The block's sums: every thread leaves (energy, max |F|) in the
        // corner staging area (not read after the cell phase) and wave 0
        // adds them, four per lane in fixed order, then across the wave.
        // max |F| is never NaN here (a NaN force was mapped to +inf).
        static_assert(2 * kTileV * sizeof(double) <= sizeof(sh_corner), "tail sums");
        double *se = reinterpret_cast<double *>(sh_corner);
        double *sm = se + kTileV;
        se[tid] = el + ec;
        sm[tid] = mf;
        __syncthreads();
        __shared__ int s_last;
        if (tid < 64) {
            double e = ((se[tid] + se[tid + 64]) + se[tid + 128]) + se[tid + 192];
            double m = fmax(fmax(sm[tid], sm[tid + 64]), fmax(sm[tid + 128], sm[tid + 192]));
            e = wave_sum(e);
            m = wave_max_plain(m);
            if (tid == 0) {
                a.part[blockIdx.x] = double2{e, m};
                s_last = a.finish ? last_block(&a.ctl->arrive) : 0;
            }
        }
        if (a.finish) {  // small grids: the last block finishes the scalars
            __syncthreads();
            if (s_last) finish_reductions<0>(a, gridDim.x, sh, false);
        }
    }
}

// ---------------------------------------------------------------------- T1
template <typename PosT, typename M>
__global__ __launch_bounds__(kBlock) void k_t1(DevTissue t, PosT *X, DevParams<PosT> p, M *cap,
                                               LoopCtl *ctl, int32_t *list_g, double l_min,
                                               double l_new) {
    __shared__ int32_t buf[kT1SortCap];
    __shared__ int32_t extra[kT1Extra];
    __shared__ int32_t scan[kBlock];
    __shared__ int s_changed;
    if (ctl->done) return;
    const int n = (int)ctl->t1_count;
    if (n == 0) return;
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    int32_t *arr = np2 <= kT1SortCap ? buf : list_g;
    // corner index -> edge id (each thread reads and writes only its own
    // slots, so converting in place when arr == list_g is safe)
    for (int i = threadIdx.x; i < np2; i += blockDim.x)
        arr[i] = i < n ? t.he_edge[t.corner_he[list_g[i]]] : INT_MAX;
    __syncthreads();
    block_bitonic(arr, np2);
    if (threadIdx.x < 64) {  // one wave runs the pass
        T1Counts r = t1_sequential<PosT, M>(t, X, p, cap, arr, n, extra, l_min, l_new);
        if (threadIdx.x == 0) {
        ctl->n_t1 += r.swaps;
        ctl->n_stretch += r.stretches;
        if (r.overflow) ctl->t1_overflow = r.overflow;
        ctl->t1_count = 0;
        s_changed = r.relocated;
        if (r.changed) ctl->topo_changed = 1;
        if (r.overflow == 2) ctl->done = 1;  // stop the loop; the host reports it
        }
    }
    __syncthreads();
    if (s_changed) {  // rows moved to the pool: compact them again
        const int bad = rebuild_rows_block(t, scan);
        if (threadIdx.x == 0 && bad) {
            ctl->t1_overflow = 2;
            ctl->done = 1;
        }
    }
}

// ------------------------------------------------------ scalar reductions
// A Krylov step ends with a sum over all vertices followed by scalar work
// (step lengths, rotations, stopping tests).  Each block stores its partial;
// grids of up to kLastBlockMax blocks finish in the last block to arrive,
// larger grids in a one-block k_fin launch (thousands of device-scope
// arrivals would serialise).  The scalar work is a functor run once, by one
// thread, on the total.

template <class Fin>
__device__ __forceinline__ void reduce_tail(double val, double *part, LoopCtl *ctl,
                                            double *sh, Fin fin) {
    const double bs = block_sum(val, sh);
    __shared__ int s_last;
    if (threadIdx.x == 0) {
        part[blockIdx.x] = bs;
        s_last = gridDim.x <= (unsigned)kLastBlockMax ? last_block(&ctl->arrive) : 0;
    }
    __syncthreads();
    if (s_last) {
        const double tot = block_sum_array(part, gridDim.x, 1, sh);
        if (threadIdx.x == 0) fin(ctl, tot);
    }
}

template <class Fin>
__global__ __launch_bounds__(1024) void k_fin(const double *__restrict__ part, int n,
                                              LoopCtl *ctl, Fin fin) {
    if (ctl->done) return;
    __shared__ double sh[1024 / 64];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
    const double tot = block_sum(v, sh);
    if (threadIdx.x == 0) fin(ctl, tot);
}

template <class Fin>
static void launch_fin(unsigned grid, const double *part, LoopCtl *ctl, Fin fin, hipStream_t s) {
    if (grid > (unsigned)kLastBlockMax)
        hipLaunchKernelGGL((k_fin<Fin>), dim3(1), dim3(1024), 0, s, part, (int)grid, ctl, fin);
}

// q.Hq of the HVP: CG's step length (and its curvature check); MINRES's
// Lanczos coefficient alpha.
struct FinPAp {
    __device__ void operator()(LoopCtl *ctl, double pAp) const {
        ctl->pAp = pAp;
        if (ctl->solver == 0) {  // CG: stop on non-positive curvature
            if (!(pAp > 0.0)) {
                ctl->done = 1;
                ctl->status = VTX_CG_NEG_CURVATURE;
            } else {
                ctl->alpha = ctl->rr / pAp;
            }
        }
    }
};

// -------------------------------------------------------------------- HVP
template <typename PosT, typename M>
__global__ __launch_bounds__(kBlock) void k_hvp_cell(DevTissue t, const PosT *__restrict__ X,
                                                     DevParams<PosT> p,
                                                     const double *__restrict__ v,
                                                     M *__restrict__ aux, LoopCtl *ctl) {
    if (ctl && ctl->done) return;
    const int c = xcd_block() * kBlock + threadIdx.x;
    if (c >= t.n_cell) return;
    hvp_cell_one<PosT, M>(t, X, p, v, aux, c);
}

template <typename PosT, typename M>
__global__ __launch_bounds__(kBlock) void k_hvp_vertex(DevTissue t, const PosT *__restrict__ X,
                                                       DevParams<PosT> p,
                                                       const M *__restrict__ cap,
                                                       const M *__restrict__ aux,
                                                       const double *__restrict__ v,
                                                       double *__restrict__ Hv,
                                                       double *__restrict__ dpart,
                                                       LoopCtl *ctl) {
    if (ctl && ctl->done) return;
    __shared__ double sh[kBlock / 64];
    const int i = xcd_block() * kBlock + threadIdx.x;
    double dot = 0.0;
    if (i < t.n_vert) dot = hvp_vertex_one<PosT, M>(t, X, p, cap, aux, v, Hv, i);
    if (dpart) reduce_tail(dot, dpart, ctl, sh, FinPAp{});
}

// --------------------------------------------------------------------- CG
// Sum over vertices of a 2-vector field -> ctl->nudge_mean (as a mean).
__global__ __launch_bounds__(kBlock) void k_mean2(const double *__restrict__ a, int nv,
                                                  double *__restrict__ part, LoopCtl *ctl,
                                                  double *mean_out) {
    __shared__ double sh[kBlock / 64];
    double sx = 0.0, sy = 0.0;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < nv; v += gridDim.x * kBlock) {
        sx += a[2 * (int64_t)v];
        sy += a[2 * (int64_t)v + 1];
    }
    const double bx = block_sum(sx, sh);
    const double by = block_sum(sy, sh);
    __shared__ int s_last;
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = bx;
        part[2 * blockIdx.x + 1] = by;
        s_last = last_block(&ctl->arrive2);
    }
    __syncthreads();
    if (s_last) {
        const double ax = block_sum_array(part, gridDim.x, 2, sh);
        const double ay = block_sum_array(part + 1, gridDim.x, 2, sh);
        if (threadIdx.x == 0) {
            mean_out[0] = ax / (double)nv;
            mean_out[1] = ay / (double)nv;
        }
    }
}

// v <- v - mean  (in place); also usable to produce r = b - mean.
__global__ __launch_bounds__(kBlock) void k_sub_mean(const double *__restrict__ a,
                                                     double *__restrict__ out, int nv,
                                                     const double *mean) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= nv) return;
    out[2 * (int64_t)v] = a[2 * (int64_t)v] - mean[0];
    out[2 * (int64_t)v + 1] = a[2 * (int64_t)v + 1] - mean[1];
}

struct FinCgInit {
    __device__ void operator()(LoopCtl *ctl, double s) const {
        ctl->rr = s;
        ctl->rr0 = s;
        ctl->rel_res = s > 0.0 ? 1.0 : 0.0;
        if (!(s > 0.0)) {
            ctl->done = 1;
            ctl->status = VTX_CONVERGED;
        }
    }
};

// r = b - mean(b), p = r, x = 0, rr = r . r
__global__ __launch_bounds__(kBlock) void k_cg_init(const double *__restrict__ b, int nv,
                                                    const double *mean, double *__restrict__ x,
                                                    double *__restrict__ r,
                                                    double *__restrict__ q,
                                                    double *__restrict__ part, LoopCtl *ctl) {
    __shared__ double sh[kBlock / 64];
    const int v = blockIdx.x * kBlock + threadIdx.x;
    double rr = 0.0;
    if (v < nv) {
        const double rx = b[2 * (int64_t)v] - mean[0], ry = b[2 * (int64_t)v + 1] - mean[1];
        r[2 * (int64_t)v] = rx;
        r[2 * (int64_t)v + 1] = ry;
        q[2 * (int64_t)v] = rx;
        q[2 * (int64_t)v + 1] = ry;
        x[2 * (int64_t)v] = 0.0;
        x[2 * (int64_t)v + 1] = 0.0;
        rr = rx * rx + ry * ry;
    }
    reduce_tail(rr, part, ctl, sh, FinCgInit{});
}

struct FinCgUpdate {
    __device__ void operator()(LoopCtl *ctl, double s) const {
        ctl->beta_cg = s / ctl->rr;
        ctl->rr = s;
        ctl->cg_iter += 1;
        ctl->rel_res = sqrt(s / ctl->rr0);
        if (sqrt(s) <= ctl->tol * sqrt(ctl->rr0)) {
            ctl->done = 1;
            ctl->status = VTX_CONVERGED;
        } else if (ctl->cg_iter >= ctl->max_iter) {
            ctl->done = 1;
            ctl->status = VTX_CG_MAXITER;
        }
    }
};

// x += alpha q, r -= alpha Aq, then beta = r.r / rr and the stopping tests.
__global__ __launch_bounds__(kBlock) void k_cg_update(double *__restrict__ x,
                                                      double *__restrict__ r,
                                                      const double *__restrict__ q,
                                                      const double *__restrict__ Aq, int nv,
                                                      double *__restrict__ part, LoopCtl *ctl) {
    if (ctl->done) return;
    __shared__ double sh[kBlock / 64];
    const int v = blockIdx.x * kBlock + threadIdx.x;
    const double al = ctl->alpha;
    double rr = 0.0;
    if (v < nv) {
        const int64_t k = 2 * (int64_t)v;
        x[k] += al * q[k];
        x[k + 1] += al * q[k + 1];
        const double r0 = r[k] - al * Aq[k], r1 = r[k + 1] - al * Aq[k + 1];
        r[k] = r0;
        r[k + 1] = r1;
        rr = r0 * r0 + r1 * r1;
    }
    reduce_tail(rr, part, ctl, sh, FinCgUpdate{});
}

__global__ __launch_bounds__(kBlock) void k_cg_dir(const double *__restrict__ r,
                                                   double *__restrict__ q, int nv,
                                                   LoopCtl *ctl) {
    if (ctl->done) return;
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= nv) return;
    const double be = ctl->beta_cg;
    const int64_t k = 2 * (int64_t)v;
    q[k] = r[k] + be * q[k];
    q[k + 1] = r[k + 1] + be * q[k + 1];
}

// ------------------------------------------------------------ contractions
template <typename PosT>
__global__ __launch_bounds__(kBlock) void k_contract_lambda(DevTissue t, const PosT *X,
                                                            const double *mu, double *g) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e < t.n_edge) g[e] = contract_lambda_one<PosT>(t, X, mu, e);
}

template <typename PosT>
__global__ __launch_bounds__(kBlock) void k_contract_p0(DevTissue t, const PosT *X,
                                                        DevParams<PosT> p, const double *mu,
                                                        double *g) {
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c < t.n_cell) g[c] = contract_p0_one<PosT>(t, X, p, mu, c);
}

template <typename PosT>
__global__ __launch_bounds__(kBlock) void k_edge_len(DevTissue t, const PosT *X, double *len) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= t.n_edge) return;
    const int32_t *r = t.he + 8 * (int64_t)t.edge_he[e];
    const int s = r[HS], q = r[HG];
    const double dx = pdiff<double>((double)X[2 * (int64_t)q], (double)X[2 * (int64_t)s], r[HOX], t.Lx);
    const double dy = pdiff<double>((double)X[2 * (int64_t)q + 1], (double)X[2 * (int64_t)s + 1], r[HOY], t.Ly);
    len[e] = sqrt(dx * dx + dy * dy);
}

// Exact (double) area and perimeter of every cell, walking the table.
template <typename PosT>
__global__ __launch_bounds__(kBlock) void k_cell_exact(DevTissue t, const PosT *X, double *A,
                                                       double *P) {
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= t.n_cell) return;
    PosOverride<PosT> none{-1, -1, 0, 0, 0, 0};
    double a, per;
    cell_walk<PosT>(t, X, t.cell_he[c], none, a, per);
    if (A) A[c] = a;
    if (P) P[c] = per;
}

// EP estimates from the two nudged states.
template <typename PosT>
__global__ __launch_bounds__(kBlock) void k_ep_lambda(DevTissue t, const PosT *Xp,
                                                      const PosT *Xm, double beta, double *g) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= t.n_edge) return;
    const int32_t *r = t.he + 8 * (int64_t)t.edge_he[e];
    const int s = r[HS], q = r[HG];
    double l[2];
    const PosT *Xs[2] = {Xp, Xm};
    for (int a = 0; a < 2; ++a) {
        const PosT *X = Xs[a];
        const double dx = pdiff<double>((double)X[2 * (int64_t)q], (double)X[2 * (int64_t)s], r[HOX], t.Lx);
        const double dy = pdiff<double>((double)X[2 * (int64_t)q + 1], (double)X[2 * (int64_t)s + 1], r[HOY], t.Ly);
        l[a] = sqrt(dx * dx + dy * dy);
    }
    g[e] = (l[0] - l[1]) / beta;
}

template <typename PosT>
__global__ __launch_bounds__(kBlock) void k_ep_p0(DevTissue t, const PosT *Xp, const PosT *Xm,
                                                  DevParams<PosT> p, double beta, double *g) {
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= t.n_cell) return;
    PosOverride<PosT> none{-1, -1, 0, 0, 0, 0};
    double a, pp, pm;
    cell_walk<PosT>(t, Xp, t.cell_he[c], none, a, pp);
    cell_walk<PosT>(t, Xm, t.cell_he[c], none, a, pm);
    g[c] = -2.0 * (double)p.kp(c) * (pp - pm) / beta;
}

// Sensitivity right-hand side -(d2E/dX dtheta) d for a parameter direction
// d.  theta = lambda: the line term's mixed derivative along d is the
// gradient of sum_e d_e l_e, so the RHS is the force of tensions d alone.
// theta = P0: d/dP0_c of 2K_P (P_c - P0_c) grad P_c is -2K_P grad P_c, so the
// RHS is minus the force of perimeter coefficients cP_c = 2K_P d_c alone.
// k_sens_cap writes those per-cell coefficients (cA = 0), k_sens_rhs forms
// the vertex force from them with the shared force code.
template <typename PosT>
__global__ __launch_bounds__(kBlock) void k_sens_cap(DevTissue t, DevParams<PosT> p,
                                                     const double *d, int theta, double *cap) {
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= t.n_cell) return;
    st2(cap, c, 0.0, theta == VTX_THETA_P0 ? 2.0 * (double)p.kp(c) * d[c] : 0.0);
}

template <typename PosT>
__global__ __launch_bounds__(kBlock) void k_sens_rhs(DevTissue t, const PosT *X,
                                                     DevParams<PosT> p, const double *cap,
                                                     double sgn, double *rhs) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= t.n_vert) return;
    Star<PosT, double> s;
    PosT xi, yi;
    load_star<PosT, double>(t, X, p, cap, v, s, xi, yi);
    double fx, fy;
    star_force<PosT, double>(s, fx, fy);
    st2(rhs, v, sgn * fx, sgn * fy);
}

// v2v cost and gradient (minimum image).
template <typename PosT>
__global__ __launch_bounds__(kBlock) void k_v2v(DevTissue t, const PosT *X, const PosT *Xt,
                                                double *grad, double *part, LoopCtl *ctl,
                                                double *C_out) {
    __shared__ double sh[kBlock / 64];
    double c = 0.0;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < t.n_vert; v += gridDim.x * kBlock) {
        const double dx = min_image((double)X[2 * (int64_t)v] - (double)Xt[2 * (int64_t)v], t.Lx);
        const double dy = min_image((double)X[2 * (int64_t)v + 1] - (double)Xt[2 * (int64_t)v + 1], t.Ly);
        c += dx * dx + dy * dy;
        if (grad) {
            grad[2 * (int64_t)v] = dx / (double)t.n_vert;
            grad[2 * (int64_t)v + 1] = dy / (double)t.n_vert;
        }
    }
    if (C_out) {
        const double bs = block_sum(c, sh);
        __shared__ int s_last;
        if (threadIdx.x == 0) {
            part[blockIdx.x] = bs;
            s_last = last_block(&ctl->arrive);
        }
        __syncthreads();
        if (s_last) {
            const double s = block_sum_array(part, gridDim.x, 1, sh);
            if (threadIdx.x == 0) *C_out = s / (2.0 * (double)t.n_vert);
        }
    }
}

// g . X: the linear nudge energy (g the double cost gradient, X the
// positions in their own precision) or a dot product of two double fields
template <typename PosT>
__global__ __launch_bounds__(kBlock) void k_dot_pos(const double *g, const PosT *X, int nv,
                                                    double *part, LoopCtl *ctl, double *out) {
    __shared__ double sh[kBlock / 64];
    double c = 0.0;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < nv; v += gridDim.x * kBlock)
        c += (double)g[2 * (int64_t)v] * (double)X[2 * (int64_t)v] +
             (double)g[2 * (int64_t)v + 1] * (double)X[2 * (int64_t)v + 1];
    const double bs = block_sum(c, sh);
    __shared__ int s_last;
    if (threadIdx.x == 0) {
        part[blockIdx.x] = bs;
        s_last = last_block(&ctl->arrive);
    }
    __syncthreads();
    if (s_last) {
        const double s = block_sum_array(part, gridDim.x, 1, sh);
        if (threadIdx.x == 0) *out = s;
    }
}

// mean of a position-typed 2-vector field (linear nudge) into mean_out
template <typename PosT>
__global__ __launch_bounds__(kBlock) void k_mean_pos(const PosT *a, int nv, double *part,
                                                     LoopCtl *ctl, double *mean_out) {
    __shared__ double sh[kBlock / 64];
    double sx = 0.0, sy = 0.0;
    for (int v = blockIdx.x * kBlock + threadIdx.x; v < nv; v += gridDim.x * kBlock) {
        sx += (double)a[2 * (int64_t)v];
        sy += (double)a[2 * (int64_t)v + 1];
    }
    const double bx = block_sum(sx, sh);
    const double by = block_sum(sy, sh);
    __shared__ int s_last;
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = bx;
        part[2 * blockIdx.x + 1] = by;
        s_last = last_block(&ctl->arrive2);
    }
    __syncthreads();
    if (s_last) {
        const double ax = block_sum_array(part, gridDim.x, 2, sh);
        const double ay = block_sum_array(part + 1, gridDim.x, 2, sh);
        if (threadIdx.x == 0) {
            mean_out[0] = ax / (double)nv;
            mean_out[1] = ay / (double)nv;
        }
    }
}

// ----------------------------------------------------------------- MINRES
// Minimum-residual Krylov solve of H x = P b for symmetric, possibly
// indefinite H (Paige and Saunders; the paper's solver for implicit
// differentiation).  Vectors (double [n_vert][2]) in the CG workspace:
// x, q (Lanczos vector q_k), qp (q_{k-1}), z (H q_k, then the next Lanczos
// direction), w1, w2 (the two previous search directions).  One step:
// z = H q with alpha = q.Hq fused into the HVP (k_hvp_vertex), then
// k_mr_lanczos (z -= alpha q + beta qp, beta' = |z|, the Givens rotation of
// the new tridiagonal column and the residual recurrence, in the last
// block), then k_mr_update (new search direction, x step, next q).
struct MinresVecs {
    double *x, *q, *qp, *z, *w1, *w2;
};

struct FinMrInit {
    __device__ void operator()(LoopCtl *ctl, double s2) const {
        const double b1 = sqrt(s2);
        ctl->mr_beta1 = b1;
        ctl->mr_phibar = b1;
        ctl->mr_beta = 0.0;
        ctl->mr_c1 = ctl->mr_c2 = 1.0;
        ctl->mr_s1 = ctl->mr_s2 = 0.0;
        ctl->mr_noop = 1;
        ctl->rel_res = b1 > 0.0 ? 1.0 : 0.0;
        if (!(b1 > 0.0)) {
            ctl->done = 1;
            ctl->status = VTX_CONVERGED;
        }
    }
};

// The new tridiagonal column (beta, alpha, beta_next) meets the two previous
// rotations, then a new rotation removes beta_next; the residual recurrence
// and the stopping tests follow.
struct FinMrLanczos {
    __device__ void operator()(LoopCtl *ctl, double s2) const {
        const double alpha = ctl->pAp, beta = ctl->mr_beta;
        const double beta_next = sqrt(s2);
        const double eps = ctl->mr_s2 * beta;
        const double dbar = ctl->mr_c2 * beta;
        const double delta = ctl->mr_c1 * dbar + ctl->mr_s1 * alpha;
        const double gbar = -ctl->mr_s1 * dbar + ctl->mr_c1 * alpha;
        const double gamma = sqrt(gbar * gbar + beta_next * beta_next);
        ctl->cg_iter += 1;
        if (!(gamma > 0.0)) {  // singular tridiagonal: no further progress
            ctl->mr_noop = 1;
            ctl->done = 1;
            ctl->status = ctl->rel_res <= ctl->tol ? VTX_CONVERGED : VTX_CG_MAXITER;
            return;
        }
        const double c = gbar / gamma, s = beta_next / gamma;
        ctl->mr_delta = delta;
        ctl->mr_eps = eps;
        ctl->mr_gamma = gamma;
        ctl->mr_tau = c * ctl->mr_phibar;
        ctl->mr_beta_next = beta_next;
        ctl->mr_phibar = -s * ctl->mr_phibar;
        ctl->mr_c2 = ctl->mr_c1;
        ctl->mr_s2 = ctl->mr_s1;
        ctl->mr_c1 = c;
        ctl->mr_s1 = s;
        ctl->mr_beta = beta_next;
        ctl->mr_noop = 0;
        const double rel = fabs(ctl->mr_phibar) / ctl->mr_beta1;
        ctl->rel_res = rel;
        if (rel <= ctl->tol) {
            ctl->done = 1;
            ctl->status = VTX_CONVERGED;
        } else if (!(beta_next > 0.0) || ctl->cg_iter >= ctl->max_iter) {
            ctl->done = 1;
            ctl->status = VTX_CG_MAXITER;
        }
    }
};

// z = P b (b minus its mean) into q, |P b|^2 -> beta1 and the initial state.
__global__ __launch_bounds__(kBlock) void k_mr_init(const double *__restrict__ b, int nv,
                                                    const double *mean, MinresVecs m,
                                                    double *__restrict__ part, LoopCtl *ctl) {
    __shared__ double sh[kBlock / 64];
    const int v = blockIdx.x * kBlock + threadIdx.x;
    double ss = 0.0;
    if (v < nv) {
        const int64_t k = 2 * (int64_t)v;
        const double rx = b[k] - mean[0], ry = b[k + 1] - mean[1];
        m.q[k] = rx;
        m.q[k + 1] = ry;
        ss = rx * rx + ry * ry;
    }
    reduce_tail(ss, part, ctl, sh, FinMrInit{});
}

// q /= beta1; x = qp = w1 = w2 = 0.
__global__ __launch_bounds__(kBlock) void k_mr_init2(int nv, MinresVecs m, const LoopCtl *ctl) {
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= nv) return;
    const double b1 = ctl->mr_beta1;
    const double inv = b1 > 0.0 ? 1.0 / b1 : 0.0;
    for (int c = 0; c < 2; ++c) {
        const int64_t k = 2 * (int64_t)v + c;
        m.q[k] *= inv;
        m.x[k] = m.qp[k] = m.w1[k] = m.w2[k] = 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void k_mr_lanczos(int nv, MinresVecs m,
                                                       double *__restrict__ part, LoopCtl *ctl) {
    if (ctl->done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) ctl->mr_noop = 1;
        return;
    }
    __shared__ double sh[kBlock / 64];
    const int v = blockIdx.x * kBlock + threadIdx.x;
    const double alpha = ctl->pAp, beta = ctl->mr_beta;
    double ss = 0.0;
    if (v < nv) {
        for (int c = 0; c < 2; ++c) {
            const int64_t k = 2 * (int64_t)v + c;
            const double zk = m.z[k] - (alpha * m.q[k] + beta * m.qp[k]);
            m.z[k] = zk;
            ss += zk * zk;
        }
    }
    reduce_tail(ss, part, ctl, sh, FinMrLanczos{});
}

__global__ __launch_bounds__(kBlock) void k_mr_update(int nv, MinresVecs m, const LoopCtl *ctl) {
    if (ctl->mr_noop) return;
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= nv) return;
    const double delta = ctl->mr_delta, eps = ctl->mr_eps, gamma = ctl->mr_gamma;
    const double tau = ctl->mr_tau, bn = ctl->mr_beta_next;
    for (int c = 0; c < 2; ++c) {
        const int64_t k = 2 * (int64_t)v + c;
        const double qk = m.q[k];
        const double w = (qk - delta * m.w1[k] - eps * m.w2[k]) / gamma;
        m.x[k] += tau * w;
        m.w2[k] = m.w1[k];
        m.w1[k] = w;
        m.qp[k] = qk;
        m.q[k] = bn > 0.0 ? m.z[k] / bn : 0.0;
    }
}

// ================================================================ launchers
static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <typename PosT>
static DevParams<PosT> dev_params(const ParamsRaw &r) {
    DevParams<PosT> p;
    p.KA = (const PosT *)r.KA;
    p.A0 = (const PosT *)r.A0;
    p.KP = (const PosT *)r.KP;
    p.P0 = (const PosT *)r.P0;
    p.lam = (const PosT *)r.lam;
    p.KA_s = (PosT)r.KA_s;
    p.A0_s = (PosT)r.A0_s;
    p.KP_s = (PosT)r.KP_s;
    p.P0_s = (PosT)r.P0_s;
    p.lam_s = (PosT)r.lam_s;
    return p;
}

template <typename PosT, typename M>
static void eval_impl(const DevTissue &t, const Workspace &w, const void *X, const ParamsRaw &pr,
                      double *E, void *F, double *maxf, hipStream_t s) {
    auto p = dev_params<PosT>(pr);
    LoopCtl *ectl = w.ctl + 1;
    const unsigned gc = blocks_for(t.n_cell), gv = blocks_for(t.n_vert);
    hipLaunchKernelGGL((k_cell<PosT, M>), dim3(gc), dim3(kBlock), 0, s, t, (const PosT *)X, p,
                       (M *)w.cap, w.partials, ectl, (int32_t *)nullptr, (M)0,
                       E ? (int)F_ENERGY : 0, (const PosT *)nullptr, (double *)nullptr);
    VertexArgs a{};
    a.ctl = ectl;
    a.epart_cell = w.partials;
    a.n_epart_cell = (int)gc;
    a.part = (double2 *)w.mpart;
    a.finish = gv <= (unsigned)kLastBlockMax;
    a.E_out = E;
    a.maxf_out = maxf;
    hipLaunchKernelGGL((k_vertex<PosT, M, 0>), dim3(gv), dim3(kBlock), 0, s, t, (const PosT *)X,
                       (PosT *)F, p, (const M *)w.cap, a);
    if (!a.finish && (E || maxf))
        hipLaunchKernelGGL((k_finish<0>), dim3(1), dim3(1024), 0, s, a, (int)gv);
}

template <typename PosT, typename M>
static void eval_fused_impl(const DevTissue &t, const Workspace &w, const TileTables &tt,
                            const void *X, const ParamsRaw &pr, double *E, void *F, double *maxf,
                            hipStream_t s) {
    auto p = dev_params<PosT>(pr);
    const unsigned g = (unsigned)n_tiles_for(t.n_vert);
    VertexArgs a{};
    a.ctl = w.ctl + 1;
    a.part = (double2 *)w.mpart;
    a.finish = g <= (unsigned)kLastBlockMax;
    a.E_out = E;
    a.maxf_out = maxf;
    hipLaunchKernelGGL((k_eval_fused<PosT, M>), dim3(g), dim3(kTileV), 0, s, t, (const PosT *)X,
                       (PosT *)F, p, tt, a);
    if (!a.finish && (E || maxf))
        hipLaunchKernelGGL((k_finish<0>), dim3(1), dim3(1024), 0, s, a, (int)g);
}

void launch_eval_fused(const DevTissue &t, const Workspace &w, const TileTables &tt, int mode,
                       const void *X, const ParamsRaw &p, double *E, void *F, double *maxf,
                       hipStream_t s) {
    if (mode == VTX_F32) eval_fused_impl<float, float>(t, w, tt, X, p, E, F, maxf, s);
    else if (mode == VTX_F64) eval_fused_impl<double, double>(t, w, tt, X, p, E, F, maxf, s);
    else eval_fused_impl<double, float>(t, w, tt, X, p, E, F, maxf, s);
}

void launch_tile_build(const DevTissue &t, const TileTables &tt, hipStream_t s) {
    const int64_t g = n_tiles_for(t.n_vert);
    if (g > 0) hipLaunchKernelGGL(k_tile_build, dim3((unsigned)g), dim3(kTileV), 0, s, t, tt);
}

void launch_eval(const DevTissue &t, const Workspace &w, int mode, const void *X,
                 const ParamsRaw &p, double *E, void *F, double *maxf, hipStream_t s) {
    if (mode == VTX_F32) eval_impl<float, float>(t, w, X, p, E, F, maxf, s);
    else if (mode == VTX_F64) eval_impl<double, double>(t, w, X, p, E, F, maxf, s);
    else eval_impl<double, float>(t, w, X, p, E, F, maxf, s);
}

template <typename PosT, typename M>
static void pass_impl(const DevTissue &t, const Workspace &w, const void *X, const ParamsRaw &pr,
                      void *coeffs, const void *coeffs_in, void *F, double *maxf, hipStream_t s) {
    auto p = dev_params<PosT>(pr);
    LoopCtl *ectl = w.ctl + 1;
    if (coeffs)
        hipLaunchKernelGGL((k_cell<PosT, M>), dim3(blocks_for(t.n_cell)), dim3(kBlock), 0, s, t,
                           (const PosT *)X, p, (M *)coeffs, (double *)nullptr, ectl,
                           (int32_t *)nullptr, (M)0, 0, (const PosT *)nullptr, (double *)nullptr);
    if (coeffs_in) {
        const unsigned gv = blocks_for(t.n_vert);
        VertexArgs a{};
        a.ctl = ectl;
        a.maxf_out = maxf;
        a.part = (double2 *)w.mpart;
        a.finish = gv <= (unsigned)kLastBlockMax;
        hipLaunchKernelGGL((k_vertex<PosT, M, 0>), dim3(gv), dim3(kBlock), 0, s, t,
                           (const PosT *)X, (PosT *)F, p, (const M *)coeffs_in, a);
        if (!a.finish && maxf)
            hipLaunchKernelGGL((k_finish<0>), dim3(1), dim3(1024), 0, s, a, (int)gv);
    }
}

void launch_cell_pass(const DevTissue &t, const Workspace &w, int mode, const void *X,
                      const ParamsRaw &p, void *coeffs, hipStream_t s) {
    if (mode == VTX_F32) pass_impl<float, float>(t, w, X, p, coeffs, nullptr, nullptr, nullptr, s);
    else if (mode == VTX_F64) pass_impl<double, double>(t, w, X, p, coeffs, nullptr, nullptr, nullptr, s);
    else pass_impl<double, float>(t, w, X, p, coeffs, nullptr, nullptr, nullptr, s);
}

void launch_vertex_pass(const DevTissue &t, const Workspace &w, int mode, const void *X,
                        const ParamsRaw &p, const void *coeffs, void *F, double *maxf,
                        hipStream_t s) {
    if (mode == VTX_F32) pass_impl<float, float>(t, w, X, p, nullptr, coeffs, F, maxf, s);
    else if (mode == VTX_F64) pass_impl<double, double>(t, w, X, p, nullptr, coeffs, F, maxf, s);
    else pass_impl<double, float>(t, w, X, p, nullptr, coeffs, F, maxf, s);
}

template <typename PosT, typename M>
static void relax_iter_impl(const DevTissue &t, const Workspace &w, void *Xc, void *Xn, int cur,
                            const ParamsRaw &pr, const RelaxArgs &ra, hipStream_t s) {
    auto p = dev_params<PosT>(pr);
    LoopCtl *ctl = w.ctl;
    const unsigned gc = blocks_for(t.n_cell), gv = blocks_for(t.n_vert);
    int flags = 0;
    if (ra.t1_enable) flags |= F_T1DET;
    if (ra.nudge == 1) flags |= F_NUDGE_V2V;
    // detection threshold slightly above l_min: the exact FP64 test is in k_t1
    const M lmin2 = (M)(ra.l_min * ra.l_min * (1.0 + 1e-4));
    hipLaunchKernelGGL((k_cell<PosT, M>), dim3(gc), dim3(kBlock), 0, s, t, (const PosT *)Xc, p,
                       (M *)w.cap, (double *)nullptr, ctl, w.t1_list, lmin2, flags,
                       (const PosT *)ra.X_target, w.partials);
    if (ra.t1_enable)
        hipLaunchKernelGGL((k_t1<PosT, M>), dim3(1), dim3(kBlock), 0, s, t, (PosT *)Xc, p,
                           (M *)w.cap, ctl, w.t1_list, ra.l_min, ra.l_new);
    VertexArgs a{};
    a.ctl = ctl;
    a.eta = ra.eta;
    a.cur = cur;
    a.nudge = ra.nudge;
    a.beta = ra.beta;
    a.Xt = ra.X_target;
    a.g_lin = ra.g_lin;
    a.part = (double2 *)w.mpart;
    a.finish = gv <= (unsigned)kLastBlockMax;
    hipLaunchKernelGGL((k_vertex<PosT, M, 1>), dim3(gv), dim3(kBlock), 0, s, t,
                       (const PosT *)Xc, (PosT *)Xn, p, (const M *)w.cap, a);
    if (!a.finish) hipLaunchKernelGGL((k_finish<1>), dim3(1), dim3(1024), 0, s, a, (int)gv);
}

void launch_relax_iter(const DevTissue &t, const Workspace &w, int mode, void *Xc, void *Xn,
                       int cur, const ParamsRaw &p, const RelaxArgs &ra, hipStream_t s) {
    if (mode == VTX_F32) relax_iter_impl<float, float>(t, w, Xc, Xn, cur, p, ra, s);
    else if (mode == VTX_F64) relax_iter_impl<double, double>(t, w, Xc, Xn, cur, p, ra, s);
    else relax_iter_impl<double, float>(t, w, Xc, Xn, cur, p, ra, s);
}

template <typename PosT, typename M>
static void t1_impl(const DevTissue &t, const Workspace &w, void *X, const ParamsRaw &pr,
                    double l_min, double l_new, hipStream_t s) {
    auto p = dev_params<PosT>(pr);
    LoopCtl *ectl = w.ctl + 1;
    const unsigned gc = blocks_for(t.n_cell);
    const M lmin2 = (M)(l_min * l_min * (1.0 + 1e-4));
    hipLaunchKernelGGL((k_cell<PosT, M>), dim3(gc), dim3(kBlock), 0, s, t, (const PosT *)X, p,
                       (M *)w.cap, (double *)nullptr, ectl, w.t1_list, lmin2, (int)F_T1DET,
                       (const PosT *)nullptr, (double *)nullptr);
    hipLaunchKernelGGL((k_t1<PosT, M>), dim3(1), dim3(kBlock), 0, s, t, (PosT *)X, p,
                       (M *)w.cap, ectl, w.t1_list, l_min, l_new);
}

void launch_t1(const DevTissue &t, const Workspace &w, int mode, void *X, const ParamsRaw &p,
               double l_min, double l_new, hipStream_t s) {
    if (mode == VTX_F32) t1_impl<float, float>(t, w, X, p, l_min, l_new, s);
    else if (mode == VTX_F64) t1_impl<double, double>(t, w, X, p, l_min, l_new, s);
    else t1_impl<double, float>(t, w, X, p, l_min, l_new, s);
}

template <typename PosT, typename M>
static void cap_impl(const DevTissue &t, const Workspace &w, const void *X, const ParamsRaw &pr,
                     hipStream_t s) {
    auto p = dev_params<PosT>(pr);
    hipLaunchKernelGGL((k_cell<PosT, M>), dim3(blocks_for(t.n_cell)), dim3(kBlock), 0, s, t,
                       (const PosT *)X, p, (M *)w.cap, (double *)nullptr, w.ctl + 1,
                       (int32_t *)nullptr, (M)0, 0, (const PosT *)nullptr, (double *)nullptr);
}

void launch_cell_coeffs(const DevTissue &t, const Workspace &w, int mode, const void *X,
                        const ParamsRaw &p, hipStream_t s) {
    if (mode == VTX_F32) cap_impl<float, float>(t, w, X, p, s);
    else if (mode == VTX_F64) cap_impl<double, double>(t, w, X, p, s);
    else cap_impl<double, float>(t, w, X, p, s);
}

template <typename PosT, typename M>
static void hvp_impl(const DevTissue &t, const Workspace &w, const void *X, const ParamsRaw &pr,
                     const double *v, double *Hv, double *dpart, LoopCtl *ctl, hipStream_t s) {
    auto p = dev_params<PosT>(pr);
    hipLaunchKernelGGL((k_hvp_cell<PosT, M>), dim3(blocks_for(t.n_cell)), dim3(kBlock), 0, s, t,
                       (const PosT *)X, p, v, (M *)w.cell_aux, ctl);
    const unsigned gv = blocks_for(t.n_vert);
    hipLaunchKernelGGL((k_hvp_vertex<PosT, M>), dim3(gv), dim3(kBlock), 0, s, t,
                       (const PosT *)X, p, (const M *)w.cap, (const M *)w.cell_aux, v, Hv,
                       dpart, ctl);
    if (dpart) launch_fin(gv, dpart, ctl, FinPAp{}, s);
}

void launch_hvp(const DevTissue &t, const Workspace &w, int mode, const void *X,
                const ParamsRaw &p, const double *v, double *Hv, double *dpart, LoopCtl *ctl,
                hipStream_t s) {
    if (mode == VTX_F32) hvp_impl<float, float>(t, w, X, p, v, Hv, dpart, ctl, s);
    else if (mode == VTX_F64) hvp_impl<double, double>(t, w, X, p, v, Hv, dpart, ctl, s);
    else hvp_impl<double, float>(t, w, X, p, v, Hv, dpart, ctl, s);
}

void launch_cg_init(const Workspace &w, int nv, const double *b, hipStream_t s) {
    double *x = w.cg, *r = w.cg + 2 * (int64_t)nv, *q = w.cg + 4 * (int64_t)nv;
    const unsigned gv = blocks_for(nv);
    const unsigned gm = gv < (unsigned)kRedBlocks ? gv : (unsigned)kRedBlocks;
    hipLaunchKernelGGL(k_mean2, dim3(gm), dim3(kBlock), 0, s, b, nv, w.partials2, w.ctl,
                       w.scal);
    hipLaunchKernelGGL(k_cg_init, dim3(gv), dim3(kBlock), 0, s, b, nv, (const double *)w.scal,
                       x, r, q, w.partials, w.ctl);
    launch_fin(gv, w.partials, w.ctl, FinCgInit{}, s);
}

void launch_cg_iter(const DevTissue &t, const Workspace &w, int mode, const void *X,
                    const ParamsRaw &p, hipStream_t s) {
    const int nv = t.n_vert;
    double *x = w.cg, *r = w.cg + 2 * (int64_t)nv, *q = w.cg + 4 * (int64_t)nv,
           *Aq = w.cg + 6 * (int64_t)nv;
    launch_hvp(t, w, mode, X, p, q, Aq, w.partials, w.ctl, s);
    const unsigned gv = blocks_for(nv);
    hipLaunchKernelGGL(k_cg_update, dim3(gv), dim3(kBlock), 0, s, x, r, (const double *)q,
                       (const double *)Aq, nv, w.partials, w.ctl);
    launch_fin(gv, w.partials, w.ctl, FinCgUpdate{}, s);
    hipLaunchKernelGGL(k_cg_dir, dim3(gv), dim3(kBlock), 0, s, (const double *)r, q, nv, w.ctl);
}

static MinresVecs minres_vecs(const Workspace &w, int nv) {
    const int64_t n = 2 * (int64_t)nv;
    return MinresVecs{w.cg, w.cg + n, w.cg + 2 * n, w.cg + 3 * n, w.cg + 4 * n, w.cg + 5 * n};
}

void launch_minres_init(const Workspace &w, int nv, const double *b, hipStream_t s) {
    const unsigned gv = blocks_for(nv);
    const unsigned gm = gv < (unsigned)kRedBlocks ? gv : (unsigned)kRedBlocks;
    const MinresVecs m = minres_vecs(w, nv);
    hipLaunchKernelGGL(k_mean2, dim3(gm), dim3(kBlock), 0, s, b, nv, w.partials2, w.ctl,
                       w.scal);
    hipLaunchKernelGGL(k_mr_init, dim3(gv), dim3(kBlock), 0, s, b, nv, (const double *)w.scal,
                       m, w.partials, w.ctl);
    launch_fin(gv, w.partials, w.ctl, FinMrInit{}, s);
    hipLaunchKernelGGL(k_mr_init2, dim3(gv), dim3(kBlock), 0, s, nv, m, (const LoopCtl *)w.ctl);
}

void launch_minres_iter(const DevTissue &t, const Workspace &w, int mode, const void *X,
                        const ParamsRaw &p, hipStream_t s) {
    const int nv = t.n_vert;
    const MinresVecs m = minres_vecs(w, nv);
    launch_hvp(t, w, mode, X, p, m.q, m.z, w.partials, w.ctl, s);
    const unsigned gv = blocks_for(nv);
    hipLaunchKernelGGL(k_mr_lanczos, dim3(gv), dim3(kBlock), 0, s, nv, m, w.partials, w.ctl);
    launch_fin(gv, w.partials, w.ctl, FinMrLanczos{}, s);
    hipLaunchKernelGGL(k_mr_update, dim3(gv), dim3(kBlock), 0, s, nv, m, (const LoopCtl *)w.ctl);
}

void launch_project(const Workspace &w, int nv, double *x, hipStream_t s) {
    const unsigned gv = blocks_for(nv);
    const unsigned gm = gv < (unsigned)kRedBlocks ? gv : (unsigned)kRedBlocks;
    hipLaunchKernelGGL(k_mean2, dim3(gm), dim3(kBlock), 0, s, (const double *)x, nv, w.partials2,
                       w.ctl + 1, w.scal + 2);
    hipLaunchKernelGGL(k_sub_mean, dim3(gv), dim3(kBlock), 0, s, (const double *)x, x, nv,
                       (const double *)(w.scal + 2));
}

template <typename PosT>
static void contract_impl(const DevTissue &t, const void *X, const ParamsRaw &pr, int theta,
                          const double *mu, double *g, hipStream_t s) {
    if (theta == VTX_THETA_LAMBDA)
        hipLaunchKernelGGL((k_contract_lambda<PosT>), dim3(blocks_for(t.n_edge)), dim3(kBlock), 0,
                           s, t, (const PosT *)X, mu, g);
    else
        hipLaunchKernelGGL((k_contract_p0<PosT>), dim3(blocks_for(t.n_cell)), dim3(kBlock), 0, s,
                           t, (const PosT *)X, dev_params<PosT>(pr), mu, g);
}

void launch_contract(const DevTissue &t, int mode, const void *X, const ParamsRaw &p, int theta,
                     const double *mu, double *g, hipStream_t s) {
    if (mode == VTX_F32) contract_impl<float>(t, X, p, theta, mu, g, s);
    else contract_impl<double>(t, X, p, theta, mu, g, s);
}

template <typename PosT>
static void ep_impl(const DevTissue &t, const void *Xp, const void *Xm, const ParamsRaw &pr,
                    int theta, double beta, double *g, hipStream_t s) {
    if (theta == VTX_THETA_LAMBDA)
        hipLaunchKernelGGL((k_ep_lambda<PosT>), dim3(blocks_for(t.n_edge)), dim3(kBlock), 0, s, t,
                           (const PosT *)Xp, (const PosT *)Xm, beta, g);
    else
        hipLaunchKernelGGL((k_ep_p0<PosT>), dim3(blocks_for(t.n_cell)), dim3(kBlock), 0, s, t,
                           (const PosT *)Xp, (const PosT *)Xm, dev_params<PosT>(pr), beta, g);
}

void launch_ep(const DevTissue &t, int mode, const void *Xp, const void *Xm, const ParamsRaw &p,
               int theta, double beta, double *g, hipStream_t s) {
    if (mode == VTX_F32) ep_impl<float>(t, Xp, Xm, p, theta, beta, g, s);
    else ep_impl<double>(t, Xp, Xm, p, theta, beta, g, s);
}

void launch_edge_len(const DevTissue &t, int mode, const void *X, double *len, hipStream_t s) {
    if (mode == VTX_F32)
        hipLaunchKernelGGL((k_edge_len<float>), dim3(blocks_for(t.n_edge)), dim3(kBlock), 0, s, t,
                           (const float *)X, len);
    else
        hipLaunchKernelGGL((k_edge_len<double>), dim3(blocks_for(t.n_edge)), dim3(kBlock), 0, s, t,
                           (const double *)X, len);
}

void launch_cell_exact(const DevTissue &t, int mode, const void *X, double *A, double *P,
                       hipStream_t s) {
    if (mode == VTX_F32)
        hipLaunchKernelGGL((k_cell_exact<float>), dim3(blocks_for(t.n_cell)), dim3(kBlock), 0, s,
                           t, (const float *)X, A, P);
    else
        hipLaunchKernelGGL((k_cell_exact<double>), dim3(blocks_for(t.n_cell)), dim3(kBlock), 0, s,
                           t, (const double *)X, A, P);
}

void launch_v2v(const DevTissue &t, const Workspace &w, int mode, const void *X, const void *Xt,
                double *C, double *grad, hipStream_t s) {
    const unsigned gv0 = blocks_for(t.n_vert);
    const unsigned gv = gv0 < (unsigned)kRedBlocks ? gv0 : (unsigned)kRedBlocks;
    if (mode == VTX_F32)
        hipLaunchKernelGGL((k_v2v<float>), dim3(gv), dim3(kBlock), 0, s, t, (const float *)X,
                           (const float *)Xt, grad, w.partials2, w.ctl + 1, C);
    else
        hipLaunchKernelGGL((k_v2v<double>), dim3(gv), dim3(kBlock), 0, s, t, (const double *)X,
                           (const double *)Xt, grad, w.partials2, w.ctl + 1, C);
}

void launch_sens_rhs(const DevTissue &t, const Workspace &w, const void *X, const ParamsRaw &pr,
                     int theta, const double *d, double *rhs, hipStream_t s) {
    // double positions only (VTX_F64 / VTX_MIXED)
    DevParams<double> p = dev_params<double>(pr);
    hipLaunchKernelGGL(k_sens_cap<double>, dim3(blocks_for(t.n_cell)), dim3(kBlock), 0, s, t, p,
                       d, theta, w.cell_aux);
    DevParams<double> q = p;
    q.lam = theta == VTX_THETA_LAMBDA ? d : nullptr;
    q.lam_s = 0.0;
    hipLaunchKernelGGL(k_sens_rhs<double>, dim3(blocks_for(t.n_vert)), dim3(kBlock), 0, s, t,
                       (const double *)X, q, (const double *)w.cell_aux,
                       theta == VTX_THETA_LAMBDA ? 1.0 : -1.0, rhs);
}

void launch_dot_pos(const Workspace &w, int mode, int nv, const double *g, const void *X,
                    double *out, hipStream_t s) {
    const unsigned gv0 = blocks_for(nv);
    const unsigned gv = gv0 < (unsigned)kRedBlocks ? gv0 : (unsigned)kRedBlocks;
    if (mode == VTX_F32)
        hipLaunchKernelGGL((k_dot_pos<float>), dim3(gv), dim3(kBlock), 0, s, g,
                           (const float *)X, nv, w.partials2, w.ctl + 1, out);
    else
        hipLaunchKernelGGL((k_dot_pos<double>), dim3(gv), dim3(kBlock), 0, s, g,
                           (const double *)X, nv, w.partials2, w.ctl + 1, out);
}

void launch_mean_pos(const Workspace &w, int mode, int nv, const void *a, double *mean_out,
                     hipStream_t s) {
    const unsigned gv = blocks_for(nv);
    const unsigned gm = gv < (unsigned)kRedBlocks ? gv : (unsigned)kRedBlocks;
    if (mode == VTX_F32)
        hipLaunchKernelGGL((k_mean_pos<float>), dim3(gm), dim3(kBlock), 0, s, (const float *)a, nv,
                           w.partials2, w.ctl + 1, mean_out);
    else
        hipLaunchKernelGGL((k_mean_pos<double>), dim3(gm), dim3(kBlock), 0, s, (const double *)a,
                           nv, w.partials2, w.ctl + 1, mean_out);
}

}  // namespace vtx
