// Batched relaxation of many independent periodic tissues in one persistent
// launch (VertAX, arXiv 2604.06896, Methods, "Simulation engine", applied
// per tissue).  One workgroup owns one tissue at a time and runs the whole
// loop -- cell pass, T1 pass, vertex pass with the gradient-descent step,
// convergence test -- with workgroup barriers only; tissues are taken from a
// device work queue in descending size so the largest start first.
#include <algorithm>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include "vtx_device.h"
#include "vtx_launch.h"

using namespace vtx;

struct vtx_tissue_s;  // defined in vtx_api.hip; only its handle is used here

namespace vtx {
// Accessors implemented in vtx_api.hip.
const DevTissue &tissue_dev(vtx_tissue t);
const Workspace &tissue_ws(vtx_tissue t);
int64_t tissue_size(vtx_tissue t);
int set_error(int code, const char *msg);
}  // namespace vtx

struct vtx_batch_s {
    std::vector<vtx_tissue> ts;
    std::vector<int32_t> order;  // tissue indices by descending size
    void *items;                 // device BatchItem[n]
    int32_t *order_d;
    unsigned int *queue;
    vtx_relax_result *res_d;
    hipStream_t cap_stream;
};

namespace vtx {

struct BatchItem {
    DevTissue t;
    void *X;
    void *xbuf;
    void *cap;
    int32_t *t1_list;
    ParamsRaw p;
};

struct BatchOpts {
    double eta, tol, l_min, l_new;
    int64_t patience, max_iter;
    int t1_enable;
};

template <typename PosT>
__device__ __forceinline__ DevParams<PosT> to_dev(const ParamsRaw &r) {
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

__global__ void k_reset_queue(unsigned int *q) { *q = 0u; }

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
    __shared__ int s_item, s_done, s_changed, s_rbuf;
    const M lmin2 = (M)(o.l_min * o.l_min * (1.0 + 1e-4));
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int slot = s_item;
        __syncthreads();
        if (slot >= n) return;
        const int idx = order[slot];
        const BatchItem &B = items[idx];
        const DevTissue t = B.t;
        const DevParams<PosT> p = to_dev<PosT>(B.p);
        PosT *bufs[2] = {(PosT *)B.X, (PosT *)B.xbuf};
        M *cap = (M *)B.cap;
        int cur = 0;
        int64_t iter = 0, count = 0, n_t1 = 0, n_st = 0;
        int status = VTX_NOT_CONVERGED, result_buf = 0;
        double last_mf = 0.0;
        for (;;) {
            PosT *Xc = bufs[cur], *Xn = bufs[cur ^ 1];
            if (threadIdx.x == 0) s_cnt = 0u;
            __syncthreads();
            // cell pass
            for (int c = threadIdx.x; c < t.n_cell; c += blockDim.x) {
                const int rb = t.row_ptr[c], nn = t.row_ptr[c + 1] - rb;
                PosT A, P;  // in the position precision, as in the grid kernels
                cell_geom<PosT, PosT>(
                    t, Xc, nn, [&](int k) { return t.corner[rb + k]; }, rb, A, P,
                    o.t1_enable != 0, (PosT)lmin2, B.t1_list, &s_cnt);
                st2(cap, c, (M)((PosT)2 * p.ka(c) * (A - p.a0(c))),
                    (M)((PosT)2 * p.kp(c) * (P - p.p0(c))));
            }
            __syncthreads();
            // T1 pass
            const int ncand = (int)s_cnt;
            if (ncand > 0) {
                int np2 = 1;
                while (np2 < ncand) np2 <<= 1;
                int32_t *arr = np2 <= kT1SortCap ? sort_buf : B.t1_list;
                for (int i = threadIdx.x; i < np2; i += blockDim.x)
                    arr[i] = i < ncand ? t.he_edge[t.corner_he[B.t1_list[i]]] : INT_MAX;
                __syncthreads();
                block_bitonic(arr, np2);
                if (threadIdx.x == 0) {
                    T1Counts r = t1_sequential<PosT, M>(t, Xc, p, cap, arr, ncand, extra,
                                                        o.l_min, o.l_new);
                    n_t1 += r.swaps;
                    n_st += r.stretches;
                    s_changed = r.changed;
                }
                __syncthreads();
                if (s_changed) rebuild_rows_block(t, scan);
                __syncthreads();
            }
            // vertex pass with the step
            double mf = 0.0;
            for (int v = threadIdx.x; v < t.n_vert; v += blockDim.x) {
                Star<PosT, M> s;
                PosT xi, yi;
                load_star<PosT, M>(t, Xc, p, cap, v, s, xi, yi);
                M fx, fy;
                star_force<PosT, M>(s, fx, fy);
                mf = fmax(mf, fmax(fabs((double)fx), fabs((double)fy)));
                if (!(fx == fx) || !(fy == fy)) mf = INFINITY;
                st2(Xn, v, (PosT)((double)xi + o.eta * (double)fx),
                    (PosT)((double)yi + o.eta * (double)fy));
            }
            const double m = block_max(mf, sh);
            if (threadIdx.x == 0) {
                ++iter;
                last_mf = m;
                int done = 0;
                if (!(m <= 1.7976931348623157e308)) {
                    done = 1;
                    status = VTX_E_NONFINITE;
                    result_buf = cur;
                } else {
                    count = m < o.tol ? count + 1 : 0;
                    if (count >= o.patience) {
                        done = 1;
                        status = VTX_CONVERGED;
                        result_buf = cur;
                    } else if (iter >= o.max_iter) {
                        done = 1;
                        status = VTX_NOT_CONVERGED;
                        result_buf = cur ^ 1;
                    }
                }
                s_done = done;
                s_rbuf = result_buf;
            }
            __syncthreads();
            if (s_done) break;
            cur ^= 1;
        }
        const int rbuf = s_rbuf;
        if (rbuf == 1)
            for (int k = threadIdx.x; k < 2 * t.n_vert; k += blockDim.x)
                ((PosT *)B.X)[k] = ((PosT *)B.xbuf)[k];
        __syncthreads();
        // energy at the returned positions
        double e = 0.0;
        const PosT *Xr = (const PosT *)B.X;
        for (int c = threadIdx.x; c < t.n_cell; c += blockDim.x) {
            const int rb = t.row_ptr[c], nn = t.row_ptr[c + 1] - rb;
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
        const double E = block_sum(e, sh);
        if (threadIdx.x == 0) {
            vtx_relax_result r;
            r.iters = iter;
            r.n_t1 = n_t1;
            r.n_stretch = n_st;
            r.max_f = last_mf;
            r.energy = E;
            r.status = status;
            res[idx] = r;
        }
        __syncthreads();
    }
}

}  // namespace vtx

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
    hipError_t e = hipMalloc(&b->items, sizeof(BatchItem) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&b->order_d, sizeof(int32_t) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&b->queue, sizeof(unsigned int));
    if (e == hipSuccess) e = hipMalloc((void **)&b->res_d, sizeof(vtx_relax_result) * n);
    if (e == hipSuccess)
        e = hipMemcpy(b->order_d, b->order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        vtx_batch_destroy(b);
        return set_error(VTX_E_HIP, hipGetErrorString(e));
    }
    *out = b;
    return VTX_OK;
}

int vtx_batch_destroy(vtx_batch b) {
    if (!b) return set_error(VTX_E_ARG, "null batch");
    (void)hipDeviceSynchronize();
    if (b->items) (void)hipFree(b->items);
    if (b->order_d) (void)hipFree(b->order_d);
    if (b->queue) (void)hipFree(b->queue);
    if (b->res_d) (void)hipFree(b->res_d);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return VTX_OK;
}

int vtx_batch_relax(vtx_batch b, int32_t mode, void *const *X, const vtx_params *p,
                    const vtx_relax_opts *o, int32_t schedule, int32_t block_threads,
                    vtx_relax_result *res, void *stream) {
    if (!b || !X || !p || !o || !res) return set_error(VTX_E_ARG, "null argument");
    if (mode != VTX_F32 && mode != VTX_F64 && mode != VTX_MIXED)
        return set_error(VTX_E_ARG, "bad precision mode");
    if (schedule != 0) return set_error(VTX_E_ARG, "only schedule 0 (block per tissue) exists");
    if (block_threads != 256 && block_threads != 512 && block_threads != 1024)
        return set_error(VTX_E_ARG, "block_threads must be 256, 512 or 1024");
    if (o->beta != 0.0) return set_error(VTX_E_ARG, "batched relaxation takes no nudge");
    if (!(o->eta > 0) || !(o->tol >= 0) || o->patience < 1 || o->max_iter < 1)
        return set_error(VTX_E_ARG, "bad relax options");
    if (o->t1_enable && !(o->l_min > 0 && o->l_new > 0))
        return set_error(VTX_E_ARG, "T1 needs l_min > 0 and l_new > 0");
    const int n = (int)b->ts.size();
    std::vector<BatchItem> items(n);
    for (int i = 0; i < n; ++i) {
        if (!X[i]) return set_error(VTX_E_ARG, "null X in batch");
        const Workspace &w = tissue_ws(b->ts[i]);
        items[i].t = tissue_dev(b->ts[i]);
        items[i].X = X[i];
        items[i].xbuf = w.xbuf;
        items[i].cap = w.cap;
        items[i].t1_list = w.t1_list;
        const vtx_params &q = p[i];
        items[i].p = ParamsRaw{q.KA, q.A0, q.KP, q.P0, q.lam, q.KA_s, q.A0_s, q.KP_s, q.P0_s, q.lam_s};
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(b->items, items.data(), sizeof(BatchItem) * n,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return set_error(VTX_E_HIP, hipGetErrorString(e));
    BatchOpts bo{o->eta, o->tol, o->l_min, o->l_new, o->patience, o->max_iter, o->t1_enable};
    // reset of the queue + the persistent launch, captured once as a graph
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return set_error(VTX_E_HIP, hipGetErrorString(e));
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(1), 0, b->cap_stream, b->queue);
    const BatchItem *it = (const BatchItem *)b->items;
    const dim3 grid(n), block(block_threads);
    if (mode == VTX_F32)
        hipLaunchKernelGGL((k_batch_relax<float, float>), grid, block, 0, b->cap_stream, it,
                           b->order_d, n, b->queue, bo, b->res_d);
    else if (mode == VTX_F64)
        hipLaunchKernelGGL((k_batch_relax<double, double>), grid, block, 0, b->cap_stream, it,
                           b->order_d, n, b->queue, bo, b->res_d);
    else
        hipLaunchKernelGGL((k_batch_relax<double, float>), grid, block, 0, b->cap_stream, it,
                           b->order_d, n, b->queue, bo, b->res_d);
    e = hipStreamEndCapture(b->cap_stream, &g);
    if (e != hipSuccess) return set_error(VTX_E_HIP, hipGetErrorString(e));
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(ge, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(res, b->res_d, sizeof(vtx_relax_result) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) return set_error(VTX_E_HIP, hipGetErrorString(e));
    for (int i = 0; i < n; ++i)
        if (res[i].status == VTX_E_NONFINITE) {
            res[i].status = VTX_NOT_CONVERGED;
            return set_error(VTX_E_NONFINITE, "non-finite forces in a batched relaxation");
        }
    return VTX_OK;
}

}  // extern "C"
