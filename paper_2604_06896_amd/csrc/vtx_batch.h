// Declarations shared by the batched sources of libvtx: the per-tissue work
// items of the persistent batch kernels, their options, and block-level
// helpers.
#pragma once

#include "vtx_device.h"
#include "vtx_launch.h"

struct vtx_tissue_s;  // defined in vtx_api.hip; only its handle is used here

namespace vtx {
// Accessors implemented in vtx_api.hip.
const DevTissue &tissue_dev(vtx_tissue t);
const Workspace &tissue_ws(vtx_tissue t);
int64_t tissue_size(vtx_tissue t);
int64_t tissue_cells(vtx_tissue t);
double *tissue_ep_buf(vtx_tissue t);
int set_error(int code, const char *msg);
// Rebuild the tissue's fused-evaluation tables after its topology changed
// (on stream s, in order with the change).
int tissue_topology_changed(vtx_tissue t, hipStream_t s);
}  // namespace vtx

namespace vtx {

struct BatchItem {
    DevTissue t;
    void *X;
    void *xbuf;
    void *cap;
    int32_t *t1_list;
    ParamsRaw p;
    // nudge (equilibrium propagation): beta * C with C the v2v cost to Xt or
    // the linear cost g_lin . X; the mean of grad C is removed
    const void *Xt;
    const double *g_lin;
    double beta;
};

// One tissue of a batched adjoint: H mu = P b by CG, then the contraction.
struct GradItem {
    DevTissue t;
    const void *X;
    ParamsRaw p;
    const double *b;     // dC/dX [n_vert][2]
    double *cg;          // x, r, q, Aq: 4 x [n_vert][2]
    void *cap;
    void *aux;
    double *g;           // output [n_edge] or [n_cell]
};

struct GradOpts {
    double tol;
    int64_t max_iter;
    int theta;
    int minres;  // 0: CG, 1: MINRES
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

// Block-wide sum returned to every thread: the wave sums go to LDS and every
// thread adds them in wave order, so the result equals block_sum's (thread
// 0's) in all threads without a broadcast round.
__device__ __forceinline__ double block_allsum(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();  // `sh` may still be read by the previous reduction
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) r += sh[w];
    return r;
}

// Two block_allsum sums with one pair of barriers (each component added in
// the same order as block_allsum's); workgroups of up to 512 threads, `sh`
// holds 16 doubles.
__device__ __forceinline__ double2 block_allsum2(double a, double b, double *sh) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();  // `sh` may still be read by the previous reduction
    if (lane == 0) {
        sh[wid] = a;
        sh[8 + wid] = b;
    }
    __syncthreads();
    double ra = 0.0, rb = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) {
        ra += sh[w];
        rb += sh[8 + w];
    }
    return double2{ra, rb};
}

// Exclusive prefix sum of one int per thread over the workgroup (up to 16
// waves); `sh` holds 16 ints.  Also returns the total.
__device__ __forceinline__ int block_exclusive_scan(int v, int *sh, int &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int s = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(s, off, 64);
        if (lane >= off) s += u;
    }
    if (lane == 63 || threadIdx.x == blockDim.x - 1) sh[w] = s;
    __syncthreads();
    int base = 0, tot = 0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) {
        const int x = sh[i];
        if (i < w) base += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return base + s - v;
}

}  // namespace vtx

namespace vtx {
// Batched adjoint with each tissue split over K workgroups (vtx_batch_mb.hip).
int mb_no_fit_status();
size_t mb_group_bytes();
hipError_t mb_capacity(int *max_blocks, int *lds_bytes);
hipError_t mb_launch(const GradItem *items, const int32_t *order, int n, const GradOpts &o,
                     int K, int n_groups, int lds_bytes, vtx_grad_result *res_d, void *groups,
                     hipStream_t s);
// Batched relaxation without T1 with each tissue split over K workgroups.
hipError_t mb_relax_capacity(int mode, int *max_blocks, int *lds_bytes);
hipError_t mb_relax_launch(int mode, const BatchItem *items, const int32_t *order, int n,
                           const BatchOpts &o, int K, int n_groups, int lds_bytes,
                           vtx_relax_result *res_d, void *groups, hipStream_t s);
}  // namespace vtx
