// Internal declarations shared by the HIP sources of libvtx (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vtx.h"

namespace vtx {

// ------------------------------------------------------------------ packing
// Vertex ids carry a 4-bit periodic image code in their top bits:
// bits 28-29 hold (ox + 1), bits 30-31 hold (oy + 1).
constexpr int kIdBits = 28;
constexpr uint32_t kIdMask = (1u << kIdBits) - 1u;
constexpr int kBlock = 256;          // threads per block of the grid kernels
constexpr int kT1SortCap = 4096;     // T1 candidates sorted in LDS
constexpr int kT1Extra = 256;        // pending re-checks during one T1 pass
constexpr int kRedBlocks = 128;      // grid of the grid-stride reduction kernels
constexpr int kRowSlack = 2;         // spare slots per row after a compaction
constexpr int kRowExtra = 4;         // spare slots of a row moved to the pool

// Status of an estimate built from two relaxations: an error (negative)
// wins, otherwise the worse of the two outcomes.
__host__ __device__ inline int combine_status(int a, int b) {
    return (a < 0 || b < 0) ? (a < b ? a : b) : (a > b ? a : b);
}

__host__ __device__ inline int32_t pack_id(int32_t id, int ox, int oy) {
    return (int32_t)((uint32_t)id | ((uint32_t)((ox + 1) | ((oy + 1) << 2)) << kIdBits));
}
__host__ __device__ inline int32_t id_of(int32_t w) { return (int32_t)((uint32_t)w & kIdMask); }
__host__ __device__ inline int ox_of(int32_t w) { return (int)(((uint32_t)w >> kIdBits) & 3u) - 1; }
__host__ __device__ inline int oy_of(int32_t w) {
    return (int)(((uint32_t)w >> (kIdBits + 2)) & 3u) - 1;
}

enum { HP = 0, HN, HT, HS, HG, HF, HOX, HOY };  // half-edge table columns

// ------------------------------------------------------- device structures
struct DevTissue {
    int32_t n_vert, n_cell, n_edge, n_he;
    double Lx, Ly;
    int32_t *he;         // [n_he][8] current topology
    int32_t *he_edge;    // [n_he] edge id of each half-edge
    int32_t *edge_he;    // [n_edge] lower half-edge of each edge
    int32_t *row_ptr;    // [n_cell + 1] start of each cell's corner row
    int32_t *row_cap;    // [n_cell] slots of each row (nsides[c] corners + spare)
    int32_t *pool_top;   // device int: next free slot of the relocation pool
    int32_t pool_start;  // first slot of the pool (rows above it are relocated)
    int32_t corner_cap;  // slots in corner / corner_he
    int32_t *corner;     // [n_he] packed vertex id + image relative to corner 0
    int32_t *corner_he;  // [n_he] half-edge leaving each corner
    int32_t *nsides;     // [n_cell]
    int32_t *cell_he;    // [n_cell] one half-edge of each cell
    // Vertex stars (3 counter-clockwise slots k per vertex): neighbour nb_k
    // (packed id + image), sector cell c_k (between neighbours k and k+1) and
    // edge e_k, packed so that the vertex pass reads them with three loads:
    //   [0, 4n)   int4 per vertex {nb_0, nb_1, nb_2, c_0}
    //   [4n, 8n)  int4 per vertex {c_1, c_2, e_0, e_1}
    //   [8n, 9n)  e_2
    // (see star_nb_at / star_cell_at / star_edge_at).
    int32_t *star;
    int32_t *star_he;    // [3][n_vert] outgoing half-edges, counter-clockwise
};

__host__ __device__ inline int64_t star_nb_at(int64_t /*n*/, int k, int64_t v) { return 4 * v + k; }
__host__ __device__ inline int64_t star_cell_at(int64_t n, int k, int64_t v) {
    return k == 0 ? 4 * v + 3 : 4 * n + 4 * v + (k - 1);
}
__host__ __device__ inline int64_t star_edge_at(int64_t n, int k, int64_t v) {
    return k < 2 ? 4 * n + 4 * v + 2 + k : 8 * n + v;
}

template <typename P>
struct DevParams {
    const P *KA, *A0, *KP, *P0, *lam;
    P KA_s, A0_s, KP_s, P0_s, lam_s;
    __device__ __forceinline__ P ka(int c) const { return KA ? KA[c] : KA_s; }
    __device__ __forceinline__ P a0(int c) const { return A0 ? A0[c] : A0_s; }
    __device__ __forceinline__ P kp(int c) const { return KP ? KP[c] : KP_s; }
    __device__ __forceinline__ P p0(int c) const { return P0 ? P0[c] : P0_s; }
    __device__ __forceinline__ P lm(int e) const { return lam ? lam[e] : lam_s; }
};

// Device control block of an iterative loop (relaxation or CG).  Only the
// library's kernels touch it; the host reads it between graph launches.
struct LoopCtl {
    unsigned int arrive;           // blocks of the current launch that finished
    unsigned int arrive2;
    int32_t done;
    int32_t status;
    int32_t result_buf;            // 0: caller's X, 1: library buffer
    int32_t topo_changed;
    int64_t iter;
    int64_t max_iter, patience, count;
    double tol;
    double last_maxf;
    int64_t n_t1, n_stretch;
    uint32_t t1_count;             // candidates appended in the current pass
    int32_t t1_overflow;
    double nudge_mean[2];
    // CG scalars
    double rr, rr0, pAp, alpha, beta_cg, rel_res;
    int64_t cg_iter;
    // MINRES scalars (solver 1): Lanczos off-diagonal, the two previous
    // Givens rotations, the residual recurrence, and the step's update
    int32_t solver;                // 0: CG (curvature check in the HVP), 1: MINRES
    int32_t mr_noop;               // the update kernel of this step has nothing to do
    double mr_beta1, mr_beta, mr_c1, mr_s1, mr_c2, mr_s2, mr_phibar;
    double mr_delta, mr_eps, mr_gamma, mr_tau, mr_beta_next;
};

// Tables of the fused evaluation (k_eval_fused), a tile-local copy of the
// mesh.  Vertex tile b is the kTileV consecutive vertices from b * kTileV.
// Its cells (every cell around one of its vertices, at most kTileCap) are
// listed in slot b of `cells`, bit 31 set where tile b owns the cell (holds
// its corner 0) so that each cell energy is counted once, bit 30 where the
// cell crosses the box (a corner carries a nonzero image).  Its halo lists
// the other vertices those cells and the tile's edges reach.  Local vertex
// index j < kTileV is vertex b * kTileV + j, j >= kTileV is halo[j - kTileV].
// Corner rows and star neighbours are stored as 16-bit local references:
// local index in the low 12 bits, the periodic image (as in pack_id) in the
// top 4.  Per vertex, `fstar` = {nb_0 | nb_1 << 16, nb_2 | (a neighbour
// carries a nonzero image) << 16, local cells (10 bits each), e_0} and
// `fe` = [2][n_vert] {e_1, e_2}.  A tile whose halo or
// corner rows do not fit (info.z = 1) is evaluated from the global star and
// rows instead.  Everything is derived from the star and the corner rows and
// rebuilt whenever the topology changes.
constexpr int kTileV = 256;
constexpr int kTileCap = 3 * kTileV;        // cells per tile
constexpr int kHaloCap = 768;               // halo vertices per tile
constexpr int kCornerCap = 2048;            // corner references per tile
constexpr int kCstartPad = kTileCap + 8;    // row starts per tile (uint16)
constexpr uint32_t kZeroImage = 5u;           // image field of pack_id(id, 0, 0)
constexpr uint32_t kCellOwner = 0x80000000u;  // cells[]: the tile owns the cell
constexpr uint32_t kCellImage = 0x40000000u;  // cells[]: a corner has a nonzero image
struct TileTables {
    int32_t *cells;     // [n_tiles][kTileCap]
    int4 *info;         // [n_tiles] {cells, halo vertices, global fallback, corners}
    int32_t *halo;      // [n_tiles][kHaloCap]
    uint16_t *cstart;   // [n_tiles][kCstartPad] row start of each cell, then the end
    uint16_t *corners;  // [n_tiles][kCornerCap]
    int4 *fstar;        // [n_vert]
    int32_t *fe;        // [2][n_vert]
};
__host__ __device__ inline int64_t n_tiles_for(int64_t n_vert) {
    return (n_vert + kTileV - 1) / kTileV;
}
// 16-bit local reference <-> packed local id + image
__host__ __device__ inline int32_t unpack_local(uint32_t r) {
    return (int32_t)((r & 0xfffu) | ((r >> 12) << kIdBits));
}
__host__ __device__ inline uint32_t pack_local(int32_t local, int32_t w) {
    return (uint32_t)local | (((uint32_t)w >> kIdBits) << 12);
}

struct Workspace {
    void *xbuf;          // second position buffer (double [n_vert][2])
    double *cap;         // per-cell (cA, cP) in the arithmetic type, sized for double
    double *cell_aux;    // per-cell auxiliaries (HVP: dA, dP), double [n_cell][2]
    double *partials;    // per-block partial sums (double)
    double *partials2;
    double *mpart;       // per-block (energy, max |F|) partials, double2
    int32_t *t1_list;    // [n_edge] candidate corner indices
    LoopCtl *ctl;        // device control block
    LoopCtl *ctl_host;   // pinned host mirror
    double *cg;          // CG vectors: x, r, p, Ap (double [4][n_vert][2])
    double *scal;        // device scalars
    hipStream_t cap_stream;
};

// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD
// b mod 8), and each XCD has its own L2.  Renumbering blocks so that each
// XCD gets one contiguous eighth of the work keeps the neighbour gathers of
// spatially ordered cells and vertices inside one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block() {
    const int G = gridDim.x, b = blockIdx.x;
    const int per = G / kXcds;
    if (b >= per * kXcds) return b;
    return (b % kXcds) * per + b / kXcds;
}

// ------------------------------------------------------ small device maths
// xa + w*L - xb with the periodic shift applied exactly: the operand next to
// the box face is moved by L first (exact by Sterbenz's lemma when it lies
// within [L/2, 2L]), then two nearby values are subtracted.
// Written with selects rather than branches so that gathers around it stay
// in one basic block and can all be in flight together.
template <typename T>
__host__ __device__ __forceinline__ T pdiff(T xa, T xb, int w, T L) {
    const T a = w < 0 ? xa - L : xa;
    const T b = w > 0 ? xb - L : xb;
    return a - b;
}

// Edge length from its square, and length with inverse.  In FP32 they come
// from the hardware square root and reciprocal square root (each within
// about 1 ulp), which replace the much longer correctly rounded sequences
// of sqrtf and 1/l; in FP64 from sqrt and a division.  Every kernel takes
// its FP32 lengths from these, so all paths round alike.  A zero length
// gives inverse 0.
__device__ __forceinline__ float len_of(float l2) { return __builtin_amdgcn_sqrtf(l2); }
__device__ __forceinline__ double len_of(double l2) { return sqrt(l2); }
__device__ __forceinline__ void len_inv(float l2, float &l, float &inv) {
    inv = l2 > 0.0f ? __builtin_amdgcn_rsqf(l2) : 0.0f;
    l = l2 * inv;
}
__device__ __forceinline__ void len_inv(double l2, double &l, double &inv) {
    l = sqrt(l2);
    inv = l > 0.0 ? 1.0 / l : 0.0;
}
// num / |d| for |d|^2 = l2 > 0
__device__ __forceinline__ float over_len(float num, float l2) {
    return num * __builtin_amdgcn_rsqf(l2);
}
__device__ __forceinline__ double over_len(double num, double l2) { return num / sqrt(l2); }

// The same for the Hessian-vector products, where the FP64 inverse length
// comes from the hardware reciprocal square root refined by two Newton
// steps (y += y (1 - l2 y^2) / 2, each squaring the relative error): a few
// ulp from the correctly rounded 1/sqrt, at a third of the instructions of
// sqrt and a division.  FP32 is as above.
__device__ __forceinline__ double inv_len_hvp(double l2) {
    double y = __builtin_amdgcn_rsq(l2);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double e = fma(-l2, y * y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}
__device__ __forceinline__ void len_inv_hvp(float l2, float &l, float &inv) {
    len_inv(l2, l, inv);
}
__device__ __forceinline__ void len_inv_hvp(double l2, double &l, double &inv) {
    inv = l2 > 0.0 ? inv_len_hvp(l2) : 0.0;
    l = l2 * inv;
}
__device__ __forceinline__ float over_len_hvp(float num, float l2) { return over_len(num, l2); }
__device__ __forceinline__ double over_len_hvp(double num, double l2) {
    return num * inv_len_hvp(l2);
}

__device__ __forceinline__ double min_image(double d, double L) {
    return d - L * floor(d / L + 0.5);
}

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

template <typename T>
__device__ __forceinline__ typename Vec2<T>::type ld2(const T *p, int64_t i) {
    return reinterpret_cast<const typename Vec2<T>::type *>(p)[i];
}
template <typename T>
__device__ __forceinline__ void st2(T *p, int64_t i, T x, T y) {
    typename Vec2<T>::type v;
    v.x = x;
    v.y = y;
    reinterpret_cast<typename Vec2<T>::type *>(p)[i] = v;
}

// ------------------------------------------------------------ reductions
// Wave-wide reductions of a double with DPP lane moves (no LDS traffic):
// pairs of lanes (xor 1, xor 2 in each quad), then the two quads of each
// 8-lane half-row (half-row mirror), then the two halves of each 16-lane
// row (row mirror); every lane then holds its row's total, and the four
// row totals are read with readlane.  The order of operations is fixed, so
// the result is deterministic, and it is the same in every lane.  All 64
// lanes must be active.
template <int Ctrl>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, Ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), Ctrl, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ double first_lane_f64(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7-i within 8
constexpr int kDppMirror = 0x140;     // lane i <-> 15-i within 16

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
    v += dpp_f64<kDppHalfMirror>(v);
    v += dpp_f64<kDppMirror>(v);
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}
// Max that keeps NaN visible (fmax drops a NaN operand).
__device__ __forceinline__ double nanmax(double a, double b) {
    return (a != a || b != b) ? __longlong_as_double(0x7ff8000000000000ll) : fmax(a, b);
}
__device__ __forceinline__ double wave_max(double v) {
    v = nanmax(v, dpp_f64<kDppXor1>(v));
    v = nanmax(v, dpp_f64<kDppXor2>(v));
    v = nanmax(v, dpp_f64<kDppHalfMirror>(v));
    v = nanmax(v, dpp_f64<kDppMirror>(v));
    return nanmax(nanmax(readlane_f64(v, 0), readlane_f64(v, 16)),
                  nanmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// Max over the wave of values that are never NaN (no NaN checks).
__device__ __forceinline__ double wave_max_plain(double v) {
    v = fmax(v, dpp_f64<kDppXor1>(v));
    v = fmax(v, dpp_f64<kDppXor2>(v));
    v = fmax(v, dpp_f64<kDppHalfMirror>(v));
    v = fmax(v, dpp_f64<kDppMirror>(v));
    return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)),
                fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// Block-wide sum of a double (fixed order: deterministic for a fixed block size).
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) r += sh[w];
    }
    return r;  // valid in thread 0
}

__device__ __forceinline__ double block_max(double v, double *sh) {
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) r = nanmax(r, sh[w]);
    }
    return r;
}

// Sum of `s` and max of `m` over the block with one barrier; `sh` holds
// 2 doubles per wave and must not be in use by the block.  Valid in thread 0.
__device__ __forceinline__ double2 block_sum_max(double s, double m, double *sh) {
    s = wave_sum(s);
    m = wave_max(m);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        sh[2 * wid] = s;
        sh[2 * wid + 1] = m;
    }
    __syncthreads();
    double2 r{0.0, 0.0};
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) {
            r.x += sh[2 * w];
            r.y = nanmax(r.y, sh[2 * w + 1]);
        }
    }
    return r;
}

__device__ __forceinline__ double ld_acquire(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of part[0..n) by all threads of one block in a fixed order (each
// thread a fixed strided subset, then the fixed-order block reduction), so
// the result does not depend on which block performs it.  Valid in thread 0.
__device__ __forceinline__ double block_sum_array(const double *part, int n, int stride,
                                                  double *sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += ld_acquire(part + (int64_t)i * stride);
    return block_sum(s, sh);
}

// Called by thread 0 of each of n blocks after the block's results are
// stored (and after a barrier, so the block's other stores have reached the
// cache): returns true in exactly one of them (the last to arrive), which
// then sees every block's stores.  Arrivals only release; the acquire is taken once, by the
// last block.  On this multi-XCD part a device-scope release writes back the
// XCD's L2 and an acquire invalidates it, so each costs tens of ns.  The
// counter is reset by the last block.
__device__ __forceinline__ bool last_of(unsigned int *counter, unsigned int n) {
    const unsigned int prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE,
                                                     __HIP_MEMORY_SCOPE_AGENT);
    const bool last = prev == n - 1;
    if (last) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return last;
}
__device__ __forceinline__ bool last_block(unsigned int *counter) {
    return last_of(counter, gridDim.x);
}

}  // namespace vtx
