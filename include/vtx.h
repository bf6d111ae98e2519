/*
 * vtx.h -- C ABI of an MI355X (gfx950) library for the periodic 2-D vertex
 * model of confluent epithelia described in VertAX (arXiv 2604.06896).
 *
 * The library evaluates the energy
 *
 *     E(X, theta) = sum_cells [ K_A (A - A0)^2 + K_P (P - P0)^2 ]
 *                 + sum_edges lambda * l
 *
 * (Methods, "Vertex model formulation": equation E1 with the line-tension
 * term of equation E2) and its per-vertex forces F = -grad_X E, relaxes a
 * tissue to mechanical equilibrium by gradient descent with T1 neighbour
 * exchanges (Methods, "Simulation engine" and "T1 transitions"), and
 * returns the gradient of an outer cost with respect to the mechanical
 * parameters at that equilibrium (Methods, "Gradient computation methods":
 * implicit differentiation in adjoint form, and centred equilibrium
 * propagation).
 *
 * Conventions shared by every call
 *  - Topology is the paper's half-edge table (Methods, "System state and
 *    data structure"): int32 [n_he][8] with columns prev, next, twin,
 *    source, target, face, x-offset, y-offset.  The offsets (each -1, 0 or
 *    +1) give the periodic image of the target, so the edge vector of
 *    half-edge h is X[tgt] + (ox*Lx, oy*Ly) - X[src].  Faces are traversed
 *    counter-clockwise (a cell lies left of its half-edges); vertices are
 *    3-valent.
 *  - Edges are numbered 0..n_edge-1 in ascending order of the lower
 *    half-edge id of each twin pair; lambda and edge gradients use this
 *    numbering.
 *  - X (vertex positions) and F (forces) are device arrays [n_vert][2]
 *    (x, y interleaved).  Their element type is set by the precision mode:
 *      VTX_F32    float  X and F, float arithmetic;
 *      VTX_F64    double X and F, double arithmetic;
 *      VTX_MIXED  double X and F; local coordinate differences are rounded
 *                 to float and the force arithmetic is float.
 *    In every mode energy totals, the max-force convergence test, CG dot
 *    products, step sizes and T1 decisions are computed in double.
 *  - Parameter arrays (vtx_params) are device arrays with the element type
 *    of X; a NULL array means "use the scalar field".
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    Calls that return results through device pointers are asynchronous in
 *    stream order and allocate nothing, so they can be captured in a HIP
 *    graph.  Calls that return results through host pointers synchronise
 *    the stream.
 *  - Every call returns VTX_OK (0) or a negative error code; the message of
 *    the last error of the calling thread is returned by vtx_last_error().
 *    Memory is owned by the caller except for tissue and batch handles,
 *    which own their topology and all workspaces (allocated at creation).
 */
#ifndef VTX_H
#define VTX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes (negative) */
#define VTX_OK 0
#define VTX_E_ARG (-1)        /* invalid argument (null pointer, size, mode) */
#define VTX_E_TOPOLOGY (-2)   /* half-edge table is not a valid periodic 3-valent tiling */
#define VTX_E_CAPACITY (-3)   /* a size exceeds a library limit */
#define VTX_E_HIP (-4)        /* HIP runtime error */
#define VTX_E_NONFINITE (-5)  /* a NaN or infinity appeared in the forces */

/* statuses (reported in result structs; not errors) */
#define VTX_CONVERGED 0
#define VTX_NOT_CONVERGED 1
#define VTX_CG_NEG_CURVATURE 2
#define VTX_CG_MAXITER 3

/* precision modes */
#define VTX_F32 0
#define VTX_F64 1
#define VTX_MIXED 2

/* parameter selectors */
#define VTX_THETA_LAMBDA 0   /* theta = per-edge line tensions lambda_e   */
#define VTX_THETA_P0 1       /* theta = per-cell preferred perimeters P0_c */

/* hypergradient estimators */
/* Schedules of vtx_batch_relax. */
#define VTX_SCHED_AUTO (-1)     /* choose by timed trials (vtx_batch_autotune)       */
#define VTX_SCHED_PERSISTENT 0  /* one persistent launch, one workgroup per tissue   */
#define VTX_SCHED_GRID 1        /* each tissue in turn on the whole GPU (vtx_relax)  */
#define VTX_SCHED_SPLIT 2       /* each tissue over several cooperating workgroups   */

#define VTX_GRAD_ADJOINT 0     /* implicit differentiation, adjoint form, CG */
#define VTX_GRAD_EP_CENTRED 1  /* centred equilibrium propagation            */
#define VTX_GRAD_EP_FORWARD 2  /* first-order (one-sided) equilibrium propagation */
#define VTX_GRAD_ADJOINT_MINRES 3 /* implicit differentiation, adjoint form, MINRES */

typedef struct vtx_tissue_s *vtx_tissue;
typedef struct vtx_batch_s *vtx_batch;

/* Mechanical parameters: per-cell K_A, A0, K_P, P0 and per-edge lambda
 * (Methods, "Vertex model formulation"; parameters may be heterogeneous,
 * Results, "Energy functions"). */
typedef struct {
    const void *KA, *A0, *KP, *P0;  /* device [n_cell] or NULL */
    const void *lam;                /* device [n_edge] or NULL */
    double KA_s, A0_s, KP_s, P0_s, lam_s;
} vtx_params;

/* Gradient-descent options (Methods, "Simulation engine").
 *   X <- X + eta * F,  stop when max_k |F_k| < tol on `patience`
 *   consecutive iterations (max over all 2*n_vert components) or after
 *   max_iter force evaluations.  One iteration is: T1 pass (if enabled),
 *   forces, convergence test, step.
 * T1 (Methods, "T1 transitions"): every iteration, edges with length
 *   l < l_min are visited in ascending edge id; each is either stretched to
 *   length l_new along its direction or exchanged for an orthogonal edge of
 *   length l_new through the same midpoint, whichever gives the strictly
 *   lower total energy (ties keep the stretch); the exchange is not
 *   considered if a cell losing the edge is a triangle or the four cells
 *   around it are not distinct.
 * Nudge (Methods, "Equilibrium propagation"): if beta != 0 the relaxed
 *   energy is E + beta*C with C the v2v cost to X_target (device, same
 *   element type as X) or, if X_target is NULL, the linear cost g_lin . X
 *   (g_lin: double device array [n_vert][2]).
 *   The mean of grad C over the vertices is removed from the nudge force
 *   (rigid translations do not change any EP estimate and are otherwise
 *   stiffened only by beta/n_vert).  A nudge cannot be combined with T1. */
typedef struct {
    double eta, tol;
    int64_t patience, max_iter;
    int32_t t1_enable;
    double l_min, l_new;
    double beta;
    const void *X_target;
    const void *g_lin;
    int32_t chunk;   /* iterations per captured graph launch (0 = 256) */
} vtx_relax_opts;

typedef struct {
    int64_t iters;      /* force evaluations performed */
    int64_t n_t1;       /* accepted neighbour exchanges */
    int64_t n_stretch;  /* short edges stretched instead */
    double max_f;       /* max |F| component of the last evaluation */
    double energy;      /* E (+ beta*C) at the returned positions */
    int32_t status;     /* VTX_CONVERGED or VTX_NOT_CONVERGED */
} vtx_relax_result;

typedef struct {
    int32_t method;        /* VTX_GRAD_ADJOINT(_MINRES), VTX_GRAD_EP_CENTRED or _FORWARD */
    int32_t theta;         /* VTX_THETA_LAMBDA or VTX_THETA_P0 */
    double cg_tol;         /* relative residual |r| / |P b| */
    int64_t cg_max_iter;
    double beta;           /* EP nudge (relaxations at +-beta/2) */
    vtx_relax_opts ep_relax; /* EP relaxation options (beta fields ignored) */
} vtx_grad_opts;

typedef struct {
    int64_t cg_iters;
    double cg_rel_res;     /* recursive relative residual at exit */
    int32_t status;        /* VTX_CONVERGED, VTX_CG_NEG_CURVATURE, VTX_CG_MAXITER,
                              or for EP the worse of the two relaxation statuses */
    vtx_relax_result ep_plus, ep_minus;
} vtx_grad_result;

/* ------------------------------------------------------------ tissues */

/* Create a tissue handle from a host half-edge table.  Validates the table
 * (twin involution with reversed ends and negated offsets, prev/next
 * inverse, source(next(h)) = target(h), faces of >= 3 sides whose offsets
 * sum to zero, 3-valent vertices, offsets in {-1,0,1}, no edge from a
 * vertex to its own image) and stages the device layouts: cell->corner
 * rows, vertex stars and the edge list.  The caller keeps ownership of
 * `he`.  Errors: VTX_E_ARG, VTX_E_TOPOLOGY, VTX_E_CAPACITY (n_vert >= 2^28,
 * a cell spanning more than one periodic image), VTX_E_HIP. */
int vtx_tissue_create(const int32_t *he, int64_t n_he, int64_t n_vert, int64_t n_cell,
                      double Lx, double Ly, vtx_tissue *out);
int vtx_tissue_destroy(vtx_tissue t);
/* Sizes of a tissue (any pointer may be NULL). */
int vtx_tissue_sizes(vtx_tissue t, int64_t *n_vert, int64_t *n_cell, int64_t *n_edge,
                     int64_t *n_he);
/* Layout of the fused evaluation's tile tables (a diagnostic): stats[0] =
 * vertex tiles (256 vertices each), stats[1] = cells listed over all tiles
 * (a border cell is listed by every tile around it), stats[2] = halo
 * vertices over all tiles, stats[3] = corner references over all tiles,
 * stats[4] = tiles evaluated from global memory because their halo or rows
 * overflow the fixed slots.  stats: host int64_t[5].  Synchronises the
 * device. */
int vtx_tissue_tile_stats(vtx_tissue t, int64_t *stats);
/* Copy the current half-edge table (it changes under T1) to host memory
 * [n_he][8].  Synchronises the device. */
int vtx_tissue_get_topology(vtx_tissue t, int32_t *he_out);
/* Replace the topology by a host table of the same sizes (validated as at
 * creation). */
int vtx_tissue_set_topology(vtx_tissue t, const int32_t *he);

/* Energy and forces at X (Methods, "Vertex model formulation"), in one
 * fused launch per tile of 256 vertices (plus a one-block finish for the
 * scalars of large tissues).  F equals vtx_cell_coeffs followed by
 * vtx_vertex_forces bit for bit; E equals the sum of the cell and edge
 * energies up to the order of summation (fixed: deterministic).
 * E_dev: device double scalar or NULL; F: device [n_vert][2] or NULL;
 * maxf_dev: device double scalar (max |F| component) or NULL.
 * Asynchronous; graph-capturable (a graph stays valid across topology
 * changes: the tile tables are rebuilt in place, in stream order, by every
 * call that changes the topology). */
int vtx_energy_forces(vtx_tissue t, int32_t mode, const void *X, const vtx_params *p,
                      double *E_dev, void *F, double *maxf_dev, void *stream);

/* vtx_energy_forces for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with their scratch (per-tile
 * partial sums, control blocks) in a fixed device array of the library
 * (about 17 KiB, held on every GPU the library runs on until the process
 * ends) instead of the tissue's workspace.  Allocates nothing and issues no
 * memset (a small kernel clears the control blocks).  Limit: at most 262144
 * vertices (131072 cells), else VTX_E_CAPACITY.
 * All calls on one GPU share that array, so calls that overlap on one GPU
 * (different streams, threads or tissues) race; serialise them.  Arguments,
 * outputs and errors as vtx_energy_forces.  Asynchronous. */
int vtx_energy_forces_noalloc(vtx_tissue t, int32_t mode, const void *X, const vtx_params *p,
                              double *E_dev, void *F, double *maxf_dev, void *stream);

/* Cell pass alone: per-cell coefficients (cA, cP) = (2 K_A (A - A0),
 * 2 K_P (P - P0)) at X, i.e. minus the cell pressure and the cortical
 * tension of each cell (derivatives of E with respect to A and P; Methods,
 * "Vertex model formulation").  coeffs: device [n_cell][2], float for
 * VTX_F32 and VTX_MIXED, double for VTX_F64.  Asynchronous. */
int vtx_cell_coeffs(vtx_tissue t, int32_t mode, const void *X, const vtx_params *p,
                    void *coeffs, void *stream);

/* Vertex pass alone: forces F at X from cell coefficients produced by
 * vtx_cell_coeffs for the same X and parameters (each 3-valent vertex
 * gathers its 3 neighbours, 3 cells and 3 edge tensions; no atomics).
 * F: device [n_vert][2] (element type of X); maxf_dev: device double or
 * NULL.  vtx_energy_forces is vtx_cell_coeffs followed by this call, plus
 * the energy.  Asynchronous. */
int vtx_vertex_forces(vtx_tissue t, int32_t mode, const void *X, const vtx_params *p,
                      const void *coeffs, void *F, double *maxf_dev, void *stream);

/* Per-cell area and perimeter at X (double device arrays [n_cell], either
 * may be NULL).  Asynchronous. */
int vtx_cell_geometry(vtx_tissue t, int32_t mode, const void *X, double *A_dev,
                      double *P_dev, void *stream);

/* Per-edge lengths at X (double device array [n_edge]).  Asynchronous. */
int vtx_edge_lengths(vtx_tissue t, int32_t mode, const void *X, double *len_dev,
                     void *stream);

/* Relax X in place to mechanical equilibrium (Methods, "Simulation
 * engine").  The loop runs on the device in captured graphs of `chunk`
 * iterations; the host reads an 8-byte status between chunks.  T1 mutates
 * the tissue's topology.  `res` is a host struct; synchronises. */
int vtx_relax(vtx_tissue t, int32_t mode, void *X, const vtx_params *p,
              const vtx_relax_opts *o, vtx_relax_result *res, void *stream);

/* One T1 pass over X (Methods, "T1 transitions"), with the rules of
 * vtx_relax_opts.  Mutates X and the topology; counts are returned in host
 * memory (either may be NULL); synchronises. */
int vtx_t1(vtx_tissue t, int32_t mode, void *X, const vtx_params *p, double l_min,
           double l_new, int64_t *n_swap, int64_t *n_stretch, void *stream);

/* Hessian-vector product H v at X (H = d2E/dX2); v and Hv are double device
 * arrays [n_vert][2].  Asynchronous. */
int vtx_hvp(vtx_tissue t, int32_t mode, const void *X, const vtx_params *p, const double *v,
            double *Hv, void *stream);

/* Gradient of an outer cost C with respect to theta at the equilibrium
 * X_star (Methods, "Implicit differentiation (ID)" and "Equilibrium
 * propagation (EP)").
 *   ADJOINT: solves H mu = P dC_dX by CG on the zero-mean subspace
 *     (P removes the per-component mean; rigid translations are null
 *     vectors of H) and returns  dC_dtheta = -(d2E/dX dtheta)^T mu.
 *     dC_dX is a double device array [n_vert][2] (the backward of any cost).
 *     CG stops with VTX_CG_NEG_CURVATURE if H is not positive definite.
 *   ADJOINT_MINRES: the same with MINRES (Paige-Saunders; the paper's
 *     solver, Methods, ID), which needs H symmetric only; cg_tol bounds the
 *     recursive residual |P b - H mu| / |P b|.
 *   EP_CENTRED: relaxes E + (beta/2) C and E - (beta/2) C from X_star and
 *     returns (dE/dtheta(X+) - dE/dtheta(X-)) / beta, where C is the v2v
 *     cost to X_target when given (device, element type of X) and the
 *     linear cost dC_dX . X otherwise.
 *   EP_FORWARD: the first-order estimator: relaxes E + beta C from X_star
 *     and returns (dE/dtheta(X_beta) - dE/dtheta(X_star)) / beta (bias
 *     O(beta) against O(beta^2) for the centred one); res->ep_minus is
 *     zero.
 * The explicit partial d_theta C is not added (zero for costs of X only).
 * dC_dtheta: double device array [n_edge] (lambda) or [n_cell] (P0).
 * `res` is a host struct; synchronises. */
int vtx_param_grad(vtx_tissue t, int32_t mode, const void *X_star, const vtx_params *p,
                   const double *dC_dX, const void *X_target, const vtx_grad_opts *o,
                   double *dC_dtheta, vtx_grad_result *res, void *stream);

/* v2v cost C = 1/(2 n_vert) sum_k |x_k - x_target,k|^2 (minimum periodic
 * image; Methods, "Geometric vertex-to-vertex (v2v) cost") and its gradient
 * (x_k - x_target,k)/n_vert.  C_dev: device double scalar or NULL; grad:
 * double device [n_vert][2] or NULL.  Asynchronous. */
int vtx_v2v(vtx_tissue t, int32_t mode, const void *X, const void *X_target, double *C_dev,
            double *grad, void *stream);

/* Forward (sensitivity) implicit differentiation along one parameter
 * direction d (Methods, "Implicit differentiation (ID)": one linear solve
 * per direction, where the adjoint needs one in total).  Solves
 *   H w = -(d2E/dX dtheta) d
 * by CG on the zero-mean subspace (w = dX_star/dtheta . d) and writes the
 * directional derivative  dC_dX . w  to the double device scalar dC_dd
 * (the explicit partial d_theta C . d is not added).  d is a double device
 * array [n_edge] (theta = lambda) or [n_cell] (theta = P0); dC_dX a double
 * device array [n_vert][2]; dX_dd, if not NULL, receives w (double device
 * [n_vert][2]).  Only o->theta, o->cg_tol, o->cg_max_iter and o->method
 * (VTX_GRAD_ADJOINT_MINRES selects MINRES, anything else CG) are read; the
 * iterations, residual and status go to res (host, may be NULL).  Needs
 * double positions (VTX_F64 or VTX_MIXED).  Synchronises. */
int vtx_param_sens(vtx_tissue t, int32_t mode, const void *X_star, const vtx_params *p,
                   const double *d, const double *dC_dX, const vtx_grad_opts *o, double *dC_dd,
                   double *dX_dd, vtx_grad_result *res, void *stream);

/* ------------------------------------------------------------- batches */

/* Group independent tissues for batched relaxation.  The handles stay
 * owned by the caller and must outlive the batch. */
int vtx_batch_create(const vtx_tissue *ts, int32_t n, vtx_batch *out);
int vtx_batch_destroy(vtx_batch b);

/* Relax every tissue of the batch (each with its own X, parameters and the
 * shared options; Methods, "Simulation engine", per tissue).  Schedules:
 *   VTX_SCHED_PERSISTENT  one persistent launch captured in a graph, one
 *                         workgroup of `block_threads` (256, 512 or 1024;
 *                         0 chooses) threads per tissue looping the whole
 *                         relaxation, tissues taken from a device work
 *                         queue in descending size.  With 512 threads (or
 *                         0), a batch whose tissues all have at most 1024
 *                         cells and fit the per-workgroup LDS (both
 *                         position buffers, cell coefficients, corner rows)
 *                         runs a kernel that keeps them there and the vertex
 *                         stars in registers, T1 passes included; 0 takes
 *                         1024 threads otherwise;
 *   VTX_SCHED_GRID        each tissue in turn through vtx_relax (all
 *                         workgroups of the GPU on one tissue; suits a few
 *                         large tissues); block_threads is ignored;
 *   VTX_SCHED_SPLIT       T1 off only: each tissue split over K = block_threads
 *                         (1, 2, 4 or 8; 0 chooses) cooperating 512-thread
 *                         workgroups of one cooperative launch, each owning a
 *                         contiguous range of vertices and the cells around
 *                         them in LDS, with one barrier between the
 *                         workgroups of a tissue per iteration (max |F| and
 *                         the boundary positions); suits a few tissues of up
 *                         to 8192 vertices.  0 takes the largest K with at
 *                         most 64 workgroups in all and 200 vertices per
 *                         part: a barrier between more workgroups costs
 *                         several microseconds on this part.  A tissue one
 *                         part cannot hold is relaxed by the persistent
 *                         schedule instead.  Returns VTX_E_HIP if a wait
 *                         between workgroups times out (20 s);
 *   VTX_SCHED_AUTO        vtx_batch_autotune first, then its choice.
 * Every schedule gives the same iterates as vtx_relax on each tissue (the
 * reported energy is summed in another order by the split schedule).  X
 * and p are host arrays of n entries (device pointers inside).  Results go
 * to the host array res[n]; synchronises.  Nudges are not supported here. */
int vtx_batch_relax(vtx_batch b, int32_t mode, void *const *X, const vtx_params *p,
                    const vtx_relax_opts *o, int32_t schedule, int32_t block_threads,
                    vtx_relax_result *res, void *stream);

/* Choose the schedule of vtx_batch_relax for this batch, mode, X, p and o
 * from timed trials on copies of the positions (T1 off, `trial_iters`
 * iterations, no convergence test): the persistent schedule with 256, 512
 * and 1024 threads on all tissues, the grid schedule on the (up to) two
 * largest tissues, extrapolated to the batch, and, when o has T1 off, the
 * split schedule with 2, 4 and 8 workgroups per tissue.  X is not
 * modified; the trial buffers are allocated and freed here.  Writes the
 * choice to *schedule and *block_threads and, if trial_ms is not NULL, the
 * seven projected times in milliseconds (persistent 256, 512, 1024, grid,
 * split 2, 4, 8; -1 for a split trial not run).  Synchronises. */
int vtx_batch_autotune(vtx_batch b, int32_t mode, void *const *X, const vtx_params *p,
                       const vtx_relax_opts *o, int32_t trial_iters, int32_t *schedule,
                       int32_t *block_threads, double *trial_ms, void *stream);

/* Hypergradients of every tissue of the batch (see vtx_param_grad).
 * ADJOINT / ADJOINT_MINRES: one persistent launch, one workgroup of
 * `block_threads` (256, 512 or 1024; 0 chooses) per tissue running the
 * whole Krylov solve and the contraction; a tissue whose positions, solve
 * vector and per-cell coefficients fit in the device's per-workgroup LDS
 * keeps them there, and with workgroups of at most 512 threads a CG solve of
 * a tissue with at most two cells and four vertices per thread also keeps
 * its corner rows in LDS and its stars, solution and residual in registers
 * (same arithmetic in every form).  0 takes 512 threads when every tissue
 * has that form, else 1024.  EP_CENTRED / EP_FORWARD: batched nudged
 * relaxations (vtx_batch_relax with a per-tissue nudge, workgroups of
 * `block_threads`; 0 takes the LDS-resident relaxation of vtx_batch_relax
 * when every tissue fits it, else 1024 threads) and one estimate launch.
 * block_threads = -K (K = 1, 2, 4 or 8) splits each tissue over K
 * cooperating 512-thread workgroups of one cooperative launch instead: for
 * ADJOINT (FP64 only) each part keeps the constant geometry of the
 * Hessian-vector product of its vertices and cells in LDS and registers and
 * the parts meet at two barriers per CG step; for EP the nudged relaxations
 * take the split schedule of vtx_batch_relax.  A barrier between many
 * workgroups costs several microseconds on this part, so splitting pays for
 * a few tissues, not for a full device of them; a tissue one part cannot
 * hold falls back to one workgroup.  X_star, p, dC_dX, X_target
 * and dC_dtheta are host arrays of n entries (device pointers inside; dC_dX
 * or X_target may be NULL as for vtx_param_grad).  Results go to the host
 * array res[n]; synchronises.  Errors: VTX_E_ARG (null arrays, bad mode,
 * theta, method, options or block_threads), VTX_E_HIP (also: a wait between
 * the workgroups of a split tissue timed out). */
int vtx_batch_param_grad(vtx_batch b, int32_t mode, void *const *X_star, const vtx_params *p,
                         const double *const *dC_dX, const void *const *X_target,
                         const vtx_grad_opts *o, double *const *dC_dtheta, int32_t block_threads,
                         vtx_grad_result *res, void *stream);

/* Message of the last error on the calling thread (never NULL). */
const char *vtx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VTX_H */
