// Launchers of the libvtx kernels (implemented in vtx_kernels.hip and
// vtx_batch.hip); all are asynchronous on the given stream.
#pragma once

#include "vtx_internal.h"

namespace vtx {

struct ParamsRaw {
    const void *KA, *A0, *KP, *P0, *lam;
    double KA_s, A0_s, KP_s, P0_s, lam_s;
};

struct RelaxArgs {
    double eta;
    int t1_enable;
    double l_min, l_new;
    int nudge;  // 0 none, 1 v2v (X_target), 2 linear (g_lin)
    double beta;
    const void *X_target;
    const void *g_lin;
};

void launch_eval(const DevTissue &t, const Workspace &w, int mode, const void *X,
                 const ParamsRaw &p, double *E, void *F, double *maxf, hipStream_t s);
void launch_eval_fused(const DevTissue &t, const Workspace &w, const TileTables &tt, int mode,
                       const void *X, const ParamsRaw &p, double *E, void *F, double *maxf,
                       hipStream_t s);
void launch_tile_build(const DevTissue &t, const TileTables &tt, hipStream_t s);
void launch_cell_pass(const DevTissue &t, const Workspace &w, int mode, const void *X,
                      const ParamsRaw &p, void *coeffs, hipStream_t s);
void launch_vertex_pass(const DevTissue &t, const Workspace &w, int mode, const void *X,
                        const ParamsRaw &p, const void *coeffs, void *F, double *maxf,
                        hipStream_t s);
void launch_relax_iter(const DevTissue &t, const Workspace &w, int mode, void *Xc, void *Xn,
                       int cur, const ParamsRaw &p, const RelaxArgs &ra, hipStream_t s);
void launch_t1(const DevTissue &t, const Workspace &w, int mode, void *X, const ParamsRaw &p,
               double l_min, double l_new, hipStream_t s);
void launch_cell_coeffs(const DevTissue &t, const Workspace &w, int mode, const void *X,
                        const ParamsRaw &p, hipStream_t s);
void launch_hvp(const DevTissue &t, const Workspace &w, int mode, const void *X,
                const ParamsRaw &p, const double *v, double *Hv, double *dpart, LoopCtl *ctl,
                hipStream_t s);
void launch_sens_rhs(const DevTissue &t, const Workspace &w, const void *X, const ParamsRaw &pr,
                     int theta, const double *d, double *rhs, hipStream_t s);
void launch_minres_init(const Workspace &w, int nv, const double *b, hipStream_t s);
void launch_minres_iter(const DevTissue &t, const Workspace &w, int mode, const void *X,
                        const ParamsRaw &p, hipStream_t s);
void launch_cg_init(const Workspace &w, int nv, const double *b, hipStream_t s);
void launch_cg_iter(const DevTissue &t, const Workspace &w, int mode, const void *X,
                    const ParamsRaw &p, hipStream_t s);
void launch_project(const Workspace &w, int nv, double *x, hipStream_t s);
void launch_contract(const DevTissue &t, int mode, const void *X, const ParamsRaw &p, int theta,
                     const double *mu, double *g, hipStream_t s);
void launch_ep(const DevTissue &t, int mode, const void *Xp, const void *Xm, const ParamsRaw &p,
               int theta, double beta, double *g, hipStream_t s);
void launch_edge_len(const DevTissue &t, int mode, const void *X, double *len, hipStream_t s);
void launch_cell_exact(const DevTissue &t, int mode, const void *X, double *A, double *P,
                       hipStream_t s);
void launch_v2v(const DevTissue &t, const Workspace &w, int mode, const void *X, const void *Xt,
                double *C, double *grad, hipStream_t s);
void launch_dot_pos(const Workspace &w, int mode, int nv, const double *g, const void *X,
                    double *out, hipStream_t s);
void launch_mean_pos(const Workspace &w, int mode, int nv, const void *a, double *mean_out,
                     hipStream_t s);

}  // namespace vtx
