// Internal declarations for batched independent instances.
#pragma once

#include <algorithm>
#include <vector>

#include "hdg_internal.hpp"

// Per-instance descriptor (device copy). Offsets are in elements of each concatenated array.
struct InstDesc {
    int M, D, P, PF, L, nu, nq, nt, nb, S, R, C, NW, KD, ne, nf;
    int64_t e0, f0;                 // first global element / face of the instance
    int64_t off[11];                // Minv, Bd, Cd, D, E, F, G, H, J, ru, rt
    int64_t kbar_off, rbar_off, local_off, du_off, dq_off;
    int64_t K_off, nbr_off, vec_off, f2e_off, e2f_off, binv_off;
};

struct BatchElemPtrs {
    const double *Minv, *Bd, *Cd, *D, *E, *F, *G, *H, *J, *ru, *rt;
};

// Per-instance GMRES state (device). 48 bytes: beta sits at a multiple of 8 bytes.
struct BatchCtl {
    int done, k, nonfinite, pad;
    double beta, est, pad2, pad3;
};

struct BatchDev {
    InstDesc* desc = nullptr;
    int32_t* eid = nullptr;         // [total_ne] instance of each element
    int32_t* fid = nullptr;         // [total_nf]
    int32_t* dof_inst = nullptr;    // [total_dof]
    int32_t* blk_inst = nullptr;    // [nblk] reduction chunks (never straddle instances)
    int64_t* blk_lo = nullptr;
    int64_t* blk_hi = nullptr;
    int32_t* ib0 = nullptr;         // [n_inst] first / one-past-last chunk of each instance
    int32_t* ib1 = nullptr;
    int n_inst = 0, nblk = 0;
    int64_t total_ne = 0, total_nf = 0, total_dof = 0;
    size_t max_cond_lds = 0, max_rec_lds = 0;
    int max_nb = 0, max_snb = 0, max_R = 0;
};

// Batched element residuals / Jacobian blocks (scalar convection-diffusion models): per
// instance its sizes, the offsets of its parts of the concatenated geometry arrays and of
// the batch arrays it reads and writes, and its model coefficients.
struct ElemInst {
    int P, PF, L, D, Qv, Qf;
    int64_t e0;
    int64_t g_wdet, g_dphix, g_phi, g_phif, g_psi, g_ndA, g_dA, g_src, g_uD;
    int64_t e2f_off, u_off, uh_off, q_off;
    int64_t out_off[11];            // Minv, Bd, Cd, D, E, F, G, H, J, ru, rt
    double nu, tau, beta[3], gamma[3];
    double c;                       // time-term factor of the instance (0: steady)
};

struct ElemBatchArgs {
    hdg_elem_geom g;                // concatenated arrays (nqv, nqf unused)
    const int32_t* e2f;
    const double *u, *uhat, *u_prev;   // u_prev: batch array like u (read where c != 0)
    const double* r_extra;             // batch array like u, or null (known stage term)
    hdg_elem_arrays out;
    int* bad;
    int residual_only, keep_mass;
};

size_t element_batch_lds_bytes(int P, int PF, int L, int D, int nqv, int nqf);
hdg_status element_blocks_batch_run(hdg_ctx ctx, int64_t total_ne, const ElemInst* inst_dev, const int32_t* eid,
                                    const ElemBatchArgs& a, size_t lds);
hdg_status residual_norm_batch_run(hdg_ctx ctx, int n_inst, const InstDesc* desc, const double* ru, const double* rt,
                                   const int32_t* f2e, double* norms);
hdg_status newton_update_batch_run(hdg_ctx ctx, int n_inst, const InstDesc* desc, const double* alpha,
                                   const double* du, double* u, const double* x, double* uhat);

hdg_status batch_launch_condense(hdg_ctx ctx, const BatchDev& b, const BatchElemPtrs& in, double* Kbar, double* rbar,
                                 double* local, int* bad, int grid);
hdg_status batch_launch_assemble(hdg_ctx ctx, const BatchDev& b, const int32_t* f2e, const int32_t* e2f,
                                 const double* Kbar, const double* rbar, double* K64, float* K32, int32_t* nbr,
                                 double* r);
hdg_status batch_launch_face(hdg_ctx ctx, const BatchDev& b, const void* M1, bool fp32, const int32_t* nbr,
                             bool bj_only, const double* x, double* out, double s0, const double* X, double a0,
                             const BatchCtl* ctl);
hdg_status batch_launch_bj(hdg_ctx ctx, const BatchDev& b, const double* K64, double* B64, float* B32, int* bad);
hdg_status seg_multidot(hdg_ctx ctx, const BatchDev& b, const double* V, size_t ldv, int J, const double* w,
                        double* part, const BatchCtl* ctl);
hdg_status seg_reduce(hdg_ctx ctx, const BatchDev& b, const double* part, int J, double* out, int ldo, bool add,
                      double* copy_to, int ldc, const BatchCtl* ctl);
hdg_status seg_multiaxpy(hdg_ctx ctx, const BatchDev& b, const double* V, size_t ldv, int J, const double* h,
                         int ldh, double sign, double* w, const BatchCtl* ctl, bool use_kdev);
hdg_status seg_sumsq(hdg_ctx ctx, const BatchDev& b, const double* w, double* part, const BatchCtl* ctl);
hdg_status seg_scale(hdg_ctx ctx, const BatchDev& b, double* v, const double* denom, int ld_denom,
                     const BatchCtl* ctl);
hdg_status seg_cycle_init(hdg_ctx ctx, const BatchDev& b, const double* part, BatchCtl* ctl, double* g, int ldg,
                          int jmax, const double* target);
hdg_status seg_givens(hdg_ctx ctx, const BatchDev& b, const double* part, BatchCtl* ctl, double* H, int ldh, int mcols,
                      double* cs, double* sn, double* g, int ldg, int j, int jmax, const double* target);
hdg_status seg_backsolve(hdg_ctx ctx, const BatchDev& b, const BatchCtl* ctl, const double* H, int ldh, int mcols,
                         const double* g, int ldg, double* y);
hdg_status batch_launch_recover(hdg_ctx ctx, const BatchDev& b, const double* local, const double* Minv,
                                const double* Bd, const double* Cd, const int32_t* e2f, const double* xhat,
                                double* du, double* dq);
