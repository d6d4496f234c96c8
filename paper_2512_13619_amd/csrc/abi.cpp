// C ABI entry points of libhdg.so: argument validation on the host, then the
// launchers. No C++ exception crosses this boundary.
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <vector>

#include "hdg_internal.hpp"

hdg_status solve_run(hdg_ctx ctx, const hdg_dims* d, const double* K64, const float* K32, const int32_t* nbr,
                     const double* b, double* x, const hdg_solve_opts* o, hdg_solve_stats* stats);
hdg_status poly_apply_run(hdg_ctx ctx, const hdg_dims* d, const double* K64, const float* K32, const int32_t* nbr,
                          const double* B64, const float* B32, int precision, int npoly, const double* tre,
                          const double* tim, const double* y, double* z);
hdg_status op_apply_run(hdg_ctx ctx, const hdg_dims* d, const void* M1, bool m1_32, const int32_t* nbr, int S1,
                        const double* x, double* y);
hdg_status cheb_apply_run(hdg_ctx ctx, const hdg_dims* d, const double* K64, const float* K32, const int32_t* nbr,
                          const double* B64, const float* B32, int precision, int P, double alpha, double beta,
                          const double* y, double* z);

void* ws_get(hdg_ctx ctx, WsSlot slot, size_t bytes, hdg_status* st) {
    *st = HDG_OK;
    if (bytes == 0) bytes = 64;
    if (ctx->ws_bytes[slot] >= bytes) return ctx->ws[slot];
    if (slot == WS_BINV64 || slot == WS_BINV32 || slot == WS_KFOLD) ctx->bj_key.valid = false;
    if (ctx->ws[slot]) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->ws[slot]);
        ctx->ws[slot] = nullptr;
        ctx->ws_bytes[slot] = 0;
    }
    void* p = nullptr;
    const size_t rounded = (bytes + 4095) / 4096 * 4096;
    if (hipMalloc(&p, rounded) != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        ctx->err = "device workspace allocation of " + std::to_string(rounded) + " bytes failed";
        *st = HDG_ERR_NOMEM;
        return nullptr;
    }
    ctx->ws[slot] = p;
    ctx->ws_bytes[slot] = rounded;
    return p;
}

namespace {

#define GUARD_BEGIN try {
#define GUARD_END                                 \
    }                                             \
    catch (const std::bad_alloc&) {               \
        ctx->err = "host allocation failed";      \
        return HDG_ERR_NOMEM;                     \
    }                                             \
    catch (const std::exception& ex) {            \
        ctx->err = ex.what();                     \
        return HDG_ERR_ARG;                       \
    }                                             \
    catch (...) {                                 \
        ctx->err = "unknown internal error";      \
        return HDG_ERR_ARG;                       \
    }

hdg_status set_err(hdg_ctx ctx, hdg_status st, const char* msg) {
    ctx->err = msg;
    return st;
}

hdg_status check_dims(hdg_ctx ctx, const hdg_dims* d, bool need_elems, bool need_faces) {
    if (!d) return set_err(ctx, HDG_ERR_ARG, "dims is NULL");
    if (d->ncomp < 1 || d->dim < 1 || d->dim > 3 || d->npe < 1 || d->npf < 1 || d->nlfe < 2 || d->nlfe > 6)
        return set_err(ctx, HDG_ERR_SHAPE, "dims: need ncomp>=1, 1<=dim<=3, npe>=1, npf>=1, 2<=nlfe<=6");
    if (d->ne < 0 || d->nf < 0) return set_err(ctx, HDG_ERR_SHAPE, "dims: negative ne or nf");
    if (need_elems && d->ne < 1) return set_err(ctx, HDG_ERR_SHAPE, "dims: ne must be >= 1");
    if (need_faces && d->nf < 1) return set_err(ctx, HDG_ERR_SHAPE, "dims: nf must be >= 1");
    if (d->ncomp * d->npf > 256) return set_err(ctx, HDG_ERR_SHAPE, "dims: face block edge M*P_F above 256");
    return HDG_OK;
}

// Layout of the residual norm's device scratch (in doubles): the assembled trace residual
// (padded to 64), the element rows' and the trace rows' block partials, two norms.
struct NormScratch {
    size_t nu_all, nface, nfa;
    int nb_u, nb_f;
    size_t total() const { return nfa + (size_t)nb_u + (size_t)nb_f + 2; }
};
NormScratch norm_scratch(const hdg_dims* d) {
    NormScratch s;
    s.nu_all = (size_t)d->ne * d->ncomp * d->npe;
    s.nface = (size_t)d->nf * d->ncomp * d->npf;
    s.nfa = (s.nface + 63) / 64 * 64;
    s.nb_u = krylov_nblk(s.nu_all);
    s.nb_f = krylov_nblk(s.nface);
    return s;
}

hdg_status residual_norm_check(hdg_ctx ctx, const hdg_dims* dims, const int32_t* f2e, const double* ru,
                               const double* rt, const double* norm_h, size_t* need) {
    hdg_status st = check_dims(ctx, dims, true, true);
    if (st != HDG_OK) return st;
    if (!f2e || !ru || !rt || !norm_h) return set_err(ctx, HDG_ERR_ARG, "hdg_residual_norm: NULL pointer");
    *need = norm_scratch(dims).total();
    return HDG_OK;
}

// ||R|| with the scratch at `base` (norm_scratch(dims).total() doubles): every entry the
// kernels read is written first by this call, so nothing needs clearing.
hdg_status residual_norm_run(hdg_ctx ctx, const hdg_dims* dims, const int32_t* f2e, const double* ru,
                             const double* rt, double* base, double* norm_h) {
    const NormScratch s = norm_scratch(dims);
    double* rf = base;
    double* part_u = base + s.nfa;
    double* part_f = part_u + s.nb_u;
    double* nrm = part_f + s.nb_f;
    hdg_status st;
    if ((st = assemble_rhs_run(ctx, dims, f2e, nullptr, rt, rf)) != HDG_OK) return st;
    if ((st = vec_sumsq_partial(ctx, ru, s.nu_all, part_u, s.nb_u, nullptr)) != HDG_OK) return st;
    if ((st = krylov_store_norm(ctx, part_u, s.nb_u, nrm)) != HDG_OK) return st;
    if ((st = vec_sumsq_partial(ctx, rf, s.nface, part_f, s.nb_f, nullptr)) != HDG_OK) return st;
    if ((st = krylov_store_norm(ctx, part_f, s.nb_f, nrm + 1)) != HDG_OK) return st;
    double h[2] = {0.0, 0.0};
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(h, nrm, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HDG_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    *norm_h = std::sqrt(h[0] * h[0] + h[1] * h[1]);
    return HDG_OK;
}

}  // namespace

extern "C" {

hdg_status hdg_create(hdg_ctx* out, int device, void* hip_stream) {
    if (!out) return HDG_ERR_ARG;
    *out = nullptr;
    hdg_ctx c = new (std::nothrow) hdg_ctx_s();
    if (!c) return HDG_ERR_NOMEM;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        delete c;
        return HDG_ERR_HIP;
    }
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return HDG_ERR_HIP;
    }
    // the device address of this GPU's fixed scratch (hdg_residual_norm_noalloc)
    if (noalloc_scratch_init(device) != HDG_OK) {
        delete c;
        return HDG_ERR_HIP;
    }
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return HDG_OK;
}

hdg_status hdg_destroy(hdg_ctx ctx) {
    if (!ctx) return HDG_ERR_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (int s = 0; s < WS_NSLOTS; ++s)
        if (ctx->ws[s]) (void)hipFree(ctx->ws[s]);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return HDG_OK;
}

hdg_status hdg_set_stream(hdg_ctx ctx, void* hip_stream) {
    if (!ctx) return HDG_ERR_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return HDG_OK;
}

const char* hdg_last_error(hdg_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

hdg_status hdg_release_workspace(hdg_ctx ctx) {
    if (!ctx) return HDG_ERR_ARG;
    (void)hipStreamSynchronize(ctx->stream);
    for (int s = 0; s < WS_NSLOTS; ++s) {
        if (ctx->ws[s]) (void)hipFree(ctx->ws[s]);
        ctx->ws[s] = nullptr;
        ctx->ws_bytes[s] = 0;
    }
    ctx->bj_key = BjSetupKey{};
    return HDG_OK;
}

size_t hdg_local_size(const hdg_dims* d) {
    if (!d) return 0;
    const size_t nu = (size_t)d->ncomp * d->npe, nt = (size_t)d->nlfe * d->ncomp * d->npf;
    return nu * (nu + nt + 1);
}

hdg_status hdg_condense(hdg_ctx ctx, const hdg_dims* dims, int64_t ne_chunk, const hdg_elem_blocks* in,
                        double* Kbar, double* rbar, double* local) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, false);
    if (st != HDG_OK) return st;
    if (ne_chunk < 0) return set_err(ctx, HDG_ERR_SHAPE, "ne_chunk must be >= 0");
    if (ne_chunk == 0) return HDG_OK;
    if (ne_chunk > 0x7fffffff) return set_err(ctx, HDG_ERR_SHAPE, "ne_chunk too large");
    if (!in || !in->Minv || !in->Bd || !in->Cd || !in->D || !in->E || !in->F || !in->G || !in->H || !in->J ||
        !in->ru || !in->rt || !Kbar || !rbar || !local)
        return set_err(ctx, HDG_ERR_ARG, "hdg_condense: NULL input or output pointer");
    if ((size_t)dims->ncomp * dims->npe > 4096)
        return set_err(ctx, HDG_ERR_SHAPE, "hdg_condense: nu above 4096");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return condense_run(ctx, dims, ne_chunk, in, Kbar, rbar, local);
    GUARD_END
}

hdg_status hdg_condense_keep(hdg_ctx ctx, const hdg_dims* dims, int64_t ne_chunk, const hdg_elem_blocks* in,
                             double* Kbar, double* rbar, double* local, double* Hbar, int32_t* ipiv) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, false);
    if (st != HDG_OK) return st;
    if (ne_chunk < 0) return set_err(ctx, HDG_ERR_SHAPE, "ne_chunk must be >= 0");
    if (ne_chunk == 0) return HDG_OK;
    if (ne_chunk > 0x7fffffff) return set_err(ctx, HDG_ERR_SHAPE, "ne_chunk too large");
    if (!in || !in->Minv || !in->Bd || !in->Cd || !in->D || !in->E || !in->F || !in->G || !in->H || !in->J ||
        !in->ru || !in->rt || !Kbar || !rbar || !local || !Hbar || !ipiv)
        return set_err(ctx, HDG_ERR_ARG, "hdg_condense_keep: NULL input or output pointer");
    if ((size_t)dims->ncomp * dims->npe > 4096)
        return set_err(ctx, HDG_ERR_SHAPE, "hdg_condense_keep: nu above 4096");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return condense_run(ctx, dims, ne_chunk, in, Kbar, rbar, local, Hbar, ipiv);
    GUARD_END
}

hdg_status hdg_condense_rhs(hdg_ctx ctx, const hdg_dims* dims, int64_t ne_chunk, double* local, const double* Hbar,
                            const int32_t* ipiv, const double* ru, const double* rt, double* rbar) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, false);
    if (st != HDG_OK) return st;
    if (ne_chunk < 0) return set_err(ctx, HDG_ERR_SHAPE, "ne_chunk must be >= 0");
    if (ne_chunk == 0) return HDG_OK;
    if (ne_chunk > 0x7fffffff) return set_err(ctx, HDG_ERR_SHAPE, "ne_chunk too large");
    if (!local || !Hbar || !ipiv || !ru || !rt || !rbar)
        return set_err(ctx, HDG_ERR_ARG, "hdg_condense_rhs: NULL pointer");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return condense_rhs_run(ctx, dims, ne_chunk, local, Hbar, ipiv, ru, rt, rbar);
    GUARD_END
}

hdg_status hdg_assemble_rhs(hdg_ctx ctx, const hdg_dims* dims, const int32_t* f2e, const int32_t* perm,
                            const double* rbar, double* r) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, true, true);
    if (st != HDG_OK) return st;
    if (!f2e || !rbar || !r) return set_err(ctx, HDG_ERR_ARG, "hdg_assemble_rhs: NULL pointer");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return assemble_rhs_run(ctx, dims, f2e, perm, rbar, r);
    GUARD_END
}

hdg_status hdg_assemble_blocks(hdg_ctx ctx, const hdg_dims* dims, const int32_t* f2e, const int32_t* e2f,
                               const int32_t* perm, const double* Kbar, const double* rbar, double* K64, float* K32,
                               int32_t* nbr, double* r) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, true, true);
    if (st != HDG_OK) return st;
    if (!f2e || !e2f || !Kbar || !rbar || !K64 || !nbr || !r)
        return set_err(ctx, HDG_ERR_ARG, "hdg_assemble_blocks: NULL pointer");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return assemble_run(ctx, dims, f2e, e2f, perm, Kbar, rbar, K64, K32, nbr, r);
    GUARD_END
}

hdg_status hdg_gmres_solve(hdg_ctx ctx, const hdg_dims* dims, const double* K64, const float* K32,
                           const int32_t* nbr, const double* r, double* x, const hdg_solve_opts* o,
                           hdg_solve_stats* stats) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, true);
    if (st != HDG_OK) return st;
    if (!o || !stats) return set_err(ctx, HDG_ERR_ARG, "hdg_gmres_solve: NULL opts or stats");
    if (!K64 || !nbr || !r || !x) return set_err(ctx, HDG_ERR_ARG, "hdg_gmres_solve: NULL matrix/vector pointer");
    if (o->restart < 1 || o->restart > 200) return set_err(ctx, HDG_ERR_ARG, "restart must be in [1, 200]");
    if (o->max_iters < 0) return set_err(ctx, HDG_ERR_ARG, "max_iters must be >= 0");
    if (!(o->rtol >= 0.0) || !(o->atol >= 0.0)) return set_err(ctx, HDG_ERR_ARG, "rtol/atol must be >= 0");
    if (o->prec < HDG_PREC_NONE || o->prec > HDG_PREC_ILU_ASM) return set_err(ctx, HDG_ERR_ARG, "unknown prec");
    if (o->prec == HDG_PREC_ILU_ASM && !ilu_matches(o->ilu_asm, dims))
        return set_err(ctx, HDG_ERR_ARG, "HDG_PREC_ILU_ASM needs opts.ilu_asm built for these dims");
    if (o->orth < HDG_ORTH_CGS2 || o->orth > HDG_ORTH_DCGS2) return set_err(ctx, HDG_ERR_ARG, "unknown orth");
    if (o->precision != HDG_FP64 && o->precision != HDG_MIXED)
        return set_err(ctx, HDG_ERR_ARG, "precision must be HDG_FP64 or HDG_MIXED");
    if (o->precision == HDG_MIXED && !K32) return set_err(ctx, HDG_ERR_ARG, "mixed precision needs K32");
    const bool poly = o->prec == HDG_PREC_BJ_POLY || o->prec == HDG_PREC_BJ_CHEB || o->prec == HDG_PREC_ASM_POLY ||
                      o->prec == HDG_PREC_ASM_CHEB;
    const bool schwarz = o->prec == HDG_PREC_ASM || o->prec == HDG_PREC_ASM_POLY || o->prec == HDG_PREC_ASM_CHEB;
    if (schwarz) {
        if (!o->asm_f2e || !o->asm_e2f || !o->asm_inv64 || (o->precision == HDG_MIXED && !o->asm_inv32))
            return set_err(ctx, HDG_ERR_ARG, "additive Schwarz needs asm_inv64 (and asm_inv32 when mixed), asm_f2e and asm_e2f");
        if (dims->ne <= 0) return set_err(ctx, HDG_ERR_SHAPE, "additive Schwarz needs dims->ne > 0");
    }
    if (poly && (o->poly_degree < 1 || o->poly_degree > 64))
        return set_err(ctx, HDG_ERR_ARG, "poly_degree must be in [1, 64]");
    if (poly && !o->poly_v0) return set_err(ctx, HDG_ERR_ARG, "polynomial preconditioner needs poly_v0");
    if (o->resid_hist_len > 0 && !o->resid_hist_h) return set_err(ctx, HDG_ERR_ARG, "resid_hist_h is NULL");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return solve_run(ctx, dims, K64, K32, nbr, r, x, o, stats);
    GUARD_END
}

hdg_status hdg_recover_local(hdg_ctx ctx, const hdg_dims* dims, const double* local, const double* Minv,
                             const double* Bd, const double* Cd, const int32_t* e2f, const int32_t* perm,
                             const double* xhat, double* du, double* dq) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, false);
    if (st != HDG_OK) return st;
    if (dims->ne == 0) return HDG_OK;
    if (!local || !Minv || !Bd || !Cd || !e2f || !xhat || !du || !dq)
        return set_err(ctx, HDG_ERR_ARG, "hdg_recover_local: NULL pointer");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return recover_run(ctx, dims, local, Minv, Bd, Cd, e2f, perm, xhat, du, dq);
    GUARD_END
}

hdg_status hdg_newton_update(hdg_ctx ctx, int64_t n, double alpha, const double* delta, double* state) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    if (n < 0) return set_err(ctx, HDG_ERR_SHAPE, "n must be >= 0");
    if (n == 0) return HDG_OK;
    if (!delta || !state) return set_err(ctx, HDG_ERR_ARG, "hdg_newton_update: NULL pointer");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return axpy_run(ctx, n, alpha, delta, state);
    GUARD_END
}

hdg_status hdg_element_blocks(hdg_ctx ctx, const hdg_dims* dims, const hdg_elem_geom* g, const hdg_conv_diff* m,
                              const hdg_time_term* tt, const int32_t* e2f, const double* u, const double* uhat,
                              int32_t flags, const hdg_elem_arrays* out) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, false);
    if (st != HDG_OK) return st;
    if (!g || !m || !out) return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks: NULL argument struct");
    if (dims->ncomp != 1) return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks: scalar models only (ncomp = 1)");
    if (g->nqv < 1 || g->nqf < 1) return set_err(ctx, HDG_ERR_SHAPE, "hdg_element_blocks: nqv and nqf must be >= 1");
    if (dims->ne == 0) return HDG_OK;
    if (!g->wdet || !g->dphix || !g->phi || !g->phif || !g->psi || !g->ndA || !g->dA || !g->src || !g->uD ||
        !g->bnd || !e2f || !u || !uhat || !out->ru || !out->rt)
        return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks: NULL pointer");
    const bool residual_only = (flags & HDG_ELEM_RESIDUAL_ONLY) != 0;
    if (flags & ~(HDG_ELEM_RESIDUAL_ONLY | HDG_ELEM_KEEP_MASS))
        return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks: unknown flags");
    if ((flags & HDG_ELEM_KEEP_MASS) && !out->Minv)
        return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks: HDG_ELEM_KEEP_MASS needs the kept Minv");
    if (!residual_only && (!out->Minv || !out->Bd || !out->Cd || !out->D || !out->E || !out->F || !out->G ||
                           !out->H || !out->J))
        return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks: NULL matrix output (residual_only = 0)");
    if (tt && !std::isfinite(tt->c))
        return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks: time-term factor c is not finite");
    if (tt && tt->c != 0.0 && !tt->u_prev)
        return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks: time term with c != 0 needs u_prev");
    if (element_blocks_lds_bytes(dims, g->nqv, g->nqf) > 65536)
        return set_err(ctx, HDG_ERR_SHAPE, "hdg_element_blocks: element data exceed 64 KiB of LDS");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    int* status = (int*)ws_get(ctx, WS_STATUS, 64, &st);
    if (!status) return st;
    const int big = 0x7fffffff;
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(status, &big, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    if ((st = element_blocks_run(ctx, dims, g, m, tt, e2f, u, uhat, flags, out, status)) != HDG_OK) return st;
    int bad = big;
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(&bad, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HDG_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    if (bad != big) {
        ctx->err = "hdg_element_blocks: non-positive mass-matrix pivot in element " + std::to_string(bad);
        return HDG_ERR_SINGULAR;
    }
    return HDG_OK;
    GUARD_END
}

hdg_status hdg_element_blocks_sys(hdg_ctx ctx, const hdg_dims* dims, const hdg_elem_geom* g, const hdg_sys_model* m,
                                  const hdg_time_term* tt, const int32_t* e2f, const double* u, const double* uhat,
                                  int32_t flags, const hdg_elem_arrays* out) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, false);
    if (st != HDG_OK) return st;
    if (!g || !m || !out) return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks_sys: NULL argument struct");
    if (dims->dim != 3) return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks_sys: dim must be 3");
    if (!((m->kind == HDG_MODEL_ELASTICITY && dims->ncomp == 3) ||
          (m->kind == HDG_MODEL_NAVIER_STOKES && dims->ncomp == 5)))
        return set_err(ctx, HDG_ERR_ARG,
                       "hdg_element_blocks_sys: model must be elasticity (ncomp 3) or Navier-Stokes (ncomp 5)");
    if (m->kind == HDG_MODEL_NAVIER_STOKES && !(m->Re > 0.0 && m->Pr > 0.0 && m->gamma > 1.0))
        return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks_sys: need Re > 0, Pr > 0, gamma > 1");
    if (!std::isfinite(m->tau)) return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks_sys: tau is not finite");
    if (g->nqv < 1 || g->nqf < 1)
        return set_err(ctx, HDG_ERR_SHAPE, "hdg_element_blocks_sys: nqv and nqf must be >= 1");
    if (dims->ne == 0) return HDG_OK;
    if (!g->wdet || !g->dphix || !g->phi || !g->phif || !g->psi || !g->ndA || !g->dA || !g->src || !g->uD ||
        !g->bnd || !e2f || !u || !uhat || !out->ru || !out->rt)
        return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks_sys: NULL pointer");
    const bool residual_only = (flags & HDG_ELEM_RESIDUAL_ONLY) != 0;
    if (flags & ~(HDG_ELEM_RESIDUAL_ONLY | HDG_ELEM_KEEP_MASS))
        return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks_sys: unknown flags");
    if ((flags & HDG_ELEM_KEEP_MASS) && !out->Minv)
        return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks_sys: HDG_ELEM_KEEP_MASS needs the kept Minv");
    if (!residual_only && (!out->Minv || !out->Bd || !out->Cd || !out->D || !out->E || !out->F || !out->G ||
                           !out->H || !out->J))
        return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks_sys: NULL matrix output (residual_only = 0)");
    if (tt && !std::isfinite(tt->c))
        return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks_sys: time-term factor c is not finite");
    if (tt && tt->c != 0.0 && !tt->u_prev)
        return set_err(ctx, HDG_ERR_ARG, "hdg_element_blocks_sys: time term with c != 0 needs u_prev");
    if (element_sys_lds_bytes(dims, g->nqv, g->nqf) > 150 * 1024)
        return set_err(ctx, HDG_ERR_SHAPE, "hdg_element_blocks_sys: element data exceed 150 KiB of LDS");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    const size_t per = element_sys_ws_doubles(dims, g->nqv, g->nqf);
    int64_t chunk = (int64_t)(((size_t)1 << 30) / (per * sizeof(double)));
    if (chunk < 1) chunk = 1;
    if (chunk > dims->ne) chunk = dims->ne;
    double* ws = (double*)ws_get(ctx, WS_ELEM_SYS, sizeof(double) * per * (size_t)chunk, &st);
    if (!ws) return st;
    int* status = (int*)ws_get(ctx, WS_STATUS, 64, &st);
    if (!status) return st;
    const int big = 0x7fffffff;
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(status, &big, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    for (int64_t e0 = 0; e0 < dims->ne; e0 += chunk) {
        const int64_t n = (dims->ne - e0) < chunk ? (dims->ne - e0) : chunk;
        if ((st = element_sys_run(ctx, dims, g, m, tt, e2f, u, uhat, flags, out, status, ws, e0, n)) != HDG_OK)
            return st;
    }
    int bad = big;
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(&bad, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HDG_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    if (bad != big) {
        ctx->err = "hdg_element_blocks_sys: non-positive mass-matrix pivot in element " + std::to_string(bad);
        return HDG_ERR_SINGULAR;
    }
    return HDG_OK;
    GUARD_END
}

hdg_status hdg_residual_norm(hdg_ctx ctx, const hdg_dims* dims, const int32_t* f2e, const double* ru,
                             const double* rt, double* norm_h) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    size_t need = 0;
    hdg_status st = residual_norm_check(ctx, dims, f2e, ru, rt, norm_h, &need);
    if (st != HDG_OK) return st;
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    double* base = (double*)ws_get(ctx, WS_NEWTON, sizeof(double) * need, &st);
    if (!base) return st;
    return residual_norm_run(ctx, dims, f2e, ru, rt, base, norm_h);
    GUARD_END
}

hdg_status hdg_residual_norm_noalloc(hdg_ctx ctx, const hdg_dims* dims, const int32_t* f2e, const double* ru,
                                     const double* rt, double* norm_h) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    size_t need = 0;
    hdg_status st = residual_norm_check(ctx, dims, f2e, ru, rt, norm_h, &need);
    if (st != HDG_OK) return st;
    if (need > NOALLOC_SCRATCH_DOUBLES)
        return set_err(ctx, HDG_ERR_ARG,
                       "hdg_residual_norm_noalloc: ncomp*npf*nf plus reduction partials exceed the fixed "
                       "scratch of 2^21 doubles (use hdg_residual_norm)");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    double* base = noalloc_scratch(ctx->device);
    if (!base) return set_err(ctx, HDG_ERR_HIP, "hdg_residual_norm_noalloc: no scratch address for this device");
    return residual_norm_run(ctx, dims, f2e, ru, rt, base, norm_h);
    GUARD_END
}

hdg_status hdg_matvec(hdg_ctx ctx, const hdg_dims* dims, const double* K64, const float* K32, const int32_t* nbr,
                      int32_t precision, const double* x, double* y) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, true);
    if (st != HDG_OK) return st;
    const bool m32 = precision == HDG_MIXED;
    if ((m32 ? (const void*)K32 : (const void*)K64) == nullptr || !nbr || !x || !y)
        return set_err(ctx, HDG_ERR_ARG, "hdg_matvec: NULL pointer");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return op_apply_run(ctx, dims, m32 ? (const void*)K32 : (const void*)K64, m32, nbr, 2 * dims->nlfe - 1, x, y);
    GUARD_END
}

hdg_status hdg_autotune(hdg_ctx ctx, const hdg_dims* dims, const double* K64, const float* K32, const int32_t* nbr,
                        const double* Binv64, const float* Binv32, int32_t reps, int32_t* n_tuned_h) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, true);
    if (st != HDG_OK) return st;
    if (!K64 || !nbr) return set_err(ctx, HDG_ERR_ARG, "hdg_autotune: K64 and nbr are required");
    if (reps < 1 || reps > 1000) return set_err(ctx, HDG_ERR_ARG, "hdg_autotune: reps must be in [1, 1000]");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    const int nb = dims->ncomp * dims->npf, L = dims->nlfe, S = 2 * L - 1, nf = dims->nf;
    const size_t N = (size_t)nf * nb;
    double* x = (double*)ws_get(ctx, WS_VEC, sizeof(double) * 2 * N, &st);
    if (!x) return st;
    double* y = x + N;
    HDG_HIP_CHECK(ctx, hipMemsetAsync(x, 0, sizeof(double) * N, ctx->stream));
    int n = 0;
    double us = 0.0;
    struct V {
        const void* M1;
        bool m1_32;
        const int32_t* nbr;
        int S1;
        const void* M2;
        bool m2_32;
    };
    const V vars[6] = {{K64, false, nbr, S, nullptr, false},       {K32, true, nbr, S, nullptr, false},
                       {Binv64, false, nullptr, 1, nullptr, false}, {Binv32, true, nullptr, 1, nullptr, false},
                       {K64, false, nbr, S, Binv64, false},         {K32, true, nbr, S, Binv32, true}};
    for (int v = 0; v < 6; ++v) {
        const V& c = vars[v];
        if (!c.M1 || (v >= 4 && !c.M2)) continue;
        if ((st = face_autotune(ctx, nf, nb, c.S1, L, c.M1, c.m1_32, c.nbr, c.M2, c.m2_32, x, y, reps, &us)) !=
            HDG_OK)
            return st;
        ++n;
    }
    if (!tune_save()) return set_err(ctx, HDG_ERR_ARG, "hdg_autotune: could not write the HDG_TUNE_CACHE file");
    if (n_tuned_h) *n_tuned_h = n;
    return HDG_OK;
    GUARD_END
}

size_t hdg_tune_table(char* buf_h, size_t len) {
    try {
        const std::string t = tune_json();
        if (buf_h && len > 0) {
            const size_t k = t.size() < len - 1 ? t.size() : len - 1;
            std::memcpy(buf_h, t.data(), k);
            buf_h[k] = '\0';
        }
        return t.size() + 1;
    } catch (...) {
        return 0;
    }
}

hdg_status hdg_bj_setup(hdg_ctx ctx, const hdg_dims* dims, const double* K64, double* Binv64, float* Binv32) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, true);
    if (st != HDG_OK) return st;
    if (!K64 || !Binv64) return set_err(ctx, HDG_ERR_ARG, "hdg_bj_setup: NULL pointer");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    int* status = (int*)ws_get(ctx, WS_STATUS, 64, &st);
    if (!status) return st;
    const int big = 0x7fffffff;
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(status, &big, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    st = bj_invert(ctx, dims->nf, dims->ncomp * dims->npf, 2 * dims->nlfe - 1, K64, Binv64, Binv32, status);
    if (st != HDG_OK) return st;
    int bad = big;
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(&bad, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HDG_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    if (bad != big) {
        ctx->err = "block-Jacobi: zero or non-finite pivot in the diagonal block of face " + std::to_string(bad);
        return HDG_ERR_SINGULAR;
    }
    return HDG_OK;
    GUARD_END
}

hdg_status hdg_bj_apply(hdg_ctx ctx, const hdg_dims* dims, const double* Binv64, const float* Binv32,
                        int32_t precision, const double* y, double* z) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, true);
    if (st != HDG_OK) return st;
    const bool m32 = precision == HDG_MIXED;
    if ((m32 ? (const void*)Binv32 : (const void*)Binv64) == nullptr || !y || !z)
        return set_err(ctx, HDG_ERR_ARG, "hdg_bj_apply: NULL pointer");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return op_apply_run(ctx, dims, m32 ? (const void*)Binv32 : (const void*)Binv64, m32, nullptr, 1, y, z);
    GUARD_END
}

hdg_status hdg_asm_setup(hdg_ctx ctx, const hdg_dims* dims, const double* Kbar, const double* K64,
                         const int32_t* e2f, double* inv64, float* inv32) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, true);
    if (st != HDG_OK) return st;
    if (dims->ne == 0) return HDG_OK;
    if (!Kbar || !K64 || !e2f || (!inv64 && !inv32)) return set_err(ctx, HDG_ERR_ARG, "hdg_asm_setup: NULL pointer");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return asm_setup_run(ctx, dims, Kbar, K64, e2f, inv64, inv32);
    GUARD_END
}

hdg_status hdg_asm_apply(hdg_ctx ctx, const hdg_dims* dims, const double* inv64, const float* inv32,
                         int32_t precision, const int32_t* f2e, const int32_t* e2f, const double* y, double* z) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, true);
    if (st != HDG_OK) return st;
    const bool m32 = precision == HDG_MIXED;
    if ((m32 ? (const void*)inv32 : (const void*)inv64) == nullptr || !f2e || !e2f || !y || !z || y == z)
        return set_err(ctx, HDG_ERR_ARG, "hdg_asm_apply: NULL or aliased pointer");
    if (dims->ne <= 0) return set_err(ctx, HDG_ERR_SHAPE, "hdg_asm_apply: dims->ne must be > 0");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return asm_apply_run(ctx, dims, m32 ? (const void*)inv32 : (const void*)inv64, m32, f2e, e2f, y, z);
    GUARD_END
}

hdg_status hdg_poly_apply(hdg_ctx ctx, const hdg_dims* dims, const double* K64, const float* K32,
                          const int32_t* nbr, const double* Binv64, const float* Binv32, int32_t precision,
                          int32_t npoly, const double* tre, const double* tim, const double* y, double* z) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, true);
    if (st != HDG_OK) return st;
    const bool m32 = precision == HDG_MIXED;
    if ((m32 ? (const void*)K32 : (const void*)K64) == nullptr || !nbr || !y || !z || y == z ||
        (m32 ? (const void*)Binv32 : (const void*)Binv64) == nullptr)
        return set_err(ctx, HDG_ERR_ARG, "hdg_poly_apply: NULL or aliased pointer");
    if (npoly < 0 || npoly > 64 || (npoly > 0 && (!tre || !tim)))
        return set_err(ctx, HDG_ERR_ARG, "hdg_poly_apply: npoly must be in [0, 64] with theta arrays");
    for (int i = 0; i < npoly; ++i) {
        if (tre[i] == 0.0 && tim[i] == 0.0) return set_err(ctx, HDG_ERR_ARG, "hdg_poly_apply: zero Ritz value");
        if (tim[i] != 0.0 && (i + 1 >= npoly || tim[i] < 0.0 || tre[i + 1] != tre[i] || tim[i + 1] != -tim[i]))
            return set_err(ctx, HDG_ERR_ARG, "hdg_poly_apply: complex values must come as adjacent (a+ib, a-ib)");
        if (tim[i] != 0.0) ++i;
    }
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return poly_apply_run(ctx, dims, K64, K32, nbr, Binv64, Binv32, precision, npoly, tre, tim, y, z);
    GUARD_END
}

hdg_status hdg_cheb_apply(hdg_ctx ctx, const hdg_dims* dims, const double* K64, const float* K32,
                          const int32_t* nbr, const double* Binv64, const float* Binv32, int32_t precision,
                          int32_t degree, double alpha, double beta, const double* y, double* z) {
    if (!ctx) return HDG_ERR_ARG;
    GUARD_BEGIN
    hdg_status st = check_dims(ctx, dims, false, true);
    if (st != HDG_OK) return st;
    const bool m32 = precision == HDG_MIXED;
    if ((m32 ? (const void*)K32 : (const void*)K64) == nullptr || !nbr || !y || !z || y == z ||
        (m32 ? (const void*)Binv32 : (const void*)Binv64) == nullptr)
        return set_err(ctx, HDG_ERR_ARG, "hdg_cheb_apply: NULL or aliased pointer");
    if (degree < 1 || degree > 64) return set_err(ctx, HDG_ERR_ARG, "hdg_cheb_apply: degree must be in [1, 64]");
    if (!(alpha > 0.0) || !(beta > alpha) || !std::isfinite(beta))
        return set_err(ctx, HDG_ERR_ARG, "hdg_cheb_apply: need 0 < alpha < beta < inf");
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    return cheb_apply_run(ctx, dims, K64, K32, nbr, Binv64, Binv32, precision, degree, alpha, beta, y, z);
    GUARD_END
}

int hdg_hessenberg_eigvals(int n, const double* H_h, int ld, double* wr, double* wi) {
    if (n < 1 || !H_h || !wr || !wi || ld < n) return -1;
    try {
        std::vector<double> H((size_t)n * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) H[(size_t)i * n + j] = (j >= i - 1) ? H_h[(size_t)i * ld + j] : 0.0;
        return hessenberg_eigvals(n, H.data(), n, wr, wi);
    } catch (...) {
        return -3;
    }
}

int hdg_harmonic_ritz(int P, const double* H_h, double drop_rel, double* tre, double* tim, int* n_out) {
    if (P < 1 || !H_h || !tre || !tim || !n_out) return -1;
    try {
        return harmonic_ritz_leja(P, H_h, drop_rel, tre, tim, n_out);
    } catch (...) {
        return -3;
    }
}

int hdg_poly_roots(int P, const double* H_h, double drop_rel, double* tre, double* tim, int* n_out, int* n_added) {
    if (P < 1 || !H_h || !tre || !tim || !n_out || !n_added) return -1;
    try {
        return poly_roots(P, H_h, drop_rel, tre, tim, n_out, n_added);
    } catch (...) {
        return -3;
    }
}

}  // extern "C"
