// Preconditioned restarted FGMRES driver (Sections 3.1-3.4, 4.4-4.7).
//
// Right-preconditioned flexible GMRES(m): the cycle-start residual r = b - K64 x
// is always formed in FP64 from the FP64 matrix; inside a cycle the operator and
// the preconditioner use either the FP64 data or (mixed precision) the FP32
// matrix and FP32 block inverses with FP64 vectors, so every restart is a step
// of iterative refinement. Orthogonalisation (CGS2 / CGS / MGS), the Hessenberg
// Givens update and the solution update are FP64.
//
// Host/device traffic: the host enqueues a whole cycle (FP64 residual, all m
// Arnoldi steps, back substitution, update), optionally as one captured hipGraph;
// every in-cycle kernel reads a device "done" word and returns at once after
// convergence, so the host synchronises once per cycle.
//
// Preconditioners (z = Prec(y)):
//   BJ       z_f = P_f^{-1} y_f                                   (Section 4.5)
//   BJ-PP(P) z = p(B) t, t = M^{-1} y, B = M^{-1} K, with the Leja-ordered
//            harmonic Ritz values of B (Section 4.7). The recurrence
//              real theta:  w += q/theta,           q <- q - Bq/theta
//              pair a+-ib:  w += (2a q - Bq)/|theta|^2,
//                           q <- q - (2a/|theta|^2) Bq + (1/|theta|^2) B^2 q
//            runs in fused face kernels (K-product, block-Jacobi and the vector
//            updates in one pass); the last q update is skipped, so P roots cost
//            P-1 applications of B. (The pair update of q follows from the product
//            form of the polynomial; the printed version of that line lacks the
//            Bq term.)
//   BJ-Cheb  Chebyshev acceleration of degree P on B over [alpha, beta] with
//            beta = 1.05 max Re(theta), alpha = max(min Re(theta), beta/1000).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "hdg_internal.hpp"

namespace {

// Preconditioner M^{-1} inside an operator: identity (block-Jacobi folded into K), block-Jacobi,
// or element-patch additive Schwarz.
enum { PK_IDENTITY = 0, PK_BJ = 1, PK_ASM = 2, PK_ILU = 3 };

struct Op {
    int nf, nb, S, L;
    size_t N;
    const void* K;        // operator matrix (K64 or K32)
    bool k32;
    const void* Binv;     // block-Jacobi inverses (64 or 32)
    bool b32;
    const int32_t* nbr;
    int pk = PK_BJ;
    // additive Schwarz
    const void* asm_inv = nullptr;
    bool asm32 = false;
    const int32_t* unbr = nullptr;
    const int32_t* f2e = nullptr;
    double* zu = nullptr;
    double* tmp = nullptr;
    int64_t ne = 0;
    const hdg_ilu_asm_s* ilu = nullptr;   // ILU-ASM factors
};

FaceEpilogue epi0() {
    FaceEpilogue e;
    for (int o = 0; o < 3; ++o) {
        e.out[o] = nullptr;
        e.X[o] = nullptr;
        e.Y[o] = nullptr;
        e.s[o] = e.a[o] = e.b[o] = 0.0;
    }
    return e;
}

// out = s*(M1 x) [+ a X + b Y] with M1 = K (product) ...
hdg_status op_matvec(hdg_ctx ctx, const Op& op, const double* x, double* y, const int* skip) {
    FaceEpilogue e = epi0();
    e.out[0] = y;
    e.s[0] = 1.0;
    return face_op(ctx, op.nf, op.nb, op.S, op.L, op.K, op.k32, op.nbr, nullptr, false, x, e, skip);
}

// out = epilogue(M^{-1} y)
hdg_status op_bj(hdg_ctx ctx, const Op& op, const double* y, const FaceEpilogue& e, const int* skip) {
    if (op.pk == PK_ASM)
        return asm_apply_op(ctx, op.nf, op.nb, op.L, op.ne, op.asm_inv, op.asm32, op.unbr, op.f2e, op.zu, y, e, skip);
    if (op.pk == PK_ILU) return ilu_apply_op(ctx, op.ilu, y, e, skip);
    const void* M = op.pk == PK_BJ ? op.Binv : nullptr;      // nullptr: identity
    return face_op(ctx, op.nf, op.nb, 1, op.L, M, op.b32, nullptr, nullptr, false, y, e, skip);
}

// out = epilogue(M^{-1} K x): one fused kernel for block-Jacobi (and the identity), the
// product then the Schwarz operator otherwise
hdg_status op_B(hdg_ctx ctx, const Op& op, const double* x, const FaceEpilogue& e, const int* skip) {
    if (op.pk == PK_ASM || op.pk == PK_ILU) {
        hdg_status st = op_matvec(ctx, op, x, op.tmp, skip);
        if (st != HDG_OK) return st;
        return op_bj(ctx, op, op.tmp, e, skip);
    }
    const void* M2 = op.pk == PK_BJ ? op.Binv : nullptr;
    return face_op(ctx, op.nf, op.nb, op.S, op.L, op.K, op.k32, op.nbr, M2, op.b32, x, e, skip);
}

struct PolyPlan {
    int kind = HDG_PREC_BJ;        // BJ_POLY or BJ_CHEB
    std::vector<double> tre, tim;  // Leja-ordered Ritz values
    int P = 0;
    double alpha = 0, beta = 0;    // Chebyshev interval
};

// work vectors: 5 x ld
hdg_status poly_apply(hdg_ctx ctx, const Op& op, const PolyPlan& pl, const double* y, double* z, double* work,
                      size_t ld, const int* skip) {
    double* t = work;
    double* qa = work + ld;
    double* qb = work + 2 * ld;
    double* ub = work + 3 * ld;
    double* xc = work + 4 * ld;
    hdg_status st;
    if (pl.kind == HDG_PREC_BJ_CHEB) {
        const double th = 0.5 * (pl.beta + pl.alpha), de = 0.5 * (pl.beta - pl.alpha);
        const double s1 = th / de;
        double rho = 1.0 / s1;
        double* r = t;
        double* dcur = qa;
        double* dnext = qb;
        FaceEpilogue e = epi0();
        e.out[0] = r;
        e.s[0] = 1.0;
        e.out[1] = dcur;
        e.s[1] = 1.0 / th;
        if ((st = op_bj(ctx, op, y, e, skip)) != HDG_OK) return st;
        bool xinit = false;
        for (int k = 1; k < pl.P; ++k) {
            const double rn = 1.0 / (2.0 * s1 - rho);
            FaceEpilogue f = epi0();
            f.out[0] = r;  f.s[0] = -1.0; f.X[0] = r; f.a[0] = 1.0;
            f.out[1] = dnext; f.s[1] = -2.0 * rn / de; f.X[1] = dcur; f.a[1] = rn * rho; f.Y[1] = r; f.b[1] = 2.0 * rn / de;
            f.out[2] = xc; f.s[2] = 0.0; f.X[2] = xinit ? xc : nullptr; f.a[2] = 1.0; f.Y[2] = dcur; f.b[2] = 1.0;
            if ((st = op_B(ctx, op, dcur, f, skip)) != HDG_OK) return st;
            xinit = true;
            std::swap(dcur, dnext);
            rho = rn;
        }
        return vec_lincomb(ctx, op.N, z, 1.0, xinit ? xc : nullptr, 1.0, dcur, skip);
    }
    // harmonic-Ritz polynomial
    FaceEpilogue e = epi0();
    e.out[0] = t;
    e.s[0] = 1.0;
    if ((st = op_bj(ctx, op, y, e, skip)) != HDG_OK) return st;
    const int n = (int)pl.tre.size();
    if (n == 0) return vec_lincomb(ctx, op.N, z, 1.0, t, 0.0, nullptr, skip);
    const double* q = t;
    bool winit = false;
    int j = 0;
    while (j < n) {
        const bool pair = pl.tim[j] != 0.0;
        const int width = pair ? 2 : 1;
        const bool last = j + width >= n;
        double* qn = (q == qa) ? qb : qa;
        if (!pair) {
            const double th = pl.tre[j];
            if (last) {
                if ((st = vec_lincomb(ctx, op.N, z, 1.0, winit ? z : nullptr, 1.0 / th, q, skip)) != HDG_OK) return st;
            } else {
                FaceEpilogue f = epi0();
                f.out[0] = qn; f.s[0] = -1.0 / th; f.X[0] = q; f.a[0] = 1.0;
                f.out[1] = z;  f.s[1] = 0.0; f.X[1] = winit ? z : nullptr; f.a[1] = 1.0; f.Y[1] = q; f.b[1] = 1.0 / th;
                if ((st = op_B(ctx, op, q, f, skip)) != HDG_OK) return st;
                q = qn;
            }
        } else {
            const double a = pl.tre[j];
            const double m2 = pl.tre[j] * pl.tre[j] + pl.tim[j] * pl.tim[j];
            FaceEpilogue f = epi0();
            f.out[0] = z; f.s[0] = -1.0 / m2; f.X[0] = winit ? z : nullptr; f.a[0] = 1.0; f.Y[0] = q; f.b[0] = 2.0 * a / m2;
            if (!last) { f.out[1] = ub; f.s[1] = 1.0; }
            if ((st = op_B(ctx, op, q, f, skip)) != HDG_OK) return st;
            if (!last) {
                FaceEpilogue g = epi0();
                g.out[0] = qn; g.s[0] = 1.0 / m2; g.X[0] = q; g.a[0] = 1.0; g.Y[0] = ub; g.b[0] = -2.0 * a / m2;
                if ((st = op_B(ctx, op, ub, g, skip)) != HDG_OK) return st;
                q = qn;
            }
        }
        winit = true;
        j += width;
    }
    return HDG_OK;
}

hdg_status prec_apply(hdg_ctx ctx, const Op& op, int prec, const PolyPlan& pl, const double* y, double* z,
                      double* work, size_t ld, const int* skip) {
    if (prec == HDG_PREC_NONE) return vec_lincomb(ctx, op.N, z, 1.0, y, 0.0, nullptr, skip);
    if (prec == HDG_PREC_BJ || prec == HDG_PREC_ASM || prec == HDG_PREC_ILU_ASM) {
        FaceEpilogue e = epi0();
        e.out[0] = z;
        e.s[0] = 1.0;
        return op_bj(ctx, op, y, e, skip);
    }
    return poly_apply(ctx, op, pl, y, z, work, ld, skip);
}

// hipEvents owned for the duration of one solve (timing only)
struct EventPool {
    std::vector<hipEvent_t> e;
    hdg_status create(int n) {
        e.assign(n, nullptr);
        for (auto& x : e)
            if (hipEventCreate(&x) != hipSuccess) { x = nullptr; return HDG_ERR_HIP; }
        return HDG_OK;
    }
    ~EventPool() {
        for (auto x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

struct SolveWs {
    double *V, *Z, *work, *part;
    GmresCtl* ctl;
    double *H, *cs, *sn, *g, *y, *h2, *hist, *bnorm;
    double *Hu, *coef;          // delayed CGS2: unrotated Hessenberg, update coefficients
    size_t ld;
    int nblk, ldh;
};

// zcols: columns of Z (m for the flexible form; the delayed-CGS2 form keeps no Z and
// uses two columns as temporaries)
hdg_status alloc_solve_ws(hdg_ctx ctx, size_t N, int m, int P, int zcols, SolveWs* w) {
    hdg_status st;
    w->ld = (N + 63) / 64 * 64;
    const int mv = std::max(m, P);
    w->V = (double*)ws_get(ctx, WS_KRYLOV_V, sizeof(double) * w->ld * (size_t)(mv + 1), &st);
    if (!w->V) return st;
    w->Z = (double*)ws_get(ctx, WS_KRYLOV_Z, sizeof(double) * w->ld * (size_t)zcols, &st);
    if (!w->Z) return st;
    w->work = (double*)ws_get(ctx, WS_VEC, sizeof(double) * w->ld * 5, &st);
    if (!w->work) return st;
    w->nblk = krylov_nblk(N);
    w->part = (double*)ws_get(ctx, WS_PART, sizeof(double) * (size_t)w->nblk * (2 * mv + 4), &st);
    if (!w->part) return st;
    w->ldh = mv + 1;
    const size_t nctl = 8 + 2 * (size_t)w->ldh * mv + 6 * (size_t)(mv + 2) + 3 * (size_t)w->ldh + 1;
    char* base = (char*)ws_get(ctx, WS_CTL, sizeof(double) * nctl + sizeof(GmresCtl), &st);
    if (!base) return st;
    w->ctl = (GmresCtl*)base;
    double* p = (double*)(base + sizeof(GmresCtl));
    w->H = p; p += (size_t)w->ldh * mv;
    w->cs = p; p += mv + 2;
    w->sn = p; p += mv + 2;
    w->g = p; p += mv + 2;
    w->y = p; p += mv + 2;
    w->h2 = p; p += mv + 2;
    w->hist = p; p += mv + 2;
    w->Hu = p; p += (size_t)w->ldh * mv;
    w->coef = p; p += 3 * (size_t)w->ldh + 1;
    w->bnorm = p;
    return HDG_OK;
}

hdg_status orthogonalise(hdg_ctx ctx, const SolveWs& w, size_t N, int j, int orth, const int* skip) {
    hdg_status st;
    double* wv = w.V + (size_t)(j + 1) * w.ld;
    double* col = w.H + (size_t)j * w.ldh;
    if (orth == HDG_ORTH_MGS) {
        for (int i = 0; i <= j; ++i) {
            if ((st = vec_multidot(ctx, w.V + (size_t)i * w.ld, w.ld, 1, wv, N, w.part, w.nblk, skip)) != HDG_OK) return st;
            if ((st = vec_reduce(ctx, w.part, 1, w.nblk, col + i, nullptr, skip)) != HDG_OK) return st;
            if ((st = vec_multiaxpy(ctx, w.V + (size_t)i * w.ld, w.ld, 1, col + i, -1.0, wv, N, skip)) != HDG_OK) return st;
        }
        return HDG_OK;
    }
    if ((st = vec_multidot(ctx, w.V, w.ld, j + 1, wv, N, w.part, w.nblk, skip)) != HDG_OK) return st;
    if ((st = vec_reduce(ctx, w.part, j + 1, w.nblk, col, nullptr, skip)) != HDG_OK) return st;
    if ((st = vec_multiaxpy(ctx, w.V, w.ld, j + 1, col, -1.0, wv, N, skip)) != HDG_OK) return st;
    if (orth == HDG_ORTH_CGS2) {
        if ((st = vec_multidot(ctx, w.V, w.ld, j + 1, wv, N, w.part, w.nblk, skip)) != HDG_OK) return st;
        if ((st = vec_reduce(ctx, w.part, j + 1, w.nblk, w.h2, col, skip)) != HDG_OK) return st;
        if ((st = vec_multiaxpy(ctx, w.V, w.ld, j + 1, w.h2, -1.0, wv, N, skip)) != HDG_OK) return st;
    }
    return HDG_OK;
}

// One MGS Arnoldi cycle of length P on B = M^{-1} K from v0; returns H (P+1) x P row-major on the host.
hdg_status arnoldi_setup(hdg_ctx ctx, const Op& op, const SolveWs& w, const double* v0, int P,
                         std::vector<double>& Hh, int* Peff) {
    hdg_status st;
    const size_t N = op.N;
    if ((st = vec_sumsq_partial(ctx, v0, N, w.part, w.nblk, nullptr)) != HDG_OK) return st;
    if ((st = krylov_store_norm(ctx, w.part, w.nblk, w.bnorm + 1)) != HDG_OK) return st;
    if ((st = krylov_scale_by(ctx, w.V, v0, N, w.bnorm + 1, nullptr)) != HDG_OK) return st;
    for (int j = 0; j < P; ++j) {
        double* wv = w.V + (size_t)(j + 1) * w.ld;
        FaceEpilogue e = epi0();
        e.out[0] = wv;
        e.s[0] = 1.0;
        if ((st = op_B(ctx, op, w.V + (size_t)j * w.ld, e, nullptr)) != HDG_OK) return st;
        if ((st = orthogonalise(ctx, w, N, j, HDG_ORTH_MGS, nullptr)) != HDG_OK) return st;
        if ((st = vec_sumsq_partial(ctx, wv, N, w.part, w.nblk, nullptr)) != HDG_OK) return st;
        double* hn = w.H + (size_t)j * w.ldh + (j + 1);
        if ((st = krylov_store_norm(ctx, w.part, w.nblk, hn)) != HDG_OK) return st;
        if ((st = krylov_scale_by(ctx, wv, wv, N, hn, nullptr)) != HDG_OK) return st;
    }
    std::vector<double> Hc((size_t)w.ldh * P);
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(Hc.data(), w.H, sizeof(double) * Hc.size(), hipMemcpyDeviceToHost, ctx->stream));
    HDG_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    // stop at a breakdown: h_{j+1,j} zero, or below 1e-12 of the norm of B v_j (the column's
    // 2-norm), where rounding leaves a vector with no direction of its own; use the leading block
    int pe = P;
    for (int j = 0; j < P; ++j) {
        double c2 = 0.0;
        for (int i = 0; i <= j + 1; ++i) c2 += Hc[(size_t)j * w.ldh + i] * Hc[(size_t)j * w.ldh + i];
        const double h = Hc[(size_t)j * w.ldh + j + 1];
        if (!(h > 1e-12 * std::sqrt(c2))) { pe = j + 1; break; }
    }
    // only rows 0..j+1 of column j are ever written on the device; the rest of
    // the Hessenberg matrix is zero by definition, not whatever the workspace holds
    Hh.assign((size_t)(pe + 1) * pe, 0.0);
    for (int j = 0; j < pe; ++j)
        for (int i = 0; i <= j + 1; ++i) Hh[(size_t)i * pe + j] = Hc[(size_t)j * w.ldh + i];
    *Peff = pe;
    return HDG_OK;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

void hdg_solve_opts_default(hdg_solve_opts* o) {
    std::memset(o, 0, sizeof(*o));
    o->restart = 50;
    o->max_iters = 1000;
    o->rtol = 1e-8;
    o->atol = 0.0;
    o->prec = HDG_PREC_BJ;
    o->poly_degree = 10;
    o->orth = HDG_ORTH_CGS2;
    o->precision = HDG_FP64;
}

hdg_status solve_run(hdg_ctx ctx, const hdg_dims* d, const double* K64, const float* K32, const int32_t* nbr,
                     const double* b, double* x, const hdg_solve_opts* o, hdg_solve_stats* stats) {
    const double t0 = now_s();
    const bool timed = o->time_phases != 0;
    const bool use_graph = o->use_graph && !timed;
    CaptureStreamScope cap;
    if (use_graph) HDG_HIP_CHECK(ctx, cap.begin(ctx));
    std::memset(stats, 0, sizeof(*stats));
    const int nb = d->ncomp * d->npf, L = d->nlfe, S = 2 * L - 1, nf = d->nf;
    const size_t N = (size_t)nf * nb;
    const bool mixed = o->precision == HDG_MIXED;
    const int m = o->restart;
    const bool poly = o->prec == HDG_PREC_BJ_POLY || o->prec == HDG_PREC_BJ_CHEB || o->prec == HDG_PREC_ASM_POLY ||
                      o->prec == HDG_PREC_ASM_CHEB;
    const bool schwarz = o->prec == HDG_PREC_ASM || o->prec == HDG_PREC_ASM_POLY || o->prec == HDG_PREC_ASM_CHEB;
    const int P = poly ? o->poly_degree : 0;
    hdg_status st;
    SolveWs w;
    const bool dcgs2 = o->orth == HDG_ORTH_DCGS2;
    if ((st = alloc_solve_ws(ctx, N, m, P, dcgs2 ? 2 : m, &w)) != HDG_OK) return st;
    Op op;
    op.nf = nf; op.nb = nb; op.S = S; op.L = L; op.N = N; op.nbr = nbr;
    op.K = mixed ? (const void*)K32 : (const void*)K64;
    op.k32 = mixed;
    op.Binv = nullptr;
    op.b32 = mixed;
    Op op64 = op;
    op64.K = K64;
    op64.k32 = false;
    if (schwarz) {
        // element-patch additive Schwarz: unit neighbour table, unit results, work vector
        const int64_t ne = d->ne;
        const size_t nunit = (size_t)ne * L;
        const size_t bytes = sizeof(int32_t) * nunit * L + sizeof(double) * (nunit * nb + N) + 256;
        char* base = (char*)ws_get(ctx, WS_ASM, bytes, &st);
        if (!base) return st;
        double* zu = (double*)base;
        double* tmp = zu + nunit * nb;
        int32_t* unbr = (int32_t*)(tmp + N);
        if ((st = asm_unit_nbr(ctx, ne, L, o->asm_e2f, unbr)) != HDG_OK) return st;
        op.pk = op64.pk = PK_ASM;
        op.asm_inv = mixed ? (const void*)o->asm_inv32 : (const void*)o->asm_inv64;
        op.asm32 = mixed;
        op64.asm_inv = o->asm_inv64;
        op64.asm32 = false;
        op.unbr = op64.unbr = unbr;
        op.f2e = op64.f2e = o->asm_f2e;
        op.zu = op64.zu = zu;
        op.tmp = op64.tmp = tmp;
        op.ne = op64.ne = ne;
    } else if (o->prec == HDG_PREC_ILU_ASM) {
        // multi-element subdomains with block ILU(0): factors held by the handle
        op.pk = op64.pk = PK_ILU;
        op.ilu = op64.ilu = o->ilu_asm;
        op.tmp = op64.tmp = ilu_tmp(o->ilu_asm);
    } else if (o->prec != HDG_PREC_NONE) {
        double* B64 = (double*)ws_get(ctx, WS_BINV64, sizeof(double) * (size_t)nf * nb * nb, &st);
        if (!B64) return st;
        float* B32 = nullptr;
        if (mixed) {
            B32 = (float*)ws_get(ctx, WS_BINV32, sizeof(float) * (size_t)nf * nb * nb, &st);
            if (!B32) return st;
        }
        BjSetupKey want;
        want.valid = true;
        want.mixed = mixed;
        want.K64 = K64;
        want.nbr = nbr;
        want.nf = nf;
        want.nb = nb;
        want.S = S;
        const BjSetupKey& have = ctx->bj_key;
        if (o->reuse_setup) {
            // the inverses (and folded blocks) of an earlier solve on the same matrix
            if (!(have.valid && have.mixed == mixed && have.K64 == K64 && have.nbr == nbr && have.nf == nf &&
                  have.nb == nb && have.S == S)) {
                ctx->err = "reuse_setup: this context holds no block-Jacobi setup of this matrix and precision";
                return HDG_ERR_ARG;
            }
        } else {
            ctx->bj_key.valid = false;
            int* status = (int*)ws_get(ctx, WS_STATUS, 64, &st);
            if (!status) return st;
            const int big = 0x7fffffff;
            HDG_HIP_CHECK(ctx, hipMemcpyAsync(status, &big, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
            if ((st = bj_invert(ctx, nf, nb, S, K64, B64, B32, status)) != HDG_OK) return st;
            int bad = big;
            HDG_HIP_CHECK(ctx, hipMemcpyAsync(&bad, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
            HDG_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
            if (bad != big) {
                ctx->err = "block-Jacobi: zero or non-finite pivot in the diagonal block of face " + std::to_string(bad);
                return HDG_ERR_SINGULAR;
            }
            ctx->bj_key = want;
        }
        op.Binv = mixed ? (const void*)B32 : (const void*)B64;
        op64.Binv = B64;
        op64.b32 = false;
    }
    // operator of the Arnoldi steps: K, or the folded K M^{-1} blocks
    bool fold = o->fold_prec != 0 && dcgs2 && o->prec != HDG_PREC_NONE && !schwarz && o->prec != HDG_PREC_ILU_ASM;
    // the preconditioner the Arnoldi steps apply: o->prec, or its base (block-Jacobi or additive
    // Schwarz alone) when the polynomial setup falls back
    int prec = o->prec;
    Op opi = op;
    if (fold) {
        const size_t nblk_el = (size_t)nf * S * nb * nb;
        const bool had_fold = o->reuse_setup && ctx->bj_key.valid && ctx->bj_key.fold;
        void* Kf = ws_get(ctx, WS_KFOLD, nblk_el * (mixed ? sizeof(float) : sizeof(double)), &st);
        if (!Kf) return st;
        if (!(had_fold && ctx->bj_key.valid)) {
            if ((st = fold_bj(ctx, nf, nb, S, K64, nbr, op64.Binv ? (const double*)op64.Binv : nullptr, Kf,
                              mixed)) != HDG_OK)
                return st;
            // the inverses are those of this matrix either way (computed or checked above)
            ctx->bj_key.valid = true;
            ctx->bj_key.mixed = mixed;
            ctx->bj_key.K64 = K64;
            ctx->bj_key.nbr = nbr;
            ctx->bj_key.nf = nf;
            ctx->bj_key.nb = nb;
            ctx->bj_key.S = S;
            ctx->bj_key.fold = true;
        }
        opi.K = Kf;
        opi.k32 = mixed;
        opi.Binv = nullptr;
        opi.pk = PK_IDENTITY;
    }
    // ||b||
    if ((st = vec_sumsq_partial(ctx, b, N, w.part, w.nblk, nullptr)) != HDG_OK) return st;
    if ((st = krylov_store_norm(ctx, w.part, w.nblk, w.bnorm)) != HDG_OK) return st;
    double bnorm = 0.0;
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(&bnorm, w.bnorm, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HDG_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    if (!std::isfinite(bnorm)) {
        ctx->err = "right-hand side contains NaN or Inf";
        return HDG_ERR_NONFINITE;
    }
    const double target = std::max(o->rtol * bnorm, o->atol);
    // polynomial preconditioner setup
    PolyPlan plan;
    plan.kind = (o->prec == HDG_PREC_BJ_CHEB || o->prec == HDG_PREC_ASM_CHEB) ? HDG_PREC_BJ_CHEB : HDG_PREC_BJ_POLY;
    if (poly) {
        std::vector<double> Hh;
        int pe = 0;
        if ((st = arnoldi_setup(ctx, op, w, o->poly_v0, P, Hh, &pe)) != HDG_OK) return st;
        std::vector<double> tre(pe + 4), tim(pe + 4);
        int nt = 0, nadd = 0;
        // the Chebyshev interval needs only the extreme values: no added roots there
        const int rc = plan.kind == HDG_PREC_BJ_CHEB
                           ? harmonic_ritz_leja(pe, Hh.data(), 1e-12, tre.data(), tim.data(), &nt)
                           : poly_roots(pe, Hh.data(), 1e-12, tre.data(), tim.data(), &nt, &nadd);
        if (rc != 0) {
            ctx->err = "polynomial preconditioner: eigenvalue iteration did not converge";
            return HDG_ERR_SINGULAR;
        }
        if (pe < P) stats->fallback_flags |= HDG_FALLBACK_PP_BREAKDOWN;
        if (nt - nadd < pe) stats->fallback_flags |= HDG_FALLBACK_PP_SMALL_RITZ;
        if (nadd > 0) stats->fallback_flags |= HDG_FALLBACK_PP_ADDED_ROOT;
        plan.tre.assign(tre.begin(), tre.begin() + nt);
        plan.tim.assign(tim.begin(), tim.begin() + nt);
        plan.P = P;
        stats->npoly = std::min(nt, 64);
        for (int i = 0; i < stats->npoly; ++i) {
            stats->theta_re[i] = plan.tre[i];
            stats->theta_im[i] = plan.tim[i];
        }
        if (plan.kind == HDG_PREC_BJ_CHEB && nt > 0) {
            double lo = INFINITY, hi = -INFINITY;
            for (int i = 0; i < nt; ++i) { lo = std::min(lo, plan.tre[i]); hi = std::max(hi, plan.tre[i]); }
            plan.beta = 1.05 * hi;
            plan.alpha = std::max(lo, plan.beta / 1000.0);
            if (!(plan.beta > 0.0) || !(plan.alpha < plan.beta)) stats->fallback_flags |= HDG_FALLBACK_PP_NO_INTERVAL;
            stats->cheb_alpha = plan.alpha;
            stats->cheb_beta = plan.beta;
        }
        // an Arnoldi breakdown, dropped (near-zero) Ritz values or no positive Chebyshev interval:
        // the polynomial is not trusted and the solve runs with its base preconditioner alone
        if (stats->fallback_flags & (HDG_FALLBACK_PP_BREAKDOWN | HDG_FALLBACK_PP_SMALL_RITZ |
                                     HDG_FALLBACK_PP_NO_INTERVAL)) {
            stats->fallback_flags |= HDG_FALLBACK_PP_TO_BASE;
            prec = schwarz ? HDG_PREC_ASM : HDG_PREC_BJ;
        }
    }
    stats->t_setup = now_s() - t0;
    int iters = 0, cycles = 0, hl = 0;
    auto hist_push = [&](double v) {
        if (o->resid_hist_h && hl < o->resid_hist_len) o->resid_hist_h[hl] = v;
        ++hl;
    };
    GmresCtl hc;
    hdg_status result = HDG_NOT_CONVERGED;
    std::vector<double> hbuf(m + 2);
    const int* skip = &w.ctl->done;
    // phase timing: events at the start of the preconditioner, the matvec and the
    // orthogonalisation of each Arnoldi step, and at the step's end
    EventPool ev;
    if (timed && (st = ev.create(6 * m)) != HDG_OK) {
        ctx->err = "hipEventCreate failed";
        return st;
    }
    auto mark = [&](int j, int k) -> hdg_status {
        if (timed) HDG_HIP_CHECK(ctx, hipEventRecord(ev.e[6 * j + k], ctx->stream));
        return HDG_OK;
    };
    // Events of step j: 0/1 preconditioner, 2/3 matvec, 4/5 orthogonalisation. Where a phase
    // starts or ends with an instrumented kernel the event is recorded at that kernel's own
    // start or end (no separate marker); arm() hands them to the next such launch and
    // settle() records any that no launch took.
    auto arm = [&](hipEvent_t s0, hipEvent_t s1) {
        if (timed) {
            ctx->ext_start = s0;
            ctx->ext_stop = s1;
        }
    };
    auto settle = [&]() -> hdg_status {
        if (!timed) return HDG_OK;
        hipEvent_t s0, s1;
        take_ext_events(ctx, &s0, &s1);
        if (s0) HDG_HIP_CHECK(ctx, hipEventRecord(s0, ctx->stream));
        if (s1) HDG_HIP_CHECK(ctx, hipEventRecord(s1, ctx->stream));
        return HDG_OK;
    };
    auto timed_matvec = [&](int j, const Op& o2, const double* xin, double* yout) -> hdg_status {
        arm(timed ? ev.e[6 * j + 2] : nullptr, timed ? ev.e[6 * j + 3] : nullptr);
        hdg_status s3 = op_matvec(ctx, o2, xin, yout, skip);
        hdg_status s4 = settle();
        return s3 != HDG_OK ? s3 : s4;
    };
    // the preconditioner is timed only where a step applies one (not with block-Jacobi folded)
    bool prec_timed = !(fold && prec == HDG_PREC_BJ);
    // Delayed-CGS2 steps of one cycle (right preconditioning with a fixed preconditioner,
    // no Z): step j applies B = K M^{-1} to vt_j, one inner-product sweep, the coefficient
    // kernel (delayed pass for vt_j, column j-1 and its Givens rotation, new column), one
    // update sweep; a final sweep closes column jmax-1; then x += M^{-1} V y.
    auto enqueue_dcgs2_steps = [&](int jmax) -> hdg_status {
        hdg_status s2;
        double* zt = w.Z;
        double* tv = w.Z + w.ld;
        for (int j = 0; j < jmax; ++j) {
            double* vj = w.V + (size_t)j * w.ld;
            double* wv = w.V + (size_t)(j + 1) * w.ld;
            const double* src = zt;
            if (fold && prec == HDG_PREC_BJ) {
                src = vj;    // folded: nothing left to apply
            } else {
                // block-Jacobi is one face-operator kernel; a polynomial takes a marker at its end
                const bool one_kernel = opi.pk != PK_ASM && prec == HDG_PREC_BJ;
                arm(timed ? ev.e[6 * j] : nullptr, timed && one_kernel ? ev.e[6 * j + 1] : nullptr);
                if ((s2 = prec_apply(ctx, opi, prec, plan, vj, zt, w.work, w.ld, skip)) != HDG_OK) return s2;
                if ((s2 = settle()) != HDG_OK) return s2;
                if (!one_kernel && (s2 = mark(j, 1)) != HDG_OK) return s2;
            }
            if ((s2 = timed_matvec(j, opi, src, wv)) != HDG_OK) return s2;
            arm(timed ? ev.e[6 * j + 4] : nullptr, nullptr);
            if ((s2 = vec_multidot2(ctx, w.V, w.ld, j + 1, vj, wv, N, w.part, w.nblk, skip)) != HDG_OK) return s2;
            if ((s2 = settle()) != HDG_OK) return s2;
            if ((s2 = krylov_dcgs2_coef(ctx, w.ctl, w.part, w.nblk, j, 0, w.Hu, w.H, w.ldh, w.cs, w.sn, w.g, w.coef,
                                        w.ldh, w.hist)) != HDG_OK)
                return s2;
            arm(nullptr, timed ? ev.e[6 * j + 5] : nullptr);
            if ((s2 = vec_dcgs2_update(ctx, w.V, w.ld, j, vj, wv, w.coef, w.ldh, N, skip)) != HDG_OK) return s2;
            if ((s2 = settle()) != HDG_OK) return s2;
        }
        double* vm = w.V + (size_t)jmax * w.ld;
        if ((s2 = vec_multidot2(ctx, w.V, w.ld, jmax + 1, vm, nullptr, N, w.part, w.nblk, skip)) != HDG_OK) return s2;
        if ((s2 = krylov_dcgs2_coef(ctx, w.ctl, w.part, w.nblk, jmax, 1, w.Hu, w.H, w.ldh, w.cs, w.sn, w.g, w.coef,
                                    w.ldh, w.hist)) != HDG_OK)
            return s2;
        if ((s2 = krylov_backsolve(ctx, w.ctl, w.H, w.ldh, w.g, w.y)) != HDG_OK) return s2;
        if (prec == HDG_PREC_NONE) return vec_multiaxpy(ctx, w.V, w.ld, jmax, w.y, 1.0, x, N, nullptr, &w.ctl->k);
        if ((s2 = vec_lincomb(ctx, N, tv, 0.0, nullptr, 0.0, nullptr, nullptr)) != HDG_OK) return s2;
        if ((s2 = vec_multiaxpy(ctx, w.V, w.ld, jmax, w.y, 1.0, tv, N, nullptr, &w.ctl->k)) != HDG_OK) return s2;
        if (!fold) {
            if ((s2 = prec_apply(ctx, op, prec, plan, tv, zt, w.work, w.ld, nullptr)) != HDG_OK) return s2;
            return vec_lincomb(ctx, N, x, 1.0, x, 1.0, zt, nullptr);
        }
        // folded: x += M^{-1} q(K M^{-1}) (V y), q = 1 for block-Jacobi, the polynomial otherwise
        const double* u = tv;
        if (prec != HDG_PREC_BJ) {
            if ((s2 = prec_apply(ctx, opi, prec, plan, tv, zt, w.work, w.ld, nullptr)) != HDG_OK) return s2;
            u = zt;
        }
        FaceEpilogue e = epi0();
        e.out[0] = x;
        e.s[0] = 1.0;
        e.X[0] = x;
        e.a[0] = 1.0;
        return op_bj(ctx, op64, u, e, nullptr);
    };
    // One restart cycle, entirely on the stream: FP64 residual, Arnoldi steps
    // (skipped on the device once converged), back substitution, x += Z y.
    auto enqueue_cycle = [&](int jmax) -> hdg_status {
        hdg_status s2;
        FaceEpilogue e = epi0();
        e.out[0] = w.V;
        e.s[0] = -1.0;
        e.X[0] = b;
        e.a[0] = 1.0;
        if ((s2 = face_op(ctx, nf, nb, S, L, K64, false, nbr, nullptr, false, x, e, nullptr)) != HDG_OK) return s2;
        if ((s2 = vec_sumsq_partial(ctx, w.V, N, w.part, w.nblk, nullptr)) != HDG_OK) return s2;
        if ((s2 = krylov_cycle_init(ctx, w.ctl, w.part, w.nblk, w.g, jmax, target)) != HDG_OK) return s2;
        if ((s2 = krylov_scale_by(ctx, w.V, w.V, N, &w.ctl->beta, skip)) != HDG_OK) return s2;
        if (dcgs2) return enqueue_dcgs2_steps(jmax);
        for (int j = 0; j < jmax; ++j) {
            double* vj = w.V + (size_t)j * w.ld;
            double* zj = w.Z + (size_t)j * w.ld;
            double* wv = w.V + (size_t)(j + 1) * w.ld;
            if ((s2 = mark(j, 0)) != HDG_OK) return s2;
            if ((s2 = prec_apply(ctx, op, prec, plan, vj, zj, w.work, w.ld, skip)) != HDG_OK) return s2;
            if ((s2 = mark(j, 1)) != HDG_OK) return s2;
            if ((s2 = timed_matvec(j, op, zj, wv)) != HDG_OK) return s2;
            if ((s2 = mark(j, 4)) != HDG_OK) return s2;
            if (o->orth == HDG_ORTH_CGS2 && j + 1 <= 64) {
                // CGS2 with three reads of the basis: dots, (axpy + second dots), (axpy + norm)
                double* col = w.H + (size_t)j * w.ldh;
                if ((s2 = vec_multidot(ctx, w.V, w.ld, j + 1, wv, N, w.part, w.nblk, skip)) != HDG_OK) return s2;
                if ((s2 = vec_reduce(ctx, w.part, j + 1, w.nblk, col, nullptr, skip)) != HDG_OK) return s2;
                if ((s2 = vec_axpy_dot(ctx, w.V, w.ld, j + 1, col, wv, N, w.part, w.nblk, skip)) != HDG_OK) return s2;
                if ((s2 = vec_reduce(ctx, w.part, j + 1, w.nblk, w.h2, col, skip)) != HDG_OK) return s2;
                if ((s2 = vec_axpy_sumsq(ctx, w.V, w.ld, j + 1, w.h2, wv, N, w.part, w.nblk, skip)) != HDG_OK) return s2;
            } else {
                if ((s2 = orthogonalise(ctx, w, N, j, o->orth, skip)) != HDG_OK) return s2;
                if ((s2 = vec_sumsq_partial(ctx, wv, N, w.part, w.nblk, skip)) != HDG_OK) return s2;
            }
            if ((s2 = krylov_givens(ctx, w.ctl, w.part, w.nblk, w.H, w.ldh, w.cs, w.sn, w.g, j, w.hist)) != HDG_OK)
                return s2;
            if ((s2 = krylov_scale_by(ctx, wv, wv, N, w.H + (size_t)j * w.ldh + j + 1, skip)) != HDG_OK) return s2;
            if ((s2 = mark(j, 5)) != HDG_OK) return s2;
        }
        if ((s2 = krylov_backsolve(ctx, w.ctl, w.H, w.ldh, w.g, w.y)) != HDG_OK) return s2;
        return vec_multiaxpy(ctx, w.Z, w.ld, jmax, w.y, 1.0, x, N, nullptr, &w.ctl->k);
    };
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool mixed_now = mixed, have_prev = false;
    double prev_beta = 0.0, prev_est = 0.0;
    auto drop_graph = [&]() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
    };
    while (true) {
        const int jmax = std::max(0, std::min(m, o->max_iters - iters));
        if (use_graph && jmax == m) {
            if (!gexec) {
                HDG_HIP_CHECK(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
                st = enqueue_cycle(jmax);
                hipGraph_t g = nullptr;
                const hipError_t ec = hipStreamEndCapture(ctx->stream, &g);
                if (st != HDG_OK) { if (g) (void)hipGraphDestroy(g); return st; }
                if (ec != hipSuccess) {
                    ctx->err = std::string("graph capture failed: ") + hipGetErrorString(ec);
                    return HDG_ERR_HIP;
                }
                graph = g;
                if (hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
                    drop_graph();
                    ctx->err = "graph instantiation failed";
                    return HDG_ERR_HIP;
                }
            }
            if (hipGraphLaunch(gexec, ctx->stream) != hipSuccess) {
                drop_graph();
                ctx->err = "graph launch failed";
                return HDG_ERR_HIP;
            }
        } else {
            if ((st = enqueue_cycle(jmax)) != HDG_OK) { drop_graph(); return st; }
        }
        const hipError_t e1 = hipMemcpyAsync(&hc, w.ctl, sizeof(hc), hipMemcpyDeviceToHost, ctx->stream);
        const hipError_t e2 = hipMemcpyAsync(hbuf.data(), w.hist, sizeof(double) * (size_t)std::max(jmax, 1),
                                             hipMemcpyDeviceToHost, ctx->stream);
        const hipError_t e3 = hipStreamSynchronize(ctx->stream);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
            drop_graph();
            ctx->err = "reading the GMRES status failed";
            return HDG_ERR_HIP;
        }
        hist_push(hc.beta);
        for (int i = 0; i < hc.k; ++i) hist_push(hbuf[i]);
        if (timed) {
            // steps at or beyond hc.k returned at once on the device flag: not counted
            const int nsteps = (dcgs2 && hc.k > 0 && hc.k < jmax) ? hc.k + 1 : hc.k;
            for (int j = 0; j < nsteps && j < jmax; ++j) {
                float a = 0.f, b2 = 0.f, c = 0.f;
                const bool pt = !dcgs2 || prec_timed;
                if ((pt && hipEventElapsedTime(&a, ev.e[6 * j], ev.e[6 * j + 1]) != hipSuccess) ||
                    hipEventElapsedTime(&b2, ev.e[6 * j + 2], ev.e[6 * j + 3]) != hipSuccess ||
                    hipEventElapsedTime(&c, ev.e[6 * j + 4], ev.e[6 * j + 5]) != hipSuccess) {
                    drop_graph();
                    ctx->err = "reading the phase timers failed";
                    return HDG_ERR_HIP;
                }
                stats->t_prec += 1e-3 * a;
                stats->t_matvec += 1e-3 * b2;
                stats->t_orth += 1e-3 * c;
                ++stats->n_timed;
            }
        }
        stats->rel_resid_true = bnorm > 0 ? hc.beta / bnorm : 0.0;
        // Iterative refinement on the mixed path: if the last cycle's inner iteration reduced its
        // (FP32-operator) residual estimate well below what the true FP64 residual now shows, and the
        // true residual fell by less than half, the FP32 operator limits the refinement: the
        // remaining cycles apply the FP64 blocks and inverses.
        if (mixed && !mixed_now && hc.k > 0) ++stats->fp64_cycles;
        if (mixed_now && have_prev && hc.beta > 0.5 * prev_beta && hc.beta > 2.0 * prev_est && hc.beta > target) {
            mixed_now = false;
            stats->fallback_flags |= HDG_FALLBACK_MIXED_TO_FP64;
            op = op64;
            opi = op64;
            fold = false;
            prec_timed = true;
            drop_graph();
        }
        if (hc.k > 0) {
            have_prev = true;
            prev_beta = hc.beta;
            prev_est = hc.est;
        }
        if (hc.nonfinite) {
            ctx->err = "residual or Arnoldi data became NaN or Inf";
            result = HDG_ERR_NONFINITE;
            break;
        }
        if (hc.k == 0) {
            result = hc.beta <= target ? HDG_OK : HDG_NOT_CONVERGED;
            break;
        }
        iters += hc.k;
        ++cycles;
        stats->rel_resid_est = bnorm > 0 ? hc.est / bnorm : 0.0;
    }
    drop_graph();
    stats->iters = iters;
    stats->cycles = cycles;
    stats->converged = result == HDG_OK;
    stats->hist_len = std::min(hl, o->resid_hist_len);
    stats->t_total = now_s() - t0;
    return result;
}

// Test hook: z = p(B) M^{-1} y for given Ritz values.
hdg_status poly_apply_run(hdg_ctx ctx, const hdg_dims* d, const double* K64, const float* K32, const int32_t* nbr,
                          const double* B64, const float* B32, int precision, int npoly, const double* tre,
                          const double* tim, const double* y, double* z) {
    const int nb = d->ncomp * d->npf, L = d->nlfe, S = 2 * L - 1, nf = d->nf;
    const size_t N = (size_t)nf * nb;
    hdg_status st;
    SolveWs w;
    if ((st = alloc_solve_ws(ctx, N, 1, 1, 1, &w)) != HDG_OK) return st;
    Op op;
    const bool mixed = precision == HDG_MIXED;
    op.nf = nf; op.nb = nb; op.S = S; op.L = L; op.N = N; op.nbr = nbr;
    op.K = mixed ? (const void*)K32 : (const void*)K64;
    op.k32 = mixed;
    op.Binv = mixed ? (const void*)B32 : (const void*)B64;
    op.b32 = mixed;
    PolyPlan pl;
    pl.kind = HDG_PREC_BJ_POLY;
    pl.tre.assign(tre, tre + npoly);
    pl.tim.assign(tim, tim + npoly);
    pl.P = npoly;
    return poly_apply(ctx, op, pl, y, z, w.work, w.ld, nullptr);
}

// Test hook: z = Chebyshev acceleration of degree P on B = M^{-1} K over [alpha, beta], applied to M^{-1} y.
hdg_status cheb_apply_run(hdg_ctx ctx, const hdg_dims* d, const double* K64, const float* K32, const int32_t* nbr,
                          const double* B64, const float* B32, int precision, int P, double alpha, double beta,
                          const double* y, double* z) {
    const int nb = d->ncomp * d->npf, L = d->nlfe, S = 2 * L - 1, nf = d->nf;
    const size_t N = (size_t)nf * nb;
    hdg_status st;
    SolveWs w;
    if ((st = alloc_solve_ws(ctx, N, 1, 1, 1, &w)) != HDG_OK) return st;
    Op op;
    const bool mixed = precision == HDG_MIXED;
    op.nf = nf; op.nb = nb; op.S = S; op.L = L; op.N = N; op.nbr = nbr;
    op.K = mixed ? (const void*)K32 : (const void*)K64;
    op.k32 = mixed;
    op.Binv = mixed ? (const void*)B32 : (const void*)B64;
    op.b32 = mixed;
    PolyPlan pl;
    pl.kind = HDG_PREC_BJ_CHEB;
    pl.P = P;
    pl.alpha = alpha;
    pl.beta = beta;
    return poly_apply(ctx, op, pl, y, z, w.work, w.ld, nullptr);
}

hdg_status op_apply_run(hdg_ctx ctx, const hdg_dims* d, const void* M1, bool m1_32, const int32_t* nbr, int S1,
                        const double* x, double* y) {
    FaceEpilogue e = epi0();
    e.out[0] = y;
    e.s[0] = 1.0;
    return face_op(ctx, d->nf, d->ncomp * d->npf, S1, d->nlfe, M1, m1_32, nbr, nullptr, false, x, e, nullptr);
}

// Test hook: z = sum_e R_e^T (P^e)^{-1} R_e y.
hdg_status asm_apply_run(hdg_ctx ctx, const hdg_dims* d, const void* inv, bool inv32, const int32_t* f2e,
                         const int32_t* e2f, const double* y, double* z) {
    const int nb = d->ncomp * d->npf, L = d->nlfe, nf = d->nf;
    const int64_t ne = d->ne;
    const size_t nunit = (size_t)ne * L;
    hdg_status st;
    char* base = (char*)ws_get(ctx, WS_ASM, sizeof(int32_t) * nunit * L + sizeof(double) * nunit * nb + 256, &st);
    if (!base) return st;
    double* zu = (double*)base;
    int32_t* unbr = (int32_t*)(zu + nunit * nb);
    if ((st = asm_unit_nbr(ctx, ne, L, e2f, unbr)) != HDG_OK) return st;
    FaceEpilogue e = epi0();
    e.out[0] = z;
    e.s[0] = 1.0;
    return asm_apply_op(ctx, nf, nb, L, ne, inv, inv32, unbr, f2e, zu, y, e, nullptr);
}
