// Internal declarations shared by the HIP translation units of libhdg.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "hdg.h"

typedef double double4_t __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Context: stream, error text and a cache of device workspace buffers.
enum WsSlot {
    WS_T_BOTTOM = 0,   // condensation: bottom (trace) rows of the elimination matrix
    WS_W,              // condensation: M^{-1}[B_d | C_d]
    WS_STATUS,         // small int status words (singular element/face ...)
    WS_BINV64,
    WS_BINV32,
    WS_KRYLOV_V,       // Arnoldi basis (m+1) x N
    WS_KRYLOV_Z,       // preconditioned vectors m x N
    WS_VEC,            // work vectors for the preconditioners
    WS_PART,           // reduction partials
    WS_CTL,            // GMRES device control block + Hessenberg/Givens state
    WS_KFOLD,          // right-preconditioned operator blocks K M^{-1}
    WS_ASM,            // additive Schwarz: unit neighbour table, unit results, a work vector
    WS_NEWTON,         // residual norm: assembled trace residual and reduction partials
    WS_NEWTON_BATCH,   // batched element generation / norms / updates: descriptors, norms, steps
    WS_ELEM_SYS,       // element generation of M-component models: per-point flux data of a chunk
    WS_LU,             // condensation: inverted diagonal blocks of L and U, row permutations
    WS_NSLOTS
};

// What the block-Jacobi workspace (WS_BINV64/32 and, with fold, WS_KFOLD) holds after a
// solve, so that a later solve on the same matrix may reuse it.
struct BjSetupKey {
    bool valid = false, fold = false, mixed = false;
    const void *K64 = nullptr, *K32 = nullptr, *nbr = nullptr;
    int nf = 0, nb = 0, S = 0;
};

struct hdg_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream for graph capture (created on first use)
    std::string err;
    void* ws[WS_NSLOTS] = {};
    size_t ws_bytes[WS_NSLOTS] = {};
    BjSetupKey bj_key;
    // phase timing: the next instrumented kernel launch (face operator, delayed-CGS2 sweeps)
    // records ext_start at its start and ext_stop at its end (hipExtLaunchKernelGGL) if they
    // are set, and clears them
    hipEvent_t ext_start = nullptr, ext_stop = nullptr;
};

inline void take_ext_events(hdg_ctx ctx, hipEvent_t* start, hipEvent_t* stop) {
    *start = ctx->ext_start;
    *stop = ctx->ext_stop;
    ctx->ext_start = ctx->ext_stop = nullptr;
}

// Runs the enclosing scope on the context's private capture stream: the caller's
// stream (possibly the legacy null stream, which cannot be captured) is drained
// first and the private stream is drained before the caller's is restored.
struct CaptureStreamScope {
    hdg_ctx ctx;
    hipStream_t saved = nullptr;
    bool active = false;
    hipError_t begin(hdg_ctx c) {
        ctx = c;
        if (!c->cap_stream) {
            hipError_t e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return e;
        }
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return e;
        saved = c->stream;
        c->stream = c->cap_stream;
        active = true;
        return hipSuccess;
    }
    ~CaptureStreamScope() {
        if (active) {
            (void)hipStreamSynchronize(ctx->stream);
            ctx->stream = saved;
        }
    }
};

// Returns a device buffer of at least `bytes` for `slot` (grows, never shrinks).
void* ws_get(hdg_ctx ctx, WsSlot slot, size_t bytes, hdg_status* st);

// Measured launch configurations (tune.cpp): key -> (a, b); HDG_TUNE_CACHE names a JSON file
// the table is read from on first use and written back by tune_save.
bool tune_get(const std::string& key, int* a, int* b);
void tune_put(const std::string& key, int a, int b, double us);
bool tune_have_entries();
std::string tune_json();
bool tune_save();
hdg_status face_autotune(hdg_ctx ctx, int nf, int nb, int S1, int nlfe, const void* M1, bool m1_fp32,
                         const int32_t* nbr1, const void* M2, bool m2_fp32, const double* x, double* y, int reps,
                         double* best_us);

// Fixed per-device scratch of the allocation-free entry point (k_noalloc.hip): 16 MiB.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = size_t(1) << 21;
hdg_status noalloc_scratch_init(int device);   // with `device` current; once per device
double* noalloc_scratch(int device);           // nullptr before noalloc_scratch_init

#define HDG_HIP_CHECK(ctx, call)                                                   \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            (ctx)->err = std::string("HIP error: ") + hipGetErrorString(e_) +      \
                         " at " + __FILE__ + ":" + std::to_string(__LINE__);       \
            return HDG_ERR_HIP;                                                    \
        }                                                                          \
    } while (0)

#define HDG_LAUNCH_CHECK(ctx) HDG_HIP_CHECK(ctx, hipGetLastError())

static inline int div_up(long long a, long long b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Face-block operator (block matvec / block-Jacobi / fused polynomial step).
//
// For face f with neighbour slots s < S1 (nbr1 == nullptr: S1 = 1 and slot 0 = f):
//   u_f = sum_s M1[f][s] x_{nbr1[f][s]}            (column-major nb x nb blocks)
//   if M2: u_f <- M2[f] u_f                          (block-Jacobi after the product)
// then for o = 0..2 with out[o] != nullptr:
//   out[o]_f = s[o] u_f + a[o] X[o]_f + b[o] Y[o]_f  (X/Y may be nullptr = 0)
// All outputs are computed from the inputs before any is written, so an output
// may alias a face-local input (X or Y) but never the gathered vector x.
struct FaceEpilogue {
    double* out[3];
    const double* X[3];
    const double* Y[3];
    double s[3], a[3], b[3];
};

hdg_status face_op(hdg_ctx ctx, int nf, int nb, int S1, int nlfe, const void* M1, bool m1_fp32,
                   const int32_t* nbr1, const void* M2, bool m2_fp32, const double* x,
                   const FaceEpilogue& epi, const int* skip_flag);

// ---------------------------------------------------------------------------
// Vector kernels (Krylov). Reductions give each block a chunk of krylov_chunk(n) entries:
// 2048, halved (down to 256) while that leaves fewer than 512 blocks, so that short vectors
// still spread over the chip; nblk must be krylov_nblk(n). `skip` (device flag, may be null):
// the kernel returns at once when *skip != 0; `J_dev` (may be null) overrides J with a
// device value.
__host__ __device__ static inline int krylov_chunk(size_t n) {
    int c = 2048;
    while (c > 256 && (n + c - 1) / c < 512) c >>= 1;
    return c;
}
static inline int krylov_nblk(size_t n) {
    const size_t c = (size_t)krylov_chunk(n);
    return (int)((n + c - 1) / c > 0 ? (n + c - 1) / c : 1);
}
hdg_status vec_multidot(hdg_ctx ctx, const double* V, size_t ldv, int J, const double* w, size_t n,
                        double* part, int nblk, const int* skip);
hdg_status vec_reduce(hdg_ctx ctx, const double* part, int J, int nblk, double* out, double* add_to,
                      const int* skip);
hdg_status vec_multiaxpy(hdg_ctx ctx, const double* V, size_t ldv, int J, const double* h, double sign,
                         double* w, size_t n, const int* skip, const int* J_dev = nullptr);
hdg_status vec_sumsq_partial(hdg_ctx ctx, const double* w, size_t n, double* part, int nblk, const int* skip);
// Fused CGS2 second pass (J <= 64): w -= V h1 with partial dots V^T w; w -= V h2 with partial ||w||^2.
hdg_status vec_multidot2(hdg_ctx ctx, const double* V, size_t ldv, int J, const double* x1, const double* x2,
                         size_t n, double* part, int nblk, const int* skip);
hdg_status vec_dcgs2_update(hdg_ctx ctx, const double* V, size_t ldv, int j, double* vj, double* wt,
                            const double* coef, int ldc, size_t n, const int* skip);
hdg_status vec_axpy_dot(hdg_ctx ctx, const double* V, size_t ldv, int J, const double* h1, double* w, size_t n,
                        double* part, int nblk, const int* skip);
hdg_status vec_axpy_sumsq(hdg_ctx ctx, const double* V, size_t ldv, int J, const double* h2, double* w, size_t n,
                          double* part, int nblk, const int* skip);
hdg_status vec_lincomb(hdg_ctx ctx, size_t n, double* out, double a, const double* X, double b,
                       const double* Y, const int* skip);

// GMRES device control block.
struct GmresCtl {
    int done;           // 1: stop the cycle (converged, breakdown or step budget)
    int k;              // Arnoldi steps completed in this cycle
    int jmax;           // step budget for this cycle
    int nonfinite;
    double target;      // absolute residual target
    double beta;        // cycle-start residual norm
    double est;         // latest Givens residual estimate
    double pad;
};
hdg_status krylov_cycle_init(hdg_ctx ctx, GmresCtl* ctl, const double* part, int nblk, double* g,
                             int jmax, double target);
hdg_status krylov_scale_by(hdg_ctx ctx, double* v, const double* src, size_t n, const double* denom,
                           const int* skip);
hdg_status krylov_givens(hdg_ctx ctx, GmresCtl* ctl, const double* part, int nblk, double* H, int ldh,
                         double* cs, double* sn, double* g, int j, double* hist);
hdg_status krylov_backsolve(hdg_ctx ctx, const GmresCtl* ctl, const double* H, int ldh, const double* g,
                            double* y);
hdg_status krylov_dcgs2_coef(hdg_ctx ctx, GmresCtl* ctl, const double* part, int nblk, int j, int finish, double* Hu,
                             double* H, int ldh, double* cs, double* sn, double* g, double* coef, int ldc,
                             double* hist);
hdg_status krylov_store_norm(hdg_ctx ctx, const double* part, int nblk, double* dst);

// ---------------------------------------------------------------------------
// Block-Jacobi batched inverse (Gauss-Jordan with partial pivoting).
// Additive Schwarz (Section 4.6): subdomain inverses inv[e][l][l'][col][row] (FP64 and/or
// FP32), the unit neighbour table, and z = sum_e R_e^T (P^e)^{-1} R_e y with the epilogue
// applied per face entry (zu: ne*L*nb scratch).
hdg_status asm_setup_run(hdg_ctx ctx, const hdg_dims* d, const double* Kbar, const double* K64, const int32_t* e2f,
                         double* inv64, float* inv32);
hdg_status asm_unit_nbr(hdg_ctx ctx, int64_t ne, int L, const int32_t* e2f, int32_t* unbr);
hdg_status asm_apply_run(hdg_ctx ctx, const hdg_dims* d, const void* inv, bool inv32, const int32_t* f2e,
                         const int32_t* e2f, const double* y, double* z);
hdg_status asm_apply_op(hdg_ctx ctx, int nf, int nb, int L, int64_t ne, const void* inv, bool inv32,
                        const int32_t* unbr, const int32_t* f2e, double* zu, const double* y, const FaceEpilogue& epi,
                        const int* skip);
// Kf[f][s] = K[f][s] Binv[nbr(f,s)] (the right-preconditioned block row), FP64 products.
hdg_status fold_bj(hdg_ctx ctx, int nf, int nb, int S, const double* K64, const int32_t* nbr, const double* B64,
                   void* out, bool out_fp32);
hdg_status bj_invert(hdg_ctx ctx, int nf, int nb, int S, const double* K64, double* B64, float* B32,
                     int* bad_face);

// Condensation, assembly, recovery launchers.
hdg_status condense_run(hdg_ctx ctx, const hdg_dims* d, int64_t ne, const hdg_elem_blocks* in,
                        double* Kbar, double* rbar, double* local, double* Hbar = nullptr, int32_t* ipiv = nullptr);
hdg_status condense_rhs_run(hdg_ctx ctx, const hdg_dims* d, int64_t ne, double* local, const double* Hbar,
                            const int32_t* ipiv, const double* ru, const double* rt, double* rbar);
hdg_status assemble_rhs_run(hdg_ctx ctx, const hdg_dims* d, const int32_t* f2e, const int32_t* perm,
                            const double* rbar, double* r);
hdg_status assemble_run(hdg_ctx ctx, const hdg_dims* d, const int32_t* f2e, const int32_t* e2f,
                        const int32_t* perm, const double* Kbar, const double* rbar, double* K64,
                        float* K32, int32_t* nbr, double* r);
hdg_status recover_run(hdg_ctx ctx, const hdg_dims* d, const double* local, const double* Minv,
                       const double* Bd, const double* Cd, const int32_t* e2f, const int32_t* perm,
                       const double* xhat, double* du, double* dq);
hdg_status axpy_run(hdg_ctx ctx, int64_t n, double alpha, const double* x, double* y);

// ILU-ASM (k_ilu.hip): out = epilogue(sum_l R_l^T (L_l U_l)^{-1} R_l y).
hdg_status ilu_apply_op(hdg_ctx ctx, const hdg_ilu_asm_s* h, const double* y, const FaceEpilogue& e,
                        const int* skip);
double* ilu_tmp(const hdg_ilu_asm_s* h);
bool ilu_matches(const hdg_ilu_asm_s* h, const hdg_dims* d);

// Element residuals / Jacobian blocks (k_element.hip). `bad` receives the first element
// whose mass matrix has a non-positive pivot (atomicMin; initialise it to INT_MAX).
size_t element_blocks_lds_bytes(const hdg_dims* d, int nqv, int nqf);
hdg_status element_blocks_run(hdg_ctx ctx, const hdg_dims* d, const hdg_elem_geom* g, const hdg_conv_diff* m,
                              const hdg_time_term* tt, const int32_t* e2f, const double* u, const double* uhat,
                              int flags, const hdg_elem_arrays* out, int* bad);

// Host-side eigenvalues / harmonic Ritz values (ritz.cpp).
int hessenberg_eigvals(int n, double* H, int ld, double* wr, double* wi);
int harmonic_ritz_leja(int P, const double* H, double drop_rel, double* tre, double* tim, int* nout);
int poly_roots(int P, const double* H, double drop_rel, double* tre, double* tim, int* nout, int* nadded);

// Element residuals / Jacobian blocks of M-component models (k_element_sys.hip).
size_t element_sys_lds_bytes(const hdg_dims* d, int nqv, int nqf);
size_t element_sys_ws_doubles(const hdg_dims* d, int nqv, int nqf);
hdg_status element_sys_run(hdg_ctx ctx, const hdg_dims* d, const hdg_elem_geom* g, const hdg_sys_model* m,
                           const hdg_time_term* tt, const int32_t* e2f, const double* u, const double* uhat,
                           int32_t flags, const hdg_elem_arrays* out, int* bad, double* ws, int64_t e0, int64_t n);
