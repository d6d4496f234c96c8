/*
 * hdg.h -- C ABI of the MI355X (gfx950) HDG hot-path library (libhdg.so).
 *
 * The library implements the data-parallel hot path of an HDG solver:
 *   (1) static condensation of element unknowns into element trace Schur
 *       complements                          Section 2.3 (eq. 13-b, 13-c), Section 4.1-4.2 (eq. w15-w22)
 *   (2) face-based assembly of the trace system in dense face blocks
 *                                              Section 2.4, Section 4.2
 *   (3) preconditioned restarted (F)GMRES on the face-block matrix with
 *       block-Jacobi and polynomial (harmonic-Ritz/Leja or Chebyshev)
 *       preconditioners                      Sections 3.1-3.4, 4.3-4.7
 *   (4) local recovery of (du, dq)           Section 2.3 (recovery equation), eq. w19, eq. w16
 *   (5) the Newton update                    Section 2.3 (Newton iterate), Section 4.4
 *
 * Conventions (all entry points):
 *   - Array arguments are DEVICE pointers (gfx950 global memory) owned by the
 *     caller, unless the name ends in _h (host memory). The library never frees
 *     caller memory. It owns only the opaque context and its internal workspace.
 *   - Arrays are C row-major (last index fastest) unless stated otherwise.
 *   - Work is enqueued on the context's stream; entry points that must read a
 *     device status (singular pivots, convergence) synchronise that stream.
 *   - Errors: argument and shape errors are detected on the host before any
 *     launch and leave every output untouched. A negative status is an error,
 *     a positive status is a warning with valid outputs. hdg_last_error()
 *     returns a message naming the offending element/face when there is one.
 *     No C++ exception crosses this interface.
 *   - A context is used by one host thread at a time.
 *
 * Dimensions (the paper's symbols): M components, D space dimensions, P_E
 * element basis functions, P_F face basis functions, N_lfe faces per element.
 *   nq = M*D*P_E, nu = M*P_E, nt = M*P_F*N_lfe, nb = M*P_F, S = 2*N_lfe - 1,
 *   N_dof = nb * N_F.
 * Dof orders: u (m, i) -> m*P_E + i; q (m, d, i) -> (m*D + d)*P_E + i;
 *   element trace (l, m, j) -> (l*M + m)*P_F + j; face vector (m, j) -> m*P_F + j.
 */
#ifndef HDG_H
#define HDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hdg_ctx_s* hdg_ctx;

typedef enum {
    HDG_OK = 0,
    HDG_NOT_CONVERGED = 1,      /* warning: solve stopped at max_iters; x holds the last iterate */
    HDG_ERR_ARG = -1,           /* null pointer / bad option value */
    HDG_ERR_SHAPE = -2,         /* inconsistent dimensions or unsupported size */
    HDG_ERR_SINGULAR = -3,      /* zero or non-finite pivot (element or face named in hdg_last_error) */
    HDG_ERR_NONFINITE = -4,     /* NaN/Inf in a residual or right-hand side */
    HDG_ERR_HIP = -5,           /* HIP runtime error */
    HDG_ERR_NOMEM = -6          /* device workspace allocation failed */
} hdg_status;

/* Mesh/space sizes: N_E, N_F, M, D, P_E, P_F, N_lfe (Section 2.4, Section 4.1). */
typedef struct {
    int32_t ne, nf, ncomp, dim, npe, npf, nlfe;
} hdg_dims;

/* Context. `device` is the HIP device ordinal; `hip_stream` a hipStream_t or NULL
 * for the null stream. The context allocates its workspace lazily on that device. */
hdg_status  hdg_create(hdg_ctx* out, int device, void* hip_stream);
hdg_status  hdg_destroy(hdg_ctx ctx);
hdg_status  hdg_set_stream(hdg_ctx ctx, void* hip_stream);
const char* hdg_last_error(hdg_ctx ctx);
/* Releases the context's cached device workspace (it is re-allocated on demand). */
hdg_status  hdg_release_workspace(hdg_ctx ctx);

/* ---------------------------------------------------------------------------
 * (1) Static condensation -- Section 2.3 eq. 13-b/13-c, Section 4.1 eq. w15-w19,
 *     Section 4.2 eq. w21-w22.
 *
 * Per element e (the caller may pass a chunk of elements by offsetting every
 * pointer and setting ne_chunk):
 *   Minv [ne][P_E][P_E]        inverse element mass matrix (M^e)^{-1}
 *   Bd   [ne][D][P_E][P_E]     B_d[i][j] = int dphi_i/dx_d phi_j  (derivative on the test
 *                              function: the q-equation reads M q_dm + B_d u_m + C_d uhat_m = 0)
 *   Cd   [ne][D][P_E][N_lfe*P_F]  C_d[i][(l,j)] = -int_{face l} phi_i psi_j n_d
 *   D [ne][nu][nq], E [ne][nu][nu], F [ne][nu][nt]     u-equation blocks
 *   G [ne][nt][nq], H [ne][nt][nu], J [ne][nt][nt]     trace-equation blocks
 *   ru [ne][nu], rt [ne][nt]                           right-hand sides (r_q = 0)
 * The q block is A = I_{MD} (x) M^e and B, C are component-diagonal (eq. w16).
 *
 * Computes  Ebar = E - D A^{-1} B,  Fbar = F - D A^{-1} C,  Hbar = H - G A^{-1} B,
 *           Jbar = J - G A^{-1} C,  Kbar = Jbar - Hbar Ebar^{-1} Fbar,
 *           rbar = rt - Hbar Ebar^{-1} ru.
 * Outputs:
 *   Kbar  [ne][nt][nt]   element trace Schur complement (row = trace test dof)
 *   rbar  [ne][nt]
 *   local [ne][nu][nu+nt+1]   the local solver for recovery (eq. w19): rows hold
 *         [L\U | Ebar^{-1} Fbar | Ebar^{-1} ru] with P Ebar = L U (partial pivoting,
 *         the unit lower L below the diagonal with every interchange applied to it).
 * Errors: HDG_ERR_SINGULAR if some Ebar has a zero/non-finite pivot (first
 * such element named). Synchronises the stream to read that status. */
typedef struct {
    const double *Minv, *Bd, *Cd, *D, *E, *F, *G, *H, *J, *ru, *rt;
} hdg_elem_blocks;

size_t     hdg_local_size(const hdg_dims* dims);   /* doubles per element of `local` */
hdg_status hdg_condense(hdg_ctx ctx, const hdg_dims* dims, int64_t ne_chunk,
                        const hdg_elem_blocks* in, double* Kbar, double* rbar, double* local);

/* (1b) Stage reuse -- Section 2.2 (the stages of a DIRK scheme solve systems with the
 *     same matrix and new right-hand sides, so matrices and preconditioners carry over)
 *     with the condensed right-hand side of Section 4.1 eq. w19 / Section 4.2 eq. w22.
 *
 * hdg_condense_keep: hdg_condense that also keeps what a later right-hand side needs:
 *   Hbar [ne][nt][nu]  Hbar = H - G A^{-1} B, the trace rows' coupling to the element
 *                      unknowns after the q-elimination;
 *   ipiv [ne][nu]      row interchanges of the elimination: at step k the rows at
 *                      (element-local) positions k and ipiv[k] >= k were exchanged;
 *   local holds the unit lower L below the diagonal of its first nu columns, with every
 *         interchange applied to every column of L (P Ebar = L U as LAPACK's getrf leaves
 *         it; hdg_condense leaves the same there).
 *   All outputs are caller-owned device buffers; the same errors as hdg_condense.
 * hdg_condense_rhs: for new right-hand sides ru [ne][nu], rt [ne][nt] of the same element
 *   matrices: x_r = Ebar^{-1} ru = U^{-1} L^{-1} P ru (P: the interchanges of ipiv in
 *   order) replaces the last column of `local`, and rbar = rt - Hbar x_r. `local`, Hbar
 *   and ipiv must come from hdg_condense_keep on the same dims. Enqueued only, no
 *   synchronisation; no pivots are re-checked. */
hdg_status hdg_condense_keep(hdg_ctx ctx, const hdg_dims* dims, int64_t ne_chunk,
                             const hdg_elem_blocks* in, double* Kbar, double* rbar, double* local,
                             double* Hbar, int32_t* ipiv);
hdg_status hdg_condense_rhs(hdg_ctx ctx, const hdg_dims* dims, int64_t ne_chunk, double* local,
                            const double* Hbar, const int32_t* ipiv, const double* ru, const double* rt,
                            double* rbar);

/* ---------------------------------------------------------------------------
 * (2) Face-block assembly -- Section 2.4, Section 4.2.
 *
 *   f2e  [nf][4]  (e1, l1, e2, l2); e2 = l2 = -1 on boundary faces. e1 < e2.
 *   e2f  [ne][N_lfe]  global face of local face l of element e.
 *   perm [ne][N_lfe][P_F] or NULL: element-local face dof holding canonical face
 *        dof j (NULL = identity: element traces already in face order).
 *   Kbar, rbar as produced by hdg_condense.
 * Outputs (face f, slot s):
 *   K64 [nf][S][nb][nb]  block coupling face f to face nbr[f][s], stored
 *        COLUMN-major: K64[f][s][col][row] (the paper's order M x P_F x M x P_F x S x N_F,
 *        first index fastest). Slot 0 = f itself (sum of both elements' diagonal
 *        blocks); slots 1..N_lfe-1 = the other faces of e1 in local order; slots
 *        N_lfe..2N_lfe-2 = the other faces of e2 (empty on boundary faces).
 *   K32 [nf][S][nb][nb]  optional (NULL to skip) FP32 rounding of K64.
 *   nbr [nf][S]  neighbour face per slot, -1 = empty slot (never read).
 *   r   [nf][nb] assembled right-hand side. */
hdg_status hdg_assemble_blocks(hdg_ctx ctx, const hdg_dims* dims,
                               const int32_t* f2e, const int32_t* e2f, const int32_t* perm,
                               const double* Kbar, const double* rbar,
                               double* K64, float* K32, int32_t* nbr, double* r);
/* hdg_assemble_rhs: r alone (the same sums as hdg_assemble_blocks) for a new rbar, e.g. a
 * later DIRK stage whose matrix is unchanged (Section 2.2). One wave per face, no atomics. */
hdg_status hdg_assemble_rhs(hdg_ctx ctx, const hdg_dims* dims, const int32_t* f2e, const int32_t* perm,
                            const double* rbar, double* r);

/* ---------------------------------------------------------------------------
 * (3) Preconditioned restarted FGMRES on K x = r -- Sections 3.1-3.4, 4.3-4.7.
 *
 * Right-preconditioned flexible GMRES(restart): every cycle starts from the true
 * FP64 residual r - K64 x; it stops when ||r - K64 x||_2 <= max(rtol*||r||_2, atol)
 * or after max_iters Arnoldi steps. The Hessenberg/Givens update runs on the
 * device in FP64; a whole cycle is enqueued at once (or replayed as one captured
 * hipGraph when use_graph = 1) and the host reads one status word per cycle.
 * With use_graph = 1 the solve drains the context's stream, runs on a private
 * stream of the context (so the caller's stream may be the legacy null stream)
 * and drains that stream before returning.
 *
 * precision = HDG_FP64: every operator application uses K64 and FP64 inverses.
 * precision = HDG_MIXED: inside a cycle the matvec and the preconditioner use K32
 *   and FP32 block inverses (FP64 vectors and accumulation); the cycle-start
 *   residual uses K64, so each restart is one step of iterative refinement.
 *   K32 must then be non-NULL.
 * prec: HDG_PREC_NONE, HDG_PREC_BJ (Section 4.5), HDG_PREC_BJ_POLY (BJ-PP(P):
 *   z = p(B) M^{-1} y, B = M^{-1} K, harmonic Ritz values from one MGS Arnoldi
 *   cycle of length poly_degree on B started at poly_v0, Leja order, Section 4.7),
 *   HDG_PREC_BJ_CHEB (Chebyshev acceleration of degree poly_degree on B over a real
 *   interval estimated from the same Ritz values); HDG_PREC_ASM, HDG_PREC_ASM_POLY and
 *   HDG_PREC_ASM_CHEB are the same with M^{-1} the element-patch additive Schwarz
 *   operator (Sections 3.3, 4.6), whose inverses hdg_asm_setup forms (asm_* options).
 * orth: Arnoldi orthogonalisation (Section 4.4). HDG_ORTH_CGS2 (default), HDG_ORTH_CGS
 *   and HDG_ORTH_MGS run the flexible form above (x += Z y, z_j = M^{-1} v_j kept).
 *   HDG_ORTH_DCGS2 runs right-preconditioned GMRES with the preconditioner fixed
 *   (x += M^{-1} V y, no Z) and delayed classical Gram-Schmidt with
 *   reorthogonalisation: two sweeps over the basis per step instead of three, the
 *   same iterates as CGS2 in exact arithmetic; each column of the Hessenberg matrix
 *   (and the residual estimate) is completed one step late, so a converged cycle
 *   spends one operator application that it does not use.
 * poly_v0: device vector [N_dof], the random Arnoldi start (required for the
 *   polynomial preconditioners; the caller draws it so both sides of a parity
 *   test use the same vector).
 * x: on entry the initial guess, on exit the solution.
 * Returns HDG_NOT_CONVERGED (positive) when max_iters is reached. */
enum { HDG_PREC_NONE = 0, HDG_PREC_BJ = 1, HDG_PREC_BJ_POLY = 2, HDG_PREC_BJ_CHEB = 3,
       HDG_PREC_ASM = 4, HDG_PREC_ASM_POLY = 5, HDG_PREC_ASM_CHEB = 6, HDG_PREC_ILU_ASM = 7 };
typedef struct hdg_ilu_asm_s* hdg_ilu_asm;   /* see (6b) */
enum { HDG_ORTH_CGS2 = 0, HDG_ORTH_CGS = 1, HDG_ORTH_MGS = 2, HDG_ORTH_DCGS2 = 3 };
enum { HDG_FP64 = 0, HDG_MIXED = 1 };

typedef struct {
    int32_t restart;            /* Krylov dimension m (1..200), default 50 */
    int32_t max_iters;          /* Arnoldi steps over all cycles, default 1000 */
    double  rtol, atol;
    int32_t prec;               /* HDG_PREC_* */
    int32_t poly_degree;        /* P (1..64) for BJ_POLY / BJ_CHEB */
    const double* poly_v0;      /* device [N_dof]; required for BJ_POLY / BJ_CHEB */
    int32_t orth;               /* HDG_ORTH_* */
    int32_t precision;          /* HDG_FP64 or HDG_MIXED */
    double* resid_hist_h;       /* host, optional: ||r|| at each cycle start and Givens estimates */
    int32_t resid_hist_len;
    int32_t use_graph;          /* 1: capture one restart cycle in a hipGraph and replay it */
    int32_t time_phases;        /* 1: HIP events around the preconditioner, matvec and
                                   orthogonalisation of every Arnoldi step (fills t_prec,
                                   t_matvec, t_orth, n_timed; the cycle is then enqueued
                                   directly even when use_graph = 1). Where a phase starts or
                                   ends with a face-operator or delayed-CGS2 sweep kernel, the
                                   launch itself records the event at the kernel's start or end
                                   (hipExtLaunchKernelGGL); elsewhere a plain event record. */
    int32_t fold_prec;          /* 1 (with HDG_ORTH_DCGS2 and a preconditioner): form the
                                   right-preconditioned blocks K[f][s] P_g^{-1} (g = nbr(f,s))
                                   once per solve in a workspace, FP32 on the mixed path, so a
                                   step applies one block row product instead of block-Jacobi +
                                   product (polynomial preconditioners become polynomials in
                                   K M^{-1}); x += M^{-1}(...) once per cycle. Same iterates in
                                   exact arithmetic; ignored otherwise. */
    const double* asm_inv64;    /* device, additive Schwarz inverses from hdg_asm_setup: FP64 */
    const float* asm_inv32;     /*   and FP32 (needed with HDG_MIXED) */
    const int32_t* asm_f2e;     /* device f2e and e2f as for hdg_assemble_blocks */
    const int32_t* asm_e2f;
    int32_t reuse_setup;        /* 1 (block-Jacobi family only): keep the block inverses, and the
                                   folded blocks if the earlier solve formed them, from the last
                                   solve on this context with the same K64, nbr, dims and precision
                                   (the matrix must not have changed since: Section 2.2's reuse
                                   across DIRK stages); HDG_ERR_ARG if the context holds none.
                                   Ignored for HDG_PREC_NONE and the additive Schwarz family. */
    hdg_ilu_asm ilu_asm;        /* HDG_PREC_ILU_ASM: factors from hdg_ilu_asm_create on this K64 */
} hdg_solve_opts;

typedef struct {
    int32_t iters, cycles, converged, npoly;
    double  rel_resid_true;     /* ||r - K64 x|| / ||r||, FP64 */
    double  rel_resid_est;      /* last Givens estimate / ||r|| */
    double  t_setup, t_total;   /* seconds (host clock around the stream work) */
    double  theta_re[64], theta_im[64];   /* Leja-ordered Ritz values (polynomial preconditioners) */
    int32_t hist_len;           /* entries written to resid_hist_h */
    int32_t n_timed;            /* Arnoldi steps timed (time_phases = 1), else 0 */
    double  t_prec, t_matvec, t_orth;     /* seconds of device time over the timed steps:
                                   preconditioner (0 with block-Jacobi folded into the blocks:
                                   no separate apply), the step's one matvec (events recorded at
                                   the block-matvec kernel's own start and end), and
                                   orthogonalisation + Givens + normalisation */
    double  cheb_alpha, cheb_beta;        /* Chebyshev interval [alpha, beta] of HDG_PREC_*_CHEB */
    int32_t fallback_flags;     /* HDG_FALLBACK_* bits: what the solve changed on its own */
    int32_t fp64_cycles;        /* mixed path: restart cycles run with the FP64 operator after
                                   HDG_FALLBACK_MIXED_TO_FP64 */
} hdg_solve_stats;

/* Safeguards of hdg_gmres_solve (none is in the paper, which states no safeguard for its
 * polynomial preconditioner or for precision):
 *   HDG_FALLBACK_PP_BREAKDOWN    the Arnoldi(P) cycle of the polynomial setup broke down
 *                                (h_{j+1,j} = 0) before step P;
 *   HDG_FALLBACK_PP_SMALL_RITZ   harmonic Ritz values below 1e-12 max|theta| were dropped;
 *   HDG_FALLBACK_PP_NO_INTERVAL  the Ritz values give no positive Chebyshev interval;
 *   HDG_FALLBACK_PP_TO_BASE      one of the three above: the solve ran with the base
 *                                preconditioner alone (block-Jacobi or additive Schwarz);
 *   HDG_FALLBACK_MIXED_TO_FP64   a mixed-precision restart cycle's true FP64 residual fell by
 *                                less than half and stayed above twice what that cycle's inner
 *                                (FP32-operator) iteration estimated: the FP32 matrix limits the
 *                                refinement, and the remaining cycles use K64 and FP64 inverses;
 *   HDG_FALLBACK_PP_ADDED_ROOT   the residual polynomial prod_j (1 - z/theta_j) of the harmonic
 *                                Ritz values exceeds 1 in modulus at 1.1 times the root of largest
 *                                real part (where the spectrum of M^{-1}K may still reach, and
 *                                z p(z) would turn negative): one or two more copies of that root
 *                                (and of its conjugate) were added, raising the degree by up to 4
 *                                (hdg_poly_roots computes the roots);
 *   HDG_FALLBACK_STAGNATED       (hdg_gmres_solve_batch, per instance) five restart cycles in a
 *                                row met the target in their inner estimate while the true
 *                                residual at the next restart stayed above the target and above
 *                                0.9 times the best true residual so far: the FP64 residual
 *                                cannot show more accuracy, and the instance stops early, not
 *                                converged. */
enum { HDG_FALLBACK_PP_BREAKDOWN = 1, HDG_FALLBACK_PP_SMALL_RITZ = 2, HDG_FALLBACK_PP_NO_INTERVAL = 4,
       HDG_FALLBACK_PP_TO_BASE = 8, HDG_FALLBACK_MIXED_TO_FP64 = 16, HDG_FALLBACK_STAGNATED = 32,
       HDG_FALLBACK_PP_ADDED_ROOT = 64 };

void       hdg_solve_opts_default(hdg_solve_opts* opts_h);
hdg_status hdg_gmres_solve(hdg_ctx ctx, const hdg_dims* dims,
                           const double* K64, const float* K32, const int32_t* nbr,
                           const double* r, double* x,
                           const hdg_solve_opts* opts_h, hdg_solve_stats* stats_h);

/* ---------------------------------------------------------------------------
 * (4) Local recovery -- Section 2.3 (recovery equation), eq. w19, eq. w16.
 *   du^e = Ebar^{-1}(r_u - Fbar uhat^e),  dq_{m,d} = -Minv (B_d du_m + C_d uhat_m)
 * from `local` (hdg_condense), Minv/Bd/Cd (as for hdg_condense), e2f/perm (as for
 * hdg_assemble_blocks) and the face solution xhat [nf][nb].
 * Outputs du [ne][nu], dq [ne][nq]. */
hdg_status hdg_recover_local(hdg_ctx ctx, const hdg_dims* dims, const double* local,
                             const double* Minv, const double* Bd, const double* Cd,
                             const int32_t* e2f, const int32_t* perm, const double* xhat,
                             double* du, double* dq);

/* (5) Newton update state += alpha * delta over n entries -- Section 2.3, Section 4.4. */
hdg_status hdg_newton_update(hdg_ctx ctx, int64_t n, double alpha, const double* delta, double* state);

/* (5b) Element residuals and Jacobian blocks on the device -- Section 4.1 (the element
 *     matrices as products of reference basis tables with per-point weights, Jacobian
 *     determinants and flux derivatives), Section 2.2 (weak form, numerical flux), and the
 *     residual evaluation of Section 4.4's damped Newton iteration.
 *
 * Scalar convection-diffusion models (ncomp = 1):
 *   F(u, q) = beta u^2/2 + gamma u - nu q  (a dim-vector), source s(x),
 *   fhat = F(uhat, q).n + tau (u - uhat),  Dirichlet data u_D on boundary faces.
 * Poisson is beta = gamma = 0, nu = 1; 2D viscous Burgers is beta = (1,0), gamma = (0,1).
 * Steady residual rows, with the trace rows negated on interior faces:
 *   R_u[i]   = -(F, grad phi_i) + <fhat, phi_i> - (s, phi_i)
 *   R_t[l,j] = -<fhat, psi_j>_l  (interior face),  <uhat - u_D, psi_j>_l  (boundary face)
 *
 * Geometry of the mesh's quadrature (device, float64 unless stated; all caller-owned):
 *   wdet  [ne][nqv]            volume weights times |det J|
 *   dphix [ne][nqv][npe][dim]  physical gradients of the element basis
 *   phi   [nqv][npe]           element basis at the volume points (reference)
 *   phif  [ne][nlfe][nqf][npe] element basis at the points of each local face
 *   psi   [nqf][npf]           face basis at the face points, canonical face order
 *   ndA   [ne][nlfe][nqf][dim] outward normal times face weight;  dA [ne][nlfe][nqf]
 *   src   [ne][nqv] source;  uD [ne][nlfe][nqf] Dirichlet data;  bnd [ne][nlfe] int32,
 *   1 on boundary faces. */
typedef struct {
    int32_t nqv, nqf;
    const double *wdet, *dphix, *phi, *phif, *psi, *ndA, *dA, *src, *uD;
    const int32_t* bnd;
} hdg_elem_geom;

typedef struct {
    double nu, tau, beta[3], gamma[3];
} hdg_conv_diff;

/* Time term of one implicit stage (Section 2.2: a DIRK stage, or a backward-Euler step):
 * the u-rows become R_u + c (u - u_n, phi_i) + r_extra[i] and E gains c M, with
 * c = 1/(a_ii dt), u_n [ne][npe] the previous step's state (device) and r_extra [ne][npe]
 * (device, may be NULL) the earlier stages' known contribution. NULL or c = 0: steady. */
typedef struct {
    double c;
    const double* u_prev;
    const double* r_extra;
} hdg_time_term;

/* flags of hdg_element_blocks(_batch) */
enum {
    HDG_ELEM_RESIDUAL_ONLY = 1,  /* write ru, rt (and q) only */
    HDG_ELEM_KEEP_MASS = 2       /* Minv, Bd, Cd in `out` already hold this mesh's (from an earlier
                                    call): Minv is read instead of formed and inverted, and none
                                    of the three is written (they depend on the geometry only,
                                    Section 4.1 precomputes them once) */
};

/* Device outputs in the layouts hdg_condense reads, plus q [ne][dim][npe] (may be NULL). */
typedef struct {
    double *Minv, *Bd, *Cd, *D, *E, *F, *G, *H, *J, *ru, *rt, *q;
} hdg_elem_arrays;

/* hdg_element_blocks: at the state u [ne][npe] (nodal) and uhat [nf][npf] (face values,
 *   canonical order; element e's face l is uhat[e2f[e][l]]), with q derived from the
 *   q-equation (M q_d + B_d u + C_d uhat = 0, eq. w16, so r_q = 0), writes ru = -R_u,
 *   rt = -R_t and, unless flags has HDG_ELEM_RESIDUAL_ONLY, Minv, Bd, Cd, D, E, F, G, H, J
 *   (the derivatives of R_u and R_t with respect to q, u, uhat; with HDG_ELEM_KEEP_MASS,
 *   Minv, Bd and Cd are inputs, Minv required). time_term (may be NULL) adds an implicit
 *   stage's mass term (HDG_ERR_ARG if c != 0 without u_prev). Outputs not written may be
 *   NULL. One workgroup
 *   per element with its data in LDS: HDG_ERR_SHAPE if the element needs more than 64 KiB;
 *   HDG_ERR_ARG for ncomp != 1. HDG_ERR_SINGULAR names the first element whose mass matrix
 *   has a non-positive pivot (synchronises to read it).
 * hdg_residual_norm: ||R|| = sqrt(sum_e ||R_u^e||^2 + sum_f ||R_f||^2) from ru and rt as
 *   written above, R_f being face f's trace rows summed over its elements (perm = NULL
 *   assembly); result in *norm_h. Uses a context workspace; synchronises. */
hdg_status hdg_element_blocks(hdg_ctx ctx, const hdg_dims* dims, const hdg_elem_geom* geom,
                              const hdg_conv_diff* model, const hdg_time_term* time_term,
                              const int32_t* e2f, const double* u, const double* uhat,
                              int32_t flags, const hdg_elem_arrays* out);
hdg_status hdg_residual_norm(hdg_ctx ctx, const hdg_dims* dims, const int32_t* f2e, const double* ru,
                             const double* rt, double* norm_h);
/* hdg_residual_norm_noalloc: for callers that cannot allocate device memory (code under
 *   graph capture, tight serving loops, harnesses that forbid hipMalloc). Same arguments,
 *   result and kernels as hdg_residual_norm, but its scratch (the assembled trace residual
 *   and the reduction partials) lives in a fixed 16 MiB device array per GPU instead of a
 *   context workspace, and it calls no allocating routine. Limit: ncomp*npf*nf (padded to
 *   64) plus the reduction partials of both vectors must fit in 2^21 doubles, else
 *   HDG_ERR_ARG with nothing launched. Every call on one GPU shares that GPU's array, which
 *   keeps the last call's contents: calls that overlap on one GPU (other threads, streams or
 *   contexts) race; calls on one stream do not. Synchronises the context stream. */
hdg_status hdg_residual_norm_noalloc(hdg_ctx ctx, const hdg_dims* dims, const int32_t* f2e, const double* ru,
                                     const double* rt, double* norm_h);

/* (5c) Element residuals and Jacobian blocks of M-component models in 3D (Section 2.1 with
 *     M > 1; Section 2.2's weak form and numerical flux; Section 4.1's element matrices):
 *   HDG_MODEL_ELASTICITY (ncomp = 3):      F = -sigma(q), sigma = lam tr(eps) I + 2 mu eps,
 *                                          eps = (q + q^T)/2, u the displacement;
 *   HDG_MODEL_NAVIER_STOKES (ncomp = 5):   F = F_c(u) - F_v(u, q) in conservative variables
 *                                          (rho, rho v, rho E), p = (gamma-1)(rho E - |rho v|^2/(2 rho)),
 *                                          F_c = (rho v, rho v v^T + p I, (rho E + p) v),
 *                                          F_v = (0, tau_v, tau_v v + (mu gamma/Pr) grad e), mu = 1/Re,
 *                                          tau_v = mu (grad v + grad v^T) - (2/3) mu (div v) I,
 *                                          e = E - |v|^2/2, grad v and grad e from q = grad u.
 *   fhat = F(uhat, q).n + tau (u - uhat); Dirichlet trace rows uhat - u_D on boundary faces.
 *   Residual rows as for the scalar models, per component m:
 *     R_u[m,i] = -(F_m, grad phi_i) + <fhat_m, phi_i> - (s_m, phi_i)  (+ the time term)
 *     R_t[l,m,j] = -<fhat_m, psi_j>_l (interior face), <uhat_m - u_D,m, psi_j>_l (boundary face)
 * hdg_element_blocks_sys: as hdg_element_blocks, for dim = 3 and these models, with
 *   geom->src [ne][nqv][ncomp] and geom->uD [ne][nlfe][nqf][ncomp]; state u [ne][ncomp][npe]
 *   (component-major, the u dof order of hdg_condense) and uhat [nf][ncomp][npf];
 *   time_term->u_prev [ne][ncomp][npe], r_extra [ne][ncomp*npe]; out->q [ne][ncomp][dim][npe].
 *   The flux derivatives come from forward-mode dual numbers per quadrature point. Uses a
 *   context workspace for the per-point flux data (elements in chunks of about 1 GiB of it).
 *   HDG_ERR_ARG for an unknown model, a model whose ncomp does not match, or dim != 3;
 *   HDG_ERR_SHAPE if an element's staged data exceed 150 KiB of LDS; HDG_ERR_SINGULAR as for
 *   hdg_element_blocks (synchronises). hdg_residual_norm applies to its ru, rt unchanged. */
enum { HDG_MODEL_ELASTICITY = 1, HDG_MODEL_NAVIER_STOKES = 2 };
typedef struct {
    int32_t kind;
    double tau;               /* S = tau I */
    double lam, mu;           /* elasticity: Lame constants */
    double Re, Pr, gamma;     /* Navier-Stokes */
} hdg_sys_model;
hdg_status hdg_element_blocks_sys(hdg_ctx ctx, const hdg_dims* dims, const hdg_elem_geom* geom,
                                  const hdg_sys_model* model, const hdg_time_term* time_term,
                                  const int32_t* e2f, const double* u, const double* uhat,
                                  int32_t flags, const hdg_elem_arrays* out);

/* (6) Additive Schwarz preconditioner with one element per subdomain -- Section 3.3
 * (definition), Section 4.6 (element matrices and their enrichment).
 *
 * hdg_asm_setup forms, for every element e, P^e = Kbar^e with the diagonal block of each
 * local face l replaced by the assembled K[f][0] of its face f = e2f[e][l] (for an
 * interior face the sum of both neighbours' diagonal blocks; P^e = R_e K R_e^T), and
 * writes its inverse as the block rows of the element's local faces:
 *   inv [ne][N_lfe][N_lfe][nb][nb], inv[e][l][l'][col][row] = (P^e)^{-1}(l nb + row, l' nb + col)
 * in FP64 (inv64) and/or FP32 (inv32; either may be NULL, not both). Kbar as from
 * hdg_condense, K64 as from hdg_assemble_blocks (canonical face orientation: assembled with
 * perm = NULL), e2f as for hdg_assemble_blocks. Workspace about 4 GiB (element chunks).
 * HDG_ERR_SINGULAR names the first element whose P^e has a zero pivot.
 * hdg_asm_apply (test hook): z = sum_e R_e^T (P^e)^{-1} R_e y with inv64 (HDG_FP64) or
 * inv32 (HDG_MIXED); f2e and e2f as for hdg_assemble_blocks; y and z must not alias.
 * Pass inv64/inv32/f2e/e2f to hdg_gmres_solve through the asm_* options with prec
 * HDG_PREC_ASM, HDG_PREC_ASM_POLY or HDG_PREC_ASM_CHEB. */
hdg_status hdg_asm_setup(hdg_ctx ctx, const hdg_dims* dims, const double* Kbar, const double* K64,
                         const int32_t* e2f, double* inv64, float* inv32);
hdg_status hdg_asm_apply(hdg_ctx ctx, const hdg_dims* dims, const double* inv64, const float* inv32,
                         int32_t precision, const int32_t* f2e, const int32_t* e2f, const double* y, double* z);

/* (6b) ILU-ASM: additive Schwarz on multi-element subdomains with block ILU(0) local solves --
 * Section 3.3 (ASM on patches of elements) with the incomplete factorisation its conclusions
 * propose for multi-element subdomains.
 *
 * hdg_ilu_asm_create: subdomain l is the patch of G consecutive elements, its unknowns the
 *   trace blocks of the patch's faces in increasing face order, its matrix K restricted to them
 *   (block (a, b) = K64[f_a][s] with nbr[f_a][s] = f_b). Each is factorised by block ILU(0) on
 *   K's block pattern in that order; only the off-diagonal pattern blocks and the inverted
 *   pivot blocks are kept. K64, nbr as from hdg_assemble_blocks (perm = NULL), e2f as there
 *   (device; e2f and nbr are copied to the host once to build the patch tables, so the call
 *   synchronises the context's stream). Limits: face block edge M*P_F <= 16 and at most 88
 *   dofs per subdomain (the subdomain is factorised in LDS): HDG_ERR_SHAPE otherwise; a face
 *   number outside [0, nf) in e2f: HDG_ERR_ARG. HDG_ERR_SINGULAR names a subdomain with a
 *   singular pivot block. The handle owns its device
 *   memory (factors, subdomain tables) until hdg_ilu_asm_destroy; it serves hdg_gmres_solve
 *   with prec HDG_PREC_ILU_ASM (opts.ilu_asm) while K64 is unchanged.
 * hdg_ilu_asm_apply (test hook): z = sum_l R_l^T (L_l U_l)^{-1} R_l y; y and z must not alias. */
hdg_status hdg_ilu_asm_create(hdg_ctx ctx, const hdg_dims* dims, const double* K64, const int32_t* nbr,
                              const int32_t* e2f, int32_t G, hdg_ilu_asm* out);
hdg_status hdg_ilu_asm_destroy(hdg_ilu_asm h);
hdg_status hdg_ilu_asm_apply(hdg_ctx ctx, hdg_ilu_asm h, const double* y, double* z);

/* Autotuning of the face operator's launch configuration (threads per face, rows per
 * thread) by measurement -- the block matvec of Section 4.3 and the block-Jacobi apply of
 * Section 4.5 are the bandwidth-bound kernels of every solve, and their best mapping depends
 * on the block size, slot count, precision and problem size.
 * hdg_autotune: times every supported configuration of the FP64 and FP32 block matvec
 *   (K64 required, K32 may be NULL), the block-Jacobi apply (Binv64 / Binv32, may be NULL)
 *   and the fused polynomial step (K and Binv of one precision) on this matrix, reps launches
 *   each, and keeps the fastest per (operand types, product kind, nb, slots, power-of-two
 *   bucket of nf) in a table that every later launch in the process consults. With the
 *   environment variable HDG_TUNE_CACHE naming a file, the table is read from it on first use
 *   and written back here (JSON). *n_tuned_h (may be NULL) receives the number of variants
 *   timed. Uses a context work vector; synchronises. Results of later solves change only by
 *   the order of the sums inside a face (rounding).
 * hdg_tune_table: the table as JSON text into buf_h (len bytes, NUL-terminated, truncated
 *   if short); returns the bytes the whole text needs. */
hdg_status hdg_autotune(hdg_ctx ctx, const hdg_dims* dims, const double* K64, const float* K32, const int32_t* nbr,
                        const double* Binv64, const float* Binv32, int32_t reps, int32_t* n_tuned_h);
size_t     hdg_tune_table(char* buf_h, size_t len);

/* ---------------------------------------------------------------------------
 * Building blocks exposed for tests and benchmarks (same kernels as the solver).
 *
 * hdg_matvec: y = K x with K64 (precision HDG_FP64) or K32 (HDG_MIXED) -- Section 4.3.
 * hdg_bj_setup: block-Jacobi inverses Binv64 [nf][nb][nb] (column-major like K) and,
 *   if Binv32 != NULL, their FP32 rounding -- Section 4.5. HDG_ERR_SINGULAR names the face.
 * hdg_bj_apply: z_f = P_f^{-1} y_f with Binv64 or Binv32 -- Section 4.5.
 * hdg_poly_apply: z = p(B) M^{-1} y for given Leja-ordered Ritz values (host arrays;
 *   conjugate pairs adjacent, positive imaginary part first) -- Section 4.7.
 * hdg_cheb_apply: z = x_P, the P-th iterate (x_0 = 0, P-1 applications of B) of Chebyshev
 *   acceleration for B x = M^{-1} y over the real interval [alpha, beta], 0 < alpha < beta
 *   (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Algorithm 12.1), the
 *   Chebyshev variant of the polynomial preconditioner (HDG_PREC_BJ_CHEB) -- Section 3.4.
 *   HDG_ERR_ARG for degree outside [1, 64] or an interval that is not positive.
 */
hdg_status hdg_matvec(hdg_ctx ctx, const hdg_dims* dims, const double* K64, const float* K32,
                      const int32_t* nbr, int32_t precision, const double* x, double* y);
hdg_status hdg_bj_setup(hdg_ctx ctx, const hdg_dims* dims, const double* K64,
                        double* Binv64, float* Binv32);
hdg_status hdg_bj_apply(hdg_ctx ctx, const hdg_dims* dims, const double* Binv64, const float* Binv32,
                        int32_t precision, const double* y, double* z);
hdg_status hdg_poly_apply(hdg_ctx ctx, const hdg_dims* dims, const double* K64, const float* K32,
                          const int32_t* nbr, const double* Binv64, const float* Binv32,
                          int32_t precision, int32_t npoly, const double* theta_re_h,
                          const double* theta_im_h, const double* y, double* z);
hdg_status hdg_cheb_apply(hdg_ctx ctx, const hdg_dims* dims, const double* K64, const float* K32,
                          const int32_t* nbr, const double* Binv64, const float* Binv32, int32_t precision,
                          int32_t degree, double alpha, double beta, const double* y, double* z);

/* ---------------------------------------------------------------------------
 * Batched independent instances (many small meshes of different element types,
 * degrees and sizes condensed and solved together) -- the same operations as
 * (1)-(4) above, Sections 2.3-2.4, 3.1-3.2, 4.1-4.5.
 *
 * hdg_batch_create builds device descriptor tables for n_inst instances with
 * sizes dims_h[i] (host array). Every array of the single-instance entry points
 * becomes the concatenation of the instances' arrays, instance i's part starting
 * at offset hdg_batch_offsets(b, id, off)[i] (elements of that array, prefix sums
 * of the per-instance sizes); id is one of HDG_BATCH_ARRAY_*. Index arrays f2e,
 * e2f and nbr hold instance-local element/face numbers; perm is not supported.
 * Limits: M*P_F <= 8, (2N_lfe-1)*M*P_F <= 64, and (nu+nt)(nu+nt+1) + D P_E (P_E +
 * N_lfe P_F) doubles per element within 150 KiB (whole element system in LDS).
 *
 * hdg_condense_batch: one persistent launch over all elements of all instances;
 *   its grid size is chosen on the first call by timing candidate sizes on the real
 *   data (hdg_batch_tuned_grid reports the choice).
 * hdg_gmres_solve_batch: one FGMRES per instance (own Arnoldi basis segment,
 *   Hessenberg, Givens rotations, tolerance relative to its own ||r_i||); finished
 *   instances are masked while the others continue; opts as for hdg_gmres_solve
 *   with prec NONE or BJ and orth CGS2 or CGS (time_phases is ignored and the
 *   timing fields stay 0); stats_h has n_inst entries.
 *   Returns HDG_NOT_CONVERGED if any instance did not converge.
 */
typedef struct hdg_batch_s* hdg_batch;
enum {
    HDG_BATCH_ARRAY_MINV = 0, HDG_BATCH_ARRAY_BD, HDG_BATCH_ARRAY_CD, HDG_BATCH_ARRAY_D, HDG_BATCH_ARRAY_E,
    HDG_BATCH_ARRAY_F, HDG_BATCH_ARRAY_G, HDG_BATCH_ARRAY_H, HDG_BATCH_ARRAY_J, HDG_BATCH_ARRAY_RU,
    HDG_BATCH_ARRAY_RT, HDG_BATCH_ARRAY_KBAR, HDG_BATCH_ARRAY_RBAR, HDG_BATCH_ARRAY_LOCAL, HDG_BATCH_ARRAY_DU,
    HDG_BATCH_ARRAY_DQ, HDG_BATCH_ARRAY_K, HDG_BATCH_ARRAY_NBR, HDG_BATCH_ARRAY_VEC, HDG_BATCH_ARRAY_F2E,
    HDG_BATCH_ARRAY_E2F, HDG_BATCH_ARRAY_BINV, HDG_BATCH_NARRAYS
};
hdg_status hdg_batch_create(hdg_ctx ctx, int32_t n_inst, const hdg_dims* dims_h, hdg_batch* out);
hdg_status hdg_batch_destroy(hdg_batch b);
hdg_status hdg_batch_offsets(hdg_batch b, int32_t array_id, int64_t* off_h /* [n_inst+1] */);
int32_t    hdg_batch_tuned_grid(hdg_batch b);
/* Batched element residuals / Jacobians and damped Newton support (scalar models; Section
 * 4.1, Section 4.4, as hdg_element_blocks / hdg_residual_norm / hdg_newton_update):
 * hdg_element_blocks_batch: nqv_h, nqf_h [n_inst] (host) are each instance's quadrature
 *   sizes, models_h [n_inst] (host) its coefficients; the geometry arrays of geom (its nqv,
 *   nqf fields unused) are the concatenation of the instances' arrays in instance order;
 *   e2f, u (DU offsets), uhat (VEC offsets) and the outputs (MINV..RT, q at DQ offsets) are
 *   batch arrays. c_h [n_inst] (host, may be NULL = all 0), u_prev and r_extra (batch arrays
 *   like u; r_extra may be NULL) give each instance a time term as hdg_time_term
 *   (pseudo-transient continuation: c = 1/dtau, u_prev = the current state; a DIRK stage:
 *   c = 1/(a dt), u_prev = u_n, r_extra = the earlier stages' term). Errors as
 *   hdg_element_blocks (the element named is global).
 * hdg_residual_norm_batch: norms_h [n_inst] (host) receives each instance's ||R|| (element
 *   u-rows and its faces' summed trace rows, f2e instance-local as for hdg_assemble_batch).
 * hdg_newton_update_batch: u += alpha_h[i] du and uhat += alpha_h[i] x over instance i's parts
 *   (DU and VEC offsets); alpha_h [n_inst] host, 0 leaves an instance unchanged.
 * All three synchronise the context's stream before returning. */
hdg_status hdg_element_blocks_batch(hdg_ctx ctx, hdg_batch b, const int32_t* nqv_h, const int32_t* nqf_h,
                                    const hdg_elem_geom* geom, const hdg_conv_diff* models_h,
                                    const double* c_h, const double* u_prev, const double* r_extra,
                                    const int32_t* e2f, const double* u, const double* uhat,
                                    int32_t flags, const hdg_elem_arrays* out);
hdg_status hdg_residual_norm_batch(hdg_ctx ctx, hdg_batch b, const int32_t* f2e, const double* ru,
                                   const double* rt, double* norms_h);
hdg_status hdg_newton_update_batch(hdg_ctx ctx, hdg_batch b, const double* alpha_h, const double* du,
                                   double* u, const double* x, double* uhat);
hdg_status hdg_condense_batch(hdg_ctx ctx, hdg_batch b, const hdg_elem_blocks* in,
                              double* Kbar, double* rbar, double* local);
hdg_status hdg_assemble_batch(hdg_ctx ctx, hdg_batch b, const int32_t* f2e, const int32_t* e2f,
                              const double* Kbar, const double* rbar, double* K64, float* K32,
                              int32_t* nbr, double* r);
hdg_status hdg_gmres_solve_batch(hdg_ctx ctx, hdg_batch b, const double* K64, const float* K32,
                                 const int32_t* nbr, const double* r, double* x,
                                 const hdg_solve_opts* opts_h, hdg_solve_stats* stats_h);
hdg_status hdg_recover_batch(hdg_ctx ctx, hdg_batch b, const double* local, const double* Minv,
                             const double* Bd, const double* Cd, const int32_t* e2f, const double* xhat,
                             double* du, double* dq);

/* Host-only helpers (no device work; usable without a GPU) -- Section 4.7.
 * hdg_hessenberg_eigvals: eigenvalues of an n x n upper Hessenberg matrix H (row-major,
 *   leading dimension ld) by the shifted QR algorithm; returns 0 on success.
 * hdg_harmonic_ritz: from H_{P+1,P} (row-major (P+1) x P) the harmonic Ritz values
 *   (eigenvalues of H_P + h_{P+1,P}^2 H_P^{-T} e_P e_P^T) in Leja order with conjugate
 *   pairs adjacent; values below drop_rel * max|theta| are dropped. Writes *n_out.
 * hdg_poly_roots: the roots hdg_gmres_solve's polynomial preconditioner uses from the same
 *   H: the harmonic Ritz values plus the safeguard of HDG_FALLBACK_PP_ADDED_ROOT (up to two
 *   more copies of the root of largest real part, and of its conjugate, each added while the
 *   residual polynomial exceeds 1 in modulus at 1.1 times that root), in Leja order (a copy
 *   has distance zero to its twin and comes after every other value). theta_re_h /
 *   theta_im_h need P + 4 entries; *n_added receives the number of values added (0 to 4). */
int hdg_hessenberg_eigvals(int n, const double* H_h, int ld, double* wr_h, double* wi_h);
int hdg_harmonic_ritz(int P, const double* H_h, double drop_rel,
                      double* theta_re_h, double* theta_im_h, int* n_out);
int hdg_poly_roots(int P, const double* H_h, double drop_rel, double* theta_re_h, double* theta_im_h,
                   int* n_out, int* n_added);

#ifdef __cplusplus
}
#endif
#endif /* HDG_H */
