// Element residuals and Jacobian blocks on the device for M-component models in 3D
// (Section 2.1, Section 2.2's weak form and numerical flux, Section 4.1's element matrices):
//   linear elasticity (M = 3)   F = -sigma(q), sigma = lam tr(eps) I + 2 mu eps, eps = sym(q);
//   compressible Navier-Stokes  F = F_c(u) - F_v(u, q), conservative u = (rho, rho v, rho E),
//   (M = 5)                     mu = 1/Re, Stokes hypothesis, heat flux (mu gamma / Pr) grad e.
// fhat = F(uhat, q).n + tau (u - uhat); Dirichlet trace rows uhat - u_D on boundary faces.
//
// Two kernels per chunk of elements:
//   1. k_sys_points: per element, the mass matrix and its inverse, B_d and C_d, the consistent
//      q = -M^{-1}(B_d u_m + C_d uhat_m) (eq. w16, r_q = 0), the state at the volume and face
//      quadrature points, then per point the flux and its derivatives with respect to u and q
//      by forward-mode dual numbers (one evaluation per input direction), stored weighted
//      (volume) or contracted with the scaled normal (faces) in a point workspace;
//   2. k_sys_blocks: every output entry as one sum over the points of that workspace times
//      the basis values -- the products of per-point flux data with the basis tables that
//      Section 4.1 forms (E = Psi U), evaluated per element.
// Residual rows (trace rows negated on interior faces), with an implicit stage's time term
// (c = 1/(a_ii dt), u_n, r_x):
//   R_u[m,i]   = -(F_m, grad phi_i) + <fhat_m, phi_i> - (s_m, phi_i) + c (u_m - u_n,m, phi_i) + r_x
//   R_t[l,m,j] = -<fhat_m, psi_j>_l (interior),  <uhat_m - u_D,m, psi_j>_l (Dirichlet)
// ru = -R_u, rt = -R_t; D..J their derivatives with respect to q, u and uhat.
#include <cmath>

#include "hdg_internal.hpp"

namespace {

constexpr int SBS = 256;
constexpr int SD = 3;        // space dimension of both models
constexpr int TJ = 4;        // output columns per work item

struct Dual {
    double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    const double r = 1.0 / b.v;
    return {a.v * r, (a.d - a.v * r * b.d) * r};
}
__device__ __forceinline__ Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ Dual operator+(Dual a, double s) { return {a.v + s, a.d}; }
__device__ __forceinline__ Dual operator-(Dual a, double s) { return {a.v - s, a.d}; }
__device__ __forceinline__ Dual dconst(double v) { return {v, 0.0}; }

struct SysParams {
    int kind;
    double tau, lam, mu, Re, Pr, gamma;
};

// F[a][x] of linear elasticity (u is not used)
template <class T>
__device__ __forceinline__ void flux_elasticity(const SysParams& p, const T (&u)[3], const T (&q)[3][SD],
                                                T (&F)[3][SD]) {
    (void)u;
    const T tr = q[0][0] + q[1][1] + q[2][2];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int x = 0; x < SD; ++x) {
            T s = p.mu * (q[a][x] + q[x][a]);
            if (a == x) s = s + p.lam * tr;
            F[a][x] = dconst(0.0) - s;
        }
}

// F[a][x] of the compressible Navier-Stokes equations
template <class T>
__device__ __forceinline__ void flux_navier_stokes(const SysParams& p, const T (&u)[5], const T (&q)[5][SD],
                                                   T (&F)[5][SD]) {
    const double g = p.gamma, mu = 1.0 / p.Re, kappa = mu * g / p.Pr;
    const T rho = u[0], rE = u[4];
    T v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = u[1 + a] / rho;
    const T pr = (g - 1.0) * (rE - 0.5 * (u[1] * v[0] + u[2] * v[1] + u[3] * v[2]));
    const T E = rE / rho;
    T gv[3][SD];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int x = 0; x < SD; ++x) gv[a][x] = (q[1 + a][x] - v[a] * q[0][x]) / rho;
    const T div = gv[0][0] + gv[1][1] + gv[2][2];
#pragma unroll
    for (int x = 0; x < SD; ++x) {
        const T ge = (q[4][x] - E * q[0][x]) / rho - (v[0] * gv[0][x] + v[1] * gv[1][x] + v[2] * gv[2][x]);
        F[0][x] = u[1 + x];
        T work = dconst(0.0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T tv = mu * (gv[a][x] + gv[x][a]);
            if (a == x) tv = tv - (2.0 / 3.0) * mu * div;
            T f = u[1 + a] * v[x] - tv;
            if (a == x) f = f + pr;
            F[1 + a][x] = f;
            work = work + tv * v[a];
        }
        F[4][x] = (rE + pr) * v[x] - work - kappa * ge;
    }
}

template <int M>
__device__ __forceinline__ void flux(const SysParams& p, const Dual (&u)[M], const Dual (&q)[M][SD],
                                     Dual (&F)[M][SD]) {
    if constexpr (M == 3) flux_elasticity(p, u, q, F);
    else flux_navier_stokes(p, u, q, F);
}

// Per-element sizes of the point workspace (doubles), in the order written below.
struct PointWs {
    int vF, vS, vU, vQ, fH, fB, fZ, fY, per_elem;
};
__host__ __device__ inline PointWs point_ws(int M, int Qv, int LQf) {
    PointWs w;
    int o = 0;
    w.vF = o; o += Qv * M * SD;              // w F[a][x]
    w.vS = o; o += Qv * M;                   // w (s_a - c (u - u_n)_a)
    w.vU = o; o += Qv * M * M * SD;          // w dF[a][x]/du_b            [x][a][b][xi]
    w.vQ = o; o += Qv * M * M * SD * SD;     // w dF[a][xi]/dq_bd          [x][a][b][d][xi]
    w.fH = o; o += LQf * M;                  // fhat_a
    w.fB = o; o += LQf * M;                  // dA (uhat - u_D)_a
    w.fZ = o; o += LQf * M * M;              // sum_xi dF[a][xi]/duhat_b n_xi
    w.fY = o; o += LQf * M * M * SD;         // sum_xi dF[a][xi]/dq_bd n_xi  [lx][a][b][d]
    w.per_elem = o;
    return w;
}

// LDS of k_sys_points (doubles)
struct PtsLds {
    int Mm, un, up, uh, qn, t, uq, duq, qq, uf, uhf, qf, total;
};
__host__ __device__ inline PtsLds pts_lds(int M, int P, int PF, int L, int Qv, int Qf) {
    PtsLds o;
    int k = 0;
    o.Mm = k; k += P * P;
    o.un = k; k += M * P;
    o.up = k; k += M * P;
    o.uh = k; k += L * M * PF;
    o.qn = k; k += M * SD * P;
    o.t = k;  k += M * SD * P;
    o.uq = k; k += Qv * M;
    o.duq = k; k += Qv * M;
    o.qq = k; k += Qv * M * SD;
    o.uf = k; k += L * Qf * M;
    o.uhf = k; k += L * Qf * M;
    o.qf = k; k += L * Qf * M * SD;
    o.total = k;
    return o;
}

struct SysArgs {
    hdg_elem_geom g;        // src [ne][nqv][M], uD [ne][nlfe][nqf][M]
    SysParams pm;
    const int32_t* e2f;
    const double* u;        // [ne][M][P]
    const double* uhat;     // [nf][M][PF]
    const double* u_prev;   // [ne][M][P] when c != 0
    const double* r_extra;  // [ne][M*P] or null
    double c;
    hdg_elem_arrays out;
    double* ws;             // point workspace of the chunk
    int* bad;
    int e0, P, PF, L, Qv, Qf, residual_only, keep_mass;
};

template <int M>
__global__ void __launch_bounds__(SBS) k_sys_points(SysArgs a) {
    extern __shared__ double sm[];
    const int el = blockIdx.x;
    const size_t e = (size_t)a.e0 + el;
    const int tid = threadIdx.x;
    const int P = a.P, PF = a.PF, L = a.L, Qv = a.Qv, Qf = a.Qf, LQf = L * Qf, LPF = L * PF;
    const PtsLds o = pts_lds(M, P, PF, L, Qv, Qf);
    double *Mm = sm + o.Mm, *un = sm + o.un, *up = sm + o.up, *uh = sm + o.uh, *qn = sm + o.qn, *t = sm + o.t;
    double *uq = sm + o.uq, *duq = sm + o.duq, *qq = sm + o.qq, *uf = sm + o.uf, *uhf = sm + o.uhf, *qf = sm + o.qf;
    const double* wdet = a.g.wdet + e * Qv;
    const double* dphix = a.g.dphix + e * Qv * P * SD;
    const double* phi = a.g.phi;
    const double* phif = a.g.phif + e * LQf * P;
    const double* psi = a.g.psi;
    const double* ndA = a.g.ndA + e * LQf * SD;
    const double* dA = a.g.dA + e * LQf;
    const double* src = a.g.src + e * Qv * M;
    const double* uD = a.g.uD + e * LQf * M;
    const int32_t* e2f = a.e2f + e * L;
    const double cdt = a.c;

    // 1. nodal state
    for (int k = tid; k < M * P; k += SBS) {
        un[k] = a.u[e * M * P + k];
        up[k] = cdt != 0.0 ? a.u_prev[e * M * P + k] : 0.0;
    }
    for (int k = tid; k < L * M * PF; k += SBS) {
        const int l = k / (M * PF), r = k - l * M * PF;
        uh[k] = a.uhat[(size_t)e2f[l] * M * PF + r];
    }
    // 2. mass matrix and its inverse (Gauss-Jordan in place; M is SPD), or the kept inverse
    if (a.keep_mass) {
        for (int k = tid; k < P * P; k += SBS) Mm[k] = a.out.Minv[e * P * P + k];
        __syncthreads();
    } else {
        for (int k = tid; k < P * P; k += SBS) {
            const int i = k / P, j = k - i * P;
            double s = 0.0;
            for (int x = 0; x < Qv; ++x) s += wdet[x] * phi[x * P + i] * phi[x * P + j];
            Mm[k] = s;
        }
        __syncthreads();
        for (int k = 0; k < P; ++k) {
            const double piv = Mm[k * P + k];
            if (!(piv > 0.0) || !isfinite(piv)) {
                if (tid == 0) atomicMin(a.bad, (int)e);
                return;    // uniform across the workgroup: every thread read the same pivot
            }
            const double rp = 1.0 / piv;
            for (int idx = tid; idx < P * P; idx += SBS) {
                const int i = idx / P, j = idx - i * P;
                if (i == k || j == k) continue;
                Mm[idx] -= Mm[i * P + k] * rp * Mm[k * P + j];
            }
            __syncthreads();
            for (int idx = tid; idx < P; idx += SBS) {
                if (idx != k) {
                    Mm[idx * P + k] = -Mm[idx * P + k] * rp;
                    Mm[k * P + idx] *= rp;
                }
            }
            if (tid == 0) Mm[k * P + k] = rp;
            __syncthreads();
        }
        if (a.out.Minv)
            for (int k = tid; k < P * P; k += SBS) a.out.Minv[e * P * P + k] = Mm[k];
    }
    // B_d [d][i][j] and C_d [d][i][(l,j)] (geometry only)
    if (!a.keep_mass && !a.residual_only) {
        for (int k = tid; k < SD * P * P; k += SBS) {
            const int d = k / (P * P), r = k - d * P * P, i = r / P, j = r - i * P;
            double s = 0.0;
            for (int x = 0; x < Qv; ++x) s += wdet[x] * dphix[(x * P + i) * SD + d] * phi[x * P + j];
            a.out.Bd[e * SD * P * P + k] = s;
        }
        for (int k = tid; k < SD * P * LPF; k += SBS) {
            const int d = k / (P * LPF), r = k - d * P * LPF, i = r / LPF, c = r - i * LPF;
            const int l = c / PF, j = c - l * PF;
            double s = 0.0;
            for (int x = 0; x < Qf; ++x) {
                const int lx = l * Qf + x;
                s -= ndA[lx * SD + d] * phif[lx * P + i] * psi[x * PF + j];
            }
            a.out.Cd[e * SD * P * LPF + k] = s;
        }
    }
    // 3. u, u - u_n at the volume points; u and uhat at the face points
    for (int k = tid; k < Qv * M; k += SBS) {
        const int x = k / M, m = k - x * M;
        double s = 0.0, sp = 0.0;
        for (int i = 0; i < P; ++i) {
            s += phi[x * P + i] * un[m * P + i];
            sp += phi[x * P + i] * up[m * P + i];
        }
        uq[k] = s;
        duq[k] = s - sp;
    }
    for (int k = tid; k < LQf * M; k += SBS) {
        const int lx = k / M, m = k - lx * M, l = lx / Qf, x = lx - l * Qf;
        double s = 0.0, h = 0.0;
        for (int i = 0; i < P; ++i) s += phif[lx * P + i] * un[m * P + i];
        for (int j = 0; j < PF; ++j) h += psi[x * PF + j] * uh[(l * M + m) * PF + j];
        uf[k] = s;
        uhf[k] = h;
    }
    __syncthreads();
    // 4. q = -M^{-1} (B_d u_m + C_d uhat_m), summed over the points
    for (int k = tid; k < M * SD * P; k += SBS) {
        const int m = k / (SD * P), r = k - m * SD * P, d = r / P, i = r - d * P;
        double s = 0.0;
        for (int x = 0; x < Qv; ++x) s += wdet[x] * dphix[(x * P + i) * SD + d] * uq[x * M + m];
        for (int lx = 0; lx < LQf; ++lx) s -= ndA[lx * SD + d] * phif[lx * P + i] * uhf[lx * M + m];
        t[k] = s;
    }
    __syncthreads();
    for (int k = tid; k < M * SD * P; k += SBS) {
        const int md = k / P, i = k - md * P;
        double s = 0.0;
        for (int j = 0; j < P; ++j) s += Mm[i * P + j] * t[md * P + j];
        qn[k] = -s;
        if (a.out.q) a.out.q[e * M * SD * P + k] = -s;
    }
    __syncthreads();
    // q at the points
    for (int k = tid; k < Qv * M * SD; k += SBS) {
        const int x = k / (M * SD), md = k - x * M * SD;
        double s = 0.0;
        for (int i = 0; i < P; ++i) s += phi[x * P + i] * qn[md * P + i];
        qq[k] = s;
    }
    for (int k = tid; k < LQf * M * SD; k += SBS) {
        const int lx = k / (M * SD), md = k - lx * M * SD;
        double s = 0.0;
        for (int i = 0; i < P; ++i) s += phif[lx * P + i] * qn[md * P + i];
        qf[k] = s;
    }
    __syncthreads();
    // 5. flux and its derivatives per point (one point per thread)
    const PointWs W = point_ws(M, Qv, LQf);
    double* ws = a.ws + (size_t)el * W.per_elem;
    const bool jac = !a.residual_only;
    for (int k = tid; k < Qv + LQf; k += SBS) {
        const bool vol = k < Qv;
        const int lx = k - Qv;
        Dual uu[M], qd[M][SD], F[M][SD];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            uu[m] = dconst(vol ? uq[k * M + m] : uhf[lx * M + m]);
#pragma unroll
            for (int d = 0; d < SD; ++d) qd[m][d] = dconst(vol ? qq[(k * M + m) * SD + d] : qf[(lx * M + m) * SD + d]);
        }
        flux<M>(a.pm, uu, qd, F);
        if (vol) {
            const double w = wdet[k];
#pragma unroll
            for (int m = 0; m < M; ++m) {
#pragma unroll
                for (int x = 0; x < SD; ++x) ws[W.vF + (k * M + m) * SD + x] = w * F[m][x].v;
                ws[W.vS + k * M + m] = w * (src[k * M + m] - cdt * duq[k * M + m]);
            }
        } else {
            double n[SD];
#pragma unroll
            for (int x = 0; x < SD; ++x) n[x] = ndA[lx * SD + x];
            const double da = dA[lx];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                double fn = 0.0;
#pragma unroll
                for (int x = 0; x < SD; ++x) fn += F[m][x].v * n[x];
                ws[W.fH + lx * M + m] = fn + a.pm.tau * (uf[lx * M + m] - uhf[lx * M + m]) * da;
                ws[W.fB + lx * M + m] = da * (uhf[lx * M + m] - uD[lx * M + m]);
            }
        }
        if (!jac) continue;
        // derivatives: one dual evaluation per input direction (u_b, then q_bd)
#pragma unroll 1
        for (int dir = 0; dir < M + M * SD; ++dir) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                uu[m].d = (dir == m) ? 1.0 : 0.0;
#pragma unroll
                for (int d = 0; d < SD; ++d) qd[m][d].d = (dir == M + m * SD + d) ? 1.0 : 0.0;
            }
            flux<M>(a.pm, uu, qd, F);
            const int b = dir < M ? dir : (dir - M) / SD, dq = dir < M ? -1 : (dir - M) - b * SD;
            if (vol) {
                const double w = wdet[k];
#pragma unroll
                for (int m = 0; m < M; ++m)
#pragma unroll
                    for (int x = 0; x < SD; ++x) {
                        if (dq < 0) ws[W.vU + ((k * M + m) * M + b) * SD + x] = w * F[m][x].d;
                        else ws[W.vQ + (((k * M + m) * M + b) * SD + dq) * SD + x] = w * F[m][x].d;
                    }
            } else {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    double s = 0.0;
#pragma unroll
                    for (int x = 0; x < SD; ++x) s += F[m][x].d * ndA[lx * SD + x];
                    if (dq < 0) ws[W.fZ + (lx * M + m) * M + b] = s;
                    else ws[W.fY + ((lx * M + m) * M + b) * SD + dq] = s;
                }
            }
        }
    }
}

template <int M>
__global__ void __launch_bounds__(SBS) k_sys_blocks(SysArgs a) {
    const int el = blockIdx.x;
    const size_t e = (size_t)a.e0 + el;
    const int tid = threadIdx.x;
    const int P = a.P, PF = a.PF, L = a.L, Qv = a.Qv, Qf = a.Qf, LQf = L * Qf;
    const int nu = M * P, nq = M * SD * P, nt = L * M * PF;
    const PointWs W = point_ws(M, Qv, LQf);
    const double* ws = a.ws + (size_t)el * W.per_elem;
    const double* wdet = a.g.wdet + e * Qv;
    const double* dphix = a.g.dphix + e * Qv * P * SD;
    const double* phi = a.g.phi;
    const double* phif = a.g.phif + e * LQf * P;
    const double* psi = a.g.psi;
    const double* dA = a.g.dA + e * LQf;
    const int32_t* bnd = a.g.bnd + e * L;
    const double tau = a.pm.tau, cdt = a.c;
    // ru[a][i]
    for (int k = tid; k < nu; k += SBS) {
        const int m = k / P, i = k - m * P;
        double s = 0.0;
        for (int x = 0; x < Qv; ++x) {
            double g = 0.0;
#pragma unroll
            for (int d = 0; d < SD; ++d) g += ws[W.vF + (x * M + m) * SD + d] * dphix[(x * P + i) * SD + d];
            s += g + ws[W.vS + x * M + m] * phi[x * P + i];
        }
        for (int lx = 0; lx < LQf; ++lx) s -= ws[W.fH + lx * M + m] * phif[lx * P + i];
        if (a.r_extra) s -= a.r_extra[e * nu + k];
        a.out.ru[e * nu + k] = s;
    }
    // rt[(l,a,j)]
    for (int k = tid; k < nt; k += SBS) {
        const int l = k / (M * PF), r = k - l * M * PF, m = r / PF, j = r - m * PF;
        const bool bd = bnd[l] != 0;
        double s = 0.0;
        for (int x = 0; x < Qf; ++x) {
            const int lx = l * Qf + x;
            s += (bd ? -ws[W.fB + lx * M + m] : ws[W.fH + lx * M + m]) * psi[x * PF + j];
        }
        a.out.rt[e * nt + k] = s;
    }
    if (a.residual_only) return;
    const int nJT = (P + TJ - 1) / TJ;
    // D[(a,i)][(b,d,j)] and E[(a,i)][(b,j)]: work item (a, b, slot, i, j-tile), slot d < SD for D,
    // slot SD for E
    for (int it = tid; it < M * M * (SD + 1) * P * nJT; it += SBS) {
        int r = it;
        const int jt = r % nJT; r /= nJT;
        const int i = r % P; r /= P;
        const int sl = r % (SD + 1); r /= (SD + 1);
        const int b = r % M;
        const int am = r / M;
        const int j0 = jt * TJ;
        double acc[TJ] = {};
        for (int x = 0; x < Qv; ++x) {
            double cf = 0.0;
            if (sl < SD) {
#pragma unroll
                for (int xi = 0; xi < SD; ++xi)
                    cf -= ws[W.vQ + (((x * M + am) * M + b) * SD + sl) * SD + xi] * dphix[(x * P + i) * SD + xi];
            } else {
#pragma unroll
                for (int xi = 0; xi < SD; ++xi)
                    cf -= ws[W.vU + ((x * M + am) * M + b) * SD + xi] * dphix[(x * P + i) * SD + xi];
                if (am == b) cf += cdt * wdet[x] * phi[x * P + i];
            }
#pragma unroll
            for (int jj = 0; jj < TJ; ++jj)
                if (j0 + jj < P) acc[jj] += cf * phi[x * P + j0 + jj];
        }
        for (int lx = 0; lx < LQf; ++lx) {
            const double pi = phif[lx * P + i];
            const double cf = sl < SD ? ws[W.fY + ((lx * M + am) * M + b) * SD + sl] * pi
                                      : (am == b ? tau * dA[lx] * pi : 0.0);
#pragma unroll
            for (int jj = 0; jj < TJ; ++jj)
                if (j0 + jj < P) acc[jj] += cf * phif[lx * P + j0 + jj];
        }
#pragma unroll
        for (int jj = 0; jj < TJ; ++jj) {
            const int j = j0 + jj;
            if (j >= P) continue;
            if (sl < SD) a.out.D[e * nu * nq + (size_t)(am * P + i) * nq + (b * SD + sl) * P + j] = acc[jj];
            else a.out.E[e * nu * nu + (size_t)(am * P + i) * nu + b * P + j] = acc[jj];
        }
    }
    // F[(a,i)][(l,b,j)] and H[(l,b,j)][(a,i)] (H's entry uses the same face sums with a, b swapped
    // roles: H[(l,a,j)][(b,k)] = -tau delta_ab sum dA psi_j phi_k for interior faces)
    for (int it = tid; it < nu * nt; it += SBS) {
        const int row = it / nt, c = it - row * nt;
        const int am = row / P, i = row - am * P;
        const int l = c / (M * PF), r = c - l * M * PF, b = r / PF, j = r - b * PF;
        double f = 0.0, h = 0.0;
        for (int x = 0; x < Qf; ++x) {
            const int lx = l * Qf + x;
            const double w = phif[lx * P + i] * psi[x * PF + j];
            f += (ws[W.fZ + (lx * M + am) * M + b] - (am == b ? tau * dA[lx] : 0.0)) * w;
            h += dA[lx] * w;
        }
        a.out.F[e * nu * nt + it] = f;
        // H row (l, b, j), column (a, i): nonzero only for b == a on interior faces
        a.out.H[e * nt * nu + (size_t)c * nu + row] = (bnd[l] == 0 && am == b) ? -tau * h : 0.0;
    }
    // G[(l,a,j)][(b,d,k)]
    for (int it = tid; it < nt * nq; it += SBS) {
        const int row = it / nq, c = it - row * nq;
        const int l = row / (M * PF), r = row - l * M * PF, am = r / PF, j = r - am * PF;
        const int b = c / (SD * P), r2 = c - b * SD * P, d = r2 / P, kk = r2 - d * P;
        double s = 0.0;
        if (bnd[l] == 0)
            for (int x = 0; x < Qf; ++x) {
                const int lx = l * Qf + x;
                s -= ws[W.fY + ((lx * M + am) * M + b) * SD + d] * psi[x * PF + j] * phif[lx * P + kk];
            }
        a.out.G[e * nt * nq + it] = s;
    }
    // J[(l,a,j)][(l',b,k)], block diagonal in l
    for (int it = tid; it < nt * nt; it += SBS) {
        const int row = it / nt, c = it - row * nt;
        const int l = row / (M * PF), r = row - l * M * PF, am = r / PF, j = r - am * PF;
        const int l2 = c / (M * PF), r2 = c - l2 * M * PF, b = r2 / PF, kk = r2 - b * PF;
        double s = 0.0;
        if (l == l2) {
            const bool bd = bnd[l] != 0;
            for (int x = 0; x < Qf; ++x) {
                const int lx = l * Qf + x;
                const double coef = bd ? (am == b ? dA[lx] : 0.0)
                                       : ((am == b ? tau * dA[lx] : 0.0) - ws[W.fZ + (lx * M + am) * M + b]);
                s += coef * psi[x * PF + j] * psi[x * PF + kk];
            }
        }
        a.out.J[e * nt * nt + it] = s;
    }
}

}  // namespace

size_t element_sys_lds_bytes(const hdg_dims* d, int nqv, int nqf) {
    return sizeof(double) * (size_t)pts_lds(d->ncomp, d->npe, d->npf, d->nlfe, nqv, nqf).total;
}

size_t element_sys_ws_doubles(const hdg_dims* d, int nqv, int nqf) {
    return (size_t)point_ws(d->ncomp, nqv, d->nlfe * nqf).per_elem;
}

// The two kernels over elements [e0, e0 + n) with the point workspace `ws`.
hdg_status element_sys_run(hdg_ctx ctx, const hdg_dims* d, const hdg_elem_geom* g, const hdg_sys_model* m,
                           const hdg_time_term* tt, const int32_t* e2f, const double* u, const double* uhat,
                           int32_t flags, const hdg_elem_arrays* out, int* bad, double* ws, int64_t e0, int64_t n) {
    if (n <= 0) return HDG_OK;
    SysArgs a;
    a.g = *g;
    a.pm.kind = m->kind;
    a.pm.tau = m->tau;
    a.pm.lam = m->lam;
    a.pm.mu = m->mu;
    a.pm.Re = m->Re;
    a.pm.Pr = m->Pr;
    a.pm.gamma = m->gamma;
    a.e2f = e2f;
    a.u = u;
    a.uhat = uhat;
    a.c = tt ? tt->c : 0.0;
    a.u_prev = tt ? tt->u_prev : nullptr;
    a.r_extra = tt ? tt->r_extra : nullptr;
    a.out = *out;
    a.ws = ws;
    a.bad = bad;
    a.e0 = (int)e0;
    a.P = d->npe;
    a.PF = d->npf;
    a.L = d->nlfe;
    a.Qv = g->nqv;
    a.Qf = g->nqf;
    a.residual_only = (flags & HDG_ELEM_RESIDUAL_ONLY) != 0;
    a.keep_mass = (flags & HDG_ELEM_KEEP_MASS) != 0;
    const size_t lds = element_sys_lds_bytes(d, g->nqv, g->nqf);
    const void* kp = d->ncomp == 3 ? (const void*)k_sys_points<3> : (const void*)k_sys_points<5>;
    const void* kb = d->ncomp == 3 ? (const void*)k_sys_blocks<3> : (const void*)k_sys_blocks<5>;
    if (lds > 64 * 1024) HDG_HIP_CHECK(ctx, hipFuncSetAttribute(kp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    void* args[] = {(void*)&a};
    HDG_HIP_CHECK(ctx, hipLaunchKernel(kp, dim3((unsigned)n), dim3(SBS), args, lds, ctx->stream));
    HDG_LAUNCH_CHECK(ctx);
    HDG_HIP_CHECK(ctx, hipLaunchKernel(kb, dim3((unsigned)n), dim3(SBS), args, 0, ctx->stream));
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}
