// Element residuals and Jacobian blocks on the device (Section 4.1, Section 4.4's residual
// evaluation) for scalar convection-diffusion models
//   F(u, q) = beta u^2/2 + gamma u - nu q,   fhat = F(uhat, q).n + tau (u - uhat),
// which cover Poisson (beta = gamma = 0, nu = 1) and viscous Burgers. Each element is one
// workgroup: its quadrature geometry and state are staged in LDS, the state is evaluated at
// the quadrature points (the Phi/Psi products of Section 4.1 as per-point sums), the flux
// and its derivatives are formed per point, and every output entry is one sum over the
// volume or face points. q is derived from the q-equation (M q_d + B_d u + C_d uhat = 0),
// so r_q = 0.
//
// Residual rows (the sign of the trace rows as everywhere in the library), with the time
// term of an implicit stage (c = 1/(a_ii dt), u_n, r_x; c = 0 and no r_x: steady):
//   R_u[i]   = -(F, grad phi_i) + <fhat, phi_i> - (s, phi_i) + c (u - u_n, phi_i) + r_x[i]
//   R_t[l,j] = -<fhat, psi_j>_l (interior face), <uhat - u_D, psi_j>_l (Dirichlet face)
// and ru = -R_u, rt = -R_t; D..J are their derivatives with respect to q, u and uhat.
#include "hdg_batch.hpp"

namespace {

constexpr int EBS = 256;
constexpr int TJ = 4;      // output columns per work item in the (i, j) sums

// One element's inputs and outputs, every pointer already at that element (phi and psi:
// the reference tables; uhat: the face values of the element's mesh, indexed by e2f).
struct ElemView {
    const double *wdet, *dphix, *phi, *phif, *psi, *ndA, *dA, *src, *uD;
    const int32_t *bnd, *e2f;
    const double *u, *uhat, *u_prev, *r_extra;
    double *Minv, *Bd, *Cd, *D, *E, *F, *G, *H, *J, *ru, *rt, *q;
    int P, PF, L, Dm, Qv, Qf, residual_only, keep_mass, eid;
    double nu, tau, beta[3], gamma[3], c;
    int* bad;              // first element with a non-positive mass pivot
};

struct ElemArgs {
    hdg_elem_geom g;
    hdg_conv_diff m;
    const int32_t* e2f;
    const double* u;       // [ne][P]
    const double* uhat;    // [nf][PF]
    hdg_elem_arrays out;
    double c;              // implicit-stage mass factor 1/(a_ii dt); 0: steady
    const double* u_prev;  // [ne][P], read when c != 0
    const double* r_extra; // [ne][P] or null
    int* bad;
    int ne, P, PF, L, D, residual_only, keep_mass;
};

// LDS offsets (in doubles) of the element's staged arrays
struct ElemLds {
    int phi, dphi, wdet, phif, psi, ndA, dA, src, uD, u, uh, up, M, t, q, uq, duq, qq, uf, qf, uhf, wF, wFu, fhat, Z,
        total;
};

__host__ __device__ inline ElemLds elem_lds(int P, int PF, int L, int D, int Qv, int Qf) {
    ElemLds o;
    int p = 0;
    o.phi = p;  p += Qv * P;
    o.dphi = p; p += Qv * P * D;
    o.wdet = p; p += Qv;
    o.phif = p; p += L * Qf * P;
    o.psi = p;  p += Qf * PF;
    o.ndA = p;  p += L * Qf * D;
    o.dA = p;   p += L * Qf;
    o.src = p;  p += Qv;
    o.uD = p;   p += L * Qf;
    o.u = p;    p += P;
    o.uh = p;   p += L * PF;
    o.up = p;   p += P;
    o.M = p;    p += P * P;
    o.t = p;    p += D * P;
    o.q = p;    p += D * P;
    o.uq = p;   p += Qv;
    o.duq = p;  p += Qv;
    o.qq = p;   p += Qv * D;
    o.uf = p;   p += L * Qf;
    o.qf = p;   p += L * Qf * D;
    o.uhf = p;  p += L * Qf;
    o.wF = p;   p += Qv * D;
    o.wFu = p;  p += Qv * D;
    o.fhat = p; p += L * Qf;
    o.Z = p;    p += L * Qf;
    o.total = p;
    return o;
}

// v[d] for d < 3 without dynamic indexing (which would put v in scratch memory)
__device__ __forceinline__ double sel3(const double (&v)[3], int d) { return d == 0 ? v[0] : d == 1 ? v[1] : v[2]; }

__device__ __forceinline__ void element_body(const ElemView& a, double* sm) {
    const int e = a.eid;
    const int tid = threadIdx.x;
    const int P = a.P, PF = a.PF, L = a.L, D = a.Dm, Qv = a.Qv, Qf = a.Qf;
    const int nt = L * PF;
    const ElemLds o = elem_lds(P, PF, L, D, Qv, Qf);
    double *phi = sm + o.phi, *dphi = sm + o.dphi, *wdet = sm + o.wdet, *phif = sm + o.phif, *psi = sm + o.psi;
    double *ndA = sm + o.ndA, *dA = sm + o.dA, *src = sm + o.src, *uD = sm + o.uD, *u = sm + o.u, *uh = sm + o.uh;
    double *up = sm + o.up, *duq = sm + o.duq;
    double *Mm = sm + o.M, *t = sm + o.t, *q = sm + o.q, *uq = sm + o.uq, *qq = sm + o.qq, *uf = sm + o.uf;
    double *qf = sm + o.qf, *uhf = sm + o.uhf, *wF = sm + o.wF, *wFu = sm + o.wFu, *fhat = sm + o.fhat, *Z = sm + o.Z;

    // 1. stage geometry, reference tables and state
    for (int k = tid; k < Qv * P; k += EBS) phi[k] = a.phi[k];
    for (int k = tid; k < Qv * P * D; k += EBS) dphi[k] = a.dphix[k];
    for (int k = tid; k < Qv; k += EBS) {
        wdet[k] = a.wdet[k];
        src[k] = a.src[k];
    }
    for (int k = tid; k < L * Qf * P; k += EBS) phif[k] = a.phif[k];
    for (int k = tid; k < Qf * PF; k += EBS) psi[k] = a.psi[k];
    for (int k = tid; k < L * Qf * D; k += EBS) ndA[k] = a.ndA[k];
    for (int k = tid; k < L * Qf; k += EBS) {
        dA[k] = a.dA[k];
        uD[k] = a.uD[k];
    }
    const double cdt = a.c;
    for (int k = tid; k < P; k += EBS) {
        u[k] = a.u[k];
        up[k] = cdt != 0.0 ? a.u_prev[k] : 0.0;
    }
    for (int k = tid; k < nt; k += EBS) {
        const int l = k / PF, j = k - l * PF;
        uh[k] = a.uhat[(size_t)a.e2f[l] * PF + j];
    }
    __syncthreads();

    // 2. mass matrix and its inverse (Gauss-Jordan in place; M is SPD, no interchanges), or
    //    the inverse kept from an earlier evaluation on the same mesh (state-independent)
    const int nJT = (P + TJ - 1) / TJ;    // column tiles of TJ entries: one row i per work item
    if (a.keep_mass) {
        for (int k = tid; k < P * P; k += EBS) Mm[k] = a.Minv[k];
        __syncthreads();
    } else {
        for (int it = tid; it < P * nJT; it += EBS) {
            const int i = it / nJT, j0 = (it - i * nJT) * TJ;
            double acc[TJ] = {};
            for (int x = 0; x < Qv; ++x) {
                const double wi = wdet[x] * phi[x * P + i];
#pragma unroll
                for (int jj = 0; jj < TJ; ++jj)
                    if (j0 + jj < P) acc[jj] += wi * phi[x * P + j0 + jj];
            }
#pragma unroll
            for (int jj = 0; jj < TJ; ++jj)
                if (j0 + jj < P) Mm[i * P + j0 + jj] = acc[jj];
        }
        __syncthreads();
        for (int k = 0; k < P; ++k) {
            const double piv = Mm[k * P + k];
            if (!(piv > 0.0) || !isfinite(piv)) {
                if (tid == 0) atomicMin(a.bad, e);
                return;    // uniform across the workgroup: every thread read the same pivot
            }
            const double rp = 1.0 / piv;
            // row k scaled (entry k becomes 1/piv), other rows updated with the old column k
            for (int idx = tid; idx < P * P; idx += EBS) {
                const int i = idx / P, j = idx - i * P;
                if (i == k) continue;
                const double f = Mm[i * P + k] * rp;
                if (j == k) continue;
                Mm[idx] -= f * Mm[k * P + j];
            }
            __syncthreads();
            for (int idx = tid; idx < P; idx += EBS) {
                if (idx != k) {
                    Mm[idx * P + k] = -Mm[idx * P + k] * rp;
                    Mm[k * P + idx] *= rp;
                }
            }
            if (tid == 0) Mm[k * P + k] = rp;
            __syncthreads();
        }
    }

    // 3. u and uhat at the quadrature points
    for (int k = tid; k < Qv; k += EBS) {
        double s = 0.0, sp = 0.0;
        for (int i = 0; i < P; ++i) {
            s += phi[k * P + i] * u[i];
            sp += phi[k * P + i] * up[i];
        }
        uq[k] = s;
        duq[k] = s - sp;     // u - u_n at the point (time term)
    }
    for (int k = tid; k < L * Qf; k += EBS) {
        const int l = k / Qf, x = k - l * Qf;
        double s = 0.0, h = 0.0;
        for (int i = 0; i < P; ++i) s += phif[k * P + i] * u[i];
        for (int j = 0; j < PF; ++j) h += psi[x * PF + j] * uh[l * PF + j];
        uf[k] = s;
        uhf[k] = h;
    }
    __syncthreads();

    // 4. q = -M^{-1} (B_d u + C_d uhat), with B_d u and C_d uhat summed over the points
    for (int k = tid; k < D * P; k += EBS) {
        const int d = k / P, i = k - d * P;
        double s = 0.0;
        for (int x = 0; x < Qv; ++x) s += wdet[x] * dphi[(x * P + i) * D + d] * uq[x];
        for (int lx = 0; lx < L * Qf; ++lx) s -= ndA[lx * D + d] * phif[lx * P + i] * uhf[lx];
        t[k] = s;
    }
    __syncthreads();
    for (int k = tid; k < D * P; k += EBS) {
        const int d = k / P, i = k - d * P;
        double s = 0.0;
        for (int j = 0; j < P; ++j) s += Mm[i * P + j] * t[d * P + j];
        q[k] = -s;
        if (a.q) a.q[k] = -s;
    }
    __syncthreads();

    // 5. q at the points, then the flux and its derivatives per point
    for (int k = tid; k < Qv * D; k += EBS) {
        const int x = k / D, d = k - x * D;
        double s = 0.0;
        for (int i = 0; i < P; ++i) s += phi[x * P + i] * q[d * P + i];
        qq[k] = s;
    }
    for (int k = tid; k < L * Qf * D; k += EBS) {
        const int lx = k / D, d = k - lx * D;
        double s = 0.0;
        for (int i = 0; i < P; ++i) s += phif[lx * P + i] * q[d * P + i];
        qf[k] = s;
    }
    __syncthreads();
    const double nu = a.nu, tau = a.tau;
    for (int k = tid; k < Qv * D; k += EBS) {
        const int x = k / D, d = k - x * D;
        const double v = uq[x];
        const double bt = sel3(a.beta, d), gm = sel3(a.gamma, d);
        wF[k] = wdet[x] * (bt * 0.5 * v * v + gm * v - nu * qq[k]);
        wFu[k] = wdet[x] * (bt * v + gm);
    }
    for (int lx = tid; lx < L * Qf; lx += EBS) {
        const double v = uhf[lx];
        double fn = 0.0, zn = 0.0;
        for (int d = 0; d < D; ++d) {
            const double n = ndA[lx * D + d];
            const double bt = sel3(a.beta, d), gm = sel3(a.gamma, d);
            fn += (bt * 0.5 * v * v + gm * v - nu * qf[lx * D + d]) * n;
            zn += (bt * v + gm) * n;
        }
        fhat[lx] = fn + tau * (uf[lx] - v) * dA[lx];
        Z[lx] = zn - tau * dA[lx];    // d fhat / d uhat per unit trace value
    }
    __syncthreads();

    // 6. right-hand sides ru = -R_u, rt = -R_t
    for (int i = tid; i < P; i += EBS) {
        double s = 0.0;
        for (int x = 0; x < Qv; ++x) {
            double g = 0.0;
            for (int d = 0; d < D; ++d) g += wF[x * D + d] * dphi[(x * P + i) * D + d];
            s += g + wdet[x] * (src[x] - cdt * duq[x]) * phi[x * P + i];
        }
        for (int lx = 0; lx < L * Qf; ++lx) s -= fhat[lx] * phif[lx * P + i];
        if (a.r_extra) s -= a.r_extra[i];
        a.ru[i] = s;
    }
    for (int k = tid; k < nt; k += EBS) {
        const int l = k / PF, j = k - l * PF;
        const bool bd = a.bnd[l] != 0;
        double s = 0.0;
        for (int x = 0; x < Qf; ++x) {
            const int lx = l * Qf + x;
            s += (bd ? -dA[lx] * (uhf[lx] - uD[lx]) : fhat[lx]) * psi[x * PF + j];
        }
        a.rt[k] = s;
    }
    if (a.residual_only) return;

    // 7. matrices. With dF/dq = -nu I: the volume part of D is nu B_d, and G on an interior
    // face is -nu C_d^T; the (i, j) sums over volume and face points share one pass with
    // the row's per-point values held in registers.
    const bool put_mass = !a.keep_mass;      // Minv, Bd, Cd: written unless kept
    if (put_mass)
        for (int k = tid; k < P * P; k += EBS) a.Minv[k] = Mm[k];
    for (int it = tid; it < P * nJT; it += EBS) {        // Bd, D, E
        const int i = it / nJT, j0 = (it - i * nJT) * TJ;
        double bd[3][TJ] = {}, sf[3][TJ] = {}, ev[TJ] = {}, ef[TJ] = {}, mm[TJ] = {};
        for (int x = 0; x < Qv; ++x) {
            const double wp = wdet[x] * phi[x * P + i];
            double wd[3], g = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double dp = d < D ? dphi[(x * P + i) * D + d] : 0.0;
                wd[d] = wdet[x] * dp;
                g += d < D ? wFu[x * D + d] * dp : 0.0;
            }
#pragma unroll
            for (int jj = 0; jj < TJ; ++jj) {
                const double pj = j0 + jj < P ? phi[x * P + j0 + jj] : 0.0;
#pragma unroll
                for (int d = 0; d < 3; ++d) bd[d][jj] += wd[d] * pj;
                ev[jj] -= g * pj;
                mm[jj] += wp * pj;
            }
        }
        for (int lx = 0; lx < L * Qf; ++lx) {
            const double pi = phif[lx * P + i];
            double nd[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) nd[d] = d < D ? ndA[lx * D + d] * pi : 0.0;
            const double da = dA[lx] * pi;
#pragma unroll
            for (int jj = 0; jj < TJ; ++jj) {
                const double pj = j0 + jj < P ? phif[lx * P + j0 + jj] : 0.0;
#pragma unroll
                for (int d = 0; d < 3; ++d) sf[d][jj] += nd[d] * pj;
                ef[jj] += da * pj;
            }
        }
#pragma unroll
        for (int jj = 0; jj < TJ; ++jj) {
            const int j = j0 + jj;
            if (j >= P) continue;
            for (int d = 0; d < D; ++d) {
                if (put_mass) a.Bd[(size_t)(d * P + i) * P + j] = bd[d][jj];
                a.D[(size_t)i * D * P + d * P + j] = nu * (bd[d][jj] - sf[d][jj]);
            }
            a.E[(size_t)i * P + j] = ev[jj] + tau * ef[jj] + cdt * mm[jj];
        }
    }
    for (int it = tid; it < P * nt; it += EBS) {          // Cd, F, G, H for one (i, l, j)
        const int i = it / nt, c = it - i * nt, l = c / PF, j = c - l * PF;
        double cd[3] = {}, f = 0.0, h = 0.0;
        for (int x = 0; x < Qf; ++x) {
            const int lx = l * Qf + x;
            const double w = phif[lx * P + i] * psi[x * PF + j];
#pragma unroll
            for (int d = 0; d < 3; ++d) cd[d] -= d < D ? ndA[lx * D + d] * w : 0.0;
            f += Z[lx] * w;
            h += dA[lx] * w;
        }
        const bool interior = a.bnd[l] == 0;
        for (int d = 0; d < D; ++d) {
            if (put_mass) a.Cd[(size_t)(d * P + i) * nt + c] = cd[d];
            a.G[(size_t)c * D * P + d * P + i] = interior ? -nu * cd[d] : 0.0;
        }
        a.F[(size_t)i * nt + c] = f;
        a.H[(size_t)c * P + i] = interior ? -tau * h : 0.0;
    }
    for (int k = tid; k < nt * nt; k += EBS) {              // J[(l,j)][(l',j')], block diagonal in l
        const int r = k / nt, c = k - r * nt, l = r / PF, j = r - l * PF, l2 = c / PF, j2 = c - l2 * PF;
        double s = 0.0;
        if (l == l2) {
            const bool bd = a.bnd[l] != 0;
            for (int x = 0; x < Qf; ++x) {
                const int lx = l * Qf + x;
                s += (bd ? dA[lx] : -Z[lx]) * psi[x * PF + j] * psi[x * PF + j2];
            }
        }
        a.J[k] = s;
    }
}

__global__ void __launch_bounds__(EBS) k_element_blocks(ElemArgs a) {
    extern __shared__ double sm[];
    const size_t E = blockIdx.x;
    const int P = a.P, PF = a.PF, L = a.L, D = a.D, Qv = a.g.nqv, Qf = a.g.nqf, nt = L * PF;
    ElemView v;
    v.wdet = a.g.wdet + E * Qv;
    v.dphix = a.g.dphix + E * Qv * P * D;
    v.phi = a.g.phi;
    v.phif = a.g.phif + E * L * Qf * P;
    v.psi = a.g.psi;
    v.ndA = a.g.ndA + E * L * Qf * D;
    v.dA = a.g.dA + E * L * Qf;
    v.src = a.g.src + E * Qv;
    v.uD = a.g.uD + E * L * Qf;
    v.bnd = a.g.bnd + E * L;
    v.e2f = a.e2f + E * L;
    v.u = a.u + E * P;
    v.uhat = a.uhat;
    v.u_prev = a.u_prev ? a.u_prev + E * P : nullptr;
    v.r_extra = a.r_extra ? a.r_extra + E * P : nullptr;
    const bool mats = !a.residual_only;
    v.Minv = (mats || a.keep_mass) ? a.out.Minv + E * P * P : nullptr;
    v.Bd = mats ? a.out.Bd + E * D * P * P : nullptr;
    v.Cd = mats ? a.out.Cd + E * D * P * nt : nullptr;
    v.D = mats ? a.out.D + E * P * D * P : nullptr;
    v.E = mats ? a.out.E + E * P * P : nullptr;
    v.F = mats ? a.out.F + E * P * nt : nullptr;
    v.G = mats ? a.out.G + E * nt * D * P : nullptr;
    v.H = mats ? a.out.H + E * nt * P : nullptr;
    v.J = mats ? a.out.J + E * nt * nt : nullptr;
    v.ru = a.out.ru + E * P;
    v.rt = a.out.rt + E * nt;
    v.q = a.out.q ? a.out.q + E * D * P : nullptr;
    v.P = P; v.PF = PF; v.L = L; v.Dm = D; v.Qv = Qv; v.Qf = Qf;
    v.residual_only = a.residual_only;
    v.keep_mass = a.keep_mass;
    v.eid = (int)E;
    v.nu = a.m.nu; v.tau = a.m.tau; v.c = a.c;
    for (int d = 0; d < 3; ++d) { v.beta[d] = a.m.beta[d]; v.gamma[d] = a.m.gamma[d]; }
    v.bad = a.bad;
    element_body(v, sm);
}

// Batched instances: element e belongs to instance eid[e]; its arrays sit at the instance's
// offsets plus its instance-local index times the per-element sizes.
__global__ void __launch_bounds__(EBS) k_element_blocks_batch(const ElemInst* __restrict__ inst,
                                                              const int32_t* __restrict__ eid, ElemBatchArgs a) {
    extern __shared__ double sm[];
    const int64_t e = blockIdx.x;
    const ElemInst& q = inst[eid[e]];
    const int64_t E = e - q.e0;
    const int P = q.P, PF = q.PF, L = q.L, D = q.D, Qv = q.Qv, Qf = q.Qf, nt = L * PF;
    ElemView v;
    v.wdet = a.g.wdet + q.g_wdet + E * Qv;
    v.dphix = a.g.dphix + q.g_dphix + E * Qv * P * D;
    v.phi = a.g.phi + q.g_phi;
    v.phif = a.g.phif + q.g_phif + E * L * Qf * P;
    v.psi = a.g.psi + q.g_psi;
    v.ndA = a.g.ndA + q.g_ndA + E * L * Qf * D;
    v.dA = a.g.dA + q.g_dA + E * L * Qf;
    v.src = a.g.src + q.g_src + E * Qv;
    v.uD = a.g.uD + q.g_uD + E * L * Qf;
    v.bnd = a.g.bnd + q.e2f_off + E * L;
    v.e2f = a.e2f + q.e2f_off + E * L;
    v.u = a.u + q.u_off + E * P;
    v.uhat = a.uhat + q.uh_off;
    v.u_prev = (q.c != 0.0) ? a.u_prev + q.u_off + E * P : nullptr;
    v.r_extra = a.r_extra ? a.r_extra + q.u_off + E * P : nullptr;
    const bool mats = !a.residual_only;
    v.Minv = (mats || a.keep_mass) ? a.out.Minv + q.out_off[0] + E * P * P : nullptr;
    v.Bd = mats ? a.out.Bd + q.out_off[1] + E * D * P * P : nullptr;
    v.Cd = mats ? a.out.Cd + q.out_off[2] + E * D * P * nt : nullptr;
    v.D = mats ? a.out.D + q.out_off[3] + E * P * D * P : nullptr;
    v.E = mats ? a.out.E + q.out_off[4] + E * P * P : nullptr;
    v.F = mats ? a.out.F + q.out_off[5] + E * P * nt : nullptr;
    v.G = mats ? a.out.G + q.out_off[6] + E * nt * D * P : nullptr;
    v.H = mats ? a.out.H + q.out_off[7] + E * nt * P : nullptr;
    v.J = mats ? a.out.J + q.out_off[8] + E * nt * nt : nullptr;
    v.ru = a.out.ru + q.out_off[9] + E * P;
    v.rt = a.out.rt + q.out_off[10] + E * nt;
    v.q = a.out.q ? a.out.q + q.q_off + E * D * P : nullptr;
    v.P = P; v.PF = PF; v.L = L; v.Dm = D; v.Qv = Qv; v.Qf = Qf;
    v.residual_only = a.residual_only;
    v.keep_mass = a.keep_mass;
    v.eid = (int)e;
    v.nu = q.nu; v.tau = q.tau; v.c = q.c;
    for (int d = 0; d < 3; ++d) { v.beta[d] = q.beta[d]; v.gamma[d] = q.gamma[d]; }
    v.bad = a.bad;
    element_body(v, sm);
}

// ||R|| of instance blockIdx.x: its element u-rows and its faces' summed trace rows.
__global__ void __launch_bounds__(EBS) k_residual_norm_batch(const InstDesc* __restrict__ desc,
                                                             const double* __restrict__ ru,
                                                             const double* __restrict__ rt,
                                                             const int32_t* __restrict__ f2e, double* norms) {
    __shared__ double red[EBS / 64];
    const InstDesc& q = desc[blockIdx.x];
    double acc = 0.0;
    const int64_t nuu = (int64_t)q.ne * q.nu;
    for (int64_t k = threadIdx.x; k < nuu; k += EBS) {
        const double v = ru[q.off[9] + k];
        acc += v * v;
    }
    const int64_t nfe = (int64_t)q.nf * q.nb;
    for (int64_t k = threadIdx.x; k < nfe; k += EBS) {
        const int64_t f = k / q.nb;
        const int j = (int)(k - f * q.nb);
        const int32_t* fe = f2e + q.f2e_off + 4 * f;
        double v = rt[q.off[10] + (int64_t)fe[0] * q.nt + (int64_t)fe[1] * q.nb + j];
        if (fe[2] >= 0) v += rt[q.off[10] + (int64_t)fe[2] * q.nt + (int64_t)fe[3] * q.nb + j];
        acc += v * v;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < EBS / 64; ++w) s += red[w];
        norms[blockIdx.x] = sqrt(s);
    }
}

// u += alpha_i du and uhat += alpha_i x over instance i = blockIdx.x (nothing when alpha_i = 0).
__global__ void __launch_bounds__(EBS) k_newton_update_batch(const InstDesc* __restrict__ desc,
                                                             const double* __restrict__ alpha,
                                                             const double* __restrict__ du, double* u,
                                                             const double* __restrict__ x, double* uhat) {
    const InstDesc& q = desc[blockIdx.x];
    const double al = alpha[blockIdx.x];
    if (al == 0.0) return;
    const int64_t nuu = (int64_t)q.ne * q.nu, nfe = (int64_t)q.nf * q.nb;
    for (int64_t k = threadIdx.x; k < nuu; k += EBS) u[q.du_off + k] += al * du[q.du_off + k];
    for (int64_t k = threadIdx.x; k < nfe; k += EBS) uhat[q.vec_off + k] += al * x[q.vec_off + k];
}

}  // namespace

size_t element_batch_lds_bytes(int P, int PF, int L, int D, int nqv, int nqf) {
    return sizeof(double) * (size_t)elem_lds(P, PF, L, D, nqv, nqf).total;
}

hdg_status element_blocks_batch_run(hdg_ctx ctx, int64_t total_ne, const ElemInst* inst_dev, const int32_t* eid,
                                    const ElemBatchArgs& a, size_t lds) {
    if (total_ne == 0) return HDG_OK;
    hipLaunchKernelGGL(k_element_blocks_batch, dim3((unsigned)total_ne), dim3(EBS), lds, ctx->stream, inst_dev, eid, a);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status residual_norm_batch_run(hdg_ctx ctx, int n_inst, const InstDesc* desc, const double* ru, const double* rt,
                                   const int32_t* f2e, double* norms) {
    if (n_inst == 0) return HDG_OK;
    hipLaunchKernelGGL(k_residual_norm_batch, dim3(n_inst), dim3(EBS), 0, ctx->stream, desc, ru, rt, f2e, norms);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status newton_update_batch_run(hdg_ctx ctx, int n_inst, const InstDesc* desc, const double* alpha,
                                   const double* du, double* u, const double* x, double* uhat) {
    if (n_inst == 0) return HDG_OK;
    hipLaunchKernelGGL(k_newton_update_batch, dim3(n_inst), dim3(EBS), 0, ctx->stream, desc, alpha, du, u, x, uhat);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

size_t element_blocks_lds_bytes(const hdg_dims* d, int nqv, int nqf) {
    const ElemLds o = elem_lds(d->npe, d->npf, d->nlfe, d->dim, nqv, nqf);
    return sizeof(double) * (size_t)o.total;
}

hdg_status element_blocks_run(hdg_ctx ctx, const hdg_dims* d, const hdg_elem_geom* g, const hdg_conv_diff* m,
                              const hdg_time_term* tt, const int32_t* e2f, const double* u, const double* uhat,
                              int flags, const hdg_elem_arrays* out, int* bad) {
    if (d->ne == 0) return HDG_OK;
    ElemArgs a;
    a.g = *g;
    a.m = *m;
    a.e2f = e2f;
    a.u = u;
    a.uhat = uhat;
    a.out = *out;
    a.c = tt ? tt->c : 0.0;
    a.u_prev = tt ? tt->u_prev : nullptr;
    a.r_extra = tt ? tt->r_extra : nullptr;
    a.bad = bad;
    a.ne = d->ne;
    a.P = d->npe;
    a.PF = d->npf;
    a.L = d->nlfe;
    a.D = d->dim;
    a.residual_only = (flags & HDG_ELEM_RESIDUAL_ONLY) != 0;
    a.keep_mass = (flags & HDG_ELEM_KEEP_MASS) != 0;
    const size_t lds = element_blocks_lds_bytes(d, g->nqv, g->nqf);
    hipLaunchKernelGGL(k_element_blocks, dim3(d->ne), dim3(EBS), lds, ctx->stream, a);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}
