// Batched static condensation (Section 4.1 eq. w15-w19, Section 4.2 eq. w21-w22).
//
// For each element the kernels build the (nu+nt) x (nu+nt+1) matrix
//     T = [[E F r_u], [H J r_t]] - [D; G] A^{-1} [B C 0]
//       = [[Ebar Fbar r_u], [Hbar Jbar r_t]]                       (q eliminated, r_q = 0)
// and then eliminate its first nu columns by Gaussian elimination with partial
// pivoting restricted to the Ebar rows. Afterwards the bottom-right block is
//     Kbar = Jbar - Hbar Ebar^{-1} Fbar   and the last column  rbar = r_t - Hbar Ebar^{-1} r_u,
// while the top rows hold [U | L^{-1}P Fbar | L^{-1}P r_u], which recovery uses.
//
// A^{-1} = I_{MD} (x) M^{-1} and B, C are component-diagonal (eq. w16), so
// [D;G] A^{-1} [B C] restricted to the columns of component m is
//     sum_d [D;G][:, q(m,d,:)] (M^{-1} [B_d | C_d]):
// one (nu+nt) x (D P_E) by (D P_E) x (P_E + N_lfe P_F) product per component,
// with W = M^{-1}[B_d | C_d] formed first. All products run on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64, 32x32 tiles per wave). The elimination is
// right-looking and blocked: the panel (NB columns, up to 64) is factorised in
// LDS, the panel rows of the trailing columns are solved with L11 and written
// back, and the trailing matrix is updated with MFMA from the LDS-resident L21
// and the just-written U12 rows (L2-resident).
//
// Storage of T per element: the top nu rows live directly in the caller's
// `local` buffer (row stride nu+nt+1), the bottom nt rows in a workspace.
#include <cmath>

#include "hdg_internal.hpp"

namespace {

constexpr int BS = 256;

struct CondDims {
    int M, D, P, PF, L;
    int nu, nq, nt, R, C, NW, KD;
};

// acc[bi][bj][q] holds row 16*bi + 4*q + lane/16, column 16*bj + lane%16 of a 32x32 tile
// (v_mfma_f64_16x16x4f64: A[i][k] in lane i+16k, B[k][j] in lane j+16k, D[i][j] in lane
// j+16*(i%4), register i/4).
//
// acc += A(32 x K) B(K x 32). k is taken in groups of 16: instruction s (0..3) of a
// group gives lane (i, kq) the pair A[i][kb+4kq+s], B[kb+4kq+s][j], so the four
// instructions together cover all 16 k of the group and each lane reads four
// consecutive k of its A row. The next group's operands are loaded while the current
// group's 16 MFMAs run (two register buffers). la/lb return 0 outside the matrices.
template <class LA, class LB>
__device__ __forceinline__ void mfma_32x32(const LA& la, const LB& lb, int K, double4_t (&acc)[2][2]) {
    const int lane = threadIdx.x & 63;
    const int i16 = lane & 15, kq = lane >> 4;
    double a0[4][2], b0[4][2], a1[4][2], b1[4][2];
    auto fetch = [&](double (&fa)[4][2], double (&fb)[4][2], int kb) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = kb + 4 * kq + s;
            fa[s][0] = la(i16, k);
            fa[s][1] = la(16 + i16, k);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = kb + 4 * kq + s;
            fb[s][0] = lb(k, i16);
            fb[s][1] = lb(k, 16 + i16);
        }
    };
    auto mma = [&](const double (&fa)[4][2], const double (&fb)[4][2]) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][0], fb[s][0], acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][0], fb[s][1], acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][1], fb[s][0], acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][1], fb[s][1], acc[1][1], 0, 0, 0);
        }
    };
    // (loads past K are harmless: la/lb read a clamped address and return 0)
    fetch(a0, b0, 0);
    for (int kb = 0; kb < K; kb += 32) {
        fetch(a1, b1, kb + 16);
        __builtin_amdgcn_sched_barrier(0);
        mma(a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        if (kb + 16 >= K) break;
        fetch(a0, b0, kb + 32);
        __builtin_amdgcn_sched_barrier(0);
        mma(a1, b1);
        __builtin_amdgcn_sched_barrier(0);
    }
}

__device__ __forceinline__ void acc_zero(double4_t (&acc)[2][2]) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = double4_t{0.0, 0.0, 0.0, 0.0};
}

// ---- W = M^{-1} [B_d | C_d]  per (element, d):  (P x P) (P x NW) -----------------------
__global__ __launch_bounds__(BS) void k_cond_w(CondDims cd, const double* __restrict__ Minv,
                                               const double* __restrict__ Bd, const double* __restrict__ Cd,
                                               double* __restrict__ W) {
    const long long e = blockIdx.x;
    const int d = blockIdx.y;
    const int P = cd.P, NW = cd.NW, LPF = cd.L * cd.PF;
    const double* Mi = Minv + (size_t)e * P * P;
    const double* B = Bd + ((size_t)e * cd.D + d) * P * P;
    const double* Cm = Cd + ((size_t)e * cd.D + d) * P * LPF;
    double* Wo = W + (size_t)e * cd.KD * NW + (size_t)d * P * NW;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tr = (P + 31) / 32, tc = (NW + 31) / 32;
    for (int tile = wave; tile < tr * tc; tile += BS / 64) {
        const int r0 = (tile / tc) * 32, c0 = (tile % tc) * 32;
        double4_t acc[2][2];
        acc_zero(acc);
        // operand reads are unconditional (clamped to a valid address) and masked after,
        // so a whole group of loads is issued without branches
        auto la = [&](int i, int k) -> double {
            const int r = r0 + i;
            const bool ok = r < P && k < P;
            const double v = Mi[ok ? (size_t)r * P + k : 0];
            return ok ? v : 0.0;
        };
        auto lb = [&](int k, int j) -> double {
            const int c = c0 + j;
            const bool ok = k < P && c < NW;
            const double* src = c < P ? B + (size_t)k * P + c : Cm + (size_t)k * LPF + (c - P);
            const double v = *(ok ? src : B);
            return ok ? v : 0.0;
        };
        mfma_32x32(la, lb, P, acc);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = r0 + 16 * bi + 4 * q + (lane >> 4);
                    const int c = c0 + 16 * bj + (lane & 15);
                    if (r < P && c < NW) Wo[(size_t)r * NW + c] = acc[bi][bj][q];
                }
    }
}

// Column of T for column c of W (component m): u columns of m, then m's part of each
// element-trace block l.
__device__ __forceinline__ int qelim_col(int c, int m, int P, int PF, int M, int nu) {
    if (c < P) return m * P + c;
    const int cc = c - P, l = cc / PF, j = cc - l * PF;
    return nu + (l * M + m) * PF + j;
}

// ---- T = T0 - [D;G][:, q(m,:,:)] W   per (element, component m) ----------------------------
__global__ __launch_bounds__(BS) void k_cond_qelim(CondDims cd, const double* __restrict__ Dm,
                                                   const double* __restrict__ Em, const double* __restrict__ Fm,
                                                   const double* __restrict__ Gm, const double* __restrict__ Hm,
                                                   const double* __restrict__ Jm, const double* __restrict__ ru,
                                                   const double* __restrict__ rt, const double* __restrict__ W,
                                                   double* __restrict__ top, double* __restrict__ bot) {
    const long long e = blockIdx.x;
    const int m = blockIdx.y;
    const int nu = cd.nu, nt = cd.nt, nq = cd.nq, R = cd.R, C = cd.C, NW = cd.NW, KD = cd.KD;
    const int P = cd.P, PF = cd.PF, M = cd.M;
    const double* De = Dm + (size_t)e * nu * nq + (size_t)m * KD;
    const double* Ge = Gm + (size_t)e * nt * nq + (size_t)m * KD;
    const double* We = W + (size_t)e * KD * NW;
    double* Te = top + (size_t)e * nu * C;
    double* Be = bot + (size_t)e * nt * C;
    const double* Ee = Em + (size_t)e * nu * nu;
    const double* Fe = Fm + (size_t)e * nu * nt;
    const double* He = Hm + (size_t)e * nt * nu;
    const double* Je = Jm + (size_t)e * nt * nt;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tr = (R + 31) / 32, tc = (NW + 31) / 32;
    for (int tile = wave; tile < tr * tc; tile += BS / 64) {
        const int r0 = (tile / tc) * 32, c0 = (tile % tc) * 32;
        double4_t acc[2][2];
        acc_zero(acc);
        auto la = [&](int i, int k) -> double {
            const int r = r0 + i;
            const bool ok = r < R && k < KD;
            const double* src = r < nu ? De + (size_t)r * nq + k : Ge + (size_t)(r - nu) * nq + k;
            const double v = *(ok ? src : De);
            return ok ? v : 0.0;
        };
        auto lb = [&](int k, int j) -> double {
            const int c = c0 + j;
            const bool ok = k < KD && c < NW;
            const double v = We[ok ? (size_t)k * NW + c : 0];
            return ok ? v : 0.0;
        };
        // T0 entries of this tile, loaded before the product (in flight during it)
        double t0[2][2][4];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = r0 + 16 * bi + 4 * q + (lane >> 4);
                    const int c = c0 + 16 * bj + (lane & 15);
                    const bool ok = r < R && c < NW;
                    const int tcol = qelim_col(c, m, P, PF, M, nu);
                    const double* src = r < nu ? (tcol < nu ? Ee + (size_t)r * nu + tcol : Fe + (size_t)r * nt + (tcol - nu))
                                               : (tcol < nu ? He + (size_t)(r - nu) * nu + tcol
                                                            : Je + (size_t)(r - nu) * nt + (tcol - nu));
                    t0[bi][bj][q] = *(ok ? src : Ee);
                }
        mfma_32x32(la, lb, KD, acc);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = r0 + 16 * bi + 4 * q + (lane >> 4);
                    const int c = c0 + 16 * bj + (lane & 15);
                    if (r >= R || c >= NW) continue;
                    const int tcol = qelim_col(c, m, P, PF, M, nu);
                    const double v = t0[bi][bj][q] - acc[bi][bj][q];
                    if (r < nu) Te[(size_t)r * C + tcol] = v;
                    else Be[(size_t)(r - nu) * C + tcol] = v;
                }
    }
    if (m == 0) {
        for (int r = threadIdx.x; r < R; r += BS) {
            if (r < nu) Te[(size_t)r * C + (C - 1)] = ru[(size_t)e * nu + r];
            else Be[(size_t)(r - nu) * C + (C - 1)] = rt[(size_t)e * nt + (r - nu)];
        }
    }
}

// ---- blocked elimination of the first nu columns ----------------------------------------------
// NBT: compile-time bound of the panel width (the triangular solve keeps one
// column of U12 in registers). LBS threads share the LDS panel (512 for panels of
// up to 32 columns, so eight waves hide the trailing update's memory latency).
// Dynamic LDS: the R x (NB+1) panel, then nu + 2*NBT ints for the row interchanges.
template <int NBT, int LBS>
__global__ __launch_bounds__(LBS) void k_cond_lu(CondDims cd, int NB, double* __restrict__ top,
                                                 double* __restrict__ bot, int* bad_elem, int e_off) {
    extern __shared__ double sm[];
    __shared__ double pval;
    __shared__ int pidx;
    __shared__ int ndisp;
    const long long e = blockIdx.x;
    const int nu = cd.nu, R = cd.R, C = cd.C;
    double* Te = top + (size_t)e * nu * C;
    double* Be = bot + (size_t)e * cd.nt * C;
    auto rowp = [&](int r) -> double* { return r < nu ? Te + (size_t)r * C : Be + (size_t)(r - nu) * C; };
    const int ldp = NB + 1;
    double* Pn = sm;                                   // R x ldp (panel; L21 stays here)
    int* rsrc = (int*)(sm + (size_t)R * ldp);          // [nu]: row interchanges of the panel
    int* dsrc = rsrc + nu;                             // [NBT]: displaced rows (source)
    int* ddst = dsrc + NBT;                            // [NBT]: displaced rows (destination)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    bool singular = false;
    for (int k0 = 0; k0 < nu; k0 += NB) {
        const int nbk = (nu - k0) < NB ? (nu - k0) : NB;
        const int nrow = R - k0;
        // 1. load the panel (four loads in flight per thread)
        for (int base = threadIdx.x; base < nrow * nbk; base += 4 * LBS) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = base + u * LBS;
                const int li = idx / nbk, kk = idx - li * nbk;
                v[u] = idx < nrow * nbk ? rowp(k0 + li)[k0 + kk] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = base + u * LBS;
                const int li = idx / nbk, kk = idx - li * nbk;
                if (idx < nrow * nbk) Pn[li * ldp + kk] = v[u];
            }
        }
        for (int r = threadIdx.x; r < nu - k0; r += LBS) rsrc[r] = r;
        if (threadIdx.x == 0) ndisp = 0;
        __syncthreads();
        // 2. factorise the panel (pivot rows restricted to the Ebar rows)
        for (int kk = 0; kk < nbk; ++kk) {
            if (wave == 0) {
                double best = -1.0;
                int bi = kk;
                for (int li = kk + lane; li < nu - k0; li += 64) {
                    const double v = fabs(Pn[li * ldp + kk]);
                    if (v > best || (v == best && li < bi)) { best = v; bi = li; }
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    const double ob = __shfl_xor(best, off, 64);
                    const int oi = __shfl_xor(bi, off, 64);
                    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
                }
                if (lane == 0) {
                    pidx = bi;
                    pval = Pn[bi * ldp + kk];
                    const int t = rsrc[kk];
                    rsrc[kk] = rsrc[bi];
                    rsrc[bi] = t;
                }
            }
            __syncthreads();
            const int p = pidx;
            double pv = pval;
            if (!(fabs(pv) > 0.0) || !isfinite(pv)) { singular = true; pv = 1.0; }
            if (p != kk) {
                for (int c = threadIdx.x; c < nbk; c += LBS) {
                    const double t = Pn[kk * ldp + c];
                    Pn[kk * ldp + c] = Pn[p * ldp + c];
                    Pn[p * ldp + c] = t;
                }
            }
            __syncthreads();
            const double inv = 1.0 / pv;
            for (int li = kk + 1 + threadIdx.x; li < nrow; li += LBS) {
                const double mlt = Pn[li * ldp + kk] * inv;
                Pn[li * ldp + kk] = mlt;
                for (int c = kk + 1; c < nbk; ++c) Pn[li * ldp + c] -= mlt * Pn[kk * ldp + c];
            }
            __syncthreads();
        }
        // rows at or below nbk whose content moved (at most nbk of them); the order of
        // the list does not matter, each destination appears once
        for (int r = nbk + threadIdx.x; r < nu - k0; r += LBS) {
            if (rsrc[r] != r) {
                const int q = atomicAdd(&ndisp, 1);
                dsrc[q] = rsrc[r];
                ddst[q] = r;
            }
        }
        // 3. the panel's U11 rows back to T (rows k0..k0+nbk-1 are final)
        for (int idx = threadIdx.x; idx < nbk * nbk; idx += LBS) {
            const int li = idx / nbk, kk = idx - li * nbk;
            rowp(k0 + li)[k0 + kk] = Pn[li * ldp + kk];
        }
        __syncthreads();
        // 4. row interchanges and U12 = L11^{-1} A12 on the trailing columns (one thread
        //    per column): every load of the column is issued before its first store
        const int cbeg = k0 + nbk;
        const int ncol = C - cbeg;
        const int nd = ndisp;
        for (int cl = threadIdx.x; cl < ncol; cl += LBS) {
            const int col = cbeg + cl;
            double u[NBT], dv[NBT];
#pragma unroll
            for (int t = 0; t < NBT; ++t) u[t] = t < nbk ? rowp(k0 + rsrc[t])[col] : 0.0;
#pragma unroll
            for (int q = 0; q < NBT; ++q) dv[q] = q < nd ? rowp(k0 + dsrc[q])[col] : 0.0;
#pragma unroll
            for (int q = 0; q < NBT; ++q)
                if (q < nd) rowp(k0 + ddst[q])[col] = dv[q];
            // forward substitution with the unit lower L11
#pragma unroll
            for (int kk = 1; kk < NBT; ++kk) {
                if (kk < nbk) {
                    double v = u[kk];
#pragma unroll
                    for (int q = 0; q < kk; ++q) v -= Pn[kk * ldp + q] * u[q];
                    u[kk] = v;
                }
            }
#pragma unroll
            for (int t = 0; t < NBT; ++t)
                if (t < nbk) rowp(k0 + t)[col] = u[t];
        }
        __syncthreads();
        // 5. trailing update T22 -= L21 U12 (MFMA, 32x32 tiles per wave)
        const int nrow2 = R - cbeg;
        const int tr = (nrow2 + 31) / 32, tc = (ncol + 31) / 32;
        for (int tile = wave; tile < tr * tc; tile += LBS / 64) {
            const int r0 = (tile / tc) * 32, c0 = (tile % tc) * 32;
            double4_t acc[2][2];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int r = r0 + 16 * bi + 4 * q + (lane >> 4);
                        const int c = c0 + 16 * bj + (lane & 15);
                        const bool ok = r < nrow2 && c < ncol;
                        const double v = rowp(cbeg + (ok ? r : 0))[ok ? cbeg + c : cbeg];
                        acc[bi][bj][q] = ok ? v : 0.0;
                    }
            auto la = [&](int i, int k) -> double {
                const int r = r0 + i;
                const bool ok = r < nrow2 && k < nbk;
                const double v = Pn[ok ? (nbk + r) * ldp + k : 0];
                return ok ? -v : 0.0;
            };
            auto lb = [&](int k, int j) -> double {
                const int c = c0 + j;
                const bool ok = k < nbk && c < ncol;
                const double v = rowp(k0 + (ok ? k : 0))[ok ? cbeg + c : cbeg];
                return ok ? v : 0.0;
            };
            mfma_32x32(la, lb, nbk, acc);
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int r = r0 + 16 * bi + 4 * q + (lane >> 4);
                        const int c = c0 + 16 * bj + (lane & 15);
                        if (r < nrow2 && c < ncol) rowp(cbeg + r)[cbeg + c] = acc[bi][bj][q];
                    }
        }
        __syncthreads();
    }
    if (singular && threadIdx.x == 0) atomicMin(bad_elem, e_off + (int)e);
}

__global__ __launch_bounds__(BS) void k_cond_copyout(CondDims cd, const double* __restrict__ bot,
                                                     double* __restrict__ Kbar, double* __restrict__ rbar) {
    const long long e = blockIdx.x;
    const int nt = cd.nt, nu = cd.nu, C = cd.C;
    const double* Be = bot + (size_t)e * nt * C;
    for (int idx = threadIdx.x; idx < nt * nt; idx += BS) {
        const int i = idx / nt, j = idx - i * nt;
        Kbar[(size_t)e * nt * nt + idx] = Be[(size_t)i * C + nu + j];
    }
    for (int i = threadIdx.x; i < nt; i += BS) rbar[(size_t)e * nt + i] = Be[(size_t)i * C + C - 1];
}

size_t lu_lds_bytes(const CondDims& cd, int NB) {
    return sizeof(double) * (size_t)cd.R * (NB + 1) + sizeof(int) * ((size_t)cd.nu + 2 * 64);
}

}  // namespace

hdg_status condense_run(hdg_ctx ctx, const hdg_dims* d, int64_t ne, const hdg_elem_blocks* in, double* Kbar,
                        double* rbar, double* local) {
    CondDims cd;
    cd.M = d->ncomp; cd.D = d->dim; cd.P = d->npe; cd.PF = d->npf; cd.L = d->nlfe;
    cd.nu = cd.M * cd.P; cd.nq = cd.M * cd.D * cd.P; cd.nt = cd.L * cd.M * cd.PF;
    cd.R = cd.nu + cd.nt; cd.C = cd.R + 1; cd.NW = cd.P + cd.L * cd.PF; cd.KD = cd.D * cd.P;
    if (ne <= 0) return HDG_OK;
    // panel width: the whole Ebar when it fits in LDS, else 32 or 16 columns
    const size_t lds_cap = 150 * 1024;
    int NB = 0;
    const int cands[4] = {cd.nu, 32, 16, 8};
    for (int k = 0; k < 4; ++k) {
        const int nb = cands[k] < cd.nu ? cands[k] : cd.nu;
        if (nb <= 64 && lu_lds_bytes(cd, nb) <= lds_cap) { NB = nb; break; }
    }
    if (NB == 0) {
        ctx->err = "condensation: element too large for the LDS-blocked elimination";
        return HDG_ERR_SHAPE;
    }
    // chunk elements so the workspace stays bounded (about 4 GiB)
    const size_t per_elem = sizeof(double) * ((size_t)cd.nt * cd.C + (size_t)cd.KD * cd.NW);
    int64_t chunk = (int64_t)((size_t)4 << 30) / (int64_t)per_elem;
    if (chunk < 1) chunk = 1;
    if (chunk > ne) chunk = ne;
    hdg_status st;
    double* bot = (double*)ws_get(ctx, WS_T_BOTTOM, sizeof(double) * (size_t)chunk * cd.nt * cd.C, &st);
    if (!bot) return st;
    double* W = (double*)ws_get(ctx, WS_W, sizeof(double) * (size_t)chunk * cd.KD * cd.NW, &st);
    if (!W) return st;
    int* status = (int*)ws_get(ctx, WS_STATUS, 64, &st);
    if (!status) return st;
    const int big = 0x7fffffff;
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(status, &big, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    const size_t lds = lu_lds_bytes(cd, NB);
    const void* lu_fn = NB <= 16 ? (const void*)k_cond_lu<16, 512> : NB <= 32 ? (const void*)k_cond_lu<32, 512>
                                                                               : (const void*)k_cond_lu<64, 256>;
    if (lds > 64 * 1024)
        HDG_HIP_CHECK(ctx, hipFuncSetAttribute(lu_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    for (int64_t e0 = 0; e0 < ne; e0 += chunk) {
        const int64_t n = (ne - e0) < chunk ? (ne - e0) : chunk;
        const size_t P = cd.P, LPF = (size_t)cd.L * cd.PF;
        hipLaunchKernelGGL(k_cond_w, dim3((unsigned)n, cd.D), dim3(BS), 0, ctx->stream, cd, in->Minv + e0 * P * P,
                           in->Bd + e0 * cd.D * P * P, in->Cd + e0 * cd.D * P * LPF, W);
        HDG_LAUNCH_CHECK(ctx);
        hipLaunchKernelGGL(k_cond_qelim, dim3((unsigned)n, cd.M), dim3(BS), 0, ctx->stream, cd,
                           in->D + e0 * cd.nu * cd.nq, in->E + e0 * cd.nu * cd.nu, in->F + e0 * cd.nu * cd.nt,
                           in->G + e0 * cd.nt * cd.nq, in->H + e0 * cd.nt * cd.nu, in->J + e0 * cd.nt * cd.nt,
                           in->ru + e0 * cd.nu, in->rt + e0 * cd.nt, W, local + e0 * cd.nu * cd.C, bot);
        HDG_LAUNCH_CHECK(ctx);
        if (NB <= 16)
            hipLaunchKernelGGL((k_cond_lu<16, 512>), dim3((unsigned)n), dim3(512), lds, ctx->stream, cd, NB,
                               local + e0 * cd.nu * cd.C, bot, status, (int)e0);
        else if (NB <= 32)
            hipLaunchKernelGGL((k_cond_lu<32, 512>), dim3((unsigned)n), dim3(512), lds, ctx->stream, cd, NB,
                               local + e0 * cd.nu * cd.C, bot, status, (int)e0);
        else
            hipLaunchKernelGGL((k_cond_lu<64, 256>), dim3((unsigned)n), dim3(256), lds, ctx->stream, cd, NB,
                               local + e0 * cd.nu * cd.C, bot, status, (int)e0);
        HDG_LAUNCH_CHECK(ctx);
        hipLaunchKernelGGL(k_cond_copyout, dim3((unsigned)n), dim3(BS), 0, ctx->stream, cd, bot,
                           Kbar + e0 * cd.nt * cd.nt, rbar + e0 * cd.nt);
        HDG_LAUNCH_CHECK(ctx);
    }
    int bad = big;
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(&bad, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HDG_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    if (bad != big) {
        ctx->err = "condensation: zero or non-finite pivot in Ebar of element " + std::to_string(bad);
        return HDG_ERR_SINGULAR;
    }
    return HDG_OK;
}
