// Local recovery (Section 2.3 recovery equation; Section 4.1 eq. w19 and eq. w16),
// one workgroup per element:
//   du = Ebar^{-1}(r_u - Fbar uhat) = U^{-1}(c - Y uhat)   with the factorised rows
//        [U | Y | c] = [U | L^{-1}P Fbar | L^{-1}P r_u] left by the condensation,
//   dq_{m,d} = -M^{-1}(B_d du_m + C_d uhat_m).
// Also the Newton update state += alpha * delta (Section 2.3).
//
// The back substitution runs in diagonal blocks of RB rows from the bottom: the rows of a
// block first take the already solved unknowns below it (a row-block product, all waves),
// then one wave solves the RB x RB triangle with the block's unknowns in registers.
#include "hdg_internal.hpp"

namespace {

constexpr int BS = 256;
constexpr int RB = 64;      // rows of a diagonal block of U (one per lane)
constexpr int MMAX = 8;     // components handled together in the q part

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Sum over the wave, the same value in every lane: within each row of 16 lanes the
// partners come through DPP (xor 1, xor 2, half-row and row mirrors), then the four row
// sums are added in a fixed order.
__device__ __forceinline__ double wave_sum_all(double v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// res[r] = sum_{k<n} A[(i0+r)*lda + k] v[k] for r < nr (nr <= 4), v in LDS; the loads of
// the four rows are issued together (row and column indices clamped to valid entries).
__device__ __forceinline__ void rows_dot4(const double* __restrict__ A, int lda, int i0, int nr,
                                          const double* v, int n, double (&res)[4]) {
    const int lane = threadIdx.x & 63;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < n; k0 += 64) {
        const int k = k0 + lane;
        const bool ok = k < n;
        const int kc = ok ? k : 0;
        double a[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = A[(size_t)(i0 + (r < nr ? r : 0)) * lda + kc];
        const double xv = v[kc];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] += ok ? a[r] * xv : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) res[r] = wave_sum_all(acc[r]);
}

__global__ __launch_bounds__(BS) void k_recover(int ne, int M, int D, int P, int PF, int L,
                                                const double* __restrict__ local, const double* __restrict__ Minv,
                                                const double* __restrict__ Bd, const double* __restrict__ Cd,
                                                const int32_t* __restrict__ e2f, const int32_t* __restrict__ perm,
                                                const double* __restrict__ xhat, double* __restrict__ du,
                                                double* __restrict__ dq) {
    extern __shared__ double sm[];
    const int nu = M * P, nb = M * PF, nt = L * nb, C = nu + nt + 1, LPF = L * PF;
    const long long e = blockIdx.x;
    if (e >= ne) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    constexpr int NW = BS / 64;
    double* xe = sm;                   // nt: the element's trace values, in local order
    double* t = xe + nt;               // nu: right-hand side, then du
    double* Ub = t + nu;               // RB x (RB+1): a diagonal block of U
    double* sq = Ub + RB * (RB + 1);   // NW x M x P: per-wave products of the q part
    for (int idx = threadIdx.x; idx < nt; idx += BS) {
        const int l = idx / nb, rem = idx - l * nb, m = rem / PF, j = rem - m * PF;
        const int jl = perm ? perm[((size_t)e * L + l) * PF + j] : j;
        xe[(l * M + m) * PF + jl] = xhat[(size_t)e2f[(size_t)e * L + l] * nb + rem];
    }
    __syncthreads();
    const double* Le = local + (size_t)e * nu * C;
    // t = c - Y xe, four rows per wave at a time
    for (int i0 = 4 * wave; i0 < nu; i0 += 4 * NW) {
        const int nr = nu - i0 < 4 ? nu - i0 : 4;
        double res[4];
        rows_dot4(Le + nu, C, i0, nr, xe, nt, res);
        if (lane < nr) {
            double rr = res[0];
#pragma unroll
            for (int r = 1; r < 4; ++r) rr = lane == r ? res[r] : rr;
            t[i0 + lane] = Le[(size_t)(i0 + lane) * C + nu + nt] - rr;
        }
    }
    __syncthreads();
    // U du = t, diagonal blocks of RB rows from the bottom; rows above 0 in the top block
    // are padding (identity rows that take nothing from the rows below)
    for (int top = nu; top > 0; top -= RB) {
        const int base = top - RB;
        const int lo = base > 0 ? base : 0;
        if (top < nu) {
            for (int i0 = lo + 4 * wave; i0 < top; i0 += 4 * NW) {
                const int nr = top - i0 < 4 ? top - i0 : 4;
                double res[4];
                rows_dot4(Le + top, C, i0, nr, t + top, nu - top, res);
                if (lane < nr) {
                    double rr = res[0];
#pragma unroll
                    for (int r = 1; r < 4; ++r) rr = lane == r ? res[r] : rr;
                    t[i0 + lane] -= rr;
                }
            }
        }
        for (int idx = threadIdx.x; idx < RB * RB; idx += BS) {
            const int r = idx / RB, c = idx - r * RB;
            const int gr = base + r, gc = base + c;
            Ub[r * (RB + 1) + c] = (gr >= 0 && gc >= 0) ? Le[(size_t)gr * C + gc] : (r == c ? 1.0 : 0.0);
        }
        __syncthreads();
        if (wave == 0) {
            const int g = base + lane;
            double x = g >= 0 ? t[g] : 0.0;
            double ub[RB];                       // column `lane` of the block
#pragma unroll
            for (int i = 0; i < RB; ++i) ub[i] = Ub[i * (RB + 1) + lane];
#pragma unroll
            for (int i = RB - 1; i >= 0; --i) {
                const double s = wave_sum_all(lane > i ? ub[i] * x : 0.0);
                const double xi = (read_lane(x, i) - s) / read_lane(ub[i], i);
                x = lane == i ? xi : x;
            }
            if (g >= 0) t[g] = x;
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < nu; i += BS) du[(size_t)e * nu + i] = t[i];
    // dq_{m,d} = -Minv (B_d du_m + C_d uhat_m): one d per wave, all components together
    // (B_d, C_d and Minv are read once per d)
    const double* Mi = Minv + (size_t)e * P * P;
    double* s = sq + (size_t)wave * M * P;
    for (int d = wave; d < D; d += NW) {
        const double* B = Bd + ((size_t)e * D + d) * P * P;
        const double* Cm = Cd + ((size_t)e * D + d) * P * LPF;
        for (int m0 = 0; m0 < M; m0 += MMAX) {
            const int mc = M - m0 < MMAX ? M - m0 : MMAX;
            for (int i = lane; i < P; i += 64) {
                double acc[MMAX];
#pragma unroll
                for (int q = 0; q < MMAX; ++q) acc[q] = 0.0;
                for (int j = 0; j < P; ++j) {
                    const double bij = B[(size_t)i * P + j];
#pragma unroll
                    for (int q = 0; q < MMAX; ++q)
                        if (q < mc) acc[q] += bij * t[(m0 + q) * P + j];
                }
                for (int l = 0; l < L; ++l)
                    for (int j = 0; j < PF; ++j) {
                        const double cij = Cm[(size_t)i * LPF + l * PF + j];
#pragma unroll
                        for (int q = 0; q < MMAX; ++q)
                            if (q < mc) acc[q] += cij * xe[(l * M + m0 + q) * PF + j];
                    }
#pragma unroll
                for (int q = 0; q < MMAX; ++q)
                    if (q < mc) s[q * P + i] = acc[q];
            }
            __builtin_amdgcn_wave_barrier();
            for (int i = lane; i < P; i += 64) {
                double acc[MMAX];
#pragma unroll
                for (int q = 0; q < MMAX; ++q) acc[q] = 0.0;
                for (int k = 0; k < P; ++k) {
                    const double mik = Mi[(size_t)i * P + k];
#pragma unroll
                    for (int q = 0; q < MMAX; ++q)
                        if (q < mc) acc[q] += mik * s[q * P + k];
                }
#pragma unroll
                for (int q = 0; q < MMAX; ++q)
                    if (q < mc) dq[(size_t)e * M * D * P + (size_t)((m0 + q) * D + d) * P + i] = -acc[q];
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

__global__ __launch_bounds__(BS) void k_axpy(int64_t n, double alpha, const double* __restrict__ x, double* y) {
    const int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (k < n) y[k] += alpha * x[k];
}

}  // namespace

hdg_status recover_run(hdg_ctx ctx, const hdg_dims* d, const double* local, const double* Minv, const double* Bd,
                       const double* Cd, const int32_t* e2f, const int32_t* perm, const double* xhat, double* du,
                       double* dq) {
    if (d->ne == 0) return HDG_OK;
    const int nu = d->ncomp * d->npe, nt = d->nlfe * d->ncomp * d->npf;
    const size_t lds = sizeof(double) * ((size_t)nt + nu + RB * (RB + 1) + (size_t)(BS / 64) * nu);
    if (lds > 64 * 1024)
        HDG_HIP_CHECK(ctx, hipFuncSetAttribute((const void*)k_recover, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds));
    hipLaunchKernelGGL(k_recover, dim3(d->ne), dim3(BS), lds, ctx->stream, d->ne, d->ncomp, d->dim, d->npe, d->npf,
                       d->nlfe, local, Minv, Bd, Cd, e2f, perm, xhat, du, dq);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status axpy_run(hdg_ctx ctx, int64_t n, double alpha, const double* x, double* y) {
    if (n == 0) return HDG_OK;
    hipLaunchKernelGGL(k_axpy, dim3(div_up(n, BS)), dim3(BS), 0, ctx->stream, n, alpha, x, y);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}
