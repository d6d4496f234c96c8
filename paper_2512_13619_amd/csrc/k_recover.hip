// Local recovery (Section 2.3 recovery equation; Section 4.1 eq. w19 and eq. w16),
// one workgroup per element:
//   du = Ebar^{-1}(r_u - Fbar uhat) = x_r - X uhat   with the rows [U | X | x_r] =
//        [U | Ebar^{-1} Fbar | Ebar^{-1} r_u] left by the condensation,
//   dq_{m,d} = -M^{-1}(B_d du_m + C_d uhat_m).
// Also the Newton update state += alpha * delta (Section 2.3).
#include "hdg_internal.hpp"
#include "wave_ops.hpp"

namespace {

constexpr int BS = 256;
constexpr int MMAX = 8;     // components handled together in the q part

using namespace wave_ops;

// ROWS: the q part reads the rows of [B_d | C_d] and M^{-1} along their length (M <= MMAX and
// P >= 32); otherwise one row per lane. (Two kernels: the first needs more registers.)
template <bool ROWS>
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
    double* t = xe + nt;               // nu: du
    double* sq = t + nu;               // NW x M x P: per-wave products of the q part
    for (int idx = threadIdx.x; idx < nt; idx += BS) {
        const int l = idx / nb, rem = idx - l * nb, m = rem / PF, j = rem - m * PF;
        const int jl = perm ? perm[((size_t)e * L + l) * PF + j] : j;
        xe[(l * M + m) * PF + jl] = xhat[(size_t)e2f[(size_t)e * L + l] * nb + rem];
    }
    __syncthreads();
    const double* Le = local + (size_t)e * nu * C;
    // du = x_r - X xe, four rows per wave at a time
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
    for (int i = threadIdx.x; i < nu; i += BS) du[(size_t)e * nu + i] = t[i];
    const double* Mi = Minv + (size_t)e * P * P;
    if constexpr (ROWS) {
        // dq_{m,d} = -Minv (B_d du_m + C_d uhat_m): the rows of [B_d | C_d], then of Minv, are
        // read along their length by the 64 lanes (coalesced), four rows per wave at a time,
        // against all M vectors in LDS; each row-vector sum is then reduced over the wave.
        // (Rows shorter than half a wave leave most lanes idle: those elements take the
        // row-per-lane form below.)
        double* sd = sq;                       // [D][M][P]: B_d du_m + C_d uhat_m
        const int nbt = (P + 3) / 4;
        for (int bt = wave; bt < D * nbt; bt += NW) {
            const int d = bt / nbt, i0 = (bt - d * nbt) * 4;
            const int nr = P - i0 < 4 ? P - i0 : 4;
            const double* B = Bd + ((size_t)e * D + d) * P * P;
            const double* Cm = Cd + ((size_t)e * D + d) * P * LPF;
            double acc[4][MMAX];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int q = 0; q < MMAX; ++q) acc[r][q] = 0.0;
            for (int k0 = 0; k0 < P; k0 += 64) {
                const int k = k0 + lane;
                const bool ok = k < P;
                const int kc = ok ? k : 0;
                double a[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) a[r] = B[(size_t)(i0 + (r < nr ? r : 0)) * P + kc];
#pragma unroll
                for (int q = 0; q < MMAX; ++q)
                    if (q < M) {
                        const double v = t[q * P + kc];
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[r][q] += ok ? a[r] * v : 0.0;
                    }
            }
            for (int c0 = 0; c0 < LPF; c0 += 64) {
                const int c = c0 + lane;
                const bool ok = c < LPF;
                const int cc = ok ? c : 0;
                const int l = cc / PF, j = cc - l * PF;
                double a[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) a[r] = Cm[(size_t)(i0 + (r < nr ? r : 0)) * LPF + cc];
#pragma unroll
                for (int q = 0; q < MMAX; ++q)
                    if (q < M) {
                        const double v = xe[(l * M + q) * PF + j];
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[r][q] += ok ? a[r] * v : 0.0;
                    }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int q = 0; q < MMAX; ++q)
                    if (q < M) {
                        const double v = wave_sum_all(acc[r][q]);
                        if (lane == 0 && r < nr) sd[(d * M + q) * P + i0 + r] = v;
                    }
        }
        __syncthreads();
        for (int bt = wave; bt < D * nbt; bt += NW) {
            const int d = bt / nbt, i0 = (bt - d * nbt) * 4;
            const int nr = P - i0 < 4 ? P - i0 : 4;
            double acc[4][MMAX];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int q = 0; q < MMAX; ++q) acc[r][q] = 0.0;
            for (int k0 = 0; k0 < P; k0 += 64) {
                const int k = k0 + lane;
                const bool ok = k < P;
                const int kc = ok ? k : 0;
                double a[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) a[r] = Mi[(size_t)(i0 + (r < nr ? r : 0)) * P + kc];
#pragma unroll
                for (int q = 0; q < MMAX; ++q)
                    if (q < M) {
                        const double v = sd[(d * M + q) * P + kc];
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[r][q] += ok ? a[r] * v : 0.0;
                    }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int q = 0; q < MMAX; ++q)
                    if (q < M) {
                        const double v = wave_sum_all(acc[r][q]);
                        if (lane == 0 && r < nr) dq[(size_t)e * M * D * P + (size_t)(q * D + d) * P + i0 + r] = -v;
                    }
        }
        return;
    }
    // one row per lane, one d per wave, MMAX components at a time (B_d, C_d and Minv re-read
    // per group)
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
    const size_t lds = sizeof(double) * ((size_t)nt + nu + (size_t)(BS / 64) * nu);
    const bool rows = d->ncomp <= MMAX && d->npe >= 32;
    const void* fn = rows ? (const void*)k_recover<true> : (const void*)k_recover<false>;
    if (lds > 64 * 1024)
        HDG_HIP_CHECK(ctx, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (rows)
        hipLaunchKernelGGL(k_recover<true>, dim3(d->ne), dim3(BS), lds, ctx->stream, d->ne, d->ncomp, d->dim, d->npe,
                           d->npf, d->nlfe, local, Minv, Bd, Cd, e2f, perm, xhat, du, dq);
    else
        hipLaunchKernelGGL(k_recover<false>, dim3(d->ne), dim3(BS), lds, ctx->stream, d->ne, d->ncomp, d->dim, d->npe,
                           d->npf, d->nlfe, local, Minv, Bd, Cd, e2f, perm, xhat, du, dq);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status axpy_run(hdg_ctx ctx, int64_t n, double alpha, const double* x, double* y) {
    if (n == 0) return HDG_OK;
    hipLaunchKernelGGL(k_axpy, dim3(div_up(n, BS)), dim3(BS), 0, ctx->stream, n, alpha, x, y);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}
