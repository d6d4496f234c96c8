// Local recovery (Section 2.3 recovery equation; Section 4.1 eq. w19 and eq. w16),
// one workgroup per element:
//   du = Ebar^{-1}(r_u - Fbar uhat) = U^{-1}(c - Y uhat)   with the factorised rows
//        [U | Y | c] = [U | L^{-1}P Fbar | L^{-1}P r_u] left by the condensation,
//   dq_{m,d} = -M^{-1}(B_d du_m + C_d uhat_m).
// Also the Newton update state += alpha * delta (Section 2.3).
#include "hdg_internal.hpp"

namespace {

constexpr int BS = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
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
    double* xe = sm;             // nt
    double* t = xe + nt;         // nu
    double* s = t + nu;          // P (per (m,d) temp)
    for (int idx = threadIdx.x; idx < nt; idx += BS) {
        const int l = idx / nb, rem = idx - l * nb, m = rem / PF, j = rem - m * PF;
        const int jl = perm ? perm[((size_t)e * L + l) * PF + j] : j;
        xe[(l * M + m) * PF + jl] = xhat[(size_t)e2f[(size_t)e * L + l] * nb + rem];
    }
    __syncthreads();
    const double* Le = local + (size_t)e * nu * C;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = wave; i < nu; i += BS / 64) {
        const double* row = Le + (size_t)i * C + nu;
        double acc = 0.0;
        for (int k = lane; k < nt; k += 64) acc += row[k] * xe[k];
        acc = wave_sum(acc);
        if (lane == 0) t[i] = row[nt] - acc;
    }
    __syncthreads();
    // back substitution with U (column-oriented updates)
    for (int i = nu - 1; i >= 0; --i) {
        const double ui = t[i] / Le[(size_t)i * C + i];
        __syncthreads();
        if (threadIdx.x == 0) t[i] = ui;
        for (int k = threadIdx.x; k < i; k += BS) t[k] -= Le[(size_t)k * C + i] * ui;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < nu; i += BS) du[(size_t)e * nu + i] = t[i];
    // dq_{m,d} = -Minv (B_d du_m + C_d uhat_m)
    const double* Mi = Minv + (size_t)e * P * P;
    for (int m = 0; m < M; ++m) {
        for (int d = 0; d < D; ++d) {
            const double* B = Bd + ((size_t)e * D + d) * P * P;
            const double* Cm = Cd + ((size_t)e * D + d) * P * LPF;
            for (int i = threadIdx.x; i < P; i += BS) {
                double acc = 0.0;
                for (int j = 0; j < P; ++j) acc += B[(size_t)i * P + j] * t[m * P + j];
                for (int l = 0; l < L; ++l)
                    for (int j = 0; j < PF; ++j) acc += Cm[(size_t)i * LPF + l * PF + j] * xe[(l * M + m) * PF + j];
                s[i] = acc;
            }
            __syncthreads();
            for (int i = threadIdx.x; i < P; i += BS) {
                double acc = 0.0;
                for (int k = 0; k < P; ++k) acc += Mi[(size_t)i * P + k] * s[k];
                dq[(size_t)e * M * D * P + (size_t)(m * D + d) * P + i] = -acc;
            }
            __syncthreads();
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
    const size_t lds = sizeof(double) * ((size_t)nt + nu + d->npe);
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
