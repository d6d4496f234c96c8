// Face-block operator: strided block matvec y_f = K_f x_f over the extended
// neighbour vector (Section 4.3), block-Jacobi z_f = P_f^{-1} y_f (Section 4.5),
// and the fused operator step of the polynomial preconditioner (Section 4.7:
// the recurrence's axpy/scale work folded into the product's epilogue).
//
// Mapping (gfx950, wave64): a "team" of TEAM threads owns one face. The face's
// blocks are stored column-major, K[f][s][col][row], so the face row of blocks
// is an nb x (S nb) column-major matrix streamed contiguously from HBM. Thread t
// of the team owns row (t mod nb) and column group (t div nb); with G = TEAM/nb
// groups the team reads G*nb consecutive matrix entries per step, each thread
// accumulating into its fixed row. The extended x (S nb values gathered through
// nbr) sits in LDS; the G partial sums of each row are combined in a fixed order,
// so results are bitwise reproducible. Empty slots (boundary faces) are trailing
// and are never read.
#include "hdg_internal.hpp"

namespace {

template <typename T>
__device__ __forceinline__ double ld_stream(const T* p) {
    return (double)__builtin_nontemporal_load(p);
}

struct FaceArgs {
    const void* M1;
    const int32_t* nbr1;
    const void* M2;
    const double* x;
    FaceEpilogue epi;
    const int* skip;
    int nf, nb, S1, nlfe;
};

// KIND only separates kernel symbols for profiling: 0 = block row product
// (matvec / fused step), 1 = block-diagonal product (block-Jacobi apply).
template <typename T1, typename T2, int TEAM, bool HAS_M2, int KIND>
__global__ __launch_bounds__(256) void k_face_op(FaceArgs A) {
    constexpr int FPB = 256 / TEAM;        // faces per block
    extern __shared__ double smem[];
    if (A.skip && *A.skip) return;
    const int nb = A.nb, S = A.S1;
    const int team = threadIdx.x / TEAM;
    const int t = threadIdx.x - team * TEAM;
    const long long f = (long long)blockIdx.x * FPB + team;
    const bool valid = f < A.nf;
    const int L = S * nb;
    double* xs = smem + team * L;
    double* red = smem + FPB * L;            // 256
    double* uf = red + 256 + team * nb;      // nb per team (second stage input)

    // number of leading non-empty slots (empty slots only ever trail)
    int Seff = S;
    if (valid && A.nbr1 != nullptr && S > A.nlfe && A.nbr1[f * S + A.nlfe] < 0) Seff = A.nlfe;
    const int ncols = Seff * nb;
    if (valid) {
        for (int i = t; i < ncols; i += TEAM) {
            const int s = i / nb;
            const int c = i - s * nb;
            const long long g = A.nbr1 ? (long long)A.nbr1[f * S + s] : f;
            xs[i] = A.x[g * nb + c];
        }
    }
    __syncthreads();

    const int G = TEAM / nb;
    const int grp = t / nb;
    const int row = t - grp * nb;
    double acc = 0.0;
    if (valid && grp < G) {
        const T1* Mf = static_cast<const T1*>(A.M1) + (size_t)f * S * nb * nb;
        const T1* p = Mf + (size_t)grp * nb + row;
        const size_t step = (size_t)G * nb;
        // U independent streaming loads in flight per thread (more for 4-byte entries)
        constexpr int U = sizeof(T1) == 4 ? 8 : 4;
        double a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = 0.0;
        int k = grp;
        for (; k + (U - 1) * G < ncols; k += U * G) {
            T1 m[U];
#pragma unroll
            for (int u = 0; u < U; ++u) m[u] = __builtin_nontemporal_load(p + u * step);
            // keep the U loads in flight together: without this the scheduler interleaves
            // each 4-byte load with its wait and conversion, serialising the stream
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u) a[u] += (double)m[u] * xs[k + u * G];
            p += U * step;
        }
        for (; k < ncols; k += G) {
            a[0] += ld_stream(p) * xs[k];
            p += step;
        }
#pragma unroll
        for (int u = 1; u < U; ++u) a[0] += a[u];
        acc = a[0];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    double u = 0.0;
    if (valid && t < nb) {
        for (int g2 = 0; g2 < G; ++g2) u += red[team * TEAM + g2 * nb + t];
    }
    if (HAS_M2) {
        if (valid && t < nb) uf[t] = u;
        __syncthreads();
        acc = 0.0;
        if (valid && grp < G) {
            const T2* Bf = static_cast<const T2*>(A.M2) + (size_t)f * nb * nb;
            for (int k = grp; k < nb; k += G) acc += (double)Bf[(size_t)k * nb + row] * uf[k];
        }
        __syncthreads();
        red[threadIdx.x] = acc;
        __syncthreads();
        u = 0.0;
        if (valid && t < nb) {
            for (int g2 = 0; g2 < G; ++g2) u += red[team * TEAM + g2 * nb + t];
        }
    }
    if (valid && t < nb) {
        const size_t idx = (size_t)f * nb + t;
        double v[3];
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            v[o] = A.epi.s[o] * u;
            if (A.epi.X[o]) v[o] += A.epi.a[o] * A.epi.X[o][idx];
            if (A.epi.Y[o]) v[o] += A.epi.b[o] * A.epi.Y[o][idx];
        }
#pragma unroll
        for (int o = 0; o < 3; ++o)
            if (A.epi.out[o]) A.epi.out[o][idx] = v[o];
    }
}

template <typename T1, typename T2, bool HAS_M2, int KIND>
hdg_status launch_team(hdg_ctx ctx, const FaceArgs& a) {
    int team;
    // a block row (S1 > 1) has S1*nb columns: 4 column groups keep every thread busy; a
    // block-diagonal product (S1 == 1) has only nb columns, so fewer groups give each
    // thread a longer run of loads
    const int want = (a.S1 > 1 ? 4 : 2) * a.nb;
    if (a.nb > 64 || want > 128) team = 256;
    else if (want > 64) team = 128;
    else if (want > 32) team = 64;
    else if (want > 16) team = 32;
    else team = 16;
    const int fpb = 256 / team;
    const size_t lds = sizeof(double) * ((size_t)fpb * a.S1 * a.nb + 256 + (size_t)fpb * a.nb);
    const int grid = div_up(a.nf, fpb);
    if (grid == 0) return HDG_OK;
    switch (team) {
        case 256: hipLaunchKernelGGL((k_face_op<T1, T2, 256, HAS_M2, KIND>), dim3(grid), dim3(256), lds, ctx->stream, a); break;
        case 128: hipLaunchKernelGGL((k_face_op<T1, T2, 128, HAS_M2, KIND>), dim3(grid), dim3(256), lds, ctx->stream, a); break;
        case 64:  hipLaunchKernelGGL((k_face_op<T1, T2, 64, HAS_M2, KIND>), dim3(grid), dim3(256), lds, ctx->stream, a); break;
        case 32:  hipLaunchKernelGGL((k_face_op<T1, T2, 32, HAS_M2, KIND>), dim3(grid), dim3(256), lds, ctx->stream, a); break;
        default:  hipLaunchKernelGGL((k_face_op<T1, T2, 16, HAS_M2, KIND>), dim3(grid), dim3(256), lds, ctx->stream, a); break;
    }
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

}  // namespace

hdg_status face_op(hdg_ctx ctx, int nf, int nb, int S1, int nlfe, const void* M1, bool m1_fp32,
                   const int32_t* nbr1, const void* M2, bool m2_fp32, const double* x,
                   const FaceEpilogue& epi, const int* skip_flag) {
    if (nb < 1 || nb > 256) {
        ctx->err = "face block edge M*P_F must be in [1, 256]";
        return HDG_ERR_SHAPE;
    }
    FaceArgs a;
    a.M1 = M1;
    a.nbr1 = nbr1;
    a.M2 = M2;
    a.x = x;
    a.epi = epi;
    a.skip = skip_flag;
    a.nf = nf;
    a.nb = nb;
    a.S1 = S1;
    a.nlfe = nlfe;
    if (M2 == nullptr) {
        if (nbr1 == nullptr)
            return m1_fp32 ? launch_team<float, float, false, 1>(ctx, a) : launch_team<double, double, false, 1>(ctx, a);
        return m1_fp32 ? launch_team<float, float, false, 0>(ctx, a) : launch_team<double, double, false, 0>(ctx, a);
    }
    if (m1_fp32 && m2_fp32) return launch_team<float, float, true, 0>(ctx, a);
    if (!m1_fp32 && !m2_fp32) return launch_team<double, double, true, 0>(ctx, a);
    if (m1_fp32) return launch_team<float, double, true, 0>(ctx, a);
    return launch_team<double, float, true, 0>(ctx, a);
}
