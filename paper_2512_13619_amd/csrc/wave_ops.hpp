// Wave-level helpers shared by the recovery, condensation and block-Jacobi kernels (64-lane waves).
#pragma once

#include <hip/hip_runtime.h>

namespace wave_ops {

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

// Largest v over the wave (ties: smallest i), returned in every lane. Within each row of
// 16 lanes the partners come through DPP (xor 1, xor 2, half-row and row mirrors, no LDS
// round trip); the four row results are then read as uniform values.
template <int CTRL>
__device__ __forceinline__ void argmax_dpp_step(double& v, int& i) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
    const int ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
    const int oi = __builtin_amdgcn_update_dpp(i, i, CTRL, 0xF, 0xF, false);
    const double ov = __hiloint2double(ohi, olo);
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
}

__device__ __forceinline__ void wave_argmax(double& v, int& i) {
    argmax_dpp_step<0xB1>(v, i);   // quad_perm [1,0,3,2]
    argmax_dpp_step<0x4E>(v, i);   // quad_perm [2,3,0,1]
    argmax_dpp_step<0x141>(v, i);  // row_half_mirror
    argmax_dpp_step<0x140>(v, i);  // row_mirror
    const int lo = __double2loint(v), hi = __double2hiint(v);
#pragma unroll
    for (int r = 1; r < 4; ++r) {
        const double ov = __hiloint2double(__builtin_amdgcn_readlane(hi, 16 * r), __builtin_amdgcn_readlane(lo, 16 * r));
        const int oi = __builtin_amdgcn_readlane(i, 16 * r);
        if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
    }
    // row 0's lanes started from their own row value; make every lane agree on the result
    const double v0 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 0),
                                       __builtin_amdgcn_readlane(__double2loint(v), 0));
    i = __builtin_amdgcn_readlane(i, 0);
    v = v0;
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

}  // namespace wave_ops

namespace wave_ops {

// Solves U x = y in place for the n x n upper triangle of U (row stride ld, global memory;
// entries below the diagonal are not read into the result), with y in LDS. All NT threads
// of the block call it. Diagonal blocks of 64 rows from the bottom: the block's rows first
// take the unknowns already solved below them (four rows per wave at a time), then one wave
// solves the 64 x 64 triangle with one unknown per lane. Rows above row 0 in the top block
// are padding (identity rows that take nothing from the rows below).
template <int NT>
__device__ void upper_solve_lds(const double* __restrict__ U, int ld, int n, double* y) {
    constexpr int NW = NT / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int top = n; top > 0; top -= 64) {
        const int base = top - 64;
        const int lo = base > 0 ? base : 0;
        if (top < n) {
            for (int i0 = lo + 4 * wave; i0 < top; i0 += 4 * NW) {
                const int nr = top - i0 < 4 ? top - i0 : 4;
                double res[4];
                rows_dot4(U + top, ld, i0, nr, y + top, n - top, res);
                if (lane < nr) {
                    double rr = res[0];
#pragma unroll
                    for (int r = 1; r < 4; ++r) rr = lane == r ? res[r] : rr;
                    y[i0 + lane] -= rr;
                }
            }
        }
        __syncthreads();
        if (wave == 0) {
            const int g = base + lane;
            double x = g >= 0 ? y[g] : 0.0;
            double ub[64];                 // column g of the block: ub[i] = U[base + i][g]
#pragma unroll
            for (int i = 0; i < 64; ++i) {
                const int gr = base + i;
                const bool in = gr >= 0 && g >= 0;
                const double v = U[in ? (size_t)gr * ld + g : 0];
                ub[i] = in ? v : (i == lane ? 1.0 : 0.0);
            }
#pragma unroll
            for (int i = 63; i >= 0; --i) {
                const double s = wave_sum_all(lane > i ? ub[i] * x : 0.0);
                const double xi = (read_lane(x, i) - s) / read_lane(ub[i], i);
                x = lane == i ? xi : x;
            }
            if (g >= 0) y[g] = x;
        }
        __syncthreads();
    }
}

}  // namespace wave_ops
