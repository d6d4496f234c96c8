// Block-Jacobi setup (Section 4.5): invert every diagonal face block K_ff by
// Gauss-Jordan elimination with partial pivoting. Blocks of edge <= 64: one wave per face
// with the block in its registers; larger ones: one workgroup per face, the augmented
// [K_ff | I] held in LDS. Inverses are written column-major like K (Binv[f][col][row]) in
// FP64 and optionally rounded to FP32.
#include <cmath>

#include "hdg_internal.hpp"
#include "wave_ops.hpp"

namespace {

constexpr int BS = 256;

__global__ __launch_bounds__(BS) void k_bj_invert(int nf, int nb, int S, const double* __restrict__ K,
                                                  double* __restrict__ B64, float* __restrict__ B32,
                                                  int* bad_face) {
    extern __shared__ double sm[];
    const int lda = 2 * nb + 1;          // odd stride: no LDS bank conflicts on column access
    double* A = sm;                      // nb x (2nb) augmented, row-major
    __shared__ int piv_s;
    __shared__ double pval_s;
    const long long f = blockIdx.x;
    if (f >= nf) return;
    const double* Kf = K + (size_t)f * S * nb * nb;   // slot 0, column-major
    for (int idx = threadIdx.x; idx < nb * nb; idx += BS) {
        const int c = idx / nb, r = idx - c * nb;
        A[r * lda + c] = Kf[idx];
        A[r * lda + nb + c] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    bool singular = false;
    for (int k = 0; k < nb; ++k) {
        if (threadIdx.x < 64) {
            double best = -1.0;
            int bi = k;
            for (int r = k + threadIdx.x; r < nb; r += 64) {
                const double v = fabs(A[r * lda + k]);
                if (v > best || (v == best && r < bi)) { best = v; bi = r; }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_xor(best, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
            }
            if (threadIdx.x == 0) { piv_s = bi; pval_s = A[bi * lda + k]; }
        }
        __syncthreads();
        const int p = piv_s;
        double pv = pval_s;
        if (!(fabs(pv) > 0.0) || !isfinite(pv)) { singular = true; pv = 1.0; }
        if (p != k) {
            for (int c = threadIdx.x; c < 2 * nb; c += BS) {
                const double t = A[k * lda + c];
                A[k * lda + c] = A[p * lda + c];
                A[p * lda + c] = t;
            }
        }
        __syncthreads();
        const double inv = 1.0 / pv;
        for (int c = threadIdx.x; c < 2 * nb; c += BS) A[k * lda + c] *= inv;
        __syncthreads();
        // eliminate column k from every other row
        for (int idx = threadIdx.x; idx < nb * 2 * nb; idx += BS) {
            const int r = idx / (2 * nb), c = idx - r * (2 * nb);
            if (r == k || c == k) continue;
            A[r * lda + c] -= A[r * lda + k] * A[k * lda + c];
        }
        __syncthreads();
        for (int r = threadIdx.x; r < nb; r += BS)
            if (r != k) A[r * lda + k] = 0.0;
        __syncthreads();
    }
    if (singular && threadIdx.x == 0) atomicMin(bad_face, (int)f);
    for (int idx = threadIdx.x; idx < nb * nb; idx += BS) {
        const int c = idx / nb, r = idx - c * nb;
        const double v = A[r * lda + nb + c];
        B64[(size_t)f * nb * nb + idx] = v;
        if (B32) B32[(size_t)f * nb * nb + idx] = (float)v;
    }
}

// The same inversion for nb <= NBT <= 64, one wave per face and four faces per workgroup: lane
// r holds row r of the block in registers, and the elimination runs in place (the column of
// the unit vector that the augmented form would carry is stored in the column just
// eliminated). Rows never move: each lane tracks the position its row has in the
// interchanged order, the pivot of column k is the largest |entry| among the rows not yet
// chosen (ties to the lower position, a NaN entry wins so that the face is flagged), and
// the pivot row reaches every lane through readlane. The same operations in the same order
// as the LDS kernel: the results agree bit for bit on finite blocks. At the end, row
// position i of the registers is row i of the inverse with its columns interchanged by the
// pivots; the inverse's column for each register column is found by undoing those
// interchanges in reverse order.
template <int NBT>
__global__ __launch_bounds__(BS) void k_bj_invert_w(int nf, int nb, int S, const double* __restrict__ K,
                                                    double* __restrict__ B64, float* __restrict__ B32,
                                                    int* bad_face) {
    const long long f = (long long)blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
    if (f >= nf) return;
    const int lane = threadIdx.x & 63;
    const bool row_ok = lane < nb;
    const double* Kf = K + (size_t)f * S * nb * nb;   // slot 0, column-major
    double a[NBT];
#pragma unroll
    for (int c = 0; c < NBT; ++c) {
        const bool ok = row_ok && c < nb;
        const double v = Kf[ok ? c * nb + lane : 0];
        a[c] = ok ? v : 0.0;
    }
    int pos = lane;          // position of this lane's row in the interchanged order
    bool live = row_ok;      // the row has not been a pivot row yet
    int pk = 0;              // in lane k: the position interchanged with k at step k
    bool bad = false;
#pragma unroll
    for (int k = 0; k < NBT; ++k) {
        if (k < nb) {
            double v = live ? fabs(a[k]) : -1.0;
            if (live && !(v >= 0.0)) v = INFINITY;
            int key = live ? (pos << 8) | lane : 0x7fffffff;
            wave_ops::wave_argmax(v, key);
            const int ol = key & 255, p = key >> 8;      // the pivot row's lane and position
            if (lane == k) pk = p;
            double pv = wave_ops::read_lane(a[k], ol);
            if (pos == k) pos = p;
            const bool prow = lane == ol;
            if (prow) { pos = k; live = false; }
            if (!(fabs(pv) > 0.0) || !isfinite(pv)) { bad = true; pv = 1.0; }
            const double inv = 1.0 / pv;
            const double m = prow ? 0.0 : a[k];
            a[k] = prow ? inv : -m * inv;
#pragma unroll
            for (int c = 0; c < NBT; ++c) {
                if (c != k && c < nb) {
                    const double pc = wave_ops::read_lane(a[c], ol) * inv;   // the scaled pivot row
                    a[c] = prow ? pc : fma(-m, pc, a[c]);
                }
            }
        }
    }
    if (bad && lane == 0) atomicMin(bad_face, (int)f);
    // lane j: the inverse's column that register column j holds
    int d = lane;
    for (int k = nb - 1; k >= 0; --k) {
        const int p = __builtin_amdgcn_readlane(pk, k);
        d = d == k ? p : (d == p ? k : d);
    }
    double* Bo = B64 + (size_t)f * nb * nb;
    float* Bo32 = B32 ? B32 + (size_t)f * nb * nb : nullptr;
#pragma unroll
    for (int c = 0; c < NBT; ++c) {
        if (c < nb) {
            const int col = __builtin_amdgcn_readlane(d, c);
            if (row_ok) {
                Bo[(size_t)col * nb + pos] = a[c];
                if (Bo32) Bo32[(size_t)col * nb + pos] = (float)a[c];
            }
        }
    }
}

// Right-preconditioned operator blocks (Section 3.2 with M = blockdiag(K_ff)):
//     Kf[f][s] = K[f][s] * Binv[nbr(f,s)]
// so that (K M^{-1}) x needs one block row product and no separate block-Jacobi pass.
// One wave per (face, slot), 16x16 output tiles of v_mfma_f64_16x16x4f64 over the block
// padded to a multiple of 16; FP64 products, rounded to T on output. Empty slots are skipped.
// k is taken in groups of 16 with instruction s giving lane (i, kq) the pair
// A(i, kb+4kq+s), B(kb+4kq+s, j): the sum over a group covers its 16 k, and each lane reads
// four consecutive k of the column-major B. A tile's loads are all issued before its MFMAs.
template <typename T, int KG>
__global__ __launch_bounds__(BS) void k_fold_bj(int nf, int nb, int S, const double* __restrict__ K,
                                                const int32_t* __restrict__ nbr, const double* __restrict__ Binv,
                                                T* __restrict__ out) {
    const long long pair = (long long)blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
    if (pair >= (long long)nf * S) return;
    const int g = nbr[pair];
    if (g < 0) return;
    const int lane = threadIdx.x & 63;
    const int i16 = lane & 15, kq = lane >> 4;
    const size_t bsz = (size_t)nb * nb;
    const double* A = K + (size_t)pair * bsz;       // A(row, k) = A[k*nb + row]
    const double* B = Binv + (size_t)g * bsz;       // B(k, col) = B[col*nb + k]
    T* C = out + (size_t)pair * bsz;                // C(row, col) at C[col*nb + row]
    const int nt = (nb + 15) / 16;
    for (int ti = 0; ti < nt; ++ti)
        for (int tj = 0; tj < nt; ++tj) {
            const int row = ti * 16 + i16, col = tj * 16 + i16;
            double a[KG][4], b[KG][4];
#pragma unroll
            for (int gi = 0; gi < KG; ++gi)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int k = gi * 16 + 4 * kq + u;
                    const bool oka = row < nb && k < nb, okb = col < nb && k < nb;
                    a[gi][u] = A[oka ? (size_t)k * nb + row : 0];
                    b[gi][u] = B[okb ? (size_t)col * nb + k : 0];
                }
            __builtin_amdgcn_sched_barrier(0);      // all loads in flight before the first use
            double4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int gi = 0; gi < KG; ++gi)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int k = gi * 16 + 4 * kq + u;
                    const double av = (row < nb && k < nb) ? a[gi][u] : 0.0;   // padding
                    const double bv = (col < nb && k < nb) ? b[gi][u] : 0.0;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = ti * 16 + 4 * q + (lane >> 4);
                const int c = tj * 16 + (lane & 15);
                if (r < nb && c < nb) C[(size_t)c * nb + r] = (T)acc[q];
            }
        }
}

// The same product for blocks of edge <= 16 KG (KG <= 2), computed as C^T = Binv^T A^T so
// that both operands are read along their contiguous direction and the output tile columns
// are written 16 rows at a time: Binv goes through the wave's own LDS region (coalesced
// loads, column stride nb+1), every A operand of the block is loaded from global memory up
// front, and all 16x16 tiles of the (face, slot) pair are then formed from registers and LDS.
template <typename T, int KG>
__global__ __launch_bounds__(BS) void k_fold_bj_lds(int nf, int nb, int S, const double* __restrict__ K,
                                                    const int32_t* __restrict__ nbr,
                                                    const double* __restrict__ Binv, T* __restrict__ out) {
    extern __shared__ double fsm[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long pair = (long long)blockIdx.x * (BS / 64) + wave;
    if (pair >= (long long)nf * S) return;
    const int g = nbr[pair];
    if (g < 0) return;
    const int i16 = lane & 15, kq = lane >> 4;
    const int ldb = nb + 1;
    const int bsz = nb * nb;
    double* Bs = fsm + (size_t)wave * nb * ldb;
    const double* A = K + (size_t)pair * bsz;       // A(row, k) = A[k*nb + row]
    const double* B = Binv + (size_t)g * bsz;       // B(k, col) = B[col*nb + k]
    T* C = out + (size_t)pair * bsz;                // C(row, col) at C[col*nb + row]
    constexpr int PER = (16 * KG * 16 * KG + 63) / 64;
    double bv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = lane + 64 * u;
        bv[u] = B[idx < bsz ? idx : 0];
    }
    // ao[ti][gi][s] = A(16 ti + i16, 16 gi + 4 kq + s), raw (masked at use)
    double ao[KG][KG][4];
#pragma unroll
    for (int ti = 0; ti < KG; ++ti)
#pragma unroll
        for (int gi = 0; gi < KG; ++gi)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int row = 16 * ti + i16, k = 16 * gi + 4 * kq + u;
                ao[ti][gi][u] = A[(row < nb && k < nb) ? k * nb + row : 0];
            }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = lane + 64 * u;
        if (idx < bsz) {
            const int col = idx / nb;
            Bs[col * ldb + (idx - col * nb)] = bv[u];
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int tj = 0; tj < KG; ++tj) {
        const int col = 16 * tj + i16;
        double bo[KG][4];                            // Binv^T(col, k) = Binv(k, col)
#pragma unroll
        for (int gi = 0; gi < KG; ++gi)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = 16 * gi + 4 * kq + u;
                const bool ok = col < nb && k < nb;
                const double v = Bs[ok ? col * ldb + k : 0];
                bo[gi][u] = ok ? v : 0.0;
            }
        // the KG row tiles of this column tile accumulate side by side (independent MFMA chains)
        double4_t acc[KG];
#pragma unroll
        for (int ti = 0; ti < KG; ++ti) acc[ti] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int gi = 0; gi < KG; ++gi)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = 16 * gi + 4 * kq + u;
#pragma unroll
                for (int ti = 0; ti < KG; ++ti) {
                    const double av = (16 * ti + i16 < nb && k < nb) ? ao[ti][gi][u] : 0.0;
                    acc[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(bo[gi][u], av, acc[ti], 0, 0, 0);
                }
            }
        // acc[ti][q] = C^T(16 tj + 4q + lane/16, 16 ti + lane%16)
#pragma unroll
        for (int ti = 0; ti < KG; ++ti)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = 16 * tj + 4 * q + (lane >> 4);
                const int r = 16 * ti + (lane & 15);
                if (r < nb && c < nb) C[(size_t)c * nb + r] = (T)acc[ti][q];
            }
    }
}

// The same product for blocks of edge 33..48 (KG = 3) with every operand in registers: the
// wave loads all of its A block up front (the B operand of C^T = Binv^T A^T, each lane 16
// consecutive rows of a column), then, per 16-column tile of the output, the Binv^T
// operands of that tile (four consecutive k of one column of Binv per lane) and the KG row
// tiles' products. Without LDS staging the kernel holds two waves per SIMD (the LDS form
// needs all of a block's Binv in registers before its store and holds one).
template <typename T, int KG>
__global__ __launch_bounds__(BS) void k_fold_bj_r(int nf, int nb, int S, const double* __restrict__ K,
                                                  const int32_t* __restrict__ nbr,
                                                  const double* __restrict__ Binv, T* __restrict__ out) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long pair = (long long)blockIdx.x * (BS / 64) + wave;
    if (pair >= (long long)nf * S) return;
    const int g = nbr[pair];
    if (g < 0) return;
    const int i16 = lane & 15, kq = lane >> 4;
    const int bsz = nb * nb;
    const double* A = K + (size_t)pair * bsz;
    const double* B = Binv + (size_t)g * bsz;
    T* C = out + (size_t)pair * bsz;
    double ao[KG][KG][4];
#pragma unroll
    for (int ti = 0; ti < KG; ++ti)
#pragma unroll
        for (int gi = 0; gi < KG; ++gi)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int row = 16 * ti + i16, k = 16 * gi + 4 * kq + u;
                ao[ti][gi][u] = A[(row < nb && k < nb) ? k * nb + row : 0];
            }
#pragma unroll
    for (int tj = 0; tj < KG; ++tj) {
        const int col = 16 * tj + i16;
        double bo[KG][4];
#pragma unroll
        for (int gi = 0; gi < KG; ++gi)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = 16 * gi + 4 * kq + u;
                bo[gi][u] = B[(col < nb && k < nb) ? col * nb + k : 0];
            }
        double4_t acc[KG];
#pragma unroll
        for (int ti = 0; ti < KG; ++ti) acc[ti] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int gi = 0; gi < KG; ++gi)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = 16 * gi + 4 * kq + u;
                const double bv = (col < nb && k < nb) ? bo[gi][u] : 0.0;
#pragma unroll
                for (int ti = 0; ti < KG; ++ti) {
                    const double av = (16 * ti + i16 < nb && k < nb) ? ao[ti][gi][u] : 0.0;
                    acc[ti] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv, av, acc[ti], 0, 0, 0);
                }
            }
#pragma unroll
        for (int ti = 0; ti < KG; ++ti)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = 16 * tj + 4 * q + (lane >> 4);
                const int r = 16 * ti + (lane & 15);
                if (r < nb && c < nb) C[(size_t)c * nb + r] = (T)acc[ti][q];
            }
    }
}
}  // namespace

hdg_status fold_bj(hdg_ctx ctx, int nf, int nb, int S, const double* K64, const int32_t* nbr, const double* B64,
                   void* out, bool out_fp32) {
    const long long pairs = (long long)nf * S;
    if (pairs == 0) return HDG_OK;
    const int grid = div_up(pairs, BS / 64);
    if (nb > 256) {
        ctx->err = "fold_bj: face block edge above 256";
        return HDG_ERR_SHAPE;
    }
#define HDG_FOLD(T, KG) \
    hipLaunchKernelGGL((k_fold_bj<T, KG>), dim3(grid), dim3(BS), 0, ctx->stream, nf, nb, S, K64, nbr, B64, (T*)out)
#define HDG_FOLD_R(T, KG) \
    hipLaunchKernelGGL((k_fold_bj_r<T, KG>), dim3(grid), dim3(BS), 0, ctx->stream, nf, nb, S, K64, nbr, B64, (T*)out)
#define HDG_FOLD_LDS(T, KG) \
    hipLaunchKernelGGL((k_fold_bj_lds<T, KG>), dim3(grid), dim3(BS), lds, ctx->stream, nf, nb, S, K64, nbr, B64, \
                       (T*)out)
    // KG groups of 16 k cover the (padded) block edge
    const int kg = (nb + 15) / 16;
    if (kg == 3) {
        if (out_fp32) HDG_FOLD_R(float, 3); else HDG_FOLD_R(double, 3);
        HDG_LAUNCH_CHECK(ctx);
        return HDG_OK;
    }
    if (kg <= 2) {
        const size_t lds = sizeof(double) * (BS / 64) * (size_t)nb * (nb + 1);
        if (lds > 64 * 1024) {
            const void* fn = out_fp32 ? (kg <= 1 ? (const void*)k_fold_bj_lds<float, 1> : (const void*)k_fold_bj_lds<float, 2>)
                                      : (kg <= 1 ? (const void*)k_fold_bj_lds<double, 1> : (const void*)k_fold_bj_lds<double, 2>);
            HDG_HIP_CHECK(ctx, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        }
        if (out_fp32) {
            if (kg <= 1) HDG_FOLD_LDS(float, 1); else HDG_FOLD_LDS(float, 2);
        } else {
            if (kg <= 1) HDG_FOLD_LDS(double, 1); else HDG_FOLD_LDS(double, 2);
        }
        HDG_LAUNCH_CHECK(ctx);
        return HDG_OK;
    }
    // larger blocks: tile by tile
    if (out_fp32) {
        if (kg <= 4) HDG_FOLD(float, 4); else if (kg <= 8) HDG_FOLD(float, 8); else HDG_FOLD(float, 16);
    } else {
        if (kg <= 4) HDG_FOLD(double, 4); else if (kg <= 8) HDG_FOLD(double, 8); else HDG_FOLD(double, 16);
    }
#undef HDG_FOLD
#undef HDG_FOLD_R
#undef HDG_FOLD_LDS
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status bj_invert(hdg_ctx ctx, int nf, int nb, int S, const double* K64, double* B64, float* B32,
                     int* bad_face) {
    if (nf == 0) return HDG_OK;
    if (nb <= 64) {
        const dim3 grid((unsigned)div_up((long long)nf, BS / 64));
        if (nb <= 16)
            hipLaunchKernelGGL(k_bj_invert_w<16>, grid, dim3(BS), 0, ctx->stream, nf, nb, S, K64, B64, B32, bad_face);
        else if (nb <= 32)
            hipLaunchKernelGGL(k_bj_invert_w<32>, grid, dim3(BS), 0, ctx->stream, nf, nb, S, K64, B64, B32, bad_face);
        else if (nb <= 48)
            hipLaunchKernelGGL(k_bj_invert_w<48>, grid, dim3(BS), 0, ctx->stream, nf, nb, S, K64, B64, B32, bad_face);
        else
            hipLaunchKernelGGL(k_bj_invert_w<64>, grid, dim3(BS), 0, ctx->stream, nf, nb, S, K64, B64, B32, bad_face);
        HDG_LAUNCH_CHECK(ctx);
        return HDG_OK;
    }
    const size_t lds = sizeof(double) * (size_t)nb * (2 * nb + 1);
    if (lds > 150 * 1024) {
        ctx->err = "block-Jacobi: face block too large for LDS";
        return HDG_ERR_SHAPE;
    }
    if (lds > 64 * 1024)
        HDG_HIP_CHECK(ctx, hipFuncSetAttribute((const void*)k_bj_invert,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_bj_invert, dim3(nf), dim3(BS), lds, ctx->stream, nf, nb, S, K64, B64, B32, bad_face);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}
