// Krylov vector kernels: Gram-Schmidt multi-dot / multi-axpy, norms, and the
// device-side Hessenberg/Givens update of GMRES (Section 4.4). The paper keeps
// the Hessenberg system on the CPU; here one thread on the device performs the
// same FP64 rotations so a whole restart cycle runs without host round trips.
//
// Reductions are two-stage with a fixed block count and fixed summation order,
// so every run gives bitwise identical results.
#include <cmath>

#include <hip/hip_ext.h>

#include "hdg_internal.hpp"

namespace {

constexpr int BS = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// part[i*nblk + b] = sum_{k in chunk b} V[i][k] w[k],  i < J.
// The block's slice of w is staged in LDS; each wave owns a subset of the vectors and
// streams them with U loads in flight per lane, so one wave writes each partial.
constexpr int CHUNK = 2048;        // largest chunk (krylov_chunk): the LDS staging size
constexpr int COEF_BS = 1024;      // threads of the delayed-CGS2 coefficient kernel

template <int U>
__global__ __launch_bounds__(BS) void k_multidot(const double* __restrict__ V, size_t ldv, int J,
                                                 const double* __restrict__ w, size_t n,
                                                 double* __restrict__ part, int nblk, const int* skip) {
    if (skip && *skip) return;
    __shared__ double ws[CHUNK];
    const int chunk = krylov_chunk(n);
    const size_t k0 = (size_t)blockIdx.x * chunk;
    const int len = (int)(k0 + chunk < n ? chunk : n - k0);
    for (int k = threadIdx.x; k < len; k += BS) ws[k] = w[k0 + k];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = wave; i < J; i += BS / 64) {
        const double* v = V + (size_t)i * ldv + k0;
        double acc = 0.0;
        for (int k = lane; k < len; k += 64 * U) {
            double m[U];
#pragma unroll
            for (int u = 0; u < U; ++u) m[u] = (k + 64 * u < len) ? v[k + 64 * u] : 0.0;
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (k + 64 * u < len) acc += m[u] * ws[k + 64 * u];
        }
        acc = wave_sum(acc);
        if (lane == 0) part[(size_t)i * nblk + blockIdx.x] = acc;
    }
}

// out[i] = sum_b part[i*nblk + b]; if add_to: add_to[i] += out[i]. One wave per i.
__global__ void k_reduce(const double* __restrict__ part, int J, int nblk, double* out, double* add_to,
                         const int* skip) {
    if (skip && *skip) return;
    const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= J) return;
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += part[(size_t)i * nblk + b];
    s = wave_sum(s);
    if (lane == 0) {
        if (out) out[i] = s;
        if (add_to) add_to[i] += s;
    }
}

// w[k] += sign * sum_{i<J} V[i][k] h[i]  (vectors in groups of 8 loads in flight)
__global__ __launch_bounds__(BS) void k_multiaxpy(const double* __restrict__ V, size_t ldv, int J,
                                                  const double* __restrict__ h, double sign, double* w,
                                                  size_t n, const int* skip, const int* J_dev) {
    if (skip && *skip) return;
    const size_t k = (size_t)blockIdx.x * BS + threadIdx.x;
    if (k >= n) return;
    const int JJ = J_dev ? *J_dev : J;
    double acc = 0.0;
    for (int i0 = 0; i0 < JJ; i0 += 8) {
        double m[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) m[u] = (i0 + u < JJ) ? V[(size_t)(i0 + u) * ldv + k] : 0.0;
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + u < JJ) acc += m[u] * h[i0 + u];
    }
    w[k] += sign * acc;
}

__global__ __launch_bounds__(BS) void k_sumsq(const double* __restrict__ w, size_t n, double* part, int nblk,
                                              const int* skip) {
    if (skip && *skip) return;
    __shared__ double red[BS / 64];
    const int chunk = krylov_chunk(n);
    const size_t k0 = (size_t)blockIdx.x * chunk;
    const size_t k1 = k0 + chunk < n ? k0 + chunk : n;
    double acc = 0.0;
    for (size_t k = k0 + threadIdx.x; k < k1; k += BS) acc += w[k] * w[k];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < BS / 64; ++q) s += red[q];
        part[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(BS) void k_lincomb(size_t n, double* out, double a, const double* X, double b,
                                                const double* Y, const int* skip) {
    if (skip && *skip) return;
    const size_t k = (size_t)blockIdx.x * BS + threadIdx.x;
    if (k >= n) return;
    double v = 0.0;
    if (X) v += a * X[k];
    if (Y) v += b * Y[k];
    out[k] = v;
}

__global__ __launch_bounds__(BS) void k_scale_by(double* v, const double* src, size_t n, const double* denom,
                                                 const int* skip) {
    if (skip && *skip) return;
    const size_t k = (size_t)blockIdx.x * BS + threadIdx.x;
    if (k >= n) return;
    v[k] = src[k] / *denom;
}

// Sum of the norm partials of the cycle-start residual; initialises the cycle.
__global__ void k_cycle_init(GmresCtl* ctl, const double* part, int nblk, double* g, int jmax, double target) {
    const int lane = threadIdx.x;
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += part[b];
    s = wave_sum(s);
    if (lane == 0) {
        const double beta = sqrt(s);
        ctl->beta = beta;
        ctl->est = beta;
        ctl->k = 0;
        ctl->jmax = jmax;
        ctl->target = target;
        ctl->nonfinite = !isfinite(beta);
        ctl->done = (beta <= target || !isfinite(beta) || jmax <= 0) ? 1 : 0;
        g[0] = beta;
    }
}

__global__ void k_store_norm(const double* part, int nblk, double* dst) {
    const int lane = threadIdx.x;
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += part[b];
    s = wave_sum(s);
    if (lane == 0) *dst = sqrt(s);
}

// Step j: column j of H (rows 0..j already hold the Gram-Schmidt coefficients);
// h_{j+1,j} from the norm partials; previous rotations, new rotation, residual estimate.
__global__ void k_givens(GmresCtl* ctl, const double* part, int nblk, double* H, int ldh, double* cs,
                         double* sn, double* g, int j, double* hist) {
    if (ctl->done) return;
    const int lane = threadIdx.x;
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += part[b];
    s = wave_sum(s);
    if (lane != 0) return;
    const double hn = sqrt(s);
    double* col = H + (size_t)j * ldh;     // column-major (ldh = m+1)
    col[j + 1] = hn;   // the rotated subdiagonal is zero; the slot keeps h_{j+1,j} to scale v_{j+1}
    double hjj = col[j];
    for (int i = 0; i < j; ++i) {
        const double t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = t;
    }
    hjj = col[j];
    double c = 1.0, sg = 0.0;
    if (hn != 0.0) {
        const double r = hypot(hjj, hn);
        c = hjj / r;
        sg = hn / r;
    }
    cs[j] = c;
    sn[j] = sg;
    col[j] = c * hjj + sg * hn;
    const double gj = g[j];
    g[j + 1] = -sg * gj;
    g[j] = c * gj;
    const double est = fabs(g[j + 1]);
    ctl->est = est;
    ctl->k = j + 1;
    if (hist) hist[j] = est;
    if (!isfinite(est) || !isfinite(col[j])) ctl->nonfinite = 1;
    if (est <= ctl->target || hn == 0.0 || j + 1 >= ctl->jmax || !isfinite(est)) ctl->done = 1;
}

// y = R^{-1} g over the k steps of this cycle (upper triangular R in H, column-major).
// Back substitution R y = g (R = the k x k upper triangle of the rotated H, column-major with
// leading dimension ldh) by column sweeps: y_c = r_c / R_cc, then r_i -= R_ic y_c for i < c
// in parallel. The triangle is staged in LDS (packed by columns) when it fits, else read
// from global memory column by column.
constexpr int BACKSOLVE_BS = 256;
constexpr int BACKSOLVE_LDS = 4096;     // doubles of packed triangle: k <= 90
__global__ __launch_bounds__(BACKSOLVE_BS) void k_backsolve(const GmresCtl* ctl, const double* H, int ldh,
                                                            const double* g, double* y) {
    __shared__ double tri[BACKSOLVE_LDS];
    __shared__ double r[256];
    const int k = ctl->k;
    const int tid = threadIdx.x;
    const bool staged = (long)k * (k + 1) / 2 <= BACKSOLVE_LDS;
    for (int i = tid; i < k; i += BACKSOLVE_BS) r[i] = g[i];
    if (staged)
        for (int c = 0; c < k; ++c)
            for (int i = tid; i <= c; i += BACKSOLVE_BS) tri[c * (c + 1) / 2 + i] = H[(size_t)c * ldh + i];
    __syncthreads();
    for (int c = k - 1; c >= 0; --c) {
        const double* col = staged ? tri + c * (c + 1) / 2 : H + (size_t)c * ldh;
        const double yc = r[c] / col[c];
        for (int i = tid; i < c; i += BACKSOLVE_BS) r[i] -= col[i] * yc;
        if (tid == 0) y[c] = yc;
        __syncthreads();
    }
    for (int i = k + tid; i < ldh - 1; i += BACKSOLVE_BS) y[i] = 0.0;
}

// Fused second Gram-Schmidt pass, part 1: w <- w - V h1 and partial dots V^T w
// (the new w) in one read of V. Same chunking as k_multidot, so k_reduce applies.
//
// A wave takes 64 consecutive entries (one per lane) and holds their JMAX basis values
// only while it works on them: the products V[i][k] w[k] are summed over the lanes by a
// reduce-scatter (log2(JMAX) halving steps of lane exchanges) that leaves the sum for
// column (lane mod JMAX) in the lane, so each lane keeps one accumulator instead of JMAX.
template <int JMAX>
__global__ __launch_bounds__(BS) void k_axpy_dot(const double* __restrict__ V, size_t ldv, int J,
                                                 const double* __restrict__ h1, double* __restrict__ w, size_t n,
                                                 double* __restrict__ part, int nblk, const int* skip) {
    if (skip && *skip) return;
    __shared__ double hs[JMAX];
    __shared__ double red[BS / 64][JMAX];
    for (int i = threadIdx.x; i < JMAX; i += BS) hs[i] = i < J ? h1[i] : 0.0;
    __syncthreads();
    const int chunk = krylov_chunk(n);
    const size_t k0 = (size_t)blockIdx.x * chunk;
    const size_t k1 = k0 + chunk < n ? k0 + chunk : n;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double acc = 0.0;
    for (size_t kb = k0 + (size_t)wave * 64; kb < k1; kb += BS) {
        const size_t k = kb + lane;
        const bool ok = k < k1;
        const size_t kc = ok ? k : k0;
        const double wk = w[kc];
        // all JMAX loads in flight; columns at or past J read column 0 (valid memory) and
        // drop out: hs is 0 there, and their dot products are never written
        double v[JMAX];
#pragma unroll
        for (int i = 0; i < JMAX; ++i) v[i] = V[(size_t)(i < J ? i : 0) * ldv + kc];
        __builtin_amdgcn_sched_barrier(0);
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < JMAX; ++i) s += v[i] * hs[i];
        const double wn = ok ? wk - s : 0.0;
        if (ok) w[k] = wn;
#pragma unroll
        for (int i = 0; i < JMAX; ++i) v[i] *= wn;
        // reduce-scatter: after the step with mask m a lane holds half as many sums, each
        // over twice as many lanes; the last one leaves column (lane mod JMAX) in v[0]
#pragma unroll
        for (int S = JMAX; S > 1; S >>= 1) {
            const int m = S >> 1;
            const bool up = (lane & m) != 0;
#pragma unroll
            for (int t = 0; t < S / 2; ++t) {
                const double keep = up ? v[t + S / 2] : v[t];
                const double send = up ? v[t] : v[t + S / 2];
                v[t] = keep + __shfl_xor(send, m, 64);
            }
        }
        acc += v[0];
    }
    // lanes that share a column (lane mod JMAX) hold partial sums of it
#pragma unroll
    for (int m = 32; m >= JMAX; m >>= 1) acc += __shfl_xor(acc, m, 64);
    if (lane < JMAX) red[wave][lane] = acc;
    __syncthreads();
    if (threadIdx.x < J) {
        double t = 0.0;
        for (int q = 0; q < BS / 64; ++q) t += red[q][threadIdx.x];
        part[(size_t)threadIdx.x * nblk + blockIdx.x] = t;
    }
}

// Fused second pass, part 2: w <- w - V h2 and partial sums of w^2 (the norm) in one read of V.
template <int JMAX>
__global__ __launch_bounds__(BS) void k_axpy_sumsq(const double* __restrict__ V, size_t ldv, int J,
                                                   const double* __restrict__ h2, double* __restrict__ w, size_t n,
                                                   double* __restrict__ part, int nblk, const int* skip) {
    if (skip && *skip) return;
    __shared__ double red[BS / 64];
    const int chunk = krylov_chunk(n);
    const size_t k0 = (size_t)blockIdx.x * chunk;
    const size_t k1 = k0 + chunk < n ? k0 + chunk : n;
    double acc = 0.0;
    for (size_t k = k0 + threadIdx.x; k < k1; k += BS) {
        double s = 0.0;
        for (int i0 = 0; i0 < J; i0 += 8) {
            double m[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) m[u] = (i0 + u < J) ? V[(size_t)(i0 + u) * ldv + k] : 0.0;
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (i0 + u < J) s += m[u] * h2[i0 + u];
        }
        const double wn = w[k] - s;
        w[k] = wn;
        acc += wn * wn;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < BS / 64; ++q) t += red[q];
        part[blockIdx.x] = t;
    }
}

// ---- delayed CGS2 (DCGS2) Arnoldi -------------------------------------------------------------
// One sweep of inner products per step: columns 0..J-1 of V against one or two staged
// vectors x1, x2 (the not yet reorthogonalised vt_j and wt = B vt_j). Rows [0, J) of part
// hold the partial dots with x1, rows [J, 2J) those with x2.
template <int NRHS>
__global__ __launch_bounds__(BS) void k_multidot2(const double* __restrict__ V, size_t ldv, int J,
                                                  const double* __restrict__ x1, const double* __restrict__ x2,
                                                  size_t n, double* __restrict__ part, int nblk, const int* skip) {
    if (skip && *skip) return;
    __shared__ double xs[NRHS][CHUNK];
    const int chunk = krylov_chunk(n);
    const size_t k0 = (size_t)blockIdx.x * chunk;
    const int len = (int)(k0 + chunk < n ? chunk : n - k0);
    for (int k = threadIdx.x; k < len; k += BS) {
        xs[0][k] = x1[k0 + k];
        if (NRHS == 2) xs[NRHS - 1][k] = x2[k0 + k];
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    typedef double d2 __attribute__((ext_vector_type(2)));
    constexpr int U = 4;
    for (int i = wave; i < J; i += BS / 64) {
        const double* v = V + (size_t)i * ldv + k0;
        double acc1 = 0.0, acc2 = 0.0;
        // two consecutive entries per lane (16-byte loads); len is even except at the vector's end
        for (int k = 2 * lane; k < len; k += 128 * U) {
            d2 m[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int kk = k + 128 * u;
                if (kk + 1 < len) m[u] = *reinterpret_cast<const d2*>(v + kk);
                else { m[u].x = kk < len ? v[kk] : 0.0; m[u].y = 0.0; }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int kk = k + 128 * u;
                if (kk < len) {
                    acc1 += m[u].x * xs[0][kk];
                    if (NRHS == 2) acc2 += m[u].x * xs[NRHS - 1][kk];
                }
                if (kk + 1 < len) {
                    acc1 += m[u].y * xs[0][kk + 1];
                    if (NRHS == 2) acc2 += m[u].y * xs[NRHS - 1][kk + 1];
                }
            }
        }
        acc1 = wave_sum(acc1);
        if (NRHS == 2) acc2 = wave_sum(acc2);
        if (lane == 0) {
            part[(size_t)i * nblk + blockIdx.x] = acc1;
            if (NRHS == 2) part[(size_t)(J + i) * nblk + blockIdx.x] = acc2;
        }
    }
}

// Step j of the delayed CGS2 Arnoldi process, one block. It first adds up the sweep's block
// partials (part[i*nblk + b]) into the inner products d: d[i] = V_i . vt_j (i <= j; i < j is
// the delayed projection a, i = j is alpha) and d[J + i] = V_i . wt (c, gamma), J = j + 1. rho = sqrt(alpha - a.a) normalises
// the reorthogonalised v_j; column j-1 of the unrotated Hessenberg Hu gains a and rho and
// is then rotated into H (Givens, residual estimate). Unless finish, the new column
//     h = ([c; (gamma - a.c)/rho] - t)/rho,  t = Hu[:j+1, :j] a,
// goes to Hu, and coef receives what the update sweep needs: a (j values) at coef[0..],
// b = t/rho + h (j+1 values) at coef[ldc..], 1/rho at coef[2 ldc].
__global__ __launch_bounds__(COEF_BS) void k_dcgs2_coef(GmresCtl* ctl, const double* __restrict__ part, int nblk,
                                                        int j, int finish, double* Hu, double* H, int ldh,
                                                        double* cs, double* sn, double* g, double* coef, int ldc,
                                                        double* hist, int hs_ld) {
    if (ctl->done) return;
    extern __shared__ double hstage[];  // (j-1) x hs_ld when hs_ld > 0
    __shared__ double ds[2 * 201];      // restart lengths up to 200
    __shared__ double tsh[201];
    __shared__ double hcol[202];        // column j-1 of Hu (rows 0..j)
    __shared__ double css[201], sns[201];
    __shared__ double sh_rho;
    __shared__ int sh_stop;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int J = j + 1;
    // the block partials of the inner-product sweep, one wave per sum (each lane adds its
    // blocks in increasing order), three sums per pass so that each lane has 36 loads in
    // flight, and everything the serial part needs
    const int nout = finish ? J : 2 * J;
    constexpr int NW = COEF_BS / 64, CS = 3, CU = 12;
    for (int i0 = wave; i0 < nout; i0 += CS * NW) {
        double acc[CS];
#pragma unroll
        for (int q = 0; q < CS; ++q) acc[q] = 0.0;
        for (int b0 = 0; b0 < nblk; b0 += CU * 64) {
            double m[CS][CU];
#pragma unroll
            for (int q = 0; q < CS; ++q) {
                const int i = i0 + q * NW;
                const double* pi = part + (size_t)(i < nout ? i : i0) * nblk;
#pragma unroll
                for (int u = 0; u < CU; ++u) {
                    const int b = b0 + 64 * u + lane;
                    m[q][u] = b < nblk ? pi[b] : 0.0;
                }
            }
#pragma unroll
            for (int q = 0; q < CS; ++q)
#pragma unroll
                for (int u = 0; u < CU; ++u) acc[q] += m[q][u];
        }
#pragma unroll
        for (int q = 0; q < CS; ++q) {
            const double sacc = wave_sum(acc[q]);
            const int i = i0 + q * NW;
            if (lane == 0 && i < nout) ds[i] = sacc;
        }
    }
    // columns 0..j-2 of Hu (rows 0..j) staged in LDS when they fit (hs_ld = j+1, else 0)
    if (hs_ld > 0) {
        for (int idx = tid; idx < (j - 1) * hs_ld; idx += COEF_BS) {
            const int q = idx / hs_ld;
            hstage[idx] = Hu[(size_t)q * ldh + (idx - q * hs_ld)];
        }
    }
    if (j > 0 && wave == 0) {
        for (int i = lane; i < j; i += 64) {
            hcol[i] = Hu[(size_t)(j - 1) * ldh + i];
            css[i] = cs[i];
            sns[i] = sn[i];
        }
    }
    __syncthreads();
    double rho = 0.0, ac = 0.0;
    if (wave == 0) {
        double aa = 0.0;
        for (int i = lane; i < j; i += 64) {
            aa += ds[i] * ds[i];
            if (!finish) ac += ds[i] * ds[J + i];
        }
        aa = wave_sum(aa);
        ac = wave_sum(ac);
        // delayed pass for column j-1: Hu[:j, j-1] += a, Hu[j, j-1] = rho
        const double r2 = ds[j] - aa;
        rho = r2 > 0.0 ? sqrt(r2) : 0.0;
        if (j > 0) {
            for (int i = lane; i < j; i += 64) {
                hcol[i] += ds[i];
                Hu[(size_t)(j - 1) * ldh + i] = hcol[i];
            }
            if (lane == 0) {
                hcol[j] = rho;
                Hu[(size_t)(j - 1) * ldh + j] = rho;
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        int stop = 0;
        if (j > 0) {
            // Givens: previous rotations, a new one, the residual estimate (column j-1)
            const int c0 = j - 1;
            double* col = H + (size_t)c0 * ldh;
            double hprev = hcol[0];
            for (int i = 0; i < c0; ++i) {
                const double hn = hcol[i + 1];
                const double t = css[i] * hprev + sns[i] * hn;
                col[i] = t;
                hprev = -sns[i] * hprev + css[i] * hn;
            }
            const double hjj = hprev, hn = hcol[c0 + 1];
            double c = 1.0, sg = 0.0;
            if (hn != 0.0) {
                const double r = hypot(hjj, hn);
                c = hjj / r;
                sg = hn / r;
            }
            cs[c0] = c;
            sn[c0] = sg;
            col[c0] = c * hjj + sg * hn;
            col[c0 + 1] = 0.0;
            const double gj = g[c0];
            g[c0 + 1] = -sg * gj;
            g[c0] = c * gj;
            const double est = fabs(g[c0 + 1]);
            ctl->est = est;
            ctl->k = j;
            if (hist) hist[c0] = est;
            if (!isfinite(est) || !isfinite(col[c0])) ctl->nonfinite = 1;
            if (est <= ctl->target || !isfinite(est)) stop = 1;
        }
        if (!(rho > 0.0) || !isfinite(rho)) stop = 1;   // breakdown: the space is invariant
        if (finish) stop = 1;
        if (stop) ctl->done = 1;
        sh_rho = rho;
        sh_stop = stop;
    }
    __syncthreads();
    if (sh_stop) return;
    if (wave != 0) return;     // the rest is one wave's work (no barriers below)
    const double irho = 1.0 / sh_rho;
    // t = Hu[:j+1, :j] a over the Hessenberg pattern (row i has entries in columns q >= i-1
    // only; nothing below the subdiagonal is ever read): column j-1 from LDS, the others
    // read eight at a time
    for (int i = lane; i <= j; i += 64) {
        double t = 0.0;
        const int qe = j - 1;
        for (int q0 = i > 0 ? i - 1 : 0; q0 < qe; q0 += 8) {
            double m[8];
            if (hs_ld > 0) {
#pragma unroll
                for (int u = 0; u < 8; ++u) m[u] = hstage[(q0 + u < qe ? q0 + u : q0) * hs_ld + i];
            } else {
#pragma unroll
                for (int u = 0; u < 8; ++u) m[u] = Hu[(size_t)(q0 + u < qe ? q0 + u : q0) * ldh + i];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q0 + u < qe) t += m[u] * ds[q0 + u];
        }
        if (j > 0 && i <= j) t += hcol[i] * ds[j - 1];
        tsh[i] = t;
    }
    // (each lane reads back only the tsh entries it wrote)
    for (int i = lane; i <= j; i += 64) {
        const double ci = i < j ? ds[J + i] : (ds[J + j] - ac) * irho;
        const double h = (ci - tsh[i]) * irho;
        Hu[(size_t)j * ldh + i] = h;
        coef[ldc + i] = tsh[i] * irho + h;
        if (i < j) coef[i] = ds[i];
    }
    if (lane == 0) coef[2 * ldc] = irho;
}

// The update sweep of step j, one read of V_0..V_{j-1}:
//     v_j = (vt_j - V_{<j} a) / rho           (written over vt_j),
//     vt_{j+1} = wt / rho - V_{<j} b_{<j} - v_j b_j   (written over wt).
// Two consecutive entries per thread (16-byte loads), eight columns in flight.
__global__ __launch_bounds__(BS) void k_dcgs2_update(const double* __restrict__ V, size_t ldv, int j,
                                                     double* vj, double* wt, const double* __restrict__ coef,
                                                     int ldc, size_t n, const int* skip) {
    if (skip && *skip) return;
    const size_t k = 2 * ((size_t)blockIdx.x * BS + threadIdx.x);
    if (k >= n) return;
    const double* a = coef;
    const double* b = coef + ldc;
    const double irho = coef[2 * ldc];
    if (k + 1 >= n) {      // odd tail entry
        double s1 = 0.0, s2 = 0.0;
        for (int i = 0; i < j; ++i) {
            const double m = V[(size_t)i * ldv + k];
            s1 += m * a[i];
            s2 += m * b[i];
        }
        const double v = (vj[k] - s1) * irho;
        vj[k] = v;
        wt[k] = wt[k] * irho - s2 - v * b[j];
        return;
    }
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 vt = *reinterpret_cast<const d2*>(vj + k);
    const d2 w = *reinterpret_cast<const d2*>(wt + k);
    double s1x = 0.0, s1y = 0.0, s2x = 0.0, s2y = 0.0;
    for (int i0 = 0; i0 < j; i0 += 8) {
        d2 m[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            m[u] = *reinterpret_cast<const d2*>(V + (size_t)(i0 + u < j ? i0 + u : 0) * ldv + k);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + u < j) {
                s1x += m[u].x * a[i0 + u];
                s1y += m[u].y * a[i0 + u];
                s2x += m[u].x * b[i0 + u];
                s2y += m[u].y * b[i0 + u];
            }
    }
    d2 v, o;
    v.x = (vt.x - s1x) * irho;
    v.y = (vt.y - s1y) * irho;
    o.x = w.x * irho - s2x - v.x * b[j];
    o.y = w.y * irho - s2y - v.y * b[j];
    *reinterpret_cast<d2*>(vj + k) = v;
    *reinterpret_cast<d2*>(wt + k) = o;
}

}  // namespace

hdg_status vec_axpy_dot(hdg_ctx ctx, const double* V, size_t ldv, int J, const double* h1, double* w, size_t n,
                        double* part, int nblk, const int* skip) {
    if (J <= 8)
        hipLaunchKernelGGL(k_axpy_dot<8>, dim3(nblk), dim3(BS), 0, ctx->stream, V, ldv, J, h1, w, n, part, nblk, skip);
    else if (J <= 16)
        hipLaunchKernelGGL(k_axpy_dot<16>, dim3(nblk), dim3(BS), 0, ctx->stream, V, ldv, J, h1, w, n, part, nblk, skip);
    else if (J <= 32)
        hipLaunchKernelGGL(k_axpy_dot<32>, dim3(nblk), dim3(BS), 0, ctx->stream, V, ldv, J, h1, w, n, part, nblk, skip);
    else
        hipLaunchKernelGGL(k_axpy_dot<64>, dim3(nblk), dim3(BS), 0, ctx->stream, V, ldv, J, h1, w, n, part, nblk, skip);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status vec_axpy_sumsq(hdg_ctx ctx, const double* V, size_t ldv, int J, const double* h2, double* w, size_t n,
                          double* part, int nblk, const int* skip) {
    if (J <= 16)
        hipLaunchKernelGGL(k_axpy_sumsq<16>, dim3(nblk), dim3(BS), 0, ctx->stream, V, ldv, J, h2, w, n, part, nblk, skip);
    else if (J <= 32)
        hipLaunchKernelGGL(k_axpy_sumsq<32>, dim3(nblk), dim3(BS), 0, ctx->stream, V, ldv, J, h2, w, n, part, nblk, skip);
    else
        hipLaunchKernelGGL(k_axpy_sumsq<64>, dim3(nblk), dim3(BS), 0, ctx->stream, V, ldv, J, h2, w, n, part, nblk, skip);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status vec_multidot2(hdg_ctx ctx, const double* V, size_t ldv, int J, const double* x1, const double* x2,
                         size_t n, double* part, int nblk, const int* skip) {
    if (J <= 0) return HDG_OK;
    hipEvent_t es, ee;
    take_ext_events(ctx, &es, &ee);
    if (es || ee) {
        if (x2)
            hipExtLaunchKernelGGL(k_multidot2<2>, dim3(nblk), dim3(BS), 0, ctx->stream, es, ee, 0, V, ldv, J, x1, x2,
                                  n, part, nblk, skip);
        else
            hipExtLaunchKernelGGL(k_multidot2<1>, dim3(nblk), dim3(BS), 0, ctx->stream, es, ee, 0, V, ldv, J, x1, x2,
                                  n, part, nblk, skip);
    } else if (x2) {
        hipLaunchKernelGGL(k_multidot2<2>, dim3(nblk), dim3(BS), 0, ctx->stream, V, ldv, J, x1, x2, n, part, nblk,
                           skip);
    } else {
        hipLaunchKernelGGL(k_multidot2<1>, dim3(nblk), dim3(BS), 0, ctx->stream, V, ldv, J, x1, x2, n, part, nblk,
                           skip);
    }
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status krylov_dcgs2_coef(hdg_ctx ctx, GmresCtl* ctl, const double* part, int nblk, int j, int finish, double* Hu,
                             double* H, int ldh, double* cs, double* sn, double* g, double* coef, int ldc,
                             double* hist) {
    // the columns of Hu the new column's product reads go through LDS when they fit in 48 KiB
    const int hs_ld = (j >= 2 && (size_t)(j - 1) * (j + 1) * sizeof(double) <= 48 * 1024) ? j + 1 : 0;
    const size_t lds = hs_ld ? (size_t)(j - 1) * hs_ld * sizeof(double) : 0;
    hipLaunchKernelGGL(k_dcgs2_coef, dim3(1), dim3(COEF_BS), lds, ctx->stream, ctl, part, nblk, j, finish, Hu, H, ldh,
                       cs, sn, g, coef, ldc, hist, hs_ld);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status vec_dcgs2_update(hdg_ctx ctx, const double* V, size_t ldv, int j, double* vj, double* wt,
                            const double* coef, int ldc, size_t n, const int* skip) {
    // two entries per thread: vj, wt and the columns of V must be 16-byte aligned (the basis
    // columns start at multiples of ldv, a multiple of 64 doubles)
    hipEvent_t es, ee;
    take_ext_events(ctx, &es, &ee);
    const dim3 grid(div_up((long long)(n + 1) / 2, BS));
    if (es || ee)
        hipExtLaunchKernelGGL(k_dcgs2_update, grid, dim3(BS), 0, ctx->stream, es, ee, 0, V, ldv, j, vj, wt, coef, ldc,
                              n, skip);
    else
        hipLaunchKernelGGL(k_dcgs2_update, grid, dim3(BS), 0, ctx->stream, V, ldv, j, vj, wt, coef, ldc, n, skip);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status vec_multidot(hdg_ctx ctx, const double* V, size_t ldv, int J, const double* w, size_t n,
                        double* part, int nblk, const int* skip) {
    if (J <= 0) return HDG_OK;
    hipLaunchKernelGGL(k_multidot<8>, dim3(nblk), dim3(BS), 0, ctx->stream, V, ldv, J, w, n, part, nblk, skip);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status vec_reduce(hdg_ctx ctx, const double* part, int J, int nblk, double* out, double* add_to,
                      const int* skip) {
    if (J <= 0) return HDG_OK;
    hipLaunchKernelGGL(k_reduce, dim3(div_up(J, 4)), dim3(256), 0, ctx->stream, part, J, nblk, out, add_to, skip);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status vec_multiaxpy(hdg_ctx ctx, const double* V, size_t ldv, int J, const double* h, double sign,
                         double* w, size_t n, const int* skip, const int* J_dev) {
    if ((J <= 0 && !J_dev) || n == 0) return HDG_OK;
    hipLaunchKernelGGL(k_multiaxpy, dim3(div_up((long long)n, BS)), dim3(BS), 0, ctx->stream, V, ldv, J, h, sign,
                       w, n, skip, J_dev);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status vec_sumsq_partial(hdg_ctx ctx, const double* w, size_t n, double* part, int nblk, const int* skip) {
    hipLaunchKernelGGL(k_sumsq, dim3(nblk), dim3(BS), 0, ctx->stream, w, n, part, nblk, skip);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status vec_lincomb(hdg_ctx ctx, size_t n, double* out, double a, const double* X, double b,
                       const double* Y, const int* skip) {
    if (n == 0) return HDG_OK;
    hipLaunchKernelGGL(k_lincomb, dim3(div_up((long long)n, BS)), dim3(BS), 0, ctx->stream, n, out, a, X, b, Y,
                       skip);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status krylov_cycle_init(hdg_ctx ctx, GmresCtl* ctl, const double* part, int nblk, double* g, int jmax,
                             double target) {
    hipLaunchKernelGGL(k_cycle_init, dim3(1), dim3(64), 0, ctx->stream, ctl, part, nblk, g, jmax, target);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status krylov_scale_by(hdg_ctx ctx, double* v, const double* src, size_t n, const double* denom,
                           const int* skip) {
    hipLaunchKernelGGL(k_scale_by, dim3(div_up((long long)n, BS)), dim3(BS), 0, ctx->stream, v, src, n, denom,
                       skip);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status krylov_givens(hdg_ctx ctx, GmresCtl* ctl, const double* part, int nblk, double* H, int ldh,
                         double* cs, double* sn, double* g, int j, double* hist) {
    hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, ctx->stream, ctl, part, nblk, H, ldh, cs, sn, g, j, hist);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status krylov_backsolve(hdg_ctx ctx, const GmresCtl* ctl, const double* H, int ldh, const double* g,
                            double* y) {
    if (ldh - 1 > 256) {
        ctx->err = "back substitution: Krylov dimension above 256";
        return HDG_ERR_ARG;
    }
    hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(BACKSOLVE_BS), 0, ctx->stream, ctl, H, ldh, g, y);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status krylov_store_norm(hdg_ctx ctx, const double* part, int nblk, double* dst) {
    hipLaunchKernelGGL(k_store_norm, dim3(1), dim3(64), 0, ctx->stream, part, nblk, dst);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}
