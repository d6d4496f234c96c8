// Batched independent instances (many small uneven meshes, degrees and element
// types in one set of launches): condensation in one persistent launch with the
// whole element system in LDS, face-parallel assembly, a face-block operator
// whose faces carry their instance's block size, and segmented Krylov kernels
// with per-instance reductions, Givens updates and convergence masks.
//
// The arithmetic per element/face/instance is the same as in the single-instance
// kernels (Section 4.1 eq. w15-w19, Section 4.2 eq. w21-w22, Section 4.3-4.5);
// only the indexing differs: every element, face and vector entry looks up its
// instance descriptor.
#include <cmath>

#include "hdg_batch.hpp"

namespace {

constexpr int BS = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---- condensation: one element per workgroup iteration, all in LDS ------------------------
__global__ __launch_bounds__(BS) void k_batch_condense(const InstDesc* __restrict__ desc,
                                                       const int32_t* __restrict__ eid, int64_t total_ne,
                                                       BatchElemPtrs in, double* __restrict__ Kbar,
                                                       double* __restrict__ rbar, double* __restrict__ local,
                                                       int* bad_elem) {
    extern __shared__ double sm[];
    __shared__ int pidx;
    __shared__ double pval;
    for (int64_t g = blockIdx.x; g < total_ne; g += gridDim.x) {
        const InstDesc& q = desc[eid[g]];
        const int64_t le = g - q.e0;
        const int P = q.P, D = q.D, M = q.M, PF = q.PF, L = q.L;
        const int nu = q.nu, nq = q.nq, nt = q.nt, R = q.R, C = q.C, NW = q.NW, KD = q.KD, LPF = L * PF;
        double* T = sm;                        // R x C (row stride C)
        double* W = sm + (size_t)R * C;        // KD x NW
        const double* Mi = in.Minv + q.off[0] + le * P * P;
        const double* Bd = in.Bd + q.off[1] + le * D * P * P;
        const double* Cd = in.Cd + q.off[2] + le * D * P * LPF;
        const double* Dm = in.D + q.off[3] + le * nu * nq;
        const double* Em = in.E + q.off[4] + le * nu * nu;
        const double* Fm = in.F + q.off[5] + le * nu * nt;
        const double* Gm = in.G + q.off[6] + le * nt * nq;
        const double* Hm = in.H + q.off[7] + le * nt * nu;
        const double* Jm = in.J + q.off[8] + le * nt * nt;
        const double* ru = in.ru + q.off[9] + le * nu;
        const double* rt = in.rt + q.off[10] + le * nt;
        // W = Minv [B_d | C_d]
        for (int idx = threadIdx.x; idx < KD * NW; idx += BS) {
            const int r = idx / NW, c = idx - r * NW;
            const int d = r / P, i = r - d * P;
            double acc = 0.0;
            for (int k = 0; k < P; ++k) {
                const double b = c < P ? Bd[((size_t)d * P + k) * P + c] : Cd[((size_t)d * P + k) * LPF + (c - P)];
                acc += Mi[(size_t)i * P + k] * b;
            }
            W[idx] = acc;
        }
        __syncthreads();
        // T = T0 - X W  column-mapped per component
        for (int idx = threadIdx.x; idx < R * (nu + nt); idx += BS) {
            const int r = idx / (nu + nt), tcol = idx - r * (nu + nt);
            int m, c;
            if (tcol < nu) {
                m = tcol / P;
                c = tcol - m * P;
            } else {
                const int t2 = tcol - nu, l = t2 / (M * PF), rem = t2 - l * M * PF;
                m = rem / PF;
                c = P + l * PF + (rem - m * PF);
            }
            const double* X = r < nu ? Dm + (size_t)r * nq : Gm + (size_t)(r - nu) * nq;
            double acc = 0.0;
            for (int kk = 0; kk < KD; ++kk) acc += X[m * KD + kk] * W[(size_t)kk * NW + c];
            double t0;
            if (r < nu) t0 = tcol < nu ? Em[(size_t)r * nu + tcol] : Fm[(size_t)r * nt + (tcol - nu)];
            else t0 = tcol < nu ? Hm[(size_t)(r - nu) * nu + tcol] : Jm[(size_t)(r - nu) * nt + (tcol - nu)];
            T[(size_t)r * C + tcol] = t0 - acc;
        }
        for (int r = threadIdx.x; r < R; r += BS) T[(size_t)r * C + C - 1] = r < nu ? ru[r] : rt[r - nu];
        __syncthreads();
        // eliminate the first nu columns, pivots among the Ebar rows
        bool singular = false;
        for (int k = 0; k < nu; ++k) {
            if (threadIdx.x < 64) {
                double best = -1.0;
                int bi = k;
                for (int i = k + threadIdx.x; i < nu; i += 64) {
                    const double v = fabs(T[(size_t)i * C + k]);
                    if (v > best || (v == best && i < bi)) { best = v; bi = i; }
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    const double ob = __shfl_xor(best, off, 64);
                    const int oi = __shfl_xor(bi, off, 64);
                    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
                }
                if (threadIdx.x == 0) { pidx = bi; pval = T[(size_t)bi * C + k]; }
            }
            __syncthreads();
            const int p = pidx;
            double pv = pval;
            if (!(fabs(pv) > 0.0) || !isfinite(pv)) { singular = true; pv = 1.0; }
            if (p != k)
                for (int c = k + threadIdx.x; c < C; c += BS) {
                    const double t = T[(size_t)k * C + c];
                    T[(size_t)k * C + c] = T[(size_t)p * C + c];
                    T[(size_t)p * C + c] = t;
                }
            __syncthreads();
            const double inv = 1.0 / pv;
            for (int i = k + 1 + threadIdx.x; i < R; i += BS) T[(size_t)i * C + k] *= inv;
            __syncthreads();
            const int w = C - k - 1;
            for (int idx = threadIdx.x; idx < (R - k - 1) * w; idx += BS) {
                const int i = k + 1 + idx / w, c = k + 1 + idx % w;
                T[(size_t)i * C + c] -= T[(size_t)i * C + k] * T[(size_t)k * C + c];
            }
            __syncthreads();
        }
        if (singular && threadIdx.x == 0) atomicMin(bad_elem, (int)g);
        double* lo = local + q.local_off + le * nu * C;
        for (int idx = threadIdx.x; idx < nu * C; idx += BS) lo[idx] = T[idx];
        double* Ko = Kbar + q.kbar_off + le * nt * nt;
        for (int idx = threadIdx.x; idx < nt * nt; idx += BS) {
            const int i = idx / nt, j = idx - i * nt;
            Ko[idx] = T[(size_t)(nu + i) * C + nu + j];
        }
        for (int i = threadIdx.x; i < nt; i += BS) rbar[q.rbar_off + le * nt + i] = T[(size_t)(nu + i) * C + C - 1];
        __syncthreads();
    }
}

// ---- assembly --------------------------------------------------------------------------------
__global__ __launch_bounds__(BS) void k_batch_assemble(const InstDesc* __restrict__ desc,
                                                       const int32_t* __restrict__ fid, int64_t total_nf,
                                                       const int32_t* __restrict__ f2e, const int32_t* __restrict__ e2f,
                                                       const double* __restrict__ Kbar, const double* __restrict__ rbar,
                                                       double* __restrict__ K64, float* __restrict__ K32,
                                                       int32_t* __restrict__ nbr, double* __restrict__ r) {
    __shared__ int se[16], slr[16], slc[16];
    for (int64_t g = blockIdx.x; g < total_nf; g += gridDim.x) {
        const InstDesc& q = desc[fid[g]];
        const int64_t f = g - q.f0;
        const int M = q.M, PF = q.PF, L = q.L, nb = q.nb, S = q.S, nt = q.nt;
        const int32_t* f2 = f2e + q.f2e_off + 4 * f;
        const int e1 = f2[0], l1 = f2[1], e2 = f2[2], l2 = f2[3];
        if (threadIdx.x == 0) {
            int s = 0;
            se[s] = e1; slr[s] = l1; slc[s] = l1; ++s;
            for (int l = 0; l < L; ++l)
                if (l != l1) { se[s] = e1; slr[s] = l1; slc[s] = l; ++s; }
            for (int l = 0; l < L; ++l) {
                if (e2 >= 0) {
                    if (l != l2) { se[s] = e2; slr[s] = l2; slc[s] = l; ++s; }
                } else if (l != 0) {
                    se[s] = -1; slr[s] = 0; slc[s] = 0; ++s;
                }
            }
        }
        __syncthreads();
        for (int s = threadIdx.x; s < S; s += BS) {
            int gg = -1;
            if (s == 0) gg = (int)f;
            else if (se[s] >= 0) gg = e2f[q.e2f_off + (int64_t)se[s] * L + slc[s]];
            nbr[q.nbr_off + f * S + s] = gg;
        }
        const int64_t blk = (int64_t)nb * nb;
        for (int s = 0; s < S; ++s) {
            const int e = se[s];
            double* out = K64 + q.K_off + (f * S + s) * blk;
            float* out32 = K32 ? K32 + q.K_off + (f * S + s) * blk : nullptr;
            for (int idx = threadIdx.x; idx < (int)blk; idx += BS) {
                const int c = idx / nb, rr = idx - c * nb;
                double v = 0.0;
                if (e >= 0) {
                    const int mr = rr / PF, jr = rr - mr * PF, mc = c / PF, jc = c - mc * PF;
                    const double* Ke = Kbar + q.kbar_off + (int64_t)e * nt * nt;
                    v = Ke[(int64_t)((slr[s] * M + mr) * PF + jr) * nt + (slc[s] * M + mc) * PF + jc];
                    if (s == 0 && e2 >= 0) {
                        const double* K2 = Kbar + q.kbar_off + (int64_t)e2 * nt * nt;
                        v += K2[(int64_t)((l2 * M + mr) * PF + jr) * nt + (l2 * M + mc) * PF + jc];
                    }
                }
                out[idx] = v;
                if (out32) out32[idx] = (float)v;
            }
        }
        for (int rr = threadIdx.x; rr < nb; rr += BS) {
            const int m = rr / PF, j = rr - m * PF;
            double v = rbar[q.rbar_off + (int64_t)e1 * nt + (l1 * M + m) * PF + j];
            if (e2 >= 0) v += rbar[q.rbar_off + (int64_t)e2 * nt + (l2 * M + m) * PF + j];
            r[q.vec_off + f * nb + rr] = v;
        }
        __syncthreads();
    }
}

// ---- face-block operator -----------------------------------------------------------------------
// u_f = sum_s M1[f][s] x_{nbr[f][s]} (or the block-diagonal product when bj_only), then
// out_f = s0 u_f + a0 X_f (X may be null); faces of finished instances are skipped.
template <typename T>
__global__ __launch_bounds__(BS) void k_batch_face(const InstDesc* __restrict__ desc,
                                                   const int32_t* __restrict__ fid, int64_t total_nf,
                                                   const T* __restrict__ M1, const int32_t* __restrict__ nbr,
                                                   int bj_only, const double* __restrict__ x, double* out,
                                                   double s0, const double* X, double a0,
                                                   const BatchCtl* ctl) {
    constexpr int TEAM = 32, FPB = BS / TEAM;
    extern __shared__ double sm[];
    const int team = threadIdx.x / TEAM, t = threadIdx.x % TEAM;
    const int64_t g = (int64_t)blockIdx.x * FPB + team;
    const bool valid = g < total_nf;
    int inst = valid ? fid[g] : 0;
    const InstDesc& q = desc[inst];
    const bool live = valid && !(ctl && ctl[inst].done);
    const int nb = q.nb, S = bj_only ? 1 : q.S;
    const int64_t f = g - q.f0;
    double* xs = sm + (size_t)team * 64;       // S*nb <= 64 per face
    double* red = sm + (size_t)FPB * 64;
    int Seff = S;
    if (live && !bj_only && S > q.L && nbr[q.nbr_off + f * S + q.L] < 0) Seff = q.L;
    const int ncols = Seff * nb;
    if (live)
        for (int i = t; i < ncols; i += TEAM) {
            const int s = i / nb, c = i - s * nb;
            const int64_t gg = bj_only ? f : nbr[q.nbr_off + f * S + s];
            xs[i] = x[q.vec_off + gg * nb + c];
        }
    __syncthreads();
    const int G = TEAM / nb, grp = t / nb, row = t - grp * nb;
    double acc = 0.0;
    if (live && grp < G) {
        const T* Mf = M1 + (bj_only ? q.binv_off : q.K_off) + f * S * nb * nb;
        for (int k = grp; k < ncols; k += G) acc += (double)Mf[(int64_t)k * nb + row] * xs[k];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (live && t < nb) {
        double u = 0.0;
        for (int g2 = 0; g2 < G; ++g2) u += red[team * TEAM + g2 * nb + t];
        const int64_t idx = q.vec_off + f * nb + t;
        double v = s0 * u;
        if (X) v += a0 * X[idx];
        out[idx] = v;
    }
}

// ---- block-Jacobi inverses (Gauss-Jordan, partial pivoting), one face per workgroup -------------
__global__ __launch_bounds__(BS) void k_batch_bj(const InstDesc* __restrict__ desc, const int32_t* __restrict__ fid,
                                                 int64_t total_nf, const double* __restrict__ K, double* B64,
                                                 float* B32, int* bad_face) {
    __shared__ double A[16 * 33];
    __shared__ int ps;
    for (int64_t g = blockIdx.x; g < total_nf; g += gridDim.x) {
        const InstDesc& q = desc[fid[g]];
        const int64_t f = g - q.f0;
        const int nb = q.nb, lda = 2 * nb + 1;
        const double* Kf = K + q.K_off + f * q.S * nb * nb;
        for (int idx = threadIdx.x; idx < nb * nb; idx += BS) {
            const int c = idx / nb, r = idx - c * nb;
            A[r * lda + c] = Kf[idx];
            A[r * lda + nb + c] = (r == c) ? 1.0 : 0.0;
        }
        __syncthreads();
        bool singular = false;
        for (int k = 0; k < nb; ++k) {
            if (threadIdx.x == 0) {
                int p = k;
                for (int r = k + 1; r < nb; ++r)
                    if (fabs(A[r * lda + k]) > fabs(A[p * lda + k])) p = r;
                ps = p;
            }
            __syncthreads();
            const int p = ps;
            if (p != k)
                for (int c = threadIdx.x; c < 2 * nb; c += BS) {
                    const double t = A[k * lda + c];
                    A[k * lda + c] = A[p * lda + c];
                    A[p * lda + c] = t;
                }
            __syncthreads();
            double pv = A[k * lda + k];
            if (!(fabs(pv) > 0.0) || !isfinite(pv)) { singular = true; pv = 1.0; }
            __syncthreads();
            for (int c = threadIdx.x; c < 2 * nb; c += BS) A[k * lda + c] /= pv;
            __syncthreads();
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
        if (singular && threadIdx.x == 0) atomicMin(bad_face, (int)g);
        for (int idx = threadIdx.x; idx < nb * nb; idx += BS) {
            const int c = idx / nb, r = idx - c * nb;
            B64[q.binv_off + f * nb * nb + idx] = A[r * lda + nb + c];
            if (B32) B32[q.binv_off + f * nb * nb + idx] = (float)A[r * lda + nb + c];
        }
        __syncthreads();
    }
}

// ---- segmented Krylov kernels -------------------------------------------------------------------
// Block b covers entries [blk_lo[b], blk_hi[b]) of instance blk_inst[b] (chunks never straddle
// two instances). part[i * nblk + b].
__global__ __launch_bounds__(BS) void k_seg_multidot(const int32_t* __restrict__ blk_inst,
                                                     const int64_t* __restrict__ blk_lo, const int64_t* __restrict__ blk_hi,
                                                     const double* __restrict__ V, size_t ldv, int J,
                                                     const double* __restrict__ w, double* part, int nblk,
                                                     const BatchCtl* ctl) {
    __shared__ double red[64][BS / 64];
    const int b = blockIdx.x;
    if (ctl && ctl[blk_inst[b]].done) return;
    const int64_t k0 = blk_lo[b], k1 = blk_hi[b];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i0 = 0; i0 < J; i0 += 64) {
        const int ni = (J - i0) < 64 ? (J - i0) : 64;
        for (int ii = 0; ii < ni; ++ii) {
            const double* v = V + (size_t)(i0 + ii) * ldv;
            double acc = 0.0;
            for (int64_t k = k0 + threadIdx.x; k < k1; k += BS) acc += v[k] * w[k];
            acc = wave_sum(acc);
            if (lane == 0) red[ii][wave] = acc;
        }
        __syncthreads();
        if (threadIdx.x < ni) {
            double s = 0.0;
            for (int q = 0; q < BS / 64; ++q) s += red[threadIdx.x][q];
            part[(size_t)(i0 + threadIdx.x) * nblk + b] = s;
        }
        __syncthreads();
    }
}

// out[inst * ldo + i] (= or +=) sum of part[i][b] over the instance's blocks; one wave per (inst, i)
__global__ void k_seg_reduce(const int32_t* __restrict__ ib0, const int32_t* __restrict__ ib1, int n_inst,
                             const double* __restrict__ part, int J, int nblk, double* out, int ldo, int add,
                             double* copy_to, int ldc, const BatchCtl* ctl) {
    const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= n_inst * J) return;
    const int inst = w / J, i = w - inst * J;
    if (ctl && ctl[inst].done) return;
    double s = 0.0;
    for (int b = ib0[inst] + lane; b < ib1[inst]; b += 64) s += part[(size_t)i * nblk + b];
    s = wave_sum(s);
    if (lane == 0) {
        if (copy_to) copy_to[(size_t)inst * ldc + i] = s;
        if (add) out[(size_t)inst * ldo + i] += s;
        else out[(size_t)inst * ldo + i] = s;
    }
}

// w[k] += sign * sum_{i<J} V[i][k] h[inst(k)][i], J = Jdev[inst] when given
__global__ __launch_bounds__(BS) void k_seg_multiaxpy(const int32_t* __restrict__ dof_inst, const double* V,
                                                      size_t ldv, int J, const double* h, int ldh, double sign,
                                                      double* w, size_t n, const BatchCtl* ctl, int use_kdev) {
    const size_t k = (size_t)blockIdx.x * BS + threadIdx.x;
    if (k >= n) return;
    const int inst = dof_inst[k];
    if (ctl && !use_kdev && ctl[inst].done) return;
    const int JJ = use_kdev ? ctl[inst].k : J;
    const double* hh = h + (size_t)inst * ldh;
    double acc = 0.0;
    for (int i = 0; i < JJ; ++i) acc += V[(size_t)i * ldv + k] * hh[i];
    w[k] += sign * acc;
}

__global__ __launch_bounds__(BS) void k_seg_sumsq(const int32_t* __restrict__ blk_inst,
                                                  const int64_t* __restrict__ blk_lo, const int64_t* __restrict__ blk_hi,
                                                  const double* __restrict__ w, double* part, const BatchCtl* ctl) {
    __shared__ double red[BS / 64];
    const int b = blockIdx.x;
    if (ctl && ctl[blk_inst[b]].done) return;
    double acc = 0.0;
    for (int64_t k = blk_lo[b] + threadIdx.x; k < blk_hi[b]; k += BS) acc += w[k] * w[k];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[b] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(BS) void k_seg_scale(const int32_t* __restrict__ dof_inst, double* v, size_t n,
                                                  const double* denom, int ld_denom, const BatchCtl* ctl) {
    const size_t k = (size_t)blockIdx.x * BS + threadIdx.x;
    if (k >= n) return;
    const int inst = dof_inst[k];
    if (ctl[inst].done) return;
    v[k] /= denom[(size_t)inst * ld_denom];
}

// per instance: beta from the residual partials, cycle state
__global__ void k_seg_cycle_init(const int32_t* __restrict__ ib0, const int32_t* __restrict__ ib1, int n_inst,
                                 const double* part, BatchCtl* ctl, double* g, int ldg, int jmax,
                                 const double* target) {
    const int inst = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (inst >= n_inst) return;
    double s = 0.0;
    for (int b = ib0[inst] + lane; b < ib1[inst]; b += 64) s += part[b];
    s = wave_sum(s);
    if (lane == 0) {
        BatchCtl& c = ctl[inst];
        const double beta = sqrt(s);
        c.beta = beta;
        c.est = beta;
        c.k = 0;
        c.nonfinite = !isfinite(beta);
        c.done = (beta <= target[inst] || !isfinite(beta) || jmax <= 0) ? 1 : 0;
        g[(size_t)inst * ldg] = beta;
    }
}

__global__ void k_seg_givens(const int32_t* __restrict__ ib0, const int32_t* __restrict__ ib1, int n_inst,
                             const double* part, BatchCtl* ctl, double* H, int ldh, int mcols, double* cs,
                             double* sn, double* g, int ldg, int j, int jmax, const double* target) {
    const int inst = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (inst >= n_inst) return;
    BatchCtl& c = ctl[inst];
    if (c.done) return;
    double s = 0.0;
    for (int b = ib0[inst] + lane; b < ib1[inst]; b += 64) s += part[b];
    s = wave_sum(s);
    if (lane != 0) return;
    const double hn = sqrt(s);
    double* Hi = H + (size_t)inst * ldh * mcols;
    double* col = Hi + (size_t)j * ldh;
    double* csi = cs + (size_t)inst * ldg;
    double* sni = sn + (size_t)inst * ldg;
    double* gi = g + (size_t)inst * ldg;
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double t = csi[i] * col[i] + sni[i] * col[i + 1];
        col[i + 1] = -sni[i] * col[i] + csi[i] * col[i + 1];
        col[i] = t;
    }
    const double hjj = col[j];
    double cc = 1.0, sg = 0.0;
    if (hn != 0.0) {
        const double r = hypot(hjj, hn);
        cc = hjj / r;
        sg = hn / r;
    }
    csi[j] = cc;
    sni[j] = sg;
    col[j] = cc * hjj + sg * hn;
    const double gj = gi[j];
    gi[j + 1] = -sg * gj;
    gi[j] = cc * gj;
    const double est = fabs(gi[j + 1]);
    c.est = est;
    c.k = j + 1;
    if (!isfinite(est)) c.nonfinite = 1;
    if (est <= target[inst] || hn == 0.0 || j + 1 >= jmax || !isfinite(est)) c.done = 1;
}

__global__ void k_seg_backsolve(int n_inst, const BatchCtl* ctl, const double* H, int ldh, int mcols,
                                const double* g, int ldg, double* y) {
    const int inst = blockIdx.x * blockDim.x + threadIdx.x;
    if (inst >= n_inst) return;
    const int k = ctl[inst].k;
    const double* Hi = H + (size_t)inst * ldh * mcols;
    const double* gi = g + (size_t)inst * ldg;
    double* yi = y + (size_t)inst * ldg;
    for (int i = k - 1; i >= 0; --i) {
        double s = gi[i];
        for (int c = i + 1; c < k; ++c) s -= Hi[(size_t)c * ldh + i] * yi[c];
        yi[i] = s / Hi[(size_t)i * ldh + i];
    }
}

// ---- recovery ------------------------------------------------------------------------------------
__global__ __launch_bounds__(BS) void k_batch_recover(const InstDesc* __restrict__ desc,
                                                      const int32_t* __restrict__ eid, int64_t total_ne,
                                                      const double* __restrict__ local, const double* __restrict__ Minv,
                                                      const double* __restrict__ Bd, const double* __restrict__ Cd,
                                                      const int32_t* __restrict__ e2f, const double* __restrict__ xhat,
                                                      double* __restrict__ du, double* __restrict__ dq) {
    extern __shared__ double sm[];
    for (int64_t g = blockIdx.x; g < total_ne; g += gridDim.x) {
        const InstDesc& q = desc[eid[g]];
        const int64_t le = g - q.e0;
        const int P = q.P, D = q.D, M = q.M, PF = q.PF, L = q.L, nu = q.nu, nt = q.nt, nb = q.nb, C = q.C;
        const int LPF = L * PF;
        double* xe = sm;
        double* t = xe + nt;
        double* s = t + nu;
        for (int idx = threadIdx.x; idx < nt; idx += BS) {
            const int l = idx / nb, rem = idx - l * nb;
            xe[idx] = xhat[q.vec_off + (int64_t)e2f[q.e2f_off + le * L + l] * nb + rem];
        }
        __syncthreads();
        const double* Le = local + q.local_off + le * nu * C;
        for (int i = threadIdx.x; i < nu; i += BS) {
            const double* row = Le + (size_t)i * C + nu;
            double acc = 0.0;
            for (int k = 0; k < nt; ++k) acc += row[k] * xe[k];
            t[i] = row[nt] - acc;
        }
        __syncthreads();
        for (int i = nu - 1; i >= 0; --i) {
            const double ui = t[i] / Le[(size_t)i * C + i];
            __syncthreads();
            if (threadIdx.x == 0) t[i] = ui;
            for (int k = threadIdx.x; k < i; k += BS) t[k] -= Le[(size_t)k * C + i] * ui;
            __syncthreads();
        }
        for (int i = threadIdx.x; i < nu; i += BS) du[q.du_off + le * nu + i] = t[i];
        const double* Mi = Minv + q.off[0] + le * P * P;
        for (int m = 0; m < M; ++m)
            for (int d = 0; d < D; ++d) {
                const double* B = Bd + q.off[1] + (le * D + d) * P * P;
                const double* Cm = Cd + q.off[2] + (le * D + d) * P * LPF;
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
                    dq[q.dq_off + le * q.nq + (int64_t)(m * D + d) * P + i] = -acc;
                }
                __syncthreads();
            }
        __syncthreads();
    }
}

}  // namespace

// ---- launchers ---------------------------------------------------------------------------------------
hdg_status batch_launch_condense(hdg_ctx ctx, const BatchDev& b, const BatchElemPtrs& in, double* Kbar, double* rbar,
                                 double* local, int* bad, int grid) {
    const size_t lds = sizeof(double) * b.max_cond_lds;
    if (lds > 64 * 1024)
        HDG_HIP_CHECK(ctx, hipFuncSetAttribute((const void*)k_batch_condense,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_batch_condense, dim3(grid), dim3(BS), lds, ctx->stream, b.desc, b.eid, b.total_ne, in, Kbar,
                       rbar, local, bad);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status batch_launch_assemble(hdg_ctx ctx, const BatchDev& b, const int32_t* f2e, const int32_t* e2f,
                                 const double* Kbar, const double* rbar, double* K64, float* K32, int32_t* nbr,
                                 double* r) {
    const int grid = (int)std::min<int64_t>(b.total_nf, 65536);
    hipLaunchKernelGGL(k_batch_assemble, dim3(grid), dim3(BS), 0, ctx->stream, b.desc, b.fid, b.total_nf, f2e, e2f,
                       Kbar, rbar, K64, K32, nbr, r);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status batch_launch_face(hdg_ctx ctx, const BatchDev& b, const void* M1, bool fp32, const int32_t* nbr,
                             bool bj_only, const double* x, double* out, double s0, const double* X, double a0,
                             const BatchCtl* ctl) {
    const int fpb = BS / 32;
    const int grid = (int)((b.total_nf + fpb - 1) / fpb);
    const size_t lds = sizeof(double) * ((size_t)fpb * 64 + BS);
    if (fp32)
        hipLaunchKernelGGL(k_batch_face<float>, dim3(grid), dim3(BS), lds, ctx->stream, b.desc, b.fid, b.total_nf,
                           (const float*)M1, nbr, bj_only ? 1 : 0, x, out, s0, X, a0, ctl);
    else
        hipLaunchKernelGGL(k_batch_face<double>, dim3(grid), dim3(BS), lds, ctx->stream, b.desc, b.fid, b.total_nf,
                           (const double*)M1, nbr, bj_only ? 1 : 0, x, out, s0, X, a0, ctl);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status batch_launch_bj(hdg_ctx ctx, const BatchDev& b, const double* K64, double* B64, float* B32, int* bad) {
    const int grid = (int)std::min<int64_t>(b.total_nf, 65536);
    hipLaunchKernelGGL(k_batch_bj, dim3(grid), dim3(BS), 0, ctx->stream, b.desc, b.fid, b.total_nf, K64, B64, B32,
                       bad);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status seg_multidot(hdg_ctx ctx, const BatchDev& b, const double* V, size_t ldv, int J, const double* w,
                        double* part, const BatchCtl* ctl) {
    if (J <= 0) return HDG_OK;
    hipLaunchKernelGGL(k_seg_multidot, dim3(b.nblk), dim3(BS), 0, ctx->stream, b.blk_inst, b.blk_lo, b.blk_hi, V, ldv,
                       J, w, part, b.nblk, ctl);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status seg_reduce(hdg_ctx ctx, const BatchDev& b, const double* part, int J, double* out, int ldo, bool add,
                      double* copy_to, int ldc, const BatchCtl* ctl) {
    if (J <= 0) return HDG_OK;
    const int waves = b.n_inst * J;
    hipLaunchKernelGGL(k_seg_reduce, dim3(div_up(waves, 4)), dim3(256), 0, ctx->stream, b.ib0, b.ib1, b.n_inst, part,
                       J, b.nblk, out, ldo, add ? 1 : 0, copy_to, ldc, ctl);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status seg_multiaxpy(hdg_ctx ctx, const BatchDev& b, const double* V, size_t ldv, int J, const double* h,
                         int ldh, double sign, double* w, const BatchCtl* ctl, bool use_kdev) {
    hipLaunchKernelGGL(k_seg_multiaxpy, dim3(div_up((long long)b.total_dof, BS)), dim3(BS), 0, ctx->stream,
                       b.dof_inst, V, ldv, J, h, ldh, sign, w, (size_t)b.total_dof, ctl, use_kdev ? 1 : 0);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status seg_sumsq(hdg_ctx ctx, const BatchDev& b, const double* w, double* part, const BatchCtl* ctl) {
    hipLaunchKernelGGL(k_seg_sumsq, dim3(b.nblk), dim3(BS), 0, ctx->stream, b.blk_inst, b.blk_lo, b.blk_hi, w, part,
                       ctl);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status seg_scale(hdg_ctx ctx, const BatchDev& b, double* v, const double* denom, int ld_denom,
                     const BatchCtl* ctl) {
    hipLaunchKernelGGL(k_seg_scale, dim3(div_up((long long)b.total_dof, BS)), dim3(BS), 0, ctx->stream, b.dof_inst, v,
                       (size_t)b.total_dof, denom, ld_denom, ctl);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status seg_cycle_init(hdg_ctx ctx, const BatchDev& b, const double* part, BatchCtl* ctl, double* g, int ldg,
                          int jmax, const double* target) {
    hipLaunchKernelGGL(k_seg_cycle_init, dim3(div_up(b.n_inst, 4)), dim3(256), 0, ctx->stream, b.ib0, b.ib1, b.n_inst,
                       part, ctl, g, ldg, jmax, target);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status seg_givens(hdg_ctx ctx, const BatchDev& b, const double* part, BatchCtl* ctl, double* H, int ldh, int mcols,
                      double* cs, double* sn, double* g, int ldg, int j, int jmax, const double* target) {
    hipLaunchKernelGGL(k_seg_givens, dim3(div_up(b.n_inst, 4)), dim3(256), 0, ctx->stream, b.ib0, b.ib1, b.n_inst,
                       part, ctl, H, ldh, mcols, cs, sn, g, ldg, j, jmax, target);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status seg_backsolve(hdg_ctx ctx, const BatchDev& b, const BatchCtl* ctl, const double* H, int ldh, int mcols,
                         const double* g, int ldg, double* y) {
    hipLaunchKernelGGL(k_seg_backsolve, dim3(div_up(b.n_inst, 64)), dim3(64), 0, ctx->stream, b.n_inst, ctl, H, ldh,
                       mcols, g, ldg, y);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status batch_launch_recover(hdg_ctx ctx, const BatchDev& b, const double* local, const double* Minv,
                                const double* Bd, const double* Cd, const int32_t* e2f, const double* xhat,
                                double* du, double* dq) {
    const int grid = (int)std::min<int64_t>(b.total_ne, 65536);
    const size_t lds = sizeof(double) * b.max_rec_lds;
    hipLaunchKernelGGL(k_batch_recover, dim3(grid), dim3(BS), lds, ctx->stream, b.desc, b.eid, b.total_ne, local, Minv,
                       Bd, Cd, e2f, xhat, du, dq);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}
