// Face-based assembly of the trace system (Section 4.2): each face is handled
// by one workgroup that gathers the matching (nb x nb) blocks of the element
// Schur complements of its one or two neighbours and writes the face's S slots
// of K (column-major blocks) and its part of r. Every output entry has exactly
// one writer, so there are no atomics and the result is deterministic.
#include "hdg_internal.hpp"

namespace {

constexpr int BS = 256;

__global__ __launch_bounds__(BS) void k_assemble(int nf, int M, int PF, int L, const int32_t* __restrict__ f2e,
                                                 const int32_t* __restrict__ e2f, const int32_t* __restrict__ perm,
                                                 const double* __restrict__ Kbar, const double* __restrict__ rbar,
                                                 double* __restrict__ K64, float* __restrict__ K32,
                                                 int32_t* __restrict__ nbr, double* __restrict__ r, int nbuf) {
    const int nb = M * PF;
    const int S = 2 * L - 1;
    const int nt = L * nb;
    const long long f = blockIdx.x;
    if (f >= nf) return;
    const int e1 = f2e[4 * f + 0], l1 = f2e[4 * f + 1];
    const int e2 = f2e[4 * f + 2], l2 = f2e[4 * f + 3];
    // slot -> (element, row local face, column local face)
    __shared__ int se[64], slr[64], slc[64];
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
        int g = -1;
        if (s == 0) g = (int)f;
        else if (se[s] >= 0) g = e2f[(size_t)se[s] * L + slc[s]];
        nbr[f * S + s] = g;
    }
    // local trace index of canonical face dof (m, j) on local face l of element e
    auto tix = [&](int e, int l, int m, int j) -> int {
        const int jl = perm ? perm[((size_t)e * L + l) * PF + j] : j;
        return (l * M + m) * PF + jl;
    };
    const size_t blk = (size_t)nb * nb;
    // dynamic LDS: nbuf tiles of nb x (nb+1) (row-major gather, column-major write), then the
    // row and column trace indices of every slot's block (and of the second element's
    // diagonal block), formed once so that the gathers read Kbar without a perm lookup
    extern __shared__ double tile[];
    const int ldt = nb + 1;
    int* ridx = reinterpret_cast<int*>(tile + (size_t)nbuf * nb * ldt);   // [S + 1][nb]
    int* cidx = ridx + (size_t)(S + 1) * nb;                              // [S + 1][nb]
    for (int idx = threadIdx.x; idx < (S + 1) * nb; idx += BS) {
        const int s = idx / nb, rr = idx - s * nb;
        const int m = rr / PF, j = rr - m * PF;
        if (s < S) {
            const int e = se[s];
            ridx[idx] = e >= 0 ? tix(e, slr[s], m, j) : 0;
            cidx[idx] = e >= 0 ? tix(e, slc[s], m, j) : 0;
        } else {
            ridx[idx] = e2 >= 0 ? tix(e2, l2, m, j) : 0;
            cidx[idx] = ridx[idx];
        }
    }
    __syncthreads();
    // slot s's block gathered into tile buffer s % nbuf (consecutive threads read consecutive
    // columns of a row of Kbar)
    auto gather = [&](int s) {
        const int e = se[s];
        if (e < 0) return;
        double* tb = tile + (size_t)(s % nbuf) * nb * ldt;
        const double* Ke = Kbar + (size_t)e * nt * nt;
        const double* K2 = (s == 0 && e2 >= 0) ? Kbar + (size_t)e2 * nt * nt : nullptr;
        const int* ri = ridx + s * nb;
        const int* ci = cidx + s * nb;
        const int* ri2 = ridx + S * nb;
        for (int idx = threadIdx.x; idx < (int)blk; idx += BS) {
            const int rr = idx / nb, c = idx - rr * nb;
            double v = Ke[(size_t)ri[rr] * nt + ci[c]];
            if (K2) v += K2[(size_t)ri2[rr] * nt + ri2[c]];
            tb[rr * ldt + c] = v;
        }
    };
    auto write = [&](int s) {
        double* out = K64 + ((size_t)f * S + s) * blk;
        float* out32 = K32 ? K32 + ((size_t)f * S + s) * blk : nullptr;
        if (se[s] < 0) {
            for (int idx = threadIdx.x; idx < (int)blk; idx += BS) {
                out[idx] = 0.0;
                if (out32) out32[idx] = 0.0f;
            }
            return;
        }
        const double* tb = tile + (size_t)(s % nbuf) * nb * ldt;
        for (int idx = threadIdx.x; idx < (int)blk; idx += BS) {
            const int c = idx / nb, rr = idx - c * nb;          // column-major: idx = c*nb + rr
            const double v = tb[rr * ldt + c];
            out[idx] = v;
            if (out32) out32[idx] = (float)v;
        }
    };
    if (nbuf == 2) {
        // the next slot's loads are in flight while this slot's block is written
        gather(0);
        __syncthreads();
        for (int s = 0; s < S; ++s) {
            if (s + 1 < S) gather(s + 1);
            write(s);
            __syncthreads();
        }
    } else {
        for (int s = 0; s < S; ++s) {
            gather(s);
            __syncthreads();
            write(s);
            __syncthreads();
        }
    }
    for (int rr = threadIdx.x; rr < nb; rr += BS) {
        const int m = rr / PF, j = rr - m * PF;
        double v = rbar[(size_t)e1 * nt + tix(e1, l1, m, j)];
        if (e2 >= 0) v += rbar[(size_t)e2 * nt + tix(e2, l2, m, j)];
        r[f * nb + rr] = v;
    }
}

// The right-hand side alone: r_f = rbar^{e1}_{l1} + rbar^{e2}_{l2} (the same sums as above),
// one wave per face.
__global__ __launch_bounds__(BS) void k_assemble_rhs(int nf, int M, int PF, int L, const int32_t* __restrict__ f2e,
                                                     const int32_t* __restrict__ perm,
                                                     const double* __restrict__ rbar, double* __restrict__ r) {
    const int nb = M * PF, nt = L * nb;
    const long long f = (long long)blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
    if (f >= nf) return;
    const int lane = threadIdx.x & 63;
    const int e1 = f2e[4 * f + 0], l1 = f2e[4 * f + 1];
    const int e2 = f2e[4 * f + 2], l2 = f2e[4 * f + 3];
    for (int rr = lane; rr < nb; rr += 64) {
        const int m = rr / PF, j = rr - m * PF;
        const int j1 = perm ? perm[((size_t)e1 * L + l1) * PF + j] : j;
        double v = rbar[(size_t)e1 * nt + (l1 * M + m) * PF + j1];
        if (e2 >= 0) {
            const int j2 = perm ? perm[((size_t)e2 * L + l2) * PF + j] : j;
            v += rbar[(size_t)e2 * nt + (l2 * M + m) * PF + j2];
        }
        r[f * nb + rr] = v;
    }
}

}  // namespace

hdg_status assemble_rhs_run(hdg_ctx ctx, const hdg_dims* d, const int32_t* f2e, const int32_t* perm,
                            const double* rbar, double* r) {
    if (d->nf == 0) return HDG_OK;
    const long long grid = ((long long)d->nf + BS / 64 - 1) / (BS / 64);
    hipLaunchKernelGGL(k_assemble_rhs, dim3((unsigned)grid), dim3(BS), 0, ctx->stream, d->nf, d->ncomp, d->npf,
                       d->nlfe, f2e, perm, rbar, r);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status assemble_run(hdg_ctx ctx, const hdg_dims* d, const int32_t* f2e, const int32_t* e2f,
                        const int32_t* perm, const double* Kbar, const double* rbar, double* K64, float* K32,
                        int32_t* nbr, double* r) {
    if (d->nf == 0) return HDG_OK;
    const int nb = d->ncomp * d->npf;
    // two tile buffers for small blocks (at most 32 KiB of LDS in all, so that several faces
    // still share a CU), else one
    const int S = 2 * d->nlfe - 1;
    const size_t tile = sizeof(double) * (size_t)nb * (nb + 1);
    const size_t tabs = sizeof(int) * 2 * (size_t)(S + 1) * nb;
    const int nbuf = 2 * tile + tabs <= 32 * 1024 ? 2 : 1;
    const size_t lds = nbuf * tile + tabs;
    if (lds > 64 * 1024)
        HDG_HIP_CHECK(ctx, hipFuncSetAttribute((const void*)k_assemble, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds));
    hipLaunchKernelGGL(k_assemble, dim3(d->nf), dim3(BS), lds, ctx->stream, d->nf, d->ncomp, d->npf, d->nlfe, f2e,
                       e2f, perm, Kbar, rbar, K64, K32, nbr, r, nbuf);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}
