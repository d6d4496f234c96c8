// ILU-ASM: additive Schwarz on multi-element subdomains with block ILU(0) local solves
// (Section 3.3's ASM with the incomplete factorisation its conclusions propose).
//
// Subdomain l is the patch of G consecutive elements; its unknowns are the trace blocks of
// the patch's faces in increasing face order, its matrix K_l = R_l K R_l^T (block (a, b) =
// K[f_a][s] with nbr[f_a][s] = f_b). Setup: one workgroup per subdomain loads K_l densely
// into LDS together with its block pattern and runs right-looking block ILU(0) on that
// pattern (for each k: D_k = A_kk^{-1}; A_ik <- A_ik D_k for pattern blocks below; A_ij -=
// A_ik A_kj where (i, j) is in the pattern), which gives the same factors as the row-wise
// order for a fixed pattern. Only the off-diagonal pattern blocks are stored, grouped by
// block column (the L blocks of column k, then its U blocks), with U_ik stored as D_i U_ik,
// and the inverted diagonal blocks D_i. Apply: per subdomain, forward substitution with the
// unit lower factor column by column, x <- D x, then x_i -= (D_i U_ik) x_k column by column
// from the last; every face then sums the results of the (one or two) subdomains that hold
// it, with the face operator's epilogue.
#include <algorithm>
#include <vector>

#include "hdg_internal.hpp"

struct hdg_ilu_asm_s {
    int device = 0;
    int nsub = 0, nb = 0, nf = 0, G = 0, max_m = 0, max_n = 0;
    size_t solve_lds = 0;
    size_t N = 0;
    int32_t *sub_off = nullptr, *sub_faces = nullptr, *face_sub = nullptr;
    int64_t* blk_off = nullptr;       // per subdomain: first stored block
    int32_t *bij = nullptr, *cptr = nullptr, *cmid = nullptr;
    double *fac = nullptr, *dinv = nullptr, *zsub = nullptr, *tmp = nullptr;
    std::vector<void*> allocs;
};

namespace {

constexpr int IBS = 256;
constexpr int ILU_MAX_M = 88;      // n_faces * nb of a subdomain: (88^2) doubles of LDS
constexpr int ILU_MAX_NB = 16;

__global__ void __launch_bounds__(IBS) k_ilu_factor(const double* __restrict__ K64, const int32_t* __restrict__ nbr,
                                                    int S, int nb, const int32_t* __restrict__ sub_off,
                                                    const int32_t* __restrict__ sub_faces, double* fac,
                                                    const int64_t* __restrict__ blk_off,
                                                    const int32_t* __restrict__ bij, double* dinv, int* bad) {
    extern __shared__ double sm[];
    const int sub = blockIdx.x;
    const int tid = threadIdx.x;
    const int f0 = sub_off[sub], n = sub_off[sub + 1] - f0, m = n * nb;
    const int32_t* faces = sub_faces + f0;
    double* A = sm;                               // m x m, row-major
    double* Dk = A + (size_t)m * m;               // nb x nb: inverse of the current pivot block
    double* W = Dk + nb * nb;                     // nb x 2nb: Gauss-Jordan work
    unsigned char* pat = (unsigned char*)(W + 2 * nb * nb);   // n x n
    __shared__ int sing;
    for (int k = tid; k < m * m; k += IBS) A[k] = 0.0;
    for (int k = tid; k < n * n; k += IBS) pat[k] = 0;
    if (tid == 0) sing = 0;
    __syncthreads();
    // the local matrix: block (a, b) from slot s of face f_a with nbr = f_b
    for (int as = tid; as < n * S; as += IBS) {
        const int a = as / S, s = as - a * S;
        const int g = nbr[(size_t)faces[a] * S + s];
        if (g < 0) continue;
        int b = -1;
        for (int q = 0; q < n; ++q)
            if (faces[q] == g) { b = q; break; }
        if (b < 0) continue;
        pat[a * n + b] = 1;
        const double* blk = K64 + ((size_t)faces[a] * S + s) * nb * nb;   // [col][row]
        for (int c = 0; c < nb; ++c)
            for (int r = 0; r < nb; ++r) A[(size_t)(a * nb + r) * m + b * nb + c] = blk[c * nb + r];
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        // D_k = A_kk^{-1}: Gauss-Jordan with partial pivoting by one thread (nb <= 16)
        if (tid == 0) {
            for (int r = 0; r < nb; ++r)
                for (int c = 0; c < nb; ++c) {
                    W[r * 2 * nb + c] = A[(size_t)(k * nb + r) * m + k * nb + c];
                    W[r * 2 * nb + nb + c] = r == c ? 1.0 : 0.0;
                }
            for (int c = 0; c < nb && !sing; ++c) {
                int p = c;
                for (int r = c + 1; r < nb; ++r)
                    if (fabs(W[r * 2 * nb + c]) > fabs(W[p * 2 * nb + c])) p = r;
                const double pv = W[p * 2 * nb + c];
                if (!(fabs(pv) > 0.0) || !isfinite(pv)) { sing = 1; break; }
                if (p != c)
                    for (int q = 0; q < 2 * nb; ++q) {
                        const double t = W[c * 2 * nb + q];
                        W[c * 2 * nb + q] = W[p * 2 * nb + q];
                        W[p * 2 * nb + q] = t;
                    }
                const double ip = 1.0 / pv;
                for (int q = 0; q < 2 * nb; ++q) W[c * 2 * nb + q] *= ip;
                for (int r = 0; r < nb; ++r) {
                    if (r == c) continue;
                    const double fr = W[r * 2 * nb + c];
                    if (fr != 0.0)
                        for (int q = 0; q < 2 * nb; ++q) W[r * 2 * nb + q] -= fr * W[c * 2 * nb + q];
                }
            }
            for (int r = 0; r < nb; ++r)
                for (int c = 0; c < nb; ++c) Dk[r * nb + c] = W[r * 2 * nb + nb + c];
        }
        __syncthreads();
        if (sing) {
            if (tid == 0) atomicMin(bad, sub);
            return;     // uniform: every thread read the same flag after the barrier
        }
        // D_k goes to dinv and over A_kk, which no later step reads
        for (int q = tid; q < nb * nb; q += IBS) {
            dinv[((size_t)(f0 + k) * nb) * nb + q] = Dk[q];
            A[(size_t)(k * nb + q / nb) * m + k * nb + q % nb] = Dk[q];
        }
        // L_ik = A_ik D_k below the pivot (one thread per row of a block: reads, then writes its row)
        for (int ir = tid; ir < (n - k - 1) * nb; ir += IBS) {
            const int i = k + 1 + ir / nb, r = ir % nb;
            if (!pat[i * n + k]) continue;
            double* row = A + (size_t)(i * nb + r) * m + k * nb;
            double v[ILU_MAX_NB];
            for (int t = 0; t < nb; ++t) v[t] = row[t];
            for (int c = 0; c < nb; ++c) {
                double s = 0.0;
                for (int t = 0; t < nb; ++t) s += v[t] * Dk[t * nb + c];
                row[c] = s;
            }
        }
        __syncthreads();
        // A_ij -= L_ik A_kj on the pattern (i, j > k)
        const int rest = n - k - 1;
        for (int idx = tid; idx < rest * rest * nb * nb; idx += IBS) {
            const int ij = idx / (nb * nb), rc = idx - ij * nb * nb;
            const int i = k + 1 + ij / rest, j = k + 1 + ij % rest, r = rc / nb, c = rc % nb;
            if (!pat[i * n + k] || !pat[k * n + j] || !pat[i * n + j]) continue;
            const double* lik = A + (size_t)(i * nb + r) * m + k * nb;
            double s = 0.0;
            for (int t = 0; t < nb; ++t) s += lik[t] * A[(size_t)(k * nb + t) * m + j * nb + c];
            A[(size_t)(i * nb + r) * m + j * nb + c] -= s;
        }
        __syncthreads();
    }
    // the stored blocks: L_ik as factored, U_ik scaled to D_i U_ik
    const int nb2 = nb * nb;
    const int64_t b0 = blk_off[sub], nblk = blk_off[sub + 1] - b0;
    for (int64_t q = tid; q < nblk * nb2; q += IBS) {
        const int64_t b = q / nb2;
        const int rc = (int)(q - b * nb2), r = rc / nb, c = rc - r * nb;
        const int code = bij[b0 + b], i = code >> 16, k = code & 0xffff;
        double v;
        if (i > k) {
            v = A[(size_t)(i * nb + r) * m + k * nb + c];
        } else {
            v = 0.0;
            for (int t = 0; t < nb; ++t)
                v += A[(size_t)(i * nb + r) * m + i * nb + t] * A[(size_t)(i * nb + t) * m + k * nb + c];
        }
        fac[(b0 + b) * nb2 + rc] = v;
    }
}

// One workgroup of SBS threads per subdomain: 64 (one wave) when a subdomain has at most 64
// rows, else 128, so that a substitution step gives one row to each thread. Its stored blocks, their (row, column) codes, the column pointers and
// the inverted diagonal blocks are first copied to LDS with coalesced loads, so every
// substitution step reads LDS only and the dependent steps do not wait on HBM.
template <int SBS>
__global__ void __launch_bounds__(SBS) k_ilu_solve(const double* __restrict__ y, int nb,
                                                   const int32_t* __restrict__ sub_off,
                                                   const int32_t* __restrict__ sub_faces,
                                                   const double* __restrict__ fac,
                                                   const int64_t* __restrict__ blk_off,
                                                   const int32_t* __restrict__ bij,
                                                   const int32_t* __restrict__ cptr,
                                                   const int32_t* __restrict__ cmid,
                                                   const double* __restrict__ dinv, double* zsub, const int* skip) {
    if (skip && *skip) return;
    extern __shared__ double sm[];
    const int sub = blockIdx.x, tid = threadIdx.x;
    const int f0 = sub_off[sub], n = sub_off[sub + 1] - f0, m = n * nb, nb2 = nb * nb;
    const int64_t b0 = blk_off[sub];
    const int nblk = (int)(blk_off[sub + 1] - b0);
    const int32_t* faces = sub_faces + f0;
    double* Bs = sm;                          // nblk blocks nb x nb
    double* Ds = Bs + (size_t)nblk * nb2;     // n blocks nb x nb
    double* xa = Ds + (size_t)n * nb2;        // m: y, then L^{-1} y
    double* xb = xa + m;                      // m: the result
    int32_t* code = (int32_t*)(xb + m);       // nblk
    int32_t* cp = code + nblk;                // n + 1
    int32_t* cm = cp + n + 1;                 // n
    const double* Fg = fac + b0 * nb2;
    const double* Dg = dinv + (size_t)f0 * nb2;
    for (int q = tid; q < nblk * nb2; q += SBS) Bs[q] = Fg[q];
    for (int q = tid; q < n * nb2; q += SBS) Ds[q] = Dg[q];
    for (int q = tid; q < nblk; q += SBS) code[q] = bij[b0 + q];
    for (int q = tid; q <= n; q += SBS) cp[q] = cptr[f0 + sub + q];
    for (int q = tid; q < n; q += SBS) cm[q] = cmid[f0 + q];
    for (int q = tid; q < m; q += SBS) xa[q] = y[(size_t)faces[q / nb] * nb + q % nb];
    __syncthreads();
    for (int k = 0; k < n; ++k) {               // unit block-lower, column k: x_i -= L_ik x_k
        const double* xk = xa + k * nb;
        const int bl = cp[k];
        for (int q = tid; q < (cm[k] - bl) * nb; q += SBS) {
            const int b = bl + q / nb, r = q % nb;
            const double* L = Bs + (size_t)b * nb2 + r * nb;
            double s = 0.0;
            for (int c = 0; c < nb; ++c) s += L[c] * xk[c];
            xa[(code[b] >> 16) * nb + r] -= s;
        }
        __syncthreads();
    }
    for (int q = tid; q < m; q += SBS) {         // x = D y
        const int i = q / nb, r = q - i * nb;
        const double* D = Ds + (size_t)i * nb2 + r * nb;
        double s = 0.0;
        for (int c = 0; c < nb; ++c) s += D[c] * xa[i * nb + c];
        xb[q] = s;
    }
    __syncthreads();
    for (int k = n - 1; k > 0; --k) {           // column k of D U: x_i -= (D_i U_ik) x_k, i < k
        const double* xk = xb + k * nb;
        const int bu = cm[k];
        for (int q = tid; q < (cp[k + 1] - bu) * nb; q += SBS) {
            const int b = bu + q / nb, r = q % nb;
            const double* U = Bs + (size_t)b * nb2 + r * nb;
            double s = 0.0;
            for (int c = 0; c < nb; ++c) s += U[c] * xk[c];
            xb[(code[b] >> 16) * nb + r] -= s;
        }
        __syncthreads();
    }
    for (int q = tid; q < m; q += SBS) zsub[(size_t)f0 * nb + q] = xb[q];
}

// every face sums the (one or two) subdomain results that hold it; face epilogue as k_face_op
__global__ void __launch_bounds__(IBS) k_ilu_gather(int nf, int nb, const int32_t* __restrict__ face_sub,
                                                    const double* __restrict__ zsub, FaceEpilogue epi,
                                                    const int* skip) {
    if (skip && *skip) return;
    const size_t idx = (size_t)blockIdx.x * IBS + threadIdx.x;
    if (idx >= (size_t)nf * nb) return;
    const size_t f = idx / nb;
    const int t = (int)(idx - f * nb);
    double u = 0.0;
    for (int q = 0; q < 2; ++q) {
        const int p = face_sub[2 * f + q];
        if (p >= 0) u += zsub[(size_t)p * nb + t];
    }
    double v[3];
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        v[o] = epi.s[o] * u;
        if (epi.X[o]) v[o] += epi.a[o] * epi.X[o][idx];
        if (epi.Y[o]) v[o] += epi.b[o] * epi.Y[o][idx];
    }
#pragma unroll
    for (int o = 0; o < 3; ++o)
        if (epi.out[o]) epi.out[o][idx] = v[o];
}

size_t factor_lds(int max_m, int max_n, int nb) {
    return sizeof(double) * ((size_t)max_m * max_m + 3 * (size_t)nb * nb) + (size_t)max_n * max_n + 16;
}

template <typename T>
T* upload(hdg_ilu_asm h, const std::vector<T>& v, hipError_t* err) {
    void* p = nullptr;
    *err = hipMalloc(&p, std::max<size_t>(sizeof(T) * v.size(), 16));
    if (*err != hipSuccess) return nullptr;
    h->allocs.push_back(p);
    if (!v.empty()) *err = hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
    return (T*)p;
}

template <typename T>
T* dev_alloc(hdg_ilu_asm h, size_t n, hipError_t* err) {
    void* p = nullptr;
    *err = hipMalloc(&p, std::max<size_t>(sizeof(T) * n, 16));
    if (*err != hipSuccess) return nullptr;
    h->allocs.push_back(p);
    return (T*)p;
}

void free_handle(hdg_ilu_asm h) {
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    for (void* p : h->allocs) (void)hipFree(p);
    delete h;
}

}  // namespace

hdg_status ilu_apply_op(hdg_ctx ctx, const hdg_ilu_asm_s* h, const double* y, const FaceEpilogue& e,
                        const int* skip) {
    if (h->max_m <= 64)
        hipLaunchKernelGGL(k_ilu_solve<64>, dim3(h->nsub), dim3(64), h->solve_lds, ctx->stream, y, h->nb, h->sub_off,
                           h->sub_faces, h->fac, h->blk_off, h->bij, h->cptr, h->cmid, h->dinv, h->zsub, skip);
    else
        hipLaunchKernelGGL(k_ilu_solve<128>, dim3(h->nsub), dim3(128), h->solve_lds, ctx->stream, y, h->nb,
                           h->sub_off, h->sub_faces, h->fac, h->blk_off, h->bij, h->cptr, h->cmid, h->dinv, h->zsub,
                           skip);
    HDG_LAUNCH_CHECK(ctx);
    const size_t n = (size_t)h->nf * h->nb;
    if (n == 0) return HDG_OK;
    hipLaunchKernelGGL(k_ilu_gather, dim3((unsigned)div_up((long long)n, IBS)), dim3(IBS), 0, ctx->stream, h->nf,
                       h->nb, h->face_sub, h->zsub, e, skip);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

double* ilu_tmp(const hdg_ilu_asm_s* h) { return h->tmp; }
bool ilu_matches(const hdg_ilu_asm_s* h, const hdg_dims* d) {
    return h && h->nf == d->nf && h->nb == d->ncomp * d->npf;
}

extern "C" {

hdg_status hdg_ilu_asm_create(hdg_ctx ctx, const hdg_dims* d, const double* K64, const int32_t* nbr,
                              const int32_t* e2f, int32_t G, hdg_ilu_asm* out) {
    if (!ctx || !out) return HDG_ERR_ARG;
    *out = nullptr;
    if (!d || !K64 || !nbr || !e2f || G < 1) {
        ctx->err = "hdg_ilu_asm_create: NULL argument or G < 1";
        return HDG_ERR_ARG;
    }
    const int nb = d->ncomp * d->npf, L = d->nlfe, S = 2 * L - 1;
    if (d->ne < 1 || d->nf < 1 || nb < 1 || nb > ILU_MAX_NB) {
        ctx->err = "hdg_ilu_asm_create: need ne, nf >= 1 and a face block edge M*P_F of at most 16";
        return HDG_ERR_SHAPE;
    }
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    // subdomains from the element-to-face table (host copy)
    std::vector<int32_t> e2f_h((size_t)d->ne * L);
    HDG_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    HDG_HIP_CHECK(ctx, hipMemcpy(e2f_h.data(), e2f, sizeof(int32_t) * e2f_h.size(), hipMemcpyDeviceToHost));
    std::vector<int32_t> nbr_h((size_t)d->nf * S);
    HDG_HIP_CHECK(ctx, hipMemcpy(nbr_h.data(), nbr, sizeof(int32_t) * nbr_h.size(), hipMemcpyDeviceToHost));
    std::vector<int32_t> sub_off(1, 0), sub_faces, face_sub((size_t)d->nf * 2, -1);
    std::vector<int64_t> blk_off(1, 0);
    std::vector<int32_t> bij, cptr, cmid;
    std::vector<unsigned char> pat;
    int max_m = 0, max_n = 0;
    size_t solve_lds = 0;
    for (int64_t e0 = 0; e0 < d->ne; e0 += G) {
        const int64_t e1 = std::min<int64_t>(e0 + G, d->ne);
        std::vector<int32_t> fs(e2f_h.begin() + e0 * L, e2f_h.begin() + e1 * L);
        std::sort(fs.begin(), fs.end());
        fs.erase(std::unique(fs.begin(), fs.end()), fs.end());
        const int n = (int)fs.size();
        if (fs.front() < 0 || fs.back() >= d->nf) {
            ctx->err = "hdg_ilu_asm_create: e2f holds a face number outside [0, nf)";
            return HDG_ERR_ARG;
        }
        if (n * nb > ILU_MAX_M) {
            ctx->err = "hdg_ilu_asm_create: a subdomain has " + std::to_string(n) + " faces x " + std::to_string(nb) +
                       " dofs, more than 88 (LDS); use a smaller G";
            return HDG_ERR_SHAPE;
        }
        for (int a = 0; a < n; ++a) {
            const size_t p = sub_faces.size() + a;
            int32_t* slot = &face_sub[(size_t)fs[a] * 2];
            if (slot[0] < 0) slot[0] = (int32_t)p;
            else if (slot[1] < 0) slot[1] = (int32_t)p;
            else {
                ctx->err = "hdg_ilu_asm_create: a face lies in more than two subdomains";
                return HDG_ERR_ARG;
            }
        }
        // off-diagonal blocks of K's pattern inside the subdomain, by column: L part, then U part
        pat.assign((size_t)n * n, 0);
        for (int a = 0; a < n; ++a)
            for (int sl = 0; sl < S; ++sl) {
                const int32_t g = nbr_h[(size_t)fs[a] * S + sl];
                const auto it = std::lower_bound(fs.begin(), fs.end(), g);
                if (g >= 0 && it != fs.end() && *it == g) pat[(size_t)a * n + (it - fs.begin())] = 1;
            }
        const size_t first = bij.size();
        for (int k = 0; k < n; ++k) {
            cptr.push_back((int32_t)(bij.size() - first));
            for (int a = k + 1; a < n; ++a)
                if (pat[(size_t)a * n + k]) bij.push_back((a << 16) | k);
            cmid.push_back((int32_t)(bij.size() - first));
            for (int a = 0; a < k; ++a)
                if (pat[(size_t)a * n + k]) bij.push_back((a << 16) | k);
        }
        cptr.push_back((int32_t)(bij.size() - first));
        const size_t nblk = bij.size() - first;
        solve_lds = std::max(solve_lds, sizeof(double) * ((nblk + n) * nb * nb + 2 * (size_t)n * nb) +
                                            sizeof(int32_t) * (nblk + 2 * (size_t)n + 1));
        sub_faces.insert(sub_faces.end(), fs.begin(), fs.end());
        sub_off.push_back((int32_t)sub_faces.size());
        blk_off.push_back((int64_t)bij.size());
        max_m = std::max(max_m, n * nb);
        max_n = std::max(max_n, n);
    }
    hdg_ilu_asm h = new (std::nothrow) hdg_ilu_asm_s();
    if (!h) return HDG_ERR_NOMEM;
    h->device = ctx->device;
    h->nsub = (int)sub_off.size() - 1;
    h->nb = nb;
    h->nf = d->nf;
    h->G = G;
    h->max_m = max_m;
    h->max_n = max_n;
    h->solve_lds = solve_lds;
    h->N = (size_t)d->nf * nb;
    hipError_t err = hipSuccess;
    h->sub_off = upload(h, sub_off, &err);
    if (err == hipSuccess) h->sub_faces = upload(h, sub_faces, &err);
    if (err == hipSuccess) h->face_sub = upload(h, face_sub, &err);
    if (err == hipSuccess) h->blk_off = upload(h, blk_off, &err);
    if (err == hipSuccess) h->bij = upload(h, bij, &err);
    if (err == hipSuccess) h->cptr = upload(h, cptr, &err);
    if (err == hipSuccess) h->cmid = upload(h, cmid, &err);
    if (err == hipSuccess) h->fac = dev_alloc<double>(h, bij.size() * nb * nb, &err);
    if (err == hipSuccess) h->dinv = dev_alloc<double>(h, sub_faces.size() * nb * nb, &err);
    if (err == hipSuccess) h->zsub = dev_alloc<double>(h, sub_faces.size() * nb, &err);
    if (err == hipSuccess) h->tmp = dev_alloc<double>(h, h->N, &err);
    hdg_status st;
    int* status = err == hipSuccess ? (int*)ws_get(ctx, WS_STATUS, 64, &st) : nullptr;
    if (err != hipSuccess || !status) {
        ctx->err = err != hipSuccess ? std::string("hdg_ilu_asm_create: ") + hipGetErrorString(err) : ctx->err;
        free_handle(h);
        return HDG_ERR_NOMEM;
    }
    // from here on every error return releases the handle's device memory
    auto fail_hip = [&](hipError_t e, int line) {
        ctx->err = std::string("HIP error: ") + hipGetErrorString(e) + " at " + __FILE__ + ":" + std::to_string(line);
        free_handle(h);
        return HDG_ERR_HIP;
    };
    const int big = 0x7fffffff;
    err = hipMemcpyAsync(status, &big, sizeof(int), hipMemcpyHostToDevice, ctx->stream);
    if (err != hipSuccess) return fail_hip(err, __LINE__);
    const size_t lds = factor_lds(max_m, max_n, nb);
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute((const void*)k_ilu_factor, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    if (h->solve_lds > 64 * 1024) {
        (void)hipFuncSetAttribute((const void*)k_ilu_solve<64>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)h->solve_lds);
        (void)hipFuncSetAttribute((const void*)k_ilu_solve<128>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)h->solve_lds);
    }
    hipLaunchKernelGGL(k_ilu_factor, dim3(h->nsub), dim3(IBS), lds, ctx->stream, K64, nbr, S, nb, h->sub_off,
                       h->sub_faces, h->fac, h->blk_off, h->bij, h->dinv, status);
    if (hipGetLastError() != hipSuccess) {
        ctx->err = "hdg_ilu_asm_create: factorisation launch failed";
        free_handle(h);
        return HDG_ERR_HIP;
    }
    int bad = big;
    err = hipMemcpyAsync(&bad, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
    if (err != hipSuccess) return fail_hip(err, __LINE__);
    err = hipStreamSynchronize(ctx->stream);
    if (err != hipSuccess) return fail_hip(err, __LINE__);
    if (bad != big) {
        ctx->err = "hdg_ilu_asm_create: singular pivot block in subdomain " + std::to_string(bad);
        free_handle(h);
        return HDG_ERR_SINGULAR;
    }
    *out = h;
    return HDG_OK;
}

hdg_status hdg_ilu_asm_destroy(hdg_ilu_asm h) {
    if (!h) return HDG_ERR_ARG;
    free_handle(h);
    return HDG_OK;
}

hdg_status hdg_ilu_asm_apply(hdg_ctx ctx, hdg_ilu_asm h, const double* y, double* z) {
    if (!ctx || !h || !y || !z) return HDG_ERR_ARG;
    HDG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
    FaceEpilogue e;
    for (int o = 0; o < 3; ++o) {
        e.out[o] = nullptr;
        e.X[o] = e.Y[o] = nullptr;
        e.s[o] = e.a[o] = e.b[o] = 0.0;
    }
    e.out[0] = z;
    e.s[0] = 1.0;
    return ilu_apply_op(ctx, h, y, e, nullptr);
}

}  // extern "C"
