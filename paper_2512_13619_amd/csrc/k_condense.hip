// Batched static condensation (Section 4.1 eq. w15-w19, Section 4.2 eq. w21-w22).
//
// For each element the kernels build the (nu+nt) x (nu+nt+1) matrix
//     T = [[E F r_u], [H J r_t]] - [D; G] A^{-1} [B C 0]
//       = [[Ebar Fbar r_u], [Hbar Jbar r_t]]                       (q eliminated, r_q = 0)
// then factorise Ebar with partial pivoting (P Ebar = L U) and solve on the Ebar rows, so
// that they hold [U | X | x_r] with X = Ebar^{-1} Fbar and x_r = Ebar^{-1} r_u (eq. w19,
// which recovery uses directly), and finally
//     Kbar = Jbar - Hbar X   and   rbar = r_t - Hbar x_r                  (eq. w22).
//
// A^{-1} = I_{MD} (x) M^{-1} and B, C are component-diagonal (eq. w16), so
// [D;G] A^{-1} [B C] restricted to the columns of component m is
//     sum_d [D;G][:, q(m,d,:)] (M^{-1} [B_d | C_d]):
// one (nu+nt) x (D P_E) by (D P_E) x (P_E + N_lfe P_F) product per component,
// with W = M^{-1}[B_d | C_d] formed first. All products run on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64). Three stages:
//   1. q-elimination: LDS-staged 64x64 tiles (one block per element and tile, the M
//      components' products in one pipeline), giving [[Ebar Fbar r_u], [Hbar Jbar r_t]];
//   2. on the Ebar rows only: right-looking blocked LU of the first nu columns (panels
//      factorised in one wave's registers, trailing updates on the matrix cores; for
//      nu <= 64 one wave per element holds the whole block), then block substitution
//      X = U^{-1} (L^{-1} P [Fbar | r_u]) with inverted 32x32 diagonal blocks;
//   3. Schur product Kbar = Jbar - Hbar X, rbar = r_t - Hbar x_r, of depth nu: fused into
//      the substitution's slabs for nu <= 192, else LDS-staged 64x64 tiles.
//
// Storage of T per element: the top nu rows live directly in the caller's
// `local` buffer (row stride nu+nt+1), the bottom nt rows in a workspace.
#include <cmath>

#include "hdg_internal.hpp"
#include "wave_ops.hpp"

namespace {

constexpr int BS = 256;

struct CondDims {
    int M, D, P, PF, L;
    int nu, nq, nt, R, C, NW, KD;
};

// acc[bi][bj][q] holds row 16*bi + 4*q + lane/16, column 16*bj + lane%16 of a 32x32 tile
// (v_mfma_f64_16x16x4f64: A[i][k] in lane i+16k, B[k][j] in lane j+16k, D[i][j] in lane
// j+16*(i%4), register i/4).
//
// acc += A(32 x K) B(K x 32). k is taken in groups of 16: instruction s (0..3) of a
// group gives lane (i, kq) the pair A[i][kb+4kq+s], B[kb+4kq+s][j], so the four
// instructions together cover all 16 k of the group and each lane reads four
// consecutive k of its A row. The next group's operands are loaded while the current
// group's 16 MFMAs run (two register buffers). la/lb return 0 outside the matrices.
template <class LA, class LB>
__device__ __forceinline__ void mfma_32x32(const LA& la, const LB& lb, int K, double4_t (&acc)[2][2]) {
    const int lane = threadIdx.x & 63;
    const int i16 = lane & 15, kq = lane >> 4;
    double a0[4][2], b0[4][2], a1[4][2], b1[4][2];
    auto fetch = [&](double (&fa)[4][2], double (&fb)[4][2], int kb) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = kb + 4 * kq + s;
            fa[s][0] = la(i16, k);
            fa[s][1] = la(16 + i16, k);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = kb + 4 * kq + s;
            fb[s][0] = lb(k, i16);
            fb[s][1] = lb(k, 16 + i16);
        }
    };
    auto mma = [&](const double (&fa)[4][2], const double (&fb)[4][2]) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][0], fb[s][0], acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][0], fb[s][1], acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][1], fb[s][0], acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][1], fb[s][1], acc[1][1], 0, 0, 0);
        }
    };
    // (loads past K are harmless: la/lb read a clamped address and return 0)
    fetch(a0, b0, 0);
    for (int kb = 0; kb < K; kb += 32) {
        fetch(a1, b1, kb + 16);
        __builtin_amdgcn_sched_barrier(0);
        mma(a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        if (kb + 16 >= K) break;
        fetch(a0, b0, kb + 32);
        __builtin_amdgcn_sched_barrier(0);
        mma(a1, b1);
        __builtin_amdgcn_sched_barrier(0);
    }
}

__device__ __forceinline__ void acc_zero(double4_t (&acc)[2][2]) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = double4_t{0.0, 0.0, 0.0, 0.0};
}

// ---- LDS-staged 64x64 tile product -----------------------------------------------------------
// acc += A(64 x K) B(K x 64) for the tile whose corner is (m0, n0): 256 threads, wave w owns
// the 32x32 quadrant (rows 32*(w/2), columns 32*(w%2)) in the mfma_32x32 layout. K is
// taken in chunks of 32 staged through LDS (double-buffered; a chunk's global loads are
// issued two chunks ahead). A is stored k-major in LDS (row
// stride 65 to spread the transposing writes over the banks), B as it is. Entries
// outside the matrices read as 0.
constexpr int GT = 64, GK = 32, GLDA = GT + 1, GLDB = GT;
constexpr size_t GEMM_LDS = sizeof(double) * 2 * (GK * GLDA + GK * GLDB);

// A row-major matrix whose rows [0, split) start at p0 and rows [split, rows) at p1
// (same row stride ld).
struct MatA {
    const double* p0;
    const double* p1;
    int split, ld, rows, cols;
};
// A row-major matrix at p with row stride ld.
struct MatB {
    const double* p;
    int ld, rows, cols;
};

__device__ __forceinline__ void gemm_tile64(const MatA& A, const MatB& B, int m0, int n0, double* lds,
                                            double4_t (&acc)[2][2]) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int i16 = lane & 15, kq = lane >> 4;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int K = A.cols;
    // staging roles: A rows m0 + (tid>>5) + 8u at column k0 + (tid&31); B rows
    // k0 + (tid>>6) + 4u at column n0 + (tid&63)
    const int ka = tid & 31, jb = tid & 63;
    const double* arow[8];
    bool aok[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int r = m0 + (tid >> 5) + 8 * u;
        aok[u] = r < A.rows;
        const int rr = aok[u] ? r : 0;
        arow[u] = rr < A.split ? A.p0 + (size_t)rr * A.ld : A.p1 + (size_t)(rr - A.split) * A.ld;
    }
    const bool bok_c = n0 + jb < B.cols;
    const double* bcol = B.p + (bok_c ? n0 + jb : 0);
    // raw loads (clamped addresses); the masks are applied when the values go to LDS, so
    // no load has to complete before the MFMAs of the current chunk are issued. Two
    // register sets: a chunk's loads are issued two chunks before its MFMAs, so their
    // latency is covered by a whole chunk of MFMAs.
    double ra[2][8], rb[2][8];
    int kst[2] = {0, 0};               // k0 of the chunk held in set s
    auto gload = [&](int s, int k0) {
        kst[s] = k0;
        const int k = k0 + ka;
        const int kc = k < K ? k : 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) ra[s][u] = arow[u][kc];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int kb = k0 + (tid >> 6) + 4 * u;
            rb[s][u] = bcol[(size_t)(kb < B.rows ? kb : 0) * B.ld];
        }
    };
    auto lstore = [&](int s, int b) {
        double* As = lds + b * (GK * GLDA);
        double* Bs = lds + 2 * GK * GLDA + b * (GK * GLDB);
        const bool kok = kst[s] + ka < K;
#pragma unroll
        for (int u = 0; u < 8; ++u) As[ka * GLDA + (tid >> 5) + 8 * u] = (kok && aok[u]) ? ra[s][u] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int kb = kst[s] + (tid >> 6) + 4 * u;
            Bs[((tid >> 6) + 4 * u) * GLDB + jb] = (bok_c && kb < B.rows) ? rb[s][u] : 0.0;
        }
    };
    auto compute = [&](int b) {
        const double* As = lds + b * (GK * GLDA);
        const double* Bs = lds + 2 * GK * GLDA + b * (GK * GLDB);
        double a[8][2], bb[8][2];
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const int k = 4 * ks + kq;
            a[ks][0] = As[k * GLDA + wr + i16];
            a[ks][1] = As[k * GLDA + wr + 16 + i16];
            bb[ks][0] = Bs[k * GLDB + wc + i16];
            bb[ks][1] = Bs[k * GLDB + wc + 16 + i16];
        }
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks][0], bb[ks][0], acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks][0], bb[ks][1], acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks][1], bb[ks][0], acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks][1], bb[ks][1], acc[1][1], 0, 0, 0);
        }
    };
    const int nch = (K + GK - 1) / GK;
    gload(0, 0);
    if (nch > 1) gload(1, GK);
    lstore(0, 0);
    __syncthreads();
    // even chunks in LDS buffer 0 (their loads in set 0), odd ones in buffer 1 (set 1)
    for (int c = 0; c < nch; c += 2) {
        if (c + 2 < nch) gload(0, (c + 2) * GK);
        compute(0);
        if (c + 1 < nch) lstore(1, 1);
        __syncthreads();
        if (c + 1 >= nch) break;
        if (c + 3 < nch) gload(1, (c + 3) * GK);
        compute(1);
        if (c + 2 < nch) lstore(0, 0);
        __syncthreads();
    }
}

// Blocks are dealt round-robin to the 8 XCDs; renumber them so that each XCD walks a
// contiguous range of tiles (the tiles of one element then share that XCD's L2).
__device__ __forceinline__ long long xcd_linear(long long nblk) {
    const long long b = blockIdx.x;
    const long long per = nblk / 8;
    return (b % 8) * per + b / 8;
}

// ---- W = M^{-1} [B_d | C_d]  per (element, d):  (P x P) (P x NW) -----------------------
__global__ __launch_bounds__(BS) void k_cond_w(CondDims cd, const double* __restrict__ Minv,
                                               const double* __restrict__ Bd, const double* __restrict__ Cd,
                                               double* __restrict__ W) {
    const long long e = blockIdx.x;
    const int d = blockIdx.y;
    const int P = cd.P, NW = cd.NW, LPF = cd.L * cd.PF;
    const double* Mi = Minv + (size_t)e * P * P;
    const double* B = Bd + ((size_t)e * cd.D + d) * P * P;
    const double* Cm = Cd + ((size_t)e * cd.D + d) * P * LPF;
    double* Wo = W + (size_t)e * cd.KD * NW + (size_t)d * P * NW;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tr = (P + 31) / 32, tc = (NW + 31) / 32;
    for (int tile = wave; tile < tr * tc; tile += BS / 64) {
        const int r0 = (tile / tc) * 32, c0 = (tile % tc) * 32;
        double4_t acc[2][2];
        acc_zero(acc);
        // operand reads are unconditional (clamped to a valid address) and masked after,
        // so a whole group of loads is issued without branches
        auto la = [&](int i, int k) -> double {
            const int r = r0 + i;
            const bool ok = r < P && k < P;
            const double v = Mi[ok ? (size_t)r * P + k : 0];
            return ok ? v : 0.0;
        };
        auto lb = [&](int k, int j) -> double {
            const int c = c0 + j;
            const bool ok = k < P && c < NW;
            const double* src = c < P ? B + (size_t)k * P + c : Cm + (size_t)k * LPF + (c - P);
            const double v = *(ok ? src : B);
            return ok ? v : 0.0;
        };
        mfma_32x32(la, lb, P, acc);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = r0 + 16 * bi + 4 * q + (lane >> 4);
                    const int c = c0 + 16 * bj + (lane & 15);
                    if (r < P && c < NW) Wo[(size_t)r * NW + c] = acc[bi][bj][q];
                }
    }
}

// Column of T for column c of W (component m): u columns of m, then m's part of each
// element-trace block l.
__device__ __forceinline__ int qelim_col(int c, int m, int P, int PF, int M, int nu) {
    if (c < P) return m * P + c;
    const int cc = c - P, l = cc / PF, j = cc - l * PF;
    return nu + (l * M + m) * PF + j;
}

// ---- T = T0 - [D;G][:, q(m,:,:)] W   per (element, 64x64 tile), every component m ------------
// One block per (element, row tile, column tile); the M components' products run through one
// pipeline: chunk c of the stream is component c / nch, depth slice (c % nch) * QK of the
// product [D;G][:, q(m,:,:)] (rows m0.., columns m KD..) times W (the same W for every
// component), so the next component's first slices are loaded while the current one's last
// ones are multiplied, and a block fills its pipeline once instead of once per component.
// Each component's result, T0 minus the product, goes to its own columns of T (qelim_col)
// when its last slice is done. Slices are 16 deep (33 KB of LDS, double-buffered), so three
// blocks share a CU and hide each other's barrier and load waits. nblk is a multiple of 8
// (trailing blocks exit).
constexpr int QK = 16;
constexpr size_t QLDS = sizeof(double) * 2 * (QK * GLDA + QK * GLDB);
template <bool V2>
__global__ __launch_bounds__(BS, 3) void k_cond_qelim(CondDims cd, long long ntile, int tm_n, int tn_n,
                                                   const double* __restrict__ Dm, const double* __restrict__ Em,
                                                   const double* __restrict__ Fm, const double* __restrict__ Gm,
                                                   const double* __restrict__ Hm, const double* __restrict__ Jm,
                                                   const double* __restrict__ ru, const double* __restrict__ rt,
                                                   const double* __restrict__ W, double* __restrict__ top,
                                                   double* __restrict__ bot) {
    extern __shared__ double lds[];
    const long long Lb = xcd_linear(gridDim.x);
    if (Lb >= ntile) return;
    const int per_e = tm_n * tn_n;
    const long long e = Lb / per_e;
    const int rem = (int)(Lb - e * per_e);
    const int m0 = (rem / tn_n) * GT, n0 = (rem % tn_n) * GT;
    const int nu = cd.nu, nt = cd.nt, nq = cd.nq, R = cd.R, C = cd.C, NW = cd.NW, KD = cd.KD;
    const int P = cd.P, PF = cd.PF, M = cd.M;
    const double* We = W + (size_t)e * KD * NW;
    double* Te = top + (size_t)e * nu * C;
    double* Be = bot + (size_t)e * nt * C;
    const double* Ee = Em + (size_t)e * nu * nu;
    const double* Fe = Fm + (size_t)e * nu * nt;
    const double* He = Hm + (size_t)e * nt * nu;
    const double* Je = Jm + (size_t)e * nt * nt;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i16 = lane & 15, kq = lane >> 4;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int r0 = m0 + wr, c0 = n0 + wc;
    const int nch = (KD + QK - 1) / QK;
    const int nall = M * nch;
    // staging roles (8-byte form): A rows m0 + (tid>>4) + 16u at depth k0 + (tid&15); B rows
    // k0 + (tid>>6) + 4u at column n0 + (tid&63); the 16-byte form halves the threads per row and
    // doubles the rows per thread. Rows of A past R and columns of B past NW are read at clamped
    // addresses and left unmasked: they only reach rows and columns of the tile that are never
    // stored. Depth past KD (a ragged last slice) reads clamped A and zeroed B, so those products
    // vanish.
    const bool ragged = (KD % QK) != 0;
    int kst = 0;
    typedef double d2_t __attribute__((ext_vector_type(2)));
    // V2 (nq, KD and NW even): 16-byte loads of two consecutive depths of a row of [D;G] and of
    // two consecutive columns of W, half the load instructions of the 8-byte form
    const int ka = V2 ? 2 * (tid & 7) : (tid & 15), jb = V2 ? 2 * (tid & 31) : (tid & 63);
    constexpr int NA = V2 ? 2 : 4;                 // rows of [D;G] per thread
    const int arow0 = V2 ? (tid >> 3) : (tid >> 4), astep = V2 ? 32 : 16;
    const double* arow[NA];
#pragma unroll
    for (int u = 0; u < NA; ++u) {
        const int r = m0 + arow0 + astep * u;
        const int rr = r < R ? r : R - 1;
        arow[u] = rr < nu ? Dm + ((size_t)e * nu + rr) * nq : Gm + ((size_t)e * nt + (rr - nu)) * nq;
    }
    const int brow0 = V2 ? (tid >> 5) : (tid >> 6), bstep = V2 ? 8 : 4;
    const int jc = V2 ? (n0 + jb < NW ? n0 + jb : NW - 2) : (n0 + jb < NW ? n0 + jb : NW - 1);
    const double* bcol = We + jc;
    double ra[4], rb[4];
    // loads of stream chunk c (past the stream: its last chunk again) into the staging registers;
    // every pass of the loop issues the same loads, so the wait before each LDS store covers
    // exactly the chunk that store writes
    auto gload = [&](int c) __attribute__((always_inline)) {
        c = c < nall ? c : nall - 1;
        const int m = c / nch, k0 = (c - m * nch) * QK;
        kst = k0;
        const int k = k0 + ka;
        if constexpr (V2) {
            const int kc = m * KD + (k < KD ? k : KD - 2);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const d2_t v = *reinterpret_cast<const d2_t*>(arow[u] + kc);
                ra[2 * u] = v.x;
                ra[2 * u + 1] = v.y;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int kb = k0 + brow0 + bstep * u;
                const d2_t v = *reinterpret_cast<const d2_t*>(bcol + (size_t)(kb < KD ? kb : KD - 1) * NW);
                rb[2 * u] = v.x;
                rb[2 * u + 1] = v.y;
            }
        } else {
            const int kc = m * KD + (k < KD ? k : KD - 1);
#pragma unroll
            for (int u = 0; u < 4; ++u) ra[u] = arow[u][kc];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int kb = k0 + brow0 + bstep * u;
                rb[u] = bcol[(size_t)(kb < KD ? kb : KD - 1) * NW];
            }
        }
    };
    auto lstore = [&](int b) __attribute__((always_inline)) {
        double* As = lds + b * (QK * GLDA);
        double* Bs = lds + 2 * QK * GLDA + b * (QK * GLDB);
        if constexpr (V2) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                As[ka * GLDA + arow0 + astep * u] = ra[2 * u];
                As[(ka + 1) * GLDA + arow0 + astep * u] = ra[2 * u + 1];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int kl = brow0 + bstep * u;
                const bool z = ragged && kst + kl >= KD;
                d2_t v;
                v.x = z ? 0.0 : rb[2 * u];
                v.y = z ? 0.0 : rb[2 * u + 1];
                *reinterpret_cast<d2_t*>(Bs + kl * GLDB + jb) = v;
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) As[ka * GLDA + arow0 + astep * u] = ra[u];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int kb = kst + brow0 + bstep * u;      // uniform over the wave
                Bs[(brow0 + bstep * u) * GLDB + jb] = (ragged && kb >= KD) ? 0.0 : rb[u];
            }
        }
    };
    double4_t acc[2][2];
    acc_zero(acc);
    const bool wact = r0 < R && c0 < NW;   // the wave's quadrant holds part of the element's block
    auto compute = [&](int b) __attribute__((always_inline)) {
        if (!wact) return;
        const double* As = lds + b * (QK * GLDA);
        const double* Bs = lds + 2 * QK * GLDA + b * (QK * GLDB);
        {   // one 16-deep slice: four k-steps of four products
            double a[4][2], bb[4][2];
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int k = 4 * ks + kq;
                a[ks][0] = As[k * GLDA + wr + i16];
                a[ks][1] = As[k * GLDA + wr + 16 + i16];
                bb[ks][0] = Bs[k * GLDB + wc + i16];
                bb[ks][1] = Bs[k * GLDB + wc + 16 + i16];
            }
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks][0], bb[ks][0], acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks][0], bb[ks][1], acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks][1], bb[ks][0], acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks][1], bb[ks][1], acc[1][1], 0, 0, 0);
            }
        }
    };
    // this lane's two columns of the quadrant: T's column for component m is cb[bj] + m * cs[bj]
    // (u columns of m: c + m P; trace columns: nu + (l M + m) PF + j, l = (c - P) / PF)
    int cb[2], cs[2];
    bool cu[2], cin[2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        const int c = c0 + 16 * bj + (lane & 15);
        cin[bj] = c < NW;
        cu[bj] = c < P;
        const int cc = c - P, l = cc / PF, j = cc - l * PF;
        cb[bj] = cu[bj] ? c : nu + l * M * PF + j;
        cs[bj] = cu[bj] ? P : PF;
    }
    // T = T0 - product for component m. T0 (E, F, H or J at T's column) is loaded when the
    // component's last slice is issued, so its latency is covered by that slice's products.
    double t0[2][4][2];
    auto load_t0 = [&](int m) __attribute__((always_inline)) {
        if (!wact) return;
        int rl = r0 + (lane >> 4);
        asm volatile("" : "+v"(rl));   // the row addresses are formed here, not kept live across the loop
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = rl + 16 * bi + 4 * q;
                const bool rok = r < R, top_row = r < nu;
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    const int tcol = cb[bj] + m * cs[bj];
                    const double* src = top_row ? (cu[bj] ? Ee + (size_t)r * nu + tcol : Fe + (size_t)r * nt + (tcol - nu))
                                                : (cu[bj] ? He + (size_t)(r - nu) * nu + tcol
                                                          : Je + (size_t)(r - nu) * nt + (tcol - nu));
                    t0[bi][q][bj] = *((rok && cin[bj]) ? src : Ee);
                }
            }
    };
    auto store_t = [&](int m) __attribute__((always_inline)) {
        if (!wact) return;
        int rl = r0 + (lane >> 4);
        asm volatile("" : "+v"(rl));
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = rl + 16 * bi + 4 * q;
                if (r >= R) continue;
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    if (!cin[bj]) continue;
                    const int tcol = cb[bj] + m * cs[bj];
                    const double v = t0[bi][q][bj] - acc[bi][bj][q];
                    if (r < nu) Te[(size_t)r * C + tcol] = v;
                    else Be[(size_t)(r - nu) * C + tcol] = v;
                }
            }
        acc_zero(acc);
    };
    // stream chunk c in LDS buffer c % 2; chunk c + 1's loads are in flight while chunk c is
    // multiplied (a store into a buffer past the stream is never read)
    gload(0);
    lstore(0);
    gload(1);
    __syncthreads();
#pragma unroll 1
    for (int c = 0; c < nall; c += 2) {
        const bool last0 = (c % nch) == nch - 1, last1 = ((c + 1) % nch) == nch - 1;
        compute(0);
        lstore(1);
        gload(c + 2);
        if (last0) { load_t0(c / nch); store_t(c / nch); }
        __syncthreads();
        if (c + 1 >= nall) break;
        compute(1);
        lstore(0);
        gload(c + 3);
        if (last1) { load_t0((c + 1) / nch); store_t((c + 1) / nch); }
        __syncthreads();
    }
    // the right-hand-side column (once per element and row tile)
    if (n0 == 0) {
        for (int r = m0 + tid; r < m0 + GT && r < R; r += BS) {
            if (r < nu) Te[(size_t)r * C + (C - 1)] = ru[(size_t)e * nu + r];
            else Be[(size_t)(r - nu) * C + (C - 1)] = rt[(size_t)e * nt + (r - nu)];
        }
    }
}

// v from lane l (l uniform), as a uniform value
__device__ __forceinline__ double lane_value(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Orders the LDS accesses of one wave: its lanes exchange data through LDS without a
// block barrier (the LDS executes one wave's operations in issue order).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Entry c of row slot os of lane ol, as a uniform value (os, ol uniform).
// (Each slot is read from lane ol, then the uniform results are selected: a select between
// the slots' registers would let the compiler turn it into an indexed load and keep the panel
// in scratch memory.)
template <int RPL, int NBT>
__device__ __forceinline__ double panel_entry(const double (&a)[RPL][NBT], int os, int c, int ol) {
    double x = lane_value(a[0][c], ol);
#pragma unroll
    for (int r = 1; r < RPL; ++r) {
        const double y = lane_value(a[r][c], ol);
        x = os == r ? y : x;
    }
    return x;
}

// LU with partial pivoting of a panel (nrow rows, nbk <= NBT columns) held in one wave's
// registers: lane l holds the rows l + 64 r (r < RPL) in a[r], pos[r] = l + 64 r on entry. No
// row moves while the panel is factorised: each lane tracks where its rows stand in the
// interchanged order (pos), and the pivot of column kk is the largest |entry| among the rows
// not yet chosen, ties going to the lower position (what a search down the interchanged column
// finds). The multipliers and the rank-1 update run on registers; the pivot row reaches every
// lane through readlane. ipiv[kk] (if given) receives ipiv_off plus the position interchanged
// with kk at step kk. Returns whether a pivot was zero or not finite.
template <int NBT, int RPL>
__device__ __forceinline__ bool lu_regs(double (&a)[RPL][NBT], int (&pos)[RPL], int nrow, int nbk, int32_t* ipiv,
                                        int ipiv_off) {
    bool bad = false;
    const int lane = threadIdx.x & 63;
    bool live[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) live[r] = lane + 64 * r < nrow;
#pragma unroll
    for (int kk = 0; kk < NBT; ++kk) {
        if (kk < nbk) {
            double best = -1.0;
            int key = 0x7fffffff;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                // a NaN entry wins (the pivot check then flags the element): some live row is
                // always chosen
                double v = live[r] ? fabs(a[r][kk]) : -1.0;
                if (live[r] && !(v >= 0.0)) v = INFINITY;
                const int k = (pos[r] << 8) | (lane + 64 * r);
                if (v > best || (v == best && k < key)) { best = v; key = k; }
            }
            wave_ops::wave_argmax(best, key);
            const int ob = key & 255, p = key >> 8;
            const int ol = ob & 63, os = ob >> 6;
            double pv = panel_entry(a, os, kk, ol);
            if (ipiv && lane == 0) ipiv[kk] = ipiv_off + p;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                if (pos[r] == kk) pos[r] = p;
                if (lane == ol && r == os) { pos[r] = kk; live[r] = false; }
            }
            if (!(fabs(pv) > 0.0) || !isfinite(pv)) { bad = true; pv = 1.0; }
            const double inv = 1.0 / pv;
            double m[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                m[r] = live[r] ? a[r][kk] * inv : 0.0;
                if (live[r]) a[r][kk] = m[r];
            }
#pragma unroll
            for (int c = 0; c < NBT; ++c) {
                if (c > kk) {   // (constant trip count: both loops unroll, a stays in registers)
                    const double pc = panel_entry(a, os, c, ol);
#pragma unroll
                    for (int r = 0; r < RPL; ++r) a[r][c] = fma(-m[r], pc, a[r][c]);
                }
            }
        }
    }
    return bad;
}

// lu_regs on a panel in LDS (row stride ldp): loaded into registers, factorised, written back
// in the interchanged order; rsrc[position] receives the row's index before the interchanges.
template <int NBT, int RPL>
__device__ __forceinline__ bool panel_lu_regs(double* Pn, int ldp, int nrow, int nbk, int* rsrc, int32_t* ipiv,
                                              int ipiv_off) {
    const int lane = threadIdx.x & 63;
    double a[RPL][NBT];
    int pos[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int li = lane + 64 * r;
        pos[r] = li;
#pragma unroll
        for (int c = 0; c < NBT; ++c) {
            const bool ok = li < nrow && c < nbk;
            const double v = Pn[ok ? li * ldp + c : 0];
            a[r][c] = ok ? v : 0.0;
        }
    }
    const bool bad = lu_regs<NBT, RPL>(a, pos, nrow, nbk, ipiv, ipiv_off);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int li = lane + 64 * r;
        if (li < nrow) {
#pragma unroll
            for (int c = 0; c < NBT; ++c)
                if (c < nbk) Pn[pos[r] * ldp + c] = a[r][c];
            rsrc[pos[r]] = li;
        }
    }
    return bad;
}

// ---- LU of Ebar and X = Ebar^{-1} [Fbar | r_u] on the Ebar rows ------------------------------
// Works on the top nu rows of T only (row stride C): [Ebar | Fbar | r_u] becomes
// [L\U | X | x_r] with P Ebar = L U. The trace rows are not touched: they keep
// [Hbar | Jbar | r_t] for the Schur product Kbar = Jbar - Hbar X. Three kernels:
//   1. k_cond_getrf, one block per element: right-looking blocked LU of the nu x nu block
//      with partial pivoting, panels of NB columns. The panel is factorised by one wave (in
//      its registers, or in LDS for large elements), then the panel's interchanges are
//      applied to every other column of the block (the earlier columns of L included, so L
//      ends as LAPACK's getrf leaves it), U12 = L11^{-1} A12 (one thread per column) and the
//      trailing update A22 -= L21 U12 runs on the matrix cores. The interchanges go to ipiv
//      (step k exchanged positions k and ipiv[k]) and, composed, to perm (row i of P Ebar is
//      row perm[i] of Ebar);
//   2. k_cond_trinv, one block per (element, 32-row block): the inverses of the unit lower
//      and upper 32 x 32 diagonal blocks of L and U;
//   3. k_cond_getrs, one block per (element, slab of the nt + 1 right-hand-side columns): the
//      slab is gathered in the interchanged row order into LDS, and Y = U^{-1} L^{-1} Y runs
//      by 32-row blocks, each a product with the inverted diagonal block and an update of
//      the remaining rows, all on the matrix cores.

// Kernel 1: LU of the nu x nu block of the Ebar rows (see above). NBT: compile-time bound of
// the panel width; RPL: rows per lane of the register panel (0: the panel is factorised in
// LDS). Dynamic LDS: the nu x (NB+1) panel, then ints: rsrc [nu] (row interchanges of the
// panel), dsrc/ddst [NBT] (displaced rows), gperm/gtmp [nu] (composed interchanges).
template <int NBT, int LBS, int RPL>
__global__ __launch_bounds__(LBS, LBS == 256 ? (RPL * NBT >= 64 ? 2 : 3) : 1) void k_cond_getrf(
    CondDims cd, int NB, double* __restrict__ top, int* bad_elem, int e_off, int32_t* __restrict__ ipiv_out,
    int32_t* __restrict__ perm_out) {
    extern __shared__ double sm[];
    __shared__ int ndisp;
    __shared__ int sing;
    const long long e = blockIdx.x;
    const int nu = cd.nu, C = cd.C;
    double* Te = top + (size_t)e * nu * C;
    const int ldp = NB + 1;
    double* Pn = sm;                                   // nu x ldp: the panel
    int* rsrc = (int*)(sm + (size_t)nu * ldp);         // [nu]
    int* dsrc = rsrc + nu;                             // [NBT]
    int* ddst = dsrc + NBT;                            // [NBT]
    int* gperm = ddst + NBT;                           // [nu]
    int* gtmp = gperm + nu;                            // [nu]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x == 0) sing = 0;
    for (int r = threadIdx.x; r < nu; r += LBS) gperm[r] = r;
    for (int k0 = 0; k0 < nu; k0 += NB) {
        const int nbk = (nu - k0) < NB ? (nu - k0) : NB;
        const int nrow = nu - k0;
        // 1. load the panel (four loads in flight per thread)
        for (int base = threadIdx.x; base < nrow * nbk; base += 4 * LBS) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = base + u * LBS;
                const int li = idx / nbk, kk = idx - li * nbk;
                v[u] = idx < nrow * nbk ? Te[(size_t)(k0 + li) * C + k0 + kk] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = base + u * LBS;
                const int li = idx / nbk, kk = idx - li * nbk;
                if (idx < nrow * nbk) Pn[li * ldp + kk] = v[u];
            }
        }
        for (int r = threadIdx.x; r < nrow; r += LBS) rsrc[r] = r;
        if (threadIdx.x == 0) ndisp = 0;
        __syncthreads();
        // 2. one wave factorises the panel (pivot rows among the panel's rows): in its registers
        //    when every lane holds at most RPL rows, else in LDS
        if (RPL > 0 && wave == 0) {
            const bool bad = panel_lu_regs<NBT, (RPL > 0 ? RPL : 1)>(Pn, ldp, nrow, nbk, rsrc,
                                                                     ipiv_out + (size_t)e * nu + k0, k0);
            if (bad && lane == 0) sing = 1;
        }
        if (RPL == 0 && wave == 0) {
            bool bad = false;
            for (int kk = 0; kk < nbk; ++kk) {
                double best = -1.0;
                int bi = kk;
                for (int li = kk + lane; li < nrow; li += 64) {
                    const double v = fabs(Pn[li * ldp + kk]);
                    if (v > best || (v == best && li < bi)) { best = v; bi = li; }
                }
                wave_ops::wave_argmax(best, bi);
                double pv = Pn[bi * ldp + kk];
                if (lane == 0) {
                    if (ipiv_out) ipiv_out[(size_t)e * nu + k0 + kk] = k0 + bi;
                    const int t = rsrc[kk];
                    rsrc[kk] = rsrc[bi];
                    rsrc[bi] = t;
                }
                if (!(fabs(pv) > 0.0) || !isfinite(pv)) { bad = true; pv = 1.0; }
                if (bi != kk) {
                    for (int c = lane; c < nbk; c += 64) {
                        const double t = Pn[kk * ldp + c];
                        Pn[kk * ldp + c] = Pn[bi * ldp + c];
                        Pn[bi * ldp + c] = t;
                    }
                }
                wave_lds_sync();
                const double inv = 1.0 / pv;
                // rank-1 update of the rows below, CW columns at a time: the pivot row's and the
                // lane's row entries are all loaded before any is written (independent LDS loads in
                // flight instead of one read-modify-write chain per entry)
                constexpr int CW = NBT < 32 ? NBT : 32;
                for (int cb = 0; cb < nbk; cb += CW) {
                    if (cb + CW <= kk + 1) continue;
                    double prow[CW];
#pragma unroll
                    for (int c = 0; c < CW; ++c) {
                        const int cc = cb + c;
                        prow[c] = Pn[kk * ldp + ((cc > kk && cc < nbk) ? cc : kk)];
                    }
                    for (int li = kk + 1 + lane; li < nrow; li += 64) {
                        double* row = Pn + li * ldp;
                        double r[CW];
#pragma unroll
                        for (int c = 0; c < CW; ++c) {
                            const int cc = cb + c;
                            r[c] = row[(cc > kk && cc < nbk) ? cc : kk];
                        }
                        const double mlt = row[kk] * inv;
#pragma unroll
                        for (int c = 0; c < CW; ++c) {
                            const int cc = cb + c;
                            if (cc > kk && cc < nbk) row[cc] = r[c] - mlt * prow[c];
                        }
                    }
                }
                for (int li = kk + 1 + lane; li < nrow; li += 64) Pn[li * ldp + kk] *= inv;
                wave_lds_sync();
            }
            if (bad && lane == 0) sing = 1;
        }
        __syncthreads();
        // rows at or below nbk whose content moved (at most nbk of them); the order of
        // the list does not matter, each destination appears once
        for (int r = nbk + threadIdx.x; r < nrow; r += LBS) {
            if (rsrc[r] != r) {
                const int q = atomicAdd(&ndisp, 1);
                dsrc[q] = rsrc[r];
                ddst[q] = r;
            }
        }
        // 3. the factorised panel back to T (U11 and the multipliers L21), and the panel's
        //    interchanges composed into gperm
        for (int idx = threadIdx.x; idx < nrow * nbk; idx += LBS) {
            const int li = idx / nbk, kk = idx - li * nbk;
            Te[(size_t)(k0 + li) * C + k0 + kk] = Pn[li * ldp + kk];
        }
        for (int r = threadIdx.x; r < nrow; r += LBS) gtmp[r] = gperm[k0 + rsrc[r]];
        __syncthreads();
        for (int r = threadIdx.x; r < nrow; r += LBS) gperm[k0 + r] = gtmp[r];
        // 4. the panel's interchanges on every other column of the block (rows k0..): the
        //    columns left of the panel (earlier multipliers) are only permuted, the trailing
        //    ones also get U12 = L11^{-1} A12 (one thread per column)
        const int cbeg = k0 + nbk;
        const int ncol = k0 + (nu - cbeg);
        const int nd = ndisp;
        // the pivot rows' offsets from row k0 are read from LDS once, before any global load
        // (reads past the valid entries stay inside the LDS allocation and are replaced by row 0)
        int rs[NBT];
#pragma unroll
        for (int t = 0; t < NBT; ++t) rs[t] = rsrc[t];
#pragma unroll
        for (int t = 0; t < NBT; ++t) rs[t] = (t < nbk ? rs[t] : 0) * C;
        for (int cl = threadIdx.x; cl < ncol; cl += LBS) {
            const bool trailing = cl >= k0;
            double* Tc = Te + (size_t)k0 * C + (trailing ? cbeg + (cl - k0) : cl);   // this column, from row k0 on
            double u[NBT];
#pragma unroll
            for (int t = 0; t < NBT; ++t) u[t] = Tc[rs[t]];
            // displaced rows: sources lie among the first nbk rows, destinations below them, and
            // the pivot rows are already loaded; eight moves at a time, their loads issued together
            for (int q0 = 0; q0 < nd; q0 += 8) {
                double mv[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) mv[q] = Tc[(size_t)dsrc[q0 + q < nd ? q0 + q : q0] * C];
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (q0 + q < nd) Tc[(size_t)ddst[q0 + q] * C] = mv[q];
            }
            if (trailing) {
                // forward substitution with the unit lower L11
#pragma unroll
                for (int kk = 1; kk < NBT; ++kk) {
                    if (kk < nbk) {
                        double v = u[kk];
#pragma unroll
                        for (int q = 0; q < kk; ++q) v -= Pn[kk * ldp + q] * u[q];
                        u[kk] = v;
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < NBT; ++t)
                if (t < nbk) Tc[(size_t)t * C] = u[t];
        }
        __syncthreads();
        // 5. trailing update of the block (MFMA, 32x32 tiles per wave)
        const int na = nu - cbeg;
        const int ta_c = (na + 31) / 32;
        const int tA = ta_c * ta_c;
        for (int tile = wave; tile < tA; tile += LBS / 64) {
            const int r0 = cbeg + (tile / ta_c) * 32;
            const int c0 = cbeg + (tile % ta_c) * 32;
            double4_t acc[2][2];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int r = r0 + 16 * bi + 4 * q + (lane >> 4);
                        const int c = c0 + 16 * bj + (lane & 15);
                        const bool ok = r < nu && c < nu;
                        const double v = Te[ok ? (size_t)r * C + c : (size_t)cbeg * C + cbeg];
                        acc[bi][bj][q] = ok ? v : 0.0;
                    }
            auto la = [&](int i, int k) -> double {
                const int r = r0 + i;
                const bool ok = r < nu && k < nbk;
                const double v = Pn[ok ? (r - k0) * ldp + k : 0];
                return ok ? -v : 0.0;
            };
            auto lb = [&](int k, int j) -> double {
                const int c = c0 + j;
                const bool ok = k < nbk && c < nu;
                const double v = Te[ok ? (size_t)(k0 + k) * C + c : (size_t)k0 * C + cbeg];
                return ok ? v : 0.0;
            };
            mfma_32x32(la, lb, nbk, acc);
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int r = r0 + 16 * bi + 4 * q + (lane >> 4);
                        const int c = c0 + 16 * bj + (lane & 15);
                        if (r < nu && c < nu) Te[(size_t)r * C + c] = acc[bi][bj][q];
                    }
        }
        __syncthreads();
    }
    for (int r = threadIdx.x; r < nu; r += LBS) perm_out[(size_t)e * nu + r] = gperm[r];
    if (sing && threadIdx.x == 0) atomicMin(bad_elem, e_off + (int)e);
}

// Kernel 1 for nu <= NBT <= 64: one wave per element factorises the whole nu x nu block in its
// registers (lane l holds row l), no LDS and no block barrier; the rows of L\U are written back
// in the interchanged order (the right-hand-side columns stay in place: the solve gathers them
// through perm).
template <int NBT>
__global__ __launch_bounds__(64) void k_cond_getrf_w(CondDims cd, double* __restrict__ top, int* bad_elem,
                                                     int e_off, int32_t* __restrict__ ipiv_out,
                                                     int32_t* __restrict__ perm_out) {
    const long long e = blockIdx.x;
    const int nu = cd.nu, C = cd.C;
    double* Te = top + (size_t)e * nu * C;
    const int lane = threadIdx.x & 63;
    const int rl = lane < nu ? lane : nu - 1;
    double a[1][NBT];
    int pos[1] = {lane};
#pragma unroll
    for (int c = 0; c < NBT; ++c) {
        const bool ok = lane < nu && c < nu;
        const double v = Te[(size_t)rl * C + (c < nu ? c : 0)];
        a[0][c] = ok ? v : 0.0;
    }
    const bool bad = lu_regs<NBT, 1>(a, pos, nu, nu, ipiv_out + (size_t)e * nu, 0);
    if (lane < nu) {
#pragma unroll
        for (int c = 0; c < NBT; ++c)
            if (c < nu) Te[(size_t)pos[0] * C + c] = a[0][c];
        perm_out[(size_t)e * nu + pos[0]] = lane;
    }
    if (bad && lane == 0) atomicMin(bad_elem, e_off + (int)e);
}

// Kernel 2: inverses of the 32 x 32 diagonal blocks of L (unit lower) and U (upper), one
// block of 64 threads per (element, block row): thread t < 32 forms column t of inv(L_kb),
// thread 32 + t column t of inv(U_kb), with the blocks in LDS. A last partial block (nu not
// a multiple of 32) is completed with the identity. Output dinv[e][kb][0 / 1][32][32]
// (row-major).
__global__ __launch_bounds__(64) void k_cond_trinv(CondDims cd, const double* __restrict__ top,
                                                   double* __restrict__ dinv) {
    __shared__ double blk[32][33];
    const int nu = cd.nu, C = cd.C;
    const int nkb = (nu + 31) / 32;
    const long long e = blockIdx.x / nkb;
    const int kb = (int)(blockIdx.x - e * nkb);
    const int r0 = kb * 32, rb = (nu - r0) < 32 ? (nu - r0) : 32;
    const double* Te = top + (size_t)e * nu * C;
    for (int idx = threadIdx.x; idx < 32 * 32; idx += 64) {
        const int i = idx >> 5, j = idx & 31;
        const bool ok = i < rb && j < rb;
        const double v = Te[ok ? (size_t)(r0 + i) * C + r0 + j : 0];
        blk[i][j] = ok ? v : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    const int t = threadIdx.x & 31;
    double x[32];
    if (threadIdx.x < 32) {
        // L x = e_t, L unit lower
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            double v = i == t ? 1.0 : 0.0;
#pragma unroll
            for (int j = 0; j < i; ++j) v -= blk[i][j] * x[j];
            x[i] = v;
        }
    } else {
        // U x = e_t, U upper
#pragma unroll
        for (int i = 31; i >= 0; --i) {
            double v = i == t ? 1.0 : 0.0;
#pragma unroll
            for (int j = i + 1; j < 32; ++j) v -= blk[i][j] * x[j];
            x[i] = v / blk[i][i];
        }
    }
    double* out = dinv + ((size_t)e * nkb + kb) * 2048 + (threadIdx.x < 32 ? 0 : 1024);
#pragma unroll
    for (int i = 0; i < 32; ++i) out[i * 32 + t] = x[i];
}

// Kernel 3: Y = U^{-1} L^{-1} P Y on the right-hand-side columns, one block per (element,
// slab of sw <= 32 columns). LDS: the slab, nu rows x SLAB_LD.
constexpr int SLAB_LD = 33;

__global__ __launch_bounds__(256, 2) void k_cond_getrs(CondDims cd, long long nblk, int nsl, int sw,
                                                       double* __restrict__ top, const int32_t* __restrict__ perm,
                                                       const double* __restrict__ dinv) {
    extern __shared__ double Y[];
    const long long Lb = xcd_linear(gridDim.x);
    if (Lb >= nblk) return;
    const long long e = Lb / nsl;
    const int s = (int)(Lb - e * nsl);
    const int nu = cd.nu, C = cd.C;
    const int c0 = nu + s * sw;
    const int ncs = (C - c0) < sw ? (C - c0) : sw;
    double* Te = top + (size_t)e * nu * C;
    const int32_t* pe = perm + (size_t)e * nu;
    const int nkb = (nu + 31) / 32;
    const double* De = dinv + (size_t)e * nkb * 2048;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // the slab's rows in the interchanged order
    for (int idx = threadIdx.x; idx < nu * 32; idx += 256) {
        const int i = idx >> 5, j = idx & 31;
        const bool ok = j < ncs;
        const double v = Te[(size_t)pe[i] * C + c0 + (ok ? j : 0)];
        Y[i * SLAB_LD + j] = ok ? v : 0.0;
    }
    __syncthreads();
    // Y_kb <- inv(diagonal block) Y_kb, by one wave (a 32 x 32 x 32 product)
    auto diag = [&](int kb, int which) {
        const int r0 = kb * 32;
        const int rb = (nu - r0) < 32 ? (nu - r0) : 32;
        const double* Di = De + (size_t)kb * 2048 + which * 1024;
        double4_t acc[2][2];
        acc_zero(acc);
        auto la = [&](int i, int k) -> double {
            const bool ok = k < 32;
            const double v = Di[i * 32 + (ok ? k : 0)];
            return ok ? v : 0.0;
        };
        auto lb = [&](int k, int j) -> double {
            const bool ok = k < rb;
            const double v = Y[(r0 + (ok ? k : 0)) * SLAB_LD + j];
            return ok ? v : 0.0;
        };
        mfma_32x32(la, lb, 32, acc);
        wave_lds_sync();
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = 16 * bi + 4 * q + (lane >> 4);
                    const int c = 16 * bj + (lane & 15);
                    if (r < rb) Y[(r0 + r) * SLAB_LD + c] = acc[bi][bj][q];
                }
    };
    // Y_t -= A[rows of block t][columns of block kb] Y_kb (A = L below the diagonal, U above)
    auto update = [&](int t, int kb) {
        const int rr = t * 32, r0 = kb * 32;
        const int rb = (nu - r0) < 32 ? (nu - r0) : 32;
        double4_t acc[2][2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = rr + 16 * bi + 4 * q + (lane >> 4);
                    const int c = 16 * bj + (lane & 15);
                    const bool ok = r < nu;
                    const double v = Y[(ok ? r : 0) * SLAB_LD + c];
                    acc[bi][bj][q] = ok ? v : 0.0;
                }
        auto la = [&](int i, int k) -> double {
            const int r = rr + i;
            const bool ok = r < nu && k < rb;
            const double v = Te[ok ? (size_t)r * C + r0 + k : 0];
            return ok ? -v : 0.0;
        };
        auto lb = [&](int k, int j) -> double {
            const bool ok = k < rb;
            const double v = Y[(r0 + (ok ? k : 0)) * SLAB_LD + j];
            return ok ? v : 0.0;
        };
        mfma_32x32(la, lb, rb, acc);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = rr + 16 * bi + 4 * q + (lane >> 4);
                    const int c = 16 * bj + (lane & 15);
                    if (r < nu) Y[r * SLAB_LD + c] = acc[bi][bj][q];
                }
    };
    // forward: L (unit lower), 32-row blocks from the top
    for (int kb = 0; kb < nkb; ++kb) {
        if (wave == 0) diag(kb, 0);
        __syncthreads();
        for (int t = kb + 1 + wave; t < nkb; t += 4) update(t, kb);
        __syncthreads();
    }
    // backward: U, 32-row blocks from the bottom
    for (int kb = nkb - 1; kb >= 0; --kb) {
        if (wave == 0) diag(kb, 1);
        __syncthreads();
        for (int t = wave; t < kb; t += 4) update(t, kb);
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < nu * 32; idx += 256) {
        const int i = idx >> 5, j = idx & 31;
        if (j < ncs) Te[(size_t)i * C + c0 + j] = Y[i * SLAB_LD + j];
    }
}

// Order of the block products of the register-resident solve (k_cond_getrs_b): forward with
// L by 32-row blocks from the top, then backward with U from the bottom.
struct SolveOp {
    int kind;   // 0: Y_kb <- inv(L_kb) Y_kb, 1: Y_kb <- inv(U_kb) Y_kb, 2: Y_t -= T_t,kb Y_kb
    int t, kb;
};

template <int NKB>
struct SolvePlan {
    static constexpr int N = NKB * (NKB + 1);
    SolveOp op[N];
    constexpr SolvePlan() : op() {
        int n = 0;
        for (int kb = 0; kb < NKB; ++kb) {
            op[n++] = SolveOp{0, kb, kb};
            for (int t = kb + 1; t < NKB; ++t) op[n++] = SolveOp{2, t, kb};
        }
        for (int kb = NKB - 1; kb >= 0; --kb) {
            op[n++] = SolveOp{1, kb, kb};
            for (int t = 0; t < kb; ++t) op[n++] = SolveOp{2, t, kb};
        }
    }
};

// Kernel 3 for elements of NKB <= 6 blocks of 32 rows (nu <= 192), with the Schur product
// fused: one block of four waves per 64 consecutive right-hand-side columns of one element,
// one 16-column slab per wave. The slab lives in the wave's registers in the matrix cores'
// accumulator layout (row 16 bi + 4 q + lane/16, column lane%16 of 32-row block t in
// Y[t][bi][q]); that layout is also the B-operand layout of a product whose k runs as
// 16 bi + 4 q + lane/16, so each product A Y_kb reads Y_kb where it lies. The products run in
// a fixed order: the solve (inverted diagonal block times Y_kb, or a block of L / U times
// -Y_kb), then, for each 32-row block of the trace rows, [Jbar | r_t] - Hbar X for the slab's
// columns. Each A block (32 x 32) is loaded once per block, with 16-byte coalesced loads, into
// LDS (rows padded to 34: the operand reads, 16 rows x 4 columns per instruction, hit distinct
// banks), double-buffered with one barrier per product. Output: X and x_r into T's top rows,
// Kbar and rbar for the slab's columns.
constexpr int ALD = 34;

// (Two blocks per CU, 256 VGPRs each; the five-block variants spill a few registers at that
// size and still run faster than at one block per CU: 18.4 -> 15.8 ms for the Navier-Stokes
// hexes. The six-block variant with a partial last block would spill far more and runs one
// block per CU.)
template <int NKB, bool FULL>
__global__ __launch_bounds__(256, (NKB == 6 && !FULL) ? 1 : 2) void k_cond_getrs_b(CondDims cd, long long nblk, int nbe,
                                                         double* __restrict__ top, const double* __restrict__ bot,
                                                         const int32_t* __restrict__ perm,
                                                         const double* __restrict__ dinv, double* __restrict__ Kbar,
                                                         double* __restrict__ rbar) {
    __shared__ double As[2][32 * ALD];
    const long long Lb = xcd_linear(gridDim.x);
    if (Lb >= nblk) return;
    const long long e = Lb / nbe;
    const int b = (int)(Lb - e * nbe);
    const int nu = cd.nu, nt = cd.nt, C = cd.C;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, i16 = lane & 15, kq = lane >> 4;
    const int g0 = 64 * b + 16 * wave;                   // the slab's first right-hand-side column
    const int ncs = (C - nu - g0) < 16 ? (C - nu - g0) : 16;   // may be <= 0: an idle slab
    double* __restrict__ Te = top + (size_t)e * nu * C;
    const double* __restrict__ Be = bot + (size_t)e * nt * C;
    const int32_t* __restrict__ pe = perm + (size_t)e * nu;
    const double* __restrict__ De = dinv + (size_t)e * NKB * 2048;
    const int cl = ncs <= 0 ? 0 : g0 + (i16 < ncs ? i16 : ncs - 1);   // this lane's column (clamped)
    const double cmask = i16 < ncs ? 1.0 : 0.0;
    double4_t Y[NKB][2];
#pragma unroll
    for (int t = 0; t < NKB; ++t)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = 32 * t + 16 * bi + 4 * q + kq;
                const int rc = FULL ? r : (r < nu ? r : nu - 1);
                const double v = Te[pe[rc] * C + nu + cl];
                Y[t][bi][q] = v * (FULL || r < nu ? cmask : 0.0);
            }
    // cooperative tile load: thread (row tr = tid / 8, columns 4 (tid % 8) .. +3) of the 32 x 32 A
    const int tr = threadIdx.x >> 3, tc = 4 * (threadIdx.x & 7);
    // A = a 32 x 32 block of M (row stride C, rows [r0, r0 + 32) clamped below rmax, columns
    // [k0, k0 + 32) masked beyond kmax), zero outside
    auto gload_blk = [&](const double* __restrict__ M, int r0, int rmax, int k0, int kmax, bool full,
                         double (&v)[4]) {
        const int r = r0 + tr;
        const int rc = full ? r : (r < rmax ? r : rmax - 1);
        const double* __restrict__ row = M + rc * C + k0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = tc + u;
            if (full) {
                v[u] = row[k];
            } else {
                const int kb = kmax - k0;
                const double x = row[k < kb ? k : kb - 1];
                v[u] = x * ((r < rmax && k < kb) ? 1.0 : 0.0);
            }
        }
    };
    auto gload = [&](const SolveOp& o, double (&v)[4]) {
        if (o.kind < 2) {
            const double* __restrict__ Di = De + o.kb * 2048 + o.kind * 1024 + tr * 32 + tc;
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = Di[u];
        } else {
            gload_blk(Te, 32 * o.t, nu, 32 * o.kb, nu, FULL, v);
        }
    };
    auto lstore = [&](int buf, const double (&v)[4]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) As[buf][tr * ALD + tc + u] = v[u];
    };
    // out += A B, A from LDS buffer buf (lane (i16, kq): A[16 ai + i16][16 bi + 4 q + kq])
    auto mma = [&](double4_t (&out)[2], int buf, const double4_t (&B)[2]) {
        double a[2][4][2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int ai = 0; ai < 2; ++ai) a[bi][q][ai] = As[buf][(16 * ai + i16) * ALD + 16 * bi + 4 * q + kq];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int ai = 0; ai < 2; ++ai)
                    out[ai] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi][q][ai], B[bi][q], out[ai], 0, 0, 0);
    };
    constexpr SolvePlan<NKB> plan;
    constexpr int NS = SolvePlan<NKB>::N;
    const int ntb = (nt + 31) / 32;
    const bool tfull = FULL && nt % 32 == 0;
    double4_t nY[2];   // -Y_kb of the latest diagonal step
    double v[4];
    gload(plan.op[0], v);
    lstore(0, v);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const int buf = i & 1;
        if (i + 1 < NS) gload(plan.op[i + 1 < NS ? i + 1 : 0], v);
        else gload_blk(Be, 0, nt, 0, nu, tfull, v);       // first block of Hbar
        const SolveOp o = plan.op[i];
        if (o.kind == 2) {
            mma(Y[o.t], buf, nY);
        } else {
            double4_t nw[2] = {double4_t{0.0, 0.0, 0.0, 0.0}, double4_t{0.0, 0.0, 0.0, 0.0}};
            mma(nw, buf, Y[o.kb]);
            Y[o.kb][0] = nw[0];
            Y[o.kb][1] = nw[1];
            nY[0] = -nw[0];   // the updates that follow subtract T Y_kb
            nY[1] = -nw[1];
        }
        lstore(buf ^ 1, v);
        __syncthreads();
    }
    // X and x_r of the slab back to T
    if (ncs > 0) {
#pragma unroll
        for (int t = 0; t < NKB; ++t)
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = 32 * t + 16 * bi + 4 * q + kq;
                    if ((FULL || r < nu) && i16 < ncs) Te[r * C + nu + g0 + i16] = Y[t][bi][q];
                }
    }
    // -X, the B operand of the Schur products
#pragma unroll
    for (int t = 0; t < NKB; ++t) {
        Y[t][0] = -Y[t][0];
        Y[t][1] = -Y[t][1];
    }
    // [Kbar | rbar] = [Jbar | r_t] - Hbar X for the slab's columns, 32 trace rows at a time
    const int g = cl;                                    // column of [Jbar | r_t] (clamped)
    int par = NS & 1;                                    // the buffer holding the next A block
    for (int rt = 0; rt < ntb; ++rt) {
        double4_t acc[2];
#pragma unroll
        for (int ai = 0; ai < 2; ++ai)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = 32 * rt + 16 * ai + 4 * q + kq;
                const int rc = r < nt ? r : nt - 1;
                acc[ai][q] = Be[rc * C + nu + g];
            }
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
            // the next A block: Hbar block (rt, kb + 1), or (rt + 1, 0)
            const bool last = kb + 1 == NKB && rt + 1 == ntb;
            if (!last) {
                if (kb + 1 < NKB) gload_blk(Be, 32 * rt, nt, 32 * (kb + 1), nu, tfull, v);
                else gload_blk(Be, 32 * (rt + 1), nt, 0, nu, tfull, v);
            }
            mma(acc, par, Y[kb]);
            if (!last) lstore(par ^ 1, v);
            __syncthreads();
            par ^= 1;
        }
        if (ncs > 0 && i16 < ncs) {
            const int gc = g0 + i16;
#pragma unroll
            for (int ai = 0; ai < 2; ++ai)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = 32 * rt + 16 * ai + 4 * q + kq;
                    if (r < nt) {
                        if (gc < nt) Kbar[((size_t)e * nt + r) * nt + gc] = acc[ai][q];
                        else rbar[(size_t)e * nt + r] = acc[ai][q];
                    }
                }
        }
    }
}

// ---- Kbar = Jbar - Hbar X, rbar = r_t - Hbar x_r   per (element, 64x64 tile) ----------------
// Hbar = the trace rows' first nu columns, X and x_r = the Ebar rows' columns nu.. after the
// elimination and back substitution: one product of depth nu.
__global__ __launch_bounds__(BS, 2) void k_cond_schur(CondDims cd, long long ntile, int tm_n, int tn_n,
                                                   const double* __restrict__ top, const double* __restrict__ bot,
                                                   double* __restrict__ Kbar, double* __restrict__ rbar) {
    extern __shared__ double lds[];
    const long long L = xcd_linear(gridDim.x);
    if (L >= ntile) return;
    const int per_e = tm_n * tn_n;
    const long long e = L / per_e;
    const int rem = (int)(L - e * per_e);
    const int m0 = (rem / tn_n) * GT, n0 = (rem % tn_n) * GT;
    const int nu = cd.nu, nt = cd.nt, C = cd.C;
    const double* Te = top + (size_t)e * nu * C;
    const double* Be = bot + (size_t)e * nt * C;
    const MatA Am{Be, Be, nt, C, nt, nu};
    const MatB Bm{Te + nu, C, nu, nt};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = m0 + (wave >> 1) * 32, c0 = n0 + (wave & 1) * 32;
    double j0[2][2][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + 16 * bi + 4 * q + (lane >> 4);
                const int c = c0 + 16 * bj + (lane & 15);
                const bool ok = r < nt && c < nt;
                j0[bi][bj][q] = Be[ok ? (size_t)r * C + nu + c : 0];
            }
    double4_t acc[2][2];
    acc_zero(acc);
    gemm_tile64(Am, Bm, m0, n0, lds, acc);
    double* Ke = Kbar + (size_t)e * nt * nt;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + 16 * bi + 4 * q + (lane >> 4);
                const int c = c0 + 16 * bj + (lane & 15);
                if (r < nt && c < nt) Ke[(size_t)r * nt + c] = j0[bi][bj][q] - acc[bi][bj][q];
            }
    // rbar for this row tile: four lanes per row, fixed-order combination
    if (n0 == 0) {
        const int r = m0 + (threadIdx.x >> 2), part = threadIdx.x & 3;
        double sum = 0.0;
        if (r < nt)
            for (int k = part; k < nu; k += 4) sum += Be[(size_t)r * C + k] * Te[(size_t)k * C + C - 1];
        sum += __shfl_xor(sum, 1, 64);
        sum += __shfl_xor(sum, 2, 64);
        if (r < nt && part == 0) rbar[(size_t)e * nt + r] = Be[(size_t)r * C + C - 1] - sum;
    }
}

// Hbar (the trace rows' first nu columns, which the elimination leaves as they are), per
// element, out of the workspace into a caller buffer [n][nt][nu].
__global__ __launch_bounds__(BS) void k_copy_hbar(CondDims cd, const double* __restrict__ bot,
                                                  double* __restrict__ Hbar) {
    const long long e = blockIdx.x;
    const int nu = cd.nu, nt = cd.nt, C = cd.C;
    for (int idx = threadIdx.x; idx < nt * nu; idx += BS) {
        const int t = idx / nu, r = idx - t * nu;
        Hbar[(size_t)e * nt * nu + idx] = bot[((size_t)e * nt + t) * C + r];
    }
}

// Right-hand side of the condensation for a new (r_u, r_t) with the factors a previous
// elimination of the same element matrices left (the stages of a DIRK step solve systems
// with the same matrix and new right-hand sides, Section 2.2):
//     c = L^{-1} P r_u   (all interchanges in order, then the unit lower L by blocks of NB
//                         rows: the block's triangle, then its multipliers below it),
//     x_r = U^{-1} c,    rbar = r_t - Hbar x_r.
// x_r replaces the last column of `local` (recovery reads it). One block per element, the
// vector in LDS.
__global__ __launch_bounds__(BS) void k_cond_rhs(CondDims cd, int NB, double* __restrict__ local,
                                                 const double* __restrict__ Hbar, const int32_t* __restrict__ ipiv,
                                                 const double* __restrict__ ru, const double* __restrict__ rt,
                                                 double* __restrict__ rbar) {
    extern __shared__ double y[];          // nu
    const long long e = blockIdx.x;
    const int nu = cd.nu, nt = cd.nt, C = cd.C;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double* Te = local + (size_t)e * nu * C;
    const int32_t* pv = ipiv + (size_t)e * nu;
    for (int i = threadIdx.x; i < nu; i += BS) y[i] = ru[(size_t)e * nu + i];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int kk = 0; kk < nu; ++kk) {
            const int p = pv[kk];
            if (p != kk) {
                const double a = y[kk];
                y[kk] = y[p];
                y[p] = a;
            }
        }
    }
    __syncthreads();
    for (int k0 = 0; k0 < nu; k0 += NB) {
        const int nbk = (nu - k0) < NB ? (nu - k0) : NB;
        if (wave == 0) {
            // the block's unit lower triangle: lane t holds y[k0+t]
            double yt = lane < nbk ? y[k0 + lane] : 0.0;
            for (int kk = 0; kk + 1 < nbk; ++kk) {
                const bool below = lane > kk && lane < nbk;
                const double l = Te[(size_t)(k0 + (below ? lane : kk)) * C + k0 + kk];
                const double ykk = lane_value(yt, kk);
                yt -= below ? l * ykk : 0.0;
            }
            if (lane < nbk) y[k0 + lane] = yt;
        }
        __syncthreads();
        // rows below the block
        for (int i = k0 + nbk + threadIdx.x; i < nu; i += BS) {
            const double* li = Te + (size_t)i * C + k0;
            double acc = 0.0;
            for (int kk = 0; kk < nbk; ++kk) acc += li[kk] * y[k0 + kk];
            y[i] -= acc;
        }
        __syncthreads();
    }
    wave_ops::upper_solve_lds<BS>(Te, C, nu, y);
    for (int i = threadIdx.x; i < nu; i += BS) Te[(size_t)i * C + C - 1] = y[i];
    // rbar = r_t - Hbar x_r, four rows per wave at a time
    for (int t0 = 4 * wave; t0 < nt; t0 += 4 * (BS / 64)) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int r0 = 0; r0 < nu; r0 += 64) {
            const int r = r0 + lane;
            const bool ok = r < nu;
            const double yv = y[ok ? r : 0];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = t0 + q < nt ? t0 + q : nt - 1;
                const double a = Hbar[((size_t)e * nt + t) * nu + (ok ? r : 0)];
                acc[q] += ok ? a * yv : 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double v = acc[q];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0 && t0 + q < nt) rbar[(size_t)e * nt + t0 + q] = rt[(size_t)e * nt + t0 + q] - v;
        }
    }
}

size_t lu_lds_bytes(const CondDims& cd, int NB) {
    return sizeof(double) * (size_t)cd.nu * (NB + 1) + sizeof(int) * (3 * (size_t)cd.nu + 2 * 64);
}

// LDS of the right-hand-side solve: one slab of the element's nu rows
size_t getrs_lds_bytes(const CondDims& cd) { return sizeof(double) * (size_t)cd.nu * SLAB_LD; }

// Workspace of the elimination per element: the inverted diagonal blocks, perm and ipiv.
size_t lu_ws_bytes_per_elem(const CondDims& cd) {
    const size_t nkb = (cd.nu + 31) / 32;
    return sizeof(double) * nkb * 2048 + 2 * sizeof(int32_t) * cd.nu;
}

// Panel width of the factorisation: all nu columns when nu <= 32 (one panel), else 16 (8 when
// the panel does not fit in LDS); 0 when even 8 does not fit or a slab of the right-hand-side
// solve does not. (Measured on the 192-unknown elasticity elements: panels of 16 factorised in
// registers condense in 90 ms, of 32 in registers in 94 ms, of 16 / 32 in LDS in 92 / 98 ms;
// on the 50-unknown Navier-Stokes tets, panels of 16 on 256 threads in 112 ms where one panel
// of 50 on 128 threads took 203 ms.)
int pick_panel(const CondDims& cd) {
    const size_t lds_cap = 150 * 1024;
    if (getrs_lds_bytes(cd) > lds_cap) return 0;
    if (cd.nu <= 32) return cd.nu;
    if (lu_lds_bytes(cd, 16) <= lds_cap) return 16;
    if (lu_lds_bytes(cd, 8) <= lds_cap) return 8;
    return 0;
}

// The factorisation kernel: for nu <= 64 one wave per element with the whole block in its
// registers (k_cond_getrf_w; on the 50-unknown Navier-Stokes tets it replaced panels of 16 on
// four waves); else four waves per element (several elements share a CU: the panel of one is
// factorised while others run on the matrix cores), panels of at most 256 rows factorised in
// one wave's registers (at most four rows per lane), larger ones in LDS.
const void* getrf_kernel(const CondDims& cd, int NB, int* threads) {
    if (cd.nu <= 64) {
        *threads = 64;
        return cd.nu <= 32 ? (const void*)k_cond_getrf_w<32> : (const void*)k_cond_getrf_w<64>;
    }
    *threads = 256;
    switch ((cd.nu + 63) / 64) {
        case 2: return (const void*)k_cond_getrf<16, 256, 2>;
        case 3: return (const void*)k_cond_getrf<16, 256, 3>;
        case 4: return (const void*)k_cond_getrf<16, 256, 4>;
        default: return (const void*)k_cond_getrf<16, 256, 0>;
    }
}

hdg_status set_kernel_lds(hdg_ctx ctx, const CondDims& cd, int NB) {
    const size_t lds = lu_lds_bytes(cd, NB);
    int threads = 0;
    const void* lu_fn = getrf_kernel(cd, NB, &threads);
    if (cd.nu > 64 && lds > 64 * 1024)
        HDG_HIP_CHECK(ctx, hipFuncSetAttribute(lu_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (getrs_lds_bytes(cd) > 64 * 1024)
        HDG_HIP_CHECK(ctx, hipFuncSetAttribute((const void*)k_cond_getrs, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)getrs_lds_bytes(cd)));
    HDG_HIP_CHECK(ctx, hipFuncSetAttribute((const void*)k_cond_schur, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)GEMM_LDS));
    return HDG_OK;
}

// Stages 2 and 3 on n elements whose matrices T are in place (top rows at `top`, row stride
// cd.C, trace rows at `bot`): LU of Ebar (L and U left in the first nu columns of the top
// rows) and X = Ebar^{-1}[Fbar | r_u] in their other columns, then the Schur product into
// Kout [n][nt][nt] and rout [n][nt]. A zero pivot records e_off + element in status. ipiv
// (optional, [n][nu]) receives the row interchanges; without it they go to the workspace.
hdg_status eliminate_and_schur(hdg_ctx ctx, const CondDims& cd, int NB, int64_t n, double* top, double* bot,
                               double* Kout, double* rout, int* status, int64_t e_off, int32_t* ipiv = nullptr) {
    hdg_status st;
    const int nkb = (cd.nu + 31) / 32;
    double* dinv = (double*)ws_get(ctx, WS_LU, lu_ws_bytes_per_elem(cd) * (size_t)n, &st);
    if (!dinv) return st;
    int32_t* perm = (int32_t*)(dinv + (size_t)n * nkb * 2048);
    int32_t* ipw = ipiv ? ipiv : perm + (size_t)n * cd.nu;
    int threads = 0;
    const void* lu_fn = getrf_kernel(cd, NB, &threads);
    int e_off_i = (int)e_off;
    if (cd.nu <= 64) {
        void* args[] = {(void*)&cd, (void*)&top, (void*)&status, (void*)&e_off_i, (void*)&ipw, (void*)&perm};
        HDG_HIP_CHECK(ctx, hipLaunchKernel(lu_fn, dim3((unsigned)n), dim3(threads), args, 0, ctx->stream));
    } else {
        void* args[] = {(void*)&cd, (void*)&NB, (void*)&top, (void*)&status, (void*)&e_off_i, (void*)&ipw,
                        (void*)&perm};
        HDG_HIP_CHECK(ctx, hipLaunchKernel(lu_fn, dim3((unsigned)n), dim3(threads), args, lu_lds_bytes(cd, NB),
                                           ctx->stream));
    }
    HDG_LAUNCH_CHECK(ctx);
    hipLaunchKernelGGL(k_cond_trinv, dim3((unsigned)(n * nkb)), dim3(64), 0, ctx->stream, cd, (const double*)top,
                       dinv);
    HDG_LAUNCH_CHECK(ctx);
    const int ncx = cd.C - cd.nu;
    if (nkb <= 6) {
        // four slabs of 16 columns per block, in registers, sharing each A block through LDS;
        // the Schur product fused
        const int nbe = div_up(ncx, 64);
        const long long nb_all = (long long)n * nbe;
        const long long gridb = (nb_all + 7) / 8 * 8;
        const void* fns[2][6] = {
            {(const void*)k_cond_getrs_b<1, false>, (const void*)k_cond_getrs_b<2, false>,
             (const void*)k_cond_getrs_b<3, false>, (const void*)k_cond_getrs_b<4, false>,
             (const void*)k_cond_getrs_b<5, false>, (const void*)k_cond_getrs_b<6, false>},
            {(const void*)k_cond_getrs_b<1, true>, (const void*)k_cond_getrs_b<2, true>,
             (const void*)k_cond_getrs_b<3, true>, (const void*)k_cond_getrs_b<4, true>,
             (const void*)k_cond_getrs_b<5, true>, (const void*)k_cond_getrs_b<6, true>}};
        const void* fn = fns[cd.nu % 32 == 0 ? 1 : 0][nkb - 1];
        const double* bc = bot;
        const int32_t* pc = perm;
        const double* dc = dinv;
        void* a3[] = {(void*)&cd, (void*)&nb_all, (void*)&nbe, (void*)&top, (void*)&bc, (void*)&pc, (void*)&dc,
                      (void*)&Kout, (void*)&rout};
        HDG_HIP_CHECK(ctx, hipLaunchKernel(fn, dim3((unsigned)gridb), dim3(BS), a3, 0, ctx->stream));
        HDG_LAUNCH_CHECK(ctx);
        return HDG_OK;
    }
    // larger elements: one block per slab of at most 32 columns in LDS (balanced, none empty),
    // then the Schur product on the tile engine
    const int sw = div_up(ncx, div_up(ncx, 32));
    const int nsl = div_up(ncx, sw);
    const long long nslab = (long long)n * nsl;
    hipLaunchKernelGGL(k_cond_getrs, dim3((unsigned)((nslab + 7) / 8 * 8)), dim3(BS), getrs_lds_bytes(cd), ctx->stream,
                       cd, nslab, nsl, sw, top, (const int32_t*)perm, (const double*)dinv);
    HDG_LAUNCH_CHECK(ctx);
    const int tm_n = div_up(cd.nt, GT);
    const long long ntile = (long long)n * tm_n * tm_n;
    const long long nblk = (ntile + 7) / 8 * 8;
    hipLaunchKernelGGL(k_cond_schur, dim3((unsigned)nblk), dim3(BS), GEMM_LDS, ctx->stream, cd, ntile, tm_n, tm_n,
                       top, bot, Kout, rout);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

// ---- additive Schwarz subdomain inverses (Section 4.6) -----------------------------------------
// T = [[P, I, 0], [I, 0, 0]] with P the element's enriched Schur complement: eliminating the
// first nt columns leaves -P^{-1} where the Schur complement would be.
//   P = Kbar^e, except that the diagonal block of each local face l is the assembled K_ff of
//   its face f = e2f[e][l] (= Kbar^{e1}_{l1 l1} + Kbar^{e2}_{l2 l2}; one term on a boundary).
__global__ __launch_bounds__(BS) void k_asm_fill(int nb, int L, const double* __restrict__ Kbar,
                                                 const double* __restrict__ K64, int S, const int32_t* __restrict__ e2f,
                                                 double* __restrict__ top, double* __restrict__ bot) {
    const long long e = blockIdx.x;
    const int nt = L * nb, C = 2 * nt + 1;
    const double* Ke = Kbar + (size_t)e * nt * nt;
    double* Te = top + (size_t)e * nt * C;
    double* Be = bot + (size_t)e * nt * C;
    for (int idx = threadIdx.x; idx < nt * C; idx += BS) {
        const int r = idx / C, c = idx - r * C;
        double v = 0.0, w = 0.0;
        if (c < nt) {
            const int lr = r / nb, lc = c / nb;
            if (lr == lc) {
                const long long f = e2f[e * L + lr];
                v = K64[((size_t)f * S) * nb * nb + (size_t)(c - lc * nb) * nb + (r - lr * nb)];
            } else {
                v = Ke[(size_t)r * nt + c];
            }
            w = (c == r) ? 1.0 : 0.0;
        } else if (c < 2 * nt) {
            v = (c - nt == r) ? 1.0 : 0.0;
        }
        Te[idx] = v;
        Be[idx] = w;
    }
}

// inv[e][l][l'][col][row] = P^{-1}(l nb + row, l' nb + col) = -Kout[e][l nb + row][l' nb + col]
// (the block row of unit (e, l), blocks column-major, as the face operator streams them).
__global__ __launch_bounds__(BS) void k_asm_store(int nb, int L, const double* __restrict__ Kout,
                                                  double* __restrict__ inv64, float* __restrict__ inv32) {
    const long long e = blockIdx.x;
    const int nt = L * nb;
    const size_t base = (size_t)e * nt * nt;
    for (int idx = threadIdx.x; idx < nt * nt; idx += BS) {
        // idx enumerates the output order: l, l', col, row
        int rem = idx;
        const int row = rem % nb; rem /= nb;
        const int col = rem % nb; rem /= nb;
        const int lp = rem % L; rem /= L;
        const int l = rem;
        const double v = -Kout[base + (size_t)(l * nb + row) * nt + (lp * nb + col)];
        if (inv64) inv64[base + idx] = v;
        if (inv32) inv32[base + idx] = (float)v;
    }
}

}  // namespace

hdg_status condense_run(hdg_ctx ctx, const hdg_dims* d, int64_t ne, const hdg_elem_blocks* in, double* Kbar,
                        double* rbar, double* local, double* Hbar_out, int32_t* ipiv) {
    CondDims cd;
    cd.M = d->ncomp; cd.D = d->dim; cd.P = d->npe; cd.PF = d->npf; cd.L = d->nlfe;
    cd.nu = cd.M * cd.P; cd.nq = cd.M * cd.D * cd.P; cd.nt = cd.L * cd.M * cd.PF;
    cd.R = cd.nu + cd.nt; cd.C = cd.R + 1; cd.NW = cd.P + cd.L * cd.PF; cd.KD = cd.D * cd.P;
    if (ne <= 0) return HDG_OK;
    const int NB = pick_panel(cd);
    if (NB == 0) {
        ctx->err = "condensation: element too large for the LDS-blocked elimination";
        return HDG_ERR_SHAPE;
    }
    // chunk elements so the workspace stays bounded (about 4 GiB)
    const size_t per_elem = sizeof(double) * ((size_t)cd.nt * cd.C + (size_t)cd.KD * cd.NW) + lu_ws_bytes_per_elem(cd);
    int64_t chunk = (int64_t)((size_t)4 << 30) / (int64_t)per_elem;
    if (chunk < 1) chunk = 1;
    if (chunk > ne) chunk = ne;
    hdg_status st;
    double* bot = (double*)ws_get(ctx, WS_T_BOTTOM, sizeof(double) * (size_t)chunk * cd.nt * cd.C, &st);
    if (!bot) return st;
    double* W = (double*)ws_get(ctx, WS_W, sizeof(double) * (size_t)chunk * cd.KD * cd.NW, &st);
    if (!W) return st;
    int* status = (int*)ws_get(ctx, WS_STATUS, 64, &st);
    if (!status) return st;
    const int big = 0x7fffffff;
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(status, &big, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    if ((st = set_kernel_lds(ctx, cd, NB)) != HDG_OK) return st;
    for (int64_t e0 = 0; e0 < ne; e0 += chunk) {
        const int64_t n = (ne - e0) < chunk ? (ne - e0) : chunk;
        const size_t P = cd.P, LPF = (size_t)cd.L * cd.PF;
        hipLaunchKernelGGL(k_cond_w, dim3((unsigned)n, cd.D), dim3(BS), 0, ctx->stream, cd, in->Minv + e0 * P * P,
                           in->Bd + e0 * cd.D * P * P, in->Cd + e0 * cd.D * P * LPF, W);
        HDG_LAUNCH_CHECK(ctx);
        {
            const int tm_n = div_up(cd.R, GT), tn_n = div_up(cd.NW, GT);
            const long long ntile = (long long)n * tm_n * tn_n;
            const long long nblk = (ntile + 7) / 8 * 8;
            // 16-byte staging loads where every row start and pair of [D;G] and W is 16-byte aligned
            // (even strides and 16-byte aligned base pointers)
            const bool v2 = cd.nq % 2 == 0 && cd.KD % 2 == 0 && cd.NW % 2 == 0 &&
                            (((uintptr_t)in->D | (uintptr_t)in->G | (uintptr_t)W) & 15) == 0;
            const void* qfn = v2 ? (const void*)k_cond_qelim<true> : (const void*)k_cond_qelim<false>;
            const double *Dp = in->D + e0 * cd.nu * cd.nq, *Ep = in->E + e0 * cd.nu * cd.nu,
                         *Fp = in->F + e0 * cd.nu * cd.nt, *Gp = in->G + e0 * cd.nt * cd.nq,
                         *Hp = in->H + e0 * cd.nt * cd.nu, *Jp = in->J + e0 * cd.nt * cd.nt, *rup = in->ru + e0 * cd.nu,
                         *rtp = in->rt + e0 * cd.nt;
            double* topp = local + e0 * cd.nu * cd.C;
            int tm_i = tm_n, tn_i = tn_n;
            long long ntile_l = ntile;
            void* qargs[] = {(void*)&cd, (void*)&ntile_l, (void*)&tm_i, (void*)&tn_i, (void*)&Dp, (void*)&Ep,
                             (void*)&Fp, (void*)&Gp, (void*)&Hp, (void*)&Jp, (void*)&rup, (void*)&rtp, (void*)&W,
                             (void*)&topp, (void*)&bot};
            HDG_HIP_CHECK(ctx, hipLaunchKernel(qfn, dim3((unsigned)nblk), dim3(BS), qargs, QLDS, ctx->stream));
            HDG_LAUNCH_CHECK(ctx);
        }
        const bool keep = Hbar_out != nullptr;
        if ((st = eliminate_and_schur(ctx, cd, NB, n, local + e0 * cd.nu * cd.C, bot, Kbar + e0 * cd.nt * cd.nt,
                                      rbar + e0 * cd.nt, status, e0, keep ? ipiv + e0 * cd.nu : nullptr)) != HDG_OK)
            return st;
        if (keep) {
            hipLaunchKernelGGL(k_copy_hbar, dim3((unsigned)n), dim3(BS), 0, ctx->stream, cd, bot,
                               Hbar_out + e0 * cd.nt * cd.nu);
            HDG_LAUNCH_CHECK(ctx);
        }
    }
    int bad = big;
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(&bad, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HDG_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    if (bad != big) {
        ctx->err = "condensation: zero or non-finite pivot in Ebar of element " + std::to_string(bad);
        return HDG_ERR_SINGULAR;
    }
    return HDG_OK;
}

hdg_status asm_setup_run(hdg_ctx ctx, const hdg_dims* d, const double* Kbar, const double* K64, const int32_t* e2f,
                         double* inv64, float* inv32) {
    const int nb = d->ncomp * d->npf, L = d->nlfe, S = 2 * L - 1;
    const int64_t ne = d->ne;
    CondDims cd{};
    cd.nu = L * nb;
    cd.nt = L * nb;
    cd.R = 2 * cd.nt;
    cd.C = cd.R + 1;
    if (ne <= 0) return HDG_OK;
    const int NB = pick_panel(cd);
    if (NB == 0) {
        ctx->err = "additive Schwarz: element trace block too large for the LDS-blocked elimination";
        return HDG_ERR_SHAPE;
    }
    const size_t per_elem = sizeof(double) * ((size_t)2 * cd.nt * cd.C + (size_t)cd.nt * cd.nt + cd.nt);
    int64_t chunk = (int64_t)((size_t)4 << 30) / (int64_t)(per_elem + lu_ws_bytes_per_elem(cd));
    if (chunk < 1) chunk = 1;
    if (chunk > ne) chunk = ne;
    hdg_status st;
    // workspace: top rows, trace rows, -P^{-1} and the (zero) right-hand-side output
    double* top = (double*)ws_get(ctx, WS_T_BOTTOM, per_elem * (size_t)chunk, &st);
    if (!top) return st;
    double* bot = top + (size_t)chunk * cd.nt * cd.C;
    double* Kout = bot + (size_t)chunk * cd.nt * cd.C;
    double* rout = Kout + (size_t)chunk * cd.nt * cd.nt;
    int* status = (int*)ws_get(ctx, WS_STATUS, 64, &st);
    if (!status) return st;
    const int big = 0x7fffffff;
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(status, &big, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    if ((st = set_kernel_lds(ctx, cd, NB)) != HDG_OK) return st;
    const size_t nt2 = (size_t)cd.nt * cd.nt;
    for (int64_t e0 = 0; e0 < ne; e0 += chunk) {
        const int64_t n = (ne - e0) < chunk ? (ne - e0) : chunk;
        hipLaunchKernelGGL(k_asm_fill, dim3((unsigned)n), dim3(BS), 0, ctx->stream, nb, L, Kbar + e0 * nt2, K64, S,
                           e2f + e0 * L, top, bot);
        HDG_LAUNCH_CHECK(ctx);
        if ((st = eliminate_and_schur(ctx, cd, NB, n, top, bot, Kout, rout, status, e0)) != HDG_OK) return st;
        hipLaunchKernelGGL(k_asm_store, dim3((unsigned)n), dim3(BS), 0, ctx->stream, nb, L, Kout,
                           inv64 ? inv64 + e0 * nt2 : nullptr, inv32 ? inv32 + e0 * nt2 : nullptr);
        HDG_LAUNCH_CHECK(ctx);
    }
    int bad = big;
    HDG_HIP_CHECK(ctx, hipMemcpyAsync(&bad, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HDG_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    if (bad != big) {
        ctx->err = "additive Schwarz: zero or non-finite pivot in the subdomain matrix of element " +
                   std::to_string(bad);
        return HDG_ERR_SINGULAR;
    }
    return HDG_OK;
}

hdg_status condense_rhs_run(hdg_ctx ctx, const hdg_dims* d, int64_t ne, double* local, const double* Hbar,
                            const int32_t* ipiv, const double* ru, const double* rt, double* rbar) {
    CondDims cd;
    cd.M = d->ncomp; cd.D = d->dim; cd.P = d->npe; cd.PF = d->npf; cd.L = d->nlfe;
    cd.nu = cd.M * cd.P; cd.nq = cd.M * cd.D * cd.P; cd.nt = cd.L * cd.M * cd.PF;
    cd.R = cd.nu + cd.nt; cd.C = cd.R + 1; cd.NW = cd.P + cd.L * cd.PF; cd.KD = cd.D * cd.P;
    if (ne <= 0) return HDG_OK;
    const int NB = pick_panel(cd);     // the panel width the elimination used
    if (NB == 0) {
        ctx->err = "condensation: element too large for the LDS-blocked elimination";
        return HDG_ERR_SHAPE;
    }
    hipLaunchKernelGGL(k_cond_rhs, dim3((unsigned)ne), dim3(BS), sizeof(double) * cd.nu, ctx->stream, cd, NB, local,
                       Hbar, ipiv, ru, rt, rbar);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}
