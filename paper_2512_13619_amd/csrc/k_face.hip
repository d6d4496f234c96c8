// Face-block operator: strided block matvec y_f = K_f x_f over the extended
// neighbour vector (Section 4.3), block-Jacobi z_f = P_f^{-1} y_f (Section 4.5),
// and the fused operator step of the polynomial preconditioner (Section 4.7:
// the recurrence's axpy/scale work folded into the product's epilogue).
//
// Mapping (gfx950, wave64): a "team" of TEAM threads owns one face. The face's
// blocks are stored column-major, K[f][s][col][row], so the face row of blocks
// is an nb x (S nb) column-major matrix streamed contiguously from HBM. Each
// thread owns VEC consecutive rows (one 16-byte load of 4 floats or 2 doubles when
// nb allows it) and a column group; with G column groups the team reads G whole
// columns, i.e. one contiguous run of G*nb entries, per step. The extended x (S nb
// values gathered through nbr) sits in LDS; the G partial sums of each row are
// combined in a fixed order, so results are bitwise reproducible. Empty slots
// (boundary faces) are trailing and are never read.
#include <hip/hip_ext.h>

#include <cstdio>
#include <string>

#include "hdg_internal.hpp"

namespace {

// VEC consecutive entries of T as one load
template <typename T, int VEC>
struct VecOf {
    typedef T type __attribute__((ext_vector_type(VEC)));
};
template <typename T>
struct VecOf<T, 1> {
    typedef T type;
};
template <typename V>
__device__ __forceinline__ double lane_of(const V& v, int i) { return (double)v[i]; }
__device__ __forceinline__ double lane_of(float v, int) { return (double)v; }
__device__ __forceinline__ double lane_of(double v, int) { return v; }

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
template <typename T1, typename T2, int TEAM, bool HAS_M2, int KIND, int VEC>
__global__ __launch_bounds__(256) void k_face_op(FaceArgs A) {
    constexpr int FPB = 256 / TEAM;        // faces per block
    typedef typename VecOf<T1, VEC>::type V1;
    extern __shared__ double smem[];
    if (A.skip && *A.skip) return;
    const int nb = A.nb, S = A.S1;
    const int team = threadIdx.x / TEAM;
    const int t = threadIdx.x - team * TEAM;
    const long long f = (long long)blockIdx.x * FPB + team;
    const bool valid = f < A.nf;
    const int L = S * nb;
    double* xs = smem + team * L;
    double* red = smem + FPB * L;                   // 256*VEC: one partial sum per (thread, row)
    double* redt = red + (size_t)team * TEAM * VEC; // this team's part, indexed group*nb + row
    double* uf = red + 256 * VEC + team * nb;       // nb per team (second stage input)

    // number of leading non-empty slots (empty slots only ever trail)
    int Seff = S;
    if (valid && A.nbr1 != nullptr && S > A.nlfe && A.nbr1[f * S + A.nlfe] < 0) Seff = A.nlfe;
    const int ncols = Seff * nb;

    const int nbv = nb / VEC;          // threads per column
    const int G = TEAM / nbv;          // column groups
    const int grp = t / nbv;
    const int r0 = (t - grp * nbv) * VEC;
    const bool active = valid && grp < G;
    const V1* p = nullptr;
    const size_t step = (size_t)G * nbv;        // in units of V1
    // U independent streaming loads in flight per thread (more for 4-byte loads)
    constexpr int U = (VEC == 1 && sizeof(T1) == 4) ? 8 : 4;
    // small blocks (one row per thread): the first U loads of the block stream and the
    // epilogue operands do not depend on x, so they are issued before the gather and their
    // latency overlaps the nbr -> x chain (a thread has only a few loads in all)
    constexpr bool PRE = VEC == 1;
    const bool pre = PRE && active && grp + (U - 1) * G < ncols;
    V1 m0[U];
    if (active) {
        const T1* Mf = static_cast<const T1*>(A.M1) + (size_t)f * S * nb * nb;
        p = reinterpret_cast<const V1*>(Mf + (size_t)grp * nb + r0);
    }
    if (pre) {
#pragma unroll
        for (int u = 0; u < U; ++u) m0[u] = __builtin_nontemporal_load(p + u * step);
    }
    // second product (HAS_M2): thread (row row2, column group grp2 of G2) needs the entries
    // Bf[k][row2], k = grp2 + j G2; the first K2 of them do not depend on x and are loaded
    // here, so their latency overlaps the first product instead of following it
    constexpr int K2 = 16;
    const int G2 = HAS_M2 ? TEAM / nb : 1;
    const int grp2 = HAS_M2 ? t / nb : 0;
    const int row2 = t - grp2 * nb;
    const bool act2 = HAS_M2 && valid && grp2 < G2;
    T2 b2[HAS_M2 ? K2 : 1];
    if (HAS_M2 && act2) {
        const T2* Bf = static_cast<const T2*>(A.M2) + (size_t)f * nb * nb;
#pragma unroll
        for (int j = 0; j < K2; ++j) {
            const int k = grp2 + j * G2;
            const T2 b = Bf[(size_t)(k < nb ? k : grp2) * nb + row2];
            b2[j] = k < nb ? b : T2(0);
        }
    }
    double ex[3], ey[3];
#pragma unroll
    for (int o = 0; o < 3; ++o) ex[o] = ey[o] = 0.0;
    if (PRE && valid && t < nb) {
        const size_t idx = (size_t)f * nb + t;
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            if (A.epi.X[o]) ex[o] = A.epi.X[o][idx];
            if (A.epi.Y[o]) ey[o] = A.epi.Y[o][idx];
        }
    }
    if (valid) {
        for (int i = t; i < ncols; i += TEAM) {
            const int s = i / nb;
            const int c = i - s * nb;
            const long long g = A.nbr1 ? (long long)A.nbr1[f * S + s] : f;
            xs[i] = A.x[g * nb + c];
        }
    }
    __syncthreads();

    double acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = 0.0;
    if (active) {
        int k = grp;
        if (pre) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double xv = xs[k + u * G];
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc[v] += lane_of(m0[u], v) * xv;
            }
            p += U * step;
            k += U * G;
        }
        for (; k + (U - 1) * G < ncols; k += U * G) {
            V1 m[U];
#pragma unroll
            for (int u = 0; u < U; ++u) m[u] = __builtin_nontemporal_load(p + u * step);
            // keep the U loads in flight together: without this the scheduler interleaves
            // each load with its wait and conversion, serialising the stream
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double xv = xs[k + u * G];
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc[v] += lane_of(m[u], v) * xv;
            }
            p += U * step;
        }
        for (; k < ncols; k += G) {
            const V1 m = __builtin_nontemporal_load(p);
            const double xv = xs[k];
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] += lane_of(m, v) * xv;
            p += step;
        }
        // index grp*nb + row, row = r0 + v
#pragma unroll
        for (int v = 0; v < VEC; ++v) redt[(size_t)t * VEC + v] = acc[v];
    }
    __syncthreads();
    double u = 0.0;
    if (valid && t < nb) {
        for (int g2 = 0; g2 < G; ++g2) u += redt[g2 * nb + t];
    }
    if (HAS_M2) {
        // second product (one thread per row and column group; entries from b2, the rest, if
        // any, loaded here), k ascending as in a plain loop
        if (valid && t < nb) uf[t] = u;
        __syncthreads();
        double acc2 = 0.0;
        if (act2) {
#pragma unroll
            for (int j = 0; j < K2; ++j) {
                const int k = grp2 + j * G2;
                if (k < nb) acc2 += (double)b2[j] * uf[k];
            }
            const T2* Bf = static_cast<const T2*>(A.M2) + (size_t)f * nb * nb;
            for (int k = grp2 + K2 * G2; k < nb; k += G2) acc2 += (double)Bf[(size_t)k * nb + row2] * uf[k];
        }
        redt[t] = acc2;
        __syncthreads();
        u = 0.0;
        if (valid && t < nb) {
            for (int g2 = 0; g2 < G2; ++g2) u += redt[g2 * nb + t];
        }
    }
    if (valid && t < nb) {
        const size_t idx = (size_t)f * nb + t;
        double v[3];
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            v[o] = A.epi.s[o] * u;
            if (A.epi.X[o]) v[o] += A.epi.a[o] * (PRE ? ex[o] : A.epi.X[o][idx]);
            if (A.epi.Y[o]) v[o] += A.epi.b[o] * (PRE ? ey[o] : A.epi.Y[o][idx]);
        }
#pragma unroll
        for (int o = 0; o < 3; ++o)
            if (A.epi.out[o]) A.epi.out[o][idx] = v[o];
    }
}

// M1 = identity: u = x, the epilogue only (one thread per entry).
__global__ __launch_bounds__(256) void k_face_identity(FaceArgs A, size_t n) {
    if (A.skip && *A.skip) return;
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n) return;
    const double u = A.x[idx];
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

// Additive Schwarz prolongation (Section 4.6): face f sums the results of its one or two
// elements' units (e1, l1) and (e2, l2), zu[(e*L + l)*nb + t], then applies the epilogue.
// Face-parallel, no atomics: bitwise reproducible.
__global__ __launch_bounds__(256) void k_asm_gather(int nf, int nb, int L, const int32_t* __restrict__ f2e,
                                                    const double* __restrict__ zu, FaceArgs A) {
    if (A.skip && *A.skip) return;
    const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (size_t)nf * nb) return;
    const size_t f = idx / nb;
    const int t = (int)(idx - f * nb);
    const int e1 = f2e[4 * f], l1 = f2e[4 * f + 1], e2 = f2e[4 * f + 2], l2 = f2e[4 * f + 3];
    double u = zu[((size_t)e1 * L + l1) * nb + t];
    if (e2 >= 0) u += zu[((size_t)e2 * L + l2) * nb + t];
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

// Neighbour table of the element units: unit (e, l) takes block l' from face e2f[e][l'].
__global__ __launch_bounds__(256) void k_asm_unit_nbr(long long ne, int L, const int32_t* __restrict__ e2f,
                                                      int32_t* __restrict__ unbr) {
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= ne * L * L) return;
    const long long e = idx / ((long long)L * L);
    const int lp = (int)(idx % L);
    unbr[idx] = e2f[e * L + lp];
}

// A configuration (threads per face, rows per thread) the kernel supports for these operands:
// the instantiated pairs, every row of the face owned by a thread, and vector loads that
// divide nb and are aligned to the matrix.
bool face_config_ok(const FaceArgs& a, size_t t1_bytes, int team, int vec) {
    const bool inst = (vec == 1 && (team == 16 || team == 32 || team == 64 || team == 128 || team == 256)) ||
                      ((vec == 2 || vec == 4) && (team == 128 || team == 256));
    if (!inst || team < a.nb || a.nb % vec != 0 || vec * t1_bytes > 16) return false;
    return reinterpret_cast<uintptr_t>(a.M1) % (vec * t1_bytes) == 0;
}

// Key of a launch configuration in the measured table: operand types, product kind, block
// size, slots per face and the power-of-two bucket of the face count.
std::string face_key(const FaceArgs& a, size_t t1_bytes, size_t t2_bytes, bool has_m2, int kind) {
    int lg = 0;
    while (lg < 40 && ((long long)1 << (lg + 1)) <= (long long)a.nf) ++lg;
    char buf[128];
    std::snprintf(buf, sizeof(buf), "face:m%zu:p%zu:m2%d:k%d:nb%d:S%d:nf2^%d", t1_bytes * 8, t2_bytes * 8,
                  has_m2 ? 1 : 0, kind, a.nb, a.S1, lg);
    return buf;
}

// Set by the tuner while it times one configuration (this thread only).
thread_local int g_force_team = 0, g_force_vec = 0;

template <typename T1, typename T2, bool HAS_M2, int KIND>
hdg_status launch_team(hdg_ctx ctx, const FaceArgs& a) {
    // 16-byte loads (4 floats or 2 doubles per thread) when nb and the matrix pointer
    // allow them, else 8-byte float pairs, else one entry per load
    int vec = 1;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(a.M1);
    for (int cand = (int)(16 / sizeof(T1)); cand > 1; cand /= 2)
        if (a.nb % cand == 0 && addr % (cand * sizeof(T1)) == 0) { vec = cand; break; }
    // columns in flight per team: a block row (S1 > 1) has S1*nb columns, a block-diagonal
    // product (S1 == 1) only nb, so it takes fewer groups and longer runs per thread
    const int groups = (a.S1 > 1 ? 4 : 2) * (vec > 1 ? 4 : 1);
    const int want = groups * (a.nb / vec);
    int team;
    if (a.nb > 64 || want > 128) team = 256;
    else if (want > 64) team = 128;
    else if (want > 32) team = 64;
    else if (want > 16) team = 32;
    else team = 16;
    if (team < 128) vec = 1;           // vector loads only for the wide teams
    if (team < a.nb / vec) team = 256;
    // a measured choice (hdg_autotune) replaces the rule above; the tuner forces its candidates
    if (g_force_team) {
        team = g_force_team;
        vec = g_force_vec;
    } else if (tune_have_entries()) {
        int tt = 0, tv = 0;
        if (tune_get(face_key(a, sizeof(T1), sizeof(T2), HAS_M2, KIND), &tt, &tv) &&
            face_config_ok(a, sizeof(T1), tt, tv)) {
            team = tt;
            vec = tv;
        }
    }
    const int fpb = 256 / team;
    const size_t lds = sizeof(double) * ((size_t)fpb * a.S1 * a.nb + 256 * (size_t)vec + (size_t)fpb * a.nb);
    const int grid = div_up(a.nf, fpb);
    if (grid == 0) return HDG_OK;
    hipEvent_t ev_start, ev_stop;
    take_ext_events(ctx, &ev_start, &ev_stop);
#define HDG_FACE_LAUNCH(TM, VC)                                                                                 \
    do {                                                                                                        \
        if (ev_start || ev_stop)                                                                                \
            hipExtLaunchKernelGGL((k_face_op<T1, T2, TM, HAS_M2, KIND, VC>), dim3(grid), dim3(256), lds,        \
                                  ctx->stream, ev_start, ev_stop, 0, a);                                        \
        else                                                                                                    \
            hipLaunchKernelGGL((k_face_op<T1, T2, TM, HAS_M2, KIND, VC>), dim3(grid), dim3(256), lds,           \
                               ctx->stream, a);                                                                 \
    } while (0)
    if (vec == 4) {
        if (team == 256) HDG_FACE_LAUNCH(256, 4); else HDG_FACE_LAUNCH(128, 4);
    } else if (vec == 2) {
        if (team == 256) HDG_FACE_LAUNCH(256, 2); else HDG_FACE_LAUNCH(128, 2);
    } else {
        switch (team) {
            case 256: HDG_FACE_LAUNCH(256, 1); break;
            case 128: HDG_FACE_LAUNCH(128, 1); break;
            case 64:  HDG_FACE_LAUNCH(64, 1); break;
            case 32:  HDG_FACE_LAUNCH(32, 1); break;
            default:  HDG_FACE_LAUNCH(16, 1); break;
        }
    }
#undef HDG_FACE_LAUNCH
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
    if (M1 == nullptr) {
        // identity operator (a preconditioner folded into the operator blocks)
        if (M2 != nullptr || nbr1 != nullptr) {
            ctx->err = "face operator: identity M1 takes neither a second matrix nor neighbours";
            return HDG_ERR_ARG;
        }
        const size_t n = (size_t)nf * nb;
        if (n == 0) return HDG_OK;
        hipLaunchKernelGGL(k_face_identity, dim3((unsigned)div_up((long long)n, 256)), dim3(256), 0, ctx->stream, a, n);
        HDG_LAUNCH_CHECK(ctx);
        return HDG_OK;
    }
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

// Times every supported configuration of one face-operator variant (the product's operands
// as in face_op, output to y) with `reps` launches each and records the fastest in the table.
// Returns the chosen configuration's time per launch in *best_us.
hdg_status face_autotune(hdg_ctx ctx, int nf, int nb, int S1, int nlfe, const void* M1, bool m1_fp32,
                         const int32_t* nbr1, const void* M2, bool m2_fp32, const double* x, double* y, int reps,
                         double* best_us) {
    FaceArgs a;
    a.M1 = M1;
    a.nbr1 = nbr1;
    a.M2 = M2;
    a.x = x;
    a.skip = nullptr;
    a.nf = nf;
    a.nb = nb;
    a.S1 = S1;
    a.nlfe = nlfe;
    for (int o = 0; o < 3; ++o) {
        a.epi.out[o] = nullptr;
        a.epi.X[o] = nullptr;
        a.epi.Y[o] = nullptr;
        a.epi.s[o] = a.epi.a[o] = a.epi.b[o] = 0.0;
    }
    a.epi.out[0] = y;
    a.epi.s[0] = 1.0;
    const size_t b1 = m1_fp32 ? 4 : 8, b2 = M2 ? (m2_fp32 ? 4 : 8) : b1;
    const int kind = (nbr1 == nullptr && M2 == nullptr) ? 1 : 0;
    static const int cands[9][2] = {{256, 4}, {128, 4}, {256, 2}, {128, 2}, {256, 1}, {128, 1}, {64, 1}, {32, 1},
                                    {16, 1}};
    hipEvent_t e0, e1;
    HDG_HIP_CHECK(ctx, hipEventCreate(&e0));
    HDG_HIP_CHECK(ctx, hipEventCreate(&e1));
    double best = -1.0;
    int bt = 0, bv = 0;
    hdg_status st = HDG_OK;
    for (const auto& c : cands) {
        if (!face_config_ok(a, b1, c[0], c[1])) continue;
        g_force_team = c[0];
        g_force_vec = c[1];
        st = face_op(ctx, nf, nb, S1, nlfe, M1, m1_fp32, nbr1, M2, m2_fp32, x, a.epi, nullptr);   // warm-up
        if (st == HDG_OK && hipEventRecord(e0, ctx->stream) != hipSuccess) st = HDG_ERR_HIP;
        for (int r = 0; r < reps && st == HDG_OK; ++r)
            st = face_op(ctx, nf, nb, S1, nlfe, M1, m1_fp32, nbr1, M2, m2_fp32, x, a.epi, nullptr);
        if (st == HDG_OK && (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
            st = HDG_ERR_HIP;
        g_force_team = g_force_vec = 0;
        if (st != HDG_OK) break;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = HDG_ERR_HIP;
            break;
        }
        const double us = 1e3 * ms / reps;
        if (best < 0.0 || us < best) {
            best = us;
            bt = c[0];
            bv = c[1];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != HDG_OK) {
        if (ctx->err.empty()) ctx->err = "autotune: a timed launch failed";
        return st;
    }
    if (best >= 0.0) tune_put(face_key(a, b1, b2, M2 != nullptr, kind), bt, bv, best);
    *best_us = best;
    return HDG_OK;
}

hdg_status asm_unit_nbr(hdg_ctx ctx, int64_t ne, int L, const int32_t* e2f, int32_t* unbr) {
    const long long n = (long long)ne * L * L;
    if (n == 0) return HDG_OK;
    hipLaunchKernelGGL(k_asm_unit_nbr, dim3((unsigned)div_up(n, 256)), dim3(256), 0, ctx->stream, (long long)ne, L, e2f,
                       unbr);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}

hdg_status asm_apply_op(hdg_ctx ctx, int nf, int nb, int L, int64_t ne, const void* inv, bool inv32,
                        const int32_t* unbr, const int32_t* f2e, double* zu, const double* y, const FaceEpilogue& epi,
                        const int* skip) {
    // restriction + element solves: unit (e, l) = block row l of (P^e)^{-1} against y on e's faces
    FaceEpilogue e0;
    for (int o = 0; o < 3; ++o) {
        e0.out[o] = nullptr;
        e0.X[o] = nullptr;
        e0.Y[o] = nullptr;
        e0.s[o] = e0.a[o] = e0.b[o] = 0.0;
    }
    e0.out[0] = zu;
    e0.s[0] = 1.0;
    hdg_status st = face_op(ctx, (int)(ne * L), nb, L, L, inv, inv32, unbr, nullptr, false, y, e0, skip);
    if (st != HDG_OK) return st;
    // prolongation: sum over the face's elements
    FaceArgs a;
    a.M1 = nullptr;
    a.nbr1 = nullptr;
    a.M2 = nullptr;
    a.x = nullptr;
    a.epi = epi;
    a.skip = skip;
    a.nf = nf;
    a.nb = nb;
    a.S1 = 1;
    a.nlfe = L;
    const size_t n = (size_t)nf * nb;
    if (n == 0) return HDG_OK;
    hipLaunchKernelGGL(k_asm_gather, dim3((unsigned)div_up((long long)n, 256)), dim3(256), 0, ctx->stream, nf, nb, L,
                       f2e, zu, a);
    HDG_LAUNCH_CHECK(ctx);
    return HDG_OK;
}
