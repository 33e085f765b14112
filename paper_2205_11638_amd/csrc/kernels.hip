// kernels.hip -- CDNA4 (gfx950) kernels of the dual solver's hot path.
//
// Forward pass (Alg. 1, blocks B_1..B_u): for each hop l of a diagram, with F_l the
// shortest-path cost root -> node (App. B) and B_{l+1} the cost node -> 1-terminal from
// the previous backward pass (still valid: hops > l are not yet touched in this pass),
//     m^beta = min_{v in level l} F_l(v) + beta * lambda_l + B_{l+1}(child_beta(v))   (eq. 8)
//     M_new  = omega (m^1 - m^0),  lambda_new = lambda - M_new + alpha * S_i
// and F_{l+1}(w) = min over arcs (v, beta) -> w of F_l(v) + beta * lambda_new.
// The backward pass is the mirror image with B recomputed bottom-up from the terminals.
// One wavefront owns one tile of diagrams (see kernels.hpp for the layout); the current
// level's costs live in LDS, so hops need only wavefront-local synchronisation.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "kernels.hpp"

namespace dd {
namespace {

constexpr float kInf = __builtin_huge_valf();

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Order-preserving map float <-> int32 so that an integer LDS min is a float min.
__device__ __forceinline__ int f2k(float f) {
    int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ __forceinline__ float k2f(int k) { return __int_as_float(k >= 0 ? k : k ^ 0x7FFFFFFF); }

template <int P>
__device__ __forceinline__ float team_min(float v) {
#pragma unroll
    for (int o = P / 2; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}

struct TileCtx {
    int64_t nbase;
    int ebase, lbase, wbase, nlev;
};

__device__ __forceinline__ TileCtx tile_ctx(const DevTables &T, int64_t tile) {
    TileCtx c;
    c.nbase = T.node_base[tile];
    c.ebase = T.edge_base[tile];
    c.lbase = T.lev_base[tile];
    c.wbase = T.w_base[tile];
    c.nlev = T.nlev[tile];
    return c;
}

// ------------------------------------------------------------------------------------------
// Forward pass.  LDS per team: two int buffers of WL entries (F of level l, partial F of
// level l+1), interleaved over teams: index (buf * WL + k) * G + g.
// ------------------------------------------------------------------------------------------
template <int P, int RMAX, int MODE>
__global__ __launch_bounds__(256) void k_fwd(DevTables T, int64_t tile0, int64_t ntiles, int WL) {
    constexpr int G = 64 / P;
    extern __shared__ int lds_i[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane / P, p = lane % P;
    const int64_t tile = tile0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= tile0 + ntiles) return;  // uniform per wave
    int *my = lds_i + (size_t)wave * 2 * WL * G;
    const TileCtx tc = tile_ctx(T, tile);
    int cur = 0;
    if (p == 0) my[(0 * WL + 0) * G + g] = f2k(0.f);  // F(root) = 0
    float lam_prev = 0.f;
    wave_sync();
    for (int l = 0; l < tc.nlev; ++l) {
        const int W = T.widths[tc.wbase + l * G + g];
        const bool has_next = l + 1 < tc.nlev;
        const int Wn = has_next ? (int)T.widths[tc.wbase + (l + 1) * G + g] : 0;
        const int R = T.lev_rows[tc.lbase + l];
        const int64_t off = tc.nbase + T.lev_off[tc.lbase + l];
        const int64_t offn = has_next ? tc.nbase + T.lev_off[tc.lbase + l + 1] : 0;
        const int e = tc.ebase + l * G + g;
        float lam = 0.f, om = 0.f, al = 0.f, S = 0.f;
        if (W > 0) {
            lam = T.lam[e];
            al = T.alpha[e];
            S = T.S[T.evar[e]];
            if (MODE == FWD_UPDATE) om = T.omega[e];
        }
        int *nxt = my + (size_t)(cur ^ 1) * WL * G;
        const int *cb = my + (size_t)cur * WL * G;
        for (int k = p; k < Wn; k += P) nxt[k * G + g] = f2k(kInf);
        wave_sync();
        float m0 = kInf, m1 = kInf;
        uint32_t tp[RMAX];
        float fv[RMAX];
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            tp[r] = 0u;
            fv[r] = kInf;
            const int k = r * P + p;
            if (r < R && k < W) {
                const int64_t slot = off + (int64_t)r * 64 + lane;
                const float f = k2f(cb[k * G + g]);
                const uint32_t t = T.topo[slot];
                T.F[slot] = f;
                if (MODE == FWD_UPDATE) {
                    const int lo = (int)(t & 0xFFFFu), hi = (int)(t >> 16);
                    float b0 = lo == Wn ? kInf : 0.f, b1 = hi == Wn ? kInf : 0.f;
                    if (lo < Wn) b0 = T.B[offn + (int64_t)(lo / P) * 64 + g * P + (lo % P)];
                    if (hi < Wn) b1 = T.B[offn + (int64_t)(hi / P) * 64 + g * P + (hi % P)];
                    m0 = fminf(m0, f + b0);
                    m1 = fminf(m1, f + b1);
                }
                tp[r] = t;
                fv[r] = f;
            }
        }
        float lam_new;
        if (MODE == FWD_UPDATE) {
            m0 = team_min<P>(m0);
            m1 = team_min<P>(m1);
            lam_new = lam;
            if (W > 0) {
                m1 += lam;
                const float Mn = om * (m1 - m0);
                lam_new = lam - Mn + al * S;
                if (p == 0) {
                    T.lam[e] = lam_new;
                    T.M[e] = Mn;
                }
            }
        } else {
            lam_new = lam + al * S;  // flushed multipliers, no update
        }
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            const int k = r * P + p;
            if (r < R && k < W) {
                const int lo = (int)(tp[r] & 0xFFFFu), hi = (int)(tp[r] >> 16);
                if (lo < Wn) atomicMin(&nxt[lo * G + g], f2k(fv[r]));
                if (hi < Wn) atomicMin(&nxt[hi * G + g], f2k(fv[r] + lam_new));
            }
        }
        wave_sync();
        cur ^= 1;
        (void)lam_prev;
    }
}

// ------------------------------------------------------------------------------------------
// Backward pass and sweeps.  LDS per team: two float buffers (B of level l+1, B of level l).
// ------------------------------------------------------------------------------------------
template <int P, int RMAX, int MODE>
__global__ __launch_bounds__(256) void k_bwd(DevTables T, int64_t tile0, int64_t ntiles, int WL) {
    constexpr int G = 64 / P;
    extern __shared__ float lds_f[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane / P, p = lane % P;
    const int64_t tile = tile0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= tile0 + ntiles) return;
    float *my = lds_f + (size_t)wave * 2 * WL * G;
    const TileCtx tc = tile_ctx(T, tile);
    const int row = T.bdd[tile * 64 + g];
    int cur = 0;  // buffer holding B of level l+1
    for (int l = tc.nlev - 1; l >= 0; --l) {
        const int W = T.widths[tc.wbase + l * G + g];
        const int Wn = l + 1 < tc.nlev ? (int)T.widths[tc.wbase + (l + 1) * G + g] : 0;
        const int R = T.lev_rows[tc.lbase + l];
        const int64_t off = tc.nbase + T.lev_off[tc.lbase + l];
        const int e = tc.ebase + l * G + g;
        float lam = 0.f, om = 0.f, al = 0.f, S = 0.f;
        if (W > 0) {
            lam = T.lam[e];
            if (MODE == BWD_UPDATE || MODE == BWD_EN_BAR || MODE == BWD_MM) {
                al = T.alpha[e];
                S = T.S[T.evar[e]];
            }
            if (MODE == BWD_UPDATE) om = T.omega[e];
        }
        const float lam_use = (MODE == BWD_EN_BAR || MODE == BWD_MM) ? lam + al * S : lam;
        const float *bn = my + (size_t)cur * WL * G;
        float *bc = my + (size_t)(cur ^ 1) * WL * G;
        float m0 = kInf, m1 = kInf;
        float b0r[RMAX], b1r[RMAX];
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            b0r[r] = kInf;
            b1r[r] = kInf;
            const int k = r * P + p;
            if (r < R && k < W) {
                const int64_t slot = off + (int64_t)r * 64 + lane;
                const uint32_t t = T.topo[slot];
                const int lo = (int)(t & 0xFFFFu), hi = (int)(t >> 16);
                const float b0 = lo < Wn ? bn[lo * G + g] : (lo == Wn ? kInf : 0.f);
                const float b1 = hi < Wn ? bn[hi * G + g] : (hi == Wn ? kInf : 0.f);
                if (MODE == BWD_UPDATE || MODE == BWD_MM) {
                    const float f = T.F[slot];
                    m0 = fminf(m0, f + b0);
                    m1 = fminf(m1, f + b1);
                }
                b0r[r] = b0;
                b1r[r] = b1;
            }
        }
        float lam_new = lam_use;
        if (MODE == BWD_UPDATE || MODE == BWD_MM) {
            m0 = team_min<P>(m0);
            m1 = team_min<P>(m1);
            if (W > 0) {
                m1 += lam_use;
                if (MODE == BWD_UPDATE) {
                    const float Mn = om * (m1 - m0);
                    lam_new = lam - Mn + al * S;
                    if (p == 0) {
                        T.lam[e] = lam_new;
                        T.M[e] = Mn;
                    }
                } else if (p == 0) {
                    const int ce = T.slot2canon[e];
                    T.out0[ce] = m0;
                    T.out1[ce] = m1;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            const int k = r * P + p;
            if (r < R && k < W) {
                const float b = fminf(b0r[r], lam_new + b1r[r]);
                bc[k * G + g] = b;
                if (MODE == BWD_UPDATE || MODE == BWD_STORE) T.B[off + (int64_t)r * 64 + lane] = b;
            }
        }
        wave_sync();
        cur ^= 1;
    }
    if (MODE != BWD_MM && p == 0 && row >= 0) T.energies[row] = my[(size_t)cur * WL * G + g];
}

template <int P, int RMAX>
hipError_t fwd_dispatch(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s) {
    dim3 grid((unsigned)((c.ntiles + c.wpb - 1) / c.wpb)), block(64 * c.wpb);
    size_t lds = (size_t)c.wpb * 2 * c.WL * (64 / P) * sizeof(int);
    if (mode == FWD_UPDATE) hipLaunchKernelGGL((k_fwd<P, RMAX, FWD_UPDATE>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WL);
    else hipLaunchKernelGGL((k_fwd<P, RMAX, FWD_SWEEP_BAR>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WL);
    return hipGetLastError();
}

template <int P, int RMAX>
hipError_t bwd_dispatch(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s) {
    dim3 grid((unsigned)((c.ntiles + c.wpb - 1) / c.wpb)), block(64 * c.wpb);
    size_t lds = (size_t)c.wpb * 2 * c.WL * (64 / P) * sizeof(float);
    switch (mode) {
        case BWD_UPDATE: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_UPDATE>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WL); break;
        case BWD_STORE: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_STORE>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WL); break;
        case BWD_EN_LAM: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_EN_LAM>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WL); break;
        case BWD_EN_BAR: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_EN_BAR>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WL); break;
        default: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_MM>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WL); break;
    }
    return hipGetLastError();
}

#define DD_CLASSES(X) X(1, 4) X(2, 4) X(4, 4) X(8, 4) X(16, 4) X(32, 4) X(64, 4) X(64, 8) X(64, 16) X(64, 32)

__global__ void k_deferred_sum(const int32_t *__restrict__ var_ptr, const int32_t *__restrict__ var_slots,
                               const float *__restrict__ M, float *__restrict__ S, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int q = var_ptr[i]; q < var_ptr[i + 1]; ++q) s += M[var_slots[q]];
    S[i] = s;
}

__global__ void k_init_lambda(const int32_t *__restrict__ canon2slot, const int32_t *__restrict__ evar,
                              const int32_t *__restrict__ var_ptr, const float *__restrict__ c, float *lam, float *M,
                              int64_t E) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int s = canon2slot[e];
    const int v = evar[s];
    lam[s] = c[v] / (float)(var_ptr[v + 1] - var_ptr[v]);
    M[s] = 0.f;
}

__global__ void k_scatter(const int32_t *__restrict__ canon2slot, const float *__restrict__ src, float *dst,
                          int64_t E) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < E) dst[canon2slot[e]] = src[e];
}

__global__ void k_gather(const int32_t *__restrict__ canon2slot, const float *__restrict__ src, float *dst, int64_t E,
                         const float *__restrict__ alpha, const float *__restrict__ S, const int32_t *__restrict__ evar,
                         int flush) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int s = canon2slot[e];
    float v = src[s];
    if (flush) v = v + alpha[s] * S[evar[s]];
    dst[e] = v;
}

__global__ void k_seg_softmax(const int32_t *__restrict__ var_ptr, const int32_t *__restrict__ var_canon,
                              const float *__restrict__ x, float *y, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int a = var_ptr[i], b = var_ptr[i + 1];
    float mx = -kInf;
    for (int q = a; q < b; ++q) mx = fmaxf(mx, x[var_canon[q]]);
    float den = 0.f;
    for (int q = a; q < b; ++q) den += expf(x[var_canon[q]] - mx);
    for (int q = a; q < b; ++q) y[var_canon[q]] = expf(x[var_canon[q]] - mx) / den;
}

// One workgroup of 1024 threads: per-thread fp64 partial sums in a fixed stride order,
// then a fixed-shape tree in LDS, so the result does not depend on scheduling.
__global__ __launch_bounds__(1024) void k_bound_reduce(const float *__restrict__ En, int64_t m,
                                                       const float *__restrict__ M, int64_t slots, double *out) {
    __shared__ double sa[1024], sb[1024];
    const int t = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t j = t; j < m; j += 1024) a += (double)En[j];
    for (int64_t j = t; j < slots; j += 1024) b += (double)fminf(M[j], 0.f);
    sa[t] = a;
    sb[t] = b;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) {
            sa[t] += sa[t + w];
            sb[t] += sb[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = sa[0];
        out[1] = sb[0];
    }
}

__global__ void k_check_params(const float *__restrict__ om, const float *__restrict__ al, int64_t E, int32_t *flags) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const float w = om[e], a = al[e];
    if (!(w >= 0.f && w <= 1.f)) atomicOr(&flags[0], 1);
    if (!(a >= 0.f && a <= 3.0e38f)) atomicOr(&flags[1], 1);
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

bool class_supported(int P, int RMAX) {
#define DD_SUP(PP, RR) if (P == PP && RMAX == RR) return true;
    DD_CLASSES(DD_SUP)
#undef DD_SUP
    return false;
}

hipError_t launch_fwd(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s) {
    if (c.ntiles <= 0) return hipSuccess;
#define DD_FWD(PP, RR) if (c.P == PP && c.RMAX == RR) return fwd_dispatch<PP, RR>(t, c, mode, s);
    DD_CLASSES(DD_FWD)
#undef DD_FWD
    return hipErrorInvalidValue;
}

hipError_t launch_bwd(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s) {
    if (c.ntiles <= 0) return hipSuccess;
#define DD_BWD(PP, RR) if (c.P == PP && c.RMAX == RR) return bwd_dispatch<PP, RR>(t, c, mode, s);
    DD_CLASSES(DD_BWD)
#undef DD_BWD
    return hipErrorInvalidValue;
}

hipError_t launch_deferred_sum(const int32_t *var_ptr, const int32_t *var_slots, const float *M, float *S, int n,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_deferred_sum, dim3(blocks_for(n, 256)), dim3(256), 0, s, var_ptr, var_slots, M, S, n);
    return hipGetLastError();
}

hipError_t launch_init_lambda(const int32_t *canon2slot, const int32_t *evar, const int32_t *var_ptr, const float *c,
                              float *lam, float *M, int64_t E, hipStream_t s) {
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_lambda, dim3(blocks_for(E, 256)), dim3(256), 0, s, canon2slot, evar, var_ptr, c, lam, M, E);
    return hipGetLastError();
}

hipError_t launch_scatter(const int32_t *canon2slot, const float *src, float *dst, int64_t E, hipStream_t s) {
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(E, 256)), dim3(256), 0, s, canon2slot, src, dst, E);
    return hipGetLastError();
}

hipError_t launch_gather(const int32_t *canon2slot, const float *src, float *dst, int64_t E, const float *alpha,
                         const float *S, const int32_t *evar, int flush, hipStream_t s) {
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(E, 256)), dim3(256), 0, s, canon2slot, src, dst, E, alpha, S, evar,
                       flush);
    return hipGetLastError();
}

hipError_t launch_seg_softmax(const int32_t *var_ptr, const int32_t *var_canon, const float *x, float *y, int n,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_softmax, dim3(blocks_for(n, 256)), dim3(256), 0, s, var_ptr, var_canon, x, y, n);
    return hipGetLastError();
}

hipError_t launch_bound_reduce(const float *energies, int64_t m, const float *M, int64_t slots, double *out,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_bound_reduce, dim3(1), dim3(1024), 0, s, energies, m, M, slots, out);
    return hipGetLastError();
}

hipError_t launch_check_params(const float *omega, const float *alpha, int64_t E, int32_t *flags, hipStream_t s) {
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_params, dim3(blocks_for(E, 256)), dim3(256), 0, s, omega, alpha, E, flags);
    return hipGetLastError();
}

}  // namespace dd
