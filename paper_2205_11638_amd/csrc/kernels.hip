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

#include <algorithm>
#include <cfloat>

#include "device_common.hpp"
#include "kernels.hpp"

namespace dd {
namespace {

using namespace dev;

// LOOP = false: one wave per tile.  LOOP = true (update passes on a resident grid): each wave
// takes tiles w, w + stride, ... (stride = waves in the grid); tiles are sorted by decreasing
// length within a class, so striding mixes long and short ones.
template <int P, int RMAX, int MODE, bool LOOP>
__global__ __launch_bounds__(256) void k_fwd(DevTables T, int64_t tile0, int64_t ntiles, int WB, int NL) {
    constexpr int G = 64 / P;
    constexpr bool UPD = MODE == FWD_UPDATE;
    extern __shared__ float lds_f[];
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int g = lane / P, p = lane % P;
    int64_t tile = tile0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= tile0 + ntiles) return;  // uniform per wave
    for (;;) {
        float *Fb = lds_f + (size_t)wave * lds_words_pass(P, WB, NL);
        float *Bst = Fb + WB * G;
        int *meta = (int *)(Bst + WB * G);
        int *off = meta + NL * G;
        const TileCtx tc = tile_ctx(T, tile);
        preload_meta<G>(T, tc, lane, meta, off);
        const int nlev = tc.nlev;
        auto level = [&](int l) {
            Lev v{0, 0, 0};
            if (l < nlev) {
                const int w = meta[l * G + g] & 0xFFFF;
                v.W = G == 1 ? uni(w) : w;
                v.R = uni(meta[l * G] >> 16);
                v.base = tc.nbase + (int64_t)uni(off[l]);
            }
            return v;
        };
        const int mine = p * G + g;  // this lane's buffer index for k = p; row r adds r * P * G

        Lev c0 = level(0), c1 = level(1), c2 = level(2);
        uint32_t tpn[RMAX];
        float bvn[RMAX];
    #pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            tpn[r] = r < c0.R ? T.topo[c0.base + r * 64 + lane] : 0u;
            bvn[r] = (UPD && r < c1.R) ? T.B[c1.base + r * 64 + lane] : 0.f;
        }
        float lamn = T.lam[tc.ebase + g], aSn = T.aS[tc.ebase + g], omn = UPD ? T.omega[tc.ebase + g] : 0.f;
        if (p == 0) Fb[g] = 0.f;  // F(root) = 0
        wave_sync();
        for (int l = 0; l < nlev; ++l) {
            const float lam = lamn, om = omn, aS = aSn;
            uint32_t tp[RMAX];
            float fv[RMAX];
            // B of level l+1 (prefetched last hop) into LDS, with the terminals after it
    #pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                tp[r] = tpn[r];
                if (UPD && r < c1.R) Bst[mine + r * P * G] = bvn[r];
            }
            if (UPD && p == 0) {
                Bst[c1.W * G + g] = kInf;       // 0-terminal
                Bst[(c1.W + 1) * G + g] = 0.f;  // 1-terminal
            }
            // F of this level: read, store for the backward pass, clear the slots of level l+1
            float *fg = T.F + c0.base;
    #pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                const int k = r * P + p, x = mine + r * P * G;
                if (r < c0.R) {
                    fv[r] = k < c0.W ? Fb[x] : kInf;
                    if (in_level<P>(r, c0.R, lane, c0.W)) fg[r * 64 + lane] = fv[r];
                }
                if (r < c1.R) Fb[x] = kInf;
            }
            wave_sync();
            // prefetch (issued after this hop's stores): topology of l+1, B of l+2, edge data of l+1
    #pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                tpn[r] = r < c1.R ? T.topo[c1.base + r * 64 + lane] : 0u;
                bvn[r] = (UPD && r < c2.R) ? T.B[c2.base + r * 64 + lane] : 0.f;
            }
            if (l + 1 < nlev) {
                const int e = tc.ebase + (l + 1) * G + g;
                lamn = T.lam[e];
                aSn = T.aS[e];
                if (UPD) omn = T.omega[e];
            }
            float m0 = kInf, m1 = kInf;
            const uint32_t dead = (uint32_t)c1.W | ((uint32_t)c1.W << 16);
    #pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                if (r < c0.R) {
                    if (!in_level<P>(r, c0.R, lane, c0.W)) tp[r] = dead;
                    if (UPD) {
                        const float b0 = Bst[(int)(tp[r] & 0xFFFFu) * G + g];
                        const float b1 = Bst[(int)(tp[r] >> 16) * G + g];
                        m0 = fminf(m0, fv[r] + b0);
                        m1 = fminf(m1, fv[r] + b1);
                    }
                }
            }
            float lam_new;
            if (UPD) {
                m0 = team_min<P>(m0);
                m1 = team_min<P>(m1);
                lam_new = lam;
                if (c0.W > 0) {
                    m1 += lam;
                    const float Mn = om * (m1 - m0);
                    lam_new = lam - Mn + aS;
                    if (p == 0) {
                        const int e = tc.ebase + l * G + g;
                        T.lam[e] = lam_new;
                        T.M[e] = Mn;
                    }
                }
            } else {
                lam_new = MODE == FWD_SWEEP_BAR ? lam + aS : lam;  // sweep, no update
            }
    #pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                if (r < c0.R) {
                    const int lo = (int)(tp[r] & 0xFFFFu), hi = (int)(tp[r] >> 16);
                    if (lo < c1.W) lds_fmin(&Fb[lo * G + g], fv[r]);
                    if (hi < c1.W) lds_fmin(&Fb[hi * G + g], fv[r] + lam_new);
                }
            }
            wave_sync();
            c0 = c1;
            c1 = c2;
            c2 = level(l + 3);
        }
        if (!LOOP) break;
        tile += (int64_t)gridDim.x * (blockDim.x >> 6);
        if (tile >= tile0 + ntiles) break;
        wave_sync();
    }  // tiles
}

// ------------------------------------------------------------------------------------------
// Backward pass and sweeps.  The two node buffers alternate as B of level l+1 (read) and B of
// level l (written); B of a level goes to global memory at the start of the next hop, before
// that hop's prefetch, so waiting for prefetched data never waits for a fresh store.
// ------------------------------------------------------------------------------------------
template <int P, int RMAX, int MODE, bool LOOP>
__global__ __launch_bounds__(256) void k_bwd(DevTables T, int64_t tile0, int64_t ntiles, int WB, int NL) {
    constexpr int G = 64 / P;
    constexpr bool UPD = MODE == BWD_UPDATE, MM = MODE == BWD_MM;
    constexpr bool NEEDF = UPD || MM, BAR = MODE == BWD_EN_BAR || MM || MODE == BWD_STORE_BAR;
    constexpr bool STOREB = UPD || MODE == BWD_STORE || MODE == BWD_STORE_BAR;
    extern __shared__ float lds_f[];
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int g = lane / P, p = lane % P;
    int64_t tile = tile0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= tile0 + ntiles) return;
    for (;;) {
        float *buf0 = lds_f + (size_t)wave * lds_words_pass(P, WB, NL);
        int *meta = (int *)(buf0 + 2 * WB * G);
        int *off = meta + NL * G;
        const TileCtx tc = tile_ctx(T, tile);
        const int row = T.bdd[tile * 64 + g];
        preload_meta<G>(T, tc, lane, meta, off);
        const int nlev = tc.nlev;
        auto level = [&](int l) {
            Lev v{0, 0, 0};
            if (l >= 0 && l < nlev) {
                const int w = meta[l * G + g] & 0xFFFF;
                v.W = G == 1 ? uni(w) : w;
                v.R = uni(meta[l * G] >> 16);
                v.base = tc.nbase + (int64_t)uni(off[l]);
            }
            return v;
        };
        const int mine = p * G + g;

        Lev cn{0, 0, 0}, c0 = level(nlev - 1), cp = level(nlev - 2);  // levels l+1, l, l-1
        uint32_t tpn[RMAX];
        float fn[RMAX];
    #pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            tpn[r] = r < c0.R ? T.topo[c0.base + r * 64 + lane] : 0u;
            fn[r] = (NEEDF && r < c0.R) ? T.F[c0.base + r * 64 + lane] : 0.f;
        }
        const int et = tc.ebase + (nlev - 1) * G + g;
        float lamn = T.lam[et], aSn = (UPD || BAR) ? T.aS[et] : 0.f, omn = UPD ? T.omega[et] : 0.f;
        int cur = 0;  // buffer holding B of level l+1 (terminals only, below the last level)
        if (p == 0) {
            buf0[g] = kInf;
            buf0[G + g] = 0.f;
        }
        wave_sync();
        for (int l = nlev - 1; l >= 0; --l) {
            const float lam = lamn, om = omn, aS = aSn;
            uint32_t tp[RMAX];
            float fv[RMAX];
    #pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                tp[r] = tpn[r];
                fv[r] = fn[r];
            }
            const float *bn = buf0 + cur * WB * G;
            float *bc = buf0 + (cur ^ 1) * WB * G;
            // B of level l+1, computed last hop, to global memory
            if (STOREB) {
                float *bg = T.B + cn.base;
    #pragma unroll
                for (int r = 0; r < RMAX; ++r)
                    if (r < cn.R && in_level<P>(r, cn.R, lane, cn.W)) bg[r * 64 + lane] = bn[mine + r * P * G];
            }
            // prefetch level l-1
    #pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                tpn[r] = r < cp.R ? T.topo[cp.base + r * 64 + lane] : 0u;
                fn[r] = (NEEDF && r < cp.R) ? T.F[cp.base + r * 64 + lane] : 0.f;
            }
            if (l > 0) {
                const int e = tc.ebase + (l - 1) * G + g;
                lamn = T.lam[e];
                if (UPD || BAR) aSn = T.aS[e];
                if (UPD) omn = T.omega[e];
            }
            float m0 = kInf, m1 = kInf;
            const uint32_t dead = (uint32_t)cn.W | ((uint32_t)cn.W << 16);
    #pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                if (r < c0.R) {
                    if (!in_level<P>(r, c0.R, lane, c0.W)) tp[r] = dead;
                    if (NEEDF) {
                        // a lane past the level's end has two 0-terminal children: its cost is +inf
                        const float b0 = bn[(int)(tp[r] & 0xFFFFu) * G + g];
                        const float b1 = bn[(int)(tp[r] >> 16) * G + g];
                        m0 = fminf(m0, fv[r] + b0);
                        m1 = fminf(m1, fv[r] + b1);
                    }
                }
            }
            const float lam_use = BAR ? lam + aS : lam;
            float lam_new = lam_use;
            if (NEEDF) {
                m0 = team_min<P>(m0);
                m1 = team_min<P>(m1);
                if (c0.W > 0) {
                    m1 += lam_use;
                    if (UPD) {
                        const float Mn = om * (m1 - m0);
                        lam_new = lam - Mn + aS;
                        if (p == 0) {
                            const int e = tc.ebase + l * G + g;
                            T.lam[e] = lam_new;
                            T.M[e] = Mn;
                        }
                    } else if (p == 0) {
                        const int ce = T.slot2canon[tc.ebase + l * G + g];
                        T.out0[ce] = m0;
                        T.out1[ce] = m1;
                    }
                }
            }
    #pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                if (r < c0.R) {
                    // child costs read again from LDS: cheaper than keeping 2 * RMAX registers live
                    bc[mine + r * P * G] =
                        fminf(bn[(int)(tp[r] & 0xFFFFu) * G + g], lam_new + bn[(int)(tp[r] >> 16) * G + g]);
                }
            }
            if (p == 0) {
                bc[c0.W * G + g] = kInf;
                bc[(c0.W + 1) * G + g] = 0.f;
            }
            wave_sync();
            cur ^= 1;
            cn = c0;
            c0 = cp;
            cp = level(l - 2);
        }
        const float *bn = buf0 + cur * WB * G;  // B of level 0
        if (STOREB) {
            float *bg = T.B + cn.base;
    #pragma unroll
            for (int r = 0; r < RMAX; ++r)
                if (r < cn.R && in_level<P>(r, cn.R, lane, cn.W)) bg[r * 64 + lane] = bn[mine + r * P * G];
        }
        if (!MM && p == 0 && row >= 0) {
            const float e0 = bn[g];  // B(root) = E^j at the multipliers swept
            if (BAR) T.energies[row] = e0;
            else T.en_lam[row] = e0;
        }
        if (!LOOP) break;
        tile += (int64_t)gridDim.x * (blockDim.x >> 6);
        if (tile >= tile0 + ntiles) break;
        wave_sync();
    }  // tiles
}

inline unsigned full_grid(int64_t ntiles, int wpb) { return (unsigned)((ntiles + wpb - 1) / wpb); }

template <int P, int RMAX>
hipError_t fwd_dispatch(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s) {
    if (c.wpb_f < 1 || c.wpb_f > kMaxWavesPerBlock) return hipErrorInvalidConfiguration;
    const unsigned full = full_grid(c.ntiles, c.wpb_f);
    dim3 grid(full), block(64 * c.wpb_f);
    size_t lds = (size_t)c.wpb_f * lds_words_pass(P, c.WB, c.NL) * 4;
    if (mode == FWD_UPDATE && c.grid_f > 0 && (unsigned)c.grid_f < full)
        hipLaunchKernelGGL((k_fwd<P, RMAX, FWD_UPDATE, true>), dim3(c.grid_f), block, lds, s, t, c.tile0, c.ntiles,
                           c.WB, c.NL);
    else if (mode == FWD_UPDATE)
        hipLaunchKernelGGL((k_fwd<P, RMAX, FWD_UPDATE, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WB, c.NL);
    else if (mode == FWD_SWEEP_BAR)
        hipLaunchKernelGGL((k_fwd<P, RMAX, FWD_SWEEP_BAR, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WB,
                           c.NL);
    else
        hipLaunchKernelGGL((k_fwd<P, RMAX, FWD_SWEEP_LAM, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WB,
                           c.NL);
    return hipGetLastError();
}

template <int P, int RMAX>
hipError_t bwd_dispatch(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s) {
    if (c.wpb_b < 1 || c.wpb_b > kMaxWavesPerBlock) return hipErrorInvalidConfiguration;
    const unsigned full = full_grid(c.ntiles, c.wpb_b);
    dim3 grid(full), block(64 * c.wpb_b);
    size_t lds = (size_t)c.wpb_b * lds_words_pass(P, c.WB, c.NL) * 4;
    if (mode == BWD_UPDATE && c.grid_b > 0 && (unsigned)c.grid_b < full) {
        hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_UPDATE, true>), dim3(c.grid_b), block, lds, s, t, c.tile0, c.ntiles,
                           c.WB, c.NL);
        return hipGetLastError();
    }
    switch (mode) {
        case BWD_UPDATE: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_UPDATE, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WB, c.NL); break;
        case BWD_STORE: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_STORE, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WB, c.NL); break;
        case BWD_EN_LAM: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_EN_LAM, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WB, c.NL); break;
        case BWD_EN_BAR: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_EN_BAR, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WB, c.NL); break;
        case BWD_STORE_BAR: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_STORE_BAR, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WB, c.NL); break;
        default: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_MM, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WB, c.NL); break;
    }
    return hipGetLastError();
}


__global__ void k_deferred_sum(const int32_t *__restrict__ var_ptr, const int32_t *__restrict__ var_slots,
                               const float *__restrict__ M, float *__restrict__ S, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int q = var_ptr[i]; q < var_ptr[i + 1]; ++q) s += M[var_slots[q]];
    S[i] = s;
}

// aS[slot] = alpha[slot] * S[var(slot)] over all edge slots (padding slots have var -1).
__global__ void k_edge_alpha_s(const int32_t *__restrict__ evar, const float *__restrict__ alpha,
                               const float *__restrict__ S, float *__restrict__ aS, int64_t slots) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= slots) return;
    const int v = evar[e];
    aS[e] = v >= 0 ? alpha[e] * S[v] : 0.f;
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
                         const float *__restrict__ add) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int s = canon2slot[e];
    float v = src[s];
    if (add) v = v + add[s];
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

// Deterministic two-stage sum in fp64: block b sums a fixed contiguous chunk (thread-strided,
// then a fixed-shape tree), one block then sums the per-block partials in index order.
// neg_part != 0 sums min(0, x) instead of x.
__global__ __launch_bounds__(256) void k_sum_partial(const float *__restrict__ x, int64_t n, int64_t chunk,
                                                     int neg_part, double *partial) {
    __shared__ double sh[256];
    const int t = threadIdx.x;
    const int64_t a = (int64_t)blockIdx.x * chunk, b = a + chunk < n ? a + chunk : n;
    double acc = 0.0;
    for (int64_t j = a + t; j < b; j += 256) {
        const float v = x[j];
        acc += (double)(neg_part ? fminf(v, 0.f) : v);
    }
    sh[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_sum_final(const double *__restrict__ partial, int nb, double *out) {
    __shared__ double sh[256];
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int j = t; j < nb; j += 256) acc += partial[j];
    sh[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) *out = sh[0];
}

__global__ void k_check_params(const float *__restrict__ om, const float *__restrict__ al, int64_t E, int32_t *flags) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    // bit tests, so the check holds under -fno-honor-nans: an all-ones exponent is inf or NaN
    const uint32_t w = __float_as_uint(om[e]), a = __float_as_uint(al[e]);
    const bool w_nonfinite = (w & 0x7F800000u) == 0x7F800000u, a_nonfinite = (a & 0x7F800000u) == 0x7F800000u;
    const bool w_neg = (w >> 31) && (w & 0x7FFFFFFFu), a_neg = (a >> 31) && (a & 0x7FFFFFFFu);
    if (w_nonfinite || w_neg || __uint_as_float(w) > 1.f) atomicOr(&flags[0], 1);
    if (a_nonfinite || a_neg) atomicOr(&flags[1], 1);
}

// Per-segment fp64 sums (one workgroup per segment, fixed order): out[q] = sum of x (or of
// min(0, x) when neg_part) over [seg[q], seg[q+1]).  Per-instance bounds of a packed batch.
__global__ __launch_bounds__(256) void k_seg_sum(const float *__restrict__ x, const int64_t *__restrict__ seg,
                                                 int neg_part, double *out) {
    __shared__ double sh[256];
    const int t = threadIdx.x, q = blockIdx.x;
    const int64_t a = seg[q], b = seg[q + 1];
    double acc = 0.0;
    for (int64_t j = a + t; j < b; j += 256) {
        const float v = x[j];
        acc += (double)(neg_part ? fminf(v, 0.f) : v);
    }
    sh[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) out[q] = sh[0];
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <int P, int RMAX>
int pass_blocks_per_cu_t(const ClassLaunch &c, bool fwd) {
    int nb = 0;
    const int wpb = fwd ? c.wpb_f : c.wpb_b;
    const size_t lds = (size_t)wpb * lds_words_pass(P, c.WB, c.NL) * 4;
    hipError_t e = fwd ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &nb, reinterpret_cast<const void *>(&k_fwd<P, RMAX, FWD_UPDATE, true>), 64 * wpb, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &nb, reinterpret_cast<const void *>(&k_bwd<P, RMAX, BWD_UPDATE, true>), 64 * wpb, lds);
    return e == hipSuccess ? nb : 0;
}

}  // namespace

int pass_blocks_per_cu(const ClassLaunch &c, bool fwd) {
#define DD_OCC(PP, RR) if (c.P == PP && c.RMAX == RR) return pass_blocks_per_cu_t<PP, RR>(c, fwd);
    DD_CLASSES(DD_OCC)
#undef DD_OCC
    return 0;
}

hipError_t launch_seg_sum(const float *x, const int64_t *seg, int k, int neg_part, double *out, hipStream_t s) {
    if (k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_sum, dim3(k), dim3(256), 0, s, x, seg, neg_part, out);
    return hipGetLastError();
}

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

hipError_t launch_edge_alpha_s(const int32_t *evar, const float *alpha, const float *S, float *aS, int64_t slots,
                               hipStream_t s) {
    if (slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_edge_alpha_s, dim3(blocks_for(slots, 256)), dim3(256), 0, s, evar, alpha, S, aS, slots);
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

hipError_t launch_gather(const int32_t *canon2slot, const float *src, float *dst, int64_t E, const float *add,
                         hipStream_t s) {
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(E, 256)), dim3(256), 0, s, canon2slot, src, dst, E, add);
    return hipGetLastError();
}

hipError_t launch_seg_softmax(const int32_t *var_ptr, const int32_t *var_canon, const float *x, float *y, int n,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_softmax, dim3(blocks_for(n, 256)), dim3(256), 0, s, var_ptr, var_canon, x, y, n);
    return hipGetLastError();
}

hipError_t launch_sum(const float *x, int64_t n, int neg_part, double *partial, double *out, hipStream_t s) {
    const int nb = (int)std::min<int64_t>(kSumBlocks, std::max<int64_t>(1, (n + 4095) / 4096));
    const int64_t chunk = (std::max<int64_t>(n, 1) + nb - 1) / nb;
    hipLaunchKernelGGL(k_sum_partial, dim3(nb), dim3(256), 0, s, x, n, chunk, neg_part, partial);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partial, nb, out);
    return hipGetLastError();
}

hipError_t launch_check_params(const float *omega, const float *alpha, int64_t E, int32_t *flags, hipStream_t s) {
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_params, dim3(blocks_for(E, 256)), dim3(256), 0, s, omega, alpha, E, flags);
    return hipGetLastError();
}

}  // namespace dd
