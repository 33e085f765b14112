// features.hip -- per-row solver features of the appendix's feature table on CDNA4 (gfx950):
// the smoothed subproblems E_tau^j(lambda) = -tau log sum_{x in X_j} exp(-<lambda, x>/tau) and their
// gradients, the marginals P(x_l = 1) of the Gibbs distribution exp(-<lambda, x>/tau) on X_j.
//
// One wavefront per tile, as in the pass kernels.  Phase 1 sweeps the levels bottom-up in the
// (soft-min, +) semiring: Bs(v) = softmin(Bs(lo v), lambda_l + Bs(hi v)) is the smoothed cost from
// v to the 1-terminal, and Bs(root) = E_tau^j.  The Gibbs distribution conditioned on reaching v
// takes v's beta arc with probability exp(-(beta lambda_l + Bs(child_beta v) - Bs(v)) / tau); the
// two probabilities sum to 1 and are fixed by the same exponential the soft-min evaluates, so
// phase 1 stores, per node, the smaller of the two with its sign bit naming the arc it belongs to
// (clear: lo, set: hi).  Phase 2 sweeps top-down pushing probability mass from the root (mass 1)
// along both arcs, the larger share taken as 1 minus the smaller; the mass that takes hi arcs at
// level l is P(x_l = 1).  Mass is accumulated in LDS with native float adds.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace dd {
namespace {

using namespace dev;

// soft-min of the lo-arc cost a and the hi-arc cost b at temperature tau (itau = 1 / tau); q gets
// the smaller of the two arc probabilities, signed as above (an arc into an infinite cost has
// probability 0, a tie splits evenly)
__device__ __forceinline__ float softmin2(float a, float b, float tau, float itau, float &q) {
    if (a == kInf) {
        q = 0.f;
        return b;
    }
    if (b == kInf) {
        q = -0.f;
        return a;
    }
    const float m = fminf(a, b), e = expf(-fabsf(a - b) * itau);
    const float small = e * __builtin_amdgcn_rcpf(1.f + e);  // 1 + e lies in [1, 2]
    q = a <= b ? -small : small;
    return m - tau * log1pf(e);
}

template <int P, int RMAX>
__global__ __launch_bounds__(256) void k_smooth(DevTables T, float *__restrict__ Q, float tau, int bar,
                                                float *__restrict__ E_out, float *__restrict__ p_out, int64_t tile0,
                                                int64_t ntiles, int WB, int NL) {
    constexpr int G = 64 / P;
    extern __shared__ float lds_f[];
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int g = lane / P, p = lane % P;
    const int64_t tile = tile0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= tile0 + ntiles) return;
    float *nbuf = lds_f + (size_t)wave * lds_words_features(P, WB, NL);  // two node buffers
    int *meta = (int *)(nbuf + 2 * WB * G);
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
    // a level's rows (and its edge data) are loaded one hop ahead through level-sized resources:
    // every load is issued unconditionally, rows past a level load 0 and are never used
    auto rows_u = [&](const uint32_t *a, const Lev &c, uint32_t (&v)[RMAX]) {
        const rsrc_t r = buf(a + c.base, c.R * 256);
#pragma unroll
        for (int q = 0; q < RMAX; ++q) v[q] = ld1(r, (q * 64 + lane) * 4);
    };
    auto rows_f = [&](const float *a, const Lev &c, float (&v)[RMAX]) {
        const rsrc_t r = buf(a + c.base, c.R * 256);
#pragma unroll
        for (int q = 0; q < RMAX; ++q) v[q] = ld1f(r, (q * 64 + lane) * 4);
    };
    const int ne = nlev * G * 4;
    const rsrc_t lam_r = buf(T.lam + tc.ebase, ne), aS_r = buf(T.aS + tc.ebase, ne);
    auto edge_off = [&](int l) { return (max(min(l, nlev - 1), 0) * G + g) * 4; };
    const int mine = p * G + g;
    const float itau = 1.f / tau;
    // ---- phase 1: bottom-up soft-min costs (in LDS), arc probabilities stored to Q
    int cur = 0;  // buffer holding level l+1
    if (p == 0) {
        nbuf[g] = kInf;
        nbuf[G + g] = 0.f;
    }
    Lev c0 = level(nlev - 1), cn{0, 0, 0};
    uint32_t tpn[RMAX];
    rows_u(T.topo, c0, tpn);
    float lamn = ld1f(lam_r, edge_off(nlev - 1)), aSn = ld1f(aS_r, edge_off(nlev - 1));
    wave_sync();
    for (int l = nlev - 1; l >= 0; --l) {
        uint32_t tp[RMAX];
#pragma unroll
        for (int r = 0; r < RMAX; ++r) tp[r] = tpn[r];
        const float lam = bar ? lamn + aSn : lamn;
        const Lev cp = level(l - 1);
        rows_u(T.topo, cp, tpn);  // hop l-1
        lamn = ld1f(lam_r, edge_off(l - 1));
        aSn = ld1f(aS_r, edge_off(l - 1));
        const float *bn = nbuf + cur * WB * G;
        float *bc = nbuf + (cur ^ 1) * WB * G;
        const uint32_t dead = (uint32_t)cn.W | ((uint32_t)cn.W << 16);
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            if (r < c0.R) {
                const bool ok = in_level<P>(r, c0.R, lane, c0.W);
                const uint32_t t = ok ? tp[r] : dead;
                float q;
                const float v =
                    softmin2(bn[(int)(t & 0xFFFFu) * G + g], lam + bn[(int)(t >> 16) * G + g], tau, itau, q);
                bc[mine + r * P * G] = v;
                if (ok) Q[c0.base + r * 64 + lane] = q;
            }
        }
        wave_sync();  // the terminals' slots may have been written by another lane
        if (p == 0) {
            bc[c0.W * G + g] = kInf;
            bc[(c0.W + 1) * G + g] = 0.f;
        }
        wave_sync();
        cur ^= 1;
        cn = c0;
        c0 = cp;
    }
    if (p == 0 && row >= 0 && E_out) E_out[row] = nbuf[cur * WB * G + g];  // Bs(root)
    // phase 2 reads back what phase 1 stored: make the stores visible to this wave's loads
    __threadfence();
    wave_sync();
    // ---- phase 2: top-down probability mass; buffers: mass of level l (pa) and of level l+1 (pb)
    float *pa = nbuf, *pb = nbuf + WB * G;
    {
        const int R0 = uni(meta[0] >> 16);
        for (int r = 0; r < R0; ++r) pa[mine + r * P * G] = 0.f;
        if (p == 0) pa[g] = 1.f;
    }
    c0 = level(0);
    Lev c1 = level(1);
    float qn[RMAX];  // arc probabilities of the next level
    rows_u(T.topo, c0, tpn);
    rows_f(Q, c0, qn);
    wave_sync();
    for (int l = 0; l < nlev; ++l) {
        const int Wn = c1.W;
        uint32_t tp[RMAX];
        float qv[RMAX];
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            tp[r] = tpn[r];
            qv[r] = qn[r];
            if (r < c1.R) pb[mine + r * P * G] = 0.f;
        }
        // prefetch hop l+1
        rows_u(T.topo, c1, tpn);
        rows_f(Q, c1, qn);
        wave_sync();  // the next level's mass is cleared before any lane adds to it
        float hi_mass = 0.f;
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            if (r < c0.R) {
                const bool ok = in_level<P>(r, c0.R, lane, c0.W);
                const float m = ok ? pa[mine + r * P * G] : 0.f;
                if (m > 0.f) {
                    const int lo = (int)(tp[r] & 0xFFFFu), hi = (int)(tp[r] >> 16);
                    const float small = fabsf(qv[r]), large = 1.f - small;
                    const bool hi_small = signbit(qv[r]);
                    const float q1 = hi_small ? small : large;
                    if (lo < Wn) lds_fadd(&pb[lo * G + g], m * (hi_small ? large : small));
                    if (hi < Wn) lds_fadd(&pb[hi * G + g], m * q1);
                    hi_mass += m * q1;
                }
            }
        }
        hi_mass = team_sum<P>(hi_mass);
        if (p == 0 && c0.W > 0) p_out[T.slot2canon[tc.ebase + l * G + g]] = hi_mass;
        wave_sync();
        float *t = pa;
        pa = pb;
        pb = t;
        c0 = c1;
        c1 = level(l + 2);
    }
}

template <int P, int RMAX>
hipError_t smooth_dispatch(const DevTables &t, const ClassLaunch &c, float *Q, float tau, int bar, float *E_out,
                           float *p_out, hipStream_t s) {
    int wpb = c.wpb_b;
    if (wpb < 1 || wpb > kMaxWavesPerBlock) return hipErrorInvalidConfiguration;
    while (wpb > 1 && (size_t)wpb * lds_words_features(P, c.WB, c.NL) * 4 > 64 * 1024) wpb /= 2;
    dim3 grid((unsigned)((c.ntiles + wpb - 1) / wpb)), block(64 * wpb);
    const size_t lds = (size_t)wpb * lds_words_features(P, c.WB, c.NL) * 4;
    hipLaunchKernelGGL((k_smooth<P, RMAX>), grid, block, lds, s, t, Q, tau, bar, E_out, p_out, c.tile0, c.ntiles,
                       c.WB, c.NL);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_smooth(const DevTables &t, const ClassLaunch &c, float *Q, float tau, int bar, float *E_out,
                         float *p_out, hipStream_t s) {
    if (c.ntiles <= 0) return hipSuccess;
#define DD_SMOOTH(PP, RR) \
    if (c.P == PP && c.RMAX == RR) return smooth_dispatch<PP, RR>(t, c, Q, tau, bar, E_out, p_out, s);
    DD_CLASSES(DD_SMOOTH)
#undef DD_SMOOTH
    return hipErrorInvalidValue;
}

}  // namespace dd
