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
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"

namespace dd {
namespace {

using namespace dev;

// alpha * S_i of the edges an update pass visits, formed in the pass (the deferred sums S are
// complete when it starts). The variable of the next hop's edge is loaded a hop earlier, so the load
// of its S waits for nothing issued in the current hop. Padding slots (variable -1) give 0, as the
// stored alpha * S has; the pass stores the value beside the multipliers, so the stored array holds
// what the separate per-edge launch would have written. Used when the instance's form_as is set.
struct EdgeAlphaS {
    float al = 0.f, s = 0.f;  // alpha and S of the next hop's edge
    int v = -1;               // its variable
    int vn = -1;              // the variable of the edge after it
    // the value for the next hop: a rounded product, as a stored one is (no multiply-add with its use)
    __device__ __forceinline__ float value() const {
        float r = v >= 0 ? al * s : 0.f;
        __asm__("" : "+v"(r));
        return r;
    }
    // S of the next hop's edge (0 on padding), as the S-per-edge array holds it
    __device__ __forceinline__ float s_edge() const { return v >= 0 ? s : 0.f; }
    // loads for edge e, whose variable is vn, and the variable of edge e2
    __device__ __forceinline__ void prefetch(const DevTables &T, int64_t e, int64_t e2) {
        al = T.alpha[e];
        s = T.S[vn >= 0 ? vn : 0];
        v = vn;
        vn = T.evar[e2];
    }
};

// LOOP = false: one wave per tile.  LOOP = true (update passes on a resident grid): each wave
// takes tiles w, w + stride, ... (stride = waves in the grid); tiles are sorted by decreasing
// length within a class, so striding mixes long and short ones.  FAS (update modes): the pass forms
// alpha * S itself (the instance's form_as) instead of reading the stored array.
template <int P, int RMAX, int MODE, bool LOOP, bool FAS>
__global__ __launch_bounds__(256) void k_fwd(DevTables T, int64_t tile0, int64_t ntiles, int WB, int NL) {
    constexpr int G = 64 / P;
    constexpr bool REC = MODE == FWD_UPDATE_REC, UPD = MODE == FWD_UPDATE || REC;
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
        constexpr bool fas = UPD && FAS;  // this pass forms alpha * S (the instance's form_as)
        EdgeAlphaS eas;
        if (fas) eas.vn = T.evar[tc.ebase + g];  // issued first: the level table's load covers its wait
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
        float lamn = T.lam[tc.ebase + g], aSn = fas ? 0.f : T.aS[tc.ebase + g], omn = UPD ? T.omega[tc.ebase + g] : 0.f;
        if (fas) eas.prefetch(T, tc.ebase + g, tc.ebase + min(1, nlev - 1) * G + g);
        if (p == 0) Fb[g] = 0.f;  // F(root) = 0
        wave_sync();
        for (int l = 0; l < nlev; ++l) {
            const float lam = lamn, om = omn, aS = fas ? eas.value() : aSn;
            const float Se_now = fas && REC ? eas.s_edge() : 0.f;  // kept for the reverse sweeps
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
            // prefetch (issued after this hop's stores): topology of l+1, B of l+2, edge data of l+1.
            // Rows past a level load 0 without a memory access, and the last hop reloads its own
            // edge data: no branch, so no prefetched register is merged with its old value (a merge
            // would wait for the load right after issuing it).
            {
                const rsrc_t tr = buf(T.topo + c1.base, c1.R * 256), br = buf(T.B + c2.base, c2.R * 256);
    #pragma unroll
                for (int r = 0; r < RMAX; ++r) {
                    tpn[r] = ld1(tr, (r * 64 + lane) * 4);
                    if (UPD) bvn[r] = ld1f(br, (r * 64 + lane) * 4);
                }
                const int e = tc.ebase + min(l + 1, nlev - 1) * G + g;
                lamn = T.lam[e];
                if (UPD) omn = T.omega[e];
                if (fas) eas.prefetch(T, e, tc.ebase + min(l + 2, nlev - 1) * G + g);
                else aSn = T.aS[e];
            }
            float m0 = kInf, m1 = kInf;
            int k0 = INT_MAX, k1 = INT_MAX, h0 = 0, h1 = 0;  // recording: first node attaining the lane's min
            const uint32_t dead = (uint32_t)c1.W | ((uint32_t)c1.W << 16);
    #pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                if (r < c0.R) {
                    if (!in_level<P>(r, c0.R, lane, c0.W)) tp[r] = dead;
                    if (UPD) {
                        const int lo = (int)(tp[r] & 0xFFFFu), hi = (int)(tp[r] >> 16);
                        const float v0 = fv[r] + Bst[lo * G + g], v1 = fv[r] + Bst[hi * G + g];
                        if (REC) argmin_step(v0, m0, r * P + p, lo, k0, h0);
                        if (REC) argmin_step(v1, m1, r * P + p, hi, k1, h1);
                        m0 = fminf(m0, v0);
                        m1 = fminf(m1, v1);
                    }
                }
            }
            float lam_new;
            if (UPD) {
                const float lm0 = m0, lm1 = m1;
                m0 = team_min<P>(m0);
                m1 = team_min<P>(m1);
                const float M1 = m1;
                m1 += lam;
                const float d = m1 - m0;
                const float Mn = om * d;
                const bool live = c0.W > 0;  // this team's diagram has a node at level l
                lam_new = live ? lam - Mn + aS : lam;
                // stored by the team's first lane through a resource over the tile's edges: the
                // offsets of the other lanes, and of teams with no node here, fall outside it
                const int ne = nlev * G * 4, off = p == 0 && live ? (l * G + g) * 4 : ne;
                st1(buf(T.lam + tc.ebase, ne), off, lam_new);
                st1(buf(T.M + tc.ebase, ne), off, Mn);
                if (fas) st1(buf(T.aS + tc.ebase, ne), off, aS);
                if (fas && REC) st1(buf(T.Se_rec ? T.Se_rec + tc.ebase : T.lam, T.Se_rec ? ne : 0), off, Se_now);
                if (REC) record_argmins_team<P>(T, tc.ebase, ne, off, lm0, m0, k0, h0, lm1, M1, k1, h1, d);
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
template <int P, int RMAX, int MODE, bool LOOP, bool FAS>
__global__ __launch_bounds__(256) void k_bwd(DevTables T, int64_t tile0, int64_t ntiles, int WB, int NL) {
    constexpr int G = 64 / P;
    constexpr bool REC = MODE == BWD_UPDATE_REC, UPD = MODE == BWD_UPDATE || REC, MM = MODE == BWD_MM;
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
        constexpr bool fas = UPD && FAS;  // this pass forms alpha * S (the instance's form_as)
        EdgeAlphaS eas;
        if (fas) eas.vn = T.evar[tc.ebase + (tc.nlev - 1) * G + g];  // issued first, as in the forward pass
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
        float lamn = T.lam[et], aSn = (BAR || (UPD && !fas)) ? T.aS[et] : 0.f, omn = UPD ? T.omega[et] : 0.f;
        if (fas) eas.prefetch(T, et, tc.ebase + max(nlev - 2, 0) * G + g);
        int cen = MM ? T.slot2canon[et] : 0;  // canonical edge of the min-marginals (padding slots: unused)
        int cur = 0;  // buffer holding B of level l+1 (terminals only, below the last level)
        if (p == 0) {
            buf0[g] = kInf;
            buf0[G + g] = 0.f;
        }
        wave_sync();
        for (int l = nlev - 1; l >= 0; --l) {
            const float lam = lamn, om = omn, aS = fas ? eas.value() : aSn;
            const float Se_now = fas && REC ? eas.s_edge() : 0.f;  // kept for the reverse sweeps
            const int ce = cen;
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
            // prefetch level l-1 (unconditional, as in the forward pass; the first level reloads its own
            // edge data)
            {
                const rsrc_t tr = buf(T.topo + cp.base, cp.R * 256), fr = buf(T.F + cp.base, cp.R * 256);
    #pragma unroll
                for (int r = 0; r < RMAX; ++r) {
                    tpn[r] = ld1(tr, (r * 64 + lane) * 4);
                    if (NEEDF) fn[r] = ld1f(fr, (r * 64 + lane) * 4);
                }
                const int e = tc.ebase + max(l - 1, 0) * G + g;
                lamn = T.lam[e];
                if (UPD) omn = T.omega[e];
                if (fas) eas.prefetch(T, e, tc.ebase + max(l - 2, 0) * G + g);
                else if (UPD || BAR) aSn = T.aS[e];
                if (MM) cen = T.slot2canon[e];
            }
            float m0 = kInf, m1 = kInf;
            int k0 = INT_MAX, k1 = INT_MAX, h0 = 0, h1 = 0;  // recording: first node attaining the lane's min
            const uint32_t dead = (uint32_t)cn.W | ((uint32_t)cn.W << 16);
    #pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                if (r < c0.R) {
                    if (!in_level<P>(r, c0.R, lane, c0.W)) tp[r] = dead;
                    if (NEEDF) {
                        // a lane past the level's end has two 0-terminal children: its cost is +inf
                        const int lo = (int)(tp[r] & 0xFFFFu), hi = (int)(tp[r] >> 16);
                        const float v0 = fv[r] + bn[lo * G + g], v1 = fv[r] + bn[hi * G + g];
                        if (REC) argmin_step(v0, m0, r * P + p, lo, k0, h0);
                        if (REC) argmin_step(v1, m1, r * P + p, hi, k1, h1);
                        m0 = fminf(m0, v0);
                        m1 = fminf(m1, v1);
                    }
                }
            }
            const float lam_use = BAR ? lam + aS : lam;
            float lam_new = lam_use;
            if (NEEDF) {
                const float lm0 = m0, lm1 = m1;
                m0 = team_min<P>(m0);
                m1 = team_min<P>(m1);
                const float M1 = m1;
                m1 += lam_use;
                const bool live = c0.W > 0;  // this team's diagram has a node at level l
                if (UPD) {
                    const float d = m1 - m0;
                    const float Mn = om * d;
                    lam_new = live ? lam - Mn + aS : lam_new;
                    // the team's first lane stores; other offsets fall outside the tile's edges
                    const int ne = nlev * G * 4, off = p == 0 && live ? (l * G + g) * 4 : ne;
                    st1(buf(T.lam + tc.ebase, ne), off, lam_new);
                    st1(buf(T.M + tc.ebase, ne), off, Mn);
                    if (fas) st1(buf(T.aS + tc.ebase, ne), off, aS);
                    if (fas && REC)
                        st1(buf(T.Se_rec ? T.Se_rec + tc.ebase : T.lam, T.Se_rec ? ne : 0), off, Se_now);
                    if (REC) record_argmins_team<P>(T, tc.ebase, ne, off, lm0, m0, k0, h0, lm1, M1, k1, h1, d);
                } else if (p == 0 && live) {
                    T.out0[ce] = m0;
                    T.out1[ce] = m1;
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

// ------------------------------------------------------------------------------------------
// One-wave diagrams (P = 64): the same passes, laid out for wide memory operations.
// ------------------------------------------------------------------------------------------
// Each lane owns 4 consecutive nodes of a group of 256 (node k = 256 q + 4 lane + j), so
// every row of F or B moves with one 16-byte access per lane and a row of byte-coded child
// codes with one 4-byte access (decoded by child_codes; the 4-byte codes of a level without
// byte codes with one 16-byte access): a quarter of the memory instructions of one node per
// lane, whose address processing, not HBM, would otherwise bound the pass.  Levels of these
// tiles start at multiples of 4 nodes.
// A hop branches once on its level's group count Q (a binary tree of scalar compares) into a
// body unrolled over exactly Q groups, so no group carries a predicate of its own.  Node
// buffers hold RMAX rows of 64 and 64 more slots: clears and staged groups cover all RMAX
// rows without a test (slots past a level are never read), the terminal sentinels of a full
// last group fit, and arcs into a terminal send their min-update to the lane's own sink slot
// past the rows (a terminal needs no forward cost; one slot per lane keeps the atomics
// conflict free).  Global rows go through buffer resources sized to the level: an access
// past them loads 0 without touching memory or is dropped, so every load and store is issued
// unconditionally (no branch, no merge of a prefetched register with its old value, which
// would force a wait right after the load), and every path of a hop issues the same memory
// operations after its prefetch, so the next hop waits for the prefetched rows alone.  The
// multiplier and M of a hop are stored by lane 0 alone: the other lanes' offsets fall outside
// the tile.  Every level of a built diagram holds at least one node, so the update needs no
// empty-level case.  The arithmetic is that of the general kernels above; the min over a
// level's arcs is exact, so the order in which a lane visits its nodes does not matter.
// The sweeps that reverse mode reads also record each node's argmin parent arc 2 k + beta: their
// next-level buffer holds 64-bit keys (cost, code) (cost_key), so one integer min per arc forms the
// cost and, among arcs of equal cost, the lowest code (lo before hi, lowest node); the next hop
// splits the keys of its level into the F row and the code row.
template <int Q, int RMAX, int MODE, typename Prefetch>
__device__ __forceinline__ void fwd_hop_w(rsrc_t Fr, rsrc_t lam_r, rsrc_t M_r, rsrc_t rec_r, rsrc_t md_r, rsrc_t Pr,
                                          float *Fb, const float *Bst, const uint32_t (&cw)[RMAX / 4], uint32_t cb,
                                          rsrc_t traw, int lane, int out, const Lev &c0, const Lev &c1, float lam,
                                          float om, float aS, Prefetch &&prefetch) {
    constexpr bool REC = MODE == FWD_UPDATE_REC, UPD = MODE == FWD_UPDATE || REC;
    constexpr bool PAR = REC || MODE == FWD_SWEEP_LAM;
    constexpr int QM = RMAX / 4, SINK = RMAX * 64;
    const int l16 = lane16(lane);
    uint64_t *Kb = (uint64_t *)Fb;  // PAR: the keys of this level, then of level l+1
    f32x4 fv[Q];
    u32x4 t[Q];
    child_codes<Q>(cw, cb, c1.W == 0, traw, lane, t);
    if constexpr (PAR) {
        const int l32 = lane32(lane), l8 = lane8(lane);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const u64x2 a = *(const u64x2 *)((const char *)Kb + l32 + q * 2048);
            const u64x2 b = *(const u64x2 *)((const char *)Kb + l32 + q * 2048 + 16);
            fv[q] = f32x4{key_cost(a[0]), key_cost(a[1]), key_cost(b[0]), key_cost(b[1])};
            // codes of this level's nodes (every slot past the width holds 0xFFFF)
            st2(Pr, l8 + q * 512, ((uint32_t)a[0] & 0xFFFFu) | ((uint32_t)a[1] << 16),
                ((uint32_t)b[0] & 0xFFFFu) | ((uint32_t)b[1] << 16));
        }
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q) fv[q] = lds4(Fb, l16 + q * 1024);  // slots past the level's width hold +inf
    }
    // last group: this lane's slots past the level's width get two 0-terminal arcs
    const int rem = c0.W - (Q - 1) * 256 - lane * 4;
    const uint32_t dead = (uint32_t)c1.W | ((uint32_t)c1.W << 16);
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (j >= rem) t[Q - 1][j] = dead;
#pragma unroll
    for (int q = 0; q < Q; ++q) st4(Fr, l16 + q * 1024, fv[q]);  // F for the backward pass
    prefetch(l16);  // after the stores: waiting for the prefetched rows then waits for no fresh store
    if constexpr (PAR) {
        const int l32 = lane32(lane);
        const uint64_t none = cost_key(kInf, 0xFFFFu);
        const u64x2 none2 = {none, none};
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            *(u64x2 *)((char *)Kb + l32 + q * 2048) = none2;  // level l+1 accumulates here
            *(u64x2 *)((char *)Kb + l32 + q * 2048 + 16) = none2;
        }
    } else {
        const f32x4 inf4 = {kInf, kInf, kInf, kInf};
#pragma unroll
        for (int q = 0; q < QM; ++q) lds4(Fb, l16 + q * 1024) = inf4;  // F of level l+1 accumulates here
    }
    wave_sync();
    float lam_new;
    if (UPD) {
        float m0 = kInf, m1 = kInf;
        int k0 = INT_MAX, k1 = INT_MAX, h0 = 0, h1 = 0;  // recording: first node attaining the lane's min
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int lo = (int)(t[q][j] & 0xFFFFu), hi = (int)(t[q][j] >> 16);
                const float v0 = fv[q][j] + Bst[lo], v1 = fv[q][j] + Bst[hi];
                if (REC) argmin_step(v0, m0, q * 256 + (l16 >> 2) + j, lo, k0, h0);
                if (REC) argmin_step(v1, m1, q * 256 + (l16 >> 2) + j, hi, k1, h1);
                m0 = fminf(m0, v0);
                m1 = fminf(m1, v1);
            }
        const float M0 = team_min<64>(m0), M1 = team_min<64>(m1);
        const float d = (M1 + lam) - M0;
        const float Mn = om * d;
        lam_new = lam - Mn + aS;
        st1(lam_r, out, lam_new);
        st1(M_r, out, Mn);
        if (REC) record_argmins(rec_r, md_r, out, m0, M0, k0, h0, m1, M1, k1, h1, d);
    } else {
        lam_new = MODE == FWD_SWEEP_BAR ? lam + aS : lam;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int lo = (int)(t[q][j] & 0xFFFFu), hi = (int)(t[q][j] >> 16);
            if constexpr (PAR) {
                const uint32_t k2 = 2u * (uint32_t)(q * 256 + (l16 >> 2) + j);
                lds_umin64(&Kb[lo < c1.W ? lo : SINK + lane], cost_key(fv[q][j], k2));
                lds_umin64(&Kb[hi < c1.W ? hi : SINK + lane], cost_key(fv[q][j] + lam_new, k2 + 1u));
            } else {
                lds_fmin(&Fb[lo < c1.W ? lo : SINK + lane], fv[q][j]);
                lds_fmin(&Fb[hi < c1.W ? hi : SINK + lane], fv[q][j] + lam_new);
            }
        }
    wave_sync();
}

template <int RMAX, int MODE, bool LOOP>
__global__ __launch_bounds__(256) void k_fwd_w(DevTables T, int64_t tile0, int64_t ntiles, int NL) {
    constexpr bool REC = MODE == FWD_UPDATE_REC, UPD = MODE == FWD_UPDATE || REC;
    constexpr bool PAR = REC || MODE == FWD_SWEEP_LAM;
    constexpr int NB = node_buf_w(RMAX), QM = RMAX / 4;
    extern __shared__ float lds_f[];
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    int64_t tile = tile0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= tile0 + ntiles) return;  // uniform per wave
    float *Fb = lds_f + (size_t)wave * (PAR ? lds_words_pass_w_par(RMAX, NL) : lds_words_pass_w(RMAX, NL));
    float *Bst = Fb + (PAR ? 2 * NB : NB);  // PAR: Fb holds NB 64-bit keys
    int *meta = (int *)(Bst + NB);
    int *off = meta + NL;
    const f32x4 inf4 = {kInf, kInf, kInf, kInf};
    // the recording sweeps keep the level table in registers when it fits (their LDS then holds the
    // node buffers alone, and more waves fit a CU): lane k holds levels k, k + 64, k + 128, k + 192
    constexpr int NR = kParRegLevels / 64;
    static_assert(NR == 4, "the register level table is read through a four-way choice");
    const bool regs = PAR && NL <= kParRegLevels;
    int mr[NR], orr[NR];
    for (;;) {
        const TileCtx tc = tile_ctx(T, tile);
        const int nlev = tc.nlev;
        if (regs) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int l = lane + 64 * r;
                mr[r] = l < nlev ? (int)T.widths[tc.wbase + l] | (T.lev_rows[tc.lbase + l] << 16) : 0;
                orr[r] = l < nlev ? T.lev_off[tc.lbase + l] : 0;
            }
        } else {
            preload_meta<1>(T, tc, lane, meta, off);
        }
        auto level = [&](int l) {
            Lev v{0, 0, 0};
            if (l < nlev) {
                int mw, ow;
                if (regs) {
                    const int r = l >> 6;  // uniform: a choice among the lane's registers, then one lane's
                    const int ms = r == 0 ? mr[0] : r == 1 ? mr[1] : r == 2 ? mr[2] : mr[3];
                    const int os = r == 0 ? orr[0] : r == 1 ? orr[1] : r == 2 ? orr[2] : orr[3];
                    mw = __builtin_amdgcn_readlane(ms, l & 63);
                    ow = __builtin_amdgcn_readlane(os, l & 63);
                } else {
                    mw = meta[l];
                    ow = off[l];
                }
                v.W = uni(mw & 0xFFFF);
                v.R = uni(mw >> 16);
                v.base = tc.nbase + (int64_t)uni(ow);
            }
            return v;
        };
        const rsrc_t lam_r = buf(T.lam + tc.ebase, nlev * 4), M_r = buf(T.M + tc.ebase, nlev * 4);
        const rsrc_t rec_r = rec_buf<REC>(T, tc, nlev), md_r = mdiff_buf<REC>(T, tc, nlev);
        const int out0 = lane * nlev * 4;  // hop l stores at out0 + 4 l: in range for lane 0 only
        Lev c0 = level(0), c1 = level(1), c2 = level(2);
        uint32_t cwn[QM], cbn = T.lev_code[tc.lbase];  // byte codes of the level's topology
        f32x4 bvn[QM];
        {
            const int l16 = lane16(lane);
            const rsrc_t cr = buf(T.tcode + c0.base, code_row_bytes(c0)), br = buf(T.B + c1.base, row_bytes(c1));
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                cwn[q] = ld1(cr, lane * 4 + q * 256);
                bvn[q] = UPD ? ld4f(br, l16 + q * 1024) : inf4;
            }
        }
        float lamn = T.lam[tc.ebase], aSn = T.aS[tc.ebase], omn = UPD ? T.omega[tc.ebase] : 0.f;
        if constexpr (PAR) {
            const int l32 = lane32(lane);
            const uint64_t none = cost_key(kInf, 0xFFFFu);
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                u64x2 a = {none, none};
                const u64x2 b = {none, none};
                if (q == 0 && lane == 0) a[0] = cost_key(0.f, 0xFFFFu);  // F(root) = 0
                *(u64x2 *)((char *)Fb + l32 + q * 2048) = a;
                *(u64x2 *)((char *)Fb + l32 + q * 2048 + 16) = b;
            }
        } else {
            const int l16 = lane16(lane);
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                f32x4 v = inf4;
                if (q == 0 && lane == 0) v[0] = 0.f;  // F(root) = 0
                lds4(Fb, l16 + q * 1024) = v;
            }
        }
        wave_sync();
        for (int l = 0; l < nlev; ++l) {
            const float lam = lamn, om = omn, aS = aSn;
            uint32_t cw[QM];
            const uint32_t cb = uni((int)cbn);
#pragma unroll
            for (int q = 0; q < QM; ++q) cw[q] = cwn[q];
            if (UPD) {
                // B of level l+1, then its terminals
                const int l16 = lane16(lane);
#pragma unroll
                for (int q = 0; q < QM; ++q) lds4(Bst, l16 + q * 1024) = bvn[q];
                if (lane == 0) {
                    Bst[c1.W] = kInf;
                    Bst[c1.W + 1] = 0.f;
                }
            }
            // prefetch: byte codes of l+1, B of l+2, edge data of l+1 (the last hop reloads its own)
            auto prefetch = [&](int l16) {
                const rsrc_t cr = buf(T.tcode + c1.base, code_row_bytes(c1)), br = buf(T.B + c2.base, row_bytes(c2));
#pragma unroll
                for (int q = 0; q < QM; ++q) {
                    cwn[q] = ld1(cr, lane * 4 + q * 256);
                    if (UPD) bvn[q] = ld4f(br, l16 + q * 1024);
                }
                cbn = T.lev_code[tc.lbase + min(l + 1, nlev - 1)];
                const int e = tc.ebase + min(l + 1, nlev - 1);
                lamn = T.lam[e];
                aSn = T.aS[e];
                if (UPD) omn = T.omega[e];
            };
            const rsrc_t Fr = buf(T.F + c0.base, node_bytes(c0));
            // codes of this level (the root has no parent; no codes recorded: every store dropped)
            const bool codes = PAR && T.Fpar && l > 0;
            const rsrc_t Pr = buf(codes ? (const void *)(T.Fpar + c0.base) : (const void *)T.F,
                                  codes ? code_bytes(c0) : 0);
            const rsrc_t traw = buf(T.topo + c0.base, row_bytes(c0));
            with_count<1, QM>(groups(c0), [&](auto qc) {
                fwd_hop_w<decltype(qc)::value, RMAX, MODE>(Fr, lam_r, M_r, rec_r, md_r, Pr, Fb, Bst, cw, cb, traw,
                                                           lane, out0 + 4 * l, c0, c1, lam, om, aS, prefetch);
            });
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

// Backward hop of level l: bn = B of level l+1 (Wn its width: terminals at Wn, Wn+1), bc
// receives B of level l, which also goes to global memory here, from registers.
template <int Q, int RMAX, int MODE>
__device__ __forceinline__ void bwd_hop_w(const DevTables &T, rsrc_t Br, rsrc_t Cr, rsrc_t lam_r, rsrc_t M_r,
                                          rsrc_t rec_r, rsrc_t md_r, const float *bn, float *bc,
                                          const u32x4 (&tp)[RMAX / 4],
                                          const f32x4 (&fn)[RMAX / 4], int lane, int out, const Lev &c0, int Wn,
                                          float lam, float om, float aS, int ce) {
    constexpr bool REC = MODE == BWD_UPDATE_REC, UPD = MODE == BWD_UPDATE || REC, MM = MODE == BWD_MM;
    constexpr bool NEEDF = UPD || MM, BAR = MODE == BWD_EN_BAR || MM || MODE == BWD_STORE_BAR;
    constexpr bool STOREB = UPD || MODE == BWD_STORE || MODE == BWD_STORE_BAR;
    constexpr int QM = RMAX / 4;
    const int l16 = lane16(lane);
    u32x4 t[Q];
    f32x4 b0[Q], b1[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) t[q] = tp[q];
    const int rem = c0.W - (Q - 1) * 256 - lane * 4;
    const uint32_t dead = (uint32_t)Wn | ((uint32_t)Wn << 16);
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (j >= rem) t[Q - 1][j] = dead;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            b0[q][j] = bn[(int)(t[q][j] & 0xFFFFu)];
            b1[q][j] = bn[(int)(t[q][j] >> 16)];
        }
    const float lam_use = BAR ? lam + aS : lam;
    float lam_new = lam_use;
    if (NEEDF) {
        float m0 = kInf, m1 = kInf;
        int k0 = INT_MAX, k1 = INT_MAX, h0 = 0, h1 = 0;  // recording: first node attaining the lane's min
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float v0 = fn[q][j] + b0[q][j], v1 = fn[q][j] + b1[q][j];
                if (REC) argmin_step(v0, m0, q * 256 + (l16 >> 2) + j, (int)(t[q][j] & 0xFFFFu), k0, h0);
                if (REC) argmin_step(v1, m1, q * 256 + (l16 >> 2) + j, (int)(t[q][j] >> 16), k1, h1);
                m0 = fminf(m0, v0);
                m1 = fminf(m1, v1);
            }
        const float lm0 = m0, lm1 = m1;
        m0 = team_min<64>(m0);
        m1 = team_min<64>(m1);
        const float M1 = m1;
        m1 += lam_use;
        if (UPD) {
            const float d = m1 - m0;
            const float Mn = om * d;
            lam_new = lam - Mn + aS;
            st1(lam_r, out, lam_new);
            st1(M_r, out, Mn);
            if (REC) record_argmins(rec_r, md_r, out, lm0, m0, k0, h0, lm1, M1, k1, h1, d);
        } else if (lane == 0) {
            T.out0[ce] = m0;
            T.out1[ce] = m1;
        }
    }
    f32x4 bv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[q][j] = fminf(b0[q][j], lam_new + b1[q][j]);
        lds4(bc, l16 + q * 1024) = bv[q];
    }
    if (lane == 0) {
        bc[c0.W] = kInf;
        bc[c0.W + 1] = 0.f;
    }
    if (STOREB) {
        // groups past the level fall outside Br and are dropped: the same stores on every path
        const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < QM; ++q) st4(Br, l16 + q * 1024, q < Q ? bv[q < Q ? q : 0] : z);
    }
    if constexpr (REC || MODE == BWD_STORE || MODE == BWD_STORE_BAR) {
        // the arc each node's B went through (the pull sweeps' argmin child: lo on ties), as
        // child code | beta << 15; dropped when the codes are not recorded (Cr of no size)
        const int l8 = lane8(lane);
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            uint32_t c[4] = {0u, 0u, 0u, 0u};
            if (q < Q)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int qq = q < Q ? q : 0;
                    const bool hi = lam_new + b1[qq][j] < b0[qq][j];
                    c[j] = hi ? ((t[qq][j] >> 16) | 0x8000u) : (t[qq][j] & 0xFFFFu);
                }
            st2(Cr, l8 + q * 512, c[0] | (c[1] << 16), c[2] | (c[3] << 16));
        }
    }
}

template <int RMAX, int MODE, bool LOOP>
__global__ __launch_bounds__(256) void k_bwd_w(DevTables T, int64_t tile0, int64_t ntiles, int NL) {
    constexpr bool REC = MODE == BWD_UPDATE_REC, UPD = MODE == BWD_UPDATE || REC, MM = MODE == BWD_MM;
    constexpr bool NEEDF = UPD || MM, BAR = MODE == BWD_EN_BAR || MM || MODE == BWD_STORE_BAR;
    constexpr int NB = node_buf_w(RMAX), QM = RMAX / 4;
    extern __shared__ float lds_f[];
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    int64_t tile = tile0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= tile0 + ntiles) return;
    // one node buffer: a hop reads every child's B before it writes its own level's, in order, so
    // B of level l replaces B of level l+1 in place (the terminals go after the level's width)
    float *buf0 = lds_f + (size_t)wave * lds_words_bwd_w(RMAX, NL);
    int *meta = (int *)(buf0 + NB);
    int *off = meta + NL;
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
    for (;;) {
        const TileCtx tc = tile_ctx(T, tile);
        const int row = T.bdd[tile * 64];
        preload_meta<1>(T, tc, lane, meta, off);
        const int nlev = tc.nlev;
        auto level = [&](int l) {
            Lev v{0, 0, 0};
            if (l >= 0 && l < nlev) {
                v.W = uni(meta[l] & 0xFFFF);
                v.R = uni(meta[l] >> 16);
                v.base = tc.nbase + (int64_t)uni(off[l]);
            }
            return v;
        };
        const rsrc_t lam_r = buf(T.lam + tc.ebase, nlev * 4), M_r = buf(T.M + tc.ebase, nlev * 4);
        const rsrc_t rec_r = rec_buf<REC>(T, tc, nlev), md_r = mdiff_buf<REC>(T, tc, nlev);
        const int out0 = lane * nlev * 4;  // hop l stores at out0 + 4 l: in range for lane 0 only
        Lev c0 = level(nlev - 1), cp = level(nlev - 2);  // levels l, l-1
        int Wn = 0;                                       // width of level l+1 (none below the last)
        // byte codes of the level's topology (prefetched one hop ahead) and the child codes they
        // decode to (decoded at the end of the hop before, while its LDS stores complete)
        uint32_t cwn[QM], cbn = T.lev_code[tc.lbase + nlev - 1];
        u32x4 tpn[QM];
        f32x4 fn[QM];
        // decode the prefetched codes of level c (whose next level has Wc nodes) into tpn
        auto decode = [&](const Lev &c, int Wc) {
            const rsrc_t traw = buf(T.topo + c.base, row_bytes(c));
            const uint32_t cb = uni((int)cbn);
            with_count<1, QM>(groups(c), [&](auto qc) {
                constexpr int QQ = decltype(qc)::value;
                u32x4 t[QQ];
                child_codes<QQ>(cwn, cb, Wc == 0, traw, lane, t);
#pragma unroll
                for (int q = 0; q < QQ; ++q) tpn[q] = t[q];
            });
        };
        {
            const int l16 = lane16(lane);
            const rsrc_t cr = buf(T.tcode + c0.base, code_row_bytes(c0)), fr = buf(T.F + c0.base, row_bytes(c0));
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                cwn[q] = ld1(cr, lane * 4 + q * 256);
                fn[q] = NEEDF ? ld4f(fr, l16 + q * 1024) : zero4;
            }
        }
        decode(c0, 0);
        const int et = tc.ebase + nlev - 1;
        float lamn = T.lam[et], aSn = (UPD || BAR) ? T.aS[et] : 0.f, omn = UPD ? T.omega[et] : 0.f;
        int cen = MM ? T.slot2canon[et] : 0;  // canonical edge of the min-marginals
        if (lane == 0) {  // below the last level: the terminals alone
            buf0[0] = kInf;
            buf0[1] = 0.f;
        }
        wave_sync();
        for (int l = nlev - 1; l >= 0; --l) {
            const float lam = lamn, om = omn, aS = aSn;
            const int ce = cen;
            u32x4 tp[QM];
            f32x4 fv[QM];
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                tp[q] = tpn[q];
                fv[q] = fn[q];
            }
            const float *bn = buf0;
            float *bc = buf0;
            // prefetch level l-1 (the first level reloads its own edge data)
            {
                const int l16 = lane16(lane);
                const rsrc_t cr = buf(T.tcode + cp.base, code_row_bytes(cp)), fr = buf(T.F + cp.base, row_bytes(cp));
#pragma unroll
                for (int q = 0; q < QM; ++q) {
                    cwn[q] = ld1(cr, lane * 4 + q * 256);
                    if (NEEDF) fn[q] = ld4f(fr, l16 + q * 1024);
                }
                cbn = T.lev_code[tc.lbase + max(l - 1, 0)];
                const int e = tc.ebase + max(l - 1, 0);
                lamn = T.lam[e];
                if (UPD || BAR) aSn = T.aS[e];
                if (UPD) omn = T.omega[e];
                if (MM) cen = T.slot2canon[e];
            }
            const rsrc_t Br = buf(T.B + c0.base, node_bytes(c0));
            const rsrc_t Cr = buf(T.Bch ? (const void *)(T.Bch + c0.base) : (const void *)T.B,
                                  T.Bch ? code_bytes(c0) : 0);  // no codes recorded: every store dropped
            with_count<1, QM>(groups(c0), [&](auto qc) {
                bwd_hop_w<decltype(qc)::value, RMAX, MODE>(T, Br, Cr, lam_r, M_r, rec_r, md_r, bn, bc, tp, fv, lane,
                                                           out0 + 4 * l, c0, Wn, lam, om, aS, ce);
            });
            if (l > 0) decode(cp, c0.W);
            wave_sync();
            
            Wn = c0.W;
            c0 = cp;
            cp = level(l - 2);
        }
        if (!MM && lane == 0 && row >= 0) {
            const float e0 = buf0[0];  // B(root) = E^j at the multipliers swept
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

template <int RMAX>
hipError_t fwd_dispatch_w(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s) {
    // the recording sweeps need a node buffer more per wave: at most the waves per workgroup of the
    // push-form adjoint sweep, whose LDS per wave is larger still
    const bool par = mode == FWD_UPDATE_REC || mode == FWD_SWEEP_LAM;
    const int wpb = par ? std::min(c.wpb_f, c.wpb_af) : c.wpb_f;
    const unsigned full = full_grid(c.ntiles, wpb);
    dim3 grid(full), block(64 * wpb);
    size_t lds = (size_t)wpb * (par ? lds_words_pass_w_par(RMAX, c.NL) : lds_words_pass_w(RMAX, c.NL)) * 4;
    if (mode == FWD_UPDATE && c.grid_f > 0 && (unsigned)c.grid_f < full)
        hipLaunchKernelGGL((k_fwd_w<RMAX, FWD_UPDATE, true>), dim3(c.grid_f), block, lds, s, t, c.tile0, c.ntiles, c.NL);
    else if (mode == FWD_UPDATE)
        hipLaunchKernelGGL((k_fwd_w<RMAX, FWD_UPDATE, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.NL);
    else if (mode == FWD_UPDATE_REC)
        hipLaunchKernelGGL((k_fwd_w<RMAX, FWD_UPDATE_REC, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.NL);
    else if (mode == FWD_SWEEP_BAR)
        hipLaunchKernelGGL((k_fwd_w<RMAX, FWD_SWEEP_BAR, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.NL);
    else
        hipLaunchKernelGGL((k_fwd_w<RMAX, FWD_SWEEP_LAM, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.NL);
    return hipGetLastError();
}

template <int RMAX>
hipError_t bwd_dispatch_w(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s) {
    const unsigned full = full_grid(c.ntiles, c.wpb_b);
    dim3 grid(full), block(64 * c.wpb_b);
    size_t lds = (size_t)c.wpb_b * lds_words_bwd_w(RMAX, c.NL) * 4;
    if (mode == BWD_UPDATE && c.grid_b > 0 && (unsigned)c.grid_b < full) {
        hipLaunchKernelGGL((k_bwd_w<RMAX, BWD_UPDATE, true>), dim3(c.grid_b), block, lds, s, t, c.tile0, c.ntiles, c.NL);
        return hipGetLastError();
    }
    switch (mode) {
        case BWD_UPDATE: hipLaunchKernelGGL((k_bwd_w<RMAX, BWD_UPDATE, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.NL); break;
        case BWD_UPDATE_REC: hipLaunchKernelGGL((k_bwd_w<RMAX, BWD_UPDATE_REC, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.NL); break;
        case BWD_STORE: hipLaunchKernelGGL((k_bwd_w<RMAX, BWD_STORE, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.NL); break;
        case BWD_EN_LAM: hipLaunchKernelGGL((k_bwd_w<RMAX, BWD_EN_LAM, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.NL); break;
        case BWD_EN_BAR: hipLaunchKernelGGL((k_bwd_w<RMAX, BWD_EN_BAR, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.NL); break;
        case BWD_STORE_BAR: hipLaunchKernelGGL((k_bwd_w<RMAX, BWD_STORE_BAR, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.NL); break;
        default: hipLaunchKernelGGL((k_bwd_w<RMAX, BWD_MM, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.NL); break;
    }
    return hipGetLastError();
}

template <int P, int RMAX>
hipError_t fwd_dispatch_g(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s) {
    const unsigned full = full_grid(c.ntiles, c.wpb_f);
    dim3 grid(full), block(64 * c.wpb_f);
    size_t lds = (size_t)c.wpb_f * lds_words_pass(P, c.WB, c.NL) * 4;
    auto update = [&](auto fas) {
        constexpr bool F = decltype(fas)::value;
        if (mode == FWD_UPDATE && c.grid_f > 0 && (unsigned)c.grid_f < full)
            hipLaunchKernelGGL((k_fwd<P, RMAX, FWD_UPDATE, true, F>), dim3(c.grid_f), block, lds, s, t, c.tile0,
                               c.ntiles, c.WB, c.NL);
        else if (mode == FWD_UPDATE)
            hipLaunchKernelGGL((k_fwd<P, RMAX, FWD_UPDATE, false, F>), grid, block, lds, s, t, c.tile0, c.ntiles,
                               c.WB, c.NL);
        else
            hipLaunchKernelGGL((k_fwd<P, RMAX, FWD_UPDATE_REC, false, F>), grid, block, lds, s, t, c.tile0, c.ntiles,
                               c.WB, c.NL);
    };
    if (mode == FWD_UPDATE || mode == FWD_UPDATE_REC) {
        if (t.form_as) update(std::true_type{});
        else update(std::false_type{});
    } else if (mode == FWD_SWEEP_BAR) {
        hipLaunchKernelGGL((k_fwd<P, RMAX, FWD_SWEEP_BAR, false, false>), grid, block, lds, s, t, c.tile0, c.ntiles,
                           c.WB, c.NL);
    } else {
        hipLaunchKernelGGL((k_fwd<P, RMAX, FWD_SWEEP_LAM, false, false>), grid, block, lds, s, t, c.tile0, c.ntiles,
                           c.WB, c.NL);
    }
    return hipGetLastError();
}

template <int P, int RMAX>
hipError_t bwd_dispatch_g(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s) {
    const unsigned full = full_grid(c.ntiles, c.wpb_b);
    dim3 grid(full), block(64 * c.wpb_b);
    size_t lds = (size_t)c.wpb_b * lds_words_pass(P, c.WB, c.NL) * 4;
    auto update = [&](auto fas) {
        constexpr bool F = decltype(fas)::value;
        if (mode == BWD_UPDATE && c.grid_b > 0 && (unsigned)c.grid_b < full)
            hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_UPDATE, true, F>), dim3(c.grid_b), block, lds, s, t, c.tile0,
                               c.ntiles, c.WB, c.NL);
        else if (mode == BWD_UPDATE)
            hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_UPDATE, false, F>), grid, block, lds, s, t, c.tile0, c.ntiles,
                               c.WB, c.NL);
        else
            hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_UPDATE_REC, false, F>), grid, block, lds, s, t, c.tile0, c.ntiles,
                               c.WB, c.NL);
    };
    switch (mode) {
        case BWD_UPDATE:
        case BWD_UPDATE_REC:
            if (t.form_as) update(std::true_type{});
            else update(std::false_type{});
            break;
        case BWD_STORE: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_STORE, false, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WB, c.NL); break;
        case BWD_EN_LAM: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_EN_LAM, false, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WB, c.NL); break;
        case BWD_EN_BAR: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_EN_BAR, false, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WB, c.NL); break;
        case BWD_STORE_BAR: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_STORE_BAR, false, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WB, c.NL); break;
        default: hipLaunchKernelGGL((k_bwd<P, RMAX, BWD_MM, false, false>), grid, block, lds, s, t, c.tile0, c.ntiles, c.WB, c.NL); break;
    }
    return hipGetLastError();
}


template <int P, int RMAX>
hipError_t fwd_dispatch(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s) {
    if (c.wpb_f < 1 || c.wpb_f > kMaxWavesPerBlock) return hipErrorInvalidConfiguration;
    if constexpr (P == 64) return fwd_dispatch_w<RMAX>(t, c, mode, s);
    else return fwd_dispatch_g<P, RMAX>(t, c, mode, s);
}

template <int P, int RMAX>
hipError_t bwd_dispatch(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s) {
    if (c.wpb_b < 1 || c.wpb_b > kMaxWavesPerBlock) return hipErrorInvalidConfiguration;
    if constexpr (P == 64) return bwd_dispatch_w<RMAX>(t, c, mode, s);
    else return bwd_dispatch_g<P, RMAX>(t, c, mode, s);
}


// S_i = sum of M over the edges of variable i.  TS lanes per variable (a power of two, fixed for an
// instance): lane u adds edges u, u + TS, ... of the variable in CSR order, then a fixed butterfly
// adds the TS partial sums, so S has the same bits on every call (TS = 1: one serial sum).  Teams
// keep the chain of dependent loads short for variables in many rows.  Blocks take the variables in
// plain order: the work per variable is skewed, and ranges per XCD (by count or by edges) piled an
// instance's long variables onto a few XCDs.
template <int TS>
__global__ void k_deferred_sum(const int32_t *__restrict__ var_ptr, const int32_t *__restrict__ var_slots,
                               const float *__restrict__ M, float *__restrict__ S, int n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t / TS), u = (int)(t % TS);
    const int a = i < n ? var_ptr[i] : 0, b = i < n ? var_ptr[i + 1] : 0;
    float s = strided_gather_sum<TS>(var_slots, M, a, b, u);
    for (int w = TS / 2; w > 0; w >>= 1) s += __shfl_xor(s, w, TS);  // every lane takes part
    if (i < n && u == 0) S[i] = s;
}

// aS[slot] = alpha[slot] * S[var(slot)] over all edge slots (padding slots have var -1).  A
// workgroup takes kSlotsPerThread * 256 consecutive slots, a thread every 256th of them: it issues
// all of its variable loads, then all of its S gathers, so one round trip of each serves four slots
// (a gather per thread left every wave waiting for two dependent round trips per slot).
__global__ __launch_bounds__(256) void k_edge_alpha_s(const int32_t *__restrict__ evar,
                                                      const float *__restrict__ alpha,
                                                      const float *__restrict__ S, float *__restrict__ aS,
                                                      float *__restrict__ Se, int64_t slots) {
    constexpr int K = kSlotsPerThread;
    const int64_t e0 = xcd_block(blockIdx.x, gridDim.x) * (256 * K) + threadIdx.x;
    int v[K];
    float a[K], sv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t e = e0 + 256 * k;
        v[k] = e < slots ? evar[e] : -1;
        a[k] = e < slots ? alpha[e] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) sv[k] = v[k] >= 0 ? S[v[k]] : 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t e = e0 + 256 * k;
        if (e < slots) {
            aS[e] = v[k] >= 0 ? a[k] * sv[k] : 0.f;
            if (Se) Se[e] = sv[k];
        }
    }
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

// two same-length copies in one launch (a solver state: multipliers and M)
__global__ void k_copy2(const float *__restrict__ a, float *__restrict__ ad, const float *__restrict__ b,
                        float *__restrict__ bd, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        ad[i] = a[i];
        bd[i] = b[i];
    }
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

__global__ __launch_bounds__(256) void k_sum_final(const double *__restrict__ partial, int nb, double add,
                                                   double *out) {
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
    if (t == 0) *out = sh[0] + add;
}

// Order-independent 64-bit fingerprint of a state (two float arrays a, b of n entries): the 32-bit
// pattern of word w (a[i] is word 2i, b[i] word 2i + 1) is keyed with w and mixed by the splitmix64
// finalizer (Steele, Lea and Flood, 2014), and the results are added modulo 2^64 -- the same sum in
// any order, so blocks may add their chunks separately and one block add the partial sums.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_hash_partial(const float *__restrict__ a, const float *__restrict__ b,
                                                      int64_t n, int64_t chunk, uint64_t *partial) {
    __shared__ uint64_t sh[256];
    const int t = threadIdx.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    uint64_t acc = 0;
    for (int64_t i = lo + t; i < hi; i += 256) {
        acc += mix64(((uint64_t)(2 * i) << 32 | __float_as_uint(a[i])) + 0x9E3779B97F4A7C15ull);
        acc += mix64(((uint64_t)(2 * i + 1) << 32 | __float_as_uint(b[i])) + 0x9E3779B97F4A7C15ull);
    }
    sh[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_hash_final(const uint64_t *__restrict__ partial, int nb, uint64_t *out) {
    __shared__ uint64_t sh[256];
    const int t = threadIdx.x;
    uint64_t acc = 0;
    for (int j = t; j < nb; j += 256) acc += partial[j];
    sh[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) *out = sh[0];
}

__global__ void k_hash_check(const uint64_t *__restrict__ x, const uint64_t *__restrict__ y, int32_t *flag) {
    if (threadIdx.x == 0 && *x != *y) *flag = 1;
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
    const size_t lds = (size_t)wpb * lds_words_pass_c(P, RMAX, c.WB, c.NL) * 4;
    if constexpr (P == 64) {
        const hipError_t e =
            fwd ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &nb, reinterpret_cast<const void *>(&k_fwd_w<RMAX, FWD_UPDATE, true>), 64 * wpb, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &nb, reinterpret_cast<const void *>(&k_bwd_w<RMAX, BWD_UPDATE, true>), 64 * wpb, lds);
        return e == hipSuccess ? nb : 0;
    } else {
        const hipError_t e =
            fwd ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &nb, reinterpret_cast<const void *>(&k_fwd<P, RMAX, FWD_UPDATE, true, true>), 64 * wpb, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &nb, reinterpret_cast<const void *>(&k_bwd<P, RMAX, BWD_UPDATE, true, true>), 64 * wpb, lds);
        return e == hipSuccess ? nb : 0;
    }
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
                               int team, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = blocks_for((int64_t)n * team, 256);
    switch (team) {
        case 1: hipLaunchKernelGGL(k_deferred_sum<1>, dim3(nb), dim3(256), 0, s, var_ptr, var_slots, M, S, n); break;
        case 2: hipLaunchKernelGGL(k_deferred_sum<2>, dim3(nb), dim3(256), 0, s, var_ptr, var_slots, M, S, n); break;
        case 4: hipLaunchKernelGGL(k_deferred_sum<4>, dim3(nb), dim3(256), 0, s, var_ptr, var_slots, M, S, n); break;
        case 8: hipLaunchKernelGGL(k_deferred_sum<8>, dim3(nb), dim3(256), 0, s, var_ptr, var_slots, M, S, n); break;
        case 16: hipLaunchKernelGGL(k_deferred_sum<16>, dim3(nb), dim3(256), 0, s, var_ptr, var_slots, M, S, n); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_edge_alpha_s(const int32_t *evar, const float *alpha, const float *S, float *aS, float *Se,
                               int64_t slots, hipStream_t s) {
    if (slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_edge_alpha_s, dim3(xcd_grid(blocks_for(slots, 256 * kSlotsPerThread))), dim3(256), 0, s, evar,
                       alpha, S, aS, Se,
                       slots);
    return hipGetLastError();
}

hipError_t launch_init_lambda(const int32_t *canon2slot, const int32_t *evar, const int32_t *var_ptr, const float *c,
                              float *lam, float *M, int64_t E, hipStream_t s) {
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_lambda, dim3(blocks_for(E, 256)), dim3(256), 0, s, canon2slot, evar, var_ptr, c, lam, M, E);
    return hipGetLastError();
}

hipError_t launch_copy2(const float *a, float *ad, const float *b, float *bd, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = std::min<unsigned>(blocks_for(n, 256), 8192u);
    hipLaunchKernelGGL(k_copy2, dim3(nb), dim3(256), 0, s, a, ad, b, bd, n);
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

hipError_t launch_sum(const float *x, int64_t n, int neg_part, double *partial, double *out, hipStream_t s,
                      double add) {
    const int nb = (int)std::min<int64_t>(kSumBlocks, std::max<int64_t>(1, (n + 4095) / 4096));
    const int64_t chunk = (std::max<int64_t>(n, 1) + nb - 1) / nb;
    hipLaunchKernelGGL(k_sum_partial, dim3(nb), dim3(256), 0, s, x, n, chunk, neg_part, partial);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partial, nb, add, out);
    return hipGetLastError();
}

hipError_t launch_state_hash(const float *a, const float *b, int64_t n, uint64_t *partial, uint64_t *out,
                             hipStream_t s) {
    const int nb = (int)std::min<int64_t>(kSumBlocks, std::max<int64_t>(1, (n + 4095) / 4096));
    const int64_t chunk = (std::max<int64_t>(n, 1) + nb - 1) / nb;
    hipLaunchKernelGGL(k_hash_partial, dim3(nb), dim3(256), 0, s, a, b, n, chunk, partial);
    hipLaunchKernelGGL(k_hash_final, dim3(1), dim3(256), 0, s, partial, nb, out);
    return hipGetLastError();
}

hipError_t launch_hash_check(const uint64_t *x, const uint64_t *y, int32_t *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_hash_check, dim3(1), dim3(64), 0, s, x, y, flag);
    return hipGetLastError();
}

hipError_t launch_check_params(const float *omega, const float *alpha, int64_t E, int32_t *flags, hipStream_t s) {
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_params, dim3(blocks_for(E, 256)), dim3(256), 0, s, omega, alpha, E, flags);
    return hipGetLastError();
}

}  // namespace dd
