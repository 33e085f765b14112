// adjoint.hip -- reverse mode of the dual iteration (Alg. 2, Prop. 2) on CDNA4 (gfx950).
//
// One pass of Alg. 1 on a diagram, seen as a computation graph (forward pass shown; the
// backward pass is its mirror image): B_{l+1} from the pass-input multipliers, then per hop l
//     m^beta_l = min_v F_l(v) + beta*lambda_l + B_{l+1}(child_beta v)           (eq. 8)
//     M_l = omega_l (m^1_l - m^0_l),  lambda'_l = lambda_l - M_l + alpha_l S_i    (Alg. 1)
//     F_{l+1}(w) = min over arcs (v, beta) -> w of F_l(v) + beta*lambda'_l.
// Reverse mode replaces every min by its argmin (App. B, backpropagation paragraph):
//   * the "update side" (F for a forward pass) is swept against the pass order and carries
//     the BlockUpdate adjoint of Alg. 2 at each hop: lambda'-dot collects the adjoint of the
//     hi arcs that won a min of the next level, dM = dM_out - dlambda', d_omega += dM (m1 - m0),
//     d_alpha += dlambda' S, dm^1 = omega dM = -dm^0 routed to the argmin node of each
//     min-marginal and to its child on the other side;
//   * the "fixed side" (B for a forward pass, computed from the pass-input multipliers) is swept
//     afterwards and routes what reached it to the pass-input multipliers.
// Minimum propagation comes in two forms: pull (B_l(v) = min over its two children: each node
// picks its argmin child, lo on ties) and push (F_{l+1}(w) = min over its parents: every
// parent arc whose value equals F_{l+1}(w) bids with (node index, lo before hi) in LDS and the
// lowest bid wins, so each minimum has exactly one argmin).  Argmin tests are exact float
// equalities: the stored costs and the recomputed candidates come from the same expressions.
// The argmin nodes of each hop's two min-marginals (lowest index on ties), their children and
// m^1 - m^0 are recorded by the update pass that the sweeps reverse (its recording variant).
// Contributions from one sweep to the other side travel as per-edge records
// (two node indices, two values), not as a dense per-node array.
#include <hip/hip_runtime.h>

#include <climits>
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"

namespace dd {
namespace {

using namespace dev;

// Per-edge inputs of one hop, loaded one hop ahead.  Update sweeps: the multiplier after the
// pass (lam_use), the output adjoints, omega, alpha, S of the variable, the d_alpha / d_omega
// accumulated so far, and the pass's argmin records.  Fixed sweeps: the multiplier the side was
// computed with, the dlambda_in accumulated by the update sweep, and the record (two node
// indices and adjoints) handed over by the update sweep.
struct AdjEdge {
    float lam_use, dlo, dMo, om, al, S, da, dw;
    float dl;
    int i0, i1;
    float v0, v1;
    uint32_t kc0, kc1;  // update sweeps: the pass's argmin node of m^0 | its lo child << 16, same for m^1 / hi
    float d;            // and m^1 - m^0 as the pass formed it
};

template <bool UPD>
__device__ __forceinline__ AdjEdge adj_edge(const DevTables &T, const AdjTables &A, int e, bool bar, bool rec) {
    AdjEdge x{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, -1, -1, 0.f, 0.f, 0u, 0u, 0.f};
    if (UPD) {
        x.lam_use = T.lam[e];
        x.dlo = A.dlam_out[e];
        x.dMo = A.dM_out[e];
        x.om = T.omega[e];
        x.al = T.alpha[e];
        x.S = A.Se[e];
        x.da = A.dalpha[e];
        x.dw = A.domega[e];
        x.kc0 = (uint32_t)A.mrec[2 * e];
        x.kc1 = (uint32_t)A.mrec[2 * e + 1];
        x.d = A.mdiff[e];
    } else {
        x.lam_use = A.lam_src[e];
        if (bar) x.lam_use = x.lam_use + T.aS[e];
        x.dl = A.dlam_in[e];
        if (rec) {
            x.i0 = A.rec_idx[2 * e];
            x.i1 = A.rec_idx[2 * e + 1];
            x.v0 = A.rec_val[2 * e];
            x.v1 = A.rec_val[2 * e + 1];
        }
    }
    return x;
}

// ------------------------------------------------------------------------------------------
// Push-form sweep (F side), against the level order: l = L-1 .. 0.  Every global operand of
// hop l-1 (topology, F of level l-1, edge data) is loaded during hop l; the update sweep takes
// the hop's argmins from the pass's records.
// LDS per wave: Fv, Fa (cost and adjoint of level l+1, overwritten by level l at the end of
// the hop), bid (ints), then the level table.
// ------------------------------------------------------------------------------------------
template <int P, int RMAX, bool UPD>
// (the fixed-side variant is asked for 3 waves per SIMD: measured faster; the update variant would spill)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(!UPD && RMAX <= 16 ? 3 : 1))) void k_adj_F(
    DevTables T, AdjTables A, int64_t tile0, int64_t ntiles, int WB, int NL) {
    constexpr int G = 64 / P;
    extern __shared__ float lds_f[];
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int g = lane / P, p = lane % P;
    const int64_t tile = tile0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= tile0 + ntiles) return;
    float *Fv = lds_f + (size_t)wave * lds_words_adj_F(P, WB, NL);
    float *Fa = Fv + WB * G;
    int *bid = (int *)(Fa + WB * G);
    int *meta = bid + WB * G;
    int *off = meta + NL * G;
    const TileCtx tc = tile_ctx(T, tile);
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
    Lev c0 = level(nlev - 1), c1{0, 0, 0};  // levels l and l+1 (terminals only below the last level)
    uint32_t tpn[RMAX];
    float fvn[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
        tpn[r] = r < c0.R ? T.topo[c0.base + r * 64 + lane] : 0u;
        fvn[r] = r < c0.R ? T.F[c0.base + r * 64 + lane] : kInf;
    }
    AdjEdge xn = adj_edge<UPD>(T, A, tc.ebase + (nlev - 1) * G + g, false, true);
    for (int l = nlev - 1; l >= 0; --l) {
        const int Wn = c1.W;
        const int e = tc.ebase + l * G + g;
        const AdjEdge x = xn;
        uint32_t tp[RMAX];
        float fv[RMAX];
        const uint32_t dead = (uint32_t)Wn | ((uint32_t)Wn << 16);
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            tp[r] = tpn[r];
            fv[r] = fvn[r];
            if (r < c0.R && !in_level<P>(r, c0.R, lane, c0.W)) {
                tp[r] = dead;
                fv[r] = kInf;
            }
        }
        // prefetch hop l-1: topology and F of level l-1, edge data of level l-1. Rows past the level
        // load 0 without a memory access (no row past a level is read) and the last hop reloads its
        // own edge data: no branch, so no prefetched register is merged with its old value (a merge
        // would wait for the load right after issuing it).
        const Lev cp = level(l - 1);
        {
            const rsrc_t tr = buf(T.topo + cp.base, cp.R * 256), fr = buf(T.F + cp.base, cp.R * 256);
#pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                tpn[r] = ld1(tr, (r * 64 + lane) * 4);
                fvn[r] = ld1f(fr, (r * 64 + lane) * 4);
            }
        }
        xn = adj_edge<UPD>(T, A, tc.ebase + max(l - 1, 0) * G + g, false, true);
        wave_sync();
        // bids for the argmin parent arc of every node of level l+1
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            if (r < c0.R) {
                const int k = r * P + p, lo = (int)(tp[r] & 0xFFFFu), hi = (int)(tp[r] >> 16);
                if (lo < Wn && fv[r] == Fv[lo * G + g]) lds_imin(&bid[lo * G + g], 2 * k);
                if (hi < Wn && fv[r] + x.lam_use == Fv[hi * G + g]) lds_imin(&bid[hi * G + g], 2 * k + 1);
            }
        }
        wave_sync();
        float acc[RMAX];
        float hisum = 0.f;
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            acc[r] = 0.f;
            if (r < c0.R) {
                const int k = r * P + p, lo = (int)(tp[r] & 0xFFFFu), hi = (int)(tp[r] >> 16);
                if (lo < Wn && bid[lo * G + g] == 2 * k) acc[r] += Fa[lo * G + g];
                if (hi < Wn && bid[hi * G + g] == 2 * k + 1) {
                    const float c = Fa[hi * G + g];
                    acc[r] += c;
                    hisum += c;
                }
            }
        }
        hisum = team_sum<P>(hisum);
        if (UPD) {
            // the hop's argmin nodes of the two min-marginals and their children: the pass's records
            if (c0.W > 0) {
                const int k0 = (int)(x.kc0 & 0xFFFFu), k1 = (int)(x.kc1 & 0xFFFFu);
                const int ch0 = (int)(x.kc0 >> 16), ch1 = (int)(x.kc1 >> 16);
                const float dlam_new = x.dlo + hisum;
                const float dM = x.dMo - dlam_new;
                const float diff = x.d;  // m^1 - m^0 as the pass formed it
                const float dm1 = x.om * dM, dm0 = -dm1;
                if (p == 0) {
                    A.dlam_in[e] = dlam_new + dm1;  // identity path + the hi arc of m^1 itself
                    A.g[e] = dlam_new * x.al;
                    A.dalpha[e] = x.da + dlam_new * x.S;
                    A.domega[e] = x.dw + dM * diff;
                    A.rec_idx[2 * e] = ch0 < Wn ? ch0 : -1;
                    A.rec_idx[2 * e + 1] = ch1 < Wn ? ch1 : -1;
                    A.rec_val[2 * e] = dm0;
                    A.rec_val[2 * e + 1] = dm1;
                }
#pragma unroll
                for (int r = 0; r < RMAX; ++r) {
                    const int k = r * P + p;
                    if (k == k0) acc[r] += dm0;
                    if (k == k1) acc[r] += dm1;
                }
            }
        } else if (c0.W > 0) {
            if (p == 0) A.dlam_in[e] = x.dl + hisum;
            // argmin contributions of the update sweep to F_l (record of edge l)
#pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                const int k = r * P + p;
                if (k == x.i0) acc[r] += x.v0;
                if (k == x.i1) acc[r] += x.v1;
            }
        }
        wave_sync();  // level l+1 is fully read before level l replaces it
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            if (r < c0.R) {
                const int xi = mine + r * P * G;
                Fa[xi] = acc[r];
                Fv[xi] = fv[r];
                bid[xi] = INT_MAX;
            }
        }
        wave_sync();
        c1 = c0;
        c0 = cp;
    }
}

// ------------------------------------------------------------------------------------------
// Pull-form sweep (B side), along the level order: l = 0 .. L-1, with the operands of hop l+1
// (topology of level l+1, B of level l+2, edge data) loaded during hop l; the update sweep takes
// the hop's argmins from the pass's records.
// LDS per wave: Bst (B of level l+1), Ba[2] (adjoints of levels l / l+1), level table.
// seed != 0: the adjoint of B(root) is `seed` (the lower bound's own gradient).
// ------------------------------------------------------------------------------------------
template <int P, int RMAX, bool UPD>
__global__ __launch_bounds__(256) void k_adj_B(DevTables T, AdjTables A, int64_t tile0, int64_t ntiles, int WB,
                                               int NL, int bar, int recs, float seed) {
    constexpr int G = 64 / P;
    extern __shared__ float lds_f[];
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int g = lane / P, p = lane % P;
    const int64_t tile = tile0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= tile0 + ntiles) return;
    float *Bst = lds_f + (size_t)wave * lds_words_adj_B(P, WB, NL);
    float *Ba = Bst + WB * G;
    int *meta = (int *)(Ba + 2 * WB * G);
    int *off = meta + NL * G;
    const TileCtx tc = tile_ctx(T, tile);
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
    int cur = 0;  // Ba[cur]: level l
    {
        const int R0 = uni(meta[0] >> 16);
        for (int r = 0; r < R0; ++r) Ba[mine + r * P * G] = 0.f;
        if (p == 0) Ba[g] = A.seed ? *A.seed : seed;  // the root is node 0 of level 0
    }
    Lev c0 = level(0), c1 = level(1);
    uint32_t tpn[RMAX];
    float bvn[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
        tpn[r] = r < c0.R ? T.topo[c0.base + r * 64 + lane] : 0u;
        bvn[r] = r < c1.R ? T.B[c1.base + r * 64 + lane] : 0.f;
    }
    AdjEdge xn = adj_edge<UPD>(T, A, tc.ebase + g, bar != 0, false);
    // record of the previous hop's edge (fixed sweeps): read through a resource over the tile's
    // edges, past it for teams with no node at that level; prec says whether there is one
    const int ne8 = recs ? nlev * G * 8 : 0;
    const rsrc_t ri = buf(recs ? (const void *)(A.rec_idx + 2 * (int64_t)tc.ebase) : (const void *)A.dlam_in, ne8);
    const rsrc_t rv = buf(recs ? (const void *)(A.rec_val + 2 * (int64_t)tc.ebase) : (const void *)A.dlam_in, ne8);
    bool prec = false;
    int pi0 = -1, pi1 = -1;
    float pv0 = 0.f, pv1 = 0.f;
    for (int l = 0; l < nlev; ++l) {
        const int Wn = c1.W;
        const int e = tc.ebase + l * G + g;
        const AdjEdge x = xn;
        float *ba0 = Ba + cur * WB * G, *ba1 = Ba + (cur ^ 1) * WB * G;
        // fixed side: argmin contributions of the update sweep to B_l (record of edge l-1)
        if (!UPD && p == 0 && prec) {
            if (pi0 >= 0) ba0[pi0 * G + g] += pv0;
            if (pi1 >= 0) ba0[pi1 * G + g] += pv1;
        }
        uint32_t tp[RMAX];
        const uint32_t dead = (uint32_t)Wn | ((uint32_t)Wn << 16);
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            tp[r] = tpn[r];
            if (r < c0.R && !in_level<P>(r, c0.R, lane, c0.W)) tp[r] = dead;
            if (r < c1.R) {
                Bst[mine + r * P * G] = bvn[r];
                ba1[mine + r * P * G] = 0.f;
            }
        }
        if (p == 0) {
            Bst[Wn * G + g] = kInf;
            Bst[(Wn + 1) * G + g] = 0.f;
        }
        // prefetch hop l+1: topology of level l+1, B of level l+2, edge data of level l+1, the record
        // of edge l. Rows past a level load 0 without a memory access and the last hop reloads its
        // own edge data: no branch, so no prefetched register is merged with its old value.
        const Lev c2 = level(l + 2);
        {
            const rsrc_t tr = buf(T.topo + c1.base, c1.R * 256), br = buf(T.B + c2.base, c2.R * 256);
#pragma unroll
            for (int r = 0; r < RMAX; ++r) {
                tpn[r] = ld1(tr, (r * 64 + lane) * 4);
                bvn[r] = ld1f(br, (r * 64 + lane) * 4);
            }
        }
        xn = adj_edge<UPD>(T, A, tc.ebase + min(l + 1, nlev - 1) * G + g, bar != 0, false);
        if (!UPD) {
            prec = recs && c0.W > 0;
            const int o8 = c0.W > 0 ? (l * G + g) * 8 : ne8;
            pi0 = (int)ld1(ri, o8);
            pi1 = (int)ld1(ri, o8 + 4);
            pv0 = ld1f(rv, o8);
            pv1 = ld1f(rv, o8 + 4);
        }
        wave_sync();
        float hisum = 0.f;
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            if (r < c0.R) {
                const int lo = (int)(tp[r] & 0xFFFFu), hi = (int)(tp[r] >> 16);
                const float b0 = Bst[lo * G + g], b1 = x.lam_use + Bst[hi * G + g];
                const float d = ba0[mine + r * P * G];
                const bool take_hi = b1 < b0;  // the pass formed min(b0, b1): lo on ties
                const int ch = take_hi ? hi : lo;
                if (ch < Wn) lds_fadd(&ba1[ch * G + g], d);
                if (take_hi) hisum += d;
            }
        }
        hisum = team_sum<P>(hisum);
        if (UPD) {
            // the hop's argmin nodes of the two min-marginals: the pass's records
            const int k0 = (int)(x.kc0 & 0xFFFFu), k1 = (int)(x.kc1 & 0xFFFFu);
            if (c0.W > 0) {
                const float dlam_new = x.dlo + hisum;
                const float dM = x.dMo - dlam_new;
                const float diff = x.d;  // m^1 - m^0 as the pass formed it
                const float dm1 = x.om * dM, dm0 = -dm1;
#pragma unroll
                for (int r = 0; r < RMAX; ++r) {
                    if (r < c0.R) {
                        const int k = r * P + p;
                        const int lo = (int)(tp[r] & 0xFFFFu), hi = (int)(tp[r] >> 16);
                        if (k == k0 && lo < Wn) lds_fadd(&ba1[lo * G + g], dm0);
                        if (k == k1 && hi < Wn) lds_fadd(&ba1[hi * G + g], dm1);
                    }
                }
                if (p == 0) {
                    A.dlam_in[e] = dlam_new + dm1;
                    A.g[e] = dlam_new * x.al;
                    A.dalpha[e] = x.da + dlam_new * x.S;
                    A.domega[e] = x.dw + dM * diff;
                    A.rec_idx[2 * e] = k0;  // argmin nodes of level l: F_l side contributions
                    A.rec_idx[2 * e + 1] = k1;
                    A.rec_val[2 * e] = dm0;
                    A.rec_val[2 * e + 1] = dm1;
                }
            }
        } else if (c0.W > 0 && p == 0) {
            A.dlam_in[e] = x.dl + hisum;
        }
        wave_sync();
        cur ^= 1;
        c0 = c1;
        c1 = c2;
    }
}

// ------------------------------------------------------------------------------------------
// Pull-form sweep of one-wave diagrams (P = 64), laid out like the wide pass kernels: a lane
// owns nodes k = 256 q + 4 lane + j of level l (the node indices of the general sweep, so the
// argmin keys and the records are the same), rows move with one 16-byte access per lane through
// level-sized buffer resources, every prefetch is issued unconditionally, and each hop branches
// once on its group count.
// The adjoint of B lives on minimizing paths only: a node hands its whole adjoint to one child,
// and the update sweep adds two per level, so a level holds a handful of nonzero adjoints
// whatever its width.  A hop therefore first lists them (children and adjoint of each nonzero
// node, in wave order, written over the level's own adjoint buffer once it has been read) and
// routes the list with one lane per entry, instead of a routing step for every node.  A level
// whose nonzero adjoints overflow the list is routed node by node by the owning lanes.  The
// update sweep takes the hop's argmin nodes of the two min-marginals, their children and
// m^1 - m^0 from the records of the replayed (or stored) pass, so it reads no F at all.  Float
// sums (LDS adds, the hi-arc sum) may be added in another order than in the general sweep; the
// mins and the argmin tests are exact.
// ------------------------------------------------------------------------------------------
template <bool UPD>
struct AdjIn;
template <>
struct AdjIn<true> {  // multiplier after the pass, output adjoints, omega, alpha, S, sums, the pass's records
    float lam, dlo, dMo, om, al, S, da, dw;
    uint32_t kc0, kc1;  // argmin node of m^0 | its lo child << 16; the same for m^1 and the hi child
    float d;            // m^1 - m^0 as the pass formed it
};
template <>
struct AdjIn<false> {  // multiplier of the fixed side, alpha*S and dlambda_in so far
    float lam_src, aS, dl;
};

template <bool UPD>
__device__ __forceinline__ AdjIn<UPD> adj_in(const DevTables &T, const AdjTables &A, int e) {
    AdjIn<UPD> x;
    if constexpr (UPD) {
        x.lam = T.lam[e];
        x.dlo = A.dlam_out[e];
        x.dMo = A.dM_out[e];
        x.om = T.omega[e];
        x.al = T.alpha[e];
        x.S = A.Se[e];
        x.da = A.dalpha[e];
        x.dw = A.domega[e];
        x.kc0 = (uint32_t)A.mrec[2 * e];
        x.kc1 = (uint32_t)A.mrec[2 * e + 1];
        x.d = A.mdiff[e];
    } else {
        x.lam_src = A.lam_src[e];
        x.aS = T.aS[e];
        x.dl = A.dlam_in[e];
    }
    return x;
}

// Outputs of a hop, stored by lane 0 through resources over the tile's edges: hop l stores at
// o4 + 4 l (o8 + 8 l for the two-word records), past the resource for every other lane.
struct AdjOut {
    rsrc_t dlam_in, g, dalpha, domega, rec_idx, rec_val;
    int o4, o8;
};

template <bool UPD>
__device__ __forceinline__ AdjOut adj_out(const AdjTables &A, const TileCtx &tc, int nlev, int lane) {
    AdjOut o{};
    o.dlam_in = buf(A.dlam_in + tc.ebase, nlev * 4);
    if constexpr (UPD) {
        o.g = buf(A.g + tc.ebase, nlev * 4);
        o.dalpha = buf(A.dalpha + tc.ebase, nlev * 4);
        o.domega = buf(A.domega + tc.ebase, nlev * 4);
        o.rec_idx = buf(A.rec_idx + 2 * (int64_t)tc.ebase, nlev * 8);
        o.rec_val = buf(A.rec_val + 2 * (int64_t)tc.ebase, nlev * 8);
    }
    o.o4 = lane * nlev * 4;
    o.o8 = lane * nlev * 8;
    return o;
}

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

// lanes below this one whose bit is set in a wave mask
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <int Q, int RMAX, bool UPD>
__device__ __forceinline__ void adjB_hop_w(const float *Bst, float *ba0, float *ba1, const u32x4 (&tp)[RMAX / 4],
                                           int lane, const Lev &c0, int Wn, float lam_use, const AdjIn<UPD> &x,
                                           const AdjOut &o, int l, int cap) {
    constexpr int CAP = node_buf_w(RMAX) / 2;  // list entries that fit in a node buffer
    const int l16 = lane16(lane);
    u32x4 t[Q];
    f32x4 d[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        t[q] = tp[q];
        d[q] = lds4(ba0, l16 + q * 1024);  // slots past the level's width hold 0
    }
    // last group: this lane's slots past the level's width get two 0-terminal arcs
    const int rem = c0.W - (Q - 1) * 256 - lane * 4;
    const uint32_t dead = (uint32_t)Wn | ((uint32_t)Wn << 16);
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (j >= rem) t[Q - 1][j] = dead;
    wave_sync();  // every lane has read ba0: the list overwrites it
    // the level's nonzero adjoints: children at [0, CAP) and adjoint at [CAP, 2 CAP) of ba0
    uint32_t *lt = (uint32_t *)ba0;
    float *lv = ba0 + CAP;
    int n = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool nz = d[q][j] != 0.f;
            const uint64_t m = __builtin_amdgcn_ballot_w64(nz);
            const int pos = n + lanes_below(m);
            if (nz && pos < CAP) {
                lt[pos] = t[q][j];
                lv[pos] = d[q][j];
            }
            n += (int)__builtin_popcountll(m);
        }
    wave_sync();
    float hisum = 0.f;
    auto route = [&](uint32_t tt, float dv) {
        const int lo = (int)(tt & 0xFFFFu), hi = (int)(tt >> 16);
        const float b0 = Bst[lo], b1 = lam_use + Bst[hi];
        const bool take_hi = b1 < b0;  // the pass formed min(b0, b1): lo on ties
        const int ch = take_hi ? hi : lo;
        if (ch < Wn) lds_fadd(&ba1[ch], dv);
        if (take_hi) hisum += dv;
    };
    if (n <= min(cap, CAP)) {
        for (int c = 0; c < n; c += 64)
            if (c + lane < n) route(lt[c + lane], lv[c + lane]);
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (d[q][j] != 0.f) route(t[q][j], d[q][j]);
    }
    hisum = team_sum<64>(hisum);
    if constexpr (UPD) {
        // the pass's argmin nodes of the two min-marginals and their children (recorded)
        const int K0 = (int)(x.kc0 & 0xFFFFu), K1 = (int)(x.kc1 & 0xFFFFu);
        const int r0 = (int)(x.kc0 >> 16), r1 = (int)(x.kc1 >> 16);
        const float dlam_new = x.dlo + hisum;
        const float dM = x.dMo - dlam_new;
        const float dm1 = x.om * dM, dm0 = -dm1;
        wave_sync();  // after the routed adjoints (a fixed order of the float adds)
        if (lane == 0 && r0 < Wn) lds_fadd(&ba1[r0], dm0);
        if (lane == 0 && r1 < Wn) lds_fadd(&ba1[r1], dm1);
        st1(o.dlam_in, o.o4 + 4 * l, dlam_new + dm1);  // identity path + the hi arc of m^1 itself
        st1(o.g, o.o4 + 4 * l, dlam_new * x.al);
        st1(o.dalpha, o.o4 + 4 * l, x.da + dlam_new * x.S);
        st1(o.domega, o.o4 + 4 * l, x.dw + dM * x.d);
        st2(o.rec_idx, o.o8 + 8 * l, (uint32_t)K0, (uint32_t)K1);  // argmin nodes of level l: F_l side
        st2(o.rec_val, o.o8 + 8 * l, __float_as_uint(dm0), __float_as_uint(dm1));
    } else {
        st1(o.dlam_in, o.o4 + 4 * l, x.dl + hisum);
    }
}

template <int RMAX, bool UPD>
__global__ __launch_bounds__(256) void k_adj_B_w(DevTables T, AdjTables A, int64_t tile0, int64_t ntiles, int NL,
                                                 int bar, int recs, float seed, int cap) {
    constexpr int NB = node_buf_w(RMAX), QM = RMAX / 4;
    extern __shared__ float lds_f[];
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t tile = tile0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= tile0 + ntiles) return;  // uniform per wave
    float *Bst = lds_f + (size_t)wave * lds_words_adj_B_w(RMAX, NL);
    float *Ba = Bst + NB;
    int *meta = (int *)(Ba + 2 * NB);
    int *off = meta + NL;
    const TileCtx tc = tile_ctx(T, tile);
    preload_meta<1>(T, tc, lane, meta, off);
    const int nlev = tc.nlev;
    auto level = [&](int l) {
        Lev v{0, 0, 0};
        if (l < nlev) {
            v.W = uni(meta[l] & 0xFFFF);
            v.R = uni(meta[l] >> 16);
            v.base = tc.nbase + (int64_t)uni(off[l]);
        }
        return v;
    };
    const AdjOut o = adj_out<UPD>(A, tc, nlev, lane);
    // records of the update sweep (fixed sweeps with recs): a resource of no size otherwise
    const bool use_rec = !UPD && recs;
    const rsrc_t ri = buf(use_rec ? (const void *)(A.rec_idx + 2 * (int64_t)tc.ebase) : (const void *)A.dlam_in,
                          use_rec ? nlev * 8 : 0);
    const rsrc_t rv = buf(use_rec ? (const void *)(A.rec_val + 2 * (int64_t)tc.ebase) : (const void *)A.dlam_in,
                          use_rec ? nlev * 8 : 0);
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
    int cur = 0;  // Ba + cur * NB: adjoints of level l
    {
        const int l16 = lane16(lane);
#pragma unroll
        for (int q = 0; q < QM; ++q) lds4(Ba, l16 + q * 1024) = zero4;
        if (lane == 0) Ba[0] = A.seed ? *A.seed : seed;  // the root is node 0 of level 0
    }
    Lev c0 = level(0), c1 = level(1);
    u32x4 tpn[QM];
    f32x4 bvn[QM];
    {
        const int l16 = lane16(lane);
        const rsrc_t tr = buf(T.topo + c0.base, row_bytes(c0)), br = buf(T.B + c1.base, row_bytes(c1));
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            tpn[q] = ld4(tr, l16 + q * 1024);
            bvn[q] = ld4f(br, l16 + q * 1024);
        }
    }
    AdjIn<UPD> xn = adj_in<UPD>(T, A, tc.ebase);
    int pi0 = -1, pi1 = -1;  // record of the previous hop's edge (children at this level, or -1)
    float pv0 = 0.f, pv1 = 0.f;
    for (int l = 0; l < nlev; ++l) {
        const int Wn = c1.W;
        const AdjIn<UPD> x = xn;
        float *ba0 = Ba + cur * NB, *ba1 = Ba + (cur ^ 1) * NB;
        // fixed side: argmin contributions of the update sweep to B_l (record of edge l-1)
        if (use_rec && l > 0 && lane == 0) {
            if (pi0 >= 0) ba0[pi0] += pv0;
            if (pi1 >= 0) ba0[pi1] += pv1;
        }
        u32x4 tp[QM];
#pragma unroll
        for (int q = 0; q < QM; ++q) tp[q] = tpn[q];
        {
            // B of level l+1 with its terminals; the adjoints of level l+1 start at 0
            const int l16 = lane16(lane);
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                lds4(Bst, l16 + q * 1024) = bvn[q];
                lds4(ba1, l16 + q * 1024) = zero4;
            }
        }
        wave_sync();  // the terminals' slots may have been staged by another lane
        if (lane == 0) {
            Bst[Wn] = kInf;
            Bst[Wn + 1] = 0.f;
        }
        // prefetch hop l+1: topology of level l+1, B of level l+2, edge data of level l+1 (the
        // last hop reloads its own), the record of edge l
        const Lev c2 = level(l + 2);
        {
            const int l16 = lane16(lane);
            const rsrc_t tr = buf(T.topo + c1.base, row_bytes(c1)), br = buf(T.B + c2.base, row_bytes(c2));
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                tpn[q] = ld4(tr, l16 + q * 1024);
                bvn[q] = ld4f(br, l16 + q * 1024);
            }
            xn = adj_in<UPD>(T, A, tc.ebase + min(l + 1, nlev - 1));
            if (!UPD) {
                pi0 = (int)ld1(ri, 8 * l);
                pi1 = (int)ld1(ri, 8 * l + 4);
                pv0 = ld1f(rv, 8 * l);
                pv1 = ld1f(rv, 8 * l + 4);
            }
        }
        wave_sync();
        float lam_use;
        if constexpr (UPD) lam_use = x.lam;
        else lam_use = bar ? x.lam_src + x.aS : x.lam_src;
        with_count<1, QM>(groups(c0), [&](auto qc) {
            adjB_hop_w<decltype(qc)::value, RMAX, UPD>(Bst, ba0, ba1, tp, lane, c0, Wn, lam_use, x, o, l, cap);
        });
        wave_sync();
        cur ^= 1;
        c0 = c1;
        c1 = c2;
    }
}

// ------------------------------------------------------------------------------------------
// Push-form sweep of one-wave diagrams (P = 64), levels l = L-1 .. 0, in the wide layout.  The
// adjoint of F also lives on minimizing paths only (a node hands its adjoint to its argmin
// parent arc), but a node's parents are known only to the level above, so every arc of level l
// still looks up its child's adjoint; the few nodes with an arc into a nonzero one are listed
// (node, children, cost), and with one lane per entry, which reads its two child adjoints, their arcs bid
// 2k + beta for their child; a node's adjoint is the sum of the children it won.  A list that
// overflows is bid and collected by the owning lanes instead.  F and its adjoint have one buffer
// each: level l overwrites level l+1 once every value of level l+1 that the hop needs is read.  The update sweep takes the hop's argmin nodes, their children and
// m^1 - m^0 from the records of the replayed (or stored) pass, so it reads no B at all.
// LDS per wave: Fv, Fa (cost and adjoint), the bids (INT_MAX between hops: the bidding lanes clear
// what they set), the list, the level table.
// ------------------------------------------------------------------------------------------
template <bool UPD>
struct AdjInF;
template <>
struct AdjInF<true> {
    AdjIn<true> a;
};
template <>
struct AdjInF<false> {  // fixed side: the multiplier swept, dlambda_in so far, the update sweep's record
    float lam_src, dl;
    int i0, i1;
    float v0, v1;
};

template <int Q, int RMAX, bool UPD>
__device__ __forceinline__ void adjF_hop_w(float *Fv, float *Fa, int *bid, int *lk, uint32_t *lt, float *lf,
                                           const u32x4 (&tp)[RMAX / 4],
                                           const f32x4 (&fvi)[RMAX / 4], int lane,
                                           const Lev &c0, int Wn, float lam_use, const AdjInF<UPD> &x,
                                           const AdjOut &o, int l, int cap) {
    constexpr int CAP = kAdjListW;
    const int l16 = lane16(lane);
    u32x4 t[Q];
    f32x4 f[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        t[q] = tp[q];
        f[q] = fvi[q];
    }
    const int rem = c0.W - (Q - 1) * 256 - lane * 4;
    const uint32_t dead = (uint32_t)Wn | ((uint32_t)Wn << 16);
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (j >= rem) {
            t[Q - 1][j] = dead;
            f[Q - 1][j] = kInf;
        }
    // nodes with an arc into a child with a nonzero adjoint (terminal slots of Fa hold 0), in wave
    // order; the first CAP go to the list (node, children, cost); returns how many there are. Every
    // child adjoint is read first, in one straight run of LDS reads, and the list is built from the
    // flags after (a list write per node between the reads would make each read wait for the last).
    // The node values are taken afresh, so nothing derived from them is computed ahead and held in
    // registers.
    auto detect = [&]() {
        u32x4 tv[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            tv[q] = t[q];
            __asm__ volatile("" : "+v"(tv[q]));
        }
        // one flag per node of the lane: 4 Q bits (64-bit words for levels of more than 8 groups)
        using flags_t = std::conditional_t<(4 * Q > 32), uint64_t, uint32_t>;
        flags_t nzb = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t tt = tv[q][j];
                const float a0 = Fa[(int)(tt & 0xFFFFu)], a1 = Fa[(int)(tt >> 16)];
                nzb |= (flags_t)((a0 != 0.f) | (a1 != 0.f)) << (4 * q + j);
            }
        int n = 0;
        const int k4 = lane16(lane) >> 2;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool nz = (nzb >> (4 * q + j)) & 1;
                const uint64_t m = __builtin_amdgcn_ballot_w64(nz);
                const int pos = n + lanes_below(m);
                if (nz && pos < CAP) {
                    uint32_t tt = t[q][j];
                    float ff = f[q][j];
                    __asm__ volatile("" : "+v"(tt), "+v"(ff));
                    lk[pos] = q * 256 + k4 + j;
                    lt[pos] = tt;
                    lf[pos] = ff;
                }
                n += (int)__builtin_popcountll(m);
            }
        return n;
    };
    const int n = detect();
    wave_sync();
    float hisum = 0.f;
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
    if (n <= min(cap, CAP)) {
        // each listed arc whose value equals its child's cost bids 2k + beta for the child
        const bool mine = lane < n;
        const int k = mine ? lk[lane] : 0;
        const uint32_t tt = mine ? lt[lane] : 0u;
        const float ff = mine ? lf[lane] : 0.f;
        const int lo = (int)(tt & 0xFFFFu), hi = (int)(tt >> 16);
        const float a0 = mine ? Fa[lo] : 0.f, a1 = mine ? Fa[hi] : 0.f;  // level l+1 is unchanged until below
        const bool t0 = mine && a0 != 0.f && ff == Fv[lo];
        const bool t1 = mine && a1 != 0.f && ff + lam_use == Fv[hi];
        if (t0) lds_imin(&bid[lo], 2 * k);
        if (t1) lds_imin(&bid[hi], 2 * k + 1);
        wave_sync();
        const bool w0 = t0 && bid[lo] == 2 * k, w1 = t1 && bid[hi] == 2 * k + 1;
        wave_sync();  // every bid is read, every value of level l+1 too
        if (t0) bid[lo] = INT_MAX;  // the bid buffer is empty again for the next hop
        if (t1) bid[hi] = INT_MAX;
        // level l replaces level l+1 (a lane's node of level l may share a slot with another lane's child)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            lds4(Fv, l16 + q * 1024) = f[q];
            lds4(Fa, l16 + q * 1024) = zero4;
        }
        wave_sync();
        // a node is listed once: its adjoint is the sum of the children it won
        if (w0 || w1) Fa[k] = (w0 ? a0 : 0.f) + (w1 ? a1 : 0.f);
        if (w1) hisum = a1;
    } else {
        // more arcs than the list holds: every lane bids for its own arcs and collects its nodes'
        // adjoints
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                uint32_t tt = t[q][j];
                float ff = f[q][j];
                __asm__ volatile("" : "+v"(tt), "+v"(ff));
                const int k = q * 256 + (l16 >> 2) + j, lo = (int)(tt & 0xFFFFu), hi = (int)(tt >> 16);
                if (Fa[lo] != 0.f && ff == Fv[lo]) lds_imin(&bid[lo], 2 * k);
                if (Fa[hi] != 0.f && ff + lam_use == Fv[hi]) lds_imin(&bid[hi], 2 * k + 1);
            }
        wave_sync();  // the bids are in: F of level l+1 is not read again, its buffer collects
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                uint32_t tt = t[q][j];
                __asm__ volatile("" : "+v"(tt));
                const int k = q * 256 + (l16 >> 2) + j, lo = (int)(tt & 0xFFFFu), hi = (int)(tt >> 16);
                const float alo = Fa[lo], ahi = Fa[hi];
                float acc = 0.f;
                if (alo != 0.f && bid[lo] == 2 * k) acc += alo;
                if (ahi != 0.f && bid[hi] == 2 * k + 1) {
                    acc += ahi;
                    hisum += ahi;
                }
                Fv[k] = acc;
            }
        wave_sync();  // every adjoint and every bid of level l+1 is read
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            lds4(Fa, l16 + q * 1024) = lds4(Fv, l16 + q * 1024);
            lds4(Fv, l16 + q * 1024) = f[q];
#pragma unroll
            for (int j = 0; j < 4; ++j) {  // the bid buffer is empty again for the next hop
                bid[(int)(t[q][j] & 0xFFFFu)] = INT_MAX;
                bid[(int)(t[q][j] >> 16)] = INT_MAX;
            }
        }
    }
    wave_sync();
    // the terminals of level l (children codes W, W + 1 of the next hop) carry no adjoint
    if (lane == 0) {
        Fa[c0.W] = 0.f;
        Fa[c0.W + 1] = 0.f;
    }
    hisum = team_sum<64>(hisum);
    if constexpr (UPD) {
        // the pass's argmin nodes of the two min-marginals and their children (recorded)
        const AdjIn<true> &y = x.a;
        const int K0 = (int)(y.kc0 & 0xFFFFu), K1 = (int)(y.kc1 & 0xFFFFu);
        const int r0 = (int)(y.kc0 >> 16), r1 = (int)(y.kc1 >> 16);
        const float dlam_new = y.dlo + hisum;
        const float dM = y.dMo - dlam_new;
        const float diff = y.d;
        const float dm1 = y.om * dM, dm0 = -dm1;
        wave_sync();  // after the winners' adds (a fixed order of the float adds)
        if (lane == 0) lds_fadd(&Fa[K0], dm0);
        if (lane == 0) lds_fadd(&Fa[K1], dm1);
        st1(o.dlam_in, o.o4 + 4 * l, dlam_new + dm1);  // identity path + the hi arc of m^1 itself
        st1(o.g, o.o4 + 4 * l, dlam_new * y.al);
        st1(o.dalpha, o.o4 + 4 * l, y.da + dlam_new * y.S);
        st1(o.domega, o.o4 + 4 * l, y.dw + dM * diff);
        // children of the argmin nodes: B_{l+1} side contributions (-1 for a terminal)
        st2(o.rec_idx, o.o8 + 8 * l, (uint32_t)(r0 < Wn ? r0 : -1), (uint32_t)(r1 < Wn ? r1 : -1));
        st2(o.rec_val, o.o8 + 8 * l, __float_as_uint(dm0), __float_as_uint(dm1));
    } else {
        // argmin contributions of the update sweep to F_l (record of edge l)
        if (lane == 0) {
            if (x.i0 >= 0 && x.i0 < c0.W) Fa[x.i0] += x.v0;
            if (x.i1 >= 0 && x.i1 < c0.W) Fa[x.i1] += x.v1;
        }
        st1(o.dlam_in, o.o4 + 4 * l, x.dl + hisum);
    }
}

template <int RMAX, bool UPD>
__global__ __launch_bounds__(256) void k_adj_F_w(DevTables T, AdjTables A, int64_t tile0, int64_t ntiles, int NL,
                                                 int recs, int cap) {
    constexpr int NB = node_buf_w(RMAX), QM = RMAX / 4;
    extern __shared__ float lds_f[];
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t tile = tile0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= tile0 + ntiles) return;  // uniform per wave
    float *Fv = lds_f + (size_t)wave * lds_words_adj_F_w(RMAX, NL);
    float *Fa = Fv + NB;
    int *bid = (int *)(Fa + NB);  // INT_MAX between hops
    int *lk = bid + NB;
    uint32_t *lt = (uint32_t *)(lk + kAdjListW);
    float *lf = (float *)(lt + kAdjListW);
    int *meta = (int *)(lf + kAdjListW);
    int *off = meta + NL;
    const TileCtx tc = tile_ctx(T, tile);
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
    const AdjOut o = adj_out<UPD>(A, tc, nlev, lane);
    const bool use_rec = !UPD && recs;
    const rsrc_t ri = buf(use_rec ? (const void *)(A.rec_idx + 2 * (int64_t)tc.ebase) : (const void *)A.dlam_in,
                          use_rec ? nlev * 8 : 0);
    const rsrc_t rv = buf(use_rec ? (const void *)(A.rec_val + 2 * (int64_t)tc.ebase) : (const void *)A.dlam_in,
                          use_rec ? nlev * 8 : 0);
    auto edge = [&](int l) {
        AdjInF<UPD> x;
        const int e = tc.ebase + l;
        if constexpr (UPD) {
            x.a = adj_in<true>(T, A, e);
        } else {
            x.lam_src = A.lam_src[e];
            x.dl = A.dlam_in[e];
            x.i0 = (int)ld1(ri, 8 * l);  // no record: 0 bytes loaded, and use_rec is checked at use
            x.i1 = (int)ld1(ri, 8 * l + 4);
            x.v0 = ld1f(rv, 8 * l);
            x.v1 = ld1f(rv, 8 * l + 4);
        }
        return x;
    };
    {
        // level L: terminals only, no adjoint; no bids
        const int l16 = lane16(lane);
        const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
        const i32x4 none = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
#pragma unroll
        for (int q = 0; q <= QM; ++q)
            if (q < QM || lane < 16) {
                lds4(Fa, l16 + q * 1024) = zero4;
                *(i32x4 *)((char *)bid + l16 + q * 1024) = none;
            }
    }
    Lev c0 = level(nlev - 1), c1{0, 0, 0};
    u32x4 tpn[QM];
    f32x4 fvn[QM];
    {
        const int l16 = lane16(lane);
        const rsrc_t tr = buf(T.topo + c0.base, row_bytes(c0)), fr = buf(T.F + c0.base, row_bytes(c0));
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            tpn[q] = ld4(tr, l16 + q * 1024);
            fvn[q] = ld4f(fr, l16 + q * 1024);
        }
    }
    AdjInF<UPD> xn = edge(nlev - 1);
    for (int l = nlev - 1; l >= 0; --l) {
        const int Wn = c1.W;
        const AdjInF<UPD> x = xn;
        u32x4 tp[QM];
        f32x4 fv[QM];
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            tp[q] = tpn[q];
            fv[q] = fvn[q];
        }
        // prefetch hop l-1: topology and F of level l-1, edge data of level l-1 (the last hop
        // reloads its own)
        const Lev cp = level(l - 1);
        {
            const int l16 = lane16(lane);
            const rsrc_t tr = buf(T.topo + cp.base, row_bytes(cp)), fr = buf(T.F + cp.base, row_bytes(cp));
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                tpn[q] = ld4(tr, l16 + q * 1024);
                fvn[q] = ld4f(fr, l16 + q * 1024);
            }
            xn = edge(max(l - 1, 0));
        }
        wave_sync();
        float lam_use;
        if constexpr (UPD) lam_use = x.a.lam;
        else lam_use = x.lam_src;
        AdjInF<UPD> xu = x;
        if constexpr (!UPD)
            if (!use_rec) xu.i0 = xu.i1 = -1;
        with_count<1, QM>(groups(c0), [&](auto qc) {
            adjF_hop_w<decltype(qc)::value, RMAX, UPD>(Fv, Fa, bid, lk, lt, lf, tp, fv, lane, c0, Wn, lam_use,
                                                       xu, o, l, cap);
        });
        wave_sync();
        c1 = c0;
        c0 = cp;
    }
}

// Se[slot] = S[var(slot)], four slots per thread with the loads of a thread issued together, as in
// k_edge_alpha_s.
__global__ __launch_bounds__(256) void k_edge_S(const int32_t *__restrict__ evar, const float *__restrict__ S,
                                                float *__restrict__ Se, int64_t slots) {
    constexpr int K = kSlotsPerThread;
    const int64_t e0 = xcd_block(blockIdx.x, gridDim.x) * (256 * K) + threadIdx.x;
    int v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = e0 + 256 * k < slots ? evar[e0 + 256 * k] : -1;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float sv = v[k] >= 0 ? S[v[k]] : 0.f;
        if (e0 + 256 * k < slots) Se[e0 + 256 * k] = sv;
    }
}

// Adjoint of lambda_bar = lambda + alpha * S: dlambda stays, d_alpha += dlambda_bar * S_i,
// g = dlambda_bar * alpha (then dS per variable and dM per edge, as after a pass adjoint).
__global__ void k_flush_adj(const int32_t *__restrict__ evar, const float *__restrict__ S,
                            const float *__restrict__ alpha, const float *__restrict__ dlam, float *__restrict__ dalpha,
                            float *__restrict__ g, int64_t slots) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= slots) return;
    const int v = evar[e];
    const float d = v >= 0 ? dlam[e] : 0.f;
    if (v >= 0) dalpha[e] += d * S[v];
    g[e] = d * alpha[e];
}

// The per-variable transforms below run kVarLanes lanes per variable: lane u of a team visits the
// variable's edges u, u + kVarLanes, ... (var_canon order), and a fixed butterfly combines the lanes'
// partial sums or maxima, so every result has the same bits on every call.  A variable in many rows
// (a graph-matching assignment variable sits in ~42) then waits for a quarter of the dependent loads
// of a single thread.  Every lane of a wave takes part in the butterflies; lanes past n have no edges.
constexpr int kVarLanes = 4;

__device__ __forceinline__ float team_sum_v(float s) {
    for (int w = kVarLanes / 2; w > 0; w >>= 1) s += __shfl_xor(s, w, kVarLanes);
    return s;
}
__device__ __forceinline__ float team_max_v(float s) {
    for (int w = kVarLanes / 2; w > 0; w >>= 1) s = fmaxf(s, __shfl_xor(s, w, kVarLanes));
    return s;
}
struct VarTeam {
    int a, b, u;  // the variable's edge range in var_canon; this lane's offset in it
};
__device__ __forceinline__ VarTeam var_team(const int32_t *__restrict__ var_ptr, int n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t / kVarLanes), u = (int)(t % kVarLanes);
    return {i < n ? var_ptr[i] : 0, i < n ? var_ptr[i + 1] : 0, u};
}

// d c_i = sum_{e of i} dlambda_e / |J_i|  (lambda_0 = c / |J|); variables in no row: seed * [c_i < 0].
__global__ void k_dc(const int32_t *__restrict__ var_ptr, const int32_t *__restrict__ var_slots,
                     const float *__restrict__ dlam, const float *__restrict__ c, float seed, float *__restrict__ dc,
                     int n) {
    const VarTeam v = var_team(var_ptr, n);
    const int i = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kVarLanes);
    float s = 0.f;
    for (int q = v.a + v.u; q < v.b; q += kVarLanes) s += dlam[var_slots[q]];
    s = team_sum_v(s);
    if (i < n && v.u == 0) dc[i] = v.a == v.b ? (c[i] < 0.f ? seed : 0.f) : s / (float)(v.b - v.a);
}

// d alpha_hat_e = alpha_e (d alpha_e - sum_{k in J_i} alpha_k d alpha_k), canonical arrays.
__global__ void k_softmax_vjp(const int32_t *__restrict__ var_ptr, const int32_t *__restrict__ var_canon,
                              const float *__restrict__ alpha, const float *__restrict__ dalpha, float *__restrict__ out,
                              int n) {
    const VarTeam v = var_team(var_ptr, n);
    float s = 0.f;
    for (int q = v.a + v.u; q < v.b; q += kVarLanes) s += alpha[var_canon[q]] * dalpha[var_canon[q]];
    s = team_sum_v(s);
    for (int q = v.a + v.u; q < v.b; q += kVarLanes) {
        const int e = var_canon[q];
        out[e] = alpha[e] * (dalpha[e] - s);
    }
}

// Output transforms of the parameter predictor (Alg. 3): omega = sigmoid(omega_hat) per edge,
// alpha = softmax over J_i of alpha_hat, theta = theta_hat minus its mean over J_i.  Canonical edge
// arrays; var_canon = CSR of each variable's canonical edges.
__global__ void k_param_transform(const int32_t *__restrict__ var_ptr, const int32_t *__restrict__ var_canon,
                                  const float *__restrict__ wh, const float *__restrict__ ah,
                                  const float *__restrict__ th, float *__restrict__ w, float *__restrict__ al,
                                  float *__restrict__ t, int n) {
    const VarTeam v = var_team(var_ptr, n);
    float mx = -kInf, tsum = 0.f;
    for (int q = v.a + v.u; q < v.b; q += kVarLanes) {
        const int e = var_canon[q];
        mx = fmaxf(mx, ah[e]);
        if (th) tsum += th[e];
    }
    mx = team_max_v(mx);
    tsum = team_sum_v(tsum);
    float den = 0.f;
    for (int q = v.a + v.u; q < v.b; q += kVarLanes) den += expf(ah[var_canon[q]] - mx);
    den = team_sum_v(den);
    const float tmean = tsum / (float)(v.b > v.a ? v.b - v.a : 1);
    for (int q = v.a + v.u; q < v.b; q += kVarLanes) {
        const int e = var_canon[q];
        w[e] = 1.f / (1.f + expf(-wh[e]));
        al[e] = expf(ah[e] - mx) / den;
        if (th) t[e] = th[e] - tmean;
    }
}

// Adjoints of k_param_transform's inputs: d_omega_hat = d_omega * omega (1 - omega),
// d_alpha_hat = alpha (d_alpha - sum_k alpha_k d_alpha_k), d_theta_hat = d_theta minus its mean.
__global__ void k_param_transform_vjp(const int32_t *__restrict__ var_ptr, const int32_t *__restrict__ var_canon,
                                      const float *__restrict__ w, const float *__restrict__ al,
                                      const float *__restrict__ dw, const float *__restrict__ da,
                                      const float *__restrict__ dt, float *__restrict__ dwh,
                                      float *__restrict__ dah, float *__restrict__ dth, int n) {
    const VarTeam v = var_team(var_ptr, n);
    float s = 0.f, tsum = 0.f;
    for (int q = v.a + v.u; q < v.b; q += kVarLanes) {
        const int e = var_canon[q];
        s += al[e] * da[e];
        if (dt) tsum += dt[e];
    }
    s = team_sum_v(s);
    tsum = team_sum_v(tsum);
    const float tmean = tsum / (float)(v.b > v.a ? v.b - v.a : 1);
    for (int q = v.a + v.u; q < v.b; q += kVarLanes) {
        const int e = var_canon[q];
        dwh[e] = dw[e] * w[e] * (1.f - w[e]);
        dah[e] = al[e] * (da[e] - s);
        if (dt) dth[e] = dt[e] - tmean;
    }
}

// Non-parametric update (eq. 2): lambda[slot of e] += theta_hat[e] - mean over J_i of theta_hat.
__global__ void k_nonparam_update(const int32_t *__restrict__ var_ptr, const int32_t *__restrict__ var_canon,
                                  const int32_t *__restrict__ canon2slot, const float *__restrict__ th,
                                  float *__restrict__ lam, int n) {
    const VarTeam v = var_team(var_ptr, n);
    float tsum = 0.f;
    for (int q = v.a + v.u; q < v.b; q += kVarLanes) tsum += th[var_canon[q]];
    tsum = team_sum_v(tsum);
    const float tmean = tsum / (float)(v.b > v.a ? v.b - v.a : 1);
    for (int q = v.a + v.u; q < v.b; q += kVarLanes) {
        const int e = var_canon[q];
        const int sl = canon2slot[e];
        lam[sl] = lam[sl] + (th[e] - tmean);
    }
}

// sum over variables with no row of min(0, c_i)
__global__ void k_fill(float *__restrict__ x, float v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ void k_uncovered(const int32_t *__restrict__ var_ptr, const float *__restrict__ c, float *__restrict__ out,
                            int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = var_ptr[i + 1] == var_ptr[i] ? fminf(c[i], 0.f) : 0.f;
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------------------------------------------
// Reverse sweeps of one-wave diagrams that route along the argmin codes the sweeps they reverse
// recorded (DevTables::Fpar, Bch): every node's argmin parent arc (F side) or child arc (B side) is
// read from a 2-byte code row, so a hop needs neither topology nor node costs nor bids, only the
// codes of one level and the adjoint buffer in LDS.
//  * pull (B side, levels 0 .. L-1): node v hands its adjoint to its recorded child and, through a
//    hi arc, to the hi-arc sum;
//  * push (F side, levels L-1 .. 0): node w of level l+1 hands its adjoint to its recorded parent
//    arc (k, beta) of level l.  An arc has one child, so a parent receives at most one adjoint per
//    arc kind: lo arcs are written first, then hi arcs added, with no conflict and in the order
//    lo + hi of the bidding sweeps.
// The BlockUpdate adjoint, the argmin records of the pass and the hand-over records are those of
// the bidding sweeps above.
// ------------------------------------------------------------------------------------------
constexpr int lds_words_adjc_F_w(int RMAX, int NL) { return node_buf_w(RMAX) + ((2 * NL + 3) & ~3); }
// the pull sweep keeps one adjoint buffer: a hop reads its level's adjoints into registers before it
// clears the buffer and routes them into the next level there, as the push sweep does
constexpr int lds_words_adjc_B_w(int RMAX, int NL) { return node_buf_w(RMAX) + ((2 * NL + 3) & ~3); }

template <int Q, int RMAX, bool UPD>
__device__ __forceinline__ void adjcB_hop_w(float *Ba, const u32x2 (&cc)[RMAX / 4], int lane, int Wn,
                                            const AdjIn<UPD> &x, const AdjOut &o, int l) {
    constexpr int QM = RMAX / 4;
    const int l16 = lane16(lane);
    f32x4 d[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) d[q] = lds4(Ba, l16 + q * 1024);  // adjoints of level l (0 past its width)
    wave_sync();  // every adjoint of level l is read: the buffer collects level l+1
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < QM; ++q) lds4(Ba, l16 + q * 1024) = zero4;
    wave_sync();
    float hisum = 0.f;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t code = code_at(cc[q], j);
            const int ch = (int)(code & 0x7FFFu);
            if (d[q][j] != 0.f) {
                if (ch < Wn) lds_fadd(&Ba[ch], d[q][j]);
                if (code & 0x8000u) hisum += d[q][j];
            }
        }
    }
    hisum = team_sum<64>(hisum);
    if constexpr (UPD) {
        // the pass's argmin nodes of the two min-marginals and their children (recorded)
        const int K0 = (int)(x.kc0 & 0xFFFFu), K1 = (int)(x.kc1 & 0xFFFFu);
        const int r0 = (int)(x.kc0 >> 16), r1 = (int)(x.kc1 >> 16);
        const float dlam_new = x.dlo + hisum;
        const float dM = x.dMo - dlam_new;
        const float dm1 = x.om * dM, dm0 = -dm1;
        wave_sync();  // after the routed adjoints (a fixed order of the float adds)
        if (lane == 0 && r0 < Wn) lds_fadd(&Ba[r0], dm0);
        if (lane == 0 && r1 < Wn) lds_fadd(&Ba[r1], dm1);
        st1(o.dlam_in, o.o4 + 4 * l, dlam_new + dm1);  // identity path + the hi arc of m^1 itself
        st1(o.g, o.o4 + 4 * l, dlam_new * x.al);
        st1(o.dalpha, o.o4 + 4 * l, x.da + dlam_new * x.S);
        st1(o.domega, o.o4 + 4 * l, x.dw + dM * x.d);
        st2(o.rec_idx, o.o8 + 8 * l, (uint32_t)K0, (uint32_t)K1);  // argmin nodes of level l: F_l side
        st2(o.rec_val, o.o8 + 8 * l, __float_as_uint(dm0), __float_as_uint(dm1));
    } else {
        st1(o.dlam_in, o.o4 + 4 * l, x.dl + hisum);
    }
}

template <int RMAX, bool UPD>
__global__ __launch_bounds__(256) void k_adjc_B_w(DevTables T, AdjTables A, int64_t tile0, int64_t ntiles, int NL,
                                                  int recs, float seed) {
    constexpr int NB = node_buf_w(RMAX), QM = RMAX / 4;
    extern __shared__ float lds_f[];
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t tile = tile0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= tile0 + ntiles) return;  // uniform per wave
    float *Ba = lds_f + (size_t)wave * lds_words_adjc_B_w(RMAX, NL);  // adjoints of level l, in place
    int *meta = (int *)(Ba + NB);
    int *off = meta + NL;
    const TileCtx tc = tile_ctx(T, tile);
    preload_meta<1>(T, tc, lane, meta, off);
    const int nlev = tc.nlev;
    auto level = [&](int l) {
        Lev v{0, 0, 0};
        if (l < nlev) {
            v.W = uni(meta[l] & 0xFFFF);
            v.R = uni(meta[l] >> 16);
            v.base = tc.nbase + (int64_t)uni(off[l]);
        }
        return v;
    };
    const AdjOut o = adj_out<UPD>(A, tc, nlev, lane);
    const bool use_rec = !UPD && recs;
    const rsrc_t ri = buf(use_rec ? (const void *)(A.rec_idx + 2 * (int64_t)tc.ebase) : (const void *)A.dlam_in,
                          use_rec ? nlev * 8 : 0);
    const rsrc_t rv = buf(use_rec ? (const void *)(A.rec_val + 2 * (int64_t)tc.ebase) : (const void *)A.dlam_in,
                          use_rec ? nlev * 8 : 0);
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
    {
        const int l16 = lane16(lane);
#pragma unroll
        for (int q = 0; q < QM; ++q) lds4(Ba, l16 + q * 1024) = zero4;
        if (lane == 0) Ba[0] = A.seed ? *A.seed : seed;  // the root is node 0 of level 0
    }
    Lev c0 = level(0), c1 = level(1);
    u32x2 ccn[QM];
    {
        const int l8 = lane8(lane);
        const rsrc_t cr = buf(T.Bch + c0.base, code_bytes(c0));
#pragma unroll
        for (int q = 0; q < QM; ++q) ccn[q] = ld2(cr, l8 + q * 512);
    }
    AdjIn<UPD> xn = adj_in<UPD>(T, A, tc.ebase);
    int pi0 = -1, pi1 = -1;  // record of the previous hop's edge (children at this level, or -1)
    float pv0 = 0.f, pv1 = 0.f;
    for (int l = 0; l < nlev; ++l) {
        const int Wn = c1.W;
        const AdjIn<UPD> x = xn;
        // fixed side: argmin contributions of the update sweep to B_l (record of edge l-1)
        if (use_rec && l > 0 && lane == 0) {
            if (pi0 >= 0) Ba[pi0] += pv0;
            if (pi1 >= 0) Ba[pi1] += pv1;
        }
        u32x2 cc[QM];
#pragma unroll
        for (int q = 0; q < QM; ++q) cc[q] = ccn[q];
        // prefetch hop l+1: codes of level l+1, edge data of level l+1 (the last hop reloads its own),
        // the record of edge l
        {
            const int l8 = lane8(lane);
            const rsrc_t cr = buf(T.Bch + c1.base, code_bytes(c1));
#pragma unroll
            for (int q = 0; q < QM; ++q) ccn[q] = ld2(cr, l8 + q * 512);
            xn = adj_in<UPD>(T, A, tc.ebase + min(l + 1, nlev - 1));
            if (!UPD) {
                pi0 = (int)ld1(ri, 8 * l);
                pi1 = (int)ld1(ri, 8 * l + 4);
                pv0 = ld1f(rv, 8 * l);
                pv1 = ld1f(rv, 8 * l + 4);
            }
        }
        wave_sync();
        with_count<1, QM>(groups(c0), [&](auto qc) {
            adjcB_hop_w<decltype(qc)::value, RMAX, UPD>(Ba, cc, lane, Wn, x, o, l);
        });
        wave_sync();
        c0 = c1;
        c1 = level(l + 2);
    }
}

template <int Q, int RMAX, bool UPD>
__device__ __forceinline__ void adjcF_hop_w(float *Fa, const u32x2 (&cc)[RMAX / 4], int lane, const Lev &c0, int Wn,
                                            const AdjInF<UPD> &x, const AdjOut &o, int l) {
    constexpr int QM = RMAX / 4;
    const int l16 = lane16(lane);
    f32x4 a[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) a[q] = lds4(Fa, l16 + q * 1024);  // adjoints of level l+1 (0 past its width)
    wave_sync();  // every adjoint of level l+1 is read: the buffer collects level l
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < QM; ++q) lds4(Fa, l16 + q * 1024) = zero4;
    wave_sync();
    float hisum = 0.f;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t code = code_at(cc[q], j);
            const int k = (int)(code >> 1);
            if (a[q][j] != 0.f && !(code & 1u) && k < c0.W) Fa[k] = a[q][j];  // lo arcs: one per parent
        }
    wave_sync();
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t code = code_at(cc[q], j);
            const int k = (int)(code >> 1);
            if (a[q][j] != 0.f && (code & 1u) && k < c0.W) {  // hi arcs: one per parent, added to its lo share
                Fa[k] += a[q][j];
                hisum += a[q][j];
            }
        }
    hisum = team_sum<64>(hisum);
    if constexpr (UPD) {
        // the pass's argmin nodes of the two min-marginals and their children (recorded)
        const AdjIn<true> &y = x.a;
        const int K0 = (int)(y.kc0 & 0xFFFFu), K1 = (int)(y.kc1 & 0xFFFFu);
        const int r0 = (int)(y.kc0 >> 16), r1 = (int)(y.kc1 >> 16);
        const float dlam_new = y.dlo + hisum;
        const float dM = y.dMo - dlam_new;
        const float diff = y.d;
        const float dm1 = y.om * dM, dm0 = -dm1;
        wave_sync();  // after the routed adds (a fixed order of the float adds)
        if (lane == 0) lds_fadd(&Fa[K0], dm0);
        if (lane == 0) lds_fadd(&Fa[K1], dm1);
        st1(o.dlam_in, o.o4 + 4 * l, dlam_new + dm1);  // identity path + the hi arc of m^1 itself
        st1(o.g, o.o4 + 4 * l, dlam_new * y.al);
        st1(o.dalpha, o.o4 + 4 * l, y.da + dlam_new * y.S);
        st1(o.domega, o.o4 + 4 * l, y.dw + dM * diff);
        // children of the argmin nodes: B_{l+1} side contributions (-1 for a terminal)
        st2(o.rec_idx, o.o8 + 8 * l, (uint32_t)(r0 < Wn ? r0 : -1), (uint32_t)(r1 < Wn ? r1 : -1));
        st2(o.rec_val, o.o8 + 8 * l, __float_as_uint(dm0), __float_as_uint(dm1));
    } else {
        wave_sync();
        // argmin contributions of the update sweep to F_l (record of edge l)
        if (lane == 0) {
            if (x.i0 >= 0 && x.i0 < c0.W) Fa[x.i0] += x.v0;
            if (x.i1 >= 0 && x.i1 < c0.W) Fa[x.i1] += x.v1;
        }
        st1(o.dlam_in, o.o4 + 4 * l, x.dl + hisum);
    }
}

template <int RMAX, bool UPD>
__global__ __launch_bounds__(256) void k_adjc_F_w(DevTables T, AdjTables A, int64_t tile0, int64_t ntiles, int NL,
                                                  int recs) {
    constexpr int QM = RMAX / 4;
    extern __shared__ float lds_f[];
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t tile = tile0 + (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (tile >= tile0 + ntiles) return;  // uniform per wave
    float *Fa = lds_f + (size_t)wave * lds_words_adjc_F_w(RMAX, NL);
    int *meta = (int *)(Fa + node_buf_w(RMAX));
    int *off = meta + NL;
    const TileCtx tc = tile_ctx(T, tile);
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
    const AdjOut o = adj_out<UPD>(A, tc, nlev, lane);
    const bool use_rec = !UPD && recs;
    const rsrc_t ri = buf(use_rec ? (const void *)(A.rec_idx + 2 * (int64_t)tc.ebase) : (const void *)A.dlam_in,
                          use_rec ? nlev * 8 : 0);
    const rsrc_t rv = buf(use_rec ? (const void *)(A.rec_val + 2 * (int64_t)tc.ebase) : (const void *)A.dlam_in,
                          use_rec ? nlev * 8 : 0);
    auto edge = [&](int l) {
        AdjInF<UPD> x;
        const int e = tc.ebase + l;
        if constexpr (UPD) {
            x.a = adj_in<true>(T, A, e);
        } else {
            x.lam_src = 0.f;
            x.dl = A.dlam_in[e];
            x.i0 = use_rec ? (int)ld1(ri, 8 * l) : -1;
            x.i1 = use_rec ? (int)ld1(ri, 8 * l + 4) : -1;
            x.v0 = ld1f(rv, 8 * l);
            x.v1 = ld1f(rv, 8 * l + 4);
        }
        return x;
    };
    {
        // level L: terminals only, no adjoint
        const int l16 = lane16(lane);
        const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < QM; ++q) lds4(Fa, l16 + q * 1024) = zero4;
    }
    Lev c0 = level(nlev - 1), c1{0, 0, 0};
    u32x2 ccn[QM];  // codes of level l+1 (none below the last level)
#pragma unroll
    for (int q = 0; q < QM; ++q) ccn[q] = u32x2{0u, 0u};
    AdjInF<UPD> xn = edge(nlev - 1);
    for (int l = nlev - 1; l >= 0; --l) {
        const int Wn = c1.W;
        const AdjInF<UPD> x = xn;
        u32x2 cc[QM];
#pragma unroll
        for (int q = 0; q < QM; ++q) cc[q] = ccn[q];
        // prefetch hop l-1: the codes of level l, edge data of level l-1 (the last hop reloads its own)
        {
            const int l8 = lane8(lane);
            const rsrc_t cr = buf(T.Fpar + c0.base, code_bytes(c0));
#pragma unroll
            for (int q = 0; q < QM; ++q) ccn[q] = ld2(cr, l8 + q * 512);
            xn = edge(max(l - 1, 0));
        }
        wave_sync();
        with_count<1, QM>(max(groups(c1), 1), [&](auto qc) {
            adjcF_hop_w<decltype(qc)::value, RMAX, UPD>(Fa, cc, lane, c0, Wn, x, o, l);
        });
        wave_sync();
        c1 = c0;
        c0 = level(l - 1);
    }
}

template <int P, int RMAX>
hipError_t adj_dispatch(const DevTables &t, const AdjTables &a, const ClassLaunch &c, int which, int bar, int recs,
                        float seed, int dense, hipStream_t s) {
    const int cap = dense ? 0 : INT_MAX;  // list entries the one-wave sweeps may use
    if (c.wpb_af < 1 || c.wpb_af > kMaxWavesPerBlock || c.wpb_ab < 1 || c.wpb_ab > kMaxWavesPerBlock)
        return hipErrorInvalidConfiguration;
    const bool push = which == ADJ_F_UPDATE || which == ADJ_F_FIXED;
    if constexpr (P == 64) {  // one-wave diagrams: the wide sweeps only
        // along the recorded argmin codes (unless asked for the bidding sweeps' node-by-node routing)
        if (!dense && (push ? t.Fpar != nullptr : t.Bch != nullptr)) {
            if (push) {
                dim3 grid((unsigned)((c.ntiles + c.wpb_af - 1) / c.wpb_af)), block(64 * c.wpb_af);
                const size_t lds = (size_t)c.wpb_af * lds_words_adjc_F_w(RMAX, c.NL) * 4;
                if (which == ADJ_F_UPDATE)
                    hipLaunchKernelGGL((k_adjc_F_w<RMAX, true>), grid, block, lds, s, t, a, c.tile0, c.ntiles, c.NL,
                                       recs);
                else
                    hipLaunchKernelGGL((k_adjc_F_w<RMAX, false>), grid, block, lds, s, t, a, c.tile0, c.ntiles, c.NL,
                                       recs);
            } else {
                dim3 grid((unsigned)((c.ntiles + c.wpb_ab - 1) / c.wpb_ab)), block(64 * c.wpb_ab);
                const size_t lds = (size_t)c.wpb_ab * lds_words_adjc_B_w(RMAX, c.NL) * 4;
                if (which == ADJ_B_UPDATE)
                    hipLaunchKernelGGL((k_adjc_B_w<RMAX, true>), grid, block, lds, s, t, a, c.tile0, c.ntiles, c.NL,
                                       recs, seed);
                else
                    hipLaunchKernelGGL((k_adjc_B_w<RMAX, false>), grid, block, lds, s, t, a, c.tile0, c.ntiles, c.NL,
                                       recs, seed);
            }
            return hipGetLastError();
        }
        if (push) {
            dim3 grid((unsigned)((c.ntiles + c.wpb_af - 1) / c.wpb_af)), block(64 * c.wpb_af);
            const size_t lds = (size_t)c.wpb_af * lds_words_adj_F_w(RMAX, c.NL) * 4;
            if (which == ADJ_F_UPDATE)
                hipLaunchKernelGGL((k_adj_F_w<RMAX, true>), grid, block, lds, s, t, a, c.tile0, c.ntiles, c.NL, recs,
                                   cap);
            else
                hipLaunchKernelGGL((k_adj_F_w<RMAX, false>), grid, block, lds, s, t, a, c.tile0, c.ntiles, c.NL,
                                   recs, cap);
            return hipGetLastError();
        }
    } else if (push) {
        dim3 grid((unsigned)((c.ntiles + c.wpb_af - 1) / c.wpb_af)), block(64 * c.wpb_af);
        const size_t lds = (size_t)c.wpb_af * lds_words_adj_F(P, c.WB, c.NL) * 4;
        if (which == ADJ_F_UPDATE)
            hipLaunchKernelGGL((k_adj_F<P, RMAX, true>), grid, block, lds, s, t, a, c.tile0, c.ntiles, c.WB, c.NL);
        else
            hipLaunchKernelGGL((k_adj_F<P, RMAX, false>), grid, block, lds, s, t, a, c.tile0, c.ntiles, c.WB, c.NL);
        return hipGetLastError();
    }
    if constexpr (P == 64) {
        dim3 grid((unsigned)((c.ntiles + c.wpb_ab - 1) / c.wpb_ab)), block(64 * c.wpb_ab);
        const size_t lds = (size_t)c.wpb_ab * lds_words_adj_B_w(RMAX, c.NL) * 4;
        if (which == ADJ_B_UPDATE)
            hipLaunchKernelGGL((k_adj_B_w<RMAX, true>), grid, block, lds, s, t, a, c.tile0, c.ntiles, c.NL, bar, recs,
                               seed, cap);
        else
            hipLaunchKernelGGL((k_adj_B_w<RMAX, false>), grid, block, lds, s, t, a, c.tile0, c.ntiles, c.NL, bar, recs,
                               seed, cap);
    } else {
        dim3 grid((unsigned)((c.ntiles + c.wpb_ab - 1) / c.wpb_ab)), block(64 * c.wpb_ab);
        const size_t lds = (size_t)c.wpb_ab * lds_words_adj_B(P, c.WB, c.NL) * 4;
        if (which == ADJ_B_UPDATE)
            hipLaunchKernelGGL((k_adj_B<P, RMAX, true>), grid, block, lds, s, t, a, c.tile0, c.ntiles, c.WB, c.NL, bar,
                               recs, seed);
        else
            hipLaunchKernelGGL((k_adj_B<P, RMAX, false>), grid, block, lds, s, t, a, c.tile0, c.ntiles, c.WB, c.NL, bar,
                               recs, seed);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adj(const DevTables &t, const AdjTables &a, const ClassLaunch &c, int which, int bar, int recs,
                      float seed, int dense, hipStream_t s) {
    if (c.ntiles <= 0) return hipSuccess;
#define DD_ADJ(PP, RR) \
    if (c.P == PP && c.RMAX == RR) return adj_dispatch<PP, RR>(t, a, c, which, bar, recs, seed, dense, s);
    DD_CLASSES(DD_ADJ)
#undef DD_ADJ
    return hipErrorInvalidValue;
}

hipError_t launch_edge_S(const int32_t *evar, const float *S, float *Se, int64_t slots, hipStream_t s) {
    if (slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_edge_S, dim3(xcd_grid(blocks_for(slots, 256 * kSlotsPerThread))), dim3(256), 0, s, evar, S,
                       Se, slots);
    return hipGetLastError();
}

hipError_t launch_flush_adj(const int32_t *evar, const float *S, const float *alpha, const float *dlam, float *dalpha,
                            float *g, int64_t slots, hipStream_t s) {
    if (slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flush_adj, dim3(blocks_for(slots, 256)), dim3(256), 0, s, evar, S, alpha, dlam, dalpha, g,
                       slots);
    return hipGetLastError();
}

hipError_t launch_dc(const int32_t *var_ptr, const int32_t *var_slots, const float *dlam, const float *c, float seed,
                     float *dc, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dc, dim3(blocks_for((int64_t)n * kVarLanes, 256)), dim3(256), 0, s, var_ptr, var_slots, dlam, c, seed, dc, n);
    return hipGetLastError();
}

hipError_t launch_softmax_vjp(const int32_t *var_ptr, const int32_t *var_canon, const float *alpha,
                              const float *dalpha, float *out, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_softmax_vjp, dim3(blocks_for((int64_t)n * kVarLanes, 256)), dim3(256), 0, s, var_ptr, var_canon, alpha, dalpha, out,
                       n);
    return hipGetLastError();
}

hipError_t launch_param_transform(const int32_t *var_ptr, const int32_t *var_canon, const float *wh, const float *ah,
                                  const float *th, float *w, float *al, float *t, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_param_transform, dim3(blocks_for((int64_t)n * kVarLanes, 256)), dim3(256), 0, s, var_ptr, var_canon, wh, ah, th, w,
                       al, t, n);
    return hipGetLastError();
}

hipError_t launch_param_transform_vjp(const int32_t *var_ptr, const int32_t *var_canon, const float *w,
                                      const float *al, const float *dw, const float *da, const float *dt, float *dwh,
                                      float *dah, float *dth, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_param_transform_vjp, dim3(blocks_for((int64_t)n * kVarLanes, 256)), dim3(256), 0, s, var_ptr, var_canon, w, al, dw,
                       da, dt, dwh, dah, dth, n);
    return hipGetLastError();
}

hipError_t launch_nonparam_update(const int32_t *var_ptr, const int32_t *var_canon, const int32_t *canon2slot,
                                  const float *th, float *lam, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nonparam_update, dim3(blocks_for((int64_t)n * kVarLanes, 256)), dim3(256), 0, s, var_ptr, var_canon, canon2slot,
                       th, lam, n);
    return hipGetLastError();
}

hipError_t launch_fill(float *x, float v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, v, n);
    return hipGetLastError();
}

hipError_t launch_uncovered(const int32_t *var_ptr, const float *c, float *out, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_uncovered, dim3(blocks_for(n, 256)), dim3(256), 0, s, var_ptr, c, out, n);
    return hipGetLastError();
}

}  // namespace dd
