// kernels.hpp -- device data layout and kernel launchers (host-visible declarations).
//
// Layout ("tiles"): one wavefront processes one tile; its 64 lanes form G = 64/P teams of
// P lanes and each team owns one decision diagram (one constraint row).  For level l of a
// tile, node k of team g is stored at slot
//     node_base[tile] + lev_off[l] + (k / P) * 64 + g * P + (k % P)
// so the lanes of a wave read 64 consecutive slots per row of the level: every hop of
// every diagram in the tile is one coalesced sweep.  lev_rows[l] = max over teams of
// ceil(width / P) rows.  Per-edge data (lambda, M, omega, alpha, variable) of level l of
// team g is at edge slot edge_base[tile] + l * G + g.
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace dd {

enum FwdMode { FWD_UPDATE = 0, FWD_SWEEP_BAR = 1 };
enum BwdMode { BWD_UPDATE = 0, BWD_STORE = 1, BWD_EN_LAM = 2, BWD_EN_BAR = 3, BWD_MM = 4 };

struct DevTables {
    // tile tables
    const int64_t *node_base;
    const int32_t *edge_base;
    const int32_t *nlev;
    const int32_t *lev_base;  // index of the tile's first level in lev_off / lev_rows
    const int32_t *w_base;    // index of the tile's first width entry (level-major, G per level)
    const int32_t *bdd;       // [tiles * 64] row id per team (-1: empty team)
    const int32_t *lev_off;   // node offset of each level relative to node_base
    const int32_t *lev_rows;
    const uint16_t *widths;
    // nodes
    const uint32_t *topo;     // lo | hi << 16 child codes
    float *F;                 // shortest path root -> node (forward pass output)
    float *B;                 // shortest path node -> 1-terminal (backward pass output)
    // edges (slot indexed)
    float *lam;
    float *M;
    const float *omega;
    const float *alpha;
    const int32_t *evar;      // variable of each edge slot (-1: padding)
    const int32_t *slot2canon;
    const float *S;           // [n] deferred sums
    const float *aS;          // [edge slots] alpha * S of the edge's variable
    float *energies;          // [m] per-row E^j at the flushed multipliers
    float *en_lam;            // [m] per-row E^j at the current multipliers (from backward passes)
    float *out0, *out1;       // [edges] canonical min-marginal outputs
};

struct ClassLaunch {
    int P;         // team size (lanes per diagram)
    int RMAX;      // max rows (of 64 slots) per level for this class
    int WL;        // max level width in the class
    int WB;        // LDS floats per team per node buffer: WL + 2 terminals, rounded up to P
    int NL;        // max levels of a tile in the class
    int wpb_f, wpb_b;  // waves per workgroup of the forward / backward kernels
    int64_t tile0, ntiles;
    int64_t nodes, edges, rows;  // real (unpadded) counts covered by one launch, for byte accounting
};

// LDS words (4 bytes) one wavefront of the forward / backward pass kernels uses.
// per wave: two node buffers (2 * WB * G), level table (NL * G + NL), staged lambda and M (2 * NL * G)
constexpr int lds_words_pass(int P, int WB, int NL) {  // constexpr: usable in device code too
    return 2 * WB * (64 / P) + NL * (3 * (64 / P) + 1);
}

hipError_t launch_fwd(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s);
hipError_t launch_bwd(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s);
bool class_supported(int P, int RMAX);

// S_i = sum over the CSR list of edge slots of variable i of M[slot], in list order.
hipError_t launch_deferred_sum(const int32_t *var_ptr, const int32_t *var_slots, const float *M, float *S, int n,
                               hipStream_t s);
// aS[slot] = alpha[slot] * S[evar[slot]] for every edge slot (0 on padding).
hipError_t launch_edge_alpha_s(const int32_t *evar, const float *alpha, const float *S, float *aS, int64_t slots,
                               hipStream_t s);
// lambda[slot] = c_i / |J_i|, M[slot] = 0 for every canonical edge.
hipError_t launch_init_lambda(const int32_t *canon2slot, const int32_t *evar, const int32_t *var_ptr, const float *c,
                              float *lam, float *M, int64_t E, hipStream_t s);
// dst[canon2slot[e]] = src[e]
hipError_t launch_scatter(const int32_t *canon2slot, const float *src, float *dst, int64_t E, hipStream_t s);
// dst[e] = src[canon2slot[e]] (+ add[canon2slot[e]] when add is not NULL)
hipError_t launch_gather(const int32_t *canon2slot, const float *src, float *dst, int64_t E, const float *add,
                         hipStream_t s);
// softmax over each variable's edges; inputs/outputs canonical, var_canon is the CSR of canonical edge ids
hipError_t launch_seg_softmax(const int32_t *var_ptr, const int32_t *var_canon, const float *x, float *y, int n,
                              hipStream_t s);
// *out = sum of x[0..n) (or of min(0, x) when neg_part), fp64, fixed order; partial holds
// kSumBlocks doubles of scratch.
constexpr int kSumBlocks = 1024;
hipError_t launch_sum(const float *x, int64_t n, int neg_part, double *partial, double *out, hipStream_t s);
// validity check of parameters: flags[0] |= omega outside [0,1] or non-finite, flags[1] |= alpha < 0 or non-finite
hipError_t launch_check_params(const float *omega, const float *alpha, int64_t E, int32_t *flags, hipStream_t s);

}  // namespace dd
