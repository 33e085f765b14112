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

// forward: update pass; F sweep at lambda_bar (no update); F sweep at lambda (no update); update
// pass that also records each hop's min-marginal argmins (DevTables::mrec / mdiff)
enum FwdMode { FWD_UPDATE = 0, FWD_SWEEP_BAR = 1, FWD_SWEEP_LAM = 2, FWD_UPDATE_REC = 3 };
// backward: update pass; B sweep at lambda stored; energies at lambda; energies at lambda_bar;
// min-marginals at lambda_bar; B sweep at lambda_bar stored; update pass recording its argmins
enum BwdMode {
    BWD_UPDATE = 0,
    BWD_STORE = 1,
    BWD_EN_LAM = 2,
    BWD_EN_BAR = 3,
    BWD_MM = 4,
    BWD_STORE_BAR = 5,
    BWD_UPDATE_REC = 6
};

constexpr uint32_t kRawLevel = 0xFFFFFFFFu;  // lev_code of a level without byte codes

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
    // the same codes of one-wave diagrams in one byte per node (node-slot indexed like topo): the
    // step of the lo child code in the low nibble and of the hi child code in the high nibble, from
    // the node before in the level; lev_code[level] (indexed like lev_off) holds the codes of the
    // level's first node, lo | hi << 16, or kRawLevel when the steps of a level do not fit (its
    // passes read topo).  On a level whose next one is empty (codes 0 and 1, the two terminals)
    // the bytes describe 1 - code, so that those codes are non-decreasing too.
    const uint8_t *tcode;
    const uint32_t *lev_code;
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
    float *aS;                // [edge slots] alpha * S of the edge's variable
    int form_as;              // narrow update passes form alpha * S from S and store it (no separate launch)
    float *Se_rec;            // [edge slots] S of each edge's variable, written by the recording narrow passes
                              // that form alpha * S (NULL: not kept; padding slots are left as they are)
    float *energies;          // [m] per-row E^j at the flushed multipliers
    float *en_lam;            // [m] per-row E^j at the current multipliers (from backward passes)
    float *out0, *out1;       // [edges] canonical min-marginal outputs
    // recording update passes of one-wave diagrams, per edge slot: [2 slot] = lowest argmin node of
    // m^0 | its lo child << 16, [2 slot + 1] = the same for m^1 and the hi child; mdiff = m^1 - m^0
    int32_t *mrec;
    float *mdiff;
    // argmin codes of the node costs in F and B (one-wave diagrams, node-slot indexed like F and B; NULL:
    // not recorded).  Fpar[w] = 2 k + beta: the arc (node k of the level above, beta) whose value is
    // F(w) (lowest code on ties), written by the forward sweeps that the reverse sweeps read
    // (FWD_UPDATE_REC, FWD_SWEEP_LAM).  Bch[v] = child code | beta << 15: the arc that attains B(v) (lo
    // on ties), written by BWD_UPDATE_REC, BWD_STORE and BWD_STORE_BAR.
    uint16_t *Fpar;
    uint16_t *Bch;
};

struct ClassLaunch {
    int P;         // team size (lanes per diagram)
    int RMAX;      // max rows (of 64 slots) per level for this class
    int WL;        // max level width in the class
    int WB;        // LDS floats per team per node buffer: WL + 2 terminals, rounded up to P
    int NL;        // max levels of a tile in the class
    int wpb_f, wpb_b;  // waves per workgroup of the forward / backward kernels
    int wpb_af, wpb_ab;  // waves per workgroup of the push-form / pull-form adjoint sweeps
    int grid_f, grid_b;  // workgroups of the pass kernels (0: one wave per tile; else resident waves walk the tiles)
    int64_t tile0, ntiles;
    int64_t nodes, edges, rows;  // real (unpadded) counts covered by one launch, for byte accounting
};

// LDS words (4 bytes) one wavefront of the forward / backward pass kernels uses.
// per wave: two node buffers (2 * WB * G) and the level table (NL * G + NL)
// per wave of the smoothed-feature kernel: two node buffers and the level table
constexpr int lds_words_features(int P, int WB, int NL) { return 2 * WB * (64 / P) + NL * ((64 / P) + 1); }
// Smoothed energies (E_out[row], may be NULL) and Gibbs marginals (p_out, canonical) of one class at
// temperature tau, at lambda (bar = 0) or lambda + alpha*S (bar = 1); Q: node array for the
// per-node arc probabilities that the up sweep hands to the down sweep.
hipError_t launch_smooth(const DevTables &t, const ClassLaunch &c, float *Q, float tau, int bar, float *E_out,
                         float *p_out, hipStream_t s);

// Every kernel of the solver is compiled for workgroups of at most 256 threads (4 waves).
constexpr int kMaxWavesPerBlock = 4;
// edge slots per thread of the per-slot gathers of S (alpha * S, S per edge)
constexpr int kSlotsPerThread = 4;

constexpr int lds_words_pass(int P, int WB, int NL) {  // constexpr: usable in device code too
    return 2 * WB * (64 / P) + NL * ((64 / P) + 1);
}
// One-wave diagrams (P = 64) use pass kernels whose node buffers always hold RMAX whole rows
// plus 64 slots (terminal sentinels; one sink slot per lane for arcs into a terminal); a
// wave's share is a multiple of 4 words, so 16-byte LDS accesses stay aligned.
constexpr int node_buf_w(int RMAX) { return RMAX * 64 + 64; }
constexpr int lds_words_pass_w(int RMAX, int NL) { return 2 * node_buf_w(RMAX) + ((2 * NL + 3) & ~3); }
// the one-wave backward kernels: one node buffer (updated in place) and the level table
constexpr int lds_words_bwd_w(int RMAX, int NL) { return node_buf_w(RMAX) + ((2 * NL + 3) & ~3); }
// The forward sweeps that record argmin parent codes keep the next level's costs as 64-bit keys
// (cost, code): one node buffer more.
// Their level table (two words per level) stays in registers when the tile has at most
// kParRegLevels levels (lane k holds levels k, k + 64, ...), and takes LDS only beyond.
constexpr int kParRegLevels = 256;
constexpr int lds_words_pass_w_par(int RMAX, int NL) {
    return 3 * node_buf_w(RMAX) + (NL <= kParRegLevels ? 0 : ((2 * NL + 3) & ~3));
}
// LDS words per wave of the pass kernels of a class
constexpr int lds_words_pass_c(int P, int RMAX, int WB, int NL) {
    return P == 64 ? lds_words_pass_w(RMAX, NL) : lds_words_pass(P, WB, NL);
}

#define DD_CLASSES(X) \
    X(1, 4) X(2, 4) X(4, 4) X(8, 4) X(16, 4) X(32, 4) X(64, 4) X(64, 8) X(64, 12) X(64, 16) X(64, 24) X(64, 32) \
    X(64, 64)

// per wave of the adjoint sweeps: push form = cost and adjoint of one level, bids; pull form =
// staged B and the adjoints of two levels; both + the level table
constexpr int lds_words_adj_F(int P, int WB, int NL) { return 3 * WB * (64 / P) + NL * ((64 / P) + 1); }
constexpr int lds_words_adj_B(int P, int WB, int NL) { return 3 * WB * (64 / P) + NL * ((64 / P) + 1); }
// one-wave diagrams (P = 64), pull form: staged B and the adjoints of two levels in node buffers
// of RMAX rows + 64 slots, then the level table
constexpr int lds_words_adj_B_w(int RMAX, int NL) { return 3 * node_buf_w(RMAX) + ((2 * NL + 3) & ~3); }
// one-wave diagrams, push form: cost, adjoint and bids of a level, the list of nodes with an arc
// into a nonzero adjoint (node, children, cost), then the level table
constexpr int kAdjListW = 64;
// The narrow update passes form alpha * S themselves when the instance has no one-wave class and S
// fits one XCD's L2: they gather S_i per edge inside their hop chain, which pays while that gather
// hits L2; otherwise a separate launch, which gathers at full occupancy, is faster.
constexpr int64_t kFormAsMaxBytes = 4 << 20;
constexpr int lds_words_adj_F_w(int RMAX, int NL) {
    return 3 * node_buf_w(RMAX) + 3 * kAdjListW + ((2 * NL + 3) & ~3);
}
// the recording forward sweeps launch with the push-form sweep's waves per workgroup
static_assert(lds_words_pass_w_par(32, 1024) <= lds_words_adj_F_w(32, 1024), "recording sweep LDS");
constexpr int lds_words_adj_F_c(int P, int RMAX, int WB, int NL) {
    return P == 64 ? lds_words_adj_F_w(RMAX, NL) : lds_words_adj_F(P, WB, NL);
}
constexpr int lds_words_adj_B_c(int P, int RMAX, int WB, int NL) {
    return P == 64 ? lds_words_adj_B_w(RMAX, NL) : lds_words_adj_B(P, WB, NL);
}

// Arrays of the reverse sweeps (edge-slot indexed unless noted).
struct AdjTables {
    const float *lam_src;   // multipliers of a fixed-side sweep: the pass input (plus alpha*S when flushed)
    const float *dlam_out;  // adjoint of the pass-output multipliers
    const float *dM_out;    // adjoint of the pass-output M
    const float *Se;        // S of each edge's variable (update sweeps)
    float *dlam_in;         // adjoint of the pass-input multipliers (set by the update sweep, added to by the fixed one)
    float *g;               // dlambda' * alpha, summed per variable into dS
    float *dalpha, *domega; // accumulated over passes
    int32_t *rec_idx;       // [2 * slots] argmin node indices handed from one sweep to the other (-1: none)
    float *rec_val;         // [2 * slots] the adjoint values that go with them
    const int32_t *mrec;    // the replayed (or stored) pass's argmin records (update sweeps of one-wave
    const float *mdiff;     // diagrams), layout as in DevTables
    const float *seed;      // when set, the adjoint of B(root) is read here instead of the seed argument
                            // (a launch replayed from a graph then takes the value of the moment)
};

enum AdjSweep { ADJ_F_UPDATE = 0, ADJ_F_FIXED = 1, ADJ_B_UPDATE = 2, ADJ_B_FIXED = 3 };

// One reverse sweep over the tiles of a class.  bar: fixed pull sweeps use lam_src + alpha*S;
// recs: fixed sweeps add the records of the update sweep; seed: adjoint of B(root) (pull form).
// dense != 0: one-wave sweeps route every level node by node (the path of overflowing lists).
hipError_t launch_adj(const DevTables &t, const AdjTables &a, const ClassLaunch &c, int which, int bar, int recs,
                      float seed, int dense, hipStream_t s);
// Se[slot] = S[evar[slot]] (0 on padding)
hipError_t launch_edge_S(const int32_t *evar, const float *S, float *Se, int64_t slots, hipStream_t s);
hipError_t launch_flush_adj(const int32_t *evar, const float *S, const float *alpha, const float *dlam, float *dalpha,
                            float *g, int64_t slots, hipStream_t s);
hipError_t launch_dc(const int32_t *var_ptr, const int32_t *var_slots, const float *dlam, const float *c, float seed,
                     float *dc, int n, hipStream_t s);
hipError_t launch_softmax_vjp(const int32_t *var_ptr, const int32_t *var_canon, const float *alpha,
                              const float *dalpha, float *out, int n, hipStream_t s);
hipError_t launch_fill(float *x, float v, int64_t n, hipStream_t s);
// Alg. 3's output transforms and their adjoint (canonical arrays; th/t and dt/dth may be NULL).
hipError_t launch_param_transform(const int32_t *var_ptr, const int32_t *var_canon, const float *wh, const float *ah,
                                  const float *th, float *w, float *al, float *t, int n, hipStream_t s);
hipError_t launch_param_transform_vjp(const int32_t *var_ptr, const int32_t *var_canon, const float *w,
                                      const float *al, const float *dw, const float *da, const float *dt, float *dwh,
                                      float *dah, float *dth, int n, hipStream_t s);
// eq. 2 on the slot-ordered multipliers; th canonical
hipError_t launch_nonparam_update(const int32_t *var_ptr, const int32_t *var_canon, const int32_t *canon2slot,
                                  const float *th, float *lam, int n, hipStream_t s);
hipError_t launch_uncovered(const int32_t *var_ptr, const float *c, float *out, int n, hipStream_t s);

hipError_t launch_fwd(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s);
// Workgroups of the update-pass kernel of class c (at its waves per workgroup) one CU holds at once.
int pass_blocks_per_cu(const ClassLaunch &c, bool fwd);
// out[q] = fp64 sum over x[seg[q] .. seg[q+1]) (of min(0, x) when neg_part), fixed order, q < k.
hipError_t launch_seg_sum(const float *x, const int64_t *seg, int k, int neg_part, double *out, hipStream_t s);
hipError_t launch_bwd(const DevTables &t, const ClassLaunch &c, int mode, hipStream_t s);
bool class_supported(int P, int RMAX);

// S_i = sum over the CSR list of edge slots of variable i of M[slot]: `team` lanes per variable (1, 2,
// 4, 8 or 16), strided partial sums in list order, then a fixed butterfly (same bits on every call).
hipError_t launch_deferred_sum(const int32_t *var_ptr, const int32_t *var_slots, const float *M, float *S, int n,
                               int team, hipStream_t s);
// aS[slot] = alpha[slot] * S[evar[slot]] for every edge slot (0 on padding); with Se, also
// Se[slot] = S[evar[slot]] (the S per edge that the reverse sweeps read).
hipError_t launch_edge_alpha_s(const int32_t *evar, const float *alpha, const float *S, float *aS, float *Se,
                               int64_t slots, hipStream_t s);
// lambda[slot] = c_i / |J_i|, M[slot] = 0 for every canonical edge.
hipError_t launch_init_lambda(const int32_t *canon2slot, const int32_t *evar, const int32_t *var_ptr, const float *c,
                              float *lam, float *M, int64_t E, hipStream_t s);
// dst[canon2slot[e]] = src[e]
hipError_t launch_scatter(const int32_t *canon2slot, const float *src, float *dst, int64_t E, hipStream_t s);
// ad[i] = a[i], bd[i] = b[i] for i < n (one launch)
hipError_t launch_copy2(const float *a, float *ad, const float *b, float *bd, int64_t n, hipStream_t s);
// dst[e] = src[canon2slot[e]] (+ add[canon2slot[e]] when add is not NULL)
hipError_t launch_gather(const int32_t *canon2slot, const float *src, float *dst, int64_t E, const float *add,
                         hipStream_t s);
// softmax over each variable's edges; inputs/outputs canonical, var_canon is the CSR of canonical edge ids
hipError_t launch_seg_softmax(const int32_t *var_ptr, const int32_t *var_canon, const float *x, float *y, int n,
                              hipStream_t s);
// *out = add + sum of x[0..n) (or of min(0, x) when neg_part), fp64, fixed order; partial holds
// kSumBlocks doubles of scratch.
constexpr int kSumBlocks = 1024;
hipError_t launch_sum(const float *x, int64_t n, int neg_part, double *partial, double *out, hipStream_t s,
                      double add = 0.0);
// *out = order-independent 64-bit fingerprint of the state (a[0..n), b[0..n)); partial holds kSumBlocks
// words of scratch.  launch_hash_check sets *flag = 1 when *x != *y (and leaves it otherwise).
hipError_t launch_state_hash(const float *a, const float *b, int64_t n, uint64_t *partial, uint64_t *out,
                             hipStream_t s);
hipError_t launch_hash_check(const uint64_t *x, const uint64_t *y, int32_t *flag, hipStream_t s);
// validity check of parameters: flags[0] |= omega outside [0,1] or non-finite, flags[1] |= alpha < 0 or non-finite
hipError_t launch_check_params(const float *omega, const float *alpha, int64_t E, int32_t *flags, hipStream_t s);

}  // namespace dd
