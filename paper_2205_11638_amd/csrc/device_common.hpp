// device_common.hpp -- device helpers shared by the pass kernels and the adjoint kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>

#include "kernels.hpp"

namespace dd {
namespace dev {

constexpr float kInf = __builtin_huge_valf();

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Values known to be equal on every lane of the wavefront, made scalar for the compiler.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// min over the P lanes of a team (P a power of two, teams aligned to P lanes), result in
// every lane of the team.  Within 16-lane rows: DPP quad permutes and row mirrors; across
// rows: lane reads (P = 64) or one cross-row shuffle (P = 32).
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int P>
__device__ __forceinline__ float team_min(float v) {
    if (P >= 2) v = fminf(v, dpp<0xB1>(v));    // quad_perm [1,0,3,2]: lanes i, i^1
    if (P >= 4) v = fminf(v, dpp<0x4E>(v));    // quad_perm [2,3,0,1]: lanes i, i^2
    if (P >= 8) v = fminf(v, dpp<0x141>(v));   // row_half_mirror: the two quads of 8 lanes
    if (P >= 16) v = fminf(v, dpp<0x140>(v));  // row_mirror: the two halves of 16 lanes
    if (P == 32) v = fminf(v, __shfl_xor(v, 16));
    if (P == 64) {
        const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
        const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
        const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
        const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
        v = fminf(fminf(r0, r1), fminf(r2, r3));
    }
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

// Per-wave LDS layout shared by the pass kernels (all entries 4 bytes):
//   [X: WB*G floats] [Y: WB*G floats] [meta: NL*G ints] [off: NL ints]
// meta[l*G + g] = width of team g at level l | rows of level l << 16; off[l] = level offset.
// Node buffers are interleaved over teams (index k*G + g) and hold WB >= width + 2 entries
// per team: the two past the level's width are the terminals (0-terminal = +inf, 1-terminal
// = 0), so a child code indexes the buffer directly, with no branch.  Slots past a team's
// width inside a level's rows are padding whose child codes both point at the 0-terminal,
// so every global access of a level is unconditional and in bounds.
template <int G>
__device__ __forceinline__ void preload_meta(const DevTables &T, const TileCtx &tc, int lane, int *meta, int *off) {
    const int n = tc.nlev * G;
    for (int i = lane; i < n; i += 64) meta[i] = T.widths[tc.wbase + i] | (T.lev_rows[tc.lbase + i / G] << 16);
    for (int l = lane; l < tc.nlev; l += 64) off[l] = T.lev_off[tc.lbase + l];
    wave_sync();
}

__device__ __forceinline__ void lds_fmin(float *a, float v) {
    __hip_atomic_fetch_min(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// ------------------------------------------------------------------------------------------
// Forward pass.  X = F of the current level (min-accumulated for the next one), Y = B of the
// next level staged from global memory.
// ------------------------------------------------------------------------------------------
// One-wave diagrams (P = 64) are stored nearly compactly: level l+1 starts at the first
// multiple of 4 nodes after the last node of level l, so the last row of a level also reads a
// few slots of the next level (or of the slack after the array).  Those lanes are masked on
// that row only: their topology is replaced by two 0-terminal arcs and their stores are
// skipped.  Narrower teams use levels padded to whole rows, whose padding slots already hold
// 0-terminal arcs.
template <int P>
__device__ __forceinline__ bool in_level(int r, int R, int lane, int W) {
    return P < 64 || r < R - 1 || lane < W - r * 64;
}

// Per-level scalars of a tile: this team's width, the level's rows and first slot.
struct Lev {
    int W, R;
    int64_t base;
};

// sum / integer min over the P lanes of a team, same lane pattern as team_min
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}

template <int P>
__device__ __forceinline__ float team_sum(float v) {
    if (P >= 2) v += dpp<0xB1>(v);
    if (P >= 4) v += dpp<0x4E>(v);
    if (P >= 8) v += dpp<0x141>(v);
    if (P >= 16) v += dpp<0x140>(v);
    if (P == 32) v += __shfl_xor(v, 16);
    if (P == 64) {
        const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
        const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
        const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
        const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
        v = (r0 + r1) + (r2 + r3);
    }
    return v;
}

template <int P>
__device__ __forceinline__ int team_min_i(int v) {
    if (P >= 2) v = min(v, dpp_i<0xB1>(v));
    if (P >= 4) v = min(v, dpp_i<0x4E>(v));
    if (P >= 8) v = min(v, dpp_i<0x141>(v));
    if (P >= 16) v = min(v, dpp_i<0x140>(v));
    if (P == 32) v = min(v, __shfl_xor(v, 16));
    if (P == 64) {
        const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
        const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
        v = min(min(r0, r1), min(r2, r3));
    }
    return v;
}

__device__ __forceinline__ void lds_fadd(float *a, float v) {
    __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

__device__ __forceinline__ void lds_imin(int *a, int v) {
    __hip_atomic_fetch_min(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Dispatch on a uniform count into bodies unrolled for exactly that count, and range-checked
// buffer resources (an access past a resource's size loads 0 without touching memory, or is
// dropped), so prefetches and stores can be issued unconditionally.
template <int N>
struct Count {
    static constexpr int value = N;
};

template <int LO, int HI, typename Fn>
__device__ __forceinline__ void with_count(int n, Fn &&fn) {
    if constexpr (LO == HI) {
        fn(Count<LO>{});
    } else {
        constexpr int MID = (LO + HI) / 2;
        if (n <= MID) with_count<LO, MID>(n, fn);
        else with_count<MID + 1, HI>(n, fn);
    }
}

// gfx9-family buffer resource word 3: 32-bit data format, raw (byte) addressing, range checked
constexpr int kBufWord3 = 0x00020000;
using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ rsrc_t buf(const void *base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, bytes, kBufWord3);
}
__device__ __forceinline__ u32x4 ld4(rsrc_t r, int off) { return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0); }
__device__ __forceinline__ f32x4 ld4f(rsrc_t r, int off) { return __builtin_bit_cast(f32x4, ld4(r, off)); }
__device__ __forceinline__ void st4(rsrc_t r, int off, f32x4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, 0, 0);
}
__device__ __forceinline__ uint32_t ld1(rsrc_t r, int off) { return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0); }
__device__ __forceinline__ float ld1f(rsrc_t r, int off) { return __uint_as_float(ld1(r, off)); }
__device__ __forceinline__ void st1(rsrc_t r, int off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, 0);
}
__device__ __forceinline__ f32x4 &lds4(float *base, int byte_off) { return *(f32x4 *)((char *)base + byte_off); }

// 16 * lane, made anew in each hop body: an offset shared by the bodies (or loop invariant)
// would be computed once per group ahead of them and held in one register per group, instead
// of folding the group into the instruction's offset field
__device__ __forceinline__ int lane16(int lane) {
    int v = lane * 16;
    __asm__ volatile("" : "+v"(v));
    return v;
}

// Inclusive sum over the lanes of the wave, in lane order (unsigned, wrapping): shifts by 1, 2, 4
// and 8 within each row of 16 lanes, then the row broadcasts of the wave64 DPP forms (lane 15 of
// each row into the next row for rows 1 and 3, then lane 31 into rows 2 and 3).  Lanes whose
// source falls outside take the first operand, 0.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);
    return v;
}

// Child codes (lo | hi << 16) of a lane's four nodes in each of the first Q groups of a one-wave
// level, from the level's byte codes (DevTables::tcode, one 32-bit word per lane and group, as
// loaded at byte 256 q + 4 lane of the level) and the codes of its first node (cb).  The nibbles
// are steps from the node before, so a node's codes are cb plus the steps of every node up to it:
// the lane's own steps by byte-wise prefix sums, the lanes before it by a scan of the packed lane
// totals (lo and hi in separate halves: sums stay far below 2^16), the groups before it by the scan
// totals.  Lanes past the level's width decode the bytes that follow it; their codes are replaced
// by the callers, and they only feed lanes after them.  last: the next level is empty, so the bytes
// describe 1 - code.  A level of kRawLevel reads its 4-byte codes from traw instead.
template <int Q, int QM>
__device__ __forceinline__ void child_codes(const uint32_t (&cw)[QM], uint32_t cb, bool last, rsrc_t traw, int lane,
                                            u32x4 (&t)[Q]) {
    if (cb == 0xFFFFFFFFu) {
        const int l16 = lane16(lane);
#pragma unroll
        for (int q = 0; q < Q; ++q) t[q] = ld4(traw, l16 + q * 1024);
        return;
    }
    uint32_t base = cb, k8 = 8, k16 = 16;
    // shift counts the compiler cannot see: it would fold the shifts and adds into a multiply by
    // 0x01010101, a quarter-rate instruction, instead of two shift-and-adds
    __asm__ volatile("" : "+s"(k8), "+s"(k16));
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const uint32_t w = cw[q];
        uint32_t wl = w & 0x0F0F0F0Fu, wh = (w >> 4) & 0x0F0F0F0Fu;
        wl += wl << k8;
        wl += wl << k16;
        wh += wh << k8;
        wh += wh << k16;
        const uint32_t tot = (wl >> 24) | ((wh >> 24) << 16);
        const uint32_t inc = wave_incl_sum(tot);
        const uint32_t x = base + inc - tot;
        if (q + 1 < Q) base += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
        // node j: byte j of the lo sums into bits 0-7, byte j of the hi sums into bits 16-23
#pragma unroll
        for (int j = 0; j < 4; ++j)
            t[q][j] = x + __builtin_amdgcn_perm(wh, wl, (uint32_t)j | 0x0C00u | (uint32_t)(4 + j) << 16 | 0x0C000000u);
    }
    if (last)
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) t[q][j] = 0x00010001u - t[q][j];
}

// bytes of a level's node rows (loads) and of its nodes rounded up to whole lane chunks (stores)
__device__ __forceinline__ int row_bytes(const Lev &c) { return c.R * 256; }
__device__ __forceinline__ int node_bytes(const Lev &c) { return ((c.W + 3) & ~3) * 4; }
__device__ __forceinline__ int groups(const Lev &c) { return (c.R + 3) >> 2; }
// bytes of a level's rows of byte codes (DevTables::tcode)
__device__ __forceinline__ int code_row_bytes(const Lev &c) { return c.R * 64; }


typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st2(rsrc_t r, int off, uint32_t a, uint32_t b) {
    const u32x2 v = {a, b};
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 0);
}
__device__ __forceinline__ u32x2 ld2(rsrc_t r, int off) { return __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0); }
// Argmin codes (2 bytes per node) of one-wave diagrams: a lane's four nodes 4 lane + j of group q
// are the 8 bytes at 512 q + 8 lane of the level's code row; code j is half j & 1 of word j >> 1.
__device__ __forceinline__ int lane8(int lane) {
    int v = lane * 8;
    __asm__ volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ int code_bytes(const Lev &c) { return ((c.W + 3) & ~3) * 2; }
__device__ __forceinline__ uint32_t code_at(const u32x2 &w, int j) { return (w[j >> 1] >> (16 * (j & 1))) & 0xFFFFu; }
__device__ __forceinline__ void lds_umin(uint32_t *a, uint32_t v) {
    __hip_atomic_fetch_min(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
// A cost and a 16-bit code as one 64-bit key whose unsigned order is (cost, code): the cost's bits
// are mapped to an unsigned integer of the same order (sign bit set for non-negative values, all
// bits flipped for negative ones), so one integer min gives the least cost and, among equal costs,
// the lowest code.
__device__ __forceinline__ uint64_t cost_key(float v, uint32_t code) {
    uint32_t u = __float_as_uint(v);
    if (u == 0x80000000u) u = 0u;  // -0 and +0 are one cost
    const uint32_t o = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((uint64_t)o << 32) | code;
}
__device__ __forceinline__ float key_cost(uint64_t k) {
    const uint32_t o = (uint32_t)(k >> 32);
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}
__device__ __forceinline__ void lds_umin64(uint64_t *a, uint64_t v) {
    __hip_atomic_fetch_min(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
// Workgroups go to the chip's 8 XCDs round-robin (workgroup b to XCD b mod 8), each XCD with an L2
// of its own.  xcd_block gives the workgroups on XCD x the x-th contiguous eighth of the index range
// (a bijection on [0, nb) for nb a multiple of 8), so gathers from items that are near each other in
// that range share one L2.  Launches pad the grid to a multiple of 8; the items past the range exit.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) { return (b & 7) * (nb >> 3) + (b >> 3); }
inline unsigned xcd_grid(int64_t blocks) { return (unsigned)((blocks + 7) & ~(int64_t)7); }
// 32 * lane (a lane's four 64-bit keys of a 256-node group), made anew like lane16
__device__ __forceinline__ int lane32(int lane) {
    int v = lane * 32;
    __asm__ volatile("" : "+v"(v));
    return v;
}

// Recording update passes (one-wave diagrams): each lane visits its nodes in increasing index and
// keeps the first one attaining its running minimum m of a min-marginal (call before m takes v),
// with the child code the minimum went through.
__device__ __forceinline__ void argmin_step(float v, float m, int k, int child, int &kk, int &hh) {
    if (v < m || (v == m && kk == INT_MAX)) {
        kk = k;
        hh = child;
    }
}

// The lowest node attaining each min-marginal of the hop (lm: the lane's minima, M: the wave's,
// k / h: the lane's first attaining node and its child) with its child code, and m^1 - m^0 as the
// pass formed it; lane 0 stores them (record offset 2 out, difference offset out).
__device__ __forceinline__ void record_argmins(rsrc_t rec_r, rsrc_t md_r, int out, float lm0, float M0, int k0,
                                               int h0, float lm1, float M1, int k1, int h1, float d) {
    const int K0 = team_min_i<64>(lm0 == M0 ? k0 : INT_MAX);
    const int K1 = team_min_i<64>(lm1 == M1 ? k1 : INT_MAX);
    const int c0 = __builtin_amdgcn_readlane(h0, __builtin_ctzll(__builtin_amdgcn_ballot_w64(k0 == K0)));
    const int c1 = __builtin_amdgcn_readlane(h1, __builtin_ctzll(__builtin_amdgcn_ballot_w64(k1 == K1)));
    st2(rec_r, 2 * out, (uint32_t)K0 | ((uint32_t)c0 << 16), (uint32_t)K1 | ((uint32_t)c1 << 16));
    st1(md_r, out, d);
}

// the records' resources over a tile's edges (no size when not recording)
template <bool REC>
__device__ __forceinline__ rsrc_t rec_buf(const DevTables &T, const TileCtx &tc, int nlev) {
    if constexpr (REC) return buf(T.mrec + 2 * (int64_t)tc.ebase, nlev * 8);
    else return buf(T.lam, 0);
}
template <bool REC>
__device__ __forceinline__ rsrc_t mdiff_buf(const DevTables &T, const TileCtx &tc, int nlev) {
    if constexpr (REC) return buf(T.mdiff + tc.ebase, nlev * 4);
    else return buf(T.lam, 0);
}


// The same for a team of P lanes of a narrower tile (node k = r P + p): the lowest attaining node
// and its child code are reduced as one key (node << 12 | child; nodes and child codes of these
// tiles stay below 4096), and the team's first lane stores at its edge slot's offset off (4 bytes
// per slot; other lanes pass an offset past the ne bytes of the tile's slots).
template <int P>
__device__ __forceinline__ void record_argmins_team(const DevTables &T, int ebase, int ne, int off, float lm0,
                                                    float M0, int k0, int h0, float lm1, float M1, int k1, int h1,
                                                    float d) {
    const int key0 = team_min_i<P>(lm0 == M0 && k0 != INT_MAX ? (k0 << 12) | h0 : INT_MAX);
    const int key1 = team_min_i<P>(lm1 == M1 && k1 != INT_MAX ? (k1 << 12) | h1 : INT_MAX);
    st2(buf(T.mrec + 2 * (int64_t)ebase, 2 * ne), 2 * off, (uint32_t)(key0 >> 12) | ((uint32_t)(key0 & 0xFFF) << 16),
        (uint32_t)(key1 >> 12) | ((uint32_t)(key1 & 0xFFF) << 16));
    st1(buf(T.mdiff + ebase, ne), off, d);
}

// The sum of x[idx[q]] over q = a + u, a + u + TS, ... below b, added in that order from 0 (lane u of
// a team of TS lanes summing one CSR list).  Up to four indices are loaded, then their four values,
// before any is added: a long list waits for a quarter of the dependent load round trips of the plain
// loop, and the adds (so the bits) are the plain loop's.
template <int TS>
__device__ __forceinline__ float strided_gather_sum(const int32_t *__restrict__ idx, const float *__restrict__ x,
                                                    int a, int b, int u) {
    auto ix = [&](int q) { return idx[q]; };
    float s = 0.f;
    int q = a + u;
    for (; q + 3 * TS < b; q += 4 * TS) {
        const int e0 = ix(q), e1 = ix(q + TS), e2 = ix(q + 2 * TS), e3 = ix(q + 3 * TS);
        const float x0 = x[e0], x1 = x[e1], x2 = x[e2], x3 = x[e3];
        s += x0;
        s += x1;
        s += x2;
        s += x3;
    }
    if (q < b) {  // at most three left
        const bool h1 = q + TS < b, h2 = q + 2 * TS < b;
        const int e0 = ix(q), e1 = h1 ? ix(q + TS) : 0, e2 = h2 ? ix(q + 2 * TS) : 0;
        const float x0 = x[e0], x1 = h1 ? x[e1] : 0.f, x2 = h2 ? x[e2] : 0.f;
        s += x0;
        if (h1) s += x1;
        if (h2) s += x2;
    }
    return s;
}

}  // namespace dev
}  // namespace dd
