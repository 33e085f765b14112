// dd_api.cpp -- C ABI: problem validation, parallel diagram compilation, tile packing,
// device memory and the launch sequences of the hot path.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/dd.h"
#include "bdd.hpp"
#include "instance.hpp"
#include "kernels.hpp"

using namespace dd;
using namespace ddi;

namespace ddi {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace ddi

namespace {

int worker_count() {
    const char *env = getenv("DD_THREADS");
    int n = env ? atoi(env) : (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(n, 64));
}

template <class F>
void parallel_for(int64_t n, int64_t chunk, F f) {
    int nw = (int)std::min<int64_t>(worker_count(), (n + chunk - 1) / std::max<int64_t>(chunk, 1));
    if (nw <= 1) {
        for (int64_t i = 0; i < n; ++i) f(i, 0);
        return;
    }
    std::atomic<int64_t> next(0);
    std::vector<std::thread> th;
    for (int w = 0; w < nw; ++w)
        th.emplace_back([&, w] {
            for (;;) {
                int64_t a = next.fetch_add(chunk);
                if (a >= n) break;
                int64_t b = std::min(n, a + chunk);
                for (int64_t i = a; i < b; ++i) f(i, w);
            }
        });
    for (auto &t : th) t.join();
}

int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Sorted copy of the problem's rows (canonical order: variables ascending in each row).
struct SortedRows {
    std::vector<int64_t> ptr;
    std::vector<int32_t> col, coef;
};

int validate_and_sort(const dd_problem *p, SortedRows &sr) {
    if (!p) return fail(DD_E_ARG, "problem is NULL");
    if (p->n < 0 || p->m < 0) return fail(DD_E_ARG, "negative n or m");
    if (p->n > 0 && !p->c) return fail(DD_E_ARG, "c is NULL");
    if (!p->row_ptr) return fail(DD_E_ARG, "row_ptr is NULL");
    if (p->row_ptr[0] != 0) return fail(DD_E_ARG, "row_ptr[0] must be 0");
    for (int j = 0; j < p->m; ++j)
        if (p->row_ptr[j + 1] < p->row_ptr[j]) return fail(DD_E_ARG, "row_ptr decreases at row %d", j);
    const int64_t nnz = p->row_ptr[p->m];
    if (nnz > 0 && (!p->col || !p->coef)) return fail(DD_E_ARG, "col or coef is NULL");
    if (p->m > 0 && (!p->sense || !p->rhs)) return fail(DD_E_ARG, "sense or rhs is NULL");
    if (nnz >= ((int64_t)1 << 31) - 1) return fail(DD_E_UNSUPPORTED, "more than 2^31 edges");
    for (int i = 0; i < p->n; ++i)
        if (!std::isfinite(p->c[i])) return fail(DD_E_PARAM, "c[%d] is not finite", i);
    sr.ptr.assign(p->row_ptr, p->row_ptr + p->m + 1);
    sr.col.resize(nnz);
    sr.coef.resize(nnz);
    std::atomic<int> status(DD_OK);
    std::atomic<int> bad_row(-1);
    parallel_for(p->m, 256, [&](int64_t j, int) {
        const int64_t a = p->row_ptr[j], b = p->row_ptr[j + 1];
        if (p->sense[j] < -1 || p->sense[j] > 1) {
            status = DD_E_ARG;
            bad_row = (int)j;
            return;
        }
        std::vector<std::pair<int32_t, int32_t>> v;
        v.reserve(b - a);
        for (int64_t q = a; q < b; ++q) {
            if (p->col[q] < 0 || p->col[q] >= p->n || p->coef[q] == 0) {
                status = DD_E_ARG;
                bad_row = (int)j;
                return;
            }
            v.emplace_back(p->col[q], p->coef[q]);
        }
        std::sort(v.begin(), v.end());
        for (size_t t = 0; t < v.size(); ++t) {
            if (t && v[t].first == v[t - 1].first) {
                status = DD_E_ARG;
                bad_row = (int)j;
                return;
            }
            sr.col[a + t] = v[t].first;
            sr.coef[a + t] = v[t].second;
        }
    });
    if (status != DD_OK)
        return fail(DD_E_ARG, "row %d: bad sense, variable out of range, zero coefficient or duplicate variable",
                    (int)bad_row);
    return DD_OK;
}

constexpr int64_t kLdsPerCU = 160 * 1024;

struct HostPlan {
    std::vector<ClassLaunch> classes;
    // tiles
    std::vector<int64_t> node_base;
    std::vector<int32_t> edge_base, nlev, lev_base, w_base, bdd;
    std::vector<int32_t> lev_off, lev_rows;
    std::vector<uint32_t> lev_code;  // codes of each level's first node, or kRawLevel
    std::vector<uint16_t> widths;
    std::vector<uint8_t> tcode;      // byte codes of one-wave levels (node-slot indexed)
    int64_t coded_levels = 0, raw_levels = 0;
    std::vector<int32_t> tile_P;
    int64_t node_slots = 0, edge_slots = 0, node_alloc = 0;
    // edges
    std::vector<int32_t> canon2slot, slot2canon, evar;
    std::vector<int32_t> var_ptr, var_slots, var_canon;
    std::vector<int32_t> var_perm;  // the library's number of each variable (see build_plan)
};

}  // namespace


namespace ddi {

template <class T_>
int upload(dd_instance *h, T_ **dst, const std::vector<T_> &src, hipStream_t s) {
    int st = h->alloc(dst, src.size());
    if (st) return st;
    if (!src.empty()) HIP_TRY(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T_), hipMemcpyHostToDevice, s));
    return DD_OK;
}

// Byte codes of the one-wave levels (DevTables::tcode, lev_code): nodes are numbered in increasing
// partial sum, so a level's lo and hi child codes are non-decreasing in the node number, with the
// 0-terminal (code Wn) after every node of the level below, and they mostly step by 0 or 1.  Each
// node gets the two steps from the node before as nibbles; the first node's codes go to lev_code.
// The last level (codes 0 = 0-terminal, 1 = 1-terminal) is coded as 1 - code, which is
// non-decreasing there too.  A level whose steps fall outside 0..15 keeps kRawLevel and is read
// from the 4-byte codes.
void encode_topology(HostPlan &hp, const std::vector<uint32_t> &topo) {
    hp.lev_code.assign(hp.lev_off.size(), kRawLevel);
    hp.tcode.assign((size_t)hp.node_alloc, 0);
    const int64_t ntiles = (int64_t)hp.nlev.size();
    std::vector<int64_t> coded(ntiles, 0), raw(ntiles, 0);
    parallel_for(ntiles, 64, [&](int64_t t, int) {
        if (hp.tile_P[t] != 64) return;
        const int nl = hp.nlev[t];
        for (int l = 0; l < nl; ++l) {
            const int li = hp.lev_base[t] + l;
            const int64_t base = hp.node_base[t] + hp.lev_off[li];
            const int W = hp.widths[hp.w_base[t] + l];
            const bool last = l + 1 == nl;
            auto code = [&](int k) {
                const uint32_t c = topo[(size_t)(base + k)];
                return last ? 0x00010001u - c : c;
            };
            bool ok = W > 0;
            for (int k = 1; k < W && ok; ++k) {
                const uint32_t a = code(k - 1), b = code(k);
                const int dl = (int)(b & 0xFFFFu) - (int)(a & 0xFFFFu), dh = (int)(b >> 16) - (int)(a >> 16);
                ok = dl >= 0 && dl <= 15 && dh >= 0 && dh <= 15;
            }
            if (!ok) {
                ++raw[t];
                continue;
            }
            hp.lev_code[li] = code(0);
            for (int k = 1; k < W; ++k) {
                const uint32_t a = code(k - 1), b = code(k);
                hp.tcode[(size_t)(base + k)] = (uint8_t)(((b & 0xFFFFu) - (a & 0xFFFFu)) | (((b >> 16) - (a >> 16)) << 4));
            }
            ++coded[t];
        }
    });
    for (int64_t t = 0; t < ntiles; ++t) {
        hp.coded_levels += coded[t];
        hp.raw_levels += raw[t];
    }
}

int build_plan(const dd_problem *p, const SortedRows &sr, const std::vector<RowBdd> &bdds, int npl, int wpb,
               int lds_budget, const int32_t *row_group, HostPlan &hp, std::vector<uint32_t> &topo) {
    const int m = p->m;
    // class of every row
    std::vector<int> rP(m, 0), rR(m, 0);
    for (int j = 0; j < m; ++j) {
        const RowBdd &b = bdds[j];
        if (b.L == 0) continue;
        int P = std::min(64, next_pow2((b.max_width + npl - 1) / npl));
        int R = (b.max_width + P - 1) / P;
        int RMAX = 4;
        if (P == 64)
            for (int cand : {4, 8, 12, 16, 24, 32, 64, 1 << 30})
                if (cand >= R) {
                    RMAX = cand;
                    break;
                }
        if (!class_supported(P, RMAX))
            return fail(DD_E_UNSUPPORTED, "row %d: diagram width %d is wider than the kernels support (4096)", j,
                        b.max_width);
        rP[j] = P;
        rR[j] = RMAX;
    }
    // All one-wave diagrams share one launch (register tiles sized for the widest): a single
    // kernel per pass instead of one per width class, so no launch waits on another's tail.
    int wide = 0;
    for (int j = 0; j < m; ++j)
        if (rP[j] == 64) wide = std::max(wide, rR[j]);
    for (int j = 0; j < m; ++j)
        if (rP[j] == 64) rR[j] = wide;
    std::vector<int> order;
    for (int j = 0; j < m; ++j)
        if (bdds[j].L > 0) order.push_back(j);
    // within a class, rows of one locality group (a batch's programs, bucketed) stay together, so the
    // edge slots of a group are one stretch of the slot range; then longest diagrams first
    std::sort(order.begin(), order.end(), [&](int x, int y) {
        if (rP[x] != rP[y]) return rP[x] < rP[y];
        if (rR[x] != rR[y]) return rR[x] < rR[y];
        if (row_group && row_group[x] != row_group[y]) return row_group[x] < row_group[y];
        if (bdds[x].L != bdds[y].L) return bdds[x].L > bdds[y].L;
        if (bdds[x].max_width != bdds[y].max_width) return bdds[x].max_width > bdds[y].max_width;
        return x < y;
    });
    // tiles
    size_t i = 0;
    int64_t node_slots = 0, edge_slots = 0;
    while (i < order.size()) {
        const int P = rP[order[i]], RMAX = rR[order[i]], G = 64 / P;
        ClassLaunch cl{};
        cl.P = P;
        cl.RMAX = RMAX;
        cl.WL = 1;
        cl.tile0 = (int64_t)hp.nlev.size();
        size_t j = i;
        while (j < order.size() && rP[order[j]] == P && rR[order[j]] == RMAX) ++j;
        for (size_t t0 = i; t0 < j; t0 += G) {
            const size_t t1 = std::min(j, t0 + G);
            int nl = 0;
            for (size_t q = t0; q < t1; ++q) {
                cl.NL = std::max(cl.NL, bdds[order[q]].L);
                nl = std::max(nl, bdds[order[q]].L);
                cl.WL = std::max(cl.WL, bdds[order[q]].max_width);
                cl.nodes += (int64_t)bdds[order[q]].arcs.size();
                cl.edges += bdds[order[q]].L;
                cl.rows += 1;
            }
            hp.node_base.push_back(node_slots);
            if (edge_slots + (int64_t)nl * G >= ((int64_t)1 << 31)) return fail(DD_E_UNSUPPORTED, "too many edge slots");
            hp.edge_base.push_back((int32_t)edge_slots);
            hp.nlev.push_back(nl);
            hp.lev_base.push_back((int32_t)hp.lev_off.size());
            hp.w_base.push_back((int32_t)hp.widths.size());
            hp.tile_P.push_back(P);
            for (int g = 0; g < 64; ++g) hp.bdd.push_back(g < G && t0 + g < t1 ? order[t0 + g] : -1);
            int64_t off = 0;
            for (int l = 0; l < nl; ++l) {
                int R = 0, wmax = 0;
                for (int g = 0; g < G; ++g) {
                    int w = 0;
                    if (t0 + g < t1 && l < bdds[order[t0 + g]].L) w = bdds[order[t0 + g]].width[l];
                    hp.widths.push_back((uint16_t)w);
                    R = std::max(R, (w + P - 1) / P);
                    wmax = std::max(wmax, w);
                }
                if (off >= ((int64_t)1 << 31)) return fail(DD_E_UNSUPPORTED, "tile too large");
                if (R > RMAX) return fail(DD_E_UNSUPPORTED, "internal: level needs %d rows > %d", R, RMAX);
                hp.lev_off.push_back((int32_t)off);
                hp.lev_rows.push_back(R);
                // one-wave diagrams are stored nearly compactly (each level starts at a multiple
                // of 4 nodes, for 16-byte row accesses); teams of a narrower tile interleave, so
                // their levels are padded to whole rows
                off += P == 64 ? (int64_t)((wmax + 3) & ~3) : (int64_t)R * 64;
            }
            node_slots += off;
            edge_slots += (int64_t)nl * G;
        }
        cl.ntiles = (int64_t)hp.nlev.size() - cl.tile0;
        cl.WB = (cl.WL + 2 + P - 1) / P * P;
        // waves per workgroup: most resident waves per CU under the LDS budget per workgroup
        auto pick = [&](int64_t words) {
            const int64_t per_wave = words * 4;
            int best = 0, best_waves = -1;
            for (int w = 1; w <= kMaxWavesPerBlock; w *= 2) {
                if (w > wpb || w * per_wave > lds_budget) break;
                const int waves = (int)(kLdsPerCU / (w * per_wave)) * w;
                if (waves >= best_waves) {
                    best_waves = waves;
                    best = w;
                }
            }
            return best;
        };
        cl.wpb_f = pick(lds_words_pass_c(P, RMAX, cl.WB, cl.NL));
        cl.wpb_b = pick(lds_words_pass_c(P, RMAX, cl.WB, cl.NL));
        cl.wpb_af = pick(lds_words_adj_F_c(P, RMAX, cl.WB, cl.NL));
        cl.wpb_ab = pick(lds_words_adj_B_c(P, RMAX, cl.WB, cl.NL));
        if (!cl.wpb_f || !cl.wpb_b || !cl.wpb_af || !cl.wpb_ab)
            return fail(DD_E_UNSUPPORTED, "LDS need %lld bytes per wave exceeds the budget",
                        (long long)lds_words_adj_F_c(P, RMAX, cl.WB, cl.NL) * 4);
        hp.classes.push_back(cl);
        i = j;
    }
    hp.node_slots = node_slots;
    hp.node_alloc = node_slots + 64;  // the last row of a compact level may read up to 63 slots past it
    hp.edge_slots = edge_slots;
    // nodes
    topo.assign((size_t)hp.node_alloc, 0u);
    const int64_t ntiles = (int64_t)hp.nlev.size();
    parallel_for(ntiles, 64, [&](int64_t t, int) {
        const int P = hp.tile_P[t], G = 64 / P, nl = hp.nlev[t];
        for (int g = 0; g < G; ++g) {
            const int row = hp.bdd[t * 64 + g];
            const RowBdd *b = row >= 0 ? &bdds[row] : nullptr;
            const int L = b ? b->L : 0;
            size_t src = 0;
            for (int l = 0; l < nl; ++l) {
                const int64_t base = hp.node_base[t] + hp.lev_off[hp.lev_base[t] + l];
                const int W = l < L ? b->width[l] : 0;
                const int Wn = l + 1 < L ? b->width[l + 1] : 0;
                const int slots = hp.lev_rows[hp.lev_base[t] + l] * P;
                // real nodes, then padding whose two arcs lead to the 0-terminal
                for (int k = 0; k < W; ++k)
                    topo[(size_t)(base + (int64_t)(k / P) * 64 + g * P + (k % P))] = b->arcs[src++];
                if (P < 64)
                    for (int k = W; k < slots; ++k)
                        topo[(size_t)(base + (int64_t)(k / P) * 64 + g * P + (k % P))] =
                            (uint32_t)Wn | ((uint32_t)Wn << 16);
            }
        }
    });
    encode_topology(hp, topo);
    // edges
    const int64_t E = sr.ptr[m];
    hp.canon2slot.assign((size_t)E, -1);
    hp.slot2canon.assign((size_t)edge_slots, -1);
    hp.evar.assign((size_t)edge_slots, -1);
    for (int64_t t = 0; t < ntiles; ++t) {
        const int P = hp.tile_P[t], G = 64 / P;
        for (int g = 0; g < G; ++g) {
            const int row = hp.bdd[t * 64 + g];
            if (row < 0) continue;
            for (int l = 0; l < bdds[row].L; ++l) {
                const int64_t slot = hp.edge_base[t] + (int64_t)l * G + g;
                const int64_t ce = sr.ptr[row] + l;
                hp.canon2slot[ce] = (int32_t)slot;
                hp.slot2canon[slot] = (int32_t)ce;
                hp.evar[slot] = sr.col[ce];
            }
        }
    }
    // The library numbers the variables in the order they first appear in the edge slots (variables in
    // no row last): the per-variable sums handle consecutive numbers side by side, and a variable's
    // first edge then lies near those of its neighbours in the slot range, as do the S values that
    // the per-slot gathers read.  Per-variable arrays at the boundary (c, d_c) are mapped through
    // var_perm; every sum over a variable's edges keeps the canonical order.
    hp.var_perm.assign((size_t)p->n, -1);
    int32_t next = 0;
    for (int64_t slot = 0; slot < edge_slots; ++slot) {
        const int32_t v = hp.evar[slot];
        if (v >= 0 && hp.var_perm[v] < 0) hp.var_perm[v] = next++;
    }
    for (int v = 0; v < p->n; ++v)
        if (hp.var_perm[v] < 0) hp.var_perm[v] = next++;
    for (int64_t slot = 0; slot < edge_slots; ++slot)
        if (hp.evar[slot] >= 0) hp.evar[slot] = hp.var_perm[hp.evar[slot]];
    // variable -> edges (canonical order within a variable: rows ascending)
    hp.var_ptr.assign((size_t)p->n + 1, 0);
    for (int64_t e = 0; e < E; ++e) hp.var_ptr[hp.var_perm[sr.col[e]] + 1]++;
    for (int v = 0; v < p->n; ++v) hp.var_ptr[v + 1] += hp.var_ptr[v];
    hp.var_slots.assign((size_t)E, 0);
    hp.var_canon.assign((size_t)E, 0);
    std::vector<int32_t> fill(hp.var_ptr.begin(), hp.var_ptr.end() - 1);
    for (int64_t e = 0; e < E; ++e) {
        const int v = hp.var_perm[sr.col[e]];
        hp.var_canon[fill[v]] = (int32_t)e;
        hp.var_slots[fill[v]++] = hp.canon2slot[e];
    }
    return DD_OK;
}

// Bytes one launch must move by the method's own accounting (per node / per edge / per row); codes:
// the sweep also writes the argmin codes of the nodes it computes (2 bytes per node of a one-wave class).
double algorithmic_bytes(bool fwd, int mode, const ClassLaunch &c, bool codes) {
    const double N = (double)c.nodes, E = (double)c.edges, R = (double)c.rows;
    const bool writes_codes = codes && c.P == 64 &&
                              (fwd ? mode == FWD_UPDATE_REC || mode == FWD_SWEEP_LAM
                                   : mode == BWD_UPDATE_REC || mode == BWD_STORE || mode == BWD_STORE_BAR);
    const double cb = writes_codes ? 2 * N : 0.0;
    if (fwd)
        return cb + (mode == FWD_UPDATE ? 12 * N + 28 * E : mode == FWD_UPDATE_REC ? 12 * N + 40 * E : 8 * N + 16 * E);
    switch (mode) {
        case BWD_UPDATE: return 12 * N + 28 * E + 4 * R;
        case BWD_UPDATE_REC: return cb + 12 * N + 40 * E + 4 * R;
        case BWD_STORE: return cb + 8 * N + 8 * E + 4 * R;
        case BWD_EN_LAM: return 4 * N + 4 * E + 4 * R;
        case BWD_EN_BAR: return 4 * N + 16 * E + 4 * R;
        default: return cb + 8 * N + 24 * E;
    }
}


// The classes of one sweep are independent launches; all but the first run on side streams
// forked from (and joined back into) the caller's stream, so their tails overlap.
// launch(class, stream) returns hipError_t; name(class) and bytes(class) label it for profiling.
template <class L, class N, class B>
int per_class(dd_instance *h, hipStream_t s, L launch, N name, B bytes) {
    const size_t nc = h->classes.size();
    if (nc > 1) {
        HIP_TRY(hipEventRecord(h->fork, s));
        for (size_t c = 1; c < nc; ++c) HIP_TRY(hipStreamWaitEvent(h->side[c - 1], h->fork, 0));
    }
    for (size_t c = 0; c < nc; ++c) {
        const ClassLaunch &cl = h->classes[c];
        hipStream_t cs = c == 0 ? s : h->side[c - 1];
        int st = recorded(h, name(cl).c_str(), bytes(cl), cs, [&] { return launch(cl, cs); });
        if (st) return st;
    }
    for (size_t c = 1; c < nc; ++c) {
        HIP_TRY(hipEventRecord(h->join[c - 1], h->side[c - 1]));
        HIP_TRY(hipStreamWaitEvent(s, h->join[c - 1], 0));
    }
    return DD_OK;
}

// a kernel templated on the class, named as the profiler prints it
std::string kname(const char *k, const ClassLaunch &cl) {
    char name[96];
    snprintf(name, sizeof name, "%s<%d, %d>", k, cl.P, cl.RMAX);
    return name;
}

int all_classes_launch(dd_instance *h, bool fwd, int mode, hipStream_t s);

// Which node-cost array holds the costs at the current multipliers after a sweep of this mode.
void note_sweep(dd_instance *h, bool fwd, int mode) {
    if (fwd) {
        h->f_valid = mode != FWD_SWEEP_BAR;  // every forward sweep writes F; at lambda_bar it is not F(lambda)
        if (mode == FWD_UPDATE || mode == FWD_UPDATE_REC) h->b_valid = false;
    } else if (mode == BWD_UPDATE || mode == BWD_UPDATE_REC || mode == BWD_STORE) {
        h->b_valid = true;
        if (mode != BWD_STORE) h->f_valid = false;
    } else if (mode == BWD_STORE_BAR) {
        h->b_valid = false;
    }
}

int all_classes(dd_instance *h, bool fwd, int mode, hipStream_t s) {
    const int st = all_classes_launch(h, fwd, mode, s);
    if (st == DD_OK) note_sweep(h, fwd, mode);
    return st;
}

int all_classes_launch(dd_instance *h, bool fwd, int mode, hipStream_t s) {
    return per_class(
        h, s,
        [&](const ClassLaunch &cl, hipStream_t cs) {
            return fwd ? launch_fwd(h->T, cl, mode, cs) : launch_bwd(h->T, cl, mode, cs);
        },
        [&](const ClassLaunch &cl) {
            // the template arguments as the profiler prints them; the last says whether the
            // waves of a resident grid walk the tile list
            const int wpb = fwd ? cl.wpb_f : cl.wpb_b, grid = fwd ? cl.grid_f : cl.grid_b;
            const bool loop = mode == (fwd ? (int)FWD_UPDATE : (int)BWD_UPDATE) && grid > 0 &&
                              (int64_t)grid < (cl.ntiles + wpb - 1) / wpb;
            char name[96];
            if (cl.P == 64)  // one-wave tiles run the wide-row kernels
                snprintf(name, sizeof name, "%s<%d, %d, %s>", fwd ? "k_fwd_w" : "k_bwd_w", cl.RMAX, mode,
                         loop ? "true" : "false");
            else
                snprintf(name, sizeof name, "%s<%d, %d, %d, %s>", fwd ? "k_fwd" : "k_bwd", cl.P, cl.RMAX, mode,
                         loop ? "true" : "false");
            return std::string(name);
        },
        [&](const ClassLaunch &cl) {
            return algorithmic_bytes(fwd, mode, cl, fwd ? h->T.Fpar != nullptr : h->T.Bch != nullptr);
        });
}

// Reverse sweeps.  Bytes: topology and the swept side's cost (8 B/node), or for one-wave classes the
// argmin codes alone (2 B/node); update sweeps ~76 B of edge data with the pass's argmin records, fixed
// sweeps ~28 B/edge.
int adj_classes(dd_instance *h, const AdjTables &A, int which, int bar, int recs, float seed, hipStream_t s) {
    const bool upd = which == ADJ_F_UPDATE || which == ADJ_B_UPDATE;
    const char *nm = which == ADJ_F_UPDATE || which == ADJ_F_FIXED ? "k_adj_F" : "k_adj_B";
    return per_class(
        h, s, [&](const ClassLaunch &cl, hipStream_t cs) { return launch_adj(h->T, A, cl, which, bar, recs, seed, h->adj_dense, cs); },
        [&](const ClassLaunch &cl) {
            // the kernel and template arguments as the profiler prints them (one-wave sweeps that
            // route along recorded argmin codes run the k_adjc_ kernels)
            const bool push = which == ADJ_F_UPDATE || which == ADJ_F_FIXED;
            const bool coded = cl.P == 64 && !h->adj_dense && (push ? h->T.Fpar != nullptr : h->T.Bch != nullptr);
            char name[96];
            if (cl.P == 64)
                snprintf(name, sizeof name, "%s_w<%d, %s>", coded ? (push ? "k_adjc_F" : "k_adjc_B") : nm, cl.RMAX,
                         upd ? "true" : "false");
            else
                snprintf(name, sizeof name, "%s<%d, %d, %s>", nm, cl.P, cl.RMAX, upd ? "true" : "false");
            return std::string(name);
        },
        [&](const ClassLaunch &cl) {
            const bool push = which == ADJ_F_UPDATE || which == ADJ_F_FIXED;
            const bool coded = cl.P == 64 && !h->adj_dense && (push ? h->T.Fpar != nullptr : h->T.Bch != nullptr);
            const double per_node = coded ? 2.0 : 8.0;
            return upd ? per_node * cl.nodes + 76.0 * cl.edges : per_node * cl.nodes + 28.0 * cl.edges;
        });
}

int deferred(dd_instance *h, hipStream_t s) { return deferred_from(h, h->T.M, s); }

int smoothed_sweeps(dd_instance *h, float *Qs, float tau, int flushed, float *E_out, float *p_out, hipStream_t s) {
    int st;
    if (flushed && (st = deferred(h, s))) return st;
    if (E_out) HIP_TRY(launch_fill(E_out, 0.f, h->m, s));  // rows with no variable: E = 0
    return per_class(
        h, s, [&](const ClassLaunch &cl, hipStream_t cs) {
            return launch_smooth(h->T, cl, Qs, tau, flushed ? 1 : 0, E_out, p_out, cs);
        },
        [&](const ClassLaunch &cl) { return kname("k_smooth", cl); },
        // per node: topology twice, the arc probability written and read back (16 B); per edge:
        // the multipliers and alpha*S, the marginal and its index (16 B)
        [&](const ClassLaunch &cl) { return 16.0 * cl.nodes + 16.0 * cl.edges; });
}

// S_i of the given M (without alpha * S per edge)
int deferred_sum(dd_instance *h, const float *M, hipStream_t s) {
    return recorded(h, "k_deferred_sum", 8.0 * (double)h->E + 12.0 * (double)h->n, s, [&] {
        return launch_deferred_sum(h->var_ptr, h->var_slots, M, h->S, (int)h->n, h->var_team, s);
    });
}

int deferred_from(dd_instance *h, const float *M, hipStream_t s, float *Se) {
    int st = deferred_sum(h, M, s);
    if (st) return st;
    return recorded(h, "k_edge_alpha_s", (Se ? 20.0 : 16.0) * (double)h->edge_slots, s, [&] {
        return launch_edge_alpha_s(h->T.evar, h->alpha, h->S, h->aS, Se, h->edge_slots, s);
    });
}

int recompute_B(dd_instance *h, hipStream_t s) {
    int st = all_classes(h, false, BWD_STORE, s);
    h->en_lam_valid = st == DD_OK;
    return st;
}

int pass_launches(dd_instance *h, int dir, hipStream_t s) {
    // with form_as the update passes form and store alpha * S themselves
    int st = h->T.form_as ? deferred_sum(h, h->T.M, s) : deferred(h, s);
    if (st) return st;
    return all_classes(h, dir == 0, dir == 0 ? (int)FWD_UPDATE : (int)BWD_UPDATE, s);
}

}  // namespace ddi

extern "C" {

const char *dd_last_error(void) { return g_err.c_str(); }

int dd_compile_row(const dd_problem *prob, int32_t row, int32_t *width, uint32_t *arcs, int64_t cap, int64_t *nodes) {
    if (!prob || !nodes) return fail(DD_E_ARG, "NULL argument");
    if (row < 0 || row >= prob->m) return fail(DD_E_ARG, "row %d out of range", row);
    SortedRows sr;
    int st = validate_and_sort(prob, sr);
    if (st) return st;
    const int64_t a = sr.ptr[row];
    const int L = (int)(sr.ptr[row + 1] - a);
    RowBdd b;
    CompileScratch scr;
    if (L == 0) {
        *nodes = 0;
        return DD_OK;
    }
    st = compile_row(L, sr.coef.data() + a, prob->sense[row], prob->rhs[row], b, scr);
    if (st) return fail(st, "row %d: %s", row,
                        st == E_INFEASIBLE ? "infeasible" : st == E_FORCED ? "fixes a variable" : "unsupported");
    *nodes = (int64_t)b.arcs.size();
    if (width) std::copy(b.width.begin(), b.width.end(), width);
    if (arcs) {
        if (cap < (int64_t)b.arcs.size()) return fail(DD_E_ARG, "arcs capacity %lld < %zu", (long long)cap, b.arcs.size());
        std::copy(b.arcs.begin(), b.arcs.end(), arcs);
    }
    return DD_OK;
}

int dd_create(const dd_problem *prob, const dd_options *opt, void *stream, dd_instance **out) {
    return ddi::create_grouped(prob, opt, stream, nullptr, out);
}

}  // extern "C"

namespace ddi {

int create_grouped(const dd_problem *prob, const dd_options *opt, void *stream, const int32_t *row_group,
                   dd_instance **out) {
    if (!out) return fail(DD_E_ARG, "out is NULL");
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    dd_options o{};
    if (opt) o = *opt;
    const int npl = o.nodes_per_lane > 0 ? o.nodes_per_lane : 4;
    if (npl != 1 && npl != 2 && npl != 4) return fail(DD_E_ARG, "nodes_per_lane must be 1, 2 or 4");
    if (o.waves_per_block < 0 || o.waves_per_block > kMaxWavesPerBlock)
        return fail(DD_E_ARG, "waves_per_block must be 0 (default) or 1..%d", kMaxWavesPerBlock);
    const int wpb = o.waves_per_block > 0 ? o.waves_per_block : kMaxWavesPerBlock;
    const int lds_budget = o.lds_budget > 0 ? o.lds_budget : 64 * 1024;
    if (o.ckpt_every < 0) return fail(DD_E_ARG, "ckpt_every must be >= 0");
    if (o.lb_every < 0) return fail(DD_E_ARG, "lb_every must be >= 0");
    if (o.max_device_bytes < 0) return fail(DD_E_ARG, "max_device_bytes must be >= 0");
    SortedRows sr;
    int st = validate_and_sort(prob, sr);
    if (st) return st;
    const int m = prob->m;
    // compile every row
    std::vector<RowBdd> bdds((size_t)m);
    std::atomic<int> status(DD_OK), bad(-1);
    {
        int nw = worker_count();
        std::vector<CompileScratch> scr((size_t)nw);
        parallel_for(m, 32, [&](int64_t j, int w) {
            if (status != DD_OK) return;
            const int64_t a = sr.ptr[j];
            const int L = (int)(sr.ptr[j + 1] - a);
            if (L == 0) {
                const int64_t r = prob->rhs[j];
                const bool okk = prob->sense[j] < 0 ? 0 <= r : prob->sense[j] > 0 ? 0 >= r : r == 0;
                if (!okk) {
                    status = E_INFEASIBLE;
                    bad = (int)j;
                }
                return;
            }
            int r = compile_row(L, sr.coef.data() + a, prob->sense[j], prob->rhs[j], bdds[j], scr[w]);
            if (r != OK) {
                status = r;
                bad = (int)j;
            }
        });
    }
    if (status != DD_OK) {
        int c = status;
        return fail(c, "row %d: %s", (int)bad,
                    c == E_INFEASIBLE ? "no feasible assignment"
                    : c == E_FORCED   ? "fixes one of its variables (a min-marginal would be infinite)"
                                      : "diagram too wide");
    }
    HostPlan hp;
    std::vector<uint32_t> topo;
    st = build_plan(prob, sr, bdds, npl, wpb, lds_budget, row_group, hp, topo);
    if (st) return st;

    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    dd_instance *h = new dd_instance();
    h->device = device;
    if (o.ckpt_every > 0) h->ckpt_default = o.ckpt_every;
    if (o.lb_every > 0) h->lb_every = o.lb_every;
    h->max_device_bytes = o.max_device_bytes;
    h->use_graphs = o.no_graphs == 0;
    h->adj_dense = o.adj_route_dense != 0;
    h->adj_replay = o.adj_replay != 0;
    h->lds_budget = lds_budget;
    h->n = prob->n;
    h->m = m;
    h->E = sr.ptr[m];
    h->classes = hp.classes;
    std::stable_sort(h->classes.begin(), h->classes.end(),
                     [](const ClassLaunch &x, const ClassLaunch &y) { return x.nodes > y.nodes; });
    h->ntiles = (int64_t)hp.nlev.size();
    h->node_slots = hp.node_slots;
    h->coded_levels = hp.coded_levels;
    h->raw_levels = hp.raw_levels;
    h->edge_slots = hp.edge_slots;
    h->row_nodes.resize((size_t)m);
    for (int j = 0; j < m; ++j) h->row_nodes[j] = (int64_t)bdds[j].arcs.size();
    for (const RowBdd &b : bdds) {
        h->nodes += (int64_t)b.arcs.size();
        h->max_width = std::max(h->max_width, b.max_width);
        h->max_len = std::max(h->max_len, b.L);
    }
    bdds.clear();
    bdds.shrink_to_fit();
    h->edge_var.assign(sr.col.begin(), sr.col.end());
    h->edge_row.resize((size_t)h->E);
    for (int j = 0; j < m; ++j)
        for (int64_t e = sr.ptr[j]; e < sr.ptr[j + 1]; ++e) h->edge_row[e] = j;
    std::vector<float> c32((size_t)prob->n), om((size_t)h->E), al((size_t)h->E);
    for (int i = 0; i < prob->n; ++i) {
        const int v = hp.var_perm[i];
        c32[v] = (float)prob->c[i];
        if (hp.var_ptr[v + 1] == hp.var_ptr[v]) {
            h->uncovered++;
            if (prob->c[i] < 0) h->unc_const += prob->c[i];
        }
    }
    for (int64_t e = 0; e < h->E; ++e) {
        const int v = hp.var_perm[sr.col[e]];
        om[e] = 0.5f;
        al[e] = 1.0f / (float)(hp.var_ptr[v + 1] - hp.var_ptr[v]);
    }

    auto cleanup = [&](int code) {
        delete h;
        return code;
    };
#define TRY(x)              \
    do {                    \
        int r_ = (x);       \
        if (r_) return cleanup(r_); \
    } while (0)
    DevTables &T = h->T;
    TRY(upload(h, (int64_t **)&T.node_base, hp.node_base, s));
    TRY(upload(h, (int32_t **)&T.edge_base, hp.edge_base, s));
    TRY(upload(h, (int32_t **)&T.nlev, hp.nlev, s));
    TRY(upload(h, (int32_t **)&T.lev_base, hp.lev_base, s));
    TRY(upload(h, (int32_t **)&T.w_base, hp.w_base, s));
    TRY(upload(h, (int32_t **)&T.bdd, hp.bdd, s));
    TRY(upload(h, (int32_t **)&T.lev_off, hp.lev_off, s));
    TRY(upload(h, (int32_t **)&T.lev_rows, hp.lev_rows, s));
    TRY(upload(h, (uint16_t **)&T.widths, hp.widths, s));
    TRY(upload(h, (uint32_t **)&T.topo, topo, s));
    TRY(upload(h, (uint8_t **)&T.tcode, hp.tcode, s));
    TRY(upload(h, (uint32_t **)&T.lev_code, hp.lev_code, s));
    TRY(h->alloc(&T.F, (size_t)hp.node_alloc));
    TRY(h->alloc(&T.B, (size_t)hp.node_alloc));
    TRY(h->alloc(&T.lam, (size_t)hp.edge_slots));
    TRY(h->alloc(&T.M, (size_t)hp.edge_slots));
    TRY(h->alloc(&h->omega, (size_t)hp.edge_slots));
    TRY(h->alloc(&h->alpha, (size_t)hp.edge_slots));
    TRY(h->alloc(&h->aS, (size_t)hp.edge_slots));
    T.aS = h->aS;
    T.omega = h->omega;
    T.alpha = h->alpha;
    TRY(upload(h, (int32_t **)&T.evar, hp.evar, s));
    TRY(upload(h, (int32_t **)&T.slot2canon, hp.slot2canon, s));
    TRY(upload(h, &h->canon2slot, hp.canon2slot, s));
    TRY(upload(h, &h->var_ptr, hp.var_ptr, s));
    TRY(upload(h, &h->var_perm, hp.var_perm, s));
    // lanes per variable in the per-variable sums: one constant, so that a program gets the same bits
    // alone and packed into a batch with programs of other degrees
    h->var_team = dd_instance::kVarTeam;
    TRY(upload(h, &h->var_slots, hp.var_slots, s));
    TRY(upload(h, &h->var_canon, hp.var_canon, s));
    TRY(upload(h, &h->cdev, c32, s));
    TRY(h->alloc(&h->S, (size_t)prob->n));
    T.S = h->S;
    {
        bool wide = false;
        for (const ClassLaunch &c : h->classes) wide = wide || c.P == 64;
        T.form_as = !wide && (int64_t)prob->n * 4 <= dd::kFormAsMaxBytes;
    }
    TRY(h->alloc(&T.energies, (size_t)m));
    TRY(h->alloc(&T.en_lam, (size_t)m));
    TRY(h->alloc(&h->partial, (size_t)kSumBlocks));
    TRY(h->alloc(&h->tmp, (size_t)std::max<int64_t>(h->E, 1) * 2));
    TRY(h->alloc(&h->red, 4));
    TRY(h->alloc(&h->flags, 2));
    auto hip_ok = [&](hipError_t e) { return e == hipSuccess ? DD_OK : fail(DD_E_HIP, "%s", hipGetErrorString(e)); };
    for (size_t c = 1; c < h->classes.size(); ++c) {
        hipStream_t q;
        hipEvent_t ev;
        TRY(hip_ok(hipStreamCreateWithFlags(&q, hipStreamNonBlocking)));
        h->side.push_back(q);
        TRY(hip_ok(hipEventCreateWithFlags(&ev, hipEventDisableTiming)));
        h->join.push_back(ev);
    }
    TRY(hip_ok(hipEventCreateWithFlags(&h->fork, hipEventDisableTiming)));
    {
        hipError_t e = hipHostMalloc((void **)&h->red_host, 4 * sizeof(double), hipHostMallocDefault);
        if (e != hipSuccess) return cleanup(fail(DD_E_OOM, "hipHostMalloc: %s", hipGetErrorString(e)));
    }
    TRY(hip_ok(hipMemsetAsync(T.lam, 0, sizeof(float) * hp.edge_slots, s)));
    TRY(hip_ok(hipMemsetAsync(T.M, 0, sizeof(float) * hp.edge_slots, s)));
    TRY(hip_ok(hipMemsetAsync(h->omega, 0, sizeof(float) * hp.edge_slots, s)));
    TRY(hip_ok(hipMemsetAsync(h->alpha, 0, sizeof(float) * hp.edge_slots, s)));
    TRY(hip_ok(hipMemsetAsync(h->aS, 0, sizeof(float) * hp.edge_slots, s)));
    TRY(hip_ok(hipMemsetAsync(T.F, 0, sizeof(float) * hp.node_alloc, s)));
    TRY(hip_ok(hipMemsetAsync(T.B, 0, sizeof(float) * hp.node_alloc, s)));
    TRY(hip_ok(hipMemsetAsync(T.energies, 0, sizeof(float) * std::max(m, 1), s)));
    TRY(hip_ok(hipMemsetAsync(T.en_lam, 0, sizeof(float) * std::max(m, 1), s)));
    TRY(hip_ok(hipMemsetAsync(h->S, 0, sizeof(float) * std::max<int64_t>(prob->n, 1), s)));
    // default parameters (FastDOG special case), staged through tmp
    {
        float *d_om = h->tmp, *d_al = h->tmp + std::max<int64_t>(h->E, 1);
        if (h->E) {
            TRY(hip_ok(hipMemcpyAsync(d_om, om.data(), sizeof(float) * h->E, hipMemcpyHostToDevice, s)));
            TRY(hip_ok(hipMemcpyAsync(d_al, al.data(), sizeof(float) * h->E, hipMemcpyHostToDevice, s)));
            TRY(hip_ok(launch_scatter(h->canon2slot, d_om, h->omega, h->E, s)));
            TRY(hip_ok(launch_scatter(h->canon2slot, d_al, h->alpha, h->E, s)));
        }
    }
    // the host staging vectors must outlive the async copies
    TRY(hip_ok(hipStreamSynchronize(s)));
    TRY(dd_reset(h, stream));
    TRY(hip_ok(hipStreamSynchronize(s)));
#undef TRY
    *out = h;
    return DD_OK;
}

}  // namespace ddi

extern "C" {

int dd_destroy(dd_instance *h) {
    delete h;
    return DD_OK;
}

int dd_get_stats(const dd_instance *h, dd_stats *o) {
    if (!h || !o) return fail(DD_E_ARG, "NULL argument");
    o->n = h->n;
    o->m = h->m;
    o->edges = h->E;
    o->nodes = h->nodes;
    o->arcs = 2 * h->nodes;
    o->node_slots = h->node_slots;
    o->edge_slots = h->edge_slots;
    o->tiles = h->ntiles;
    o->max_width = h->max_width;
    o->max_len = h->max_len;
    o->classes = (int32_t)h->classes.size();
    o->uncovered = h->uncovered;
    o->device_bytes = h->device_bytes;
    o->coded_levels = h->coded_levels;
    o->raw_levels = h->raw_levels;
    return DD_OK;
}

int dd_edge_map(const dd_instance *h, int32_t *var_out, int32_t *row_out) {
    if (!h) return fail(DD_E_ARG, "NULL instance");
    if (var_out) std::copy(h->edge_var.begin(), h->edge_var.end(), var_out);
    if (row_out) std::copy(h->edge_row.begin(), h->edge_row.end(), row_out);
    return DD_OK;
}

int dd_set_params(dd_instance *h, const float *omega, const float *alpha, void *stream) {
    if (!h || (h->E && (!omega || !alpha))) return fail(DD_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemsetAsync(h->flags, 0, 2 * sizeof(int32_t), s));
    HIP_TRY(launch_check_params(omega, alpha, h->E, h->flags, s));
    int32_t f[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(f, h->flags, sizeof f, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (f[0]) return fail(DD_E_PARAM, "omega must lie in [0, 1]");
    if (f[1]) return fail(DD_E_PARAM, "alpha must be finite and non-negative");
    HIP_TRY(launch_scatter(h->canon2slot, omega, h->omega, h->E, s));
    HIP_TRY(launch_scatter(h->canon2slot, alpha, h->alpha, h->E, s));
    h->version++;
    return DD_OK;
}

int dd_seg_softmax(dd_instance *h, const float *alpha_hat, float *alpha_out, void *stream) {
    if (!h || (h->E && (!alpha_hat || !alpha_out))) return fail(DD_E_ARG, "NULL argument");
    HIP_TRY(launch_seg_softmax(h->var_ptr, h->var_canon, alpha_hat, alpha_out, (int)h->n, (hipStream_t)stream));
    return DD_OK;
}

int dd_reset(dd_instance *h, void *stream) {
    if (!h) return fail(DD_E_ARG, "NULL instance");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_init_lambda(h->canon2slot, h->T.evar, h->var_ptr, h->cdev, h->T.lam, h->T.M, h->E, s));
    h->version++;
    h->f_valid = h->b_valid = false;
    return recompute_B(h, s);
}

int dd_set_state(dd_instance *h, const float *lambda, const float *M, void *stream) {
    if (!h || (h->E && (!lambda || !M))) return fail(DD_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_scatter(h->canon2slot, lambda, h->T.lam, h->E, s));
    HIP_TRY(launch_scatter(h->canon2slot, M, h->T.M, h->E, s));
    h->version++;
    h->f_valid = h->b_valid = false;
    return recompute_B(h, s);
}

int dd_get_state(dd_instance *h, float *lambda_out, float *M_out, int32_t flushed, void *stream) {
    if (!h || (h->E && !lambda_out)) return fail(DD_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (flushed) {
        int st = deferred(h, s);
        if (st) return st;
    }
    HIP_TRY(launch_gather(h->canon2slot, h->T.lam, lambda_out, h->E, flushed ? h->aS : nullptr, s));
    if (M_out) HIP_TRY(launch_gather(h->canon2slot, h->T.M, M_out, h->E, nullptr, s));
    return DD_OK;
}

int dd_run_pass(dd_instance *h, int32_t direction, void *stream) {
    if (!h || (direction != 0 && direction != 1)) return fail(DD_E_ARG, "bad instance or direction");
    hipStream_t s = (hipStream_t)stream;
    // the pass reads the other side's node costs at its input multipliers (eq. 8 for hops not yet
    // visited): rebuild them when the last call left them stale (two passes of one direction in a
    // row, or a call that changed the multipliers or the arrays without a sweep)
    int st = DD_OK;
    if (direction == 0 && !h->b_valid) st = recompute_B(h, s);
    if (direction == 1 && !h->f_valid) st = all_classes(h, true, FWD_SWEEP_LAM, s);
    if (st) return st;
    // a backward pass ends with B(root) = E^j at the updated multipliers; a forward pass
    // changes the multipliers without computing it
    h->en_lam_valid = false;
    h->version++;
    st = pass_launches(h, direction, s);
    h->en_lam_valid = st == DD_OK && direction == 1;
    return st;
}

}  // extern "C"

namespace {

constexpr int kGraphChunk = 8;  // iterations per replay of the large graph

// Capture `iters` dual iterations (2 passes each) into an executable graph.  Capture runs on
// the instance's own stream (the caller's may be the legacy default stream, which cannot be
// captured); the executable graph is then launched on any stream.
int capture_iterations(dd_instance *h, int iters, hipGraphExec_t *out) {
    if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    int st = DD_OK;
    for (int t = 0; t < iters && st == DD_OK; ++t)
        for (int d = 0; d < 2 && st == DD_OK; ++d) st = pass_launches(h, d, h->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (st != DD_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st != DD_OK ? st : fail(DD_E_HIP, "graph capture: %s", hipGetErrorString(e));
    }
    const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(DD_E_HIP, "graph instantiate: %s", hipGetErrorString(ei));
    return DD_OK;
}

}  // namespace

namespace ddi {

void drop_graphs(dd_instance *h) {
    if (h->graph_one) (void)hipGraphExecDestroy(h->graph_one);
    if (h->graph_chunk) (void)hipGraphExecDestroy(h->graph_chunk);
    h->graph_one = h->graph_chunk = nullptr;
    for (dd_instance::SeqGraph &g : h->seq_graphs) (void)hipGraphExecDestroy(g.exec);
    h->seq_graphs.clear();
}

}  // namespace ddi

extern "C" {

int dd_run(dd_instance *h, int32_t T, void *stream) {
    if (!h || T < 0) return fail(DD_E_ARG, "bad instance or T");
    if (T == 0) return DD_OK;
    hipStream_t s = (hipStream_t)stream;
    if (h->prof || !h->use_graphs || T == 1) {  // eager launches (profiling brackets each one)
        for (int t = 0; t < T; ++t)
            for (int d = 0; d < 2; ++d) {
                int st = dd_run_pass(h, d, stream);
                if (st) return st;
            }
        return DD_OK;
    }
    int st;
    if (!h->b_valid && (st = recompute_B(h, s))) return st;  // what the first forward pass reads
    if (!h->graph_one && (st = capture_iterations(h, 1, &h->graph_one))) return st;
    if (T >= kGraphChunk && !h->graph_chunk && (st = capture_iterations(h, kGraphChunk, &h->graph_chunk)))
        return st;
    h->en_lam_valid = false;
    int t = 0;
    for (; t + kGraphChunk <= T; t += kGraphChunk) HIP_TRY(hipGraphLaunch(h->graph_chunk, s));
    for (; t < T; ++t) HIP_TRY(hipGraphLaunch(h->graph_one, s));
    h->version += 2 * (int64_t)T;
    h->en_lam_valid = true;
    h->b_valid = true;  // the last pass replayed was a backward pass (capture ran no sweep)
    h->f_valid = false;
    return DD_OK;
}

int dd_lower_bound(dd_instance *h, double *lb, double *dl, void *stream) {
    if (!h || !lb) return fail(DD_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    int st = deferred(h, s);
    if (st) return st;
    if ((st = all_classes(h, false, BWD_EN_BAR, s))) return st;
    auto sum = [&](const float *x, int64_t n, int neg, double *out) {
        return recorded(h, "k_sum", 4.0 * (double)n, s, [&] { return launch_sum(x, n, neg, h->partial, out, s); });
    };
    if ((st = sum(h->T.energies, h->m, 0, h->red))) return st;
    if (dl) {
        if (!h->en_lam_valid) {
            if ((st = all_classes(h, false, BWD_EN_LAM, s))) return st;
            h->en_lam_valid = true;
        }
        if ((st = sum(h->T.en_lam, h->m, 0, h->red + 2))) return st;
        if ((st = sum(h->T.M, h->edge_slots, 1, h->red + 3))) return st;
    }
    HIP_TRY(hipMemcpyAsync(h->red_host, h->red, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *lb = h->red_host[0] + h->unc_const;
    if (dl) *dl = h->red_host[2] + h->red_host[3] + h->unc_const;
    if (!std::isfinite(*lb) || (dl && !std::isfinite(*dl))) return fail(DD_E_NONFINITE, "lower bound is not finite");
    return DD_OK;
}

int dd_run_trace(dd_instance *h, int32_t T, int32_t lb_every, double *lb_dev, void *stream) {
    if (!h || T < 0) return fail(DD_E_ARG, "bad instance or T");
    const int every = lb_every > 0 ? lb_every : h->lb_every;
    if (T >= every && !lb_dev) return fail(DD_E_ARG, "lb_dev is NULL");
    hipStream_t s = (hipStream_t)stream;
    int st;
    for (int t = 0, i = 0; t < T; t += every) {
        const int n = std::min(every, T - t);
        if ((st = dd_run(h, n, stream))) return st;
        if (n < every) break;
        // the bound as dd_lower_bound computes it, with the constant added on the device
        if ((st = deferred(h, s)) || (st = all_classes(h, false, BWD_EN_BAR, s))) return st;
        double *out = lb_dev + i++;
        st = recorded(h, "k_sum", 4.0 * (double)h->m, s,
                      [&] { return launch_sum(h->T.energies, h->m, 0, h->partial, out, s, h->unc_const); });
        if (st) return st;
    }
    return DD_OK;
}

int dd_num_edges(const dd_instance *h, int64_t *E) {
    if (!h || !E) return fail(DD_E_ARG, "NULL argument");
    *E = h->E;
    return DD_OK;
}

int dd_row_energies(dd_instance *h, float *E_out, void *stream) {
    if (!h || (h->m && !E_out)) return fail(DD_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    int st = deferred(h, s);
    if (st) return st;
    if ((st = all_classes(h, false, BWD_EN_BAR, s))) return st;
    if (h->m) HIP_TRY(hipMemcpyAsync(E_out, h->T.energies, sizeof(float) * h->m, hipMemcpyDeviceToDevice, s));
    return DD_OK;
}

int dd_min_marginals(dd_instance *h, float *m0_out, float *m1_out, void *stream) {
    if (!h || (h->E && (!m0_out || !m1_out))) return fail(DD_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    int st = deferred(h, s);
    if (st) return st;
    // F at lambda_bar into the F buffer (free between passes), then m0/m1 during a B sweep at lambda_bar
    if ((st = all_classes(h, true, FWD_SWEEP_BAR, s))) return st;
    h->T.out0 = m0_out;
    h->T.out1 = m1_out;
    st = all_classes(h, false, BWD_MM, s);
    h->T.out0 = h->T.out1 = nullptr;
    return st;
}

}  // extern "C"

namespace {

// Point the tables at node-cost arrays together with their argmin codes.
void use_F(dd_instance *h, float *F, uint16_t *Fp) {
    h->T.F = F;
    h->T.Fpar = Fp;
}
void use_B(dd_instance *h, float *B, uint16_t *Bc) {
    h->T.B = B;
    h->T.Bch = Bc;
}

int adj_alloc(dd_instance *h) {
    if (h->adj_ready) return DD_OK;
    const size_t S = (size_t)h->edge_slots;
    int st;
    for (float **b : {&h->lam_in, &h->dlamA, &h->dlamB, &h->dMA, &h->dMB, &h->g, &h->dalpha, &h->domega, &h->Se})
        if ((st = h->alloc(b, S))) return st;
    if ((st = h->alloc(&h->rec_val, 2 * S))) return st;
    if ((st = h->alloc(&h->rec_idx, 2 * S))) return st;
    if ((st = h->alloc(&h->mrec, 2 * S))) return st;
    if ((st = h->alloc(&h->mdiff, S))) return st;
    HIP_TRY(hipMemset(h->mrec, 0, sizeof(int32_t) * 2 * S));
    HIP_TRY(hipMemset(h->mdiff, 0, sizeof(float) * S));
    if ((st = h->alloc(&h->scratch_n, (size_t)std::max<int64_t>(h->n, 1)))) return st;
    if ((st = h->alloc(&h->hash_tmp, 1)) || (st = h->alloc(&h->ck_flag, 1))) return st;
    // argmin codes of the instance's own node-cost arrays: recorded by the sweeps reverse mode reads
    const size_t nodes = (size_t)h->node_slots + 64;
    if ((st = h->alloc(&h->Fpar0, nodes)) || (st = h->alloc(&h->Bch0, nodes))) return st;
    HIP_TRY(hipMemset(h->Fpar0, 0, sizeof(uint16_t) * nodes));
    HIP_TRY(hipMemset(h->Bch0, 0, sizeof(uint16_t) * nodes));
    h->T.Fpar = h->Fpar0;
    h->T.Bch = h->Bch0;
    for (float *b : {h->lam_in, h->dlamA, h->dlamB, h->dMA, h->dMB, h->g, h->dalpha, h->domega, h->Se})
        HIP_TRY(hipMemset(b, 0, sizeof(float) * S));
    HIP_TRY(hipMemset(h->rec_val, 0, sizeof(float) * 2 * S));
    HIP_TRY(hipMemset(h->rec_idx, 0xFF, sizeof(int32_t) * 2 * S));
    h->adj_ready = true;
    return DD_OK;
}

int copy_slots(dd_instance *h, float *dst, const float *src, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(dst, src, sizeof(float) * h->edge_slots, hipMemcpyDeviceToDevice, s));
    return DD_OK;
}

// Launches fn with the tables pointed at the record arrays (the instance's own unless given), so its
// recording update passes write them; the tables never keep those pointers.
template <typename Fn>
int recording(dd_instance *h, Fn &&fn, int32_t *mrec = nullptr, float *mdiff = nullptr) {
    h->T.mrec = mrec ? mrec : h->mrec;
    h->T.mdiff = mdiff ? mdiff : h->mdiff;
    const int st = fn();
    h->T.mrec = nullptr;
    h->T.mdiff = nullptr;
    return st;
}

// First line of Alg. 2 with the multiplier update's alpha: dS_i = sum of g (= dlambda' alpha) over the
// edges of variable i, summed as S is in the forward direction (the deferred-sum kernel on g, into the
// per-variable scratch), then dM[slot] = dS_i for every edge slot of i (0 on padding) in slot order,
// which writes coalesced where writing each variable's total to its own slots would scatter.
int adj_deferred(dd_instance *h, float *dM, hipStream_t s) {
    int st = recorded(h, "k_deferred_sum", 8.0 * (double)h->E + 12.0 * (double)h->n, s, [&] {
        return launch_deferred_sum(h->var_ptr, h->var_slots, h->g, h->scratch_n, (int)h->n, h->var_team, s);
    });
    if (st) return st;
    return recorded(h, "k_edge_S", 12.0 * (double)h->edge_slots, s,
                    [&] { return launch_edge_S(h->T.evar, h->scratch_n, dM, h->edge_slots, s); });
}

// An update pass that records its argmins (as dd_run_pass otherwise); with Se, it keeps the S per
// edge of its input M there.
// With S_given (S of the pass-input M, kept by the forward that first ran this pass), the deferred
// sum is not formed again.
int run_pass_rec(dd_instance *h, int dir, hipStream_t s, int32_t *mrec = nullptr, float *mdiff = nullptr,
                 float *Se = nullptr, float *S_given = nullptr) {
    h->en_lam_valid = false;
    h->version++;
    float *own_S = h->S;
    if (S_given) {
        h->S = S_given;
        h->T.S = S_given;
    }
    // passes that form alpha*S themselves also write S per edge (every slot of a diagram level;
    // padding slots keep the 0 they were allocated with): only S per variable is needed first
    const bool fas = h->T.form_as != 0;
    int st = DD_OK;
    if (fas) st = S_given ? DD_OK : deferred_sum(h, h->T.M, s);
    else if (S_given)
        st = recorded(h, "k_edge_alpha_s", (Se ? 20.0 : 16.0) * (double)h->edge_slots, s, [&] {
            return launch_edge_alpha_s(h->T.evar, h->alpha, h->S, h->aS, Se, h->edge_slots, s);
        });
    else st = deferred_from(h, h->T.M, s, Se);
    if (st == DD_OK) {
        if (fas) h->T.Se_rec = Se;
        st = recording(h, [&] { return all_classes(h, dir == 0, dir == 0 ? (int)FWD_UPDATE_REC : (int)BWD_UPDATE_REC, s); },
                       mrec, mdiff);
        h->T.Se_rec = nullptr;
    }
    h->S = own_S;
    h->T.S = own_S;
    h->en_lam_valid = st == DD_OK && dir == 1;
    return st;
}

// Reverse mode of one pass.  On entry the instance state (lambda, M) is the pass input; on exit
// it is the pass output.  dlam_out/dM_out: adjoints of the outputs; dlam_in/dM_in receive the
// adjoints of the inputs; d_alpha and d_omega accumulate.
// With lam_src/M_src (slot order): the instance already holds this pass's outputs -- its
// multipliers, M and both node sides exactly as the pass left them (the side it read, computed
// from the input multipliers, and the side it rebuilt) -- and lam_src/M_src are its inputs and
// mrec_src/mdiff_src its argmin records (and Se_src, when kept, the S per edge of M_src); the
// fixed-side sweep and the replay are then skipped.  Otherwise the replay records them.
int pass_vjp(dd_instance *h, int dir, const float *dlam_out, const float *dM_out, float *dlam_in, float *dM_in,
             hipStream_t s, const float *lam_src = nullptr, const float *M_src = nullptr,
             const int32_t *mrec_src = nullptr, const float *mdiff_src = nullptr, const float *Se_src = nullptr) {
    const bool fresh = lam_src != nullptr;
    if (fresh && (!mrec_src || !mdiff_src)) return fail(DD_E_ARG, "internal: a pass adjoint needs the pass's records");
    // S of the pass-input M per edge for the update sweeps and, for the replayed update pass, alpha*S;
    // the reverse sweeps read no alpha*S, and every later reader of it recomputes it from its state
    int st = DD_OK;
    if (!fresh) {
        st = deferred_from(h, h->T.M, s, h->Se);
    } else if (!Se_src) {
        st = deferred_sum(h, M_src, s);
        if (st == DD_OK)
            st = recorded(h, "k_edge_S", 12.0 * (double)h->edge_slots, s,
                          [&] { return launch_edge_S(h->T.evar, h->S, h->Se, h->edge_slots, s); });
    }
    if (st) return st;
    // the pass-input multipliers: kept by the caller, or copied before the replay overwrites them
    if (!fresh && (st = copy_slots(h, h->lam_in, h->T.lam, s))) return st;
    AdjTables A{};
    A.lam_src = fresh ? lam_src : h->lam_in;
    A.mrec = fresh ? mrec_src : h->mrec;
    A.mdiff = fresh ? mdiff_src : h->mdiff;
    A.dlam_out = dlam_out;
    A.dM_out = dM_out;
    A.Se = Se_src ? Se_src : h->Se;
    A.dlam_in = dlam_in;
    A.g = h->g;
    A.dalpha = h->dalpha;
    A.domega = h->domega;
    A.rec_idx = h->rec_idx;
    A.rec_val = h->rec_val;
    h->en_lam_valid = false;
    if (dir == 0) {
        // fixed side B at the input multipliers, the pass replayed (F), then the two reverse sweeps
        if (!fresh && (st = all_classes(h, false, BWD_STORE, s))) return st;
        if (!fresh && (st = recording(h, [&] { return all_classes(h, true, FWD_UPDATE_REC, s); }))) return st;
        if ((st = adj_classes(h, A, ADJ_F_UPDATE, 0, 0, 0.f, s))) return st;
        if ((st = adj_classes(h, A, ADJ_B_FIXED, 0, 1, 0.f, s))) return st;
    } else {
        if (!fresh && (st = all_classes(h, true, FWD_SWEEP_LAM, s))) return st;
        if (!fresh && (st = recording(h, [&] { return all_classes(h, false, BWD_UPDATE_REC, s); }))) return st;
        if ((st = adj_classes(h, A, ADJ_B_UPDATE, 0, 0, 0.f, s))) return st;
        if ((st = adj_classes(h, A, ADJ_F_FIXED, 0, 1, 0.f, s))) return st;
    }
    return adj_deferred(h, dM_in, s);
}

int save_state(dd_instance *h, std::vector<float *> &L, std::vector<float *> &Mv, size_t i, hipStream_t s) {
    while (L.size() <= i) {
        float *a = nullptr, *b = nullptr;
        int st = h->alloc(&a, (size_t)h->edge_slots);
        if (st) return st;
        if ((st = h->alloc(&b, (size_t)h->edge_slots))) return st;
        L.push_back(a);
        Mv.push_back(b);
    }
    HIP_TRY(launch_copy2(h->T.lam, L[i], h->T.M, Mv[i], h->edge_slots, s));
    return DD_OK;
}

// Fingerprint of a state (slot-ordered lambda, M) into *out (device).
int state_hash(dd_instance *h, const float *lam, const float *M, uint64_t *out, hipStream_t s) {
    return recorded(h, "k_hash", 8.0 * (double)h->edge_slots, s, [&] {
        return launch_state_hash(lam, M, h->edge_slots, (uint64_t *)h->partial, out, s);
    });
}

// Flag (ck_flag) when the state (lam, M) does not have checkpoint i's fingerprint.
int verify_state(dd_instance *h, const float *lam, const float *M, size_t i, hipStream_t s) {
    int st = state_hash(h, lam, M, h->hash_tmp, s);
    if (st) return st;
    HIP_TRY(launch_hash_check(h->hash_tmp, h->ck_hash + i, h->ck_flag, s));
    return DD_OK;
}

int load_state(dd_instance *h, const std::vector<float *> &L, const std::vector<float *> &Mv, size_t i,
               hipStream_t s) {
    HIP_TRY(launch_copy2(L[i], h->T.lam, Mv[i], h->T.M, h->edge_slots, s));
    h->f_valid = h->b_valid = false;
    return DD_OK;
}

}  // namespace

extern "C" {

int dd_pass_vjp(dd_instance *h, int32_t direction, const float *lam_in, const float *M_in, const float *dlam_out,
                const float *dM_out, float *dlam_in, float *dM_in, float *d_alpha, float *d_omega, void *stream) {
    if (!h || (direction != 0 && direction != 1)) return fail(DD_E_ARG, "bad instance or direction");
    if (h->E && (!lam_in || !M_in || !dlam_out || !dM_out || !dlam_in || !dM_in || !d_alpha || !d_omega))
        return fail(DD_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    int st = adj_alloc(h);
    if (st) return st;
    HIP_TRY(launch_scatter(h->canon2slot, lam_in, h->T.lam, h->E, s));
    HIP_TRY(launch_scatter(h->canon2slot, M_in, h->T.M, h->E, s));
    h->f_valid = h->b_valid = false;
    HIP_TRY(launch_scatter(h->canon2slot, dlam_out, h->dlamA, h->E, s));
    HIP_TRY(launch_scatter(h->canon2slot, dM_out, h->dMA, h->E, s));
    HIP_TRY(launch_fill(h->dalpha, 0.f, h->edge_slots, s));
    HIP_TRY(launch_fill(h->domega, 0.f, h->edge_slots, s));
    h->version++;
    if ((st = pass_vjp(h, direction, h->dlamA, h->dMA, h->dlamB, h->dMB, s))) return st;
    HIP_TRY(launch_gather(h->canon2slot, h->dlamB, dlam_in, h->E, nullptr, s));
    HIP_TRY(launch_gather(h->canon2slot, h->dMB, dM_in, h->E, nullptr, s));
    HIP_TRY(launch_gather(h->canon2slot, h->dalpha, d_alpha, h->E, nullptr, s));
    HIP_TRY(launch_gather(h->canon2slot, h->domega, d_omega, h->E, nullptr, s));
    return recompute_B(h, s);
}

}  // extern "C"

namespace {

constexpr size_t kMaxSeqGraphs = 8;  // captured sequences kept per instance (the oldest goes first)

// Runs `seq(q)` -- the launches of a sequence fixed by `key` on stream q, with their host-side
// bookkeeping -- eagerly while profiling or without graphs.  Otherwise the first run with a key
// captures the sequence on the instance's own stream and replays the graph on s; later runs only
// replay it and apply the host-side effects the capture recorded (state version, side flags, table
// pointers).  The key also holds everything host code reads to choose the launches: the side flags
// and table pointers on entry and the allocation count, so a sequence that would see other buffers
// is captured anew.  A sequence must not allocate (its buffers are allocated beforehand), read device
// memory on the host or wait for the device.
template <typename Seq>
int replayed(dd_instance *h, std::vector<int64_t> key, hipStream_t s, Seq &&seq) {
    if (h->prof || !h->use_graphs) return seq(s);
    key.insert(key.end(), {h->alloc_epoch, (int64_t)h->en_lam_valid, (int64_t)h->b_valid, (int64_t)h->f_valid,
                           (int64_t)h->adj_dense, (int64_t)h->adj_replay, (int64_t)(intptr_t)h->T.F,
                           (int64_t)(intptr_t)h->T.B, (int64_t)(intptr_t)h->T.lam, (int64_t)(intptr_t)h->T.M});
    for (const dd_instance::SeqGraph &g : h->seq_graphs)
        if (g.key == key) {
            HIP_TRY(hipGraphLaunch(g.exec, s));
            h->version += g.dversion;
            h->en_lam_valid = g.en_lam_valid;
            h->b_valid = g.b_valid;
            h->f_valid = g.f_valid;
            h->T.F = g.F;
            h->T.B = g.B;
            h->T.Fpar = g.Fpar;
            h->T.Bch = g.Bch;
            h->T.lam = g.lam;
            h->T.M = g.M;
            return DD_OK;
        }
    if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    const int64_t v0 = h->version;
    HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    h->capturing = true;
    const int st = seq(h->cap_stream);
    h->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (st != DD_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st != DD_OK ? st : fail(DD_E_HIP, "sequence capture: %s", hipGetErrorString(e));
    }
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(DD_E_HIP, "sequence graph instantiate: %s", hipGetErrorString(ei));
    if (h->seq_graphs.size() >= kMaxSeqGraphs) {
        (void)hipGraphExecDestroy(h->seq_graphs.front().exec);
        h->seq_graphs.erase(h->seq_graphs.begin());
    }
    h->seq_graphs.push_back({std::move(key), x, h->version - v0, h->en_lam_valid, h->b_valid, h->f_valid, h->T.F,
                             h->T.B, h->T.lam, h->T.M, h->T.Fpar, h->T.Bch});
    HIP_TRY(hipGraphLaunch(x, s));
    return DD_OK;
}

// State arrays L[0 .. n-1], Mv[0 .. n-1] allocated (save_state fills them).
int reserve_states(dd_instance *h, std::vector<float *> &L, std::vector<float *> &Mv, size_t n) {
    while (L.size() < n) {
        float *a = nullptr, *b = nullptr;
        int st = h->alloc(&a, (size_t)h->edge_slots);
        if (st || (st = h->alloc(&b, (size_t)h->edge_slots))) return st;
        L.push_back(a);
        Mv.push_back(b);
    }
    return DD_OK;
}

// The unrolled forward with its whole trajectory kept on the device: every forward pass writes F
// into an array of its own and every backward pass B (the tables are pointed at them), and the
// state before every pass is kept.  Afterwards the instance is back on its own arrays, with B as
// the last pass left it, so any later call finds it as after an ordinary run.
// Device arrays for a stored run of n iterations: 2n + 1 node-cost arrays and each pass's argmin
// records (the states before the passes are allocated as they are saved).  Bytes still to allocate:
size_t stored_need(const dd_instance *h, int n) {
    // a node-cost array and its argmin codes
    const size_t bytes = ((size_t)h->node_slots + 64) * (sizeof(float) + sizeof(uint16_t)),
                 rec_bytes = (size_t)h->edge_slots * 12;
    size_t need = 0;
    if ((int)h->trF.size() < n) need += ((size_t)n - h->trF.size()) * bytes;
    if ((int)h->trB.size() < n + 1) need += ((size_t)n + 1 - h->trB.size()) * bytes;
    if ((int)h->tr_mrec.size() < 2 * n) need += ((size_t)2 * n - h->tr_mrec.size()) * rec_bytes;
    if ((int)h->tr_Se.size() < 2 * n) need += ((size_t)2 * n - h->tr_Se.size()) * 4 * (size_t)h->edge_slots;
    if ((int)h->tr_lam.size() < 2 * n + 1) need += ((size_t)2 * n + 1 - h->tr_lam.size()) * 8 * (size_t)h->edge_slots;
    return need;
}

// whether they fit in the free device memory with a margin of 2 GiB
bool stored_fits(const dd_instance *h, int n, size_t *need_out = nullptr, size_t *free_out = nullptr) {
    const size_t need = stored_need(h, n);
    size_t free_b = 0, total_b = 0;
    if (need && hipMemGetInfo(&free_b, &total_b) != hipSuccess) return false;
    if (need_out) *need_out = need;
    if (free_out) *free_out = free_b;
    if (need && h->max_device_bytes > 0 && h->device_bytes + (int64_t)need > h->max_device_bytes) return false;
    return need == 0 || need + ((size_t)2 << 30) <= free_b;
}

int stored_alloc(dd_instance *h, int n) {
    const size_t nodes = (size_t)h->node_slots + 64;
    int st;
    while ((int)h->trF.size() < n) {
        float *p = nullptr;
        uint16_t *c = nullptr;
        if ((st = h->alloc(&p, nodes)) || (st = h->alloc(&c, nodes))) return st;
        h->trF.push_back(p);
        h->trFp.push_back(c);
    }
    while ((int)h->trB.size() < n + 1) {
        float *p = nullptr;
        uint16_t *c = nullptr;
        if ((st = h->alloc(&p, nodes)) || (st = h->alloc(&c, nodes))) return st;
        h->trB.push_back(p);
        h->trBc.push_back(c);
    }
    while ((int)h->tr_mrec.size() < 2 * n) {
        int32_t *p = nullptr;
        float *q = nullptr;
        if ((st = h->alloc(&p, 2 * (size_t)h->edge_slots)) || (st = h->alloc(&q, (size_t)h->edge_slots))) return st;
        h->tr_mrec.push_back(p);
        h->tr_mdiff.push_back(q);
    }
    while ((int)h->tr_Se.size() < 2 * n) {
        float *p = nullptr;
        if ((st = h->alloc(&p, (size_t)h->edge_slots))) return st;
        HIP_TRY(hipMemset(p, 0, sizeof(float) * (size_t)h->edge_slots));  // padding slots hold S = 0
        h->tr_Se.push_back(p);
    }
    return DD_OK;
}

// n iterations from the current state, with B at that state already in trB[0]: forward pass t
// writes F into trF[t] and its backward pass B into trB[t + 1] (the tables are re-pointed), every
// pass records its argmins, and the state before every pass is kept.  The tables are left on the
// last arrays.  Sp (or NULL): the S of each of the 2n passes, when a forward already formed them;
// S_out (or NULL): where the passes put the S they form, for a later recomputation.
int stored_passes(dd_instance *h, int n, hipStream_t s, float *const *Sp = nullptr, float *const *S_out = nullptr) {
    float *own_S = h->S;
    auto pass = [&](int dir, int p) {
        if (S_out) {
            h->S = S_out[p];
            h->T.S = S_out[p];
        }
        const int r = run_pass_rec(h, dir, s, h->tr_mrec[p], h->tr_mdiff[p], h->tr_Se[p], Sp ? Sp[p] : nullptr);
        h->S = own_S;
        h->T.S = own_S;
        return r;
    };
    int st = save_state(h, h->tr_lam, h->tr_M, 0, s);
    for (int t = 0; t < n && st == DD_OK; ++t) {
        use_F(h, h->trF[t], h->trFp[t]);
        use_B(h, h->trB[t], h->trBc[t]);
        if ((st = pass(0, 2 * t)) || (st = save_state(h, h->tr_lam, h->tr_M, 2 * (size_t)t + 1, s))) break;
        use_B(h, h->trB[t + 1], h->trBc[t + 1]);
        if ((st = pass(1, 2 * t + 1))) break;
        st = save_state(h, h->tr_lam, h->tr_M, 2 * (size_t)t + 2, s);
    }
    return st;
}

// The reverse of stored_passes: every pass's adjoint from its stored output state, node costs and
// records -- no recomputation, no replay, no copy (the tables point at the stored arrays, which the
// reverse sweeps only read).  The tables' multipliers and M are restored; the node-cost pointers
// are left to the caller.
int stored_reverse(dd_instance *h, int n, float *&dl, float *&dm, float *&dl2, float *&dm2, hipStream_t s) {
    float *own_lam = h->T.lam, *own_M = h->T.M;
    int st = DD_OK;
    for (int t = n - 1; t >= 0 && st == DD_OK; --t) {
        use_F(h, h->trF[t], h->trFp[t]);
        use_B(h, h->trB[t + 1], h->trBc[t + 1]);  // the backward pass of iteration t
        h->T.lam = h->tr_lam[2 * t + 2];
        h->T.M = h->tr_M[2 * t + 2];
        if ((st = pass_vjp(h, 1, dl, dm, dl2, dm2, s, h->tr_lam[2 * t + 1], h->tr_M[2 * t + 1],
                           h->tr_mrec[2 * t + 1], h->tr_mdiff[2 * t + 1], h->tr_Se[2 * t + 1])))
            break;
        std::swap(dl, dl2);
        std::swap(dm, dm2);
        use_B(h, h->trB[t], h->trBc[t]);  // its forward pass
        h->T.lam = h->tr_lam[2 * t + 1];
        h->T.M = h->tr_M[2 * t + 1];
        if ((st = pass_vjp(h, 0, dl, dm, dl2, dm2, s, h->tr_lam[2 * t], h->tr_M[2 * t], h->tr_mrec[2 * t],
                           h->tr_mdiff[2 * t], h->tr_Se[2 * t])))
            break;
        std::swap(dl, dl2);
        std::swap(dm, dm2);
    }
    h->T.lam = own_lam;
    h->T.M = own_M;
    return st;
}

int forward_stored(dd_instance *h, int32_t T, double *lb, bool from_state, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = ((size_t)h->node_slots + 64) * sizeof(float);
    size_t need = 0, free_b = 0;
    if (!stored_fits(h, T, &need, &free_b))
        return fail(DD_E_OOM,
                    "a stored trajectory of %d iterations needs %.1f GB more device memory (%.1f GB free): "
                    "use checkpoints (ckpt_every >= 1)",
                    T, (double)need / 1e9, (double)free_b / 1e9);
    int st;
    if ((st = stored_alloc(h, T))) return st;
    h->F0 = h->T.F;
    h->B0 = h->T.B;
    h->fwd_stored = false;
    use_B(h, h->trB[0], h->trBc[0]);  // B at the start state goes to the first stored array
    if (from_state) {
        if ((st = recompute_B(h, s))) return st;
        h->version++;
    } else if ((st = dd_reset(h, stream))) {
        use_B(h, h->B0, h->Bch0);
        return st;
    }
    if (st == DD_OK) st = reserve_states(h, h->tr_lam, h->tr_M, 2 * (size_t)T + 1);
    if (st == DD_OK) st = replayed(h, {1, T}, s, [&](hipStream_t q) { return stored_passes(h, T, q); });
    if (st == DD_OK) st = dd_lower_bound(h, lb, nullptr, stream);
    const hipError_t e = hipMemcpyAsync(h->B0, h->trB[T], bytes, hipMemcpyDeviceToDevice, s);
    use_F(h, h->F0, h->Fpar0);
    use_B(h, h->B0, h->Bch0);
    h->b_valid = true;   // B of the final state, copied back
    h->f_valid = false;  // the instance's own F was not written
    if (st) return st;
    if (e != hipSuccess) return fail(DD_E_HIP, "copy of the final B: %s", hipGetErrorString(e));
    h->fwd_T = T;
    h->fwd_K = -1;
    h->fwd_stored = true;
    h->fwd_last_stored = false;
    h->fwd_from_state = from_state;
    h->fwd_version = h->version;
    h->fwd_serial++;
    return DD_OK;
}

int forward_unrolled(dd_instance *h, int32_t T, int32_t ckpt_every, double *lb, bool from_state, void *stream) {
    if (!h || T < 0 || !lb) return fail(DD_E_ARG, "bad instance, T or lb");
    if (ckpt_every < -1) return fail(DD_E_ARG, "ckpt_every must be >= -1");
    hipStream_t s = (hipStream_t)stream;
    int st = adj_alloc(h);
    if (st) return st;
    if (ckpt_every == -1) return forward_stored(h, T, lb, from_state, stream);
    h->fwd_stored = false;
    const int K = ckpt_every > 0 ? ckpt_every : (h->ckpt_default > 0 ? h->ckpt_default : 5);
    if (from_state) {
        // a forward pass reads B at its input multipliers
        if ((st = recompute_B(h, s))) return st;
        h->version++;
    } else if ((st = dd_reset(h, stream))) {
        return st;
    }
    const int nseg = (T + K - 1) / K;
    if (h->ck_hash_cap < (size_t)nseg + 1) {  // fingerprints of the checkpoints (the old array stays with the instance)
        const size_t cap = std::max<size_t>(64, (size_t)nseg + 1);
        if ((st = h->alloc(&h->ck_hash, cap))) return st;
        h->ck_hash_cap = cap;
    }
    if ((st = reserve_states(h, h->ck_lam, h->ck_M, (size_t)nseg + 1))) return st;
    // the S of every pass, kept for the backward sweep's recomputed segments
    while (h->fwd_S.size() < 2 * (size_t)T) {
        float *p = nullptr;
        if ((st = h->alloc(&p, (size_t)std::max<int64_t>(h->n, 1)))) return st;
        h->fwd_S.push_back(p);
    }
    // When the device holds a stored run of K iterations (the arrays the backward sweep recomputes
    // each segment into), the last segment runs with the recording passes straight into them: the
    // backward sweep then reverses it without recomputing it.  Same arithmetic, same bits.
    const int t_last = (nseg - 1) * K;
    const bool pre = nseg > 0 && !h->adj_replay && stored_fits(h, K) && stored_alloc(h, K) == DD_OK &&
                     reserve_states(h, h->tr_lam, h->tr_M, 2 * (size_t)K + 1) == DD_OK;
    // T iterations with a checkpoint (state and fingerprint) every K and one of the final state
    st = replayed(h, {2, T, K, (int64_t)pre}, s, [&](hipStream_t q) {
        auto checkpoint = [&](size_t i) {
            int r = save_state(h, h->ck_lam, h->ck_M, i, q);
            return r ? r : state_hash(h, h->ck_lam[i], h->ck_M[i], h->ck_hash + i, q);
        };
        float *own_S = h->S;
        int r = DD_OK;
        for (int t = 0; t < T && r == DD_OK; ++t) {
            if (t % K == 0 && (r = checkpoint((size_t)(t / K)))) break;
            if (pre && t == t_last) {
                float *own_F = h->T.F, *own_B = h->T.B;
                uint16_t *own_Fp = h->T.Fpar, *own_Bc = h->T.Bch;
                h->S = own_S;
                h->T.S = own_S;
                use_B(h, h->trB[0], h->trBc[0]);  // B at the checkpoint, with its argmin codes
                r = recompute_B(h, q);
                if (r == DD_OK) r = stored_passes(h, T - t_last, q, nullptr, h->fwd_S.data() + 2 * (size_t)t_last);
                use_F(h, own_F, own_Fp);
                use_B(h, own_B, own_Bc);
                break;
            }
            for (int d = 0; d < 2 && r == DD_OK; ++d) {
                h->S = h->fwd_S[2 * (size_t)t + d];  // the pass's deferred sums go here
                h->T.S = h->S;
                r = dd_run_pass(h, d, q);
            }
        }
        h->S = own_S;
        h->T.S = own_S;
        return r ? r : checkpoint((size_t)nseg);
    });
    if (st) return st;
    if (pre) {
        // the instance's own B takes the final B (its own F was not written by the recorded passes)
        const size_t bytes = ((size_t)h->node_slots + 64) * sizeof(float);
        HIP_TRY(hipMemcpyAsync(h->T.B, h->trB[T - t_last], bytes, hipMemcpyDeviceToDevice, s));
        h->b_valid = true;
        h->f_valid = false;
    }
    if ((st = dd_lower_bound(h, lb, nullptr, stream))) return st;
    h->fwd_T = T;
    h->fwd_K = K;
    h->fwd_last_stored = pre;
    h->fwd_from_state = from_state;
    h->fwd_version = h->version;
    h->fwd_serial++;
    return DD_OK;
}

// The launches of the backward sweep up to the adjoints of the start state (in dlamA / dMA: every pass
// adjoint swaps the buffer pairs, and there are 2T of them); d_alpha and d_omega accumulate in the
// slot-ordered dalpha / domega.  The seed is read from seed_dev.
int backward_core(dd_instance *h, int T, int K, bool stored, bool seg_store, bool last_stored, hipStream_t s) {
    const int nseg = (T + K - 1) / K;
    int st;
    // adjoint of the lower bound at the final state: dLB / dlambda_bar_j = argmin assignment of row j
    if (stored) st = load_state(h, h->tr_lam, h->tr_M, 2 * (size_t)T, s);
    else st = load_state(h, h->ck_lam, h->ck_M, (size_t)nseg, s);
    if (st == DD_OK && !stored) st = verify_state(h, h->T.lam, h->T.M, (size_t)nseg, s);
    if (st) return st;
    if ((st = deferred(h, s))) return st;
    // a stored trajectory keeps the final B in B0: the bound's B goes to the spare array (with its codes)
    if (stored) use_B(h, h->F0, h->Fpar0);
    st = all_classes(h, false, BWD_STORE_BAR, s);
    if (st) {
        use_B(h, h->B0, h->Bch0);
        return st;
    }
    HIP_TRY(launch_fill(h->dalpha, 0.f, h->edge_slots, s));
    HIP_TRY(launch_fill(h->domega, 0.f, h->edge_slots, s));
    HIP_TRY(launch_fill(h->dlamA, 0.f, h->edge_slots, s));
    {
        AdjTables A{};
        A.lam_src = h->T.lam;
        A.dlam_in = h->dlamA;
        A.seed = h->seed_dev;
        if ((st = adj_classes(h, A, ADJ_B_FIXED, 1, 0, 0.f, s))) return st;
    }
    // lambda_bar = lambda + alpha S(M): dlambda = dlambda_bar, d_alpha += dlambda_bar S, dM = dS
    HIP_TRY(launch_flush_adj(h->T.evar, h->S, h->alpha, h->dlamA, h->dalpha, h->g, h->edge_slots, s));
    if ((st = adj_deferred(h, h->dMA, s))) return st;
    float *dl = h->dlamA, *dm = h->dMA, *dl2 = h->dlamB, *dm2 = h->dMB;
    if (stored) {
        st = stored_reverse(h, T, dl, dm, dl2, dm2, s);
        use_F(h, h->F0, h->Fpar0);
        use_B(h, h->B0, h->Bch0);
        if (st) return st;
    }
    // checkpoint segments: when the device holds a stored run of K iterations, each segment is
    // recomputed into the stored-trajectory arrays and reversed like a stored trajectory (no pass
    // replayed); otherwise the pass inputs are recomputed and each pass is replayed for its adjoint.
    // Checkpoints are verified against the fingerprints taken when they were saved: when loaded, and
    // at the end of each recomputed segment (the recomputation must reproduce the next checkpoint).
    float *own_F = h->T.F, *own_B = h->T.B;
    uint16_t *own_Fp = h->T.Fpar, *own_Bc = h->T.Bch;
    for (int seg = stored ? -1 : nseg - 1; seg >= 0; --seg) {
        const int t0 = seg * K, t1 = std::min(T, t0 + K), np = 2 * (t1 - t0);
        if (last_stored && seg == nseg - 1) {
            // the unrolled forward ran this segment into the stored arrays
            st = stored_reverse(h, t1 - t0, dl, dm, dl2, dm2, s);
            use_F(h, own_F, own_Fp);
            use_B(h, own_B, own_Bc);
            if (st) return st;
            continue;
        }
        if ((st = load_state(h, h->ck_lam, h->ck_M, (size_t)seg, s))) return st;
        if ((st = verify_state(h, h->T.lam, h->T.M, (size_t)seg, s))) return st;
        if (seg_store) {
            use_B(h, h->trB[0], h->trBc[0]);  // B at the checkpoint goes to the first stored array
            st = recompute_B(h, s);
            if (st == DD_OK) st = stored_passes(h, t1 - t0, s, h->fwd_S.data() + 2 * (size_t)t0);
            if (st == DD_OK) st = verify_state(h, h->tr_lam[np], h->tr_M[np], (size_t)seg + 1, s);
            if (st == DD_OK) st = stored_reverse(h, t1 - t0, dl, dm, dl2, dm2, s);
            use_F(h, own_F, own_Fp);
            use_B(h, own_B, own_Bc);
            if (st) return st;
            continue;
        }
        // a forward pass reads B at its input multipliers: the backward pass before it left
        // exactly that, so rebuild it from the checkpoint (same expression, same bits)
        if ((st = recompute_B(h, s))) return st;
        // recompute the pass inputs of the segment; the last two passes record (the last one's argmins,
        // and the argmin codes of both: the last pass's reverse sweeps read the F its forward pass left)
        for (int q = 0; q < np; ++q) {
            if ((st = save_state(h, h->seg_lam, h->seg_M, (size_t)q, s))) return st;
            // (the last also keeps its input's S per edge for its adjoint)
            if ((st = q >= np - 2 ? run_pass_rec(h, q % 2, s, nullptr, nullptr, q == np - 1 ? h->Se : nullptr)
                                  : dd_run_pass(h, q % 2, s)))
                return st;
        }
        if ((st = verify_state(h, h->T.lam, h->T.M, (size_t)seg + 1, s))) return st;
        for (int q = np - 1; q >= 0; --q) {
            if (q == np - 1) {
                // the recomputation just ran this pass: its outputs and both node sides are in place
                // (a segment ends with a backward pass, whose fixed side is the F its forward pass left)
                if ((st = pass_vjp(h, q % 2, dl, dm, dl2, dm2, s, h->seg_lam[q], h->seg_M[q], h->mrec, h->mdiff,
                                   h->Se)))
                    return st;
            } else {
                if ((st = load_state(h, h->seg_lam, h->seg_M, (size_t)q, s))) return st;
                if ((st = pass_vjp(h, q % 2, dl, dm, dl2, dm2, s))) return st;
            }
            std::swap(dl, dl2);
            std::swap(dm, dm2);
        }
    }
    if (dl != h->dlamA || dm != h->dMA) return fail(DD_E_STATE, "internal: pass adjoints out of step");
    return DD_OK;
}

int backward(dd_instance *h, double dlb, float *d_omega, float *d_alpha, float *d_c, float *d_lam0, float *d_M0,
             void *stream) {
    if (!h) return fail(DD_E_ARG, "NULL instance");
    if (h->fwd_T < 0 || h->fwd_version != h->version)
        return fail(DD_E_STATE, "the backward sweep needs the state left by an unrolled forward");
    if (d_c && h->fwd_from_state)
        return fail(DD_E_ARG, "d_c needs an unrolled forward from the reset state (lambda = c/|J_i|)");
    hipStream_t s = (hipStream_t)stream;
    const bool stored = h->fwd_stored;
    const int T = h->fwd_T, K = stored ? 1 : h->fwd_K, nseg = (T + K - 1) / K;
    const float seed = (float)dlb;
    int st;
    // the buffers of the launch sequence, allocated beforehand
    if (!h->seed_dev && (st = h->alloc(&h->seed_dev, 1))) return st;
    const bool last_stored = !stored && h->fwd_last_stored;
    const bool seg_store =
        last_stored || (!stored && !h->adj_replay && nseg > 0 && stored_fits(h, K) && stored_alloc(h, K) == DD_OK);
    if (!stored && !seg_store && (st = reserve_states(h, h->seg_lam, h->seg_M, 2 * (size_t)K))) return st;
    if (seg_store && (st = reserve_states(h, h->tr_lam, h->tr_M, 2 * (size_t)K + 1))) return st;
    HIP_TRY(launch_fill(h->seed_dev, seed, 1, s));
    if (!stored) HIP_TRY(launch_fill((float *)h->ck_flag, 0.f, 1, s));
    st = replayed(h, {3, T, K, stored, seg_store, last_stored}, s,
                  [&](hipStream_t q) { return backward_core(h, T, K, stored, seg_store, last_stored, q); });
    // the other segments were recomputed into the same arrays: a later backward sweep of this forward
    // recomputes the last one too
    if (nseg > 1) h->fwd_last_stored = false;
    if (st) return st;
    float *dl = h->dlamA, *dm = h->dMA;
    // lambda_0 = c / |J_i|
    if (d_c) {  // per variable in the library's order, then in the caller's
        HIP_TRY(launch_dc(h->var_ptr, h->var_slots, dl, h->cdev, seed, h->scratch_n, (int)h->n, s));
        HIP_TRY(launch_gather(h->var_perm, h->scratch_n, d_c, h->n, nullptr, s));
    }
    if (d_lam0) HIP_TRY(launch_gather(h->canon2slot, dl, d_lam0, h->E, nullptr, s));
    if (d_M0) HIP_TRY(launch_gather(h->canon2slot, dm, d_M0, h->E, nullptr, s));
    if (d_omega) HIP_TRY(launch_gather(h->canon2slot, h->domega, d_omega, h->E, nullptr, s));
    if (d_alpha) HIP_TRY(launch_gather(h->canon2slot, h->dalpha, d_alpha, h->E, nullptr, s));
    // leave the solver at the final state of the recorded forward (a stored trajectory left the
    // final B in B0, which the backward sweep did not touch)
    if (stored) {
        if ((st = load_state(h, h->tr_lam, h->tr_M, 2 * (size_t)T, s))) return st;
        h->b_valid = true;  // B0 still holds the final B
    } else {
        if ((st = load_state(h, h->ck_lam, h->ck_M, (size_t)nseg, s))) return st;
        if ((st = recompute_B(h, s))) return st;
        int32_t *flag = (int32_t *)h->red_host;
        HIP_TRY(hipMemcpyAsync(flag, h->ck_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (*flag)
            return fail(DD_E_CHECKPOINT,
                        "a checkpoint of the unrolled forward no longer has the fingerprint taken when it was "
                        "saved, or recomputing a segment from it did not reproduce the next one");
    }
    h->fwd_version = h->version;
    return DD_OK;
}

}  // namespace

extern "C" {

int dd_forward_unrolled(dd_instance *h, int32_t T, int32_t ckpt_every, double *lb, void *stream) {
    return forward_unrolled(h, T, ckpt_every, lb, false, stream);
}

int dd_forward_unrolled_from_state(dd_instance *h, int32_t T, int32_t ckpt_every, double *lb, void *stream) {
    return forward_unrolled(h, T, ckpt_every, lb, true, stream);
}

int dd_corrupt_checkpoint(dd_instance *h, int32_t index) {
    if (!h) return fail(DD_E_ARG, "NULL instance");
    if (h->fwd_T < 0 || h->fwd_version != h->version || h->fwd_stored)
        return fail(DD_E_STATE, "no checkpointed unrolled forward is recorded");
    const int nseg = (h->fwd_T + h->fwd_K - 1) / h->fwd_K;
    if (index < 0 || index > nseg) return fail(DD_E_ARG, "checkpoint %d out of range [0, %d]", index, nseg);
    float v = 0.f;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(&v, h->ck_lam[index], sizeof v, hipMemcpyDeviceToHost));
    v += 1.f;
    HIP_TRY(hipMemcpy(h->ck_lam[index], &v, sizeof v, hipMemcpyHostToDevice));
    return DD_OK;
}

int dd_record_serial(const dd_instance *h, int64_t *serial) {
    if (!h || !serial) return fail(DD_E_ARG, "NULL argument");
    *serial = h->fwd_T >= 0 && h->fwd_version == h->version ? h->fwd_serial : -1;
    return DD_OK;
}

int dd_backward(dd_instance *h, double dlb, float *d_omega, float *d_alpha, float *d_c, void *stream) {
    return backward(h, dlb, d_omega, d_alpha, d_c, nullptr, nullptr, stream);
}

int dd_backward_state(dd_instance *h, double dlb, float *d_omega, float *d_alpha, float *d_lam0, float *d_M0,
                      void *stream) {
    return backward(h, dlb, d_omega, d_alpha, nullptr, d_lam0, d_M0, stream);
}

int dd_param_transform(dd_instance *h, const float *omega_hat, const float *alpha_hat, const float *theta_hat,
                       float *omega, float *alpha, float *theta, void *stream) {
    if (!h || (h->E && (!omega_hat || !alpha_hat || !omega || !alpha || (!theta_hat != !theta))))
        return fail(DD_E_ARG, "NULL argument");
    HIP_TRY(launch_param_transform(h->var_ptr, h->var_canon, omega_hat, alpha_hat, theta_hat, omega, alpha, theta,
                                   (int)h->n, (hipStream_t)stream));
    return DD_OK;
}

int dd_param_transform_vjp(dd_instance *h, const float *omega, const float *alpha, const float *d_omega,
                           const float *d_alpha, const float *d_theta, float *d_omega_hat, float *d_alpha_hat,
                           float *d_theta_hat, void *stream) {
    if (!h || (h->E && (!omega || !alpha || !d_omega || !d_alpha || !d_omega_hat || !d_alpha_hat ||
                        (!d_theta != !d_theta_hat))))
        return fail(DD_E_ARG, "NULL argument");
    HIP_TRY(launch_param_transform_vjp(h->var_ptr, h->var_canon, omega, alpha, d_omega, d_alpha, d_theta, d_omega_hat,
                                       d_alpha_hat, d_theta_hat, (int)h->n, (hipStream_t)stream));
    return DD_OK;
}

int dd_nonparam_update(dd_instance *h, const float *theta_hat, void *stream) {
    if (!h || (h->E && !theta_hat)) return fail(DD_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_nonparam_update(h->var_ptr, h->var_canon, h->canon2slot, theta_hat, h->T.lam, (int)h->n, s));
    h->version++;
    h->f_valid = h->b_valid = false;
    return recompute_B(h, s);
}

int dd_smoothed(dd_instance *h, float tau, int32_t flushed, float *E_out, float *p_out, void *stream) {
    if (!h || !(tau > 0.f) || !std::isfinite(tau) || (h->E && !p_out)) return fail(DD_E_ARG, "bad argument");
    int st;
    if (!h->Qs && (st = h->alloc(&h->Qs, (size_t)(h->node_slots + 64)))) return st;
    return smoothed_sweeps(h, h->Qs, tau, flushed, E_out, p_out, (hipStream_t)stream);
}

int dd_argmin_assignment(dd_instance *h, int32_t flushed, float *x_out, void *stream) {
    if (!h || (h->E && !x_out)) return fail(DD_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    int st = adj_alloc(h);
    if (st) return st;
    // a pull sweep with a unit adjoint at every root routes it along each row's minimizing path:
    // the adjoint that crosses hi arcs is x*
    if (flushed && (st = deferred(h, s))) return st;
    if ((st = all_classes(h, false, flushed ? BWD_STORE_BAR : BWD_STORE, s))) return st;
    HIP_TRY(launch_fill(h->dlamA, 0.f, h->edge_slots, s));
    AdjTables A{};
    A.lam_src = h->T.lam;
    A.dlam_in = h->dlamA;
    if ((st = adj_classes(h, A, ADJ_B_FIXED, flushed ? 1 : 0, 0, 1.f, s))) return st;
    HIP_TRY(launch_gather(h->canon2slot, h->dlamA, x_out, h->E, nullptr, s));
    return flushed ? recompute_B(h, s) : DD_OK;  // B at the multipliers again
}

int dd_solve(dd_instance *h, int32_t T, int32_t max_rounds, double rel_tol, double *lb_trace, double *ms_trace,
             int32_t *rounds, void *stream) {
    if (!h || T < 1 || max_rounds < 0 || !(rel_tol >= 0.0) || !lb_trace || !ms_trace || !rounds)
        return fail(DD_E_ARG, "bad argument");
    const auto t0 = std::chrono::steady_clock::now();
    auto elapsed_ms = [&] {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    };
    int st = dd_lower_bound(h, &lb_trace[0], nullptr, stream);
    if (st) return st;
    ms_trace[0] = elapsed_ms();
    *rounds = 0;
    for (int r = 1; r <= max_rounds; ++r) {
        if ((st = dd_run(h, T, stream))) return st;
        if ((st = dd_lower_bound(h, &lb_trace[r], nullptr, stream))) return st;  // synchronizes
        ms_trace[r] = elapsed_ms();
        *rounds = r;
        const double prev = lb_trace[r - 1];
        if ((lb_trace[r] - prev) < rel_tol * std::max(std::fabs(prev), 1e-300)) break;
    }
    return DD_OK;
}

int dd_gap_integral(const double *lb, const double *ms, int32_t k, double d_star, double *g_out,
                    double *g_integral) {
    if (!lb || !ms || k < 1 || !g_integral) return fail(DD_E_ARG, "bad argument");
    const double span = d_star - lb[0];
    double gi = 0.0;
    for (int i = 0; i < k; ++i) {
        const double g = span > 0.0 ? std::min((d_star - lb[i]) / span, 1.0) : 0.0;
        if (g_out) g_out[i] = g;
        if (i + 1 < k) gi += g * (ms[i + 1] - ms[i]) * 1e-3;  // each value holds until the next
    }
    *g_integral = gi;
    return DD_OK;
}

int dd_seg_softmax_vjp(dd_instance *h, const float *alpha, const float *d_alpha, float *d_alpha_hat, void *stream) {
    if (!h || (h->E && (!alpha || !d_alpha || !d_alpha_hat))) return fail(DD_E_ARG, "NULL argument");
    HIP_TRY(launch_softmax_vjp(h->var_ptr, h->var_canon, alpha, d_alpha, d_alpha_hat, (int)h->n, (hipStream_t)stream));
    return DD_OK;
}

int dd_set_costs(dd_instance *h, const float *c, void *stream) {
    if (!h || (h->n && !c)) return fail(DD_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    int st = adj_alloc(h);
    if (st) return st;
    HIP_TRY(launch_scatter(h->var_perm, c, h->cdev, h->n, s));  // the library's variable order
    HIP_TRY(launch_uncovered(h->var_ptr, h->cdev, h->scratch_n, (int)h->n, s));
    HIP_TRY(launch_sum(h->scratch_n, h->n, 0, h->partial, h->red, s));
    HIP_TRY(hipMemcpyAsync(h->red_host, h->red, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    h->unc_const = h->red_host[0];
    return dd_reset(h, stream);
}

int dd_row_nodes(const dd_instance *h, int64_t *nodes_out) {
    if (!h || (h->m && !nodes_out)) return fail(DD_E_ARG, "NULL argument");
    std::copy(h->row_nodes.begin(), h->row_nodes.end(), nodes_out);
    return DD_OK;
}

int dd_profile_begin(dd_instance *h, int32_t max_launches) {
    if (!h || max_launches <= 0) return fail(DD_E_ARG, "bad instance or max_launches");
    while (h->pool.size() < 2 * (size_t)max_launches) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        h->pool.push_back(e);
    }
    h->pool_used = 0;
    h->recs.clear();
    h->prof = true;
    return DD_OK;
}

int dd_profile_end(dd_instance *h, dd_kernel_time *out, int32_t cap, int32_t *count) {
    if (!h || !count) return fail(DD_E_ARG, "NULL argument");
    h->prof = false;
    HIP_TRY(hipDeviceSynchronize());
    std::vector<double> ms(h->kname.size(), 0.0);
    std::vector<int64_t> cnt(h->kname.size(), 0);
    for (const auto &r : h->recs) {
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
        ms[r.kernel] += t;
        cnt[r.kernel] += 1;
    }
    int k = 0;
    for (size_t q = 0; q < h->kname.size(); ++q) {
        if (!cnt[q]) continue;
        if (out && k < cap) {
            snprintf(out[k].name, sizeof out[k].name, "%s", h->kname[q].c_str());
            out[k].launches = cnt[q];
            out[k].total_ms = ms[q];
            out[k].bytes_per_launch = h->kbytes[q];
        }
        ++k;
    }
    *count = k;
    h->recs.clear();
    h->pool_used = 0;
    return DD_OK;
}

}  // extern "C"
