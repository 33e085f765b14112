// bdd.cpp -- linear row -> quasi-reduced ordered decision diagram (App. B).
//
// States at level l are partial sums s = sum_{p<l} a_p x_p.  Two kinds of states are
// collapsed before any node is made: states from which no completion is feasible are
// dropped (they would only lead to the 0-terminal), and states from which every
// completion is feasible become one "always true" state.  Then, bottom-up, states with
// the same (lo child, hi child) pair are merged into one node; a state whose two arcs
// both reach the 0-terminal is itself dropped.  No level is ever skipped, so every
// root-to-1 path crosses exactly one node per variable, as the paper's node sets P_i
// require.
//
// Nodes of a level are numbered in increasing partial sum: a node's children are the
// classes of s and s + a_l one level below, so both child numbers are non-decreasing in the
// node number, up to the point where they reach the 0-terminal.  The always-true node stands
// for the smallest sums of a <= row (numbered first) and the largest of a >= row (last).
#include "bdd.hpp"

#include <algorithm>
#include <climits>

namespace dd {
namespace {

constexpr int64_t kTrue = INT64_MAX;  // "every completion feasible"
constexpr int64_t kDead = INT64_MIN;  // "no completion feasible"
constexpr int kBot = -1, kTop = -2;   // child codes before level-relative encoding

struct Classifier {
    const std::vector<int64_t> &minrest, &maxrest;
    int sense;
    int64_t rhs;
    int64_t operator()(int64_t s, int l) const {
        int64_t lo = s + minrest[l], hi = s + maxrest[l];
        if (sense < 0) return lo > rhs ? kDead : (hi <= rhs ? kTrue : s);
        if (sense > 0) return hi < rhs ? kDead : (lo >= rhs ? kTrue : s);
        if (lo > rhs || hi < rhs) return kDead;
        return lo == hi ? kTrue : s;
    }
};

inline uint64_t pair_key(int c0, int c1) { return (uint64_t)(uint32_t)(c0 + 2) << 32 | (uint32_t)(c1 + 2); }

}  // namespace

int compile_row(int L, const int32_t *a, int sense, int64_t rhs, RowBdd &out, CompileScratch &scr) {
    out = RowBdd();
    if (L <= 0) return E_ARG;
    std::vector<int64_t> minrest(L + 1, 0), maxrest(L + 1, 0);
    for (int l = L - 1; l >= 0; --l) {
        if (a[l] == 0) return E_ARG;
        minrest[l] = minrest[l + 1] + std::min<int64_t>(0, a[l]);
        maxrest[l] = maxrest[l + 1] + std::max<int64_t>(0, a[l]);
    }
    const int64_t smin = minrest[0], smax = maxrest[0];
    const int64_t range = smax - smin + 1;
    if (range > (int64_t)1 << 26) return E_UNSUPPORTED;
    Classifier classify{minrest, maxrest, sense, rhs};

    // ---- forward: live partial sums per level ----
    if ((int)scr.states.size() < L + 1) scr.states.resize(L + 1);
    scr.has_true.assign(L + 1, 0);
    for (int l = 0; l <= L; ++l) scr.states[l].clear();
    {
        int64_t k = classify(0, 0);
        if (k == kDead) return E_INFEASIBLE;
        if (k == kTrue) scr.has_true[0] = 1;
        else scr.states[0].push_back(0);
    }
    for (int l = 0; l < L; ++l) {
        const std::vector<int64_t> &cur = scr.states[l];
        std::vector<int64_t> &nxt = scr.states[l + 1];
        const int64_t al = a[l];
        size_t i = 0, j = 0, n = cur.size();
        int64_t last = kDead;
        while (i < n || j < n) {  // merge cur and cur + a_l, both ascending
            int64_t v;
            if (j >= n || (i < n && cur[i] <= cur[j] + al)) v = cur[i++];
            else v = cur[j++] + al;
            if (v == last) continue;
            last = v;
            int64_t k = classify(v, l + 1);
            if (k == kDead) continue;
            if (k == kTrue) { scr.has_true[l + 1] = 1; continue; }
            nxt.push_back(k);
        }
        if (scr.has_true[l]) scr.has_true[l + 1] = 1;
        if ((int64_t)nxt.size() > kMaxWidth) return E_UNSUPPORTED;
    }
    if (!scr.has_true[L]) return E_INFEASIBLE;

    // ---- backward: merge states with equal child pairs into nodes ----
    scr.index.assign((size_t)range, kBot);
    std::vector<std::vector<uint32_t>> level_arcs(L);
    std::vector<int32_t> width(L + 1, 0);
    std::vector<int32_t> ids;
    int true_next = kTop;  // id of the always-true state one level below (the 1-terminal at level L)
    for (int l = L - 1; l >= 0; --l) {
        const std::vector<int64_t> &st = scr.states[l];
        const int64_t al = a[l];
        size_t cap = 16;
        while (cap < 2 * (st.size() + 1)) cap <<= 1;
        scr.table_keys.assign(cap, UINT64_MAX);
        scr.table_vals.resize(cap);
        std::vector<int> lo_list, hi_list;
        int W = 0;
        auto child = [&](int64_t v) -> int {
            int64_t k = classify(v, l + 1);
            if (k == kDead) return kBot;
            if (k == kTrue) return true_next;
            return scr.index[(size_t)(k - smin)];
        };
        auto node_for = [&](int c0, int c1) -> int {
            if (c0 == kBot && c1 == kBot) return kBot;
            uint64_t key = pair_key(c0, c1);
            size_t hsh = (size_t)((key * 0x9E3779B97F4A7C15ull) >> 20) & (cap - 1);
            while (scr.table_keys[hsh] != UINT64_MAX) {
                if (scr.table_keys[hsh] == key) return scr.table_vals[hsh];
                hsh = (hsh + 1) & (cap - 1);
            }
            scr.table_keys[hsh] = key;
            scr.table_vals[hsh] = W;
            lo_list.push_back(c0);
            hi_list.push_back(c1);
            return W++;
        };
        ids.resize(st.size());
        int true_here = kBot;
        const bool true_first = sense < 0;
        if (scr.has_true[l] && true_first) true_here = node_for(true_next, true_next);
        for (size_t t = 0; t < st.size(); ++t) ids[t] = node_for(child(st[t]), child(st[t] + al));
        if (scr.has_true[l] && !true_first) true_here = node_for(true_next, true_next);
        if (W > kMaxWidth) return E_UNSUPPORTED;
        // the dense index now describes this level
        for (int64_t s : scr.states[l + 1]) scr.index[(size_t)(s - smin)] = kBot;
        for (size_t t = 0; t < st.size(); ++t) scr.index[(size_t)(st[t] - smin)] = ids[t];
        true_next = true_here;
        width[l] = W;
        // encode children relative to the next level's width
        const int Wn = width[l + 1];
        std::vector<uint32_t> &arcs = level_arcs[l];
        arcs.resize(W);
        bool any_lo = false, any_hi = false;
        for (int v = 0; v < W; ++v) {
            int c0 = lo_list[v], c1 = hi_list[v];
            uint32_t e0 = c0 == kBot ? (uint32_t)Wn : c0 == kTop ? (uint32_t)Wn + 1 : (uint32_t)c0;
            uint32_t e1 = c1 == kBot ? (uint32_t)Wn : c1 == kTop ? (uint32_t)Wn + 1 : (uint32_t)c1;
            any_lo |= c0 != kBot;
            any_hi |= c1 != kBot;
            arcs[v] = e0 | (e1 << 16);
        }
        if (W == 0) return E_INFEASIBLE;
        if (!any_lo || !any_hi) return E_FORCED;
    }
    for (int64_t s : scr.states[0]) scr.index[(size_t)(s - smin)] = kBot;
    if (width[0] != 1) return E_INFEASIBLE;

    out.L = L;
    out.width.assign(width.begin(), width.begin() + L);
    size_t total = 0;
    for (int l = 0; l < L; ++l) total += width[l];
    out.arcs.reserve(total);
    for (int l = 0; l < L; ++l) {
        out.arcs.insert(out.arcs.end(), level_arcs[l].begin(), level_arcs[l].end());
        out.max_width = std::max(out.max_width, width[l]);
    }
    return OK;
}

}  // namespace dd
