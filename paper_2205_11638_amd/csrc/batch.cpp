// batch.cpp -- many binary programs packed into one device instance.
//
// The programs are concatenated into one disjoint union (variables and rows of program q
// follow those of program q-1).  Rows are the unit of work and the deferred sums S_i are
// per variable, so a pass over the union computes, for every program, exactly the pass it
// would compute alone, while the whole batch costs one launch per kernel class per pass and
// its tiles mix rows of all programs.  Per-program bounds are segmented reductions over the
// union's per-row energies.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/dd.h"
#include "instance.hpp"
#include "kernels.hpp"

using namespace ddi;

struct dd_batch {
    dd_instance *h = nullptr;
    int k = 0;
    std::vector<int64_t> var_off, row_off, edge_off;  // [k+1]
    std::vector<double> unc_const;                     // [k] sum of min(0, c_i) over the program's uncovered variables
    int64_t *row_seg = nullptr, *edge_seg = nullptr;   // device copies of row_off / edge_off
    double *sums = nullptr;                            // device [3k]
    double *sums_host = nullptr;                       // pinned [3k]

    ~dd_batch() {
        if (row_seg) (void)hipFree(row_seg);
        if (edge_seg) (void)hipFree(edge_seg);
        if (sums) (void)hipFree(sums);
        if (sums_host) (void)hipHostFree(sums_host);
        if (h) dd_destroy(h);
    }
};

extern "C" {

int dd_batch_create(const dd_problem *probs, int32_t k, const dd_options *opt, void *stream, dd_batch **out) {
    if (!out) return fail(DD_E_ARG, "out is NULL");
    *out = nullptr;
    if (k <= 0 || !probs) return fail(DD_E_ARG, "need k >= 1 programs");
    dd_batch *b = new dd_batch();
    b->k = k;
    b->var_off.assign((size_t)k + 1, 0);
    b->row_off.assign((size_t)k + 1, 0);
    b->edge_off.assign((size_t)k + 1, 0);
    for (int q = 0; q < k; ++q) {
        const dd_problem &p = probs[q];
        if (p.n < 0 || p.m < 0 || !p.row_ptr || (p.m > 0 && p.row_ptr[0] != 0)) {
            delete b;
            return fail(DD_E_ARG, "program %d: bad sizes or row_ptr", q);
        }
        b->var_off[q + 1] = b->var_off[q] + p.n;
        b->row_off[q + 1] = b->row_off[q] + p.m;
        b->edge_off[q + 1] = b->edge_off[q] + p.row_ptr[p.m];
    }
    if (b->var_off[k] >= INT32_MAX || b->row_off[k] >= INT32_MAX) {
        delete b;
        return fail(DD_E_UNSUPPORTED, "the batch has more than 2^31 variables or rows");
    }
    // the union, in host memory (validated again, row by row, by dd_create)
    const int64_t n = b->var_off[k], m = b->row_off[k], E = b->edge_off[k];
    std::vector<double> c((size_t)n);
    std::vector<int64_t> row_ptr((size_t)m + 1, 0), rhs((size_t)m);
    std::vector<int32_t> col((size_t)E), coef((size_t)E);
    std::vector<int8_t> sense((size_t)m);
    b->unc_const.assign((size_t)k, 0.0);
    for (int q = 0; q < k; ++q) {
        const dd_problem &p = probs[q];
        const int64_t v0 = b->var_off[q], r0 = b->row_off[q], e0 = b->edge_off[q];
        if ((p.n > 0 && !p.c) || (p.row_ptr[p.m] > 0 && (!p.col || !p.coef)) || (p.m > 0 && (!p.sense || !p.rhs))) {
            delete b;
            return fail(DD_E_ARG, "program %d: NULL array", q);
        }
        std::vector<char> used((size_t)p.n, 0);
        for (int64_t e = 0; e < p.row_ptr[p.m]; ++e) {
            if (p.col[e] < 0 || p.col[e] >= p.n) {
                delete b;
                return fail(DD_E_ARG, "program %d: variable out of range", q);
            }
            used[p.col[e]] = 1;
            col[e0 + e] = (int32_t)(p.col[e] + v0);
            coef[e0 + e] = p.coef[e];
        }
        for (int i = 0; i < p.n; ++i) {
            c[v0 + i] = p.c[i];
            if (!used[i] && p.c[i] < 0) b->unc_const[q] += p.c[i];
        }
        for (int j = 0; j < p.m; ++j) {
            row_ptr[r0 + j + 1] = e0 + p.row_ptr[j + 1];
            sense[r0 + j] = p.sense[j];
            rhs[r0 + j] = p.rhs[j];
        }
    }
    dd_problem u{(int32_t)n, c.data(), (int32_t)m, row_ptr.data(), col.data(), coef.data(), sense.data(), rhs.data()};
    // locality: the programs in eight buckets of about equal edge count (by the middle of each
    // program's edge range), whose rows keep to consecutive tiles.  The per-slot kernels hand each of
    // the chip's 8 L2 slices one eighth of the slot range, so each slice mostly gathers the S of its
    // own bucket's programs.
    std::vector<int32_t> group((size_t)m);
    for (int q = 0; q < k; ++q) {
        const int64_t mid2 = b->edge_off[q] + b->edge_off[q + 1];  // twice the middle
        const int g = E > 0 ? (int)std::min<int64_t>(7, (8 * mid2) / (2 * E)) : 0;
        for (int64_t j = b->row_off[q]; j < b->row_off[q + 1]; ++j) group[(size_t)j] = g;
    }
    int st = create_grouped(&u, opt, stream, group.data(), &b->h);
    if (st) {
        delete b;
        return st;
    }
    auto hip_ok = [&](hipError_t e) { return e == hipSuccess ? DD_OK : fail(DD_E_HIP, "%s", hipGetErrorString(e)); };
    hipStream_t s = (hipStream_t)stream;
    if ((st = hip_ok(hipMalloc((void **)&b->row_seg, sizeof(int64_t) * (k + 1)))) ||
        (st = hip_ok(hipMalloc((void **)&b->edge_seg, sizeof(int64_t) * (k + 1)))) ||
        (st = hip_ok(hipMalloc((void **)&b->sums, sizeof(double) * 3 * k))) ||
        (st = hip_ok(hipHostMalloc((void **)&b->sums_host, sizeof(double) * 3 * k, hipHostMallocDefault))) ||
        (st = hip_ok(hipMemcpyAsync(b->row_seg, b->row_off.data(), sizeof(int64_t) * (k + 1), hipMemcpyHostToDevice,
                                    s))) ||
        (st = hip_ok(hipMemcpyAsync(b->edge_seg, b->edge_off.data(), sizeof(int64_t) * (k + 1),
                                    hipMemcpyHostToDevice, s))) ||
        (st = hip_ok(hipStreamSynchronize(s)))) {
        delete b;
        return st;
    }
    *out = b;
    return DD_OK;
}

int dd_batch_destroy(dd_batch *b) {
    delete b;
    return DD_OK;
}

dd_instance *dd_batch_instance(dd_batch *b) { return b ? b->h : nullptr; }

int dd_batch_offsets(const dd_batch *b, int64_t *var_off, int64_t *row_off, int64_t *edge_off) {
    if (!b) return fail(DD_E_ARG, "NULL batch");
    for (int q = 0; q <= b->k; ++q) {
        if (var_off) var_off[q] = b->var_off[q];
        if (row_off) row_off[q] = b->row_off[q];
        if (edge_off) edge_off[q] = b->edge_off[q];
    }
    return DD_OK;
}

int dd_batch_run(dd_batch *b, int32_t T, void *stream) {
    if (!b) return fail(DD_E_ARG, "NULL batch");
    return dd_run(b->h, T, stream);
}

int dd_batch_lower_bounds(dd_batch *b, double *lbs, double *dls, void *stream) {
    if (!b || !lbs) return fail(DD_E_ARG, "NULL argument");
    dd_instance *h = b->h;
    hipStream_t s = (hipStream_t)stream;
    const int k = b->k;
    int st = deferred(h, s);
    if (st) return st;
    if ((st = all_classes(h, false, dd::BWD_EN_BAR, s))) return st;
    st = recorded(h, "k_seg_sum", 4.0 * (double)h->m, s,
                  [&] { return dd::launch_seg_sum(h->T.energies, b->row_seg, k, 0, b->sums, s); });
    if (st) return st;
    if (dls) {
        if (!h->en_lam_valid) {
            if ((st = all_classes(h, false, dd::BWD_EN_LAM, s))) return st;
            h->en_lam_valid = true;
        }
        HIP_TRY(dd::launch_gather(h->canon2slot, h->T.M, h->tmp, h->E, nullptr, s));
        st = recorded(h, "k_seg_sum", 4.0 * (double)h->m, s,
                      [&] { return dd::launch_seg_sum(h->T.en_lam, b->row_seg, k, 0, b->sums + k, s); });
        if (st) return st;
        st = recorded(h, "k_seg_sum", 4.0 * (double)h->E, s,
                      [&] { return dd::launch_seg_sum(h->tmp, b->edge_seg, k, 1, b->sums + 2 * k, s); });
        if (st) return st;
    }
    HIP_TRY(hipMemcpyAsync(b->sums_host, b->sums, sizeof(double) * 3 * k, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    bool finite = true;
    for (int q = 0; q < k; ++q) {
        lbs[q] = b->sums_host[q] + b->unc_const[q];
        finite = finite && std::isfinite(lbs[q]);
        if (dls) {
            dls[q] = b->sums_host[k + q] + b->sums_host[2 * k + q] + b->unc_const[q];
            finite = finite && std::isfinite(dls[q]);
        }
    }
    if (!finite) return fail(DD_E_NONFINITE, "a lower bound is not finite");
    return DD_OK;
}

}  // extern "C"
