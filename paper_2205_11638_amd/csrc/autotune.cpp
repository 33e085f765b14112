// autotune.cpp -- launch shapes of the pass kernels: query, set, and a timing autotuner with a
// text cache.
//
// A pass kernel's arithmetic does not depend on its launch shape (each wave owns whole tiles),
// so shapes trade only speed: waves per workgroup (at most 4: the kernels are compiled for 256 threads) set how many tiles share a CU's LDS
// allocation granule, and a resident grid (as many workgroups as the CUs hold at once, whose
// waves walk the tile list) replaces one wave per tile.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/dd.h"
#include "instance.hpp"
#include "kernels.hpp"

using namespace ddi;

namespace {

bool shape_ok(const dd_instance *h, const ClassLaunch &c, int wpb) {
    if (wpb < 1 || wpb > dd::kMaxWavesPerBlock) return false;
    return (int64_t)wpb * dd::lds_words_pass_c(c.P, c.RMAX, c.WB, c.NL) * 4 <= h->lds_budget;
}

std::string signature(const dd_instance *h) {
    hipDeviceProp_t prop;
    std::ostringstream o;
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) o << prop.gcnArchName;
    for (const ClassLaunch &c : h->classes) o << "|" << c.P << "," << c.RMAX << "," << c.ntiles << "," << c.nodes;
    return o.str();
}

std::string shapes_text(const dd_instance *h) {
    std::ostringstream o;
    for (size_t i = 0; i < h->classes.size(); ++i) {
        const ClassLaunch &c = h->classes[i];
        o << (i ? ";" : "") << c.wpb_f << "," << c.wpb_b << "," << c.grid_f << "," << c.grid_b;
    }
    return o.str();
}

// Parse "wf,wb,gf,gb;..." for every class; false if it does not fit the instance.
bool parse_shapes(dd_instance *h, const std::string &txt, std::vector<ClassLaunch> &out) {
    out = h->classes;
    std::istringstream in(txt);
    std::string item;
    size_t i = 0;
    while (std::getline(in, item, ';')) {
        if (i >= out.size()) return false;
        int wf, wb, gf, gb;
        if (sscanf(item.c_str(), "%d,%d,%d,%d", &wf, &wb, &gf, &gb) != 4) return false;
        if (!shape_ok(h, out[i], wf) || !shape_ok(h, out[i], wb) || gf < 0 || gb < 0) return false;
        out[i].wpb_f = wf;
        out[i].wpb_b = wb;
        out[i].grid_f = gf;
        out[i].grid_b = gb;
        ++i;
    }
    return i == out.size();
}

// Mean duration (ms) of `reps` launches of class c's update kernel in the given shape.
int time_shape(dd_instance *h, const ClassLaunch &c, bool fwd, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
               float *ms) {
    auto launch = [&] {
        return fwd ? dd::launch_fwd(h->T, c, dd::FWD_UPDATE, s) : dd::launch_bwd(h->T, c, dd::BWD_UPDATE, s);
    };
    HIP_TRY(launch());  // warm-up
    HIP_TRY(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) HIP_TRY(launch());
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    *ms = t / (float)reps;
    return DD_OK;
}

}  // namespace

extern "C" {

int dd_get_launch(const dd_instance *h, int32_t *out, int32_t cap, int32_t *count) {
    if (!h || !count || (cap > 0 && !out)) return fail(DD_E_ARG, "NULL argument");
    *count = (int32_t)h->classes.size();
    for (int i = 0; i < (int)h->classes.size() && i < cap; ++i) {
        const ClassLaunch &c = h->classes[i];
        const int32_t v[6] = {c.P, c.RMAX, c.wpb_f, c.wpb_b, c.grid_f, c.grid_b};
        std::memcpy(out + 6 * i, v, sizeof v);
    }
    return DD_OK;
}

int dd_set_launch(dd_instance *h, int32_t c, int32_t wpb_f, int32_t wpb_b, int32_t grid_f, int32_t grid_b) {
    if (!h || c < 0 || c >= (int)h->classes.size()) return fail(DD_E_ARG, "bad instance or class index");
    ClassLaunch &cl = h->classes[c];
    if (!shape_ok(h, cl, wpb_f) || !shape_ok(h, cl, wpb_b) || grid_f < 0 || grid_b < 0)
        return fail(DD_E_ARG, "class %d: waves per workgroup must be 1..%d within the LDS budget, grids >= 0", c,
                    dd::kMaxWavesPerBlock);
    cl.wpb_f = wpb_f;
    cl.wpb_b = wpb_b;
    cl.grid_f = grid_f;
    cl.grid_b = grid_b;
    drop_graphs(h);
    return DD_OK;
}

int dd_autotune(dd_instance *h, const char *cache_path, int32_t *from_cache, void *stream) {
    if (!h) return fail(DD_E_ARG, "NULL instance");
    if (from_cache) *from_cache = 0;
    const std::string sig = signature(h);
    if (cache_path) {
        std::ifstream f(cache_path);
        std::string line;
        while (std::getline(f, line)) {
            const size_t tab = line.find('\t');
            if (tab == std::string::npos || line.compare(0, tab, sig) != 0 || tab != sig.size()) continue;
            std::vector<ClassLaunch> cl;
            if (!parse_shapes(h, line.substr(tab + 1), cl)) continue;
            h->classes = cl;
            drop_graphs(h);
            if (from_cache) *from_cache = 1;
            return DD_OK;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
    // keep the state: the timed launches are real update passes
    float *lam0 = nullptr, *M0 = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const size_t bytes = sizeof(float) * (size_t)std::max<int64_t>(h->edge_slots, 1);
    auto release = [&] {
        if (lam0) (void)hipFree(lam0);
        if (M0) (void)hipFree(M0);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    auto run = [&]() -> int {
        HIP_TRY(hipMalloc((void **)&lam0, bytes));
        HIP_TRY(hipMalloc((void **)&M0, bytes));
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        HIP_TRY(hipMemcpyAsync(lam0, h->T.lam, bytes, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(M0, h->T.M, bytes, hipMemcpyDeviceToDevice, s));
        int st = deferred(h, s);
        if (st) return st;
        for (ClassLaunch &c : h->classes) {
            for (int fwd = 1; fwd >= 0; --fwd) {
                int best_w = fwd ? c.wpb_f : c.wpb_b, best_g = fwd ? c.grid_f : c.grid_b;
                float best = INFINITY;
                int reps = 0;
                for (int w = 1; w <= dd::kMaxWavesPerBlock; w *= 2) {
                    if (!shape_ok(h, c, w)) break;
                    ClassLaunch t = c;
                    t.wpb_f = t.wpb_b = w;
                    t.grid_f = t.grid_b = 0;
                    const int per_cu = dd::pass_blocks_per_cu(t, fwd != 0);
                    const int64_t full = (c.ntiles + w - 1) / w;
                    for (int resident = 0; resident < 2; ++resident) {
                        int g = 0;
                        if (resident) {
                            if (per_cu <= 0 || (int64_t)per_cu * cus >= full) continue;  // would be one wave per tile
                            g = per_cu * cus;
                        }
                        t.grid_f = t.grid_b = g;
                        if (!reps) {  // repetitions for about 3 ms of timed work per shape
                            float one = 0.f;
                            if ((st = time_shape(h, t, fwd != 0, 1, s, e0, e1, &one))) return st;
                            reps = (int)std::min(20.f, std::max(2.f, 3.f / std::max(one, 1e-3f)));
                        }
                        float ms = 0.f;
                        if ((st = time_shape(h, t, fwd != 0, reps, s, e0, e1, &ms))) return st;
                        if (ms < best) {
                            best = ms;
                            best_w = w;
                            best_g = g;
                        }
                    }
                }
                if (fwd) {
                    c.wpb_f = best_w;
                    c.grid_f = best_g;
                } else {
                    c.wpb_b = best_w;
                    c.grid_b = best_g;
                }
            }
        }
        HIP_TRY(hipMemcpyAsync(h->T.lam, lam0, bytes, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(h->T.M, M0, bytes, hipMemcpyDeviceToDevice, s));
        h->version++;
        h->f_valid = false;  // the timed passes left F at other multipliers
        if ((st = recompute_B(h, s))) return st;
        HIP_TRY(hipStreamSynchronize(s));
        return DD_OK;
    };
    const int st = run();
    release();
    if (st) return st;
    drop_graphs(h);
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        if (!f) return fail(DD_E_ARG, "cannot append to %s", cache_path);
        f << sig << '\t' << shapes_text(h) << '\n';
    }
    return DD_OK;
}

}  // extern "C"
