// instance.hpp -- host-side state of a device instance and the launch helpers shared by the
// C ABI's translation units.
#pragma once
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/dd.h"
#include "kernels.hpp"

namespace ddi {
// Record a thread-local error message and return code.
int fail(int code, const char *fmt, ...);
}  // namespace ddi

#define HIP_TRY(x)                                                                                            \
    do {                                                                                                      \
        hipError_t e_ = (x);                                                                                  \
        if (e_ != hipSuccess)                                                                                 \
            return ddi::fail(DD_E_HIP, "%s: %s (%s:%d)", #x, hipGetErrorString(e_), __FILE__, __LINE__);      \
    } while (0)

using dd::ClassLaunch;
using dd::DevTables;

struct dd_instance {
    int device = 0;
    int64_t n = 0, m = 0, E = 0, nodes = 0;
    int max_width = 0, max_len = 0, uncovered = 0;
    double unc_const = 0.0;
    int ckpt_default = 5;
    int var_team = 1;  // lanes per variable in the per-variable sums (deferred S and its adjoint)
    static constexpr int kVarTeam = 4;
    int lds_budget = 64 * 1024;  // max LDS bytes per workgroup
    int64_t max_device_bytes = 0;  // cap on the device memory the instance may hold (0: none)
    int lb_every = 1;              // default iterations between the bounds of dd_run_trace
    std::vector<ClassLaunch> classes;
    int64_t ntiles = 0, node_slots = 0, edge_slots = 0, device_bytes = 0;
    int64_t coded_levels = 0, raw_levels = 0;  // one-wave levels with and without byte codes
    std::vector<int32_t> edge_var, edge_row;  // canonical edge map (host)
    std::vector<int64_t> row_nodes;
    // profiling: event pairs recorded around launches while enabled
    struct Rec {
        int kernel;
        hipEvent_t a, b;
    };
    bool prof = false;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    std::vector<Rec> recs;
    std::vector<std::string> kname;
    std::vector<double> kbytes;
    int kernel_id(const std::string &name, double bytes) {
        for (size_t q = 0; q < kname.size(); ++q)
            if (kname[q] == name) return (int)q;
        kname.push_back(name);
        kbytes.push_back(bytes);
        return (int)kname.size() - 1;
    }
    // device buffers
    std::vector<void *> allocs;
    DevTables T{};
    int32_t *var_ptr = nullptr, *var_slots = nullptr, *var_canon = nullptr, *canon2slot = nullptr;
    int32_t *var_perm = nullptr;  // [n] the library's number of each variable (first appearance in slot order)
    float *cdev = nullptr, *S = nullptr, *aS = nullptr, *omega = nullptr, *alpha = nullptr, *tmp = nullptr;
    double *red = nullptr;   // device reduction output [4]
    double *partial = nullptr;  // [kSumBlocks] reduction scratch
    bool en_lam_valid = false;  // T.en_lam holds E^j at the current multipliers
    // T.B / T.F hold the node costs at the current multipliers: what a forward / backward update
    // pass reads (a forward pass leaves F valid and B stale, a backward pass the opposite)
    bool b_valid = false, f_valid = false;
    int64_t fwd_serial = 0;  // serial of the recorded unrolled forward (incremented by every one)
    // reverse mode (buffers allocated on first use)
    bool adj_ready = false;
    float *lam_in = nullptr, *dlamA = nullptr, *dlamB = nullptr, *dMA = nullptr, *dMB = nullptr, *g = nullptr;
    float *dalpha = nullptr, *domega = nullptr, *rec_val = nullptr, *scratch_n = nullptr, *Se = nullptr;
    float *Qs = nullptr;  // per-node arc probabilities of the smoothed sweeps (allocated on first use)
    int32_t *rec_idx = nullptr;
    int32_t *mrec = nullptr;  // argmin records of the last recording update pass (one-wave diagrams)
    float *mdiff = nullptr;
    std::vector<float *> ck_lam, ck_M;    // checkpoints of the unrolled forward (state at iterations 0, K, 2K, ..., T)
    uint64_t *ck_hash = nullptr;          // fingerprint of every checkpoint, taken when it is saved
    size_t ck_hash_cap = 0;
    uint64_t *hash_tmp = nullptr;         // [1] fingerprint of a loaded or recomputed state
    int32_t *ck_flag = nullptr;           // [1] set when a checkpoint or its recomputation does not match
    std::vector<float *> seg_lam, seg_M;  // pass-input states inside one checkpoint segment
    std::vector<float *> fwd_S;           // S of every pass of the checkpointed forward (2T arrays of n),
                                          // which a recomputed segment reproduces bit for bit
    // stored trajectory of the unrolled forward (ckpt_every = -1): the node costs every pass read or
    // wrote and the state before every pass, so the backward sweep recomputes nothing
    std::vector<float *> trF, trB;      // trF[t]: F left by forward pass t; trB[t]: B forward pass t read (t <= T)
    std::vector<float *> tr_lam, tr_M;  // state before pass q = 0 .. 2T (the last one: the final state)
    std::vector<int32_t *> tr_mrec;     // argmin records of pass q = 0 .. 2T-1
    std::vector<float *> tr_mdiff;
    std::vector<float *> tr_Se;         // S per edge slot of pass q's input M (q = 0 .. 2T-1)
    float *F0 = nullptr, *B0 = nullptr; // the instance's own node-cost arrays
    // argmin codes of the node costs (DevTables::Fpar / Bch): the instance's own, paired with F0 / B0,
    // and those of the stored trajectory's arrays (trFp[t] with trF[t], trBc[t] with trB[t])
    uint16_t *Fpar0 = nullptr, *Bch0 = nullptr;
    std::vector<uint16_t *> trFp, trBc;
    bool fwd_stored = false;
    bool fwd_last_stored = false;  // the checkpointed forward ran its last segment into the stored arrays
    int fwd_T = -1, fwd_K = 0;
    bool fwd_from_state = false;  // the recorded forward started from a given state (no reset)
    int64_t version = 0, fwd_version = -1;  // the recorded forward is valid while the state is unchanged
    double *red_host = nullptr;  // pinned
    int32_t *flags = nullptr;

    // side streams (default priority) and fork/join events for concurrent class launches
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;

    // iterations replayed from captured graphs (capture happens on cap_stream; launches go
    // to the caller's stream)
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_one = nullptr, graph_chunk = nullptr;
    bool use_graphs = true;
    // launch sequences of the unrolled forward and backward, replayed from graphs captured the first
    // time their key is seen, with the host-side effects the sequence had when it was captured
    struct SeqGraph {
        std::vector<int64_t> key;
        hipGraphExec_t exec;
        int64_t dversion;
        bool en_lam_valid, b_valid, f_valid;
        float *F, *B, *lam, *M;  // table pointers the sequence leaves
        uint16_t *Fpar, *Bch;
    };
    std::vector<SeqGraph> seq_graphs;
    bool capturing = false;   // a sequence is being captured: allocation is an internal error
    int64_t alloc_epoch = 0;  // counts allocations (a captured sequence keeps the buffers it saw)
    float *seed_dev = nullptr;  // [1] adjoint of the lower bound in the captured backward
    int adj_dense = 0;  // reverse sweeps of one-wave diagrams route node by node (check of that path)
    bool adj_replay = false;  // checkpointed backward: replay passes instead of storing segments

    ~dd_instance() {
        if (graph_one) (void)hipGraphExecDestroy(graph_one);
        if (graph_chunk) (void)hipGraphExecDestroy(graph_chunk);
        for (SeqGraph &g : seq_graphs) (void)hipGraphExecDestroy(g.exec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (hipEvent_t e : join) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        for (hipStream_t q : side) (void)hipStreamDestroy(q);
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        for (void *p : allocs) (void)hipFree(p);
        if (red_host) (void)hipHostFree(red_host);
    }
    template <class T_>
    int alloc(T_ **p, size_t count) {
        void *q = nullptr;
        size_t bytes = std::max<size_t>(count, 1) * sizeof(T_);
        if (capturing) return ddi::fail(DD_E_HIP, "internal: device allocation inside a captured launch sequence");
        if (max_device_bytes > 0 && device_bytes + (int64_t)bytes > max_device_bytes)
            return ddi::fail(DD_E_OOM,
                             "allocating %zu bytes would exceed the instance's device-memory cap "
                             "(%lld of %lld bytes held)",
                             bytes, (long long)device_bytes, (long long)max_device_bytes);
        hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess) return ddi::fail(DD_E_OOM, "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
        allocs.push_back(q);
        device_bytes += (int64_t)bytes;
        ++alloc_epoch;
        *p = (T_ *)q;
        return DD_OK;
    }
};

namespace ddi {

// Launch through `launch` (returns hipError_t); while profiling, bracket it with events on s.
template <class F>
inline int recorded(dd_instance *h, const char *name, double bytes, hipStream_t s, F launch) {
    hipEvent_t a = nullptr, b = nullptr;
    const bool rec = h->prof && h->pool_used + 2 <= h->pool.size();
    if (rec) {
        a = h->pool[h->pool_used++];
        b = h->pool[h->pool_used++];
        HIP_TRY(hipEventRecord(a, s));
    }
    hipError_t e = launch();
    if (e != hipSuccess) return fail(DD_E_HIP, "%s launch: %s", name, hipGetErrorString(e));
    if (rec) {
        HIP_TRY(hipEventRecord(b, s));
        h->recs.push_back({h->kernel_id(name, bytes), a, b});
    }
    return DD_OK;
}

// S and alpha*S of the current M (start of a pass), or of a given M (slot order); with Se, S per
// edge slot too.
int deferred(dd_instance *h, hipStream_t s);
int deferred_from(dd_instance *h, const float *M, hipStream_t s, float *Se = nullptr);
// One sweep (pass-kernel mode) over every class, classes concurrently on side streams.
int all_classes(dd_instance *h, bool fwd, int mode, hipStream_t s);
// B at the current multipliers, stored (what a forward pass reads).
int recompute_B(dd_instance *h, hipStream_t s);
// The launches of one pass (deferred sums, then the update sweep of every class); host flags untouched.
int pass_launches(dd_instance *h, int dir, hipStream_t s);
// The smoothed-subproblem sweeps of every class (arc probabilities into Qs, a node array of at least
// node_slots + 64 floats whose prior contents are never read), E_out / p_out as dd_smoothed.
int smoothed_sweeps(dd_instance *h, float *Qs, float tau, int flushed, float *E_out, float *p_out, hipStream_t s);
// dd_create with a locality group per row (row_group[j] for row j, or nullptr): within a kernel
// class the rows of one group get consecutive tiles, so their edge slots form one stretch.
int create_grouped(const dd_problem *prob, const dd_options *opt, void *stream, const int32_t *row_group,
                   dd_instance **out);
// Forget captured iteration and sequence graphs (after a change of launch shapes).
void drop_graphs(dd_instance *h);

}  // namespace ddi
