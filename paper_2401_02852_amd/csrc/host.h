// Host-side internals of libqnae.so shared by the ABI translation units:
// the context, error reporting, growable buffers, kernel timing, mixer forms
// and phase tables, and the sweep planner.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <complex>
#include <condition_variable>
#include <exception>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/qnae.h"
#include "internal.h"

namespace qnae_host {

// Sets the calling thread's error message and returns `code`.
int fail(int code, const char* fmt, ...);
const char* last_error();
// Inside a catch block: records the exception being handled as this thread's
// last error and returns QNAE_ENOMEM (host memory or threads ran out; nothing
// else throws here). Entry points end in it so that no exception leaves the
// C ABI.
int host_exception();

#define HIP_TRY(expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return ::qnae_host::fail(e_ == hipErrorOutOfMemory ? QNAE_ENOMEM : QNAE_EHIP, "%s: %s (%s:%d)", \
                                     #expr, hipGetErrorString(e_), __FILE__, __LINE__);                \
    } while (0)

// Device buffer that only grows (waits for the device before it reallocates).
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipError_t reserve(size_t need);
    void release();
};

// Pinned host buffer that only grows.
struct HostBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipError_t reserve(size_t need);
    void release();
};

// Event-timed kernel tallies (qnae_profile_*).
enum { K_COST, K_FIRST, K_MIDDLE, K_BOUNDARY, K_FINAL, K_RESIDENT, K_REDUCE, K_BATCH_COST, K_BATCH_RESIDENT,
       K_BATCH_SWEEP, K_BATCH_REDUCE, K_ADJOINT, K_KINDS };

struct Profiler {
    struct Rec {
        int kind;
        double bytes;
        hipEvent_t start, stop;
    };
    static const char* name(int k);
    bool on = false;
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    uint64_t launches[K_KINDS] = {};
    double ms[K_KINDS] = {}, bytes[K_KINDS] = {};
    hipEvent_t get();
};

constexpr int kResidentMaxN = 14;

// Bump allocator for a pinned host blob mirrored by a device buffer.
struct Blob {
    size_t size = 0;
    size_t take(size_t bytes, size_t align = 256) {
        size = (size + align - 1) / align * align;
        const size_t at = size;
        size += bytes;
        return at;
    }
};

}  // namespace qnae_host

namespace qnae_host {

// A few host threads kept for the context's lifetime. run(count, fn) calls
// fn(i) for every i in [0, count) on the workers and the calling thread and
// returns when all calls are done; one run at a time (the context is used by
// one thread at a time).
class WorkerPool {
public:
    explicit WorkerPool(int workers);
    ~WorkerPool();
    WorkerPool(const WorkerPool&) = delete;
    WorkerPool& operator=(const WorkerPool&) = delete;
    // fn(0) .. fn(count - 1) over the workers and the caller. If a call
    // throws, the items not yet started are skipped and the first exception
    // is rethrown to the caller once every worker is idle again.
    void run(int count, const std::function<void(int)>& fn);
    int size() const { return (int)threads_.size() + 1; }

private:
    void work();
    void drain();
    std::vector<std::thread> threads_;
    std::mutex mu_;
    std::condition_variable wake_, done_;
    const std::function<void(int)>* fn_ = nullptr;
    int count_ = 0;
    std::atomic<int> next_{0};
    std::exception_ptr error_;  // first exception of the current run
    int busy_ = 0;
    uint64_t generation_ = 0;
    bool stop_ = false;
};

// The plan of a batch shape (batch.cpp).
struct BatchPlan;
void free_batch_plan(BatchPlan* p);
struct BatchPlanFree {
    void operator()(BatchPlan* p) const { free_batch_plan(p); }
};

}  // namespace qnae_host

struct qnae_ctx {
    int device = 0;
    qnae_host::Profiler prof;
    // single-instance path
    qnae_host::DevBuf state, partials, luts, clauses, forms, small;  // small: zeros counter + 3 result doubles
    qnae_host::HostBuf h_luts, h_clauses, h_forms, h_small;
    // batched path: uploaded tables and work lists, states, partial sums, results
    qnae_host::DevBuf b_blob, b_states, b_partials, b_results;
    // gradient: checkpoints + adjoint state, tables, partial sums
    qnae_host::DevBuf g_states, g_blob, g_partials;
    qnae_host::HostBuf h_blob, h_results;
    hipEvent_t staging_done = nullptr;  // last async copy out of pinned staging
    // plans of recent batch shapes, with their captured launch sequences (most recent last)
    bool use_graphs = true;
    hipStream_t capture_stream = nullptr;
    std::vector<std::unique_ptr<qnae_host::BatchPlan, qnae_host::BatchPlanFree>> batch_plans;
    // batched cost builds: their own staging, so a run's host work can overlap their kernels
    qnae_host::DevBuf c_blob;
    qnae_host::HostBuf h_cblob;
    hipEvent_t cost_staging_done = nullptr;
    // sweep tile shapes chosen per (n, cost type), by qnae_autotune or qnae_set_tune
    std::map<std::pair<int, int>, qnae_tune> tunes;
    qnae_host::DevBuf tune_cost;
    // sampling: tile masses and prefix sums, uniforms and outcomes
    qnae_host::DevBuf s_dev;
    qnae_host::HostBuf h_sample;
    int tile_bits = 13;                 // tile size of the plain sweeps (log2 amplitudes)
    int min_low_run = 4;                // minimum contiguous low run (log2 amplitudes)
    int page_bit = 18;                  // first index bit above a 2 MiB page of amplitudes
    // host threads for per-instance planning of large batches (made on first use)
    std::unique_ptr<qnae_host::WorkerPool> pool;
    // qnae_qaoa_run_noalloc: the device's static scratch array (its address
    // from hipGetSymbolAddress) and fixed pinned staging, both set up by
    // qnae_create
    void* na_dev = nullptr;
    qnae_host::HostBuf na_host;
};

namespace qnae_host {

// Makes the context's device current and waits until pinned staging is free.
int enter(qnae_ctx* ctx);
// With the context's device current: looks up that device's static scratch
// array of qnae_qaoa_run_noalloc (once per device) and reserves the
// context's fixed pinned staging for it.
int noalloc_setup(qnae_ctx* ctx);
// fn(i) for i in [0, count), spread over the context's host threads when the
// work is large enough to pay for the hand-off (`items` units of it).
void parallel_for(qnae_ctx* ctx, int count, size_t items, const std::function<void(int)>& fn);
int check_cost_args(int32_t n, int32_t m, int32_t dtype);
// QNAE_EINVAL unless ptr (a device buffer the kernels access with 16-byte
// loads and stores; NULL passes) is 16-byte aligned.
int check_aligned(const void* ptr, const char* what);
// Sweep tile shape at (n, cost type): the tuned one if set, else the context defaults.
qnae_tune tune_for(const qnae_ctx* ctx, int n, int dtype);

int check_run_args(int32_t n, int32_t m, int32_t dtype, const void* cost, const double* gammas, const double* betas,
                   int32_t p);

// Launch through `fn`, bracketed by profiling events when enabled.
template <typename F>
hipError_t timed(qnae_ctx* ctx, int kind, double bytes, hipStream_t s, F&& fn) {
    Profiler& P = ctx->prof;
    if (!P.on) return fn();
    Profiler::Rec r{kind, bytes, P.get(), P.get()};
    hipError_t e = hipEventRecord(r.start, s);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(r.stop, s);
    P.pending.push_back(r);
    return e;
}

// Clause records for the cost kernel (drops clauses that can never be
// violated); returns the number written to `out` (room for m records), those
// with a variable below 5 first (*num_low, when given, of them).
int make_clause_records(const int32_t* clauses, int32_t m, int32_t k, qnae::ClauseRec* out,
                        int predicate = QNAE_PRED_NAE, int* num_low = nullptr);
// QNAE_EINVAL if some literal is 0 or outside +-[1, n].
int check_literals(const int32_t* clauses, int32_t m, int32_t n, int32_t k);

// One layer's mixer exp(-i beta X) on each of n qubits as device butterflies
// (I - i t X) per qubit, |t| <= 1, followed by X on every qubit when
// form.flip, times the scalar `scale` (cos(beta)^n, or (-i sin(beta))^n with
// the flip).
struct Layer {
    qnae::MixForm form;
    std::complex<double> scale;
};
Layer mixer_form(double beta, int n);

// scale * exp(sign i g c) for c = 0..m (sign -1 or +1) as m + 1 FP32 pairs.
void phase_row(double g, int m, std::complex<double> scale, int sign, float2* out);
// Phase tables (p tables of m + 1 entries, or one when p = 0) and per-layer
// mixer forms; returns the scalar factor left after the last layer.
std::complex<double> build_tables(int n, int m, const double* gammas, const double* betas, int p, float2* tables,
                                  qnae::MixForm* forms);
// The same with the first table scaled by `first` instead of 2^{-n/2} (a run
// that starts from a given, normalised state uses 1).
std::complex<double> build_tables_from(int n, int m, const double* gammas, const double* betas, int p,
                                       float2* tables, qnae::MixForm* forms, std::complex<double> first);

struct Group {
    std::vector<int> pos;  // global bit of each tile bit
    uint32_t mask;         // tile bits this group mixes
};

struct Op {
    int group;
    int kind;                              // qnae::SweepKind
    int pre_layer, post_layer, lut_layer;  // -1 when unused
};

// The groups in fixed storage (at most kMaxGroups: n <= 34 with tiles of at
// least 12 bits needs 4). make_group_specs allocates nothing; make_groups is
// the same as vectors.
constexpr int kMaxGroups = 8;
struct GroupSpec {
    uint8_t pos[16];  // global bit of each tile bit (TB entries)
    uint32_t mask;    // tile bits this group mixes
};
int make_group_specs(int n, int TB, int cmin, int page, int split, GroupSpec* out);
std::vector<Group> make_groups(int n, int TB, int cmin, int page, int split = 0);

// The sweeps of a depth-p solve over `ngroups` qubit groups, in order, handed
// to fn(const Op&) one at a time (allocates nothing). Each layer mixes every
// group once. The last group of a layer is fused with the next layer's phase
// and with that layer's mixing of the same group, so every layer after the
// first costs (number of groups - 1) sweeps. The first sweep starts from the
// phase table (no load), or with from_state loads a given state and applies
// phase 0 and the mixing of group 0; the last one only reads the state for
// the readout unless the final state is kept.
template <typename F>
void for_each_op(int ngroups, int p, bool from_state, F&& fn) {
    using namespace qnae;
    if (p == 0) {
        fn(Op{0, SK_P0, -1, -1, 0});
        return;
    }
    fn(from_state ? Op{0, SK_BOUNDARY, -1, 0, 0} : Op{0, SK_FIRST, -1, 0, 0});
    // groups not yet mixed for layer l, as a bit set (ascending order)
    uint32_t pending = ((1u << ngroups) - 1u) & ~1u;
    for (int l = 0;; ++l) {
        if (pending == 0u) {  // one group: the previous sweep mixed it already
            if (l == p - 1) {
                fn(Op{0, SK_FINAL, -1, -1, -1});
                return;
            }
            fn(Op{0, SK_BOUNDARY, -1, l + 1, l + 1});
            continue;
        }
        const int last = 31 - __builtin_clz(pending);  // carries the phase of layer l + 1
        for (uint32_t m = pending & ~(1u << last); m != 0u; m &= m - 1u)
            fn(Op{__builtin_ctz(m), SK_MIDDLE, l, -1, -1});
        if (l == p - 1) {
            fn(Op{last, SK_FINAL, l, -1, -1});
            return;
        }
        fn(Op{last, SK_BOUNDARY, l, l + 1, l + 1});
        pending = ((1u << ngroups) - 1u) & ~(1u << last);
    }
}
// from_state: the first sweep loads a given state instead of starting from |+>.
std::vector<Op> make_plan(int ngroups, int p, bool from_state = false);

// A tiled (n > kResidentMaxN) solve: groups, op sequence and per-layer data.
struct SweepPlan {
    int n = 0, m = 0, p = 0, TB = 13, dtype = QNAE_U8, lut_len = 1;
    bool keep = false;
    bool half = false;  // state and cost over x < 2^(n-1) (NAE global-flip symmetry)
    std::vector<Group> groups;
    std::vector<Op> ops;
    std::vector<qnae::MixForm> forms;
    std::vector<int> flips_before;  // parity of cot-form layers among 0 .. l-1
    std::complex<double> final_scale;
};

// Plans a tiled solve; `forms` are the per-layer mixer forms from build_tables.
void plan_sweeps(SweepPlan& P, int n, int m, int p, int dtype, int TB, int cmin, int page, int split, bool keep,
                 const qnae::MixForm* forms, std::complex<double> final_scale, bool from_state = false);

// Reverse pass of a gradient over L layers ("b-layers", the last forward
// layer first): each b-layer inverts the mixer of every group, then the phase.
struct AdjOp {
    int group;
    int kind;                                  // qnae::AdjointKind
    int pre_layer, phase_layer, post_layer;    // b-layer indices, -1 when unused
};
std::vector<AdjOp> make_adjoint_plan(int ngroups, int L);
// Kernel arguments of one op.
void sweep_args(const SweepPlan& P, const Op& op, float2* psi, const void* cost, const float2* luts, double* partials,
                qnae::SweepArgs* a);
// The same from the plan's scalars and arrays (forms: p entries,
// flips_before: p + 1) and the op's group (TB bit positions and mix mask).
struct PlanRef {
    int n, p, TB, lut_len;
    bool keep, half;
    const qnae::MixForm* forms;
    const int* flips_before;
    std::complex<double> final_scale;
};
void sweep_args_for(const PlanRef& P, const int* pos, uint32_t mask, const Op& op, float2* psi, const void* cost,
                    const float2* luts, double* partials, qnae::SweepArgs* a);
// Only the fields that depend on the angles (butterfly parameters, the
// final scalar factor, complemented cost reads): arguments of a plan whose
// angles changed.
void sweep_args_angles(const PlanRef& P, const Op& op, qnae::SweepArgs* a);
void sweep_args_angles(const SweepPlan& P, const Op& op, qnae::SweepArgs* a);
// Algorithmic bytes of one op and its profiling kind.
double op_bytes(const SweepPlan& P, const Op& op);
int op_profile_kind(const Op& op);

}  // namespace qnae_host
