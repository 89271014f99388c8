// Sweep tile-shape autotuning (include/qnae.h, qnae_autotune / qnae_set_tune /
// qnae_get_tune). A candidate is timed on two- and four-layer runs of the
// real sweep kernels over scratch memory: the cost diagonal of a fixed
// random 3-NAE-SAT instance with 63 clauses (so the phase-table reads spread
// over the table as in real runs; an all-zero diagonal makes every read the
// same entry), phase tables of 64 entries, angles away from the special
// values, so every sweep kind of a p >= 2 plan runs (first, middle,
// boundary, final).
#include <algorithm>
#include <chrono>
#include <string>
#include <vector>
#include <cmath>

#include "host.h"

using namespace qnae_host;
using qnae::MixForm;
using qnae::SweepArgs;

namespace qnae_host {

qnae_tune tune_for(const qnae_ctx* ctx, int n, int dtype) {
    auto it = ctx->tunes.find({n, dtype});
    if (it != ctx->tunes.end()) return it->second;
    return qnae_tune{ctx->tile_bits, ctx->min_low_run, ctx->page_bit, 0, 0.0};
}

}  // namespace qnae_host

namespace {

int check_shape(const qnae_tune& t) {
    if (t.tile_bits < 12 || t.tile_bits > 14) return fail(QNAE_EINVAL, "tile_bits=%d outside [12, 14]", t.tile_bits);
    if (t.low_run_bits < 4 || t.low_run_bits > 6)
        return fail(QNAE_EINVAL, "low_run_bits=%d outside [4, 6]", t.low_run_bits);
    if (t.page_bit < 4 || t.page_bit > 64) return fail(QNAE_EINVAL, "page_bit=%d outside [4, 64]", t.page_bit);
    if (t.split < 0 || t.split > 3) return fail(QNAE_EINVAL, "split=%d outside [0, 3]", t.split);
    return QNAE_OK;
}

// Do the groups of this shape at n have a third one (where split applies)?
bool has_split(int n, const qnae_tune& t) {
    GroupSpec spec[kMaxGroups];
    return make_group_specs(n, t.tile_bits, t.low_run_bits, t.page_bit, 0, spec) == 3;
}

// The fixed tuning instance: m clauses of 3 distinct variables below n with
// random signs, from a splitmix64 stream with a fixed seed (n >= 3).
std::vector<int32_t> tuning_clauses(int n, int m) {
    uint64_t state = 0x9e3779b97f4a7c15ull;
    auto next = [&state]() {
        uint64_t z = (state += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    };
    std::vector<int32_t> lits;
    lits.reserve((size_t)3 * m);
    for (int c = 0; c < m; ++c) {
        int v[3];
        for (int i = 0; i < 3; ++i) {
            bool fresh;
            do {
                v[i] = (int)(next() % (uint64_t)n);
                fresh = true;
                for (int j = 0; j < i; ++j) fresh = fresh && v[j] != v[i];
            } while (!fresh);
            lits.push_back((next() & 1u) ? -(v[i] + 1) : v[i] + 1);
        }
    }
    return lits;
}

int check_tune_target(int32_t n, int32_t dtype, int32_t lo) {
    if (n < lo || n > QNAE_MAX_N) return fail(QNAE_EINVAL, "n=%d outside [%d, %d]", n, lo, QNAE_MAX_N);
    if (dtype != QNAE_U8 && dtype != QNAE_U16) return fail(QNAE_EINVAL, "cost_dtype=%d is not QNAE_U8/QNAE_U16", dtype);
    return QNAE_OK;
}

}  // namespace

extern "C" {

int qnae_autotune(qnae_ctx* ctx, int32_t n, int32_t cost_dtype, int32_t reps, qnae_tune* out, void* stream) try {
    if (int rc = check_tune_target(n, cost_dtype, 1)) return rc;
    if (reps < 1 || reps > 1000) return fail(QNAE_EINVAL, "reps=%d outside [1, 1000]", reps);
    if (!out) return fail(QNAE_EINVAL, "null output pointer");
    if (int rc = enter(ctx)) return rc;
    *out = qnae_tune{0, 0, 0, 0, 0.0};
    if (n <= kResidentMaxN) return QNAE_OK;
    hipStream_t s = (hipStream_t)stream;
    // Two- and four-layer runs; a shape is ranked by its time per layer of a
    // ten-layer run, extrapolated linearly in the layer count (a two-layer
    // run alone gives its first and last sweeps two of five sweeps instead
    // of two of 21, and ranked 14-bit tiles first at n = 28 and 30, where a
    // ten-layer run on them was 2-5% slower).
    const int p = 4, p_lo = 2, m = 63, lut_len = m + 1;
    const double gammas[p] = {0.4, 0.7, 0.5, 0.3}, betas[p] = {0.3, 0.2, 0.25, 0.15};
    HIP_TRY(ctx->h_luts.reserve(sizeof(float2) * p * lut_len));
    HIP_TRY(ctx->h_forms.reserve(sizeof(MixForm) * p));
    float2* tables = (float2*)ctx->h_luts.ptr;
    MixForm* forms = (MixForm*)ctx->h_forms.ptr;
    const std::complex<double> final_scale = build_tables(n, m, gammas, betas, p, tables, forms);
    HIP_TRY(ctx->luts.reserve(sizeof(float2) * p * lut_len));
    HIP_TRY(hipMemcpyAsync(ctx->luts.ptr, tables, sizeof(float2) * p * lut_len, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx->state.reserve(sizeof(float2) << n));
    const size_t cbytes = (size_t)(cost_dtype == QNAE_U8 ? 1 : 2) << n;
    HIP_TRY(ctx->tune_cost.reserve(cbytes));
    {
        const std::vector<int32_t> lits = tuning_clauses(n, m);
        if (int rc = qnae_build_cost_diagonal(ctx, lits.data(), m, n, 3, ctx->tune_cost.ptr, cost_dtype, nullptr,
                                              stream))
            return rc;
    }
    HIP_TRY(ctx->partials.reserve(sizeof(double) * 3 * ((size_t)1 << (n - 12))));
    HIP_TRY(hipEventRecord(ctx->staging_done, s));
    hipEvent_t ev[2] = {nullptr, nullptr};
    HIP_TRY(hipEventCreate(&ev[0]));
    if (hipError_t e = hipEventCreate(&ev[1])) {
        (void)hipEventDestroy(ev[0]);
        return fail(QNAE_EHIP, "hipEventCreate: %s", hipGetErrorString(e));
    }
    auto run = [&](const SweepPlan& P, int TB) -> hipError_t {
        for (const Op& op : P.ops) {
            SweepArgs a;
            sweep_args(P, op, (float2*)ctx->state.ptr, ctx->tune_cost.ptr, (const float2*)ctx->luts.ptr,
                       (double*)ctx->partials.ptr, &a);
            if (hipError_t e = qnae::launch_sweep(TB, cost_dtype, op.kind, a, s)) return e;
        }
        return hipSuccess;
    };
    qnae_tune best{0, 0, 0, 0, 1e300};
    hipError_t err = hipSuccess;
    // Mean time of one run of a plan of `layers` layers under shape t.
    auto time_plan = [&](const qnae_tune& t, int layers, double* ms_out) -> hipError_t {
        SweepPlan P;
        plan_sweeps(P, n, m, layers, cost_dtype, t.tile_bits, t.low_run_bits, t.page_bit, t.split, false, forms,
                    final_scale);
        hipError_t e = run(P, t.tile_bits);  // warm-up
        if (e || (e = hipEventRecord(ev[0], s))) return e;
        for (int r = 0; r < reps && !e; ++r) e = run(P, t.tile_bits);
        if (e || (e = hipEventRecord(ev[1], s)) || (e = hipEventSynchronize(ev[1]))) return e;
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, ev[0], ev[1]))) return e;
        *ms_out = ms / reps;
        return hipSuccess;
    };
    qnae_tune best_of[3] = {best, best, best};  // fastest split-0 shape per tile size
    auto time_shape = [&](const qnae_tune& t) {
        double t_lo = 0.0, t_hi = 0.0;
        if ((err = time_plan(t, p_lo, &t_lo)) || (err = time_plan(t, p, &t_hi))) return;
        // (timing noise on a tiny state could make the four-layer run look no
        // slower than the two-layer one: then its own time per layer is used)
        const double ten = t_hi > t_lo ? t_lo + (10.0 - p_lo) * (t_hi - t_lo) / (p - p_lo) : t_hi * 10.0 / p;
        const qnae_tune timed{t.tile_bits, t.low_run_bits, t.page_bit, t.split, ten / 10.0};
        if (timed.ms_per_layer < best.ms_per_layer) best = timed;
        qnae_tune& b = best_of[t.tile_bits - 12];
        if (t.split == 0 && timed.ms_per_layer < b.ms_per_layer) b = timed;
    };
    for (int TB = 12; TB <= 14 && !err; ++TB)
        for (int low = 4; low <= 5 && !err; ++low)
            for (int page : {18, 64})
                if (!err) time_shape(qnae_tune{TB, low, page, 0, 0.0});
    // The splits of the fastest shape of every tile size: a split can
    // reorder the tile sizes (at n = 30, 14-bit tiles led 13-bit ones
    // without splits, and 13-bit tiles with split 1 were fastest overall).
    for (const qnae_tune& base : best_of)
        if (!err && base.tile_bits != 0 && has_split(n, base))
            for (int split = 1; split <= 3 && !err; ++split)
                time_shape(qnae_tune{base.tile_bits, base.low_run_bits, base.page_bit, split, 0.0});
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (err) return fail(QNAE_EHIP, "autotune: %s", hipGetErrorString(err));
    ctx->tunes[{n, cost_dtype}] = best;
    *out = best;
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

int qnae_set_tune(qnae_ctx* ctx, int32_t n, int32_t cost_dtype, const qnae_tune* tune) try {
    if (!ctx) return fail(QNAE_EINVAL, "null context");
    if (int rc = check_tune_target(n, cost_dtype, kResidentMaxN + 1)) return rc;
    if (!tune) {
        ctx->tunes.erase({n, cost_dtype});
        return QNAE_OK;
    }
    if (int rc = check_shape(*tune)) return rc;
    ctx->tunes[{n, cost_dtype}] =
        qnae_tune{tune->tile_bits, tune->low_run_bits, tune->page_bit, tune->split, tune->ms_per_layer};
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

int qnae_autotune_batched(qnae_ctx* ctx, const qnae_instance* inst, int32_t count, int32_t reps, qnae_tune* out,
                          void* stream) try {
    if (reps < 1 || reps > 100) return fail(QNAE_EINVAL, "reps=%d outside [1, 100]", reps);
    if (!out) return fail(QNAE_EINVAL, "null output pointer");
    if (count < 0 || (count > 0 && !inst)) return fail(QNAE_EINVAL, "bad instance array (count=%d)", count);
    if (!ctx) return fail(QNAE_EINVAL, "null context");
    *out = qnae_tune{0, 0, 0, 0, 0.0};
    // the (n, cost type) classes the shape applies to: instances on the sweep path
    std::vector<std::pair<int, int>> classes;
    int layers = 0;
    for (int i = 0; i < count; ++i) {
        layers += inst[i].p;
        if (inst[i].n <= kResidentMaxN) continue;
        const std::pair<int, int> c{inst[i].n, inst[i].cost_dtype};
        if (std::find(classes.begin(), classes.end(), c) == classes.end()) classes.push_back(c);
    }
    if (classes.empty()) return QNAE_OK;
    std::vector<qnae_result> res((size_t)count);
    const auto saved = ctx->tunes;
    qnae_tune best{0, 0, 0, 0, 1e300};
    qnae_tune best_of[3] = {best, best, best};  // fastest split-0 shape per tile size
    auto time_shape = [&](const qnae_tune& shape) -> int {
        for (const auto& c : classes) ctx->tunes[c] = shape;
        // one warm-up run plans the shape and captures its launches
        int rc = qnae_qaoa_run_batched(ctx, inst, count, res.data(), stream);
        const auto t0 = std::chrono::steady_clock::now();
        for (int r = 0; r < reps && !rc; ++r) rc = qnae_qaoa_run_batched(ctx, inst, count, res.data(), stream);
        if (rc) {
            const std::string msg = last_error();
            ctx->tunes = saved;
            return fail(rc, "autotune_batched: %s", msg.c_str());
        }
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / reps;
        const double per_layer = ms / std::max(layers, 1);
        const qnae_tune timed{shape.tile_bits, shape.low_run_bits, shape.page_bit, shape.split, per_layer};
        if (per_layer < best.ms_per_layer) best = timed;
        qnae_tune& b = best_of[shape.tile_bits - 12];
        if (shape.split == 0 && per_layer < b.ms_per_layer) b = timed;
        return QNAE_OK;
    };
    for (int TB = 12; TB <= 14; ++TB)
        for (int low = 4; low <= 5; ++low)
            for (int page : {18, 64})
                if (int rc = time_shape(qnae_tune{TB, low, page, 0, 0.0})) return rc;
    // the splits of the fastest shape of every tile size, as qnae_autotune
    for (const qnae_tune& base : best_of) {
        bool splits = false;
        for (const auto& c : classes) splits |= base.tile_bits != 0 && has_split(c.first, base);
        if (splits)
            for (int split = 1; split <= 3; ++split)
                if (int rc = time_shape(qnae_tune{base.tile_bits, base.low_run_bits, base.page_bit, split, 0.0}))
                    return rc;
    }
    for (const auto& c : classes) ctx->tunes[c] = best;
    *out = best;
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

int qnae_get_tune(qnae_ctx* ctx, int32_t n, int32_t cost_dtype, qnae_tune* out) try {
    if (!ctx || !out) return fail(QNAE_EINVAL, "null argument");
    if (int rc = check_tune_target(n, cost_dtype, kResidentMaxN + 1)) return rc;
    *out = tune_for(ctx, n, cost_dtype);
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

}  // extern "C"
