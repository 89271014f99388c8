// C ABI of libqnae.so (include/qnae.h): context, cost diagonal, single-instance
// QAOA run and kernel timing.
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "host.h"

using namespace qnae_host;
using qnae::ClauseRec;
using qnae::MixForm;
using qnae::SweepArgs;

extern "C" {

const char* qnae_last_error(const qnae_ctx*) { return last_error(); }

int qnae_create(qnae_ctx** out, int device) try {
    if (!out) return fail(QNAE_EINVAL, "null output pointer");
    *out = nullptr;
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(QNAE_EINVAL, "device %d outside [0, %d)", device, count);
    HIP_TRY(hipSetDevice(device));
    qnae_ctx* ctx = new qnae_ctx();
    ctx->device = device;
    hipError_t e = hipEventCreateWithFlags(&ctx->staging_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->cost_staging_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = ctx->small.reserve(64);
    if (e == hipSuccess) e = ctx->h_small.reserve(64);
    if (e != hipSuccess) {
        qnae_destroy(ctx);
        return fail(QNAE_EHIP, "qnae_create: %s", hipGetErrorString(e));
    }
    if (int rc = noalloc_setup(ctx)) {
        const std::string msg = last_error();
        qnae_destroy(ctx);
        return fail(rc, "qnae_create: %s", msg.c_str());
    }
    if (const char* tb = std::getenv("QNAE_TILE_BITS")) {
        const int v = std::atoi(tb);
        if (v >= 12 && v <= 14) ctx->tile_bits = v;
    }
    if (const char* gr = std::getenv("QNAE_GRAPHS")) ctx->use_graphs = std::atoi(gr) != 0;
    if (const char* pb = std::getenv("QNAE_PAGE_BIT")) {
        const int v = std::atoi(pb);
        if (v >= 4 && v <= 64) ctx->page_bit = v;
    }
    *out = ctx;
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

int qnae_destroy(qnae_ctx* ctx) try {
    if (!ctx) return QNAE_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (DevBuf* b : {&ctx->state, &ctx->partials, &ctx->luts, &ctx->clauses, &ctx->forms, &ctx->small, &ctx->b_blob,
                      &ctx->c_blob,
                      &ctx->b_states, &ctx->b_partials, &ctx->b_results, &ctx->g_states, &ctx->g_blob,
                      &ctx->g_partials, &ctx->tune_cost, &ctx->s_dev})
        b->release();
    for (HostBuf* b : {&ctx->h_luts, &ctx->h_clauses, &ctx->h_forms, &ctx->h_small, &ctx->h_blob, &ctx->h_results,
                       &ctx->h_sample, &ctx->na_host, &ctx->h_cblob})
        b->release();
    if (ctx->staging_done) (void)hipEventDestroy(ctx->staging_done);
    ctx->batch_plans.clear();  // destroys their captured launch sequences
    if (ctx->cost_staging_done) (void)hipEventDestroy(ctx->cost_staging_done);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    for (auto& r : ctx->prof.pending) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : ctx->prof.pool) (void)hipEventDestroy(e);
    delete ctx;
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

int qnae_build_cost_diagonal(qnae_ctx* ctx, const int32_t* clauses, int32_t m, int32_t n, int32_t k, void* cost_dev,
                             int32_t cost_dtype, uint64_t* num_solutions, void* stream) try {
    return qnae_build_cost_diagonal_pred(ctx, clauses, m, n, k, QNAE_PRED_NAE, cost_dev, cost_dtype, num_solutions,
                                         stream);
} catch (...) {
    return host_exception();
}

}  // extern "C"

namespace {

// Cost diagonal over x < 2^(n - half) (half: the lower half of the NAE
// diagonal, which the global-flip symmetry mirrors onto the upper half).
int build_cost(qnae_ctx* ctx, const int32_t* clauses, int32_t m, int32_t n, int32_t k, int32_t predicate,
               void* cost_dev, int32_t cost_dtype, uint64_t* num_solutions, void* stream, bool half) {
    if (predicate != QNAE_PRED_NAE && predicate != QNAE_PRED_SAT)
        return fail(QNAE_EINVAL, "predicate=%d is not QNAE_PRED_NAE/QNAE_PRED_SAT", predicate);
    if (int rc = check_cost_args(n, m, cost_dtype)) return rc;
    if (!cost_dev) return fail(QNAE_EINVAL, "null cost_dev");
    if (int rc = check_aligned(cost_dev, "cost_dev")) return rc;
    if (int rc = check_literals(clauses, m, n, k)) return rc;
    if (int rc = enter(ctx)) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int states = half ? n - 1 : n;

    HIP_TRY(ctx->h_clauses.reserve(sizeof(ClauseRec) * (size_t)(m > 0 ? m : 1)));
    ClauseRec* recs = (ClauseRec*)ctx->h_clauses.ptr;
    int nlow = 0;
    const int nrec = make_clause_records(clauses, m, k, recs, predicate, &nlow);
    HIP_TRY(ctx->clauses.reserve(sizeof(ClauseRec) * (size_t)(nrec > 0 ? nrec : 1)));
    if (nrec > 0)
        HIP_TRY(hipMemcpyAsync(ctx->clauses.ptr, recs, sizeof(ClauseRec) * nrec, hipMemcpyHostToDevice, s));
    unsigned long long* zeros = (unsigned long long*)ctx->small.ptr;
    if (num_solutions) HIP_TRY(hipMemsetAsync(zeros, 0, sizeof(unsigned long long), s));

    qnae::CostArgs a;
    a.clauses = (const ClauseRec*)ctx->clauses.ptr;
    a.num_clauses = nrec;
    a.num_low = nlow;
    a.n = states;
    a.cost = cost_dev;
    a.zeros = num_solutions ? zeros : nullptr;
    const double cost_bytes = (double)(cost_dtype == QNAE_U8 ? 1 : 2) * std::ldexp(1.0, states);
    HIP_TRY(timed(ctx, K_COST, cost_bytes, s, [&] { return qnae::launch_cost(a, cost_dtype, n > 32, s); }));
    HIP_TRY(hipEventRecord(ctx->staging_done, s));
    if (num_solutions) {
        HIP_TRY(hipMemcpyAsync(ctx->h_small.ptr, zeros, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        *num_solutions = *(unsigned long long*)ctx->h_small.ptr * (half ? 2ull : 1ull);
    }
    return QNAE_OK;
}

}  // namespace

extern "C" {

int qnae_build_cost_diagonal_pred(qnae_ctx* ctx, const int32_t* clauses, int32_t m, int32_t n, int32_t k,
                                  int32_t predicate, void* cost_dev, int32_t cost_dtype, uint64_t* num_solutions,
                                  void* stream) try {
    return build_cost(ctx, clauses, m, n, k, predicate, cost_dev, cost_dtype, num_solutions, stream, false);
} catch (...) {
    return host_exception();
}

int qnae_build_cost_diagonal_z2(qnae_ctx* ctx, const int32_t* clauses, int32_t m, int32_t n, int32_t k, void* cost_dev,
                                int32_t cost_dtype, uint64_t* num_solutions, void* stream) try {
    if (n < 2) return fail(QNAE_EINVAL, "n=%d below 2 for a half diagonal", n);
    return build_cost(ctx, clauses, m, n, k, QNAE_PRED_NAE, cost_dev, cost_dtype, num_solutions, stream, true);
} catch (...) {
    return host_exception();
}

}  // extern "C"

namespace {

// Depth-p run from |+>. half: state and cost hold x < 2^(n-1) only (NAE
// global-flip symmetry); the readout sums then count every amplitude twice.
int run(qnae_ctx* ctx, const void* cost_dev, int32_t cost_dtype, int32_t n, int32_t m, const double* gammas,
        const double* betas, int32_t p, void* state_dev, qnae_result* out, void* stream, bool half) {
    if (int rc = check_run_args(n, m, cost_dtype, cost_dev, gammas, betas, p)) return rc;
    if (!out) return fail(QNAE_EINVAL, "null result pointer");
    if (int rc = check_aligned(state_dev, "state_dev")) return rc;
    if (half && n <= kResidentMaxN)
        return fail(QNAE_EINVAL, "n=%d: half-state runs need n > %d (smaller n: qnae_qaoa_run)", n, kResidentMaxN);
    if (int rc = enter(ctx)) return rc;
    hipStream_t s = (hipStream_t)stream;
    const bool keep = state_dev != nullptr;
    const int T = p > 0 ? p : 1;
    const int lut_len = m + 1;

    HIP_TRY(ctx->h_luts.reserve(sizeof(float2) * (size_t)T * lut_len));
    HIP_TRY(ctx->h_forms.reserve(sizeof(MixForm) * (size_t)T));
    float2* tables = (float2*)ctx->h_luts.ptr;
    MixForm* forms = (MixForm*)ctx->h_forms.ptr;
    const std::complex<double> final_scale = build_tables(n, m, gammas, betas, p, tables, forms);
    const double readout_scale = std::norm(final_scale) * (half ? 2.0 : 1.0);
    const float2 store_scale = make_float2((float)final_scale.real(), (float)final_scale.imag());

    double* out_dev = (double*)((char*)ctx->small.ptr + 16);
    const double rb = std::ldexp((double)(cost_dtype == QNAE_U8 ? 1 : 2) * T + (keep ? 8.0 : 0.0), n);
    static_assert(sizeof(MixForm) == sizeof(float2), "a mixer form fills one table slot");

    if (n <= kResidentMaxN && (int64_t)T * lut_len + p <= qnae::kResidentInline) {
        // small tables travel in the kernel arguments: one launch, no copies ahead of it
        qnae::ResidentInlineArgs ia;
        qnae::ResidentArgs& a = ia.a;
        a.state_in = nullptr;
        a.cost = cost_dev;
        a.luts = nullptr;
        a.forms = nullptr;
        a.state_out = (float2*)state_dev;
        a.out = out_dev;
        a.store_scale = store_scale;
        a.n = n;
        a.p = p;
        a.lut_len = lut_len;
        std::memcpy(ia.tab, tables, sizeof(float2) * (size_t)T * lut_len);
        if (p > 0) std::memcpy(ia.tab + (size_t)T * lut_len, forms, sizeof(MixForm) * p);
        HIP_TRY(timed(ctx, K_RESIDENT, rb, s, [&] { return qnae::launch_resident_inline(cost_dtype, ia, s); }));
    } else if (n <= kResidentMaxN) {
        HIP_TRY(ctx->luts.reserve(sizeof(float2) * (size_t)T * lut_len));
        HIP_TRY(hipMemcpyAsync(ctx->luts.ptr, tables, sizeof(float2) * (size_t)T * lut_len, hipMemcpyHostToDevice, s));
        HIP_TRY(ctx->forms.reserve(sizeof(MixForm) * (size_t)T));
        if (p > 0) HIP_TRY(hipMemcpyAsync(ctx->forms.ptr, forms, sizeof(MixForm) * p, hipMemcpyHostToDevice, s));
        qnae::ResidentArgs a;
        a.state_in = nullptr;
        a.cost = cost_dev;
        a.luts = (const float2*)ctx->luts.ptr;
        a.forms = (const MixForm*)ctx->forms.ptr;
        a.state_out = (float2*)state_dev;
        a.out = out_dev;
        a.store_scale = store_scale;
        a.n = n;
        a.p = p;
        a.lut_len = lut_len;
        HIP_TRY(timed(ctx, K_RESIDENT, rb, s, [&] { return qnae::launch_resident(cost_dtype, a, s); }));
    } else {
        HIP_TRY(ctx->luts.reserve(sizeof(float2) * (size_t)T * lut_len));
        HIP_TRY(hipMemcpyAsync(ctx->luts.ptr, tables, sizeof(float2) * (size_t)T * lut_len, hipMemcpyHostToDevice, s));
        const qnae_tune tune = tune_for(ctx, n, cost_dtype);
        const int TB = tune.tile_bits;
        const int stored = half ? n - 1 : n;
        float2* psi = (float2*)state_dev;
        if (!psi) {
            HIP_TRY(ctx->state.reserve(sizeof(float2) << stored));
            psi = (float2*)ctx->state.ptr;
        }
        const int64_t blocks = 1ll << (stored - TB);
        HIP_TRY(ctx->partials.reserve(sizeof(double) * 3 * (size_t)blocks));
        SweepPlan P;
        plan_sweeps(P, n, m, p, cost_dtype, TB, tune.low_run_bits, tune.page_bit, tune.split, keep, forms,
                    final_scale);
        P.half = half;
        for (const Op& op : P.ops) {
            SweepArgs a;
            sweep_args(P, op, psi, cost_dev, (const float2*)ctx->luts.ptr, (double*)ctx->partials.ptr, &a);
            HIP_TRY(timed(ctx, op_profile_kind(op), op_bytes(P, op), s,
                          [&] { return qnae::launch_sweep(TB, cost_dtype, op.kind, a, s); }));
        }
        // a symmetric state equals its all-qubit flip: nothing to undo when half
        if (keep && !half && p > 0 && P.flips_before[p])
            HIP_TRY(timed(ctx, K_FINAL, 16.0 * std::ldexp(1.0, n), s,
                          [&] { return qnae::launch_reverse(psi, 1ull << n, s); }));
        HIP_TRY(timed(ctx, K_REDUCE, 24.0 * blocks, s, [&] {
            return qnae::launch_final_reduce((const double*)ctx->partials.ptr, blocks, out_dev, s);
        }));
    }
    HIP_TRY(hipMemcpyAsync(ctx->h_small.ptr, out_dev, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(ctx->staging_done, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double* r = (const double*)ctx->h_small.ptr;
    out->p_success = r[0] * readout_scale;
    out->expected_cost = r[1] * readout_scale;
    out->norm = r[2] * readout_scale;
    return QNAE_OK;
}

}  // namespace

extern "C" {

int qnae_qaoa_run(qnae_ctx* ctx, const void* cost_dev, int32_t cost_dtype, int32_t n, int32_t m,
                  const double* gammas, const double* betas, int32_t p, void* state_dev, qnae_result* out,
                  void* stream) try {
    return run(ctx, cost_dev, cost_dtype, n, m, gammas, betas, p, state_dev, out, stream, false);
} catch (...) {
    return host_exception();
}

int qnae_qaoa_run_z2(qnae_ctx* ctx, const void* cost_dev, int32_t cost_dtype, int32_t n, int32_t m,
                     const double* gammas, const double* betas, int32_t p, void* state_dev, qnae_result* out,
                     void* stream) try {
    return run(ctx, cost_dev, cost_dtype, n, m, gammas, betas, p, state_dev, out, stream, true);
} catch (...) {
    return host_exception();
}

int qnae_profile_enable(qnae_ctx* ctx, int on) try {
    if (!ctx) return fail(QNAE_EINVAL, "null context");
    ctx->prof.on = on != 0;
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

int qnae_profile_read(qnae_ctx* ctx, qnae_kernel_stat* out, int32_t capacity, int32_t* count) try {
    if (!ctx || !count || (capacity > 0 && !out)) return fail(QNAE_EINVAL, "null argument");
    HIP_TRY(hipSetDevice(ctx->device));
    Profiler& P = ctx->prof;
    for (Profiler::Rec& r : P.pending) {
        HIP_TRY(hipEventSynchronize(r.stop));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, r.start, r.stop));
        P.launches[r.kind] += 1;
        P.ms[r.kind] += ms;
        P.bytes[r.kind] += r.bytes;
        P.pool.push_back(r.start);
        P.pool.push_back(r.stop);
    }
    P.pending.clear();
    int c = 0;
    for (int k = 0; k < K_KINDS; ++k) {
        if (!P.launches[k]) continue;
        if (c < capacity) out[c] = {Profiler::name(k), P.launches[k], P.ms[k], P.bytes[k]};
        ++c;
        P.launches[k] = 0;
        P.ms[k] = 0.0;
        P.bytes[k] = 0.0;
    }
    *count = c;
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

}  // extern "C"
