// Batched C ABI of libqnae.so: many cost diagonals and many QAOA solves per
// launch (include/qnae.h, qnae_*_batched).
//
// A batch is planned on the host: small instances (n <= 14) run whole in one
// workgroup each; larger ones follow their own sweep plan, and step s of every
// plan goes into the same launch, one launch per (sweep kind, cost type). All
// tables and kernel arguments are packed into one pinned blob and uploaded
// with a single copy before the launches.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <utility>

#include "host.h"

using namespace qnae_host;
using qnae::ClauseRec;
using qnae::MixForm;
using qnae::SweepArgs;

extern "C" {

int qnae_build_cost_diagonal_batched(qnae_ctx* ctx, const qnae_cost_job* jobs, int32_t count, void* stream) try {
    if (count < 0 || (count > 0 && !jobs)) return fail(QNAE_EINVAL, "bad job array (count=%d)", count);
    for (int i = 0; i < count; ++i) {
        const qnae_cost_job& j = jobs[i];
        int rc = check_cost_args(j.n, j.m, j.cost_dtype);
        if (!rc && !j.cost_dev) rc = fail(QNAE_EINVAL, "null cost_dev");
        if (!rc) rc = check_aligned(j.cost_dev, "cost_dev");
        if (!rc) rc = check_literals(j.clauses, j.m, j.n, j.k);
        if (!rc && j.predicate != QNAE_PRED_NAE && j.predicate != QNAE_PRED_SAT)
            rc = fail(QNAE_EINVAL, "predicate=%d is not QNAE_PRED_NAE/QNAE_PRED_SAT", j.predicate);
        if (!rc && j.half && (j.predicate != QNAE_PRED_NAE || j.n < 2))
            rc = fail(QNAE_EINVAL, "half diagonals need the NAE predicate and n >= 2");
        if (rc) return fail(rc, "job %d: %s", i, std::string(last_error()).c_str());
    }
    if (count == 0) return QNAE_OK;
    if (int rc = enter(ctx)) return rc;
    hipStream_t s = (hipStream_t)stream;

    // Layout: clause records | zero counters | per type: CostArgs[] and first[]
    size_t total_recs = 0;
    for (int i = 0; i < count; ++i) total_recs += (size_t)jobs[i].m;
    Blob B;
    const size_t rec_at = B.take(sizeof(ClauseRec) * (total_recs ? total_recs : 1));
    const size_t zero_at = B.take(sizeof(unsigned long long) * count);
    std::vector<int> groups[4];  // (dtype, wide)
    for (int i = 0; i < count; ++i) groups[(jobs[i].cost_dtype == QNAE_U16 ? 2 : 0) + (jobs[i].n > 32 ? 1 : 0)].push_back(i);
    size_t args_at[4], first_at[4];
    for (int g = 0; g < 4; ++g) {
        args_at[g] = B.take(sizeof(qnae::CostArgs) * groups[g].size());
        first_at[g] = B.take(sizeof(uint32_t) * (groups[g].size() + 1));
    }
    HIP_TRY(ctx->h_blob.reserve(B.size));
    HIP_TRY(ctx->b_blob.reserve(B.size));
    char* h = (char*)ctx->h_blob.ptr;
    char* d = (char*)ctx->b_blob.ptr;
    ClauseRec* recs = (ClauseRec*)(h + rec_at);
    // each job's records start at the sum of the clause counts before it
    std::vector<size_t> rec_off(count);
    std::vector<int> nrec(count);
    size_t at = 0;
    for (int i = 0; i < count; ++i) {
        rec_off[i] = at;
        at += (size_t)jobs[i].m;
    }
    constexpr int kChunk = 16;  // jobs per host task
    parallel_for(ctx, (count + kChunk - 1) / kChunk, total_recs, [&](int c) {
        for (int i = c * kChunk; i < std::min(count, (c + 1) * kChunk); ++i)
            nrec[i] = make_clause_records(jobs[i].clauses, jobs[i].m, jobs[i].k, recs + rec_off[i], jobs[i].predicate);
    });
    std::memset(h + zero_at, 0, sizeof(unsigned long long) * count);
    unsigned long long* zeros_dev = (unsigned long long*)(d + zero_at);
    uint32_t blocks[4] = {0, 0, 0, 0};
    int maxc[4] = {0, 0, 0, 0};
    double bytes[4] = {0.0, 0.0, 0.0, 0.0};
    for (int g = 0; g < 4; ++g) {
        qnae::CostArgs* args = (qnae::CostArgs*)(h + args_at[g]);
        uint32_t* first = (uint32_t*)(h + first_at[g]);
        for (size_t q = 0; q < groups[g].size(); ++q) {
            const int i = groups[g][q];
            args[q].clauses = (const ClauseRec*)(d + rec_at) + rec_off[i];
            args[q].num_clauses = nrec[i];
            const int states = jobs[i].n - (jobs[i].half ? 1 : 0);
            args[q].n = states;
            args[q].cost = jobs[i].cost_dev;
            args[q].zeros = zeros_dev + i;
            first[q] = blocks[g];
            const uint64_t threads = states >= 5 ? (1ull << (states - 5)) : 1ull;
            const uint64_t nb = (threads + 255) / 256;
            if (blocks[g] + nb > 0x7fffffffull) return fail(QNAE_EINVAL, "batch too large for one grid");
            blocks[g] += (uint32_t)nb;
            maxc[g] = std::max(maxc[g], nrec[i]);
            bytes[g] += std::ldexp(jobs[i].cost_dtype == QNAE_U8 ? 1.0 : 2.0, states);
        }
        first[groups[g].size()] = blocks[g];
    }
    HIP_TRY(hipMemcpyAsync(d, h, B.size, hipMemcpyHostToDevice, s));
    for (int g = 0; g < 4; ++g) {
        if (groups[g].empty()) continue;
        HIP_TRY(timed(ctx, K_BATCH_COST, bytes[g], s, [&] {
            return qnae::launch_cost_batch((const qnae::CostArgs*)(d + args_at[g]), (const uint32_t*)(d + first_at[g]),
                                           (int)groups[g].size(), blocks[g], g >= 2 ? QNAE_U16 : QNAE_U8, maxc[g],
                                           (g & 1) != 0, s);
        }));
    }
    HIP_TRY(hipEventRecord(ctx->staging_done, s));
    bool want = false;
    for (int i = 0; i < count; ++i) want |= jobs[i].num_solutions != nullptr;
    if (want) {
        HIP_TRY(ctx->h_results.reserve(sizeof(unsigned long long) * count));
        HIP_TRY(hipMemcpyAsync(ctx->h_results.ptr, zeros_dev, sizeof(unsigned long long) * count,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const unsigned long long* z = (const unsigned long long*)ctx->h_results.ptr;
        for (int i = 0; i < count; ++i)
            if (jobs[i].num_solutions) *jobs[i].num_solutions = z[i] * (jobs[i].half ? 2ull : 1ull);
    }
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

int qnae_qaoa_run_batched(qnae_ctx* ctx, const qnae_instance* inst, int32_t count, qnae_result* out, void* stream) try {
    if (count < 0 || (count > 0 && (!inst || !out))) return fail(QNAE_EINVAL, "bad instance array (count=%d)", count);
    for (int i = 0; i < count; ++i) {
        const qnae_instance& q = inst[i];
        if (int rc = check_run_args(q.n, q.m, q.cost_dtype, q.cost_dev, q.gammas, q.betas, q.p))
            return fail(rc, "instance %d: %s", i, std::string(last_error()).c_str());
        if (int rc = check_aligned(q.state_dev, "state_dev"))
            return fail(rc, "instance %d: %s", i, std::string(last_error()).c_str());
        if (q.half && q.n <= kResidentMaxN)
            return fail(QNAE_EINVAL, "instance %d: half-state solves need n > %d", i, kResidentMaxN);
    }
    if (count == 0) return QNAE_OK;
    if (int rc = enter(ctx)) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int TB = qnae::kBatchTileBits;

    // ---- host plan ---------------------------------------------------------
    struct Job {
        bool resident;
        int T;
        size_t lut_at, form_at;       // element offsets into the table / form areas
        size_t state_at, part_at;     // element offsets into batch states / partials
        uint32_t tiles;
        SweepPlan plan;
        std::complex<double> final_scale;
    };
    std::vector<Job> jobs(count);
    size_t lut_elems = 0, form_elems = 0, state_elems = 0, part_elems = 0;
    int steps = 0;
    for (int i = 0; i < count; ++i) {
        const qnae_instance& q = inst[i];
        Job& J = jobs[i];
        J.resident = q.n <= kResidentMaxN;
        J.T = q.p > 0 ? q.p : 1;
        J.lut_at = lut_elems;
        lut_elems += (size_t)J.T * (q.m + 1);
        J.form_at = form_elems;
        form_elems += (size_t)J.T;
        const int stored = q.n - (q.half ? 1 : 0);
        J.tiles = J.resident ? 0u : 1u << (stored - TB);
        J.part_at = part_elems;
        part_elems += 3 * (size_t)J.tiles;
        J.state_at = state_elems;
        if (!J.resident && !q.state_dev) state_elems += (size_t)1 << stored;
    }
    std::vector<float2> tables(lut_elems);
    std::vector<MixForm> forms(form_elems);
    constexpr int kChunk = 16;  // instances per host task
    parallel_for(ctx, (count + kChunk - 1) / kChunk, lut_elems, [&](int c) {
        for (int i = c * kChunk; i < std::min(count, (c + 1) * kChunk); ++i) {
            const qnae_instance& q = inst[i];
            Job& J = jobs[i];
            J.final_scale =
                build_tables(q.n, q.m, q.gammas, q.betas, q.p, tables.data() + J.lut_at, forms.data() + J.form_at);
            if (!J.resident) {
                plan_sweeps(J.plan, q.n, q.m, q.p, q.cost_dtype, TB, ctx->min_low_run, ctx->page_bit,
                            q.state_dev != nullptr, forms.data() + J.form_at, J.final_scale);
                J.plan.half = q.half != 0;
            }
        }
    });
    for (int i = 0; i < count; ++i)
        if (!jobs[i].resident) steps = std::max(steps, (int)jobs[i].plan.ops.size());
    Blob B;
    const size_t lut_at = B.take(sizeof(float2) * lut_elems);
    const size_t form_at = B.take(sizeof(MixForm) * form_elems);
    // Sweep launches: step s, bucket (kind, cost type).
    struct Launch {
        int kind, dtype, step;
        bool half;
        std::vector<int> members;
        size_t args_at, first_at;
        uint32_t blocks;
        double bytes;
    };
    std::vector<Launch> launches;
    for (int st = 0; st < steps; ++st) {
        std::map<std::tuple<int, int, bool>, size_t> bucket;
        for (int i = 0; i < count; ++i) {
            const Job& J = jobs[i];
            if (J.resident || st >= (int)J.plan.ops.size()) continue;
            const auto key = std::make_tuple(J.plan.ops[st].kind, inst[i].cost_dtype, J.plan.half);
            auto it = bucket.find(key);
            if (it == bucket.end()) {
                it = bucket.emplace(key, launches.size()).first;
                launches.push_back({std::get<0>(key), std::get<1>(key), st, std::get<2>(key), {}, 0, 0, 0u, 0.0});
            }
            launches[it->second].members.push_back(i);
        }
    }
    for (Launch& L : launches) {
        L.args_at = B.take(sizeof(SweepArgs) * L.members.size());
        L.first_at = B.take(sizeof(uint32_t) * (L.members.size() + 1));
    }
    std::vector<int> res_members[2], sweep_members;
    for (int i = 0; i < count; ++i) {
        if (jobs[i].resident) res_members[inst[i].cost_dtype == QNAE_U16 ? 1 : 0].push_back(i);
        else sweep_members.push_back(i);
    }
    size_t res_at[2];
    for (int g = 0; g < 2; ++g) res_at[g] = B.take(sizeof(qnae::ResidentArgs) * res_members[g].size());
    const size_t red_part_at = B.take(sizeof(double*) * sweep_members.size());
    const size_t red_blocks_at = B.take(sizeof(uint32_t) * sweep_members.size());
    const size_t red_out_at = B.take(sizeof(double*) * sweep_members.size());

    // ---- device buffers ------------------------------------------------------
    HIP_TRY(ctx->h_blob.reserve(B.size));
    std::memcpy((char*)ctx->h_blob.ptr + lut_at, tables.data(), sizeof(float2) * lut_elems);
    std::memcpy((char*)ctx->h_blob.ptr + form_at, forms.data(), sizeof(MixForm) * form_elems);
    HIP_TRY(ctx->b_blob.reserve(B.size));
    HIP_TRY(ctx->b_states.reserve(sizeof(float2) * (state_elems ? state_elems : 1)));
    HIP_TRY(ctx->b_partials.reserve(sizeof(double) * (part_elems ? part_elems : 1)));
    HIP_TRY(ctx->b_results.reserve(sizeof(double) * 3 * count));
    HIP_TRY(ctx->h_results.reserve(sizeof(double) * 3 * count));
    char* h = (char*)ctx->h_blob.ptr;
    char* d = (char*)ctx->b_blob.ptr;
    const float2* d_luts = (const float2*)(d + lut_at);
    const MixForm* d_forms = (const MixForm*)(d + form_at);
    float2* d_states = (float2*)ctx->b_states.ptr;
    double* d_parts = (double*)ctx->b_partials.ptr;
    double* d_results = (double*)ctx->b_results.ptr;

    auto psi_of = [&](int i) -> float2* {
        return inst[i].state_dev ? (float2*)inst[i].state_dev : d_states + jobs[i].state_at;
    };
    for (Launch& L : launches) {
        SweepArgs* args = (SweepArgs*)(h + L.args_at);
        uint32_t* first = (uint32_t*)(h + L.first_at);
        for (size_t q = 0; q < L.members.size(); ++q) {
            const int i = L.members[q];
            const Job& J = jobs[i];
            const Op& op = J.plan.ops[L.step];
            sweep_args(J.plan, op, psi_of(i), inst[i].cost_dev, d_luts + J.lut_at, d_parts + J.part_at, &args[q]);
            first[q] = L.blocks;
            L.blocks += J.tiles;
            L.bytes += op_bytes(J.plan, op);
        }
        first[L.members.size()] = L.blocks;
    }
    for (int g = 0; g < 2; ++g) {
        qnae::ResidentArgs* ra = (qnae::ResidentArgs*)(h + res_at[g]);
        for (size_t q = 0; q < res_members[g].size(); ++q) {
            const int i = res_members[g][q];
            const Job& J = jobs[i];
            ra[q].state_in = nullptr;
            ra[q].cost = inst[i].cost_dev;
            ra[q].luts = d_luts + J.lut_at;
            ra[q].forms = d_forms + J.form_at;
            ra[q].state_out = (float2*)inst[i].state_dev;
            ra[q].out = d_results + 3 * (size_t)i;
            ra[q].store_scale = make_float2((float)J.final_scale.real(), (float)J.final_scale.imag());
            ra[q].n = inst[i].n;
            ra[q].p = inst[i].p;
            ra[q].lut_len = inst[i].m + 1;
        }
    }
    {
        const double** rp = (const double**)(h + red_part_at);
        uint32_t* rb = (uint32_t*)(h + red_blocks_at);
        double** ro = (double**)(h + red_out_at);
        for (size_t q = 0; q < sweep_members.size(); ++q) {
            const int i = sweep_members[q];
            rp[q] = d_parts + jobs[i].part_at;
            rb[q] = jobs[i].tiles;
            ro[q] = d_results + 3 * (size_t)i;
        }
    }

    // ---- upload and launch ---------------------------------------------------
    HIP_TRY(hipMemcpyAsync(d, h, B.size, hipMemcpyHostToDevice, s));
    // All launches of the batch; `prof` brackets each with timing events.
    auto enqueue = [&](hipStream_t st, bool prof) -> int {
        auto run = [&](int kind, double bytes, auto&& fn) -> hipError_t {
            return prof ? timed(ctx, kind, bytes, st, fn) : fn();
        };
        for (int g = 0; g < 2; ++g) {
            if (res_members[g].empty()) continue;
            double rbytes = 0.0;
            for (int i : res_members[g]) rbytes += std::ldexp((g ? 2.0 : 1.0) * jobs[i].T, inst[i].n);
            HIP_TRY(run(K_BATCH_RESIDENT, rbytes, [&] {
                return qnae::launch_resident_batch(g ? QNAE_U16 : QNAE_U8, (const qnae::ResidentArgs*)(d + res_at[g]),
                                                   (int)res_members[g].size(), st);
            }));
        }
        for (const Launch& L : launches) {
            HIP_TRY(run(K_BATCH_SWEEP, L.bytes, [&] {
                return qnae::launch_sweep_batch(L.dtype, L.kind, (const SweepArgs*)(d + L.args_at),
                                                (const uint32_t*)(d + L.first_at), (int)L.members.size(), L.blocks, st,
                                                L.half);
            }));
        }
        for (int i : sweep_members) {
            const SweepPlan& P = jobs[i].plan;
            if (P.keep && !P.half && P.p > 0 && P.flips_before[P.p])
                HIP_TRY(qnae::launch_reverse(psi_of(i), 1ull << inst[i].n, st));
        }
        if (!sweep_members.empty()) {
            HIP_TRY(run(K_BATCH_REDUCE, 24.0 * part_elems / 3, [&] {
                return qnae::launch_final_reduce_batch((const double* const*)(d + red_part_at),
                                                       (const uint32_t*)(d + red_blocks_at),
                                                       (double* const*)(d + red_out_at), (int)sweep_members.size(), st);
            }));
        }
        return QNAE_OK;
    };
    if (ctx->prof.on || !ctx->use_graphs) {
        if (int rc = enqueue(s, ctx->prof.on)) return rc;
    } else {
        // The launch sequence depends only on the batch's shape and on where
        // its arguments live, so a captured graph is replayed for a repeated
        // shape (the arguments themselves were just uploaded).
        uint64_t key = 1469598103934665603ull;
        auto mix = [&](uint64_t v) { key = (key ^ v) * 1099511628211ull; };
        mix((uint64_t)(uintptr_t)d);
        mix(B.size);
        for (int g = 0; g < 2; ++g) mix(res_members[g].size());
        for (const Launch& L : launches) {
            mix((uint64_t)L.half << 48 | (uint64_t)L.kind << 40 | (uint64_t)L.dtype << 32 | L.blocks);
            mix(L.members.size() << 32 | L.args_at);
        }
        for (int i : sweep_members) {
            const SweepPlan& P = jobs[i].plan;
            if (P.keep && !P.half && P.p > 0 && P.flips_before[P.p]) mix((uint64_t)(uintptr_t)psi_of(i) ^ inst[i].n);
        }
        mix(sweep_members.size());
        hipGraphExec_t exec = nullptr;
        for (auto& e : ctx->graphs)
            if (e.first == key) exec = e.second;
        if (!exec) {
            HIP_TRY(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
            const int rc = enqueue(ctx->capture_stream, false);
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(ctx->capture_stream, &graph);
            if (rc) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            HIP_TRY(ec);
            const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIP_TRY(ei);
            if (ctx->graphs.size() >= 16) {
                (void)hipGraphExecDestroy(ctx->graphs.front().second);
                ctx->graphs.erase(ctx->graphs.begin());
            }
            ctx->graphs.emplace_back(key, exec);
        }
        HIP_TRY(hipGraphLaunch(exec, s));
    }
    HIP_TRY(hipMemcpyAsync(ctx->h_results.ptr, d_results, sizeof(double) * 3 * count, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(ctx->staging_done, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double* r = (const double*)ctx->h_results.ptr;
    for (int i = 0; i < count; ++i) {
        const double sc = std::norm(jobs[i].final_scale) * (inst[i].half ? 2.0 : 1.0);
        out[i].p_success = r[3 * i] * sc;
        out[i].expected_cost = r[3 * i + 1] * sc;
        out[i].norm = r[3 * i + 2] * sc;
    }
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

}  // extern "C"
