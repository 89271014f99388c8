// qnae_qaoa_grad: gradient of w_psucc p_succ + w_energy E[C] by a hand-written
// adjoint pass (include/qnae.h). See adjoint.hip for the formulas.
//
// n <= 13: one workgroup does the forward pass, the readout and the reverse
// pass with both states in LDS. Larger n: the forward pass runs as one sweep
// plan that also stores the state after every `every` layers (checkpoints:
// the ends of segments); then for each segment from the last, reverse sweeps
// take lam (the first one forms lam = W psi_p) and that segment's checkpoint
// (psi, uncomputed in place) through the inverse layers, summing the inner
// products per tile.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "host.h"

using namespace qnae_host;
using qnae::MixForm;
using qnae::SweepArgs;

extern "C" {

int qnae_qaoa_grad(qnae_ctx* ctx, const void* cost_dev, int32_t cost_dtype, int32_t n, int32_t m,
                   const double* gammas, const double* betas, int32_t p, double w_psucc, double w_energy,
                   int32_t checkpoint_every, double* dgammas, double* dbetas, qnae_result* out, void* stream) try {
    if (int rc = check_run_args(n, m, cost_dtype, cost_dev, gammas, betas, p)) return rc;
    if (!out) return fail(QNAE_EINVAL, "null result pointer");
    if (p > 0 && (!dgammas || !dbetas)) return fail(QNAE_EINVAL, "null gradient arrays with p=%d", p);
    if (checkpoint_every < 0) return fail(QNAE_EINVAL, "checkpoint_every=%d < 0", checkpoint_every);
    if (!std::isfinite(w_psucc) || !std::isfinite(w_energy)) return fail(QNAE_EINVAL, "non-finite weights");
    // a segment longer than p layers is one segment (and p + every stays in range)
    const int every = checkpoint_every > 0 ? std::min(checkpoint_every, std::max(p, 1)) : 4;
    if (int rc = enter(ctx)) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int lut_len = m + 1;
    const size_t N = (size_t)1 << n;

    if (n <= 13) {
        // tables: forward phases exp(-i gamma c) (unit), (cos b, sin b)
        Blob B;
        const size_t lut_at = B.take(sizeof(float2) * (size_t)(p > 0 ? p : 1) * lut_len);
        const size_t cs_at = B.take(sizeof(float2) * (size_t)(p > 0 ? p : 1));
        const size_t out_at = B.take(sizeof(double) * (3 + 2 * (size_t)p));
        HIP_TRY(ctx->h_blob.reserve(B.size));
        HIP_TRY(ctx->g_blob.reserve(B.size));
        char* h = (char*)ctx->h_blob.ptr;
        char* d = (char*)ctx->g_blob.ptr;
        float2* lut = (float2*)(h + lut_at);
        float2* cs = (float2*)(h + cs_at);
        for (int l = 0; l < p; ++l) {
            phase_row(gammas[l], m, 1.0, -1, lut + (size_t)l * lut_len);
            cs[l] = make_float2((float)std::cos(betas[l]), (float)std::sin(betas[l]));
        }
        const int nck = p > 1 ? (p - 1) / every : 0;
        HIP_TRY(ctx->g_states.reserve(sizeof(float2) * N * (size_t)(nck > 0 ? nck : 1)));
        HIP_TRY(hipMemcpyAsync(d, h, out_at, hipMemcpyHostToDevice, s));
        qnae::ResidentGradArgs a;
        a.cost = cost_dev;
        a.luts = (const float2*)(d + lut_at);
        a.cs = (const float2*)(d + cs_at);
        a.ckpt = (float2*)ctx->g_states.ptr;
        a.out = (double*)(d + out_at);
        a.w_psucc = w_psucc;
        a.w_energy = w_energy;
        a.n = n;
        a.p = p;
        a.lut_len = lut_len;
        a.every = every;
        HIP_TRY(timed(ctx, K_RESIDENT, std::ldexp(3.0 * p, n), s, [&] { return qnae::launch_resident_grad(cost_dtype, a, s); }));
        HIP_TRY(hipMemcpyAsync(h + out_at, d + out_at, sizeof(double) * (3 + 2 * (size_t)p), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(ctx->staging_done, s));
        HIP_TRY(hipStreamSynchronize(s));
        const double* r = (const double*)(h + out_at);
        out->p_success = r[0];
        out->expected_cost = r[1];
        out->norm = r[2];
        for (int l = 0; l < p; ++l) {
            dgammas[l] = r[3 + l];
            dbetas[l] = r[3 + p + l];
        }
        return QNAE_OK;
    }

    // ---- tiled path ----------------------------------------------------------
    const int TB = qnae::kAdjointTileBits;
    const int nseg = p > 0 ? (p + every - 1) / every : 1;
    const std::vector<Group> groups = make_groups(n, TB, ctx->min_low_run, ctx->page_bit, 0);
    const uint32_t tiles = 1u << (n - TB);
    // checkpoints 0 .. nseg-1 (state after each segment), then lam
    HIP_TRY(ctx->g_states.reserve(sizeof(float2) * N * (size_t)(nseg + 1)));
    float2* ck = (float2*)ctx->g_states.ptr;
    float2* lam = ck + N * (size_t)nseg;

    // The forward pass is one plan over all p layers, in place in the last
    // checkpoint's buffer; the boundary sweep that completes the last layer
    // of segment j < nseg - 1 also stores checkpoint j.
    const int T = p > 0 ? p : 1;
    std::vector<float2> ftab((size_t)T * lut_len), btab((size_t)T * lut_len);
    std::vector<MixForm> forms(T);
    const std::complex<double> final_scale = build_tables(n, m, gammas, betas, p, ftab.data(), forms.data());
    SweepPlan F;
    plan_sweeps(F, n, m, p, cost_dtype, TB, ctx->min_low_run, ctx->page_bit, 0, true, forms.data(), final_scale);
    std::vector<int> ckpt_of(F.ops.size(), -1);  // checkpoint stored by each forward sweep
    int stored = 0;
    for (size_t q = 0; q < F.ops.size(); ++q) {
        const Op& op = F.ops[q];
        if (op.kind != qnae::SK_BOUNDARY || op.pre_layer < 0) continue;
        const int done_layers = op.lut_layer;  // its pre mixing completes layer lut_layer - 1
        if (done_layers % every == 0 && done_layers < p) {
            ckpt_of[q] = done_layers / every - 1;
            ++stored;
        }
    }
    if (stored != nseg - 1)
        return fail(QNAE_EINVAL, "n=%d: %zu qubit groups, the forward pass needs at least two", n, groups.size());

    // Reverse segments: b-layer i of segment j is forward layer b - 1 - i.
    struct Seg {
        int a, b;
        size_t blut_at;
        std::vector<AdjOp> aops;
        std::vector<Layer> inv;  // inverse mixer of b-layer i: exp(+i beta X) per qubit
    };
    std::vector<Seg> segs(nseg);
    int total_aops = 0;
    for (int j = 0; j < nseg; ++j) {
        Seg& S = segs[j];
        S.a = j * every;
        S.b = p > 0 ? std::min(p, S.a + every) : 0;
        const int L = S.b - S.a;
        // the inverse phase exp(+i gamma c) times the scalar factor the
        // inverse mixer's butterflies left out
        S.blut_at = (size_t)S.a * lut_len;
        S.inv.resize(L);
        for (int i = 0; i < L; ++i) {
            S.inv[i] = mixer_form(-betas[S.b - 1 - i], n);
            phase_row(gammas[S.b - 1 - i], m, S.inv[i].scale, +1, btab.data() + S.blut_at + (size_t)i * lut_len);
        }
        if (L > 0) S.aops = make_adjoint_plan((int)groups.size(), L);
        total_aops += (int)S.aops.size();
    }
    // The reverse pass opens with a sweep that mixes one group and forms lam.
    if (!segs[nseg - 1].aops.empty() && segs[nseg - 1].aops[0].kind != qnae::AK_MIDDLE)
        return fail(QNAE_EINVAL, "n=%d: %zu qubit groups, the reverse pass needs at least two", n, groups.size());
    Blob B;
    const size_t flut_at = B.take(sizeof(float2) * ftab.size());
    const size_t blut_at = B.take(sizeof(float2) * btab.size());
    const size_t rp_at = B.take(sizeof(double*) * (total_aops + 1));
    const size_t rb_at = B.take(sizeof(uint32_t) * (total_aops + 1));
    const size_t ro_at = B.take(sizeof(double*) * (total_aops + 1));
    const size_t res_at = B.take(sizeof(double) * 3 * (total_aops + 1));
    HIP_TRY(ctx->h_blob.reserve(B.size));
    HIP_TRY(ctx->g_blob.reserve(B.size));
    HIP_TRY(ctx->g_partials.reserve(sizeof(double) * 3 * tiles * (size_t)(total_aops + 1)));
    char* h = (char*)ctx->h_blob.ptr;
    char* d = (char*)ctx->g_blob.ptr;
    double* parts = (double*)ctx->g_partials.ptr;
    double* res_dev = (double*)(d + res_at);
    std::memcpy(h + flut_at, ftab.data(), sizeof(float2) * ftab.size());
    std::memcpy(h + blut_at, btab.data(), sizeof(float2) * btab.size());
    {
        const double** rp = (const double**)(h + rp_at);
        uint32_t* rb = (uint32_t*)(h + rb_at);
        double** ro = (double**)(h + ro_at);
        for (int q = 0; q <= total_aops; ++q) {  // entry total_aops: forward readout
            rp[q] = parts + 3 * (size_t)tiles * q;
            rb[q] = tiles;
            ro[q] = res_dev + 3 * (size_t)q;
        }
    }
    HIP_TRY(hipMemcpyAsync(d, h, B.size, hipMemcpyHostToDevice, s));
    const float2* d_flut = (const float2*)(d + flut_at);
    const float2* d_blut = (const float2*)(d + blut_at);

    // forward pass
    double* fwd_parts = parts + 3 * (size_t)tiles * total_aops;
    float2* const run = ck + N * (size_t)(nseg - 1);
    for (size_t q = 0; q < F.ops.size(); ++q) {
        const Op& op = F.ops[q];
        SweepArgs a;
        sweep_args(F, op, run, cost_dev, d_flut, fwd_parts, &a);
        if (ckpt_of[q] < 0) {
            HIP_TRY(timed(ctx, op_profile_kind(op), op_bytes(F, op), s,
                          [&] { return qnae::launch_sweep(TB, cost_dtype, op.kind, a, s); }));
            continue;
        }
        const std::complex<double> f = mixer_form(betas[op.lut_layer - 1], n).scale;
        a.ckpt = ck + N * (size_t)ckpt_of[q];
        a.ckpt_scale = make_float2((float)f.real(), (float)f.imag());
        HIP_TRY(timed(ctx, op_profile_kind(op), op_bytes(F, op) + std::ldexp(8.0, n), s,
                      [&] { return qnae::launch_sweep_ckpt(cost_dtype, a, s); }));
    }
    if (p > 0 && F.flips_before[p]) HIP_TRY(qnae::launch_reverse(run, N, s));
    // lam = W psi_p is formed by the first reverse sweep, which mixes one
    // group only (a layer spans at least two groups here, n > TB), from the
    // psi_p and cost it loads
    // reverse segments, last first. `relabel`: lam's index x holds element
    // x ^ (2^n - 1) (an odd number of cotangent forms so far); psi restarts
    // from a checkpoint in natural order at each segment, so within a segment
    // it is relabelled against lam by the value `relabel` had at the start.
    // done[i]: qubits of b-layer i mixed by earlier sweeps.
    int q = 0;
    std::vector<std::pair<int, const AdjOp*>> order;  // (segment, op) in launch order
    std::vector<double> gamma_weight;                 // per op: |F|^2 of its phase layer
    int relabel = 0;
    for (int j = nseg - 1; j >= 0; --j) {
        const Seg& S = segs[j];
        float2* psi = ck + N * (size_t)j;
        const int psi_flip = relabel;
        std::vector<int> done(S.inv.size(), 0);
        for (const AdjOp& op : S.aops) {
            const Group& g = groups[op.group];
            qnae::AdjointArgs a;
            std::memset(&a, 0, sizeof a);
            a.lam = lam;
            a.psi = psi;
            a.cost = cost_dev;
            a.lut = op.phase_layer >= 0 ? d_blut + S.blut_at + (size_t)op.phase_layer * lut_len : nullptr;
            a.partials = parts + 3 * (size_t)tiles * q;
            a.n = n;
            a.nw = n - TB;
            a.lut_len = lut_len;
            for (int i = 0; i < TB; ++i) {
                a.pos[i] = (uint8_t)g.pos[i];
                a.tile_bits |= 1ull << g.pos[i];
            }
            a.wmask = ((1ull << n) - 1ull) & ~a.tile_bits;
            a.pre_mask = op.pre_layer >= 0 ? g.mask : 0u;
            a.post_mask = op.post_layer >= 0 ? g.mask : 0u;
            const int qubits = __builtin_popcount(g.mask);
            // one qubit's |factor|^2: cos^2 (tangent form) or sin^2, 1 / (1 + t^2) either way
            auto factor2 = [&](int i) {
                const double b = betas[S.b - 1 - i];
                const double c = std::cos(b), sn = std::sin(b);
                return S.inv[i].form.flip ? sn * sn : c * c;
            };
            if (op.pre_layer >= 0) {
                const int i = op.pre_layer;
                a.pre_t = S.inv[i].form.t;
                a.pre_r = (float)factor2(i);
                a.pre_w = (float)std::pow(factor2(i), done[i]);
                done[i] += qubits;
            }
            double gw = 0.0;
            if (op.phase_layer >= 0) {
                const int i = op.phase_layer;
                relabel ^= S.inv[i].form.flip;
                a.cost_flip = relabel ? (uint64_t)N - 1ull : 0ull;
                gw = std::pow(factor2(i), n);
            }
            if (op.post_layer >= 0) {
                const int i = op.post_layer;
                a.post_t = S.inv[i].form.t;
                a.post_r = (float)factor2(i);
                a.post_w = (float)std::pow(factor2(i), done[i]);
                done[i] += qubits;
            }
            a.psi_flip = psi_flip;
            a.store_psi = op.kind == qnae::AK_END ? 0 : 1;
            const bool weigh = q == 0;
            a.w_psucc = (float)w_psucc;
            a.w_energy = (float)w_energy;
            const double cost_bytes = cost_dtype == QNAE_U8 ? 1.0 : 2.0;
            const double bytes = std::ldexp(32.0 - (a.store_psi ? 0.0 : 8.0) - (weigh ? 8.0 : 0.0) +
                                                (op.phase_layer >= 0 || weigh ? cost_bytes : 0.0),
                                            n);
            HIP_TRY(timed(ctx, K_ADJOINT, bytes, s,
                          [&] { return qnae::launch_adjoint(cost_dtype, op.kind, a, s, weigh); }));
            order.emplace_back(j, &op);
            gamma_weight.push_back(gw);
            ++q;
        }
    }
    HIP_TRY(qnae::launch_final_reduce_batch((const double* const*)(d + rp_at), (const uint32_t*)(d + rb_at),
                                            (double* const*)(d + ro_at), total_aops + 1, s));
    HIP_TRY(hipMemcpyAsync(h + res_at, d + res_at, sizeof(double) * 3 * (total_aops + 1), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(ctx->staging_done, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double* r = (const double*)(h + res_at);
    for (int l = 0; l < p; ++l) dgammas[l] = dbetas[l] = 0.0;
    for (int k = 0; k < total_aops; ++k) {
        const Seg& S = segs[order[k].first];
        const AdjOp& op = *order[k].second;
        if (op.pre_layer >= 0) dbetas[S.b - 1 - op.pre_layer] += 2.0 * r[3 * k];
        if (op.phase_layer >= 0) dgammas[S.b - 1 - op.phase_layer] += 2.0 * gamma_weight[k] * r[3 * k + 1];
        if (op.post_layer >= 0) dbetas[S.b - 1 - op.post_layer] += 2.0 * r[3 * k + 2];
    }
    const double sc = std::norm(final_scale);
    out->p_success = r[3 * total_aops] * sc;
    out->expected_cost = r[3 * total_aops + 1] * sc;
    out->norm = r[3 * total_aops + 2] * sc;
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

int qnae_qaoa_grad_batched(qnae_ctx* ctx, const qnae_grad_job* jobs, int32_t count, double w_psucc, double w_energy,
                           int32_t checkpoint_every, qnae_result* out, void* stream) try {
    if (count < 0 || (count > 0 && (!jobs || !out))) return fail(QNAE_EINVAL, "bad job array (count=%d)", count);
    if (checkpoint_every < 0) return fail(QNAE_EINVAL, "checkpoint_every=%d < 0", checkpoint_every);
    if (!std::isfinite(w_psucc) || !std::isfinite(w_energy)) return fail(QNAE_EINVAL, "non-finite weights");
    for (int i = 0; i < count; ++i) {
        const qnae_grad_job& j = jobs[i];
        int rc = check_run_args(j.n, j.m, j.cost_dtype, j.cost_dev, j.gammas, j.betas, j.p);
        if (!rc && j.p > 0 && (!j.dgammas || !j.dbetas)) rc = fail(QNAE_EINVAL, "null gradient arrays");
        if (rc) return fail(rc, "job %d: %s", i, std::string(last_error()).c_str());
    }
    if (count == 0) return QNAE_OK;
    const int every = checkpoint_every > 0 ? checkpoint_every : 4;
    if (int rc = enter(ctx)) return rc;
    hipStream_t s = (hipStream_t)stream;
    // Small jobs: per job its tables and outputs in one blob, checkpoints in
    // one device buffer, one launch per cost type.
    Blob B, C;
    std::vector<size_t> lut_at(count), cs_at(count), out_at(count), ck_at(count);
    std::vector<int> small[2];
    for (int i = 0; i < count; ++i) {
        const qnae_grad_job& j = jobs[i];
        if (j.n > 13) continue;
        const int T = j.p > 0 ? j.p : 1;
        lut_at[i] = B.take(sizeof(float2) * (size_t)T * (j.m + 1));
        cs_at[i] = B.take(sizeof(float2) * (size_t)T);
        out_at[i] = B.take(sizeof(double) * (3 + 2 * (size_t)j.p));
        const int nck = j.p > 1 ? (j.p - 1) / every : 0;
        ck_at[i] = C.take(sizeof(float2) * ((size_t)1 << j.n) * (size_t)(nck > 0 ? nck : 1));
        small[j.cost_dtype == QNAE_U16 ? 1 : 0].push_back(i);
    }
    size_t args_at[2];
    for (int g = 0; g < 2; ++g) args_at[g] = B.take(sizeof(qnae::ResidentGradArgs) * small[g].size());
    if (!small[0].empty() || !small[1].empty()) {
        HIP_TRY(ctx->h_blob.reserve(B.size));
        HIP_TRY(ctx->g_blob.reserve(B.size));
        HIP_TRY(ctx->g_states.reserve(C.size));
        char* h = (char*)ctx->h_blob.ptr;
        char* d = (char*)ctx->g_blob.ptr;
        // Tables and arguments job by job, chunks of jobs over the context's
        // host threads (each job writes only its own rows and argument slot).
        std::vector<std::pair<int, int>> work;  // (cost type, position in its launch)
        size_t entries = 0;
        for (int g = 0; g < 2; ++g)
            for (size_t q = 0; q < small[g].size(); ++q) {
                work.emplace_back(g, (int)q);
                entries += (size_t)jobs[small[g][q]].p * (size_t)(jobs[small[g][q]].m + 1);
            }
        constexpr int kChunk = 16;
        parallel_for(ctx, ((int)work.size() + kChunk - 1) / kChunk, entries, [&](int chunk) {
            const int w_end = std::min((int)work.size(), (chunk + 1) * kChunk);
            for (int w = chunk * kChunk; w < w_end; ++w) {
                const int g = work[w].first;
                const size_t q = (size_t)work[w].second;
                qnae::ResidentGradArgs* args = (qnae::ResidentGradArgs*)(h + args_at[g]);
                const int i = small[g][q];
                const qnae_grad_job& j = jobs[i];
                const int lut_len = j.m + 1;
                float2* lut = (float2*)(h + lut_at[i]);
                float2* cs = (float2*)(h + cs_at[i]);
                for (int l = 0; l < j.p; ++l) {
                    phase_row(j.gammas[l], j.m, 1.0, -1, lut + (size_t)l * lut_len);
                    cs[l] = make_float2((float)std::cos(j.betas[l]), (float)std::sin(j.betas[l]));
                }
                qnae::ResidentGradArgs& a = args[q];
                a.cost = j.cost_dev;
                a.luts = (const float2*)(d + lut_at[i]);
                a.cs = (const float2*)(d + cs_at[i]);
                a.ckpt = (float2*)((char*)ctx->g_states.ptr + ck_at[i]);
                a.out = (double*)(d + out_at[i]);
                a.w_psucc = w_psucc;
                a.w_energy = w_energy;
                a.n = j.n;
                a.p = j.p;
                a.lut_len = lut_len;
                a.every = every;
            }
        });
        HIP_TRY(hipMemcpyAsync(d, h, B.size, hipMemcpyHostToDevice, s));
        for (int g = 0; g < 2; ++g) {
            if (small[g].empty()) continue;
            double bytes = 0.0;
            for (int i : small[g]) bytes += std::ldexp(3.0 * jobs[i].p, jobs[i].n);
            HIP_TRY(timed(ctx, K_RESIDENT, bytes, s, [&] {
                return qnae::launch_resident_grad_batch(g ? QNAE_U16 : QNAE_U8,
                                                         (const qnae::ResidentGradArgs*)(d + args_at[g]),
                                                         (int)small[g].size(), s);
            }));
        }
        HIP_TRY(hipMemcpyAsync(h, d, args_at[0], hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(ctx->staging_done, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int g = 0; g < 2; ++g)
            for (int i : small[g]) {
                const qnae_grad_job& j = jobs[i];
                const double* r = (const double*)(h + out_at[i]);
                out[i].p_success = r[0];
                out[i].expected_cost = r[1];
                out[i].norm = r[2];
                for (int l = 0; l < j.p; ++l) {
                    j.dgammas[l] = r[3 + l];
                    j.dbetas[l] = r[3 + j.p + l];
                }
            }
    }
    // Large jobs: the tiled adjoint, one after another.
    for (int i = 0; i < count; ++i) {
        const qnae_grad_job& j = jobs[i];
        if (j.n <= 13) continue;
        if (int rc = qnae_qaoa_grad(ctx, j.cost_dev, j.cost_dtype, j.n, j.m, j.gammas, j.betas, j.p, w_psucc, w_energy,
                                    checkpoint_every, j.dgammas, j.dbetas, &out[i], stream))
            return fail(rc, "job %d: %s", i, std::string(last_error()).c_str());
    }
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

}  // extern "C"
