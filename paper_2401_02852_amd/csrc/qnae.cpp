// Host runtime of libqnae.so: context, argument checks, phase tables, the
// sweep planner and the C ABI declared in include/qnae.h.
#include "../../include/qnae.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <algorithm>
#include <vector>

#include "internal.h"

using qnae::ClauseRec;
using qnae::MixForm;
using qnae::SweepArgs;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(e_ == hipErrorOutOfMemory ? QNAE_ENOMEM : QNAE_EHIP, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);             \
    } while (0)

// Device buffer that only grows.
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipError_t reserve(size_t need) {
        if (need <= bytes) return hipSuccess;
        if (ptr) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return e;
            (void)hipFree(ptr);
            ptr = nullptr;
            bytes = 0;
        }
        hipError_t e = hipMalloc(&ptr, need);
        if (e == hipSuccess) bytes = need;
        return e;
    }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
};

// Pinned host buffer that only grows; an event guards reuse while an
// asynchronous copy from it may still be running.
struct HostBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipError_t reserve(size_t need) {
        if (need <= bytes) return hipSuccess;
        if (ptr) (void)hipHostFree(ptr);
        ptr = nullptr;
        bytes = 0;
        hipError_t e = hipHostMalloc(&ptr, need, hipHostMallocDefault);
        if (e == hipSuccess) bytes = need;
        return e;
    }
    void release() {
        if (ptr) (void)hipHostFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
};

constexpr int kResidentMaxN = 14;

}  // namespace

// Event-timed kernel tallies (qnae_profile_*).
struct Profiler {
    struct Rec {
        int kind;
        double bytes;
        hipEvent_t start, stop;
    };
    static constexpr int kKinds = 7;
    static const char* name(int k) {
        static const char* names[kKinds] = {"cost", "sweep_first", "sweep_middle", "sweep_boundary",
                                            "sweep_final", "resident", "final_reduce"};
        return names[k];
    }
    bool on = false;
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    uint64_t launches[kKinds] = {};
    double ms[kKinds] = {}, bytes[kKinds] = {};
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
};

struct qnae_ctx {
    int device = 0;
    Profiler prof;
    DevBuf state, partials, luts, clauses, forms, small;  // small: zeros counter + 3 result doubles
    HostBuf h_luts, h_clauses, h_forms, h_small;
    hipEvent_t staging_done = nullptr;  // last async copy out of pinned staging
    int tile_bits = 13;                 // tile size of the plain sweeps (log2 amplitudes)
    int min_low_run = 4;                // minimum contiguous low run (log2 amplitudes)
    int page_bit = 18;                  // first index bit above a 2 MiB page of amplitudes
    int persistent = 0;                 // persistent prefetching sweep grids
};

namespace {

int enter(qnae_ctx* ctx) {
    if (!ctx) return fail(QNAE_EINVAL, "null context");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipEventSynchronize(ctx->staging_done));
    return QNAE_OK;
}

enum { K_COST, K_FIRST, K_MIDDLE, K_BOUNDARY, K_FINAL, K_RESIDENT, K_REDUCE };

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

int check_cost_args(int32_t n, int32_t m, int32_t dtype) {
    if (n < 1 || n > QNAE_MAX_N) return fail(QNAE_EINVAL, "n=%d outside [1, %d]", n, QNAE_MAX_N);
    if (dtype != QNAE_U8 && dtype != QNAE_U16) return fail(QNAE_EINVAL, "cost_dtype=%d is not QNAE_U8/QNAE_U16", dtype);
    if (m < 0 || m > 65535) return fail(QNAE_EINVAL, "m=%d outside [0, 65535]", m);
    if (dtype == QNAE_U8 && m > 255) return fail(QNAE_EINVAL, "m=%d needs QNAE_U16 (QNAE_U8 holds m <= 255)", m);
    return QNAE_OK;
}

// ---------------------------------------------------------------------------
// Mixer forms and phase tables
// ---------------------------------------------------------------------------

struct Layer {
    MixForm form;
    std::complex<double> scale;  // scalar factor of the whole layer's mixer
};

// R(beta) = cos(beta) I - i sin(beta) X for every qubit. Device butterflies
// apply (I - i t X), optionally followed by X; the product of the n scalar
// factors is returned in `scale`.
Layer mixer_form(double beta, int n) {
    const double cb = std::cos(beta), sb = std::sin(beta);
    Layer L;
    if (std::fabs(sb) <= std::fabs(cb)) {
        L.form.t = (float)(sb / cb);
        L.form.flip = 0;
        L.scale = std::pow(std::complex<double>(cb, 0.0), n);
    } else {
        L.form.t = (float)(-cb / sb);
        L.form.flip = 1;
        L.scale = std::pow(std::complex<double>(0.0, -sb), n);
    }
    return L;
}

// Phase tables: table l holds prev_scale * exp(-i gamma_l c) for c = 0..m,
// where prev_scale is the previous layer's mixer factor (2^{-n/2}, the
// amplitude of |+>, for layer 0). Returns the factor left after the last layer.
std::complex<double> build_tables(int n, int m, const double* gammas, const double* betas, int p,
                                  float2* tables, MixForm* forms) {
    std::complex<double> prev(std::pow(2.0, -0.5 * n), 0.0);
    const int T = p > 0 ? p : 1;
    for (int l = 0; l < T; ++l) {
        const double g = p > 0 ? gammas[l] : 0.0;
        for (int c = 0; c <= m; ++c) {
            const std::complex<double> e = prev * std::complex<double>(std::cos(g * c), -std::sin(g * c));
            tables[(size_t)l * (m + 1) + c] = make_float2((float)e.real(), (float)e.imag());
        }
        if (p > 0) {
            const Layer L = mixer_form(betas[l], n);
            forms[l] = L.form;
            prev = L.scale;
        }
    }
    return p > 0 ? prev : std::complex<double>(1.0, 0.0);
}

// ---------------------------------------------------------------------------
// Sweep plan
// ---------------------------------------------------------------------------

struct Group {
    std::vector<int> pos;  // global bit of each tile bit
    uint32_t mask;         // tile bits this group mixes
};

struct Op {
    int group;
    int kind;                              // qnae::SweepKind
    int pre_layer, post_layer, lut_layer;  // -1 when unused
};

// Qubit groups of the sweeps. Group A holds the low run [0, cA) of x and a
// few high bits; every other group holds the low run [0, cmin) (not mixed,
// for contiguous global accesses) and a piece of the remaining high bits.
// Bits at or above `page` select a 2 MiB page of the state (8-byte
// amplitudes); a tile that spans k of them touches 2^k pages, so these bits
// are dealt out evenly over the groups to keep every tile within a few TLB
// entries.
std::vector<Group> make_groups(int n, int TB, int cmin, int page) {
    std::vector<Group> g;
    Group A;
    if (n <= TB) {
        for (int i = 0; i < TB; ++i) A.pos.push_back(i);
        A.mask = (1u << TB) - 1u;
        g.push_back(A);
        return g;
    }
    const int rest = n - TB;
    const int h = (rest + (TB - cmin) - 1) / (TB - cmin);
    std::vector<int> P;
    for (int b = std::max(page, TB); b < n; ++b) P.push_back(b);
    const int target = ((int)P.size() + h) / (h + 1);
    const int a = std::min(std::min(target, TB - cmin), (int)P.size());
    const int cA = TB - a;
    std::vector<int> atop(P.end() - a, P.end());
    for (int i = 0; i < cA; ++i) A.pos.push_back(i);
    for (int b : atop) A.pos.push_back(b);
    A.mask = (1u << TB) - 1u;
    g.push_back(A);
    // bits left for the other groups, page bits first
    std::vector<int> RP, RN;
    for (int b = cA; b < n; ++b) {
        if (std::find(atop.begin(), atop.end(), b) != atop.end()) continue;
        (b >= page ? RP : RN).push_back(b);
    }
    const int R = (int)(RP.size() + RN.size());
    std::vector<std::vector<int>> piece(h);
    std::vector<int> size(h);
    for (int i = 0; i < h; ++i) size[i] = R / h + (i < R % h ? 1 : 0);
    for (size_t q = 0; q < RP.size(); ++q) piece[q % h].push_back(RP[q]);
    size_t nx = 0;
    for (int i = 0; i < h; ++i)
        while ((int)piece[i].size() < size[i]) piece[i].push_back(RN[nx++]);
    for (int i = 0; i < h; ++i) {
        Group B;
        std::vector<int> bits = piece[i];
        // fill up to TB - cmin bits with unmixed bits just above the low run
        std::vector<int> fill;
        for (int b = cmin; (int)(bits.size() + fill.size()) < TB - cmin; ++b)
            if (std::find(bits.begin(), bits.end(), b) == bits.end()) fill.push_back(b);
        std::vector<int> all = fill;
        all.insert(all.end(), bits.begin(), bits.end());
        std::sort(all.begin(), all.end());
        for (int b = 0; b < cmin; ++b) B.pos.push_back(b);
        B.mask = 0u;
        for (int b : all) {
            if (std::find(bits.begin(), bits.end(), b) != bits.end()) B.mask |= 1u << B.pos.size();
            B.pos.push_back(b);
        }
        g.push_back(B);
    }
    return g;
}

// Each layer mixes every group once. The last group of a layer is fused with
// the next layer's phase and with that layer's mixing of the same group, so
// every layer after the first costs (number of groups - 1) sweeps. The first
// sweep starts from the phase table (no load) and the last one only reads the
// state for the readout unless the final state is kept.
std::vector<Op> make_plan(int ngroups, int p) {
    using namespace qnae;
    std::vector<Op> ops;
    if (p == 0) {
        ops.push_back({0, SK_P0, -1, -1, 0});
        return ops;
    }
    ops.push_back({0, SK_FIRST, -1, 0, 0});
    std::vector<int> pending;  // groups not yet mixed for layer l
    for (int g = 1; g < ngroups; ++g) pending.push_back(g);
    for (int l = 0;; ++l) {
        if (pending.empty()) {  // one group: the previous sweep mixed it already
            if (l == p - 1) {
                ops.push_back({0, SK_FINAL, -1, -1, -1});
                return ops;
            }
            ops.push_back({0, SK_BOUNDARY, -1, l + 1, l + 1});
            continue;
        }
        int last = pending.back();
        for (int g : pending)
            if (g != 0) last = g;
        for (int g : pending)
            if (g != last) ops.push_back({g, SK_MIDDLE, l, -1, -1});
        if (l == p - 1) {
            ops.push_back({last, SK_FINAL, l, -1, -1});
            return ops;
        }
        ops.push_back({last, SK_BOUNDARY, l, l + 1, l + 1});
        pending.clear();
        for (int g = 0; g < ngroups; ++g)
            if (g != last) pending.push_back(g);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* qnae_last_error(const qnae_ctx*) { return g_err.c_str(); }

int qnae_create(qnae_ctx** out, int device) {
    if (!out) return fail(QNAE_EINVAL, "null output pointer");
    *out = nullptr;
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(QNAE_EINVAL, "device %d outside [0, %d)", device, count);
    HIP_TRY(hipSetDevice(device));
    qnae_ctx* ctx = new qnae_ctx();
    ctx->device = device;
    hipError_t e = hipEventCreateWithFlags(&ctx->staging_done, hipEventDisableTiming);
    if (e == hipSuccess) e = ctx->small.reserve(64);
    if (e == hipSuccess) e = ctx->h_small.reserve(64);
    if (e != hipSuccess) {
        qnae_destroy(ctx);
        return fail(QNAE_EHIP, "qnae_create: %s", hipGetErrorString(e));
    }
    if (const char* tb = std::getenv("QNAE_TILE_BITS")) {
        const int v = std::atoi(tb);
        if (v >= 12 && v <= 14) ctx->tile_bits = v;
    }
    if (const char* ps = std::getenv("QNAE_PERSISTENT")) ctx->persistent = std::atoi(ps) != 0;
    if (const char* pb = std::getenv("QNAE_PAGE_BIT")) {
        const int v = std::atoi(pb);
        if (v >= 4 && v <= 64) ctx->page_bit = v;
    }
    *out = ctx;
    return QNAE_OK;
}

int qnae_destroy(qnae_ctx* ctx) {
    if (!ctx) return QNAE_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->state.release();
    ctx->partials.release();
    ctx->luts.release();
    ctx->clauses.release();
    ctx->forms.release();
    ctx->small.release();
    ctx->h_luts.release();
    ctx->h_clauses.release();
    ctx->h_forms.release();
    ctx->h_small.release();
    if (ctx->staging_done) (void)hipEventDestroy(ctx->staging_done);
    for (auto& r : ctx->prof.pending) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : ctx->prof.pool) (void)hipEventDestroy(e);
    delete ctx;
    return QNAE_OK;
}

int qnae_build_cost_diagonal(qnae_ctx* ctx, const int32_t* clauses, int32_t m, int32_t n, int32_t k,
                             void* cost_dev, int32_t cost_dtype, uint64_t* num_solutions, void* stream) {
    if (int rc = check_cost_args(n, m, cost_dtype)) return rc;
    if (k < 1 || k > 64) return fail(QNAE_EINVAL, "k=%d outside [1, 64]", k);
    if (!cost_dev) return fail(QNAE_EINVAL, "null cost_dev");
    if (m > 0 && !clauses) return fail(QNAE_EINVAL, "null clauses with m=%d", m);
    for (int64_t i = 0; i < (int64_t)m * k; ++i) {
        const int32_t l = clauses[i];
        if (l == 0 || l > n || l < -n) return fail(QNAE_EINVAL, "literal %d at index %lld outside +-[1, n=%d]", l, (long long)i, n);
    }
    if (int rc = enter(ctx)) return rc;
    hipStream_t s = (hipStream_t)stream;

    HIP_TRY(ctx->h_clauses.reserve(sizeof(ClauseRec) * (size_t)(m > 0 ? m : 1)));
    ClauseRec* recs = (ClauseRec*)ctx->h_clauses.ptr;
    int nrec = 0;
    for (int i = 0; i < m; ++i) {
        uint64_t mask = 0, pat = 0;
        bool never = false;
        for (int j = 0; j < k; ++j) {
            const int32_t l = clauses[(size_t)i * k + j];
            const uint64_t bit = 1ull << ((l > 0 ? l : -l) - 1);
            const bool neg = l < 0;
            if (mask & bit) {
                if (((pat & bit) != 0) != neg) never = true;  // x and NOT x: never all equal
            } else {
                mask |= bit;
                if (neg) pat |= bit;
            }
        }
        if (never) continue;
        ClauseRec r;
        const uint64_t mh = mask & ~31ull;
        r.mask_hi_lo = (uint32_t)mh;
        r.mask_hi_hi = (uint32_t)(mh >> 32);
        r.pat_lo = (uint32_t)pat;
        r.pat_hi = (uint32_t)(pat >> 32);
        const uint32_t lm = (uint32_t)(mask & 31u), lp = (uint32_t)(pat & 31u);
        r.zero_tab = 0u;
        r.full_tab = 0u;
        for (uint32_t j = 0; j < 32; ++j) {
            const uint32_t y = (j ^ lp) & lm;
            if (y == 0u) r.zero_tab |= 1u << j;
            if (y == lm) r.full_tab |= 1u << j;
        }
        recs[nrec++] = r;
    }
    HIP_TRY(ctx->clauses.reserve(sizeof(ClauseRec) * (size_t)(nrec > 0 ? nrec : 1)));
    if (nrec > 0)
        HIP_TRY(hipMemcpyAsync(ctx->clauses.ptr, recs, sizeof(ClauseRec) * nrec, hipMemcpyHostToDevice, s));
    unsigned long long* zeros = (unsigned long long*)ctx->small.ptr;
    if (num_solutions) HIP_TRY(hipMemsetAsync(zeros, 0, sizeof(unsigned long long), s));

    qnae::CostArgs a;
    a.clauses = (const ClauseRec*)ctx->clauses.ptr;
    a.num_clauses = nrec;
    a.n = n;
    a.cost = cost_dev;
    a.zeros = num_solutions ? zeros : nullptr;
    const double cost_bytes = (double)(cost_dtype == QNAE_U8 ? 1 : 2) * std::ldexp(1.0, n);
    HIP_TRY(timed(ctx, K_COST, cost_bytes, s, [&] { return qnae::launch_cost(a, cost_dtype, s); }));
    HIP_TRY(hipEventRecord(ctx->staging_done, s));
    if (num_solutions) {
        HIP_TRY(hipMemcpyAsync(ctx->h_small.ptr, zeros, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        *num_solutions = *(unsigned long long*)ctx->h_small.ptr;
    }
    return QNAE_OK;
}

int qnae_qaoa_run(qnae_ctx* ctx, const void* cost_dev, int32_t cost_dtype, int32_t n, int32_t m,
                  const double* gammas, const double* betas, int32_t p, void* state_dev, qnae_result* out,
                  void* stream) {
    if (int rc = check_cost_args(n, m, cost_dtype)) return rc;
    if (!cost_dev) return fail(QNAE_EINVAL, "null cost_dev");
    if (!out) return fail(QNAE_EINVAL, "null result pointer");
    if (p < 0 || p > 100000) return fail(QNAE_EINVAL, "p=%d outside [0, 100000]", p);
    if (p > 0 && (!gammas || !betas)) return fail(QNAE_EINVAL, "null angle arrays with p=%d", p);
    for (int l = 0; l < p; ++l)
        if (!std::isfinite(gammas[l]) || !std::isfinite(betas[l])) return fail(QNAE_EINVAL, "non-finite angle at layer %d", l);
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
    const double readout_scale = std::norm(final_scale);
    const float2 store_scale = make_float2((float)final_scale.real(), (float)final_scale.imag());

    HIP_TRY(ctx->luts.reserve(sizeof(float2) * (size_t)T * lut_len));
    HIP_TRY(hipMemcpyAsync(ctx->luts.ptr, tables, sizeof(float2) * (size_t)T * lut_len, hipMemcpyHostToDevice, s));
    double* out_dev = (double*)((char*)ctx->small.ptr + 16);

    if (n <= kResidentMaxN) {
        HIP_TRY(ctx->forms.reserve(sizeof(MixForm) * (size_t)T));
        if (p > 0) HIP_TRY(hipMemcpyAsync(ctx->forms.ptr, forms, sizeof(MixForm) * p, hipMemcpyHostToDevice, s));
        qnae::ResidentArgs a;
        a.cost = cost_dev;
        a.luts = (const float2*)ctx->luts.ptr;
        a.forms = (const MixForm*)ctx->forms.ptr;
        a.state_out = (float2*)state_dev;
        a.out = out_dev;
        a.store_scale = store_scale;
        a.n = n;
        a.p = p;
        a.lut_len = lut_len;
        const double rb = std::ldexp((double)(cost_dtype == QNAE_U8 ? 1 : 2) * T + (keep ? 8.0 : 0.0), n);
        HIP_TRY(timed(ctx, K_RESIDENT, rb, s, [&] { return qnae::launch_resident(cost_dtype, a, s); }));
    } else {
        const int TB = ctx->tile_bits;
        float2* psi = (float2*)state_dev;
        if (!psi) {
            HIP_TRY(ctx->state.reserve(sizeof(float2) << n));
            psi = (float2*)ctx->state.ptr;
        }
        const int64_t blocks = 1ll << (n - TB);  // upper bound on any sweep's grid
        int64_t reduce_blocks = 0;
        HIP_TRY(ctx->partials.reserve(sizeof(double) * 3 * (size_t)blocks));
        const std::vector<Group> groups = make_groups(n, TB, ctx->min_low_run, ctx->page_bit);
        const std::vector<Op> ops = make_plan((int)groups.size(), p);
        // flips_before[l]: parity of cot-form layers among 0 .. l-1
        std::vector<int> flips_before(T + 1, 0);
        for (int l = 0; l < p; ++l) flips_before[l + 1] = flips_before[l] ^ forms[l].flip;
        const int cb = cost_dtype == QNAE_U8 ? 1 : 2;
        for (const Op& op : ops) {
            const Group& g = groups[op.group];
            SweepArgs a;
            a.psi = psi;
            a.cost = cost_dev;
            a.lut = op.lut_layer >= 0 ? (const float2*)ctx->luts.ptr + (size_t)op.lut_layer * lut_len : nullptr;
            a.partials = (double*)ctx->partials.ptr;
            a.n = n;
            a.nw = n - TB;
            a.tile_bits = 0;
            for (int i = 0; i < TB; ++i) {
                a.pos[i] = (uint8_t)g.pos[i];
                a.tile_bits |= 1ull << g.pos[i];
            }
            a.wmask = ((1ull << n) - 1ull) & ~a.tile_bits;
            a.persistent = ctx->persistent;
            a.lut_len = lut_len;
            a.pre_mask = op.pre_layer >= 0 ? g.mask : 0u;
            a.post_mask = op.post_layer >= 0 ? g.mask : 0u;
            a.pre_t = op.pre_layer >= 0 ? forms[op.pre_layer].t : 0.f;
            a.post_t = op.post_layer >= 0 ? forms[op.post_layer].t : 0.f;
            a.store_scale = store_scale;
            a.store = keep ? 1 : 0;
            a.cflip = op.kind == qnae::SK_BOUNDARY ? flips_before[op.lut_layer]
                      : op.kind == qnae::SK_FINAL  ? flips_before[p]
                                                   : 0;
            double per_amp = 0.0;
            int kind = K_MIDDLE;
            switch (op.kind) {
                case qnae::SK_FIRST: per_amp = 8.0 + cb; kind = K_FIRST; break;
                case qnae::SK_MIDDLE: per_amp = 16.0; kind = K_MIDDLE; break;
                case qnae::SK_BOUNDARY: per_amp = 16.0 + cb; kind = K_BOUNDARY; break;
                default: per_amp = (op.kind == qnae::SK_FINAL ? 8.0 : 0.0) + cb + (keep ? 8.0 : 0.0); kind = K_FINAL;
            }
            uint32_t grid = 0;
            HIP_TRY(timed(ctx, kind, per_amp * std::ldexp(1.0, n), s,
                          [&] { return qnae::launch_sweep(TB, cost_dtype, op.kind, a, s, &grid); }));
            if (op.kind == qnae::SK_FINAL || op.kind == qnae::SK_P0) reduce_blocks = grid;
        }
        if (keep && p > 0 && flips_before[p])
            HIP_TRY(timed(ctx, K_FINAL, 16.0 * std::ldexp(1.0, n), s,
                          [&] { return qnae::launch_reverse(psi, 1ull << n, s); }));
        HIP_TRY(timed(ctx, K_REDUCE, 24.0 * reduce_blocks, s, [&] {
            return qnae::launch_final_reduce((const double*)ctx->partials.ptr, reduce_blocks, out_dev, s);
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

int qnae_profile_enable(qnae_ctx* ctx, int on) {
    if (!ctx) return fail(QNAE_EINVAL, "null context");
    ctx->prof.on = on != 0;
    return QNAE_OK;
}

int qnae_profile_read(qnae_ctx* ctx, qnae_kernel_stat* out, int32_t capacity, int32_t* count) {
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
    for (int k = 0; k < Profiler::kKinds; ++k) {
        if (!P.launches[k]) continue;
        if (c < capacity) out[c] = {Profiler::name(k), P.launches[k], P.ms[k], P.bytes[k]};
        ++c;
        P.launches[k] = 0;
        P.ms[k] = 0.0;
        P.bytes[k] = 0.0;
    }
    *count = c;
    return QNAE_OK;
}

}  // extern "C"
