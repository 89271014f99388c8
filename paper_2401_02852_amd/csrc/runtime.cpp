// Host runtime helpers of libqnae.so: errors, buffers, timing, argument
// checks, clause records, mixer forms and phase tables, and the sweep planner.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "host.h"

using qnae::MixForm;

namespace qnae_host {

namespace {
thread_local std::string g_err;
}  // namespace

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
    return build_tables_from(n, m, gammas, betas, p, tables, forms, std::complex<double>(std::pow(2.0, -0.5 * n), 0.0));
}

// scale * exp(sign i g c) for c = 0..m: exp(sign i g c) = exp(sign i g 16 q)
// exp(sign i g r) for c = 16 q + r, both factors from short angle-addition
// recurrences (at most 15 FP64 products from a directly computed value), and
// every entry then one independent product, instead of a sine and a cosine of
// a large argument per entry (the batched solves build tens of thousands of
// entries per call). The entries differ from a direct sine and cosine by at
// most about 1e-13 for m <= 255 and 1e-10 for m up to 65535 (the size of the
// rounding of g c itself there), far below the FP32 rounding of the entries.
// Products are written out: std::complex multiplication carries the infinity
// and NaN recovery of C99 Annex G, a library call per product.
void phase_row(double g, int m, std::complex<double> scale, int sign, float2* out) {
    const double sg = sign < 0 ? -1.0 : 1.0;
    double lo_r[16], lo_i[16];  // exp(sign i g r), r < 16
    lo_r[0] = 1.0;
    lo_i[0] = 0.0;
    const double s1r = std::cos(g), s1i = sg * std::sin(g);
    for (int r = 1; r < 16; ++r) {
        lo_r[r] = lo_r[r - 1] * s1r - lo_i[r - 1] * s1i;
        lo_i[r] = lo_r[r - 1] * s1i + lo_i[r - 1] * s1r;
    }
    const double s16r = std::cos(16.0 * g), s16i = sg * std::sin(16.0 * g);
    double hr = scale.real(), hi = scale.imag();  // scale * exp(sign i g 16 q)
    for (int q = 0; 16 * q <= m; ++q) {
        if (q > 0 && q % 16 == 0) {  // re-anchor the high factor every 256 entries
            const double a = 16.0 * g * q;
            const double cr = std::cos(a), ci = sg * std::sin(a);
            hr = scale.real() * cr - scale.imag() * ci;
            hi = scale.real() * ci + scale.imag() * cr;
        } else if (q > 0) {
            const double t = hr * s16r - hi * s16i;
            hi = hr * s16i + hi * s16r;
            hr = t;
        }
        float* const row = (float*)(out + 16 * q);  // (re, im) pairs
        const int rmax = std::min(15, m - 16 * q);
        for (int r = 0; r <= rmax; ++r) {
            row[2 * r] = (float)(hr * lo_r[r] - hi * lo_i[r]);
            row[2 * r + 1] = (float)(hr * lo_i[r] + hi * lo_r[r]);
        }
    }
}

std::complex<double> build_tables_from(int n, int m, const double* gammas, const double* betas, int p,
                                       float2* tables, MixForm* forms, std::complex<double> first) {
    std::complex<double> prev = first;
    const int T = p > 0 ? p : 1;
    for (int l = 0; l < T; ++l) {
        phase_row(p > 0 ? gammas[l] : 0.0, m, prev, -1, tables + (size_t)l * (m + 1));
        if (p > 0) {
            const Layer L = mixer_form(betas[l], n);
            forms[l] = L.form;
            prev = L.scale;
        }
    }
    return p > 0 ? prev : std::complex<double>(1.0, 0.0);
}

WorkerPool::WorkerPool(int workers) {
    try {
        for (int i = 0; i < workers; ++i) threads_.emplace_back([this] { work(); });
    } catch (...) {  // no thread may be left joinable when construction fails
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        wake_.notify_all();
        for (std::thread& t : threads_) t.join();
        throw;
    }
}

WorkerPool::~WorkerPool() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    wake_.notify_all();
    for (std::thread& t : threads_) t.join();
}

void WorkerPool::drain() {
    for (int i = next_.fetch_add(1); i < count_; i = next_.fetch_add(1)) {
        try {
            (*fn_)(i);
        } catch (...) {
            std::lock_guard<std::mutex> lk(mu_);
            if (!error_) error_ = std::current_exception();
            next_.store(count_);  // hand out no further items
        }
    }
}

void WorkerPool::work() {
    uint64_t seen = 0;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu_);
            wake_.wait(lk, [&] { return stop_ || generation_ != seen; });
            if (stop_) return;
            seen = generation_;
        }
        drain();
        std::lock_guard<std::mutex> lk(mu_);
        if (--busy_ == 0) done_.notify_all();
    }
}

void WorkerPool::run(int count, const std::function<void(int)>& fn) {
    if (count <= 0) return;
    {
        std::lock_guard<std::mutex> lk(mu_);
        fn_ = &fn;
        count_ = count;
        next_.store(0);
        busy_ = (int)threads_.size();
        ++generation_;
    }
    wake_.notify_all();
    drain();
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [&] { return busy_ == 0; });
    fn_ = nullptr;
    std::exception_ptr e = error_;
    error_ = nullptr;
    lk.unlock();
    if (e) std::rethrow_exception(e);
}

void parallel_for(qnae_ctx* ctx, int count, size_t items, const std::function<void(int)>& fn) {
    // below this much work (clause records or table entries) one thread is faster
    constexpr size_t kMinItems = 8192;
    if (count <= 1 || items < kMinItems) {
        for (int i = 0; i < count; ++i) fn(i);
        return;
    }
    if (!ctx->pool) {
        const unsigned hw = std::thread::hardware_concurrency();
        ctx->pool.reset(new WorkerPool((int)std::min(7u, hw > 1 ? hw - 1 : 1u)));
    }
    ctx->pool->run(count, fn);
}

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

const char* last_error() { return g_err.c_str(); }

int host_exception() {
    try {
        throw;
    } catch (const std::bad_alloc&) {
        return fail(QNAE_ENOMEM, "host memory allocation failed");
    } catch (const std::exception& e) {
        return fail(QNAE_ENOMEM, "host resources: %s", e.what());
    } catch (...) {
        return fail(QNAE_ENOMEM, "host resources: unknown exception");
    }
}

hipError_t DevBuf::reserve(size_t need) {
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

void DevBuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

hipError_t HostBuf::reserve(size_t need) {
    if (need <= bytes) return hipSuccess;
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
    hipError_t e = hipHostMalloc(&ptr, need, hipHostMallocDefault);
    if (e == hipSuccess) bytes = need;
    return e;
}

void HostBuf::release() {
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

const char* Profiler::name(int k) {
    static const char* names[K_KINDS] = {"cost", "sweep_first", "sweep_middle", "sweep_boundary", "sweep_final",
                                         "resident", "final_reduce", "batch_cost", "batch_resident", "batch_sweep",
                                         "batch_reduce", "adjoint"};
    return names[k];
}

hipEvent_t Profiler::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

int enter(qnae_ctx* ctx) {
    if (!ctx) return fail(QNAE_EINVAL, "null context");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipEventSynchronize(ctx->staging_done));
    return QNAE_OK;
}

int check_cost_args(int32_t n, int32_t m, int32_t dtype) {
    if (n < 1 || n > QNAE_MAX_N) return fail(QNAE_EINVAL, "n=%d outside [1, %d]", n, QNAE_MAX_N);
    if (dtype != QNAE_U8 && dtype != QNAE_U16) return fail(QNAE_EINVAL, "cost_dtype=%d is not QNAE_U8/QNAE_U16", dtype);
    if (m < 0 || m > 65535) return fail(QNAE_EINVAL, "m=%d outside [0, 65535]", m);
    if (dtype == QNAE_U8 && m > 255) return fail(QNAE_EINVAL, "m=%d needs QNAE_U16 (QNAE_U8 holds m <= 255)", m);
    return QNAE_OK;
}

int check_aligned(const void* ptr, const char* what) {
    if ((uintptr_t)ptr & 15u) return fail(QNAE_EINVAL, "%s is not 16-byte aligned", what);
    return QNAE_OK;
}

int check_run_args(int32_t n, int32_t m, int32_t dtype, const void* cost, const double* gammas, const double* betas,
                   int32_t p) {
    if (int rc = check_cost_args(n, m, dtype)) return rc;
    if (!cost) return fail(QNAE_EINVAL, "null cost_dev");
    if (int rc = check_aligned(cost, "cost_dev")) return rc;
    if (p < 0 || p > 100000) return fail(QNAE_EINVAL, "p=%d outside [0, 100000]", p);
    if (p > 0 && (!gammas || !betas)) return fail(QNAE_EINVAL, "null angle arrays with p=%d", p);
    for (int l = 0; l < p; ++l)
        if (!std::isfinite(gammas[l]) || !std::isfinite(betas[l]))
            return fail(QNAE_EINVAL, "non-finite angle at layer %d", l);
    return QNAE_OK;
}

int check_literals(const int32_t* clauses, int32_t m, int32_t n, int32_t k) {
    if (k < 1 || k > 64) return fail(QNAE_EINVAL, "k=%d outside [1, 64]", k);
    if (m > 0 && !clauses) return fail(QNAE_EINVAL, "null clauses with m=%d", m);
    for (int64_t i = 0; i < (int64_t)m * k; ++i) {
        const int32_t l = clauses[i];
        if (l == 0 || l > n || l < -n)
            return fail(QNAE_EINVAL, "literal %d at index %lld outside +-[1, n=%d]", l, (long long)i, n);
    }
    return QNAE_OK;
}

// Clause records for the cost kernel; clauses that can never be violated (a
// variable with both signs: one literal is always true and one false) are
// dropped. k-SAT clauses only get the all-false table (Section 2.2). Records
// of clauses with a variable below 5 come first (*num_low of them), in input
// order, then those on higher variables only, in input order.
int make_clause_records(const int32_t* clauses, int32_t m, int32_t k, qnae::ClauseRec* recs, int predicate,
                        int* num_low) {
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
        qnae::ClauseRec r;
        const uint64_t mh = mask & ~31ull;
        r.mask_hi_lo = (uint32_t)mh;
        r.mask_hi_hi = (uint32_t)(mh >> 32);
        r.pat_lo = (uint32_t)pat;
        r.pat_hi = (uint32_t)(pat >> 32);
        // Over the positions j of a 32-state run, the literal on low variable
        // v is false where bit v of j equals its negation flag: zero_tab is
        // the AND of those sets over the clause's low variables, full_tab
        // (every low literal true) the AND of their complements.
        static constexpr uint32_t kBitSet[5] = {0xAAAAAAAAu, 0xCCCCCCCCu, 0xF0F0F0F0u, 0xFF00FF00u, 0xFFFF0000u};
        uint32_t zero = ~0u, full = ~0u;
        for (int v = 0; v < 5; ++v) {
            if (!((mask >> v) & 1u)) continue;
            const uint32_t ones = kBitSet[v];  // positions j with bit v of j set
            zero &= ((pat >> v) & 1u) ? ones : ~ones;
            full &= ((pat >> v) & 1u) ? ~ones : ones;
        }
        r.zero_tab = zero;
        r.full_tab = predicate == QNAE_PRED_NAE ? full : 0u;
        recs[nrec++] = r;
    }
    // A clause with a low variable has zero_tab != ~0 (half the run or less).
    const qnae::ClauseRec* mid =
        std::stable_partition(recs, recs + nrec, [](const qnae::ClauseRec& r) { return r.zero_tab != ~0u; });
    if (num_low) *num_low = (int)(mid - recs);
    return nrec;
}

// Qubit groups of the sweeps. Group A holds the low run [0, cA) of x and a
// few high bits; every other group holds the low run [0, cmin) (not mixed,
// for contiguous global accesses) and a piece of the remaining high bits.
// Bits at or above `page` select a 2 MiB page of the state (8-byte
// amplitudes); a tile that spans k of them touches 2^k pages, so these bits
// are dealt out evenly over the groups to keep every tile within a few TLB
// entries. Group A takes the top page bits. The other groups take
// consecutive runs of the bits below `page` in ascending order, and
// consecutive runs of the remaining page bits in descending order, so the
// group with the lowest middle bits gets the highest page run. Measured at
// n = 30 (13-bit tiles): a tile that mixes index bits 14..17 together with
// page bits streams slowest, least so beside bits 18..21; this arrangement
// ran 3% faster than dealing the page bits out round-robin.
//
// With two groups besides A, `split` 1..3 changes which of the bits below
// `page` the second of them mixes (see qnae_tune); which split streams
// fastest depends on n (measured: 1 at n = 30, 3 at n = 31), so the tuner
// times them.
namespace {
// second[k] != 0: the second group takes bit k of the nrn bits below page
// (it takes k1 of them); false when the split does not fit, and then the
// consecutive runs stay.
bool split_second(int split, int nrn, int k1, bool* second) {
    int pick[64], np = 0;
    auto take = [&](int k) {
        for (int j = 0; j < np; ++j)
            if (pick[j] == k) return;
        if (k >= 0 && k < nrn && np < k1) pick[np++] = k;
    };
    if (split == 1 || split == 2) {
        take(split == 1 ? 1 : 0);
        for (int j = 1; j < k1; ++j) take(nrn - j);
    } else if (split == 3) {
        for (int j = 1; j <= 3 && j <= k1; ++j) take(nrn - j);
        for (int k = 0; np < k1 && k < nrn; k += 2) take(k);
    }
    if (np != k1) return false;
    for (int k = 0; k < nrn; ++k) second[k] = false;
    for (int j = 0; j < np; ++j) second[pick[j]] = true;
    return true;
}
}  // namespace

int make_group_specs(int n, int TB, int cmin, int page, int split, GroupSpec* out) {
    GroupSpec& A = out[0];
    A.mask = (1u << TB) - 1u;
    if (n <= TB) {
        for (int i = 0; i < TB; ++i) A.pos[i] = (uint8_t)i;
        return 1;
    }
    const int rest = n - TB;
    const int h = (rest + (TB - cmin) - 1) / (TB - cmin);
    // page bits: the consecutive run [max(page, TB), n); group A takes its top a
    const int first_page = std::max(page, TB);
    const int npage = std::max(0, n - first_page);
    const int target = (npage + h) / (h + 1);
    const int a = std::min(std::min(target, TB - cmin), npage);
    const int cA = TB - a;
    for (int i = 0; i < cA; ++i) A.pos[i] = (uint8_t)i;
    for (int i = 0; i < a; ++i) A.pos[cA + i] = (uint8_t)(n - a + i);
    // bits left for the other groups, page bits (RP) and the others (RN), ascending
    int RP[64], RN[64], nrp = 0, nrn = 0;
    for (int b = cA; b < n - a; ++b) (b >= page ? RP[nrp++] : RN[nrn++]) = b;
    const int R = nrp + nrn;
    // the group of each bit below page: consecutive runs in ascending order
    int rn_group[64];
    for (int i = 0, k = 0; i < h; ++i) {
        const int c = nrp / h + (i < nrp % h ? 1 : 0);
        const int size = R / h + (i < R % h ? 1 : 0);
        for (int j = c; j < size; ++j) rn_group[k++] = i;
    }
    if (h == 2 && split != 0) {
        int k1 = 0;
        for (int k = 0; k < nrn; ++k) k1 += rn_group[k] == 1;
        bool second[64];
        if (split_second(split, nrn, k1, second))
            for (int k = 0; k < nrn; ++k) rn_group[k] = second[k] ? 1 : 0;
    }
    for (int i = 0, q = nrp; i < h; ++i) {
        // consecutive page runs, evenly, top run first; then the other bits
        const int c = nrp / h + (i < nrp % h ? 1 : 0);
        q -= c;
        uint64_t bits = 0;
        for (int k = 0; k < c; ++k) bits |= 1ull << RP[q + k];
        for (int k = 0; k < nrn; ++k)
            if (rn_group[k] == i) bits |= 1ull << RN[k];
        // fill up to TB - cmin bits with unmixed bits just above the low run
        uint64_t all = bits;
        for (int b = cmin; __builtin_popcountll(all) < TB - cmin; ++b) all |= 1ull << b;
        GroupSpec& B = out[1 + i];
        B.mask = 0u;
        int np = 0;
        for (int b = 0; b < cmin; ++b) B.pos[np++] = (uint8_t)b;
        for (uint64_t m = all; m != 0ull; m &= m - 1ull) {
            const int b = __builtin_ctzll(m);
            if ((bits >> b) & 1ull) B.mask |= 1u << np;
            B.pos[np++] = (uint8_t)b;
        }
    }
    return 1 + h;
}

std::vector<Group> make_groups(int n, int TB, int cmin, int page, int split) {
    GroupSpec spec[kMaxGroups];
    const int count = make_group_specs(n, TB, cmin, page, split, spec);
    std::vector<Group> g(count);
    for (int i = 0; i < count; ++i) {
        g[i].pos.assign(spec[i].pos, spec[i].pos + TB);
        g[i].mask = spec[i].mask;
    }
    return g;
}

std::vector<Op> make_plan(int ngroups, int p, bool from_state) {
    std::vector<Op> ops;
    for_each_op(ngroups, p, from_state, [&](const Op& op) { ops.push_back(op); });
    return ops;
}

std::vector<AdjOp> make_adjoint_plan(int ngroups, int L) {
    using namespace qnae;
    std::vector<AdjOp> ops;
    std::vector<int> pending;
    for (int g = 0; g < ngroups; ++g) pending.push_back(g);
    for (int i = 0; i < L; ++i) {
        int last = pending.back();
        for (int g : pending)
            if (g != 0) last = g;
        for (int g : pending)
            if (g != last) ops.push_back({g, AK_MIDDLE, i, -1, -1});
        if (i == L - 1) {
            ops.push_back({last, AK_END, i, i, -1});
            break;
        }
        ops.push_back({last, AK_BOUNDARY, i, i, i + 1});
        pending.clear();
        for (int g = 0; g < ngroups; ++g)
            if (g != last) pending.push_back(g);
    }
    return ops;
}

void plan_sweeps(SweepPlan& P, int n, int m, int p, int dtype, int TB, int cmin, int page, int split, bool keep,
                 const qnae::MixForm* forms, std::complex<double> final_scale, bool from_state) {
    P.n = n;
    P.m = m;
    P.p = p;
    P.TB = TB;
    P.dtype = dtype;
    P.lut_len = m + 1;
    P.keep = keep;
    P.groups = make_groups(n, TB, cmin, page, split);
    P.ops = make_plan((int)P.groups.size(), p, from_state);
    P.forms.assign(forms, forms + p);
    P.flips_before.assign(p + 1, 0);
    for (int l = 0; l < p; ++l) P.flips_before[l + 1] = P.flips_before[l] ^ forms[l].flip;
    P.final_scale = final_scale;
}

void sweep_args(const SweepPlan& P, const Op& op, float2* psi, const void* cost, const float2* luts, double* partials,
                qnae::SweepArgs* a) {
    const Group& g = P.groups[op.group];
    const PlanRef ref{P.n, P.p, P.TB, P.lut_len, P.keep, P.half, P.forms.data(), P.flips_before.data(), P.final_scale};
    sweep_args_for(ref, g.pos.data(), g.mask, op, psi, cost, luts, partials, a);
}

void sweep_args_for(const PlanRef& P, const int* pos, uint32_t mask, const Op& op, float2* psi, const void* cost,
                    const float2* luts, double* partials, qnae::SweepArgs* a) {
    std::memset(a, 0, sizeof *a);
    a->psi = psi;
    a->psi_in = psi;
    a->cost = cost;
    a->lut = op.lut_layer >= 0 ? luts + (size_t)op.lut_layer * P.lut_len : nullptr;
    a->partials = partials;
    a->n = P.n;
    a->nw = P.n - P.TB;
    a->tile_bits = 0;
    for (int i = 0; i < P.TB; ++i) {
        a->pos[i] = (uint8_t)pos[i];
        a->tile_bits |= 1ull << pos[i];
    }
    a->wmask = ((1ull << P.n) - 1ull) & ~a->tile_bits;
    a->lut_len = P.lut_len;
    a->pre_mask = op.pre_layer >= 0 ? mask : 0u;
    a->post_mask = op.post_layer >= 0 ? mask : 0u;
    a->store = P.keep ? 1 : 0;
    a->half = 0;
    a->vbit = -1;
    a->mir = 0;
    if (P.half) {
        // Stored indices are x < 2^(n-1); full index x with bit n-1 set lives
        // at its complement. Bit n-1 of the plan becomes the virtual tile bit
        // (its flip mirrors the stored index); the tile index then fills the
        // stored bits outside the tile except the highest one, which the
        // virtual bit's mirror already covers.
        const uint64_t stored = (1ull << (P.n - 1)) - 1ull;
        uint64_t unit = 0;
        for (int i = 0; i < P.TB; ++i) {
            if (pos[i] == P.n - 1) a->vbit = i;
            else unit |= 1ull << pos[i];
        }
        uint64_t wm = stored & ~unit;
        if (a->vbit >= 0) wm &= ~(1ull << (63 - __builtin_clzll(wm)));
        a->half = 1;
        a->wmask = wm;
        a->tile_bits = unit;
        a->nw = P.n - 1 - P.TB;
        a->mir = stored;
    }
    sweep_args_angles(P, op, a);
}

void sweep_args_angles(const PlanRef& P, const Op& op, qnae::SweepArgs* a) {
    a->pre_t = op.pre_layer >= 0 ? P.forms[op.pre_layer].t : 0.f;
    a->post_t = op.post_layer >= 0 ? P.forms[op.post_layer].t : 0.f;
    a->store_scale = make_float2((float)P.final_scale.real(), (float)P.final_scale.imag());
    // half: the stored state is flip-symmetric, so flipped reads are the same
    a->cflip = P.half                         ? 0
               : op.kind == qnae::SK_BOUNDARY ? P.flips_before[op.lut_layer]
               : op.kind == qnae::SK_FINAL    ? P.flips_before[P.p]
                                              : 0;
}

void sweep_args_angles(const SweepPlan& P, const Op& op, qnae::SweepArgs* a) {
    const PlanRef ref{P.n, P.p, P.TB, P.lut_len, P.keep, P.half, P.forms.data(), P.flips_before.data(), P.final_scale};
    sweep_args_angles(ref, op, a);
}

double op_bytes(const SweepPlan& P, const Op& op) {
    const double cb = P.dtype == QNAE_U8 ? 1.0 : 2.0;
    double per_amp;
    switch (op.kind) {
        case qnae::SK_FIRST: per_amp = 8.0 + cb; break;
        case qnae::SK_MIDDLE: per_amp = 16.0; break;
        case qnae::SK_BOUNDARY: per_amp = 16.0 + cb; break;
        case qnae::SK_FINAL: per_amp = 8.0 + cb + (P.keep ? 8.0 : 0.0); break;
        default: per_amp = cb + (P.keep ? 8.0 : 0.0);
    }
    return per_amp * std::ldexp(1.0, P.half ? P.n - 1 : P.n);
}

int op_profile_kind(const Op& op) {
    switch (op.kind) {
        case qnae::SK_FIRST: return K_FIRST;
        case qnae::SK_MIDDLE: return K_MIDDLE;
        case qnae::SK_BOUNDARY: return K_BOUNDARY;
        default: return K_FINAL;
    }
}

}  // namespace qnae_host
