// qnae_qaoa_run_noalloc: qnae_qaoa_run for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc). The same kernels and the same sweep plan as qnae_qaoa_run, with
// every piece of device scratch (the phase tables, the mixer forms of the
// single-workgroup kernel, the per-tile readout sums and the three result
// sums) in one file-scope static device array, and host staging in a fixed
// pinned buffer the context reserved when it was created. The planning runs
// in fixed storage (make_group_specs, for_each_op), so a call allocates
// nothing, on the device or on the host.
#include <mutex>

#include "host.h"

namespace {

using qnae::MixForm;

// Scratch layout (bytes). Every call on a device shares that device's copy.
constexpr size_t kResultAt = 0;                    // 3 doubles
constexpr int kMaxTable = 1 << 18;                 // phase table entries, p * (m + 1)
constexpr size_t kTablesAt = 256;                  // float2 [kMaxTable]
constexpr int kMaxLayers = 4096;                   // p
constexpr size_t kFormsAt = kTablesAt + 8ull * kMaxTable;          // MixForm [kMaxLayers]
constexpr int kMaxTiles = 1 << 18;                 // tiles of one sweep (n - tile bits <= 18)
constexpr size_t kPartialsAt = kFormsAt + sizeof(MixForm) * kMaxLayers;  // 3 doubles per tile
constexpr size_t kScratchBytes = kPartialsAt + 24ull * kMaxTiles;        // 8.03 MiB

// Pinned host staging of a context: tables, forms, flip prefix, result.
constexpr size_t kHostTablesAt = 0;
constexpr size_t kHostFormsAt = 8ull * kMaxTable;
constexpr size_t kHostFlipsAt = kHostFormsAt + sizeof(MixForm) * kMaxLayers;
constexpr size_t kHostResultAt = (kHostFlipsAt + sizeof(int) * (kMaxLayers + 1) + 7) / 8 * 8;
constexpr size_t kHostBytes = kHostResultAt + 3 * sizeof(double);

static_assert(kFormsAt % 256 == 0 && kPartialsAt % 256 == 0, "scratch regions stay 256-byte aligned");
static_assert(kHostResultAt % 8 == 0, "result doubles stay aligned");

// The array itself. In host code its name is only a stand-in for the
// symbol: every host use goes through the device address that
// hipGetSymbolAddress returns for it (one per device, below).
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` per device

}  // namespace

namespace qnae_host {

int noalloc_setup(qnae_ctx* ctx) {
    if (ctx->device < 0 || ctx->device >= kMaxDevices)
        return fail(QNAE_EINVAL, "device %d: the static scratch table holds %d devices", ctx->device, kMaxDevices);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_scratch[ctx->device]) {
            void* ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fail(QNAE_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", ctx->device,
                            hipGetErrorString(e));
            g_scratch[ctx->device] = ptr;
        }
        ctx->na_dev = g_scratch[ctx->device];
    }
    HIP_TRY(ctx->na_host.reserve(kHostBytes));
    return QNAE_OK;
}

}  // namespace qnae_host

using namespace qnae_host;

extern "C" int qnae_qaoa_run_noalloc(qnae_ctx* ctx, const void* cost_dev, int32_t cost_dtype, int32_t n, int32_t m,
                                     const double* gammas, const double* betas, int32_t p, void* state_dev,
                                     qnae_result* out, void* stream) try {
    if (int rc = check_run_args(n, m, cost_dtype, cost_dev, gammas, betas, p)) return rc;
    if (!out) return fail(QNAE_EINVAL, "null result pointer");
    if (int rc = check_aligned(state_dev, "state_dev")) return rc;
    if (n > kResidentMaxN && !state_dev)
        return fail(QNAE_EINVAL, "n=%d: state_dev is required above n=%d (the state is the working buffer)", n,
                    kResidentMaxN);
    if (p > kMaxLayers) return fail(QNAE_EINVAL, "p=%d above the static scratch's %d layers", p, kMaxLayers);
    const int T = p > 0 ? p : 1;
    const int lut_len = m + 1;
    if ((int64_t)T * lut_len > kMaxTable)
        return fail(QNAE_EINVAL, "phase tables of %lld entries (p * (m + 1)) above the static scratch's %d",
                    (long long)T * lut_len, kMaxTable);
    if (!ctx) return fail(QNAE_EINVAL, "null context");
    const bool resident = n <= kResidentMaxN;
    const qnae_tune tune = tune_for(ctx, n, cost_dtype);
    const int TB = tune.tile_bits;
    const int64_t tiles = resident ? 0 : 1ll << (n - TB);
    if (tiles > kMaxTiles)
        return fail(QNAE_EINVAL, "n=%d with %d-bit tiles needs %lld tile sums, above the static scratch's %d (n <= %d)",
                    n, TB, (long long)tiles, kMaxTiles, 18 + TB);
    if (int rc = enter(ctx)) return rc;
    if (!ctx->na_dev || ctx->na_host.bytes < kHostBytes) return fail(QNAE_EINVAL, "context without no-alloc scratch");
    hipStream_t s = (hipStream_t)stream;
    const bool keep = state_dev != nullptr;

    char* const dev = (char*)ctx->na_dev;
    float2* const d_tables = (float2*)(dev + kTablesAt);
    MixForm* const d_forms = (MixForm*)(dev + kFormsAt);
    double* const d_partials = (double*)(dev + kPartialsAt);
    double* const d_result = (double*)(dev + kResultAt);
    char* const host = (char*)ctx->na_host.ptr;
    float2* const h_tables = (float2*)(host + kHostTablesAt);
    MixForm* const h_forms = (MixForm*)(host + kHostFormsAt);
    int* const h_flips = (int*)(host + kHostFlipsAt);
    double* const h_result = (double*)(host + kHostResultAt);

    const std::complex<double> final_scale = build_tables(n, m, gammas, betas, p, h_tables, h_forms);
    h_flips[0] = 0;
    for (int l = 0; l < p; ++l) h_flips[l + 1] = h_flips[l] ^ h_forms[l].flip;
    const double readout_scale = std::norm(final_scale);
    HIP_TRY(hipMemcpyAsync(d_tables, h_tables, sizeof(float2) * (size_t)T * lut_len, hipMemcpyHostToDevice, s));

    if (resident) {
        if (p > 0) HIP_TRY(hipMemcpyAsync(d_forms, h_forms, sizeof(MixForm) * p, hipMemcpyHostToDevice, s));
        qnae::ResidentArgs a;
        a.state_in = nullptr;
        a.cost = cost_dev;
        a.luts = d_tables;
        a.forms = d_forms;
        a.state_out = (float2*)state_dev;
        a.out = d_result;
        a.store_scale = make_float2((float)final_scale.real(), (float)final_scale.imag());
        a.n = n;
        a.p = p;
        a.lut_len = lut_len;
        HIP_TRY(qnae::launch_resident(cost_dtype, a, s));
    } else {
        GroupSpec spec[kMaxGroups];
        const int ngroups = make_group_specs(n, TB, tune.low_run_bits, tune.page_bit, tune.split, spec);
        const PlanRef plan{n, p, TB, lut_len, keep, false, h_forms, h_flips, final_scale};
        float2* const psi = (float2*)state_dev;
        hipError_t e = hipSuccess;
        for_each_op(ngroups, p, false, [&](const Op& op) {
            if (e != hipSuccess) return;
            int pos[16];
            for (int i = 0; i < TB; ++i) pos[i] = spec[op.group].pos[i];
            qnae::SweepArgs a;
            sweep_args_for(plan, pos, spec[op.group].mask, op, psi, cost_dev, d_tables, d_partials, &a);
            e = qnae::launch_sweep(TB, cost_dtype, op.kind, a, s);
        });
        HIP_TRY(e);
        if (keep && p > 0 && h_flips[p]) HIP_TRY(qnae::launch_reverse(psi, 1ull << n, s));
        HIP_TRY(qnae::launch_final_reduce(d_partials, tiles, d_result, s));
    }
    HIP_TRY(hipMemcpyAsync(h_result, d_result, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(ctx->staging_done, s));
    HIP_TRY(hipStreamSynchronize(s));
    out->p_success = h_result[0] * readout_scale;
    out->expected_cost = h_result[1] * readout_scale;
    out->norm = h_result[2] * readout_scale;
    return QNAE_OK;
} catch (...) {
    return host_exception();
}
