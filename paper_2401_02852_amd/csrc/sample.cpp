// qnae_sample (include/qnae.h): outcomes of a state for caller-supplied
// uniforms, and their costs. See sample.hip for the draw.
#include <cmath>
#include <cstdint>
#include <cstring>

#include "host.h"

using namespace qnae_host;

extern "C" {

int qnae_sample(qnae_ctx* ctx, const void* state_dev, int32_t n, const void* cost_dev, int32_t cost_dtype,
                const double* uniforms, int32_t count, uint64_t* samples, int32_t* sample_costs, void* stream) try {
    if (n < 1 || n > QNAE_MAX_N) return fail(QNAE_EINVAL, "n=%d outside [1, %d]", n, QNAE_MAX_N);
    if (count < 0 || count > (1 << 24)) return fail(QNAE_EINVAL, "count=%d outside [0, 2^24]", count);
    if (!state_dev) return fail(QNAE_EINVAL, "null state_dev");
    if ((uintptr_t)state_dev & 15u) return fail(QNAE_EINVAL, "state_dev is not 16-byte aligned");
    if (count > 0 && (!uniforms || !samples)) return fail(QNAE_EINVAL, "null uniforms or samples");
    if (cost_dev && cost_dtype != QNAE_U8 && cost_dtype != QNAE_U16)
        return fail(QNAE_EINVAL, "cost_dtype=%d is not QNAE_U8/QNAE_U16", cost_dtype);
    for (int q = 0; q < count; ++q)
        if (!(uniforms[q] >= 0.0 && uniforms[q] < 1.0))
            return fail(QNAE_EINVAL, "uniforms[%d]=%g outside [0, 1)", q, uniforms[q]);
    if (int rc = enter(ctx)) return rc;
    hipStream_t s = (hipStream_t)stream;
    const size_t T = (((size_t)1 << n) + (1u << qnae::kSampleTileBits) - 1) >> qnae::kSampleTileBits;
    Blob B;
    const size_t mass_at = B.take(sizeof(double) * T);
    const size_t pref_at = B.take(sizeof(double) * (T + 1));
    const size_t chunk_at = B.take(sizeof(double) * qnae::kSampleChunks);
    const size_t u_at = B.take(sizeof(double) * (size_t)count);
    const size_t out_at = B.take(sizeof(uint64_t) * (size_t)count);
    const size_t cost_at = B.take(sizeof(int32_t) * (size_t)count);
    HIP_TRY(ctx->s_dev.reserve(B.size));
    HIP_TRY(ctx->h_sample.reserve(B.size - u_at));
    char* d = (char*)ctx->s_dev.ptr;
    char* h = (char*)ctx->h_sample.ptr;  // mirrors the blob from u_at on
    if (count > 0) {
        std::memcpy(h, uniforms, sizeof(double) * (size_t)count);
        HIP_TRY(hipMemcpyAsync(d + u_at, h, sizeof(double) * (size_t)count, hipMemcpyHostToDevice, s));
    }
    HIP_TRY(qnae::launch_sample((const float2*)state_dev, n, cost_dev, cost_dtype, (const double*)(d + u_at), count,
                                (double*)(d + mass_at), (double*)(d + pref_at), (double*)(d + chunk_at), (uint64_t*)(d + out_at),
                                sample_costs ? (int32_t*)(d + cost_at) : nullptr, s));
    if (count > 0)
        HIP_TRY(hipMemcpyAsync(h + (out_at - u_at), d + out_at, B.size - out_at, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (count == 0) return QNAE_OK;
    const uint64_t* o = (const uint64_t*)(h + (out_at - u_at));
    if (o[0] == ~0ull) return fail(QNAE_EINVAL, "state has zero norm");
    std::memcpy(samples, o, sizeof(uint64_t) * (size_t)count);
    if (sample_costs) std::memcpy(sample_costs, h + (cost_at - u_at), sizeof(int32_t) * (size_t)count);
    return QNAE_OK;
} catch (...) {
    return host_exception();
}

}  // extern "C"
