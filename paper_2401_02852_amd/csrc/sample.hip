// Sampling bitstrings from a state (include/qnae.h, qnae_sample).
//
// Measuring the final QAOA state yields x with probability |psi(x)|^2 / norm;
// the instance running time of Section 4.2 counts such draws until one
// satisfies the instance. A draw inverts the cumulative distribution in index
// order: the outcome for a uniform u is the smallest x whose cumulative mass
// exceeds u times the total. The cumulative distribution is never stored per
// amplitude; it is kept at three levels of prefix sums from zero:
//   chunk level  C[i]: sequential sums of chunk masses (one thread);
//   tile level   P[t] = C[i] + (sequential sum of the tile masses before t in
//                its chunk), tiles of 4096 consecutive amplitudes;
//   inside a tile: per-thread sums of 16 consecutive probabilities, their
//                block-wide exclusive scan, then a walk over the 16.
// The first two are nondecreasing by construction (sequential sums of
// nonnegative terms, and FP64 addition of a fixed offset is monotone). The
// in-tile scan is a shuffle tree whose rounding may differ from a sequential
// sum, so a draw takes the highest thread with mass whose start is at or below
// its remainder and, if rounding carries the remainder past that thread's
// walk, the thread's last nonzero probability. A draw finds its tile by binary
// search over P, then its thread, then its amplitude. Probabilities are FP32
// |psi|^2, sums FP64.
#include "internal.h"

namespace qnae {
namespace {

constexpr int kTile = 1 << kSampleTileBits;  // amplitudes per tile
constexpr int kPer = kTile / 256;            // per thread, consecutive

// LDS slot of probability e: one pad slot per 16 so that threads reading
// their 16 consecutive entries fall in different banks.
__device__ __forceinline__ uint32_t pad(uint32_t e) { return e + (e >> 4); }

struct TileScan {
    double mine;   // this thread's 16 probabilities summed in order
    double excl;   // sum of the lower threads' sums (block-wide exclusive scan)
    double total;  // sum of the four wave totals in wave order
};

// Stages the probabilities of tile `tile` (amplitudes tile*4096 ..) in LDS and
// scans the per-thread sums. 256 threads.
__device__ TileScan tile_scan(const float2* __restrict__ psi, uint64_t N, uint64_t tile, float* prob,
                              double* wsum) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint64_t base = tile * (uint64_t)kTile;
    constexpr int kLoads = kTile / 512;
    // float4s (amplitude pairs) of this tile inside the state: 2048 for every
    // tile when N >= 4096, else N / 2 >= 1 (N is even). Indices past it load
    // the last pair in range and read as zero, so all loads are unconditional
    // and in flight together.
    const uint32_t lim = (uint32_t)min<uint64_t>(N - base, (uint64_t)kTile) / 2u;
    const float4* tp = (const float4*)(psi + base);  // uniform base, 32-bit offsets
    float4 q[kLoads];
#pragma unroll
    for (int i = 0; i < kLoads; ++i) {
        const uint32_t j = tid + 256u * i;
        q[i] = tp[j < lim ? j : lim - 1u];
        if (j >= lim) q[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < kLoads; ++i) {
        const uint32_t e = 2u * tid + 512u * i;
        prob[pad(e)] = fmaf(q[i].x, q[i].x, q[i].y * q[i].y);
        prob[pad(e + 1)] = fmaf(q[i].z, q[i].z, q[i].w * q[i].w);
    }
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) s += (double)prob[pad(kPer * tid + j)];
    double incl = s;
    for (int off = 1; off < 64; off <<= 1) {
        const double t = __shfl_up(incl, off);
        if (lane >= (uint32_t)off) incl += t;
    }
    const double prev = __shfl_up(incl, 1);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    double woff = 0.0;
    for (uint32_t w = 0; w < wave; ++w) woff += wsum[w];
    TileScan r;
    r.mine = s;
    r.excl = woff + (lane ? prev : 0.0);
    r.total = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
    return r;
}

__global__ __launch_bounds__(256) void tile_mass_kernel(const float2* __restrict__ psi, uint64_t N,
                                                         double* __restrict__ mass) {
    __shared__ float prob[kTile + kTile / 16];
    __shared__ double wsum[4];
    const TileScan r = tile_scan(psi, N, blockIdx.x, prob, wsum);
    if (threadIdx.x == 0) mass[blockIdx.x] = r.total;
}

// The tile level in three launches. Thread i of the first owns tiles
// [i*chunk, (i+1)*chunk) of the kSampleChunks chunks and writes their prefix
// within the chunk, from zero, and the chunk total. T and chunk are powers of
// two, so a chunk of 16 or more splits into whole runs of 16 tiles: their
// loads are issued together, then summed in tile order. The threads spread
// over 16 workgroups, as each load instruction touches 64 chunks' lines.
constexpr int kRun = 16;

__global__ __launch_bounds__(64) void chunk_run_kernel(const double* __restrict__ mass, double* __restrict__ pref,
                                                       double* __restrict__ chunk_total, uint32_t T, uint32_t chunk) {
    const uint32_t i = blockIdx.x * 64u + threadIdx.x;
    const uint32_t lo = min(T, i * chunk), hi = min(T, lo + chunk);
    double run = 0.0;
    uint32_t t = lo;
    for (; t + kRun <= hi; t += kRun) {
        double v[kRun];
#pragma unroll
        for (int j = 0; j < kRun; ++j) v[j] = mass[t + j];
#pragma unroll
        for (int j = 0; j < kRun; ++j) {
            const double mj = v[j];
            v[j] = run;
            run += mj;
        }
#pragma unroll
        for (int j = 0; j < kRun; ++j) pref[t + j] = v[j];
    }
    for (; t < hi; ++t) {
        pref[t] = run;
        run += mass[t];
    }
    chunk_total[i] = run;
}

// The chunk level: C[0] = 0 and C[i+1] = C[i] + total[i] in chunk order, in
// place over the totals, for the `used` = T / chunk chunks that hold tiles
// (the others hold none and add nothing), and P[T] = C[used]. One wave stages
// the totals in LDS; one thread adds them in order.
__global__ __launch_bounds__(64) void chunk_offset_kernel(double* __restrict__ chunk_total, double* __restrict__ pref,
                                                          uint32_t T, uint32_t used) {
    __shared__ double c[kSampleChunks];
    const uint32_t lane = threadIdx.x;
#pragma unroll
    for (int j = 0; j < kSampleChunks / 64; ++j) c[lane + 64u * j] = chunk_total[lane + 64u * j];
    __syncthreads();
    if (lane == 0) {
        double acc = 0.0;
        uint32_t q = 0;
        for (; q + kRun <= used; q += kRun) {
            double v[kRun];
#pragma unroll
            for (int j = 0; j < kRun; ++j) v[j] = c[q + j];
#pragma unroll
            for (int j = 0; j < kRun; ++j) {
                const double tj = v[j];
                v[j] = acc;
                acc += tj;
            }
#pragma unroll
            for (int j = 0; j < kRun; ++j) c[q + j] = v[j];
        }
        for (; q < used; ++q) {
            const double tq = c[q];
            c[q] = acc;
            acc += tq;
        }
        pref[T] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSampleChunks / 64; ++j) chunk_total[lane + 64u * j] = c[lane + 64u * j];
}

// P[t] = C[t / chunk] + (prefix within the chunk), one tile per thread.
__global__ __launch_bounds__(256) void chunk_add_kernel(double* __restrict__ pref, const double* __restrict__ C,
                                                        uint32_t T, uint32_t chunk_bits) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    if (t < T) pref[t] = C[t >> chunk_bits] + pref[t];
}

// One workgroup per draw.
template <typename CT>
__global__ __launch_bounds__(256) void sample_kernel(const float2* __restrict__ psi, uint64_t N,
                                                     const double* __restrict__ mass, const double* __restrict__ pref,
                                                     uint32_t T, const double* __restrict__ uniforms,
                                                     const CT* __restrict__ cost, uint64_t* __restrict__ out,
                                                     int32_t* __restrict__ out_cost) {
    __shared__ float prob[kTile + kTile / 16];
    __shared__ double wsum[4];
    __shared__ uint32_t s_tile;
    __shared__ double s_r;
    __shared__ uint32_t s_best[4];
    const uint32_t q = blockIdx.x, tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const double total = pref[T];
    if (!(total > 0.0)) {  // zero state: reported to the host as an error
        if (tid == 0) out[q] = ~0ull;
        return;
    }
    if (tid == 0) {
        const double target = uniforms[q] * total;
        uint32_t lo = 0, hi = T - 1;  // largest t with P[t] <= target (P[0] = 0)
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo + 1) / 2;
            if (pref[mid] <= target) lo = mid;
            else hi = mid - 1;
        }
        while (lo > 0 && !(mass[lo] > 0.0)) --lo;  // only past the last nonzero tile
        s_tile = lo;
        s_r = target - pref[lo];
    }
    __syncthreads();
    const uint32_t tile = s_tile;
    const double r = s_r;
    const TileScan sc = tile_scan(psi, N, tile, prob, wsum);
    // the highest thread with mass whose range starts at or below r
    const bool ok = sc.mine > 0.0 && sc.excl <= r;
    const uint64_t bal = __ballot(ok);
    if (lane == 0) s_best[wave] = bal ? (wave << 6) + 63u - (uint32_t)__builtin_clzll(bal) : 0xffffffffu;
    __syncthreads();
    uint32_t best = 0xffffffffu;
    for (int w = 3; w >= 0; --w)
        if (s_best[w] != 0xffffffffu) {
            best = s_best[w];
            break;
        }
    if (tid != best) return;
    double acc = sc.excl;
    int pick = -1, last = -1;
    for (int j = 0; j < kPer; ++j) {
        const float p = prob[pad(kPer * tid + j)];
        acc += (double)p;
        if (p > 0.f) {
            last = j;
            if (acc > r) {
                pick = j;
                break;
            }
        }
    }
    if (pick < 0) pick = last;  // rounding put r past this thread's walk
    const uint64_t x = (uint64_t)tile * kTile + (uint64_t)kPer * tid + (uint64_t)pick;
    out[q] = x;
    if (out_cost) out_cost[q] = cost ? (int32_t)cost[x] : -1;
}

}  // namespace

hipError_t launch_sample(const float2* psi, int n, const void* cost, int cost_dtype, const double* uniforms,
                         int count, double* mass, double* pref, double* chunk_scratch, uint64_t* out, int32_t* out_cost,
                         hipStream_t s) {
    const uint64_t N = 1ull << n;
    const uint32_t T = (uint32_t)((N + kTile - 1) / kTile);
    hipLaunchKernelGGL(tile_mass_kernel, dim3(T), dim3(256), 0, s, psi, N, mass);
    if (hipError_t e = hipGetLastError()) return e;
    static_assert(kSampleChunks % 64 == 0 && kSampleChunks % kRun == 0, "chunk launch shape");
    const uint32_t chunk = (T + kSampleChunks - 1) / kSampleChunks;  // T is a power of two
    const uint32_t chunk_bits = (uint32_t)__builtin_ctz(chunk);
    hipLaunchKernelGGL(chunk_run_kernel, dim3(kSampleChunks / 64), dim3(64), 0, s, mass, pref, chunk_scratch, T,
                       chunk);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(chunk_offset_kernel, dim3(1), dim3(64), 0, s, chunk_scratch, pref, T, T / chunk);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(chunk_add_kernel, dim3((T + 255) / 256), dim3(256), 0, s, pref,
                       (const double*)chunk_scratch, T, chunk_bits);
    if (hipError_t e = hipGetLastError()) return e;
    if (count == 0) return hipSuccess;
    if (cost_dtype == 2)
        hipLaunchKernelGGL(sample_kernel<uint16_t>, dim3((uint32_t)count), dim3(256), 0, s, psi, N, mass, pref, T,
                           uniforms, (const uint16_t*)cost, out, out_cost);
    else
        hipLaunchKernelGGL(sample_kernel<uint8_t>, dim3((uint32_t)count), dim3(256), 0, s, psi, N, mass, pref, T,
                           uniforms, (const uint8_t*)cost, out, out_cost);
    return hipGetLastError();
}

}  // namespace qnae
