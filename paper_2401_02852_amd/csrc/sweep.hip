// State sweeps: phase, mixer and readout on complex64 statevectors.
//
// The mixer U_B(beta) = prod_j exp(-i beta X_j) (Section 2.1; Appendix A.4)
// is a product of commuting one-qubit factors, so any subset of qubits can be
// applied in one pass. A sweep moves the state through the chip once: every
// workgroup owns a tile of 2^TB amplitudes whose indices vary on tile bits
// [0, c) and [H, H + TB - c) of x, keeps it in registers and LDS, applies the
// phase table (the diagonal exp(-i gamma C(x)), Section 3.2) and the selected
// qubit butterflies, and writes it back. The low run of 2^c amplitudes keeps
// global accesses in contiguous segments of at least 128 bytes.
//
// Inside a tile each thread holds 32 amplitudes. Three register layouts put
// different tile bits into the 5 "slot" bits of the register index, and LDS
// transposes switch between them:
//   L0  slots = e{0, 7, 8, 9, 10}, lanes = e{1..6}   (16-byte global accesses)
//   L1  slots = e{1..5},           lanes = e{0, 6..10}
//   L2  slots = e{6, 11.., 7..},   lanes = e{0..5}   (phase, readout)
// Round r mixes the tile bits it owns while they sit in slots: L0 owns
// {0, 7..10}, L1 owns {1..5}, L2 owns {6, 11 .. TB-1}.
//
// The butterfly on a pair (a, b) is own' = own - i t partner (two FMAs per
// amplitude); see MixForm for how t, the optional X and the scalar factor
// encode R(beta) = cos(beta) I - i sin(beta) X.
#include "internal.h"

namespace qnae {
namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// Butterfly on register bit S of a register array of size NE.
template <int NE, int S, bool SWAP>
__device__ __forceinline__ void bfly(float2 (&v)[NE], float t) {
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        if (j & (1 << S)) continue;
        const float2 a = v[j], b = v[j | (1 << S)];
        const float2 na = make_float2(fmaf(t, b.y, a.x), fmaf(-t, b.x, a.y));
        const float2 nb = make_float2(fmaf(t, a.y, b.x), fmaf(-t, a.x, b.y));
        if (SWAP) {
            v[j] = nb;
            v[j | (1 << S)] = na;
        } else {
            v[j] = na;
            v[j | (1 << S)] = nb;
        }
    }
}

template <bool SWAP>
__device__ __forceinline__ void mix_slots32(float2 (&v)[32], uint32_t sm, float t) {
    if (sm & 1u) bfly<32, 0, SWAP>(v, t);
    if (sm & 2u) bfly<32, 1, SWAP>(v, t);
    if (sm & 4u) bfly<32, 2, SWAP>(v, t);
    if (sm & 8u) bfly<32, 3, SWAP>(v, t);
    if (sm & 16u) bfly<32, 4, SWAP>(v, t);
}

__device__ __forceinline__ void mix32(float2 (&v)[32], uint32_t sm, const MixForm f) {
    if (sm == 0u) return;
    if (f.swap) mix_slots32<true>(v, sm, f.t);
    else mix_slots32<false>(v, sm, f.t);
}

// Tile-local element index of register slot j in each layout.
template <int TB>
struct Lay {
    static constexpr int WB = TB - 11;  // wave bits
    __device__ static __forceinline__ uint32_t e0(uint32_t lane, uint32_t wave, int j) {
        return (uint32_t)(j & 1) | (lane << 1) | ((uint32_t)(j >> 1) << 7) | (wave << 11);
    }
    __device__ static __forceinline__ uint32_t e1(uint32_t lane, uint32_t wave, int j) {
        return (lane & 1u) | ((uint32_t)j << 1) | ((lane >> 1) << 6) | (wave << 11);
    }
    __device__ static __forceinline__ uint32_t e2(uint32_t lane, uint32_t wave, int j) {
        return lane | ((uint32_t)(j & 1) << 6) | ((uint32_t)((j >> 1) & ((1 << WB) - 1)) << 11) |
               ((uint32_t)(j >> (1 + WB)) << 7) | (wave << (11 - WB));
    }
    // Thread and slot parts of e0 / e2 (disjoint bit sets, so e = t | s).
    __device__ static __forceinline__ uint32_t t0(uint32_t lane, uint32_t wave) { return (lane << 1) | (wave << 11); }
    __device__ static __forceinline__ constexpr uint32_t s0(int j) { return (uint32_t)(j & 1) | ((uint32_t)(j >> 1) << 7); }
    __device__ static __forceinline__ uint32_t t1(uint32_t lane, uint32_t wave) { return (lane & 1u) | ((lane >> 1) << 6) | (wave << 11); }
    __device__ static __forceinline__ constexpr uint32_t s1(int j) { return (uint32_t)j << 1; }
    __device__ static __forceinline__ uint32_t t2(uint32_t lane, uint32_t wave) { return lane | (wave << (11 - WB)); }
    __device__ static __forceinline__ constexpr uint32_t s2(int j) {
        return ((uint32_t)(j & 1) << 6) | ((uint32_t)((j >> 1) & ((1 << WB) - 1)) << 11) | ((uint32_t)(j >> (1 + WB)) << 7);
    }
    // Slot masks of the tile bits each round owns.
    __device__ static __forceinline__ uint32_t sm0(uint32_t m) {
        return (m & 1u) | (((m >> 7) & 15u) << 1);
    }
    __device__ static __forceinline__ uint32_t sm1(uint32_t m) { return (m >> 1) & 31u; }
    __device__ static __forceinline__ uint32_t sm2(uint32_t m) {
        return ((m >> 6) & 1u) | (((m >> 11) & ((1u << WB) - 1u)) << 1);
    }
};

// LDS position of tile element e: two padding slots after every 64 elements.
// Any 16 consecutive lanes then hit 16 distinct 8-byte bank pairs in all three
// layouts, and because the map is additive over disjoint bit sets of e, an
// address is a per-thread base plus a compile-time constant per slot.
__device__ __forceinline__ constexpr uint32_t phys(uint32_t e) { return e + 2u * (e >> 6); }
template <int TB>
constexpr uint32_t lds_elems() { return phys((1u << TB) - 1u) + 1u; }

template <int TB, int LAYOUT>
__device__ __forceinline__ void to_lds(float2* lds, const float2 (&v)[32], uint32_t lane, uint32_t wave) {
    using L = Lay<TB>;
    if (LAYOUT == 0) {
        float2* const p = lds + phys(L::t0(lane, wave));
#pragma unroll
        for (int jj = 0; jj < 16; ++jj)
            *(float4*)(p + phys(L::s0(2 * jj))) = make_float4(v[2 * jj].x, v[2 * jj].y, v[2 * jj + 1].x, v[2 * jj + 1].y);
    } else if (LAYOUT == 1) {
        float2* const p = lds + phys(L::t1(lane, wave));
#pragma unroll
        for (int j = 0; j < 32; ++j) p[phys(L::s1(j))] = v[j];
    } else {
        float2* const p = lds + phys(L::t2(lane, wave));
#pragma unroll
        for (int j = 0; j < 32; ++j) p[phys(L::s2(j))] = v[j];
    }
}

template <int TB, int LAYOUT>
__device__ __forceinline__ void from_lds(const float2* lds, float2 (&v)[32], uint32_t lane, uint32_t wave) {
    using L = Lay<TB>;
    if (LAYOUT == 0) {
        const float2* const p = lds + phys(L::t0(lane, wave));
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const float4 q = *(const float4*)(p + phys(L::s0(2 * jj)));
            v[2 * jj] = make_float2(q.x, q.y);
            v[2 * jj + 1] = make_float2(q.z, q.w);
        }
    } else if (LAYOUT == 1) {
        const float2* const p = lds + phys(L::t1(lane, wave));
#pragma unroll
        for (int j = 0; j < 32; ++j) v[j] = p[phys(L::s1(j))];
    } else {
        const float2* const p = lds + phys(L::t2(lane, wave));
#pragma unroll
        for (int j = 0; j < 32; ++j) v[j] = p[phys(L::s2(j))];
    }
}

template <int TB, typename CT>
__global__ __launch_bounds__(64 << (TB - 11)) void sweep_kernel(const SweepArgs a) {
    constexpr int WB = TB - 11;
    constexpr int NT = 64 << WB;
    using L = Lay<TB>;
    __shared__ float2 lds[lds_elems<TB>()];
    __shared__ float2 lut_s[256];
    __shared__ double red[3][1 << WB];

    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t G = gridDim.x, b = blockIdx.x;
    const uint64_t w = a.xcd_remap ? (uint64_t)(b & 7u) * (G >> 3) + (b >> 3) : (uint64_t)b;
    const int c = a.c, H = a.H;
    const uint64_t base = ((w & ((1ull << (H - c)) - 1ull)) << c) | ((w >> (H - c)) << (H + TB - c));
    const uint32_t lowmask = (1u << c) - 1u;
    // Global offset of tile element e. It is additive over disjoint bit sets
    // of e, so an address splits into a per-thread pointer and a per-slot
    // offset that is the same for every lane (scalar registers).
    auto scat = [&](uint32_t e) -> uint64_t { return (uint64_t)(e & lowmask) | ((uint64_t)(e >> c) << H); };
    float2* const p0 = a.psi + base + scat(L::t0(lane, wave));
    float2* const p2 = a.psi + base + scat(L::t2(lane, wave));

    const int flags = a.flags;
    const bool need_cost = (flags & (SW_INIT | SW_PHASE | SW_REDUCE)) != 0;
    const CT* cost = (const CT*)a.cost;
    constexpr bool LUT_LDS = sizeof(CT) == 1;

    // Cost values of the 32 amplitudes in layout L2, loaded early.
    // Packed: 4 (uint8) or 2 (uint16) cost values per register.
    constexpr int PK = 4 / (int)sizeof(CT);
    uint32_t cvp[32 / PK];
    const CT* const c2 = cost + base + scat(L::t2(lane, wave));
    if (need_cost) {
#pragma unroll
        for (int i = 0; i < 32 / PK; ++i) {
            uint32_t wv = 0u;
#pragma unroll
            for (int q = 0; q < PK; ++q) wv |= (uint32_t)c2[scat(L::s2(PK * i + q))] << (8 * sizeof(CT) * q);
            cvp[i] = wv;
        }
        if (LUT_LDS && (flags & (SW_INIT | SW_PHASE)))
            for (int i = threadIdx.x; i < a.lut_len; i += NT) lut_s[i] = a.lut[i];
    }
    // Cost values above m are a caller error; the clamp keeps table reads in bounds.
    const uint32_t lut_last = (uint32_t)a.lut_len - 1u;
    auto lut = [&](uint32_t cidx) -> float2 { return LUT_LDS ? lut_s[cidx] : a.lut[min(cidx, lut_last)]; };
    auto cval = [&](int j) -> uint32_t {
        return (cvp[j / PK] >> (8 * sizeof(CT) * (j % PK))) & (sizeof(CT) == 1 ? 0xffu : 0xffffu);
    };

    float2 v[32];
    if (flags & SW_INIT) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 32; ++j) v[j] = lut(cval(j));
    } else {
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const float4 q = *(const float4*)(p0 + scat(L::s0(2 * jj)));
            v[2 * jj] = make_float2(q.x, q.y);
            v[2 * jj + 1] = make_float2(q.z, q.w);
        }
        const uint32_t m = a.pre_mask;
        mix32(v, L::sm0(m), a.pre);
        if (L::sm1(m)) {
            to_lds<TB, 0>(lds, v, lane, wave);
            __syncthreads();
            from_lds<TB, 1>(lds, v, lane, wave);
            mix32(v, L::sm1(m), a.pre);
            __syncthreads();
            to_lds<TB, 1>(lds, v, lane, wave);
        } else {
            to_lds<TB, 0>(lds, v, lane, wave);
        }
        __syncthreads();
        from_lds<TB, 2>(lds, v, lane, wave);
        mix32(v, L::sm2(m), a.pre);
        if (flags & SW_PHASE) {
#pragma unroll
            for (int j = 0; j < 32; ++j) v[j] = cmul(v[j], lut(cval(j)));
        }
    }

    if (a.post_mask) {
        const uint32_t m = a.post_mask;
        mix32(v, L::sm2(m), a.post);
        __syncthreads();
        to_lds<TB, 2>(lds, v, lane, wave);
        __syncthreads();
        if (L::sm1(m)) {
            from_lds<TB, 1>(lds, v, lane, wave);
            mix32(v, L::sm1(m), a.post);
            __syncthreads();
            to_lds<TB, 1>(lds, v, lane, wave);
            __syncthreads();
        }
        from_lds<TB, 0>(lds, v, lane, wave);
        mix32(v, L::sm0(m), a.post);
        if (flags & SW_SCALE) {
#pragma unroll
            for (int j = 0; j < 32; ++j) v[j] = cmul(v[j], a.store_scale);
        }
#pragma unroll
        for (int jj = 0; jj < 16; ++jj)
            *(float4*)(p0 + scat(L::s0(2 * jj))) =
                make_float4(v[2 * jj].x, v[2 * jj].y, v[2 * jj + 1].x, v[2 * jj + 1].y);
        return;
    }

    if (flags & SW_REDUCE) {
        float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const float pr = fmaf(v[j].x, v[j].x, v[j].y * v[j].y);
            s2 += pr;
            const uint32_t cj = cval(j);
            s1 = fmaf((float)cj, pr, s1);
            s0 += cj == 0u ? pr : 0.f;
        }
        double d0 = s0, d1 = s1, d2 = s2;
        for (int off = 32; off > 0; off >>= 1) {
            d0 += __shfl_xor(d0, off);
            d1 += __shfl_xor(d1, off);
            d2 += __shfl_xor(d2, off);
        }
        if (lane == 0) {
            red[0][wave] = d0;
            red[1][wave] = d1;
            red[2][wave] = d2;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            double t = 0.0;
            for (int q = 0; q < (1 << WB); ++q) t += red[threadIdx.x][q];
            a.partials[(size_t)b * 3 + threadIdx.x] = t;
        }
    }
    if (flags & SW_STORE) {
        if (flags & SW_SCALE) {
#pragma unroll
            for (int j = 0; j < 32; ++j) v[j] = cmul(v[j], a.store_scale);
        }
#pragma unroll
        for (int j = 0; j < 32; ++j) p2[scat(L::s2(j))] = v[j];
    }
}

// ---------------------------------------------------------------------------
// Whole circuit in one workgroup for n <= 14 (state resident in LDS).
// ---------------------------------------------------------------------------

template <bool SWAP>
__device__ __forceinline__ void mix16(float2 (&v)[16], int nb, float t) {
    if (nb > 0) bfly<16, 0, SWAP>(v, t);
    if (nb > 1) bfly<16, 1, SWAP>(v, t);
    if (nb > 2) bfly<16, 2, SWAP>(v, t);
    if (nb > 3) bfly<16, 3, SWAP>(v, t);
}

template <typename CT>
__global__ __launch_bounds__(256) void resident_kernel(const ResidentArgs a) {
    __shared__ float2 s[1 << 14];
    __shared__ double red[3][4];
    const int n = a.n;
    const uint32_t N = 1u << n;
    const uint32_t tid = threadIdx.x;
    const CT* cost = (const CT*)a.cost;
    const int layers = a.p > 0 ? a.p : 1;
    for (int l = 0; l < layers; ++l) {
        const float2* lut = a.luts + (size_t)l * a.lut_len;
        for (uint32_t x = tid; x < N; x += 256) {
            const float2 e = lut[min((uint32_t)cost[x], (uint32_t)a.lut_len - 1u)];
            s[x] = l == 0 ? e : cmul(s[x], e);
        }
        __syncthreads();
        if (a.p == 0) break;
        const MixForm f = a.forms[l];
        for (int g0 = 0; g0 < n; g0 += 4) {
            const int nb = n - g0 < 4 ? n - g0 : 4;
            const uint32_t tasks = N >> nb;
            for (uint32_t task = tid; task < tasks; task += 256) {
                const uint32_t bs = ((task >> g0) << (g0 + nb)) | (task & ((1u << g0) - 1u));
                float2 v[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) v[i] = i < (1 << nb) ? s[bs | ((uint32_t)i << g0)] : make_float2(0.f, 0.f);
                if (f.swap) mix16<true>(v, nb, f.t);
                else mix16<false>(v, nb, f.t);
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    if (i < (1 << nb)) s[bs | ((uint32_t)i << g0)] = v[i];
            }
            __syncthreads();
        }
    }
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
    for (uint32_t x = tid; x < N; x += 256) {
        const float2 q = s[x];
        const float pr = fmaf(q.x, q.x, q.y * q.y);
        const uint32_t cx = cost[x];
        s2 += pr;
        s1 = fmaf((float)cx, pr, s1);
        s0 += cx == 0u ? pr : 0.f;
        if (a.state_out) a.state_out[x] = cmul(q, a.store_scale);
    }
    double d0 = s0, d1 = s1, d2 = s2;
    for (int off = 32; off > 0; off >>= 1) {
        d0 += __shfl_xor(d0, off);
        d1 += __shfl_xor(d1, off);
        d2 += __shfl_xor(d2, off);
    }
    if ((tid & 63u) == 0) {
        red[0][tid >> 6] = d0;
        red[1][tid >> 6] = d1;
        red[2][tid >> 6] = d2;
    }
    __syncthreads();
    if (tid < 3) a.out[tid] = red[tid][0] + red[tid][1] + red[tid][2] + red[tid][3];
}

__global__ __launch_bounds__(1024) void final_reduce_kernel(const double* partials, int64_t blocks, double* out) {
    __shared__ double red[3][16];
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int64_t i = threadIdx.x; i < blocks; i += 1024) {
        t0 += partials[3 * i];
        t1 += partials[3 * i + 1];
        t2 += partials[3 * i + 2];
    }
    for (int off = 32; off > 0; off >>= 1) {
        t0 += __shfl_xor(t0, off);
        t1 += __shfl_xor(t1, off);
        t2 += __shfl_xor(t2, off);
    }
    if ((threadIdx.x & 63u) == 0) {
        red[0][threadIdx.x >> 6] = t0;
        red[1][threadIdx.x >> 6] = t1;
        red[2][threadIdx.x >> 6] = t2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int q = 0; q < 16; ++q) t += red[threadIdx.x][q];
        out[threadIdx.x] = t;
    }
}

template <int TB>
hipError_t launch_tb(int dtype, const SweepArgs& a, hipStream_t s) {
    const uint32_t blocks = 1u << (a.n - TB);
    if (dtype == 1)
        hipLaunchKernelGGL((sweep_kernel<TB, uint8_t>), dim3(blocks), dim3(64 << (TB - 11)), 0, s, a);
    else
        hipLaunchKernelGGL((sweep_kernel<TB, uint16_t>), dim3(blocks), dim3(64 << (TB - 11)), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep(int tb, int dtype, const SweepArgs& a, hipStream_t s) {
    switch (tb) {
        case 12: return launch_tb<12>(dtype, a, s);
        case 13: return launch_tb<13>(dtype, a, s);
        case 14: return launch_tb<14>(dtype, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_resident(int dtype, const ResidentArgs& a, hipStream_t s) {
    if (dtype == 1)
        hipLaunchKernelGGL((resident_kernel<uint8_t>), dim3(1), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((resident_kernel<uint16_t>), dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_final_reduce(const double* partials, int64_t blocks, double* out, hipStream_t s) {
    hipLaunchKernelGGL(final_reduce_kernel, dim3(1), dim3(1024), 0, s, partials, blocks, out);
    return hipGetLastError();
}

}  // namespace qnae
