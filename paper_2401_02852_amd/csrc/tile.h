// Device helpers shared by the sweep and adjoint kernels: complex product,
// register butterflies, the three register layouts of a tile and the LDS
// transposes between them. See sweep.hip for the tiling scheme.
#pragma once

#include "internal.h"

namespace qnae {
namespace tile {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// Butterfly on register bit S of a register array of size NE:
// own' = own - i t partner for both members of each pair.
template <int NE, int S>
__device__ __forceinline__ void bfly(float2 (&v)[NE], float t) {
#pragma unroll
    for (int j = 0; j < NE; ++j) {
        if (j & (1 << S)) continue;
        const float2 a = v[j], b = v[j | (1 << S)];
        v[j] = make_float2(fmaf(t, b.y, a.x), fmaf(-t, b.x, a.y));
        v[j | (1 << S)] = make_float2(fmaf(t, a.y, b.x), fmaf(-t, a.x, b.y));
    }
}

// Butterflies on the register bits set in sm. UNCOND: all five run, with
// t = 0 (an exact identity) on the bits not in sm; straight-line code lets the
// compiler rename registers instead of copying each butterfly's results back
// for the next conditional block, which measured faster where most bits mix.
template <bool UNCOND = false>
__device__ __forceinline__ void mix32(float2 (&v)[32], uint32_t sm, float t) {
    if (UNCOND) {
        bfly<32, 0>(v, (sm & 1u) ? t : 0.f);
        bfly<32, 1>(v, (sm & 2u) ? t : 0.f);
        bfly<32, 2>(v, (sm & 4u) ? t : 0.f);
        bfly<32, 3>(v, (sm & 8u) ? t : 0.f);
        bfly<32, 4>(v, (sm & 16u) ? t : 0.f);
        return;
    }
    if (sm & 1u) bfly<32, 0>(v, t);
    if (sm & 2u) bfly<32, 1>(v, t);
    if (sm & 4u) bfly<32, 2>(v, t);
    if (sm & 8u) bfly<32, 3>(v, t);
    if (sm & 16u) bfly<32, 4>(v, t);
}

// Bit positions of layout L2 (tile bits held by slots, lanes and waves). For
// TB <= 13 the slots also hold tile bits 4 and 5, so a group whose low tile
// bits are an unmixed run of 4 (a high-qubit tile) mixes everything in L0 and
// L2 and skips L1.
template <int TB>
struct L2Map;
template <>
struct L2Map<14> {
    static constexpr int slot[5] = {6, 11, 12, 13, 7};
    static constexpr int lane[6] = {0, 1, 2, 3, 4, 5};
    static constexpr int wave[3] = {8, 9, 10};
};
template <>
struct L2Map<13> {
    static constexpr int slot[5] = {6, 11, 12, 4, 5};
    static constexpr int lane[6] = {0, 1, 2, 3, 7, 8};
    static constexpr int wave[2] = {9, 10};
};
template <>
struct L2Map<12> {
    static constexpr int slot[5] = {6, 11, 4, 5, 7};
    static constexpr int lane[6] = {0, 1, 2, 3, 8, 9};
    static constexpr int wave[1] = {10};
};

// Tile-local element index of register slot j in each layout, split into a
// thread part and a slot part with disjoint bits (e = t | s).
//   L0  slots = e{0, 7, 8, 9, 10}, lanes = e{1..6},  waves = e{11..}
//   L1  slots = e{1..5},           lanes = e{0, 6..10}, waves = e{11..}
//   L2  see L2Map
// Round ownership: L0 mixes tile bits {0, 7..10}; L1 mixes {1..5}; L2 mixes
// {6, 11..}, and also {4, 5} when L1 has nothing else to do (TB <= 13).
template <int TB>
struct Lay {
    static constexpr int WB = TB - 11;  // wave bits
    using M = L2Map<TB>;
    static constexpr bool L2_HAS_45 = TB <= 13;
    __device__ static __forceinline__ uint32_t t0(uint32_t lane, uint32_t wave) { return (lane << 1) | (wave << 11); }
    __device__ static __forceinline__ constexpr uint32_t s0(int j) { return (uint32_t)(j & 1) | ((uint32_t)(j >> 1) << 7); }
    __device__ static __forceinline__ uint32_t t1(uint32_t lane, uint32_t wave) {
        return (lane & 1u) | ((lane >> 1) << 6) | (wave << 11);
    }
    __device__ static __forceinline__ constexpr uint32_t s1(int j) { return (uint32_t)j << 1; }
    __device__ static __forceinline__ uint32_t t2(uint32_t lane, uint32_t wave) {
        uint32_t e = 0u;
#pragma unroll
        for (int i = 0; i < 6; ++i) e |= ((lane >> i) & 1u) << M::lane[i];
#pragma unroll
        for (int i = 0; i < WB; ++i) e |= ((wave >> i) & 1u) << M::wave[i];
        return e;
    }
    __device__ static __forceinline__ constexpr uint32_t s2(int j) {
        uint32_t e = 0u;
        for (int i = 0; i < 5; ++i) e |= (uint32_t)((j >> i) & 1) << M::slot[i];
        return e;
    }
    // Does L1 mix tile bits 4 and 5 for mask m?
    __host__ __device__ static __forceinline__ constexpr bool r1_takes_45(uint32_t m) {
        return !L2_HAS_45 || (m & 0xeu) != 0u;
    }
    // Slot masks of the tile bits each round mixes.
    __device__ static __forceinline__ uint32_t sm0(uint32_t m) { return (m & 1u) | (((m >> 7) & 15u) << 1); }
    __host__ __device__ static __forceinline__ constexpr uint32_t sm1(uint32_t m) {
        return r1_takes_45(m) ? (m >> 1) & 31u : (m >> 1) & 7u;
    }
    __device__ static __forceinline__ uint32_t sm2(uint32_t m) {
        const bool with45 = !r1_takes_45(m);
        uint32_t sm = 0u;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const int eb = M::slot[i];
            const bool own = eb == 6 || eb >= 11 || (with45 && (eb == 4 || eb == 5));
            if (own && ((m >> eb) & 1u)) sm |= 1u << i;
        }
        return sm;
    }
};

// Layouts L0 and L1 put the same tile bits (11 and up) in the wave index, so
// a transpose between them moves data only inside each wave's own quarter of
// the LDS tile. LDS operations of one wave complete in order, so such a
// transpose needs no workgroup barrier: this keeps the compiler from moving
// LDS accesses across the point (wavefront-scope fences emit no code).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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

// Plane transposes: the real parts of a tile go through LDS first, then the
// imaginary parts, so a tile needs a float per element instead of a float2
// and twice as many workgroups fit in a CU's LDS. Element e sits at float
// physf(e) = e + sum of c_i over the set bits i >= 6 of e. The coefficients
// are non-decreasing sums (so the map is one-to-one) chosen so that every
// b32 access of 32 lanes in layouts L1 and L2 and every b64 access of 32 lanes
// in layout L0 hits 32 distinct four-byte banks (rocprofv3 counted bank
// conflicts for b32 accesses of lanes 0..31 sharing a bank modulo 32, so
// that is the constraint); L0 pairs (tile bit 0) stay adjacent because bit 0
// carries no padding.
template <int TB>
struct PlanePad;
template <>
struct PlanePad<12> {
    static constexpr uint32_t c[6] = {2, 4, 16, 40, 62, 124};
};
template <>
struct PlanePad<13> {
    static constexpr uint32_t c[7] = {2, 16, 36, 72, 126, 252, 504};
};
template <>
struct PlanePad<14> {
    static constexpr uint32_t c[8] = {2, 4, 8, 16, 32, 64, 128, 256};
};
template <int TB>
__device__ __forceinline__ constexpr uint32_t physf(uint32_t e) {
    uint32_t p = e;
    for (int i = 6; i < TB; ++i) p += ((e >> i) & 1u) * PlanePad<TB>::c[i - 6];
    return p;
}
template <int TB>
constexpr uint32_t plane_elems() {
    uint32_t p = (1u << TB) - 1u;
    for (int i = 6; i < TB; ++i) p += PlanePad<TB>::c[i - 6];
    return p + 1u;
}

template <int C>
__device__ __forceinline__ float part(const float2& a) { return C == 0 ? a.x : a.y; }
template <int C>
__device__ __forceinline__ void set_part(float2& a, float x) {
    if (C == 0) a.x = x;
    else a.y = x;
}

// Component C (0 real, 1 imaginary) of the tile in layout LAYOUT to LDS.
template <int TB, int LAYOUT, int C>
__device__ __forceinline__ void to_plane(float* lds, const float2 (&v)[32], uint32_t lane, uint32_t wave) {
    using L = Lay<TB>;
    if (LAYOUT == 0) {
        float* const p = lds + physf<TB>(L::t0(lane, wave));
#pragma unroll
        for (int j = 0; j < 32; ++j) p[physf<TB>(L::s0(j))] = part<C>(v[j]);
    } else if (LAYOUT == 1) {
        float* const p = lds + physf<TB>(L::t1(lane, wave));
#pragma unroll
        for (int j = 0; j < 32; ++j) p[physf<TB>(L::s1(j))] = part<C>(v[j]);
    } else {
        float* const p = lds + physf<TB>(L::t2(lane, wave));
#pragma unroll
        for (int j = 0; j < 32; ++j) p[physf<TB>(L::s2(j))] = part<C>(v[j]);
    }
}

template <int TB, int LAYOUT, int C>
__device__ __forceinline__ void from_plane(const float* lds, float2 (&v)[32], uint32_t lane, uint32_t wave) {
    using L = Lay<TB>;
    if (LAYOUT == 0) {
        const float* const p = lds + physf<TB>(L::t0(lane, wave));
#pragma unroll
        for (int j = 0; j < 32; ++j) set_part<C>(v[j], p[physf<TB>(L::s0(j))]);
    } else if (LAYOUT == 1) {
        const float* const p = lds + physf<TB>(L::t1(lane, wave));
#pragma unroll
        for (int j = 0; j < 32; ++j) set_part<C>(v[j], p[physf<TB>(L::s1(j))]);
    } else {
        const float* const p = lds + physf<TB>(L::t2(lane, wave));
#pragma unroll
        for (int j = 0; j < 32; ++j) set_part<C>(v[j], p[physf<TB>(L::s2(j))]);
    }
}

// The tile from layout A to layout B, one plane after the other. CROSS: the
// layouts differ in the wave index, so waves exchange data (workgroup
// barriers); otherwise each wave stays inside its own quarter. The caller
// orders this against earlier LDS reads of the buffer by other waves.
template <int TB, int A, int B, bool CROSS>
__device__ __forceinline__ void relayout(float* lds, float2 (&v)[32], uint32_t lane, uint32_t wave) {
    to_plane<TB, A, 0>(lds, v, lane, wave);
    if (CROSS) __syncthreads();
    else wave_lds_sync();
    from_plane<TB, B, 0>(lds, v, lane, wave);
    if (CROSS) __syncthreads();
    else wave_lds_sync();
    to_plane<TB, A, 1>(lds, v, lane, wave);
    if (CROSS) __syncthreads();
    else wave_lds_sync();
    from_plane<TB, B, 1>(lds, v, lane, wave);
}

}  // namespace tile
}  // namespace qnae
