// Reverse pass of the gradient of F = w_psucc p_succ + w_energy E[C] with
// respect to every gamma_l and beta_l.
//
// With psi_l the state after layer l, phi_l the state after its phase,
// W = diag(w_psucc [C = 0] + w_energy C) and lam_l = (U_{l+1} .. U_p)^dagger W psi_p,
// d<psi|W|psi>/dtheta = 2 Re <psi|W d psi> gives
//   dF/dbeta_l  = 2 Im <lam_l | sum_j X_j | psi_l>,
//   mu_l        = U_B(beta_l)^dagger lam_l,   phi_l = U_B(beta_l)^dagger psi_l,
//   dF/dgamma_l = 2 Im <mu_l | C | phi_l>,
//   lam_{l-1}   = U_C(gamma_l)^dagger mu_l,   psi_{l-1} = U_C(gamma_l)^dagger phi_l
// (U_B and U_C as in Section 2.1 / Section 3.2). A reverse sweep applies the
// inverse one-qubit factors to lam and psi alike, as the forward sweeps'
// butterflies (I - i t X), |t| <= 1 (two multiply-adds per amplitude and
// qubit instead of four for the exact cos/sin form). Because X_j commutes with
// every one-qubit factor, <lam|X_j|psi> is the same before and after any of
// them is applied to both states, so the X_j terms of a qubit group are summed
// inside the sweep that inverts that group. The inverse phase of the layer is
// fused in the same way as the forward phase.
#include <type_traits>

#include "tile.h"

namespace qnae {
namespace {

using namespace tile;

// State accesses: plain, or (STREAM) nontemporal, which keeps states that do not
// fit the last-level cache from displacing what does (measured: at n = 26
// and 28 the reverse sweeps 7-9% faster with it, at n = 22, where both
// states fit the cache, 4% slower).
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ float4 ld4(const float2* p) {
    if constexpr (NT) {
        const f4v v = __builtin_nontemporal_load((const f4v*)p);
        return make_float4(v.x, v.y, v.z, v.w);
    } else {
        return *(const float4*)p;
    }
}
template <bool NT>
__device__ __forceinline__ void st4(float2* p, float4 q) {
    if constexpr (NT) {
        f4v v = {q.x, q.y, q.z, q.w};
        __builtin_nontemporal_store(v, (f4v*)p);
    } else {
        *(float4*)p = q;
    }
}
template <bool NT>
__device__ __forceinline__ void st2(float2* p, float2 q) {
    if constexpr (NT) {
        f2v v = {q.x, q.y};
        __builtin_nontemporal_store(v, (f2v*)p);
    } else {
        *p = q;
    }
}

// A reverse tile is 2^13 elements of both states over 512 threads: each
// thread holds the same 16 elements of lam and of psi (the pair terms below
// need both at one place), 64 registers of state, so two workgroups (four
// waves per SIMD) share a CU without scratch. (Holding 32 elements of each
// state at two waves per SIMD spilled 17 to 64 dwords per lane, and the
// spill traffic reached HBM: 10-25% more bytes written per reverse sweep at
// n = 26.) Element e of the tile splits into a thread part (6 lane bits,
// 3 wave bits) and a slot part (4 bits) in four layouts:
//   Q0  slots e{0, 7, 8, 9},   lanes e{1..6},             waves e{10, 11, 12}
//   Q1  slots e{1, 2, 3, 4},   lanes e{0, 6, 7, 8, 5, 9}, waves e{10, 11, 12}
//   Q2  slots e{4, 5, 6, 10},  lanes e{0, 1, 2, 3, 11, 12}, waves e{7, 8, 9}
//   Q3  slots e{4, 5, 12, 11}, lanes e{0, 1, 2, 3, 10, 6},  waves e{7, 8, 9}
// Q0 is the global layout (tile bit 0 pairs in one 16-byte access); Q0 <-> Q1
// stays inside each wave's eighth of the LDS tile, Q1 / Q0 <-> Q2 go through
// the whole tile; Q2 <-> Q3 exchanges two slot bits with lane bits 4 and 5
// in registers (lane-permute swaps, no LDS). Q0 mixes e{0, 7, 8, 9}, Q1 e{1, 2,
// 3, 4} when it is used, Q2 e{5, 6, 10} (and e4 otherwise), Q3 e{11, 12};
// groups whose low run e{0..3} is not mixed skip Q1.
struct QLay {
    static constexpr int slot[4][4] = {{0, 7, 8, 9}, {1, 2, 3, 4}, {4, 5, 6, 10}, {4, 5, 12, 11}};
    static constexpr int lane[4][6] = {{1, 2, 3, 4, 5, 6}, {0, 6, 7, 8, 5, 9}, {0, 1, 2, 3, 11, 12}, {0, 1, 2, 3, 10, 6}};
    static constexpr int wave[4][3] = {{10, 11, 12}, {10, 11, 12}, {7, 8, 9}, {7, 8, 9}};
};
constexpr int kQThreads = 512;

template <int LY>
__device__ __forceinline__ uint32_t qt(uint32_t lane, uint32_t wave) {
    uint32_t e = 0u;
#pragma unroll
    for (int i = 0; i < 6; ++i) e |= ((lane >> i) & 1u) << QLay::lane[LY][i];
#pragma unroll
    for (int i = 0; i < 3; ++i) e |= ((wave >> i) & 1u) << QLay::wave[LY][i];
    return e;
}
template <int LY>
__device__ __forceinline__ constexpr uint32_t qs(int j) {
    uint32_t e = 0u;
    for (int i = 0; i < 4; ++i) e |= (uint32_t)((j >> i) & 1) << QLay::slot[LY][i];
    return e;
}

// Slot masks of the tile bits each layout mixes, for tile mask m. USE1: the
// tile passes through Q1, which mixes e{1..4}; otherwise the masks of the
// launch hold no bit of e{0..3} (a group whose low run is not mixed) and Q2
// mixes e4.
template <bool USE1>
__device__ __forceinline__ uint32_t qsm0(uint32_t m) {
    return (USE1 ? m & 1u : 0u) | ((m >> 6) & 0xeu);
}
__device__ __forceinline__ uint32_t qsm1(uint32_t m) { return (m >> 1) & 0xfu; }
template <bool USE1>
__device__ __forceinline__ uint32_t qsm2(uint32_t m) {
    return (USE1 ? 0u : (m >> 4) & 1u) | ((m >> 4) & 6u) | ((m >> 7) & 8u);
}
__device__ __forceinline__ uint32_t qsm3(uint32_t m) { return ((m >> 10) & 4u) | ((m >> 8) & 8u); }
// Slot bits each layout can mix at all (compile time): the other slot bits
// get no butterfly and no pair term.
template <bool USE1>
constexpr uint32_t kQPoss0 = USE1 ? 0xfu : 0xeu;
constexpr uint32_t kQPoss1 = 0xfu;
template <bool USE1>
constexpr uint32_t kQPoss2 = USE1 ? 0xeu : 0xfu;
constexpr uint32_t kQPoss3 = 0xcu;

// LDS positions (two padding slots per 64 elements, as for the forward
// tiles): 16 consecutive lanes of Q1 and Q2 hit 16 distinct 8-byte bank
// pairs, 8 consecutive lanes of Q0's 16-byte accesses 8 distinct 16-byte
// groups.
template <int LY>
__device__ __forceinline__ void to_q(float2* lds, const float2 (&v)[16], uint32_t lane, uint32_t wave) {
    float2* const b = lds + phys(qt<LY>(lane, wave));
    if (LY == 0) {
#pragma unroll
        for (int jj = 0; jj < 8; ++jj)
            *(float4*)(b + phys(qs<0>(2 * jj))) = make_float4(v[2 * jj].x, v[2 * jj].y, v[2 * jj + 1].x, v[2 * jj + 1].y);
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) b[phys(qs<LY>(j))] = v[j];
    }
}
template <int LY>
__device__ __forceinline__ void from_q(const float2* lds, float2 (&v)[16], uint32_t lane, uint32_t wave) {
    const float2* const b = lds + phys(qt<LY>(lane, wave));
    if (LY == 0) {
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const float4 q = *(const float4*)(b + phys(qs<0>(2 * jj)));
            v[2 * jj] = make_float2(q.x, q.y);
            v[2 * jj + 1] = make_float2(q.z, q.w);
        }
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = b[phys(qs<LY>(j))];
    }
}

// Both states from layout FROM to layout TO through one LDS buffer. Q0 and
// Q1 keep a wave's elements in the wave's own eighth of the buffer, so a
// transpose between them needs no workgroup barrier; one from or to Q2 does,
// and one whose writes from Q2 reach every eighth first waits for the reads
// of the previous transpose into Q2.
template <int FROM, int TO>
__device__ __forceinline__ void q_xpose(float2* lds, float2 (&l)[16], float2 (&p)[16], uint32_t lane, uint32_t wave) {
    constexpr bool CROSS = FROM == 2 || TO == 2;
    auto sync = [] {
        if (CROSS) __syncthreads();
        else wave_lds_sync();
    };
    if (FROM == 2) __syncthreads();
    to_q<FROM>(lds, l, lane, wave);
    sync();
    from_q<TO>(lds, l, lane, wave);
    sync();
    to_q<FROM>(lds, p, lane, wave);
    sync();
    from_q<TO>(lds, p, lane, wave);
}

// Q2 <-> Q3: slot bit 3 (e10) trades places with lane bit 4 (e11) and slot
// bit 2 (e6) with lane bit 5 (e12). A 16-lane permute swap of registers
// (A, B) leaves rows (A0, B0, A2, B2) in A and (A1, B1, A3, B3) in B, which
// exchanges "which register" with lane bit 4; the 32-lane swap does the same
// with lane bit 5. Each is its own inverse.
__device__ __forceinline__ void swap_rows16(float& a, float& b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap_rows32(float& a, float& b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void q_swap23(float2 (&v)[16]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        swap_rows16(v[j].x, v[j | 8].x);
        swap_rows16(v[j].y, v[j | 8].y);
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j & 4) continue;
        swap_rows32(v[j].x, v[j | 4].x);
        swap_rows32(v[j].y, v[j | 4].y);
    }
}

// Im of sum over pairs on register bit S of conj(l_a) p_b + conj(l_b) p_a,
// i.e. the pairs' share of Im <l|X|p> for that bit.
template <int S>
__device__ __forceinline__ float ipair(const float2 (&l)[16], const float2 (&p)[16]) {
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j & (1 << S)) continue;
        const float2 la = l[j], lb = l[j | (1 << S)], pa = p[j], pb = p[j | (1 << S)];
        acc = fmaf(la.x, pb.y, acc);
        acc = fmaf(-la.y, pb.x, acc);
        acc = fmaf(lb.x, pa.y, acc);
        acc = fmaf(-lb.y, pa.x, acc);
    }
    return acc;
}

// One qubit of an inverse mixer on both states. The butterflies leave out a
// factor f per qubit, so after k of them both states are 1/f^k of the exact
// ones and the pair term is |f|^-2k of the exact term: w = |f|^2k restores it.
template <int S>
__device__ __forceinline__ void adj_bit(float2 (&l)[16], float2 (&p)[16], float t, float r, float& w, float& acc,
                                        bool on) {
    acc = fmaf(on ? w : 0.f, ipair<S>(l, p), acc);
    w *= r;
    bfly<16, S>(l, t);
    bfly<16, S>(p, t);
}

// The slot bits in POSS as straight-line code: a bit the group does not mix
// takes t = 0 (an exact identity), weight 0 and r = 1, so no branch splits
// the register arrays.
template <int S>
__device__ __forceinline__ void adj_bit_sel(float2 (&l)[16], float2 (&p)[16], uint32_t sm, float t, float r, float& w,
                                            float& acc) {
    const bool on = (sm >> S) & 1u;
    adj_bit<S>(l, p, on ? t : 0.f, on ? r : 1.f, w, acc, on);
}
template <uint32_t POSS>
__device__ __forceinline__ void adj_mix(float2 (&l)[16], float2 (&p)[16], uint32_t sm, float t, float r, float& w,
                                        float& acc) {
    if constexpr ((POSS & 1u) != 0u) adj_bit_sel<0>(l, p, sm, t, r, w, acc);
    if constexpr ((POSS & 2u) != 0u) adj_bit_sel<1>(l, p, sm, t, r, w, acc);
    if constexpr ((POSS & 4u) != 0u) adj_bit_sel<2>(l, p, sm, t, r, w, acc);
    if constexpr ((POSS & 8u) != 0u) adj_bit_sel<3>(l, p, sm, t, r, w, acc);
    // The pair sums are complete here: sunk below the next transpose or the
    // stores, they would hold the values from before the butterflies.
    asm volatile("" : "+v"(acc));
}

// One group's inverse mixing from layout Q0 to Q3 (pre) or from Q3 to Q0
// (post), with the group's pair terms. USE1 is chosen per launch: a branch
// around the transposes here raises the register demand from about 120 to
// 160.
template <bool USE1>
__device__ __forceinline__ void q_mix_down(float2* lds, float2 (&l)[16], float2 (&p)[16], uint32_t m, float t, float r,
                                           float& w, float& acc, uint32_t lane, uint32_t wave) {
    adj_mix<kQPoss0<USE1>>(l, p, qsm0<USE1>(m), t, r, w, acc);
    if constexpr (USE1) {
        q_xpose<0, 1>(lds, l, p, lane, wave);
        adj_mix<kQPoss1>(l, p, qsm1(m), t, r, w, acc);
        q_xpose<1, 2>(lds, l, p, lane, wave);
    } else {
        q_xpose<0, 2>(lds, l, p, lane, wave);
    }
    adj_mix<kQPoss2<USE1>>(l, p, qsm2<USE1>(m), t, r, w, acc);
    q_swap23(l);
    q_swap23(p);
    adj_mix<kQPoss3>(l, p, qsm3(m), t, r, w, acc);
}
template <bool USE1>
__device__ __forceinline__ void q_mix_up(float2* lds, float2 (&l)[16], float2 (&p)[16], uint32_t m, float t, float r,
                                         float& w, float& acc, uint32_t lane, uint32_t wave) {
    adj_mix<kQPoss3>(l, p, qsm3(m), t, r, w, acc);
    q_swap23(l);
    q_swap23(p);
    adj_mix<kQPoss2<USE1>>(l, p, qsm2<USE1>(m), t, r, w, acc);
    if constexpr (USE1) {
        q_xpose<2, 1>(lds, l, p, lane, wave);
        adj_mix<kQPoss1>(l, p, qsm1(m), t, r, w, acc);
        q_xpose<1, 0>(lds, l, p, lane, wave);
    } else {
        q_xpose<2, 0>(lds, l, p, lane, wave);
    }
    adj_mix<kQPoss0<USE1>>(l, p, qsm0<USE1>(m), t, r, w, acc);
}

// WEIGH (first sweep of the reverse pass, natural order): lam is not read but
// formed as W psi from the loaded psi and cost, which saves a pass over both
// states.
template <typename CT, int KIND, bool WEIGH, bool STREAM, bool USE1>
__global__ __launch_bounds__(kQThreads) __attribute__((amdgpu_waves_per_eu(4))) void adjoint_kernel(
    const AdjointArgs a) {
    constexpr int TB = kAdjointTileBits;
    static_assert(TB == 13, "the reverse tile layouts cover 13 tile bits");
    constexpr int NWV = kQThreads / 64;
    constexpr bool PHASE = KIND == AK_BOUNDARY || KIND == AK_END;
    constexpr bool POST = KIND == AK_BOUNDARY;
    constexpr bool LUT_LDS = sizeof(CT) == 1;
    constexpr int PK = 4 / (int)sizeof(CT);
    constexpr int NC = PHASE ? 16 / PK : 1;
    __shared__ __align__(16) float2 lds[lds_elems<TB>()];
    __shared__ float2 lut_s[PHASE && LUT_LDS ? 256 : 1];
    __shared__ double red[3][NWV];

    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t t = blockIdx.x;
    const uint32_t ntiles = 1u << a.nw;
    uint64_t bitval[TB];
#pragma unroll
    for (int i = 0; i < TB; ++i) bitval[i] = 1ull << a.pos[i];
    auto scat = [&](uint32_t e) -> uint64_t {
        uint64_t x = 0;
#pragma unroll
        for (int i = 0; i < TB; ++i)
            if ((e >> i) & 1u) x |= bitval[i];
        return x;
    };
    // Tiles dealt to the 8 XCDs round-robin in chunks of 16 consecutive tiles
    // (a bijection: ntiles is a power of two), so the XCDs work on
    // neighbouring chunks at once.
    constexpr uint32_t kChunk = 16;
    uint64_t w = ntiles >= 8 * kChunk
        ? (uint64_t)((t >> 3) / kChunk) * (8 * kChunk) + (uint64_t)(t & 7u) * kChunk + ((t >> 3) % kChunk)
        : ntiles >= 8 ? (uint64_t)(t & 7u) * (ntiles >> 3) + (t >> 3) : (uint64_t)t;
    uint64_t base = 0;
    for (uint64_t m = a.wmask; m != 0ull; m &= m - 1ull) {
        if (w & 1ull) base |= m & (~m + 1ull);
        w >>= 1;
    }

    // Element x of lam sits at x ^ flip in psi (relabelled by an odd number
    // of cotangent forms since psi was restored), and the phase reads
    // cost[x ^ a.cost_flip]. The tile's thread part t and slot part s of an
    // element have disjoint bits, so (t | s) ^ (2^n - 1) = (t ^ (2^n - 1)) - s.
    const uint64_t all = (1ull << a.n) - 1ull;
    uint32_t cvp[NC];
    if (PHASE) {
        const uint64_t ct = base + scat(qt<3>(lane, wave));
        const bool cf = a.cost_flip != 0ull;
        const CT* const c3 = (const CT*)a.cost + (cf ? ct ^ all : ct);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            uint32_t wv = 0u;
#pragma unroll
            for (int q = 0; q < PK; ++q) {
                const uint64_t d = scat(qs<3>(PK * i + q));
                wv |= (uint32_t)(cf ? c3[-(int64_t)d] : c3[d]) << (8 * sizeof(CT) * q);
            }
            cvp[i] = wv;
        }
        // Pack the cost bytes as soon as they arrive (the state loads issued
        // after them stay in flight) instead of holding one register per byte
        // until the phase step.
#pragma unroll
        for (int i = 0; i < NC; ++i) asm volatile("" : "+v"(cvp[i]));
        if (LUT_LDS)
            for (int i = threadIdx.x; i < a.lut_len; i += kQThreads) lut_s[i] = a.lut[i];
    }
    const uint32_t lut_last = (uint32_t)a.lut_len - 1u;
    auto lut = [&](uint32_t cidx) -> float2 { return LUT_LDS ? lut_s[cidx] : a.lut[min(cidx, lut_last)]; };
    auto cval = [&](int j) -> uint32_t {
        return (cvp[j / PK] >> (8 * sizeof(CT) * (j % PK))) & (sizeof(CT) == 1 ? 0xffu : 0xffffu);
    };

    // Layout Q0 pairs tile bit 0 (global bit 0) in one float4: flipped, the
    // pair (x, x + 1) sits at (x ^ (2^n - 1) ^ 1, its successor) in reverse
    // order.
    const bool pf = a.psi_flip != 0;
    float2 l[16], p[16];
    {
        const uint64_t o0 = base + scat(qt<0>(lane, wave));
        const float2* const pb = a.psi + (pf ? o0 ^ all ^ 1ull : o0);
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const uint64_t d = scat(qs<0>(2 * jj));
            const float4 qp = ld4<STREAM>(pf ? pb - d : pb + d);
            p[2 * jj] = pf ? make_float2(qp.z, qp.w) : make_float2(qp.x, qp.y);
            p[2 * jj + 1] = pf ? make_float2(qp.x, qp.y) : make_float2(qp.z, qp.w);
            if (WEIGH) {
                // lam = W psi: the pair's two costs are adjacent (tile bit 0)
                using PT = typename std::conditional<sizeof(CT) == 1, uint16_t, uint32_t>::type;
                constexpr uint32_t CB = 8 * sizeof(CT);
                const PT cc = *(const PT*)((const CT*)a.cost + o0 + d);
                const uint32_t c0 = (uint32_t)cc & ((1u << CB) - 1u), c1 = (uint32_t)cc >> CB;
                const float w0 = fmaf(a.w_energy, (float)c0, c0 == 0u ? a.w_psucc : 0.f);
                const float w1 = fmaf(a.w_energy, (float)c1, c1 == 0u ? a.w_psucc : 0.f);
                l[2 * jj] = make_float2(w0 * p[2 * jj].x, w0 * p[2 * jj].y);
                l[2 * jj + 1] = make_float2(w1 * p[2 * jj + 1].x, w1 * p[2 * jj + 1].y);
            } else {
                const float4 ql = ld4<STREAM>(a.lam + o0 + d);
                l[2 * jj] = make_float2(ql.x, ql.y);
                l[2 * jj + 1] = make_float2(ql.z, ql.w);
            }
        }
    }
    float acc_pre = 0.f, acc_g = 0.f, acc_post = 0.f;
    {
        float wt = a.pre_w;
        q_mix_down<USE1>(lds, l, p, a.pre_mask, a.pre_t, a.pre_r, wt, acc_pre, lane, wave);
        asm volatile("" : "+v"(acc_pre));
    }
    if (PHASE) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const uint32_t c = cval(j);
            const float im = fmaf(l[j].x, p[j].y, -l[j].y * p[j].x);
            acc_g = fmaf((float)c, im, acc_g);
            const float2 e = lut(c);
            l[j] = cmul(l[j], e);
            p[j] = cmul(p[j], e);
        }
        asm volatile("" : "+v"(acc_g));
    }
    // No memory access moves across this point: left to itself the compiler
    // interleaves the phase step's table reads with the inverse mixing below,
    // which raises the register demand. It orders nothing that another thread
    // depends on.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (POST) {
        float wt = a.post_w;
        q_mix_up<USE1>(lds, l, p, a.post_mask, a.post_t, a.post_r, wt, acc_post, lane, wave);
        // The pair sums are complete before the stores: left to itself the
        // compiler sinks them below the stores and holds the states' values
        // from before the last butterflies across them (40 spilled registers).
        asm volatile("" : "+v"(acc_post));
        const uint64_t o0 = base + scat(qt<0>(lane, wave));
        float2* const pb = a.psi + (pf ? o0 ^ all ^ 1ull : o0);
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const uint64_t d = scat(qs<0>(2 * jj));
            st4<STREAM>(a.lam + o0 + d, make_float4(l[2 * jj].x, l[2 * jj].y, l[2 * jj + 1].x, l[2 * jj + 1].y));
        }
        if (a.store_psi) {
            if (pf) {
#pragma unroll
                for (int jj = 0; jj < 8; ++jj)
                    st4<STREAM>(pb - scat(qs<0>(2 * jj)),
                                make_float4(p[2 * jj + 1].x, p[2 * jj + 1].y, p[2 * jj].x, p[2 * jj].y));
            } else {
#pragma unroll
                for (int jj = 0; jj < 8; ++jj)
                    st4<STREAM>(pb + scat(qs<0>(2 * jj)),
                                make_float4(p[2 * jj].x, p[2 * jj].y, p[2 * jj + 1].x, p[2 * jj + 1].y));
            }
        }
    } else {
        const uint64_t o3 = base + scat(qt<3>(lane, wave));
#pragma unroll
        for (int j = 0; j < 16; ++j) st2<STREAM>(a.lam + o3 + scat(qs<3>(j)), l[j]);
        if (a.store_psi) {
            float2* const pb = a.psi + (pf ? o3 ^ all : o3);
            if (pf) {
#pragma unroll
                for (int j = 0; j < 16; ++j) st2<STREAM>(pb - scat(qs<3>(j)), p[j]);
            } else {
#pragma unroll
                for (int j = 0; j < 16; ++j) st2<STREAM>(pb + scat(qs<3>(j)), p[j]);
            }
        }
    }
    double d0 = acc_pre, d1 = acc_g, d2 = acc_post;
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
        double sum = 0.0;
        for (int q = 0; q < NWV; ++q) sum += red[threadIdx.x][q];
        a.partials[3 * (size_t)t + threadIdx.x] = sum;
    }
}

// ---------------------------------------------------------------------------
// Whole gradient for n <= 13 in one workgroup.
// ---------------------------------------------------------------------------

// 1024 threads: the two resident states fill 128 KiB of a CU's LDS, so no
// second workgroup fits and the workgroup's own waves (four per SIMD) hide
// the LDS latency.
constexpr int kResidentGradThreads = 1024;

// Pairs (x, x | 2^j) of bit j over the resident states: first Im<l|X_j|p>
// (when l != null) then a' = c a - i s b on every state given.
__device__ __forceinline__ float resident_bit(float2* l, float2* p, uint32_t N, int j, float c, float s) {
    float acc = 0.f;
    const uint32_t bit = 1u << j;
    for (uint32_t task = threadIdx.x; task < N / 2; task += kResidentGradThreads) {
        const uint32_t x = ((task >> j) << (j + 1)) | (task & (bit - 1u));
        const uint32_t y = x | bit;
        const float2 pa = p[x], pb = p[y];
        if (l) {
            const float2 la = l[x], lb = l[y];
            acc = fmaf(la.x, pb.y, acc);
            acc = fmaf(-la.y, pb.x, acc);
            acc = fmaf(lb.x, pa.y, acc);
            acc = fmaf(-lb.y, pa.x, acc);
            l[x] = make_float2(fmaf(c, la.x, s * lb.y), fmaf(c, la.y, -s * lb.x));
            l[y] = make_float2(fmaf(c, lb.x, s * la.y), fmaf(c, lb.y, -s * la.x));
        }
        p[x] = make_float2(fmaf(c, pa.x, s * pb.y), fmaf(c, pa.y, -s * pb.x));
        p[y] = make_float2(fmaf(c, pb.x, s * pa.y), fmaf(c, pb.y, -s * pa.x));
    }
    __syncthreads();
    return acc;
}

// Sum over the workgroup: wave sums, then the wave totals in wave order.
__device__ __forceinline__ double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63u) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double sum = 0.0;
    for (int w = 0; w < kResidentGradThreads / 64; ++w) sum += red[w];
    return sum;
}

template <typename CT>
__device__ __forceinline__ void resident_grad_body(const ResidentGradArgs& a) {
    __shared__ float2 ls[1 << 13];
    __shared__ float2 ps[1 << 13];
    __shared__ double red[kResidentGradThreads / 64];
    constexpr uint32_t NT = kResidentGradThreads;
    const int n = a.n;
    const uint32_t N = 1u << n;
    const uint32_t tid = threadIdx.x;
    const CT* cost = (const CT*)a.cost;
    const uint32_t last = (uint32_t)a.lut_len - 1u;
    const float amp = __builtin_ldexpf(1.0f, -n) == 0.f ? 0.f : sqrtf(__builtin_ldexpf(1.0f, -n));
    // forward
    for (int l = 0; l < a.p; ++l) {
        const float2* lut = a.luts + (size_t)l * a.lut_len;
        for (uint32_t x = tid; x < N; x += NT) {
            const float2 e = lut[min((uint32_t)cost[x], last)];
            ps[x] = l == 0 ? make_float2(amp * e.x, amp * e.y) : cmul(ps[x], e);
        }
        __syncthreads();
        const float2 cs = a.cs[l];
        for (int j = 0; j < n; ++j) resident_bit(nullptr, ps, N, j, cs.x, cs.y);
        if ((l + 1) % a.every == 0 && l + 1 < a.p) {
            float2* ck = a.ckpt + (size_t)((l + 1) / a.every - 1) * N;
            for (uint32_t x = tid; x < N; x += NT) ck[x] = ps[x];
        }
    }
    if (a.p == 0)
        for (uint32_t x = tid; x < N; x += NT) ps[x] = make_float2(amp, 0.f);
    __syncthreads();
    // readout and lam = W psi
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (uint32_t x = tid; x < N; x += NT) {
        const float2 v = ps[x];
        const uint32_t c = cost[x];
        const float pr = fmaf(v.x, v.x, v.y * v.y);
        s2 += pr;
        s1 += (double)c * pr;
        s0 += c == 0u ? pr : 0.0;
        const float w = (float)a.w_energy * (float)c + (c == 0u ? (float)a.w_psucc : 0.f);
        ls[x] = make_float2(w * v.x, w * v.y);
    }
    s0 = block_sum(s0, red);
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    if (tid == 0) {
        a.out[0] = s0;
        a.out[1] = s1;
        a.out[2] = s2;
    }
    __syncthreads();
    // reverse
    for (int l = a.p - 1; l >= 0; --l) {
        const float2 cs = a.cs[l];
        float accb = 0.f;
        for (int j = 0; j < n; ++j) accb += resident_bit(ls, ps, N, j, cs.x, -cs.y);
        const float2* lut = a.luts + (size_t)l * a.lut_len;
        float accg = 0.f;
        for (uint32_t x = tid; x < N; x += NT) {
            const uint32_t c = cost[x];
            const float2 lv = ls[x], pv = ps[x];
            accg = fmaf((float)c, fmaf(lv.x, pv.y, -lv.y * pv.x), accg);
            const float2 e = lut[min(c, last)];
            const float2 ec = make_float2(e.x, -e.y);
            ls[x] = cmul(lv, ec);
            ps[x] = cmul(pv, ec);
        }
        const double db = block_sum((double)accb, red);
        const double dg = block_sum((double)accg, red);
        if (tid == 0) {
            a.out[3 + l] = 2.0 * dg;
            a.out[3 + a.p + l] = 2.0 * db;
        }
        if (l % a.every == 0 && l > 0) {
            const float2* ck = a.ckpt + (size_t)(l / a.every - 1) * N;
            for (uint32_t x = tid; x < N; x += NT) ps[x] = ck[x];
        }
        __syncthreads();
    }
}

template <typename CT>
__global__ __launch_bounds__(kResidentGradThreads) void resident_grad_kernel(const ResidentGradArgs a) {
    resident_grad_body<CT>(a);
}

// Many small gradients, one workgroup each.
template <typename CT>
__global__ __launch_bounds__(kResidentGradThreads) void resident_grad_batch_kernel(const ResidentGradArgs* args) {
    const ResidentGradArgs a = args[blockIdx.x];
    resident_grad_body<CT>(a);
}

template <typename CT, bool NT, bool USE1>
hipError_t launch_adjoint_q(int kind, const AdjointArgs& a, hipStream_t s, bool weigh) {
    const dim3 grid(1u << a.nw), block(kQThreads);
    if (weigh) {
        if (kind != AK_MIDDLE || a.psi_flip || a.cost_flip) return hipErrorInvalidValue;
        hipLaunchKernelGGL((adjoint_kernel<CT, AK_MIDDLE, true, NT, USE1>), grid, block, 0, s, a);
        return hipGetLastError();
    }
    switch (kind) {
        case AK_MIDDLE: hipLaunchKernelGGL((adjoint_kernel<CT, AK_MIDDLE, false, NT, USE1>), grid, block, 0, s, a); break;
        case AK_BOUNDARY:
            hipLaunchKernelGGL((adjoint_kernel<CT, AK_BOUNDARY, false, NT, USE1>), grid, block, 0, s, a);
            break;
        case AK_END: hipLaunchKernelGGL((adjoint_kernel<CT, AK_END, false, NT, USE1>), grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// A launch passes through layout Q1 when a mask it mixes has a bit of the low
// run e{0..3} (the first group's tiles).
template <typename CT, bool NT>
hipError_t launch_adjoint_ct(int kind, const AdjointArgs& a, hipStream_t s, bool weigh) {
    const uint32_t masks = a.pre_mask | (kind == AK_BOUNDARY ? a.post_mask : 0u);
    return (masks & 0xfu) != 0u ? launch_adjoint_q<CT, NT, true>(kind, a, s, weigh)
                                : launch_adjoint_q<CT, NT, false>(kind, a, s, weigh);
}

}  // namespace

// Nontemporal state accesses once the two states (16 B per amplitude) exceed
// the 256 MiB last-level cache.
hipError_t launch_adjoint(int dtype, int kind, const AdjointArgs& a, hipStream_t s, bool weigh) {
    const bool nt = a.n >= 24;
    if (dtype == 1)
        return nt ? launch_adjoint_ct<uint8_t, true>(kind, a, s, weigh)
                  : launch_adjoint_ct<uint8_t, false>(kind, a, s, weigh);
    return nt ? launch_adjoint_ct<uint16_t, true>(kind, a, s, weigh)
              : launch_adjoint_ct<uint16_t, false>(kind, a, s, weigh);
}

hipError_t launch_resident_grad_batch(int dtype, const ResidentGradArgs* args, int count, hipStream_t s) {
    if (dtype == 1)
        hipLaunchKernelGGL(resident_grad_batch_kernel<uint8_t>, dim3((uint32_t)count), dim3(kResidentGradThreads), 0, s,
                           args);
    else
        hipLaunchKernelGGL(resident_grad_batch_kernel<uint16_t>, dim3((uint32_t)count), dim3(kResidentGradThreads), 0, s,
                           args);
    return hipGetLastError();
}

hipError_t launch_resident_grad(int dtype, const ResidentGradArgs& a, hipStream_t s) {
    if (dtype == 1)
        hipLaunchKernelGGL(resident_grad_kernel<uint8_t>, dim3(1), dim3(kResidentGradThreads), 0, s, a);
    else
        hipLaunchKernelGGL(resident_grad_kernel<uint16_t>, dim3(1), dim3(kResidentGradThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace qnae
