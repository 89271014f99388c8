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
// amplitude); see MixForm for how t, the dropped X and the scalar factor
// encode R(beta) = cos(beta) I - i sin(beta) X.
#include <type_traits>

#include "tile.h"

namespace qnae {
namespace {

using namespace tile;

// Global index of tile element e = (thread part te) | (slot part se) in a
// half-state sweep with a virtual bit: the unit tile bits deposit additively
// (fwd = base + unit bits of te), and when the virtual bit of e is set the
// index is mirrored, mir - (fwd + unit bits of se). HALF = false: plain
// additive addresses.
// Every sweep streams the state through nontemporal loads and stores: each
// amplitude is touched once per sweep, and keeping it out of the caches'
// normal replacement measured faster in every kind (with the current qubit
// groups; the cost bytes, which neighbouring tiles share in the L2, keep
// ordinary loads).
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float4 ld_state(const float2* p) {
    const f4v v = __builtin_nontemporal_load((const f4v*)p);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_state(float2* p, float4 q) {
    f4v v = {q.x, q.y, q.z, q.w};
    __builtin_nontemporal_store(v, (f4v*)p);
}
__device__ __forceinline__ void st_state(float2* p, float2 q) {
    f2v v = {q.x, q.y};
    __builtin_nontemporal_store(v, (f2v*)p);
}

struct HalfAddr {
    uint64_t fwd, mir;
    bool tp;  // virtual bit in the thread part
};

// Waves per SIMD a sweep kernel is register-allocated for. The final kind's
// plane transposes leave LDS room for 4 workgroups per CU; capping its
// registers at 3 waves per SIMD keeps most of that (the other kinds fit
// their LDS-bound occupancy without a cap).
constexpr int sweep_waves(int tb, int kind, bool half) {
    if (half) return 1;
    if (tb == 14) return kind == SK_BOUNDARY || kind == SK_FINAL ? 4 : 1;
    return kind == SK_FINAL ? 3 : 1;
}

// The tile from layout A to layout B through LDS: whole float2 elements, or
// (PLANES) one component plane after the other in half the LDS. CROSS: the
// layouts differ in the wave index (workgroup barriers); otherwise each wave
// stays inside its own quarter of the tile.
template <int TB, bool PLANES, int A, int B, bool CROSS>
__device__ __forceinline__ void move(float* lds, float2 (&v)[32], uint32_t lane, uint32_t wave) {
    if constexpr (PLANES) {
        relayout<TB, A, B, CROSS>(lds, v, lane, wave);
    } else {
        to_lds<TB, A>((float2*)lds, v, lane, wave);
        if (CROSS) __syncthreads();
        else wave_lds_sync();
        from_lds<TB, B>((const float2*)lds, v, lane, wave);
    }
}

// One workgroup's work on tile t of one sweep. Readout kinds write the three
// block sums to partial[0..2]. L1M: whether the mixing passes through layout
// L1 is decided per tile from the masks (0, ragged batches), or fixed for the
// launch (1 through L1, 2 not): a branch around the transposes raises the
// register demand (with 14-bit tiles at four waves per SIMD the boundary
// kind spilled 21 instead of 3 dwords per lane, the final kind 15 instead of
// none).
template <int TB, typename CT, int KIND, bool HALF, bool CKPT = false, int L1M = 0>
__device__ __forceinline__ void sweep_tile(const SweepArgs& a, uint32_t t, double* partial) {
    constexpr int WB = TB - 11;
    constexpr int NT = 64 << WB;
    constexpr bool INIT = KIND == SK_FIRST || KIND == SK_P0;  // start from phase table 0
    constexpr bool PRE = KIND == SK_MIDDLE || KIND == SK_BOUNDARY || KIND == SK_FINAL;
    constexpr bool PHASE = KIND == SK_BOUNDARY;
    constexpr bool POST = KIND == SK_FIRST || KIND == SK_BOUNDARY;
    constexpr bool REDUCE = KIND == SK_FINAL || KIND == SK_P0;
    // Kinds that move state one way (only stored, or only read for the
    // readout) gain from more resident workgroups: their transposes go
    // through LDS one component plane at a time.
    // (Half-state final sweeps need too many registers for that to pay.)
    constexpr bool PLANES = KIND == SK_FIRST || (KIND == SK_FINAL && !HALF) ||
                            (TB == 14 && !HALF && (KIND == SK_MIDDLE || KIND == SK_BOUNDARY));
    // Straight-line butterflies in the kinds that mix the tile once and hold
    // no readout state: measured faster there (the boundary kind measured
    // slower, and the final kind needs the registers). With 14-bit tiles the
    // boundary and final kinds, capped at 128 registers, spill less with them
    // (21 and 15 dwords instead of 38 and 36): n = 33 590 -> 561 ms, n = 24
    // 0.96 -> 0.85 ms per 10-layer run.
    constexpr bool UNCOND = KIND == SK_FIRST || KIND == SK_MIDDLE ||
                            (TB == 14 && !HALF && (KIND == SK_BOUNDARY || KIND == SK_FINAL));
    // The first sweep (no cost flip) of a group without the virtual bit reads
    // its costs in layout L0 and mixes L0, L1, L2 in that order (see below).
    // Decided the same way in half and full kernels, whose addressing agrees
    // for such groups, so both give the same rounding.
    constexpr bool NEED_COST = INIT || PHASE || REDUCE;
    constexpr bool NEED_LUT = INIT || PHASE;
    constexpr bool LUT_LDS = sizeof(CT) == 1;
    constexpr int PK = 4 / (int)sizeof(CT);  // cost values per packed register
    constexpr int NC = NEED_COST ? 32 / PK : 1;
    using L = Lay<TB>;
    __shared__ __align__(16) float lds[PLANES ? plane_elems<TB>() : 2 * lds_elems<TB>()];
    __shared__ float2 lut_s[NEED_LUT && LUT_LDS ? 256 : 1];
    __shared__ double red[3][1 << WB];

    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t ntiles = 1u << a.nw;
    // Tile bit i sits at bit pos[i] of x; the tile index fills the other
    // bits (wmask, ascending). Both maps are bit deposits, so offsets are
    // additive (XOR-linear) over disjoint bit sets of e: an address splits
    // into a per-thread offset and a per-slot offset that is the same for
    // every lane (scalar registers).
    // Half sweeps: the virtual bit contributes no unit offset (bitval 0); it
    // selects the mirrored address instead.
    // (a half sweep whose group lacks bit n-1 has vbit < 0: plain addresses)
    const bool has_v = HALF && a.vbit >= 0;
    const bool first_l0 = KIND == SK_FIRST && !has_v;
    const uint32_t vb = has_v ? (uint32_t)a.vbit : 0u;
    uint64_t bitval[TB];
#pragma unroll
    for (int i = 0; i < TB; ++i) bitval[i] = (has_v && (uint32_t)i == vb) ? 0ull : 1ull << a.pos[i];
    auto scat = [&](uint32_t e) -> uint64_t {
        uint64_t x = 0;
#pragma unroll
        for (int i = 0; i < TB; ++i)
            if ((e >> i) & 1u) x |= bitval[i];
        return x;
    };
    // Consecutive tiles go to one XCD (blocks are dealt round-robin over the
    // 8 XCDs), so tiles that share cache lines of the cost diagonal share an
    // L2: each XCD takes one contiguous eighth of the tiles, except in the
    // boundary kind, where each XCD takes every eighth chunk of 32
    // consecutive tiles, so the 8 XCDs work on neighbouring chunks at once
    // (measured faster there: 3.41 -> 3.29 ms at n = 30; slower for the
    // middle kind). The tile index is deposited into the bits outside the
    // tile (scalar ALU only).
    constexpr uint32_t kChunk = 32;
    uint64_t w = (KIND == SK_BOUNDARY && ntiles >= 8 * kChunk)
                     ? (uint64_t)((t >> 3) / kChunk) * (8 * kChunk) + (uint64_t)(t & 7u) * kChunk + ((t >> 3) % kChunk)
                 : ntiles >= 8 ? (uint64_t)(t & 7u) * (ntiles >> 3) + (t >> 3)
                               : (uint64_t)t;
    uint64_t base = 0;
    for (uint64_t m = a.wmask; m != 0ull; m &= m - 1ull) {
        if (w & 1ull) base |= m & (~m + 1ull);
        w >>= 1;
    }
    auto vpar = [&](uint32_t e) -> bool { return has_v && ((e >> vb) & 1u); };
    auto haddr = [&](uint32_t te) -> HalfAddr {
        HalfAddr h;
        h.fwd = base + scat(te);
        h.mir = a.mir - h.fwd;
        h.tp = vpar(te);
        return h;
    };
    // index of element (te | se) for a thread's HalfAddr
    auto hidx = [&](const HalfAddr& h, uint32_t se) -> uint64_t {
        const uint64_t so = scat(se);
        return (h.tp != vpar(se)) ? h.mir - so : h.fwd + so;
    };

    // Cost values of the 32 amplitudes in layout L2, loaded first; packed 4
    // (uint8) or 2 (uint16) per register. With cflip the stored state is the
    // true one with every qubit flipped (see MixForm), so cost values are read
    // at the complemented index: complemented tile base, thread part and slot.
    uint32_t cvp[NC];
    if (NEED_COST && HALF && !first_l0) {
        // symmetric cost: no complemented reads, mirrored indices instead
        const HalfAddr h = haddr(L::t2(lane, wave));
        const CT* const cp = (const CT*)a.cost;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            uint32_t wv = 0u;
#pragma unroll
            for (int q = 0; q < PK; ++q) wv |= (uint32_t)cp[hidx(h, L::s2(PK * i + q))] << (8 * sizeof(CT) * q);
            cvp[i] = wv;
        }
        if (NEED_LUT && LUT_LDS)
            for (int i = threadIdx.x; i < a.lut_len; i += NT) lut_s[i] = a.lut[i];
    } else if (NEED_COST && !first_l0) {
        const bool cf = a.cflip != 0;
        const uint64_t cbase = cf ? base ^ ((((uint64_t)1 << a.n) - 1ull) ^ a.tile_bits) : base;
        const uint32_t ct = cf ? L::t2(lane, wave) ^ L::t2(63u, (1u << WB) - 1u) : L::t2(lane, wave);
        const int cj = cf ? 31 : 0;
        const CT* const c2 = (const CT*)a.cost + cbase + scat(ct);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            uint32_t wv = 0u;
#pragma unroll
            for (int q = 0; q < PK; ++q) wv |= (uint32_t)c2[scat(L::s2((PK * i + q) ^ cj))] << (8 * sizeof(CT) * q);
            cvp[i] = wv;
        }
        // With 14-bit tiles (128 registers) the bytes are packed as they
        // arrive instead of held one per register until the phase step: the
        // boundary kind then spills nothing instead of 3-4 dwords (n = 24
        // 2.05 -> 2.10e11 amp-layer updates/s). With 13-bit tiles the same
        // slowed the boundary kind (3.16 -> 3.27 ms at n = 30).
        if constexpr (TB == 14) {
#pragma unroll
            for (int i = 0; i < NC; ++i) asm volatile("" : "+v"(cvp[i]));
        }
        if (NEED_LUT && LUT_LDS)
            for (int i = threadIdx.x; i < a.lut_len; i += NT) lut_s[i] = a.lut[i];
    }
    // Cost values above m are a caller error; the clamp keeps table reads in bounds.
    const uint32_t lut_last = (uint32_t)a.lut_len - 1u;
    auto lut = [&](uint32_t cidx) -> float2 { return LUT_LDS ? lut_s[cidx] : a.lut[min(cidx, lut_last)]; };
    auto cval = [&](int j) -> uint32_t {
        return (cvp[j / PK] >> (8 * sizeof(CT) * (j % PK))) & (sizeof(CT) == 1 ? 0xffu : 0xffffu);
    };

    if (KIND == SK_FIRST && first_l0) {
        // In layout L0 the pair of a thread's slots along tile bit 0 are
        // adjacent costs, and the 64 lanes cover tile bits 1..6, so a wave
        // reads 128 consecutive cost bytes per load (layout L2 reads four
        // runs of 16). The tile is then mixed in L0, L1, L2 and stored from
        // L2; the order of the mixings within a layer does not matter.
        using PT = typename std::conditional<sizeof(CT) == 1, uint16_t, uint32_t>::type;
        const CT* const c0 = (const CT*)a.cost + base + scat(L::t0(lane, wave));
        PT cp[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) cp[jj] = *(const PT*)(c0 + scat(L::s0(2 * jj)));
        if (LUT_LDS)
            for (int i = threadIdx.x; i < a.lut_len; i += NT) lut_s[i] = a.lut[i];
        __syncthreads();  // phase table visible
        constexpr uint32_t CB = 8 * sizeof(CT);
        float2 v[32];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            v[2 * jj] = lut((uint32_t)cp[jj] & ((1u << CB) - 1u));
            v[2 * jj + 1] = lut((uint32_t)cp[jj] >> CB);
        }
        const uint32_t m = a.post_mask;
        const float tt = a.post_t;
        mix32<UNCOND>(v, L::sm0(m), tt);
        if (L1M == 1 || (L1M == 0 && L::sm1(m))) {
            move<TB, PLANES, 0, 1, false>(lds, v, lane, wave);  // inside the wave's quarter
            mix32<UNCOND>(v, L::sm1(m), tt);
            wave_lds_sync();
            move<TB, PLANES, 1, 2, true>(lds, v, lane, wave);
        } else {
            move<TB, PLANES, 0, 2, true>(lds, v, lane, wave);
        }
        mix32<UNCOND>(v, L::sm2(m), tt);
        float2* const p2 = a.psi + base + scat(L::t2(lane, wave));
#pragma unroll
        for (int j = 0; j < 32; ++j) st_state(p2 + scat(L::s2(j)), v[j]);
        return;
    }

    float2 v[32];
    if (INIT) {
        __syncthreads();  // phase table visible
#pragma unroll
        for (int j = 0; j < 32; ++j) v[j] = lut(cval(j));
    } else if (HALF) {
        // pairs along tile bit 0 (x bit 0): a mirrored pair is stored in
        // reverse order one slot lower
        const HalfAddr h = haddr(L::t0(lane, wave));
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const uint32_t se = L::s0(2 * jj);
            const bool neg = h.tp != vpar(se);
            const uint64_t so = scat(se);
            const float4 q = ld_state(a.psi_in + (neg ? h.mir - so - 1ull : h.fwd + so));
            v[2 * jj] = neg ? make_float2(q.z, q.w) : make_float2(q.x, q.y);
            v[2 * jj + 1] = neg ? make_float2(q.x, q.y) : make_float2(q.z, q.w);
        }
    } else {
        const float2* const p0 = a.psi_in + base + scat(L::t0(lane, wave));
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const float4 q = ld_state(p0 + scat(L::s0(2 * jj)));
            v[2 * jj] = make_float2(q.x, q.y);
            v[2 * jj + 1] = make_float2(q.z, q.w);
        }
    }
    if (PRE) {
        const uint32_t m = a.pre_mask;
        const float tt = a.pre_t;
        mix32<UNCOND>(v, L::sm0(m), tt);
        if (L1M == 1 || (L1M == 0 && L::sm1(m))) {
            move<TB, PLANES, 0, 1, false>(lds, v, lane, wave);  // inside the wave's quarter
            mix32<UNCOND>(v, L::sm1(m), tt);
            wave_lds_sync();
            move<TB, PLANES, 1, 2, true>(lds, v, lane, wave);
        } else {
            move<TB, PLANES, 0, 2, true>(lds, v, lane, wave);
        }
        mix32<UNCOND>(v, L::sm2(m), tt);
    }
    if (CKPT) {
        // The tile's thread part t and slot part s have disjoint bits, so
        // (t | s) ^ (2^n - 1) = (t ^ (2^n - 1)) - s.
        const uint64_t all = (1ull << a.n) - 1ull;
        const uint64_t o2 = base + scat(L::t2(lane, wave));
        const float2 f = a.ckpt_scale;
        if (a.cflip) {
            float2* const c2 = a.ckpt + (o2 ^ all);
#pragma unroll
            for (int j = 0; j < 32; ++j) st_state(c2 - scat(L::s2(j)), cmul(v[j], f));
        } else {
            float2* const c2 = a.ckpt + o2;
#pragma unroll
            for (int j = 0; j < 32; ++j) st_state(c2 + scat(L::s2(j)), cmul(v[j], f));
        }
    }
    if (PHASE) {
#pragma unroll
        for (int j = 0; j < 32; ++j) v[j] = cmul(v[j], lut(cval(j)));
    }
    if (POST) {
        const uint32_t m = a.post_mask;
        const float tt = a.post_t;
        mix32<UNCOND>(v, L::sm2(m), tt);
        if (PRE) __syncthreads();  // every wave has read its L2 part
        if (L1M == 1 || (L1M == 0 && L::sm1(m))) {
            move<TB, PLANES, 2, 1, true>(lds, v, lane, wave);
            mix32<UNCOND>(v, L::sm1(m), tt);
            wave_lds_sync();
            move<TB, PLANES, 1, 0, false>(lds, v, lane, wave);  // inside the wave's quarter
        } else {
            move<TB, PLANES, 2, 0, true>(lds, v, lane, wave);
        }
        mix32<UNCOND>(v, L::sm0(m), tt);
        if (HALF) {
            const HalfAddr h = haddr(L::t0(lane, wave));
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                const uint32_t se = L::s0(2 * jj);
                const bool neg = h.tp != vpar(se);
                const uint64_t so = scat(se);
                const float2 lo = neg ? v[2 * jj + 1] : v[2 * jj], hi = neg ? v[2 * jj] : v[2 * jj + 1];
                st_state(a.psi + (neg ? h.mir - so - 1ull : h.fwd + so), make_float4(lo.x, lo.y, hi.x, hi.y));
            }
            return;
        }
        float2* const p0 = a.psi + base + scat(L::t0(lane, wave));
#pragma unroll
        for (int jj = 0; jj < 16; ++jj)
            st_state(p0 + scat(L::s0(2 * jj)), make_float4(v[2 * jj].x, v[2 * jj].y, v[2 * jj + 1].x, v[2 * jj + 1].y));
        return;
    }
    if (REDUCE) {
        float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const float pr = fmaf(v[j].x, v[j].x, v[j].y * v[j].y);
            const uint32_t c = cval(j);
            s2 += pr;
            s1 = fmaf((float)c, pr, s1);
            s0 += c == 0u ? pr : 0.f;
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
            double sum = 0.0;
            for (int q = 0; q < (1 << WB); ++q) sum += red[threadIdx.x][q];
            partial[threadIdx.x] = sum;
        }
    }
    if (KIND == SK_MIDDLE || (REDUCE && a.store)) {
        if (REDUCE) {
#pragma unroll
            for (int j = 0; j < 32; ++j) v[j] = cmul(v[j], a.store_scale);
        }
        if (HALF) {
            const HalfAddr h = haddr(L::t2(lane, wave));
#pragma unroll
            for (int j = 0; j < 32; ++j) st_state(a.psi + hidx(h, L::s2(j)), v[j]);
        } else {
            float2* const p2 = a.psi + base + scat(L::t2(lane, wave));
#pragma unroll
            for (int j = 0; j < 32; ++j) st_state(p2 + scat(L::s2(j)), v[j]);
        }
    }
}

// One sweep over one state: block b handles tile b.
template <int TB, typename CT, int KIND, bool HALF = false, bool CKPT = false, int L1M = 0>
__global__ __launch_bounds__(64 << (TB - 11)) __attribute__((amdgpu_waves_per_eu(sweep_waves(TB, KIND, HALF)))) void sweep_kernel(
    const SweepArgs a) {
    sweep_tile<TB, CT, KIND, HALF, CKPT, L1M>(a, blockIdx.x, a.partials + 3 * (size_t)blockIdx.x);
}

// L1M of a single-state launch: 1 when a mask the kind mixes has bits that
// only layout L1 holds, else 2.
template <int TB, int KIND>
int sweep_l1_mode(const SweepArgs& a) {
    using L = Lay<TB>;
    const bool pre = KIND == SK_MIDDLE || KIND == SK_BOUNDARY || KIND == SK_FINAL;
    const bool post = KIND == SK_FIRST || KIND == SK_BOUNDARY;
    const bool l1 = (pre && L::sm1(a.pre_mask) != 0u) || (post && L::sm1(a.post_mask) != 0u);
    return l1 ? 1 : 2;
}

// Instance of work item b in a ragged batch: the largest i with first[i] <= b.
__device__ __forceinline__ int batch_item(const uint32_t* first, int count, uint32_t b) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One sweep step over many states at once (ragged): instance i owns blocks
// first[i] .. first[i+1]-1, one per tile, with its own arguments.
template <int TB, typename CT, int KIND, bool HALF>
__global__ __launch_bounds__(64 << (TB - 11)) __attribute__((amdgpu_waves_per_eu(sweep_waves(TB, KIND, HALF)))) void sweep_batch_kernel(const SweepArgs* args, const uint32_t* first,
                                                                      int count) {
    const int i = batch_item(first, count, blockIdx.x);
    const SweepArgs a = args[i];
    const uint32_t t = blockIdx.x - first[i];
    sweep_tile<TB, CT, KIND, HALF>(a, t, a.partials + 3 * (size_t)t);
}

// psi[x] <-> psi[N - 1 - x]: undoes an X on every qubit (N >= 4).
__global__ __launch_bounds__(256) void reverse_kernel(float2* psi, uint64_t N) {
    const uint64_t i = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * 2;
    if (i >= N / 2) return;
    float4* lo = (float4*)(psi + i);
    float4* hi = (float4*)(psi + (N - 2 - i));
    const float4 a = *lo, b = *hi;
    *lo = make_float4(b.z, b.w, b.x, b.y);
    *hi = make_float4(a.z, a.w, a.x, a.y);
}

// ---------------------------------------------------------------------------
// Whole circuit in one workgroup for n <= 14 (state resident in LDS).
// ---------------------------------------------------------------------------

// LDS slot of amplitude x: one pad slot per 16, so that the threads of the
// bits-0..3 pass, each holding 16 consecutive amplitudes, fall in different
// banks instead of all in one (a stride of 16 float2 is 32 banks).
__device__ __forceinline__ uint32_t rslot(uint32_t x) { return x + (x >> 4); }

// 1024 threads: one workgroup's LDS (the 136 KiB state, uint8 costs) leaves
// room for no second one on a CU, so its own waves (four per SIMD) hide the
// LDS latency.
constexpr int kResidentThreads = 1024;

// Radix-2^NBP butterfly passes of one layer over the LDS state: each task
// holds the 2^nb amplitudes of one coset of nb consecutive qubits.
template <int NBP>
__device__ __forceinline__ void resident_mix(float2* s, int n, uint32_t N, float t) {
    for (int g0 = 0; g0 < n; g0 += NBP) {
        const int nb = n - g0 < NBP ? n - g0 : NBP;
        const uint32_t tasks = N >> nb;
        for (uint32_t task = threadIdx.x; task < tasks; task += kResidentThreads) {
            const uint32_t bs = ((task >> g0) << (g0 + nb)) | (task & ((1u << g0) - 1u));
            float2 v[1 << NBP];
#pragma unroll
            for (int i = 0; i < (1 << NBP); ++i)
                v[i] = i < (1 << nb) ? s[rslot(bs | ((uint32_t)i << g0))] : make_float2(0.f, 0.f);
            if (nb > 0) bfly<(1 << NBP), 0>(v, t);
            if (NBP > 1 && nb > 1) bfly<(1 << NBP), (NBP > 1 ? 1 : 0)>(v, t);
            if (NBP > 2 && nb > 2) bfly<(1 << NBP), (NBP > 2 ? 2 : 0)>(v, t);
            if (NBP > 3 && nb > 3) bfly<(1 << NBP), (NBP > 3 ? 3 : 0)>(v, t);
#pragma unroll
            for (int i = 0; i < (1 << NBP); ++i)
                if (i < (1 << nb)) s[rslot(bs | ((uint32_t)i << g0))] = v[i];
        }
        __syncthreads();
    }
}

// Qubits per pass: four at n = 14 (1024 cosets, one per thread), three
// below (at n = 12 and 13 measured 1-2 us faster per solve than four).
constexpr int kResidentSmallNbp = 3;

template <typename CT>
__device__ __forceinline__ void resident_body(const ResidentArgs& a) {
    constexpr uint32_t NT = kResidentThreads;
    __shared__ float2 s[(1 << 14) + (1 << 10)];
    __shared__ double red[3][NT / 64];
    // uint8 costs are read from global memory once and kept beside the state
    // (16 KiB at n = 14); uint16 ones would not fit and are read per layer.
    constexpr bool COST_LDS = sizeof(CT) == 1;
    __shared__ CT cs[COST_LDS ? 1 << 14 : 1];
    const int n = a.n;
    const uint32_t N = 1u << n;
    const uint32_t tid = threadIdx.x;
    const CT* const cost_g = (const CT*)a.cost;
    if (COST_LDS) {
        for (uint32_t x = tid; x < N; x += NT) cs[x] = cost_g[x];
        __syncthreads();
    }
    const CT* const cost = COST_LDS ? cs : cost_g;
    const uint32_t last = (uint32_t)a.lut_len - 1u;
    const int layers = a.p > 0 ? a.p : 1;
    // The butterflies drop the X of the cot form; `flip` records that the
    // stored state is the true one with every qubit flipped.
    uint32_t flip = 0u;
    for (int l = 0; l < layers; ++l) {
        const float2* lut = a.luts + (size_t)l * a.lut_len;
        for (uint32_t x = tid; x < N; x += NT) {
            const float2 e = lut[min((uint32_t)cost[x ^ flip], last)];
            s[rslot(x)] = l > 0 ? cmul(s[rslot(x)], e) : a.state_in ? cmul(a.state_in[x], e) : e;
        }
        __syncthreads();
        if (a.p == 0) break;
    const MixForm f = a.forms[l];
        if (n >= 14) resident_mix<4>(s, n, N, f.t);
        else if (n == 13) resident_mix<3>(s, n, N, f.t);
        else resident_mix<kResidentSmallNbp>(s, n, N, f.t);
        if (f.flip) flip ^= N - 1u;
    }
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
    for (uint32_t x = tid; x < N; x += NT) {
        const float2 q = s[rslot(x)];
        const float pr = fmaf(q.x, q.x, q.y * q.y);
        const uint32_t cx = cost[x ^ flip];
        s2 += pr;
        s1 = fmaf((float)cx, pr, s1);
        s0 += cx == 0u ? pr : 0.f;
        if (a.state_out) a.state_out[x ^ flip] = cmul(q, a.store_scale);
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
    if (tid < 3) {
        double sum = 0.0;
        for (uint32_t w = 0; w < NT / 64; ++w) sum += red[tid][w];
        a.out[tid] = sum;
    }
}

template <typename CT>
__global__ __launch_bounds__(kResidentThreads) void resident_kernel(const ResidentArgs a) {
    resident_body<CT>(a);
}

// Tables from the kernel arguments, staged in LDS (3.5 KiB beside the
// state and costs: 156 of the CU's 160 KiB) and read through generic
// pointers.
template <typename CT>
__global__ __launch_bounds__(kResidentThreads) void resident_inline_kernel(const ResidentInlineArgs ia) {
    __shared__ float2 tab[kResidentInline];
    const int layers = ia.a.p > 0 ? ia.a.p : 1;
    const int count = layers * ia.a.lut_len + ia.a.p;
    for (int i = threadIdx.x; i < count; i += kResidentThreads) tab[i] = ia.tab[i];
    __syncthreads();
    ResidentArgs a = ia.a;
    a.luts = tab;
    a.forms = (const MixForm*)(tab + layers * ia.a.lut_len);
    resident_body<CT>(a);
}

// Many small instances, one workgroup each.
template <typename CT>
__global__ __launch_bounds__(kResidentThreads) void resident_batch_kernel(const ResidentArgs* args) {
    const ResidentArgs a = args[blockIdx.x];
    resident_body<CT>(a);
}

__device__ __forceinline__ void final_reduce_body(const double* partials, int64_t blocks, double* out) {
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

__global__ __launch_bounds__(1024) void final_reduce_kernel(const double* partials, int64_t blocks, double* out) {
    final_reduce_body(partials, blocks, out);
}

// One workgroup per instance i: blocks[i] triples at partials[i] -> outs[i].
__global__ __launch_bounds__(1024) void final_reduce_batch_kernel(const double* const* partials, const uint32_t* blocks,
                                                                   double* const* outs) {
    final_reduce_body(partials[blockIdx.x], blocks[blockIdx.x], outs[blockIdx.x]);
}

template <int TB, typename CT, int KIND, int L1M>
void launch_kind_l1(const SweepArgs& a, hipStream_t s) {
    if (a.half && a.vbit >= 0)
        hipLaunchKernelGGL((sweep_kernel<TB, CT, KIND, true, false, L1M>), dim3(1u << a.nw), dim3(64 << (TB - 11)), 0,
                           s, a);
    else
        hipLaunchKernelGGL((sweep_kernel<TB, CT, KIND, false, false, L1M>), dim3(1u << a.nw), dim3(64 << (TB - 11)), 0,
                           s, a);
}

// The L1 choice is fixed per launch, except in the first and final kinds of
// 13-bit tiles, which measured faster with the per-tile branch at n = 30
// (1.81 and 1.62 ms against 1.93 and 1.75 ms: the first kind fits four
// workgroups per CU without the branch instead of three, and that is
// slower for this write-only kind).
template <int TB, typename CT, int KIND>
hipError_t launch_kind(const SweepArgs& a, hipStream_t s) {
    if (TB == 13 && (KIND == SK_FIRST || KIND == SK_FINAL)) launch_kind_l1<TB, CT, KIND, 0>(a, s);
    else if (KIND == SK_P0 || sweep_l1_mode<TB, KIND>(a) == 2) launch_kind_l1<TB, CT, KIND, 2>(a, s);
    else launch_kind_l1<TB, CT, KIND, 1>(a, s);
    return hipGetLastError();
}

template <int TB, typename CT, int KIND>
hipError_t launch_batch_kind(const SweepArgs* args, const uint32_t* first, int count, uint32_t blocks, bool half,
                             hipStream_t s) {
    if (half)
        hipLaunchKernelGGL((sweep_batch_kernel<TB, CT, KIND, true>), dim3(blocks), dim3(64 << (TB - 11)), 0, s, args,
                           first, count);
    else
        hipLaunchKernelGGL((sweep_batch_kernel<TB, CT, KIND, false>), dim3(blocks), dim3(64 << (TB - 11)), 0, s, args,
                           first, count);
    return hipGetLastError();
}

template <int TB, typename CT>
hipError_t launch_tb(int kind, const SweepArgs& a, hipStream_t s) {
    switch (kind) {
        case SK_FIRST: return launch_kind<TB, CT, SK_FIRST>(a, s);
        case SK_MIDDLE: return launch_kind<TB, CT, SK_MIDDLE>(a, s);
        case SK_BOUNDARY: return launch_kind<TB, CT, SK_BOUNDARY>(a, s);
        case SK_FINAL: return launch_kind<TB, CT, SK_FINAL>(a, s);
        case SK_P0: return launch_kind<TB, CT, SK_P0>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int TB, typename CT>
hipError_t launch_batch_ct(int kind, const SweepArgs* args, const uint32_t* first, int count, uint32_t blocks,
                           bool half, hipStream_t s) {
    switch (kind) {
        case SK_FIRST: return launch_batch_kind<TB, CT, SK_FIRST>(args, first, count, blocks, half, s);
        case SK_MIDDLE: return launch_batch_kind<TB, CT, SK_MIDDLE>(args, first, count, blocks, half, s);
        case SK_BOUNDARY: return launch_batch_kind<TB, CT, SK_BOUNDARY>(args, first, count, blocks, half, s);
        case SK_FINAL: return launch_batch_kind<TB, CT, SK_FINAL>(args, first, count, blocks, half, s);
        case SK_P0: return launch_batch_kind<TB, CT, SK_P0>(args, first, count, blocks, half, s);
        default: return hipErrorInvalidValue;
    }
}

template <int TB>
hipError_t launch_tb_dt(int dtype, int kind, const SweepArgs& a, hipStream_t s) {
    return dtype == 1 ? launch_tb<TB, uint8_t>(kind, a, s) : launch_tb<TB, uint16_t>(kind, a, s);
}

}  // namespace

hipError_t launch_sweep(int tb, int dtype, int kind, const SweepArgs& a, hipStream_t s) {
    switch (tb) {
        case 12: return launch_tb_dt<12>(dtype, kind, a, s);
        case 13: return launch_tb_dt<13>(dtype, kind, a, s);
        case 14: return launch_tb_dt<14>(dtype, kind, a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int TB>
hipError_t launch_batch_tb(int dtype, int kind, const SweepArgs* args, const uint32_t* first, int count,
                           uint32_t blocks, hipStream_t s, bool half) {
    return dtype == 1 ? launch_batch_ct<TB, uint8_t>(kind, args, first, count, blocks, half, s)
                      : launch_batch_ct<TB, uint16_t>(kind, args, first, count, blocks, half, s);
}

hipError_t launch_sweep_batch(int tb, int dtype, int kind, const SweepArgs* args, const uint32_t* first, int count,
                              uint32_t blocks, hipStream_t s, bool half) {
    switch (tb) {
        case 12: return launch_batch_tb<12>(dtype, kind, args, first, count, blocks, s, half);
        case 13: return launch_batch_tb<13>(dtype, kind, args, first, count, blocks, s, half);
        case 14: return launch_batch_tb<14>(dtype, kind, args, first, count, blocks, s, half);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_ckpt(int dtype, const SweepArgs& a, hipStream_t s) {
    constexpr int TB = kAdjointTileBits;
    if (a.half || !a.ckpt || a.nw < 0) return hipErrorInvalidValue;
    const dim3 grid(1u << a.nw), block(64 << (TB - 11));
    const bool l1 = sweep_l1_mode<TB, SK_BOUNDARY>(a) == 1;
    if (dtype == 1) {
        if (l1) hipLaunchKernelGGL((sweep_kernel<TB, uint8_t, SK_BOUNDARY, false, true, 1>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((sweep_kernel<TB, uint8_t, SK_BOUNDARY, false, true, 2>), grid, block, 0, s, a);
    } else {
        if (l1) hipLaunchKernelGGL((sweep_kernel<TB, uint16_t, SK_BOUNDARY, false, true, 1>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((sweep_kernel<TB, uint16_t, SK_BOUNDARY, false, true, 2>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_reverse(float2* psi, uint64_t N, hipStream_t s) {
    const uint64_t threads = N / 4;
    hipLaunchKernelGGL(reverse_kernel, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s, psi, N);
    return hipGetLastError();
}

hipError_t launch_resident(int dtype, const ResidentArgs& a, hipStream_t s) {
    if (dtype == 1)
        hipLaunchKernelGGL((resident_kernel<uint8_t>), dim3(1), dim3(kResidentThreads), 0, s, a);
    else
        hipLaunchKernelGGL((resident_kernel<uint16_t>), dim3(1), dim3(kResidentThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_resident_inline(int dtype, const ResidentInlineArgs& a, hipStream_t s) {
    const int layers = a.a.p > 0 ? a.a.p : 1;
    if ((int64_t)layers * a.a.lut_len + a.a.p > kResidentInline) return hipErrorInvalidValue;
    if (dtype == 1)
        hipLaunchKernelGGL((resident_inline_kernel<uint8_t>), dim3(1), dim3(kResidentThreads), 0, s, a);
    else
        hipLaunchKernelGGL((resident_inline_kernel<uint16_t>), dim3(1), dim3(kResidentThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_resident_batch(int dtype, const ResidentArgs* args, int count, hipStream_t s) {
    if (dtype == 1)
        hipLaunchKernelGGL((resident_batch_kernel<uint8_t>), dim3(count), dim3(kResidentThreads), 0, s, args);
    else
        hipLaunchKernelGGL((resident_batch_kernel<uint16_t>), dim3(count), dim3(kResidentThreads), 0, s, args);
    return hipGetLastError();
}

hipError_t launch_final_reduce(const double* partials, int64_t blocks, double* out, hipStream_t s) {
    hipLaunchKernelGGL(final_reduce_kernel, dim3(1), dim3(1024), 0, s, partials, blocks, out);
    return hipGetLastError();
}

hipError_t launch_final_reduce_batch(const double* const* partials, const uint32_t* blocks, double* const* outs,
                                     int count, hipStream_t s) {
    hipLaunchKernelGGL(final_reduce_batch_kernel, dim3(count), dim3(1024), 0, s, partials, blocks, outs);
    return hipGetLastError();
}

}  // namespace qnae
