// Cost diagonal kernel: C(x) = number of NAE-violated clauses, for every basis
// state x (Section 3.2, eq. knaesatobj; Appendix A.2, eq. demorgannae).
//
// Bit-sliced: each thread owns an aligned run of 32 consecutive states. For one
// clause, its violation pattern over the run is a 32-bit word: the part of the
// clause on variables >= 5 is constant over the run (one compare against the
// thread's index), and the part on variables 0..4 is a per-clause table built
// on the host. The per-state counters are kept as NP bit-planes (a vertical
// counter); clauses go in eight at a time through a carry-save adder tree, so
// one clause costs about 9 integer operations per 32 states (clauses on
// variables >= 5 only are constant over the run and are counted as one
// integer instead). At the end the planes are transposed into bytes (uint8)
// or half-words (uint16) and written with 16-byte stores.
#include "internal.h"

namespace qnae {
namespace {

// Thread `tid` of one diagonal: states [32 tid, 32 tid + 32).
template <int NP, bool WIDE, bool U16>
__device__ __forceinline__ void cost_chunk(const CostArgs& a, uint64_t tid) {
    const uint64_t nthreads = a.n >= 5 ? (1ull << (a.n - 5)) : 1ull;
    uint32_t zeros = 0;
    if (tid < nthreads) {
        const uint64_t xbase = tid << 5;
        const uint32_t xlo = (uint32_t)xbase, xhi = (uint32_t)(xbase >> 32);
        uint32_t plane[NP];
#pragma unroll
        for (int b = 0; b < NP; ++b) plane[b] = 0u;
        // Violation word of clause i over the 32 states.
        auto viol = [&](int i) -> uint32_t {
            const ClauseRec r = a.clauses[i];
            const uint32_t hlo = (xlo ^ r.pat_lo) & r.mask_hi_lo;
            bool none, all;
            if (WIDE) {
                const uint32_t hhi = (xhi ^ r.pat_hi) & r.mask_hi_hi;
                none = (hlo | hhi) == 0u;
                all = (hlo == r.mask_hi_lo) && (hhi == r.mask_hi_hi);
            } else {
                none = hlo == 0u;
                all = hlo == r.mask_hi_lo;
            }
            return (none ? r.zero_tab : 0u) | (all ? r.full_tab : 0u);
        };
        // Adds carry * 2^b0 to the counter (ripple through the planes above).
        auto add_at = [&](int b0, uint32_t carry) {
#pragma unroll
            for (int b = 0; b < NP; ++b) {
                if (b < b0) continue;
                const uint32_t t = plane[b] & carry;
                plane[b] ^= carry;
                carry = t;
            }
        };
        // Full adder per bit: x + p + q = x' + 2 carry.
        auto csa = [](uint32_t& x, uint32_t p, uint32_t q) -> uint32_t {
            const uint32_t t = x ^ p;
            const uint32_t carry = (t & q) | (~t & x);
            x = t ^ q;
            return carry;
        };
        // Eight clauses at a time through a carry-save tree (7 full adders
        // into the planes of weight 1, 2 and 4, one ripple from weight 8):
        // the counter value after the block is exactly the sum it had plus
        // the eight violation bits, per state.
        int i = 0;
        for (; i + 8 <= a.num_low; i += 8) {
            const uint32_t c2a = csa(plane[0], viol(i), viol(i + 1));
            const uint32_t c2b = csa(plane[0], viol(i + 2), viol(i + 3));
            const uint32_t c2c = csa(plane[0], viol(i + 4), viol(i + 5));
            const uint32_t c2d = csa(plane[0], viol(i + 6), viol(i + 7));
            const uint32_t c4a = csa(plane[1], c2a, c2b);
            const uint32_t c4b = csa(plane[1], c2c, c2d);
            add_at(3, csa(plane[2], c4a, c4b));
        }
        for (; i < a.num_low; ++i) add_at(0, viol(i));
        // The other clauses only have variables >= 5: each is violated on all
        // 32 states of the run or on none, so they are counted as one integer
        // (about 5 operations per clause instead of 9) and the count is added
        // to every state's counter once, as a ripple-carry over the planes.
        uint32_t cnt = 0u;
        for (; i < a.num_clauses; ++i) cnt += viol(i) & 1u;
        uint32_t carry = 0u;
#pragma unroll
        for (int b = 0; b < NP; ++b) {
            const uint32_t cb = 0u - ((cnt >> b) & 1u);
            const uint32_t t = plane[b] ^ cb;
            const uint32_t nc = (plane[b] & cb) | (t & carry);
            plane[b] = t ^ carry;
            carry = nc;
        }
        const uint32_t valid = a.n >= 5 ? 0xffffffffu : ((1u << (1u << a.n)) - 1u);
        uint32_t any = 0u;
#pragma unroll
        for (int b = 0; b < NP; ++b) any |= plane[b];
        zeros = (uint32_t)__popc(~any & valid);

        if (!U16) {
            // 32 bytes: byte j = sum_b bit j of plane b, shifted to bit b.
            uint32_t word[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                uint32_t wv = 0u;
#pragma unroll
                for (int b = 0; b < NP; ++b) {
                    const uint32_t nib = (plane[b] >> (4 * q)) & 0xfu;
                    wv |= ((nib * 0x00204081u) & 0x01010101u) << b;
                }
                word[q] = wv;
            }
            uint8_t* out = (uint8_t*)a.cost + xbase;
            if (a.n >= 5) {
                ((uint4*)out)[0] = make_uint4(word[0], word[1], word[2], word[3]);
                ((uint4*)out)[1] = make_uint4(word[4], word[5], word[6], word[7]);
            } else {
                for (uint32_t j = 0; j < (1u << a.n); ++j) out[j] = (uint8_t)(word[j >> 2] >> (8 * (j & 3)));
            }
        } else {
            // 64 bytes: half-word j = sum_b bit j of plane b, shifted to bit b.
            uint32_t word[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                uint32_t wv = 0u;
#pragma unroll
                for (int b = 0; b < NP; ++b) {
                    const uint32_t pair = (plane[b] >> (2 * q)) & 3u;
                    wv |= ((pair * 0x8001u) & 0x10001u) << b;
                }
                word[q] = wv;
            }
            uint16_t* out = (uint16_t*)a.cost + xbase;
            if (a.n >= 5) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    ((uint4*)out)[q] = make_uint4(word[4 * q], word[4 * q + 1], word[4 * q + 2], word[4 * q + 3]);
            } else {
                for (uint32_t j = 0; j < (1u << a.n); ++j) out[j] = (uint16_t)(word[j >> 1] >> (16 * (j & 1)));
            }
        }
    }
    if (a.zeros) {
        __shared__ uint32_t blk;
        if (threadIdx.x == 0) blk = 0u;
        __syncthreads();
        // wave-level sum first, then one LDS atomic per wave
        uint32_t z = zeros;
        for (int off = 32; off > 0; off >>= 1) z += __shfl_xor(z, off);
        if ((threadIdx.x & 63) == 0 && z) atomicAdd(&blk, z);
        __syncthreads();
        if (threadIdx.x == 0 && blk) atomicAdd(a.zeros, (unsigned long long)blk);
    }
}

template <int NP, bool WIDE, bool U16>
__global__ __launch_bounds__(256) void cost_kernel(const CostArgs a) {
    cost_chunk<NP, WIDE, U16>(a, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Many diagonals at once: instance i owns blocks first[i] .. first[i+1]-1.
template <int NP, bool WIDE, bool U16>
__global__ __launch_bounds__(256) void cost_batch_kernel(const CostArgs* args, const uint32_t* first, int count) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const CostArgs a = args[lo];
    cost_chunk<NP, WIDE, U16>(a, (uint64_t)(blockIdx.x - first[lo]) * blockDim.x + threadIdx.x);
}

template <int NP, bool U16>
hipError_t launch_np(const CostArgs& a, bool wide, hipStream_t s) {
    const uint64_t nthreads = a.n >= 5 ? (1ull << (a.n - 5)) : 1ull;
    const uint64_t blocks = (nthreads + 255) / 256;
    if (wide)
        hipLaunchKernelGGL((cost_kernel<NP, true, U16>), dim3((uint32_t)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((cost_kernel<NP, false, U16>), dim3((uint32_t)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cost(const CostArgs& a, int dtype, bool wide, hipStream_t s) {
    // Enough planes to count up to the number of (normalised) clauses.
    const int need = 32 - __builtin_clz((unsigned)a.num_clauses | 1u);
    if (dtype == 1) {
        if (need <= 6) return launch_np<6, false>(a, wide, s);
        return launch_np<8, false>(a, wide, s);
    }
    if (need <= 12) return launch_np<12, true>(a, wide, s);
    return launch_np<16, true>(a, wide, s);
}

hipError_t launch_cost_batch(const CostArgs* args, const uint32_t* first, int count, uint32_t blocks, int dtype,
                             int max_clauses, bool wide, hipStream_t s) {
    const int need = 32 - __builtin_clz((unsigned)max_clauses | 1u);
    if (dtype == 1) {
        if (wide) hipLaunchKernelGGL((cost_batch_kernel<8, true, false>), dim3(blocks), dim3(256), 0, s, args, first, count);
        else hipLaunchKernelGGL((cost_batch_kernel<8, false, false>), dim3(blocks), dim3(256), 0, s, args, first, count);
    } else if (need <= 12) {
        if (wide) hipLaunchKernelGGL((cost_batch_kernel<12, true, true>), dim3(blocks), dim3(256), 0, s, args, first, count);
        else hipLaunchKernelGGL((cost_batch_kernel<12, false, true>), dim3(blocks), dim3(256), 0, s, args, first, count);
    } else {
        if (wide) hipLaunchKernelGGL((cost_batch_kernel<16, true, true>), dim3(blocks), dim3(256), 0, s, args, first, count);
        else hipLaunchKernelGGL((cost_batch_kernel<16, false, true>), dim3(blocks), dim3(256), 0, s, args, first, count);
    }
    return hipGetLastError();
}

}  // namespace qnae
