// Internal declarations shared by the host runtime and the HIP kernels of
// libqnae.so. Not part of the public ABI (include/qnae.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qnae {

// ---------------------------------------------------------------------------
// Cost diagonal (NAE-violated clause count per basis state)
// ---------------------------------------------------------------------------

// One clause after host normalisation. With M = the set of variables the
// clause touches and P = the variables whose literal is negated, the clause is
// violated at x exactly when ((x ^ P) & M) is 0 (all literals false) or M (all
// true). The low 5 bits are folded into two 32-bit tables over the position j
// of x inside an aligned run of 32 states: zero_tab bit j says
// ((j ^ P) & M & 31) == 0, full_tab bit j says it equals M & 31.
struct ClauseRec {
    uint32_t mask_hi_lo, mask_hi_hi;  // M with bits 0..4 cleared (low / high word)
    uint32_t pat_lo, pat_hi;          // P
    uint32_t zero_tab, full_tab;
};

struct CostArgs {
    const ClauseRec* clauses;
    int32_t num_clauses;
    int32_t n;
    void* cost;                 // uint8 or uint16 [2^n]
    unsigned long long* zeros;  // optional counter of states with cost 0
};

hipError_t launch_cost(const CostArgs& a, int dtype, hipStream_t s);

// ---------------------------------------------------------------------------
// State sweeps
// ---------------------------------------------------------------------------

// Mixer of one layer in the form used on the device. With t = tan(beta) when
// |tan(beta)| <= 1:  R(beta) = cos(beta) (I - i t X); otherwise, with
// t = -cot(beta):    R(beta) = (-i sin(beta)) X (I - i t X).
// Each butterfly therefore costs two FMAs per amplitude; `swap` applies the
// extra X, and the scalar factor is folded into the next phase table (or the
// readout).
struct MixForm {
    float t;
    int swap;
};

enum SweepFlags {
    SW_INIT = 1,    // start from the phase table instead of loading psi
    SW_PHASE = 2,   // apply the phase table between the pre- and post-mixers
    SW_REDUCE = 4,  // write block partial sums of the readout
    SW_STORE = 8,   // store psi back
    SW_SCALE = 16,  // multiply by store_scale when storing (final state)
};

struct SweepArgs {
    float2* psi;
    const void* cost;
    const float2* lut;     // phase table of this sweep (lut_len entries)
    double* partials;      // 3 doubles per block when SW_REDUCE
    int32_t n;
    int32_t c;             // tile: bits [0, c) and [H, H + TB - c)
    int32_t H;
    int32_t lut_len;
    uint32_t pre_mask;     // tile bits mixed before the phase
    uint32_t post_mask;    // tile bits mixed after the phase
    MixForm pre, post;
    float2 store_scale;
    int32_t flags;
    int32_t xcd_remap;     // spread consecutive tiles over one XCD
};

hipError_t launch_sweep(int tb, int dtype, const SweepArgs& a, hipStream_t s);

// Whole circuit for n <= 14 in one workgroup (state resident in LDS).
struct ResidentArgs {
    const void* cost;
    const float2* luts;    // p (or 1 when p = 0) tables of lut_len entries
    const MixForm* forms;  // p entries (device)
    float2* state_out;     // optional final state (scaled by store_scale)
    double* out;           // 3 doubles (unscaled sums)
    float2 store_scale;
    int32_t n, p, lut_len;
};

hipError_t launch_resident(int dtype, const ResidentArgs& a, hipStream_t s);

// Sum of 3-double block partials into out[3], FP64.
hipError_t launch_final_reduce(const double* partials, int64_t blocks, double* out, hipStream_t s);

}  // namespace qnae
