// Internal declarations shared by the host runtime and the HIP kernels of
// libqnae.so. Not part of the public ABI (include/qnae.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qnae {

// ---------------------------------------------------------------------------
// Cost diagonal (violated clause count per basis state)
// ---------------------------------------------------------------------------

// One clause after host normalisation. With M = the set of variables the
// clause touches and P = the variables whose literal is negated, the clause is
// violated at x exactly when ((x ^ P) & M) is 0 (all literals false) or M (all
// true; NAE) or only when it is 0 (k-SAT: full_tab is empty). The low 5 bits
// are folded into two 32-bit tables over the position j of x inside an aligned
// run of 32 states: zero_tab bit j says ((j ^ P) & M & 31) == 0, full_tab bit
// j says it equals M & 31.
struct ClauseRec {
    uint32_t mask_hi_lo, mask_hi_hi;  // M with bits 0..4 cleared (low / high word)
    uint32_t pat_lo, pat_hi;          // P
    uint32_t zero_tab, full_tab;
};

struct CostArgs {
    const ClauseRec* clauses;
    int32_t num_clauses;
    int32_t num_low;            // records 0 .. num_low-1 have a variable below 5; the rest only higher ones
    int32_t n;
    void* cost;                 // uint8 or uint16 [2^n]
    unsigned long long* zeros;  // optional counter of states with cost 0
};

// C(x) for x < 2^a.n. wide: clause variables reach index 32 or above
// (64-bit pattern compares), required when any variable is >= 32.
hipError_t launch_cost(const CostArgs& a, int dtype, bool wide, hipStream_t s);
// Many diagonals of one cost type: instance i owns 256-thread blocks
// first[i] .. first[i+1]-1 (32 states per thread). max_clauses bounds every
// instance's clause count; wide when some instance has n > 32.
hipError_t launch_cost_batch(const CostArgs* args, const uint32_t* first, int count, uint32_t blocks, int dtype,
                             int max_clauses, bool wide, hipStream_t s);

// ---------------------------------------------------------------------------
// State sweeps
// ---------------------------------------------------------------------------

// Mixer of one layer in the form used on the device. With t = tan(beta) when
// |tan(beta)| <= 1:  R(beta) = cos(beta) (I - i t X); otherwise, with
// t = -cot(beta):    R(beta) = (-i sin(beta)) X (I - i t X).
// Each butterfly therefore costs two FMAs per amplitude. The scalar factor is
// folded into the next phase table (or the readout). The X of the cot form
// (`flip`) is not applied: X on every qubit of the layer is a relabelling
// x -> NOT x of the stored state, so the runtime tracks the parity of flipped
// layers and reads the cost at the complemented index where it matters
// (phase and readout), undoing the relabelling only if the final state is
// returned.
struct MixForm {
    float t;
    int flip;
};

// Sweep kinds: which steps a sweep performs.
enum SweepKind {
    SK_FIRST = 0,     // phase table 0 as initial state, mix, store
    SK_MIDDLE = 1,    // load, mix, store
    SK_BOUNDARY = 2,  // load, mix (layer l), phase (l + 1), mix (l + 1), store
    SK_FINAL = 3,     // load, mix, readout partials (optional store)
    SK_P0 = 4,        // phase table 0 as state, readout (p = 0)
};

struct SweepArgs {
    float2* psi;           // state written (and read, unless psi_in is set)
    const float2* psi_in;  // state read by the load (== psi for in-place sweeps)
    const void* cost;
    const float2* lut;     // phase table of this sweep (lut_len entries)
    double* partials;      // 3 doubles per block for readout kinds
    int32_t n;
    int32_t nw;            // n - TB: block-index bits
    uint64_t tile_bits;    // global bits spanned by a tile
    uint8_t pos[16];       // tile bit i -> bit pos[i] of x (pos[0..3] = 0..3)
    uint64_t wmask;        // bits of x outside the tile (filled by the tile index)
    int32_t lut_len;
    uint32_t pre_mask;     // tile bits mixed before the phase
    uint32_t post_mask;    // tile bits mixed after the phase
    float pre_t, post_t;
    float2 store_scale;    // readout kinds with store: final scalar factor
    int32_t store;         // readout kinds: also store the state
    int32_t cflip;         // read the cost at the complemented index
    // Half-state sweeps (NAE global-flip symmetry): the state and cost hold
    // only x < 2^(n-1); the amplitude of x with bit n-1 set is the one at
    // its complement. With half set, tile bit vbit (pos[vbit] = n-1) is the
    // virtual bit: flipping it maps a stored index y to mir - y, mir =
    // 2^(n-1) - 1. Without a virtual bit (vbit < 0) a half sweep is a plain
    // sweep over n-1 bits.
    int32_t half;
    int32_t vbit;
    uint64_t mir;
    // Checkpointing boundary sweep (gradient forward pass): the state right
    // after the pre mixing, which completes a layer, times ckpt_scale (that
    // layer's mixer factor), in natural order (element x at x ^ (2^n - 1)
    // when cflip) to ckpt.
    float2* ckpt;
    float2 ckpt_scale;
};

hipError_t launch_sweep(int tb, int dtype, int kind, const SweepArgs& a, hipStream_t s);
// A boundary sweep that also stores a checkpoint (a.ckpt), 13-bit tiles,
// full state.
hipError_t launch_sweep_ckpt(int dtype, const SweepArgs& a, hipStream_t s);

// One sweep step over `count` states at once. Instance i owns blocks
// first[i] .. first[i+1]-1 (first has count+1 entries, first[count] =
// blocks), one per tile of its own geometry; args[i].partials receives 3
// doubles per tile for readout kinds. Every instance uses tiles of tb bits
// (12, 13 or 14). half: every instance is a half-state sweep (args[i].half).
hipError_t launch_sweep_batch(int tb, int dtype, int kind, const SweepArgs* args, const uint32_t* first, int count,
                              uint32_t blocks, hipStream_t s, bool half = false);
hipError_t launch_reverse(float2* psi, uint64_t N, hipStream_t s);

// Whole circuit for n <= 14 in one workgroup (state resident in LDS).
struct ResidentArgs {
    const float2* state_in;  // optional initial state (true scale); |+> when null
    const void* cost;
    const float2* luts;    // p (or 1 when p = 0) tables of lut_len entries
    const MixForm* forms;  // p entries (device)
    float2* state_out;     // optional final state (scaled by store_scale)
    double* out;           // 3 doubles (unscaled sums)
    float2 store_scale;
    int32_t n, p, lut_len;
};

hipError_t launch_resident(int dtype, const ResidentArgs& a, hipStream_t s);

// The same with the tables in the kernel arguments (no copy ahead of the
// launch): p phase tables of lut_len entries (one when p = 0), then the p
// mixer forms, each stored in one float2 slot; a.luts and a.forms unused.
constexpr int kResidentInline = 448;
struct ResidentInlineArgs {
    ResidentArgs a;
    float2 tab[kResidentInline];
};
hipError_t launch_resident_inline(int dtype, const ResidentInlineArgs& a, hipStream_t s);

// ---------------------------------------------------------------------------
// Adjoint (gradient) sweeps: the reverse pass carries the adjoint state lam
// and the forward state psi together and applies the inverse of each layer to
// both (psi is uncomputed). The inverse mixers use the forward sweeps'
// butterflies (I - i t X) with |t| <= 1: the layer's scalar factor is folded
// into its inverse phase table, the X on every qubit of the cotangent form is
// a relabelling (index x holds element x ^ (2^n - 1)), and the inner products
// taken between butterflies carry the factor the butterflies left out.
// Tiles as in the forward sweeps, TB = 13.
// ---------------------------------------------------------------------------

enum AdjointKind {
    AK_MIDDLE = 0,    // inverse mixer of one group (b-layer i)
    AK_BOUNDARY = 1,  // inverse mixer (i), inverse phase (i), inverse mixer (i + 1) of one group
    AK_END = 2,       // inverse mixer (i), inverse phase (i): last op of a reverse segment
};

struct AdjointArgs {
    float2* lam;
    float2* psi;
    const void* cost;
    const float2* lut;     // F exp(+i gamma c), c = 0 .. lut_len - 1, F the layer's mixer factor
    double* partials;      // 3 per tile: Im<lam|X|psi> (pre group), Im<lam|C|psi>, Im<lam|X|psi> (post group)
    int32_t n, nw, lut_len;
    uint64_t tile_bits, wmask;
    uint8_t pos[16];
    uint32_t pre_mask, post_mask;
    // Butterfly own' = own - i t partner. Before each butterfly the pair term
    // is added with weight w, then w *= r (r = |one qubit's factor|^2): w
    // starts at r^k for k qubits of the layer mixed by earlier sweeps.
    float pre_t, pre_r, pre_w, post_t, post_r, post_w;
    uint64_t cost_flip;  // 0 or 2^n - 1: the phase of element x reads cost[x ^ cost_flip]
    int32_t psi_flip;    // psi of element x sits at x ^ (2^n - 1) (relabelled against lam)
    int32_t store_psi;
    float w_psucc, w_energy;  // weigh: lam = (w_psucc [C = 0] + w_energy C) psi instead of a load
};

constexpr int kAdjointTileBits = 13;
// weigh: the middle kind forms lam from psi (first sweep of the reverse pass,
// no relabelling) instead of loading it.
hipError_t launch_adjoint(int dtype, int kind, const AdjointArgs& a, hipStream_t s, bool weigh = false);


// Whole gradient for n <= 13 in one workgroup (lam and psi resident in LDS):
// forward with exact butterflies (checkpoints of psi every `every` layers in
// ckpt), readout, then the reverse pass with psi refreshed at checkpoints.
struct ResidentGradArgs {
    const void* cost;
    const float2* luts;    // p forward tables exp(-i gamma_l c)
    const float2* cs;      // p (cos beta_l, sin beta_l)
    float2* ckpt;          // (p - 1) / every states of 2^n
    double* out;           // 3 readout sums, then dgamma[p], then dbeta[p]
    double w_psucc, w_energy;
    int32_t n, p, lut_len, every;
};
hipError_t launch_resident_grad(int dtype, const ResidentGradArgs& a, hipStream_t s);
// One workgroup per entry of args (count entries, all of one cost type).
hipError_t launch_resident_grad_batch(int dtype, const ResidentGradArgs* args, int count, hipStream_t s);
hipError_t launch_resident_batch(int dtype, const ResidentArgs* args, int count, hipStream_t s);

// Sum of 3-double block partials into out[3], FP64.
hipError_t launch_final_reduce(const double* partials, int64_t blocks, double* out, hipStream_t s);
// Instance i: sum of blocks[i] triples at partials[i] -> outs[i][0..2].
hipError_t launch_final_reduce_batch(const double* const* partials, const uint32_t* blocks, double* const* outs,
                                     int count, hipStream_t s);

// ---------------------------------------------------------------------------
// Sampling outcomes of a state (sample.hip)
// ---------------------------------------------------------------------------

constexpr int kSampleTileBits = 12;
constexpr int kSampleChunks = 1024;  // tile-prefix chunks
// Draw `count` outcomes of psi (2^n complex64) for the given uniforms in
// [0, 1): mass (ceil(2^n / 4096) doubles), pref (one more) and chunk
// (kSampleChunks doubles) are scratch. out[q] = ~0 marks a zero state.
// out_cost, if not null, receives C at each outcome (or -1 without a cost
// diagonal).
hipError_t launch_sample(const float2* psi, int n, const void* cost, int cost_dtype, const double* uniforms,
                         int count, double* mass, double* pref, double* chunk, uint64_t* out, int32_t* out_cost,
                         hipStream_t s);

}  // namespace qnae
