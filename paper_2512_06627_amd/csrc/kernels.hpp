// Device-side data layouts shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace fes {

// One circuit of an interpreter launch (plain check = a launch with one cone).
// Pattern space unit: a 32-bit "half-word" h holds patterns 32h .. 32h+31; each lane
// of a wave holds `K` half-words per value-file row.
struct ConeDesc {
    const Instr* prog;   // device copy of the instruction stream
    uint32_t n_instr;    // multiple of the plan's bundle size
    uint32_t n_inputs;
    uint32_t rows;       // value-file rows this cone uses
    uint32_t best_index; // index into the launch's best[] array
    uint64_t hw_begin;   // half-word range [hw_begin, hw_end)
    uint64_t hw_end;
    uint64_t hw_first;   // hw_begin rounded down to the pass size (64 * K)
    uint64_t tile_hw;    // half-words per work item (multiple of 64 * K)
    uint64_t item_begin; // first work item of this cone in the launch
    uint64_t item_end;   // one past its last work item
};
static_assert(sizeof(ConeDesc) == 72, "descriptor layout");

// Work claims are spread over C = min(kClaimCounters, waves in the grid) counters, each on
// its own 128-byte line: the wave with global index w claims from counter s = w % C and gets
// the items s, s + C, s + 2C, ... in that order.  One shared counter
// serialises every claim of the launch at the atomic unit (about 30 ns each), which bounds
// launches of many short work items; spread over separate lines the claims proceed in
// parallel, and the items still start in roughly ascending order.
constexpr uint32_t kClaimCounters = 16;
constexpr uint32_t kClaimStride = 16;  // 64-bit words from one counter to the next (128 bytes)
constexpr size_t kClaimBytes = sizeof(unsigned long long) * kClaimCounters * kClaimStride;

// Control block at the start of each launch's device buffer (all zero before a launch).
struct alignas(128) LaunchCtl {
    unsigned long long next_item[kClaimCounters * kClaimStride];  // claim counters, see above
};
static_assert(sizeof(LaunchCtl) == kClaimBytes, "control block layout");

struct InterpLaunch {
    const ConeDesc* cones;
    uint32_t num_cones;
    uint32_t rows_max;        // value-file rows per wave
    uint64_t total_items;
    LaunchCtl* ctl;
    unsigned long long* best; // per cone: lowest failing pattern, ~0 = none yet
    uint32_t* hbm_rows;       // device value files (HBM tier); null for the LDS tier
    const int* cancel;        // device-visible flag polled per work item, may be null
    // Simulation mode only (launch_interp_sim): the half-word index is a column of caller
    // input words instead of a pattern range, and every gate's value is stored.
    const uint32_t* sim_pi = nullptr;  // n rows of sim_words 32-bit words (row i = input i)
    uint32_t* sim_sig = nullptr;       // rows 0..max_var of sim_words words (row v = variable v)
    uint64_t sim_words = 0;
};

// Launch the interpreter.  K = half-words per lane per row (1, 2, 4); B = bundle size
// (1, 4, 8, 16); lds = value file in LDS (else in hbm_rows).  Returns hipSuccess or an error.
hipError_t launch_interp(const InterpLaunch& L, int K, int B, bool lds, int grid, int block,
                         hipStream_t stream);

// Simulation mode of the interpreter: one cone, bundles of B (8, or 16 with K <= 2), instruction
// flags = the variable a gate defines (0 = store nothing).  Columns [0, sim_words) are simulated
// once each.
hipError_t launch_interp_sim(const InterpLaunch& L, int K, int B, bool lds, int grid, int block, hipStream_t stream);

// Per row of a signature matrix (rows x words, row-major): the number of ones and the
// complement-normalised hash sum_k word'_k * (fmix32(k) | 1) mod 2^64, where word' is the
// row complemented when its first bit is 1.  One wave per row, grid-stride over rows.
hipError_t launch_signature_hash(const uint32_t* sig, uint64_t rows, uint64_t words, uint64_t* hash,
                                 uint64_t* ones, int grid, hipStream_t stream);

// Register tier's stream: per bundle of 4 gates, 28 words in this order
//   a[4]   operand rows with the complement flag in bit 31 (the kernel indexes registers by the
//          low 8 bits, so the flag needs no masking),
//   b[4]   the same for the second operands,
//   d[4]   destination rows; bit 31 of d[0] is set when a gate of the bundle drives an output,
//   ca[4], cb[4]  complement masks of the operands (0 or all ones),
//   xm[4]  XOR masks (all ones for a fused three-AND XOR, else 0),
//   fl[4]  the instruction flags (output polarity bits 0 and 1), read only in marked bundles.
constexpr uint32_t kRegsBundleWords = 28;
// Encode a bundled plan (bundle 4) into that layout, followed by one bundle of zeros (the kernel
// prefetches one bundle past the one it runs, so the last prefetch stays inside the stream).
void encode_regs_stream(const Plan& p, std::vector<uint32_t>& out);

// The simulation-mode variant of that layout for one call: words 20..27 hold, per gate, the
// 64-bit address of the signature row of the variable it defines (sig + variable * words), or
// `dummy` (a row of `words` words) for instructions that define none; one zero bundle follows.
void encode_sim_regs_stream(const Plan& p, const uint32_t* sig, uint64_t words, const uint32_t* dummy,
                            std::vector<uint32_t>& out);
// Simulation mode in the register tier: one cone, the stream above as the descriptor's prog,
// columns [0, sim_words) (at most 2^30) simulated once each; `regs` as for launch_interp_regs.
hipError_t launch_sim_regs(const InterpLaunch& L, int regs, int grid, hipStream_t stream);

// Register tier: value files in VGPRs (one wave per workgroup, bundles of 4, one 32-bit word per
// lane).  interp_regs_rows: the file size (104, 144 or 232 rows) that holds `rows`, 0 if none
// does, with the waves per SIMD it allows.  launch_interp_regs: `regs` is that file size.
int interp_regs_rows(uint32_t rows, int* waves_per_simd);
hipError_t launch_interp_regs(const InterpLaunch& L, int regs, int grid, hipStream_t stream);

// Largest per-workgroup dynamic LDS the interpreter may request.
size_t interp_lds_bytes(uint32_t rows, int K, int waves_per_block);

}  // namespace fes
