// Runtime model of exact simulation on MI355X and the decisions made from it.  Host only (no
// HIP): the paper predicts ES time from the gate count and the input count (linear in gates,
// exponential in inputs; Section 3.2, runtime prediction) and offloads ES to the GPU when the
// prediction exceeds 0.1 s, with safety margins in [0.5, 2] on its rules (Section 3.2,
// GPU-accelerated scheduling).  Here every check already runs on the GPU; the model, fitted
// per kernel on MI355X with a fixed launch cost, chooses between the interpreter (no compile)
// and a compiled specialized kernel, orders batched cones and predicts serving times.
#pragma once
#include <cstddef>
#include <cstdint>

namespace fes {

//  interpreter:  t = t0 + N * max(patterns / R, L), N = bundled-stream gate instructions,
//                R by the value-file tier of its `rows` (register tier files of at most 104,
//                144 and 232 rows at four, three and two waves per SIMD; LDS or device memory
//                above), L = one wave pass per gate
//  specialized:  t = t0 + LUT steps * passes / R, passes = patterns / 2048 (at least 1)
//  compile:      t = c0 + c1 * LUT steps
double model_interp_ms(uint32_t gates, uint32_t rows, double patterns);
// Tier of a value file of `rows` rows: 0..2 register tier (104, 144, 232 rows), 3 LDS or device memory.
int model_interp_tier(uint32_t rows);
double model_specialized_ms(uint32_t lut_steps, double patterns);
double model_compile_ms(uint32_t lut_steps);
// Compiles of several kernels at once (a batch's routed cones): with `helpers` compile helper
// processes (0: in this process) the programs compile side by side, so the group's wall time is
// about one program's fixed cost (plus a helper's start-up) and each kernel adds its own part
// (a per-kernel cost inside a multi-kernel program plus c1 per LUT step) over the helpers.
double model_group_compile_fixed_ms(int helpers);
double model_group_compile_kernel_ms(uint32_t lut_steps, int helpers);

// LUT steps expected for a cone of `and_gates` AND gates before its LUT program is built
// (measured covers: 0.28 LUTs per gate for the 16x16 multiplier miter, 0.23 for layered cones;
// the larger ratio is used, so compiles are not underestimated).
uint32_t model_lut_steps_estimate(uint32_t and_gates);
// A count below the LUT steps of any cone measured (0.2 per AND gate): the specialized time and
// compile it gives are optimistic, so a saving that cannot pay off with it cannot pay off at all.
uint32_t model_lut_steps_low(uint32_t and_gates);

// Longest-processing-time cost of a cone in a shared interpreter launch: its predicted
// interpreter time over its range (ms).
double lpt_cost_ms(uint32_t interp_gates, uint32_t rows, double patterns);

// The server's specialized tier: a job on the interpreter shares each step equally with the
// other `sharing` interpreter jobs, so its remaining time there is `sharing` times its
// predicted time alone.  Its specialized kernel is compiled (on a background thread, while the
// job keeps running on the interpreter) when that remaining time exceeds the predicted
// specialized time of the same work plus twice the predicted compile time: the factor is the
// paper's largest safety margin, and it also covers the wait behind other jobs' compiles.
struct TierJob {
    uint32_t interp_gates = 1;  // bundled-stream gate instructions
    uint32_t rows = 0;          // value-file rows of the interpreter's stream (its tier)
    uint32_t lut_steps = 0;     // exact when the LUT program exists, else the estimate
    double remaining_patterns = 0;
};
constexpr double kTierCompileFactor = 2.0;
bool server_wants_compile(const TierJob& j, size_t sharing, double* remaining_ms, double* compile_ms);
// Lowest remaining interpreter time (at the job's share) for which a compile could be wanted,
// whatever its LUT count: below it the LUT program need not be built to decide.
double server_compile_threshold_ms();

}  // namespace fes
