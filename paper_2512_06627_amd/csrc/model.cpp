#include "model.hpp"

#include <algorithm>

namespace fes {

// Fitted on one MI355X by least squares on relative error (plain checks of 35 seeded layered cones
// and four multiplier and MAC miters, n 12..32; paper_2512_06627_amd/calibrate.py): median (largest)
// relative error 6% (52%) interpreter, 15% (59%) specialized, 0.7% (2%) compile.  Interpreter gates are
// the instructions of its bundled stream (three-AND XORs count once); its rate depends on the tier
// that holds the value file.
namespace model {
constexpr double kInterpT0Ms = 0.0116;
constexpr uint32_t kTierRows[3] = {104, 144, 232};  // register tier files; LDS or device memory above
constexpr double kInterpRate[4] = {1.958e14, 2.126e14, 1.940e14, 4.04e13};  // gate instructions*patterns/s
constexpr double kInterpMsPerGateFloor = 2.24e-5; // one wave pass per gate: spaces below a chip's waves
constexpr double kSpecT0Ms = 0.0135;
constexpr double kSpecLutPassesPerS = 6.08e11;
constexpr double kCompileC0Ms = 101.7;
constexpr double kCompileMsPerLut = 0.00664;
// Multi-kernel programs (GPU machine host, comgr's cache off): 16 kernels of about 500 LUT steps
// 0.39 s as one program, 8 of about 4,000 0.45 s, 2 small ones 0.14-0.16 s in helpers against
// the fixed 0.10 s in the process: each kernel adds about 12 ms besides its LUT steps, and a
// helper's start-up about 45 ms.
constexpr double kCompileMsPerKernel = 12.0;
constexpr double kHelperStartMs = 45.0;
constexpr double kLutsPerGate = 0.30;
constexpr double kLutsPerGateLow = 0.20;  // below every cover measured (0.23 layered cones, 0.28 multipliers)
}  // namespace model

int model_interp_tier(uint32_t rows) {
    for (int t = 0; t < 3; ++t)
        if (rows <= model::kTierRows[t]) return t;
    return 3;
}

double model_interp_ms(uint32_t gates, uint32_t rows, double patterns) {
    const double rate = model::kInterpRate[model_interp_tier(rows)];
    return model::kInterpT0Ms + (double)gates * std::max(patterns / rate * 1e3, model::kInterpMsPerGateFloor);
}

double model_specialized_ms(uint32_t lut_steps, double patterns) {
    return model::kSpecT0Ms + (double)lut_steps * std::max(1.0, patterns / 2048.0) / model::kSpecLutPassesPerS * 1e3;
}

double model_compile_ms(uint32_t lut_steps) { return model::kCompileC0Ms + model::kCompileMsPerLut * lut_steps; }

double model_group_compile_fixed_ms(int helpers) {
    return model::kCompileC0Ms + (helpers > 0 ? model::kHelperStartMs : 0.0);
}

double model_group_compile_kernel_ms(uint32_t lut_steps, int helpers) {
    return (model::kCompileMsPerKernel + model::kCompileMsPerLut * lut_steps) / (double)std::max(1, helpers);
}

uint32_t model_lut_steps_estimate(uint32_t and_gates) {
    return (uint32_t)((double)and_gates * model::kLutsPerGate + 0.5);
}

uint32_t model_lut_steps_low(uint32_t and_gates) {
    return std::max<uint32_t>(1, (uint32_t)((double)and_gates * model::kLutsPerGateLow));
}

double lpt_cost_ms(uint32_t interp_gates, uint32_t rows, double patterns) {
    return model_interp_ms(interp_gates, rows, patterns);
}

double server_compile_threshold_ms() { return kTierCompileFactor * model_compile_ms(0); }

bool server_wants_compile(const TierJob& j, size_t sharing, double* remaining_ms, double* compile_ms) {
    const double t_interp = (double)std::max<size_t>(1, sharing) *
                            model_interp_ms(std::max<uint32_t>(1, j.interp_gates), j.rows, j.remaining_patterns);
    const double t_compile = model_compile_ms(j.lut_steps);
    if (remaining_ms) *remaining_ms = t_interp;
    if (compile_ms) *compile_ms = t_compile;
    return t_interp > model_specialized_ms(j.lut_steps, j.remaining_patterns) + kTierCompileFactor * t_compile;
}

}  // namespace fes
