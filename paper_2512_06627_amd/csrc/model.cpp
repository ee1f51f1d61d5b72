#include "model.hpp"

#include <algorithm>

namespace fes {

// Fitted on one MI355X by least squares on relative error (plain checks of 32 cones, n 12..32):
// median relative error 8% (interpreter), 16% (specialized), 1% (compile); largest 28%, 61%,
// 4%.  Interpreter gates are the instructions of its bundled stream (three-AND XORs count once).
namespace model {
constexpr double kInterpT0Ms = 0.0169;
constexpr uint32_t kInterpSlotsBreak = 140;      // rate drops above: fewer waves per CU
constexpr double kInterpRate = 4.62e13;          // gate instructions*patterns/s, value files of <= break slots
constexpr double kInterpRateLarge = 2.71e13;     // above
constexpr double kInterpMsPerGateFloor = 5.0e-5; // one wave pass per gate: spaces below a chip's waves
constexpr double kSpecT0Ms = 0.0130;
constexpr double kSpecLutPassesPerS = 6.33e11;
constexpr double kCompileC0Ms = 104.1;
constexpr double kCompileMsPerLut = 0.00649;
constexpr double kLutsPerGate = 0.30;
}  // namespace model

double model_interp_ms(uint32_t gates, uint32_t slots, double patterns) {
    const double rate = slots > model::kInterpSlotsBreak ? model::kInterpRateLarge : model::kInterpRate;
    return model::kInterpT0Ms + (double)gates * std::max(patterns / rate * 1e3, model::kInterpMsPerGateFloor);
}

double model_specialized_ms(uint32_t lut_steps, double patterns) {
    return model::kSpecT0Ms + (double)lut_steps * std::max(1.0, patterns / 2048.0) / model::kSpecLutPassesPerS * 1e3;
}

double model_compile_ms(uint32_t lut_steps) { return model::kCompileC0Ms + model::kCompileMsPerLut * lut_steps; }

uint32_t model_lut_steps_estimate(uint32_t and_gates) {
    return (uint32_t)((double)and_gates * model::kLutsPerGate + 0.5);
}

double lpt_cost_ms(uint32_t interp_gates, uint32_t slots, double patterns) {
    return model_interp_ms(interp_gates, slots, patterns);
}

double server_compile_threshold_ms() { return kTierCompileFactor * model_compile_ms(0); }

bool server_wants_compile(const TierJob& j, size_t sharing, double* remaining_ms, double* compile_ms) {
    const double t_interp = (double)std::max<size_t>(1, sharing) *
                            model_interp_ms(std::max<uint32_t>(1, j.interp_gates), j.slots, j.remaining_patterns);
    const double t_compile = model_compile_ms(j.lut_steps);
    if (remaining_ms) *remaining_ms = t_interp;
    if (compile_ms) *compile_ms = t_compile;
    return t_interp > model_specialized_ms(j.lut_steps, j.remaining_patterns) + kTierCompileFactor * t_compile;
}

}  // namespace fes
