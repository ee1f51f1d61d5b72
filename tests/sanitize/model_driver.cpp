// Host driver for the runtime model's decisions (no GPU): reads lines
//   interp_gates rows lut_steps remaining_patterns sharing
// and prints, per line, the server's tier decision and the model times it was taken from:
//   want remaining_ms compile_ms interp_alone_ms lpt_cost_ms specialized_ms
#include <cstdio>

#include "model.hpp"

int main() {
    unsigned gates, rows, luts;
    double patterns;
    unsigned long sharing;
    while (std::scanf("%u %u %u %lf %lu", &gates, &rows, &luts, &patterns, &sharing) == 5) {
        fes::TierJob j;
        j.interp_gates = gates;
        j.rows = rows;
        j.lut_steps = luts;
        j.remaining_patterns = patterns;
        double rem = 0, comp = 0;
        const bool want = fes::server_wants_compile(j, sharing, &rem, &comp);
        std::printf("%d %.9g %.9g %.9g %.9g %.9g\n", want ? 1 : 0, rem, comp, fes::model_interp_ms(gates, rows, patterns),
                    fes::lpt_cost_ms(gates, rows, patterns), fes::model_specialized_ms(luts, patterns));
    }
    return 0;
}
