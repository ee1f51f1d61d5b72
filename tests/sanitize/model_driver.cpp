// Host driver for the runtime model's decisions (no GPU).
//
// Default mode reads lines
//   interp_gates rows lut_steps remaining_patterns sharing
// and prints, per line, the server's tier decision and the model times it was taken from:
//   want remaining_ms compile_ms interp_alone_ms lpt_cost_ms specialized_ms
//
// With the argument "group" it reads lines
//   helpers k lut_steps_1 ... lut_steps_k
// and prints, per line, the predicted wall time of compiling those k kernels as a group with
// that many helper processes: the group's fixed cost plus each kernel's part.
#include <cstdio>
#include <cstring>

#include "model.hpp"

int main(int argc, char** argv) {
    if (argc > 1 && std::strcmp(argv[1], "group") == 0) {
        int helpers;
        unsigned k;
        while (std::scanf("%d %u", &helpers, &k) == 2) {
            double ms = fes::model_group_compile_fixed_ms(helpers);
            for (unsigned i = 0; i < k; ++i) {
                unsigned luts = 0;
                if (std::scanf("%u", &luts) != 1) return 1;
                ms += fes::model_group_compile_kernel_ms(luts, helpers);
            }
            std::printf("%.9g\n", ms);
        }
        return 0;
    }
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
