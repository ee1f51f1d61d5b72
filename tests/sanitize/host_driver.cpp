// Host-only driver for sanitizer builds of the planner path: AIGER reader, slot planner,
// LUT mapper and the block emitter.  For each AIGER file on the command line it prints one
// line: the file's index, then the LUT program's miter word at each requested half-word.
// Any memory or undefined-behaviour error aborts the run (AddressSanitizer / UBSan).
//
//   host_driver HW1,HW2,... file1.aig file2.aig ...
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <iterator>
#include <sstream>
#include <string>
#include <vector>

#include "runtime.hpp"

using namespace fes;

int main(int argc, char** argv) {
    if (argc < 3) return 2;
    std::vector<uint64_t> hws;
    std::stringstream ss(argv[1]);
    for (std::string tok; std::getline(ss, tok, ',');) hws.push_back(std::strtoull(tok.c_str(), nullptr, 10));
    for (int f = 2; f < argc; ++f) {
        std::ifstream in(argv[f], std::ios::binary);
        std::vector<uint8_t> bytes((std::istreambuf_iterator<char>(in)), std::istreambuf_iterator<char>());
        Aig g;
        try {
            g = parse_aiger(bytes.data(), bytes.size());
        } catch (const Error& e) {
            std::printf("%d error %d\n", f - 2, e.code);
            continue;
        }
        const Plan p1 = make_plan(g, Order::Auto, 1);
        for (uint32_t b : {1u, 4u, 8u, 16u}) {
            const Plan p = b == 1 ? p1 : make_plan(g, Order::Auto, b);
            const std::string err = validate_plan(g, p);
            if (!err.empty()) {
                std::printf("%d plan %u: %s\n", f - 2, b, err.c_str());
                return 1;
            }
        }
        std::vector<uint32_t> words;
        for (int policy : {0, 2}) {
            const LutProgram lp = make_lut_program(g, p1, policy);
            for (int dist : {1, 6})
                for (bool banks : {false, true})
                    for (int cap : {232, 24}) {  // 24 VGPRs: spills to LDS
                        std::string code;
                        BlockStats st;
                        emit_block_body(lp, cap, 64, 0, 20, dist, banks, cap < 64 ? 255 : 0, &code, &st);
                    }
            for (size_t i = 0; i < hws.size(); ++i) {
                const uint64_t h = g.num_inputs >= 5 ? hws[i] % (1ull << (g.num_inputs - 5)) : 0;
                const uint32_t w = eval_lut_program(lp, h);
                if (policy == 0) words.push_back(w);
                else if (words[i] != w) {
                    std::printf("%d policies disagree at half-word %llu\n", f - 2, (unsigned long long)h);
                    return 1;
                }
            }
        }
        std::printf("%d", f - 2);
        for (uint32_t w : words) std::printf(" %u", w);
        std::printf("\n");
    }
    return 0;
}
