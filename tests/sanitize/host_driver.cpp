// Host-only driver for sanitizer builds of the planner path: AIGER reader, slot planner,
// LUT mapper, block emitter, simulation plan and sub-miter extraction.  For each AIGER file on
// the command line it prints a line with the file's index and the LUT program's miter word at
// each requested half-word, then a line "<index> sweep <targets> <FNV-1a of the sub-miters>".
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
            const Aig fused = fuse_xors(g);  // interpreter plans of bundles > 1 use the fused copy
            const std::string ferr = validate_plan(fused, make_plan(fused, Order::Auto, b));
            if (!ferr.empty()) {
                std::printf("%d fused plan %u: %s\n", f - 2, b, ferr.c_str());
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

        // Simulation plan (every gate: outputs plus gates that feed nothing), validated.
        Aig all = g;
        std::vector<uint8_t> read(all.max_var() + 1, 0);
        for (uint32_t k = 0; k < all.num_ands(); ++k) read[all.and_r0[k] >> 1] = read[all.and_r1[k] >> 1] = 1;
        for (uint32_t o : all.outputs) read[o >> 1] = 1;
        for (uint32_t k = 0; k < all.num_ands(); ++k)
            if (!read[all.num_inputs + 1 + k]) all.outputs.push_back(2 * (all.num_inputs + 1 + k));
        const Plan ps = make_plan(all, Order::Auto, 8);
        const std::string perr = validate_plan(all, ps);
        if (!perr.empty() || ps.num_ands_tfi != g.num_ands()) {
            std::printf("%d simulation plan: %s\n", f - 2, perr.c_str());
            return 1;
        }
        // Sub-miters: classes by equal normalised signatures over four words per input
        // (word k of input i = (i + 1) * 0x9E3779B1 + k * 0x85EBCA77 mod 2^32), then every target.
        const uint32_t V = g.max_var(), W = 4;
        std::vector<uint32_t> sig((size_t)(V + 1) * W, 0);
        for (uint32_t i = 0; i < g.num_inputs; ++i)
            for (uint32_t k = 0; k < W; ++k) sig[(size_t)(i + 1) * W + k] = (i + 1) * 0x9E3779B1u + k * 0x85EBCA77u;
        for (uint32_t k = 0; k < g.num_ands(); ++k) {
            const uint32_t v = g.num_inputs + 1 + k, a = g.and_r0[k], b = g.and_r1[k];
            for (uint32_t w = 0; w < W; ++w)
                sig[(size_t)v * W + w] = (sig[(size_t)(a >> 1) * W + w] ^ (0u - (a & 1u))) &
                                         (sig[(size_t)(b >> 1) * W + w] ^ (0u - (b & 1u)));
        }
        std::vector<uint32_t> cls(V + 1);
        std::vector<uint8_t> pol(V + 1);
        std::vector<std::pair<std::vector<uint32_t>, uint32_t>> seen;
        for (uint32_t v = 0; v <= V; ++v) {
            pol[v] = sig[(size_t)v * W] & 1u;
            std::vector<uint32_t> norm(W);
            for (uint32_t w = 0; w < W; ++w) norm[w] = sig[(size_t)v * W + w] ^ (0u - pol[v]);
            cls[v] = v;
            for (auto& e : seen)
                if (e.first == norm) {
                    cls[v] = e.second;
                    break;
                }
            if (cls[v] == v) seen.push_back({norm, v});
        }
        uint64_t h = 0xcbf29ce484222325ull, targets = 0;
        for (uint32_t v = g.num_inputs + 1; v <= V; ++v) {
            if (cls[v] == v) continue;
            std::vector<uint32_t> ins;
            const std::string text = submiter_aag(g, cls.data(), pol.data(), V + 1, v, &ins);
            const Aig back = parse_aiger((const uint8_t*)text.data(), text.size());  // must read back
            if (back.num_inputs != ins.size()) return 1;
            for (unsigned char ch : text) h = (h ^ ch) * 0x100000001b3ull;
            ++targets;
        }
        std::printf("%d sweep %llu %llu\n", f - 2, (unsigned long long)targets, (unsigned long long)h);
    }
    return 0;
}
