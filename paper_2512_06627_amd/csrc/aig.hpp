// AIG model and AIGER reader of the GPU path.
//
// After loading, variables are renumbered densely: var 0 is constant false,
// vars 1..n are the primary inputs in file order (input i drives bit i of the
// pattern index), and vars n+1..n+A are the AND gates in a topological order.
// Literal = 2*var + complement (the AIGER convention; paper, Section 2.1
// represents circuits as latch-free AIGs).
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace fes {

struct Aig {
    uint32_t num_inputs = 0;
    std::vector<uint32_t> and_r0;  // fanin literals of AND k (var num_inputs + 1 + k)
    std::vector<uint32_t> and_r1;
    std::vector<uint32_t> outputs; // output literals
    // Nonzero entry k: gate k computes lit(and_r0[k]) XOR lit(and_r1[k]) instead of the AND
    // (interpreter plans of a fused copy only; empty = every gate is an AND).
    std::vector<uint8_t> xor_gate;
    bool is_xor(uint32_t k) const { return k < xor_gate.size() && xor_gate[k]; }
    uint32_t num_ands() const { return (uint32_t)and_r0.size(); }
    uint32_t max_var() const { return num_inputs + num_ands(); }
};

// Status codes shared with the C ABI.
enum Status : int {
    kOk = 0,
    kErrParse = -1,
    kErrUnsupported = -2,
    kErrNoMem = -3,
    kErrDevice = -4,
    kErrInvalid = -5,
    kCancelled = -6,
    kTimeout = -7,
    kRejected = -8,
};

struct Error {
    int code;
    std::string msg;
};

// Parse ASCII ("aag") or binary ("aig") AIGER.  Throws Error.
Aig parse_aiger(const uint8_t* bytes, size_t len);

}  // namespace fes
