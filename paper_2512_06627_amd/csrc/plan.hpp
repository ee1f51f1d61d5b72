// Planner: output cone, evaluation order, reference-count slot map and the
// branch-free instruction stream.
//
// The paper compiles the circuit into a compact, branch-free instruction
// stream whose registers are reused under reference-count guidance, so the
// live storage follows the circuit's minimal cut instead of its size
// (Section 3.3, "Instructionalized ES"; Table 5).  Here the same idea is a
// host-side plan: every AND gate of the output cone gets a slot that is
// released when its last reader has executed, and the lowest free slot is
// taken next.  The interpreter kernels address slots as rows of a per-wave
// value file (LDS or device memory); the specialized kernel turns each slot
// into a register variable.
#pragma once
#include <cstdint>
#include <vector>

#include "aig.hpp"

namespace fes {

// Row layout of a value file: row 0 = constant false, rows 1..n = primary
// inputs, rows n+1 .. n+S = slots, row n+S+1 = sink for output-only steps.
struct Instr {
    uint32_t a;      // row of fanin 0; bit 31 = complement
    uint32_t b;      // row of fanin 1; bit 31 = complement
    uint32_t d;      // destination row
    uint32_t flags;  // kOutPos: miter |= value; kOutNeg: miter |= ~value; kXor: a XOR b, not a AND b
};
static_assert(sizeof(Instr) == 16, "instruction must stay 16 bytes");

enum : uint32_t { kCompl = 0x80000000u, kRowMask = 0x7FFFFFFFu, kOutPos = 1u, kOutNeg = 2u, kXor = 4u };

enum class Order : int { Auto = 0, DfsLabel = 1, DfsFanin0 = 2, File = 3 };

struct Plan {
    uint32_t bundle = 1;      // instructions per bundle: all operands of a bundle are read before
                              // any of its results is written, so a bundle holds independent gates
    uint32_t num_inputs = 0;
    uint32_t num_ands_file = 0;
    uint32_t num_ands_tfi = 0;
    uint32_t num_outputs = 0;
    uint32_t levels = 0;
    uint32_t peak_slots = 0;  // S
    uint32_t rows = 0;        // n + S + 2
    Order order_used = Order::Auto;
    std::vector<Instr> prog;  // bundles of `bundle` instructions: one per cone AND, one per output
                              // that is not an AND's own value, no-ops padding the last bundle
    uint32_t num_gate_instrs = 0;  // instructions that are not padding
    std::vector<uint32_t> order;   // AND gates (index into the AIG) in evaluation order
    std::vector<uint32_t> instr_gate;  // per prog entry: the AND gate it computes, or UINT32_MAX
                                       // (output-only step or padding)
};

// XOR fusion for interpreter plans (the three-AND XOR as one instruction): a gate
// v = ~t1 & ~t2 with t1 = x & y and t2 = ~x & ~y, where t1 and t2 have no other reader,
// equals x XOR y.  The copy keeps every variable's number; v becomes an XOR gate over
// (x, y), and t1, t2 drop out of the output cone.
Aig fuse_xors(const Aig& g);

// bundle = 1: sequential stream.  bundle > 1: list-scheduled so that the gates of a
// bundle do not read each other, keeping the chosen order as the priority.
Plan make_plan(const Aig& g, Order order = Order::Auto, uint32_t bundle = 1);

// Program of the specialized kernel: the cone mapped onto the three-input LUT instruction
// of gfx950 (v_bitop3_b32, result bit = table[4*src0 + 2*src1 + src2]).
//  * a value that depends only on inputs 0..4 and constants is the same 32-bit word in
//    every lane and pass ("word"): it is computed here, at plan time;
//  * a value that depends only on inputs 11.. (bits of the wave's base index), words and
//    constants is wave-uniform: it is computed on the scalar unit from two operands;
//  * every other gate becomes one VALU LUT over at most three leaves, absorbing fan-ins
//    that feed nothing else, so a LUT may stand for several AND gates.
struct LutRef {
    enum Kind : uint8_t { Input = 0, Word = 1, Uniform = 2, Varying = 3 } kind;
    uint32_t index;  // Input: input number; Word: index into words; Uniform/Varying: value id
};
struct LutStep {
    enum Op : uint8_t { Lut = 0, ScalarAnd = 1, Output = 2 } op;
    uint8_t table;       // Lut: truth table over (leaf0, leaf1, leaf2); ScalarAnd: bit0/bit1 = complement a/b
    uint8_t nleaves;     // Lut: 1..3 distinct leaves
    LutRef leaf[3];      // Lut: leaves; ScalarAnd: leaf[0], leaf[1]; Output: leaf[0]
    uint32_t dst;        // value id written (Lut: Varying, ScalarAnd: Uniform)
    bool out_neg;        // Output: accumulate the complement
};
struct LutProgram {
    uint32_t num_inputs = 0;
    std::vector<uint32_t> words;  // plan-time constant words
    std::vector<LutStep> steps;   // in evaluation order
    uint32_t num_values = 0;      // value ids used
    uint32_t lut_steps = 0, scalar_steps = 0, absorbed_gates = 0, folded_gates = 0;
    bool always_fails = false;    // an output is constant true
};
// scalar_policy: 0 = every wave-uniform gate on the scalar unit; 1 = only those without
// plan-time-word operands; 2 = none (all gates in VALU LUTs).
LutProgram make_lut_program(const Aig& g, const Plan& order_from, int scalar_policy = 0);

// Miter word of the LUT program at half-word hw (host evaluation, for validation).
uint32_t eval_lut_program(const LutProgram& lp, uint64_t hw);

// Check the slot map: every operand row holds the value it names when read,
// and no live value is overwritten.  Returns an empty string when consistent.
std::string validate_plan(const Aig& g, const Plan& p);

}  // namespace fes
