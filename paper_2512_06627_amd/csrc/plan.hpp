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
    uint32_t flags;  // kOutPos: miter |= value; kOutNeg: miter |= ~value
};
static_assert(sizeof(Instr) == 16, "instruction must stay 16 bytes");

enum : uint32_t { kCompl = 0x80000000u, kRowMask = 0x7FFFFFFFu, kOutPos = 1u, kOutNeg = 2u };

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
};

// bundle = 1: sequential stream.  bundle > 1: list-scheduled so that the gates of a
// bundle do not read each other, keeping the chosen order as the priority.
Plan make_plan(const Aig& g, Order order = Order::Auto, uint32_t bundle = 1);

// Check the slot map: every operand row holds the value it names when read,
// and no live value is overwritten.  Returns an empty string when consistent.
std::string validate_plan(const Aig& g, const Plan& p);

}  // namespace fes
