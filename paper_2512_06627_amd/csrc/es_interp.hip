// Generic exact-simulation interpreter for gfx950.
//
// Work decomposition: the pattern space of each cone is cut into work items
// (tiles) of `tile_hw` half-words (32 patterns each).  Every wave claims items
// in ascending order from one counter, so low patterns are simulated first and
// a wave can drop an item that starts above the lowest failure found so far.
//
// Value file: each wave owns rows_max rows; a row holds one node value for the
// wave's 64 lanes * K half-words (lane-major, K consecutive 32-bit words per
// lane).  Row 0 is constant false, rows 1..n the primary inputs (rewritten
// each pass from the half-word index, so no input patterns are stored), the
// remaining rows are the planner's slots.  Each lane touches only its own
// column, so no barrier is ever needed.
//
// Instruction stream: bundles of B instructions (16 bytes each) read with
// scalar loads (the stream is wave-uniform).  All operands of a bundle are
// loaded before any result is stored, which is what lets the planner put
// independent gates in one bundle and reuse freed slots inside it.
//
// Miter and early exit: results flagged as outputs are ORed into the lane's
// miter word.  After each pass a wave ballot finds the lowest lane with a
// nonzero word; its lowest set bit is the wave's lowest failing pattern and is
// folded into best[] with atomicMin.  The paper's ES checks every assignment
// and reports a distinguishing pattern (Sections 2.1, 2.2, 3.3); this kernel
// reports the lowest one, which makes the answer independent of scheduling.
//
// Simulation mode (kSim): the logic simulation that opens a sweeping flow
// (Section 2.3, step 1).  The "half-word" index is a column of caller input
// words: input i's row holds sim_pi[i][column] instead of the pattern-index
// mask, each gate instruction's flags name the variable it defines, and its
// value is stored to that variable's signature row.  Rows 0..n of the
// signature are written too (constant false, the input words), so the output
// is the value of every variable.  No miter, no early exit.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fes {
namespace {

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Wave-uniform data (descriptors, the instruction stream) is read through the constant
// address space so that it is fetched with scalar loads into SGPRs.
#define FES_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const FES_CONST T* as_const(const T* p) {
    return (const FES_CONST T*)(p);
}

template <int K>
struct alignas(4 * K) Words {
    uint32_t w[K];
};

// Value of primary input i on the 32 patterns of half-word hw.  Inputs 0..4 select a bit
// inside the 32-bit word; input i >= 5 is bit i-5 of hw, the same for all 32 patterns.
__device__ __forceinline__ uint32_t pi_word(uint32_t i, uint64_t hw) {
    switch (i) {
        case 0: return 0xAAAAAAAAu;
        case 1: return 0xCCCCCCCCu;
        case 2: return 0xF0F0F0F0u;
        case 3: return 0xFF00FF00u;
        case 4: return 0xFFFF0000u;
        default: return 0u - (uint32_t)((hw >> (i - 5)) & 1u);
    }
}

template <int K, int B, bool kLds, bool kSim>
__global__ void __launch_bounds__(1024) es_interp_kernel(InterpLaunch L) {
    extern __shared__ uint32_t lds_file[];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    constexpr uint32_t kRowWords = 64u * K;
    uint32_t* file;
    if constexpr (kLds) {
        file = lds_file + (size_t)wave * L.rows_max * kRowWords;
    } else {
        const size_t gw = (size_t)blockIdx.x * (blockDim.x >> 6) + wave;
        file = L.hbm_rows + gw * L.rows_max * kRowWords;
    }
    uint32_t* col = file + lane * K;  // row r of this lane: col + r * kRowWords
    using V = Words<K>;

    // Control flow stays wave-uniform: every lane takes part in the claim (lane 0 adds 1,
    // the others 0) and in the atomicMin (all lanes hold the same value), so no branch
    // depends on the lane and every loop exit is a scalar branch.
    const uint32_t wave_gid = blockIdx.x * (blockDim.x >> 6) + wave;
    // A grid with fewer waves than counters uses one counter per wave, so every counter in
    // use has a wave and every item is claimed.
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    const uint32_t nclaim = waves < kClaimCounters ? waves : kClaimCounters;
    const uint32_t claim = __builtin_amdgcn_readfirstlane(wave_gid % nclaim);  // wave-uniform
    unsigned long long* const counter = &L.ctl->next_item[claim * kClaimStride];
    for (;;) {
        const uint64_t k = uniform64(atomicAdd(counter, lane == 0 ? 1ull : 0ull));
        const uint64_t item = claim + k * nclaim;
        if (item >= L.total_items) break;
        if (L.cancel && __builtin_amdgcn_readfirstlane(
                            __hip_atomic_load(L.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)))
            break;

        const FES_CONST ConeDesc* cones = as_const(L.cones);
        uint32_t lo = 0, hi = L.num_cones - 1;  // cone holding this item (uniform search)
        while (lo < hi) {
            uint32_t mid = (lo + hi + 1) >> 1;
            if (cones[mid].item_begin <= item) lo = mid; else hi = mid - 1;
        }
        const FES_CONST ConeDesc* c = cones + lo;
        unsigned long long* best = &L.best[c->best_index];
        const uint64_t hw_begin = c->hw_begin, hw_end = c->hw_end;
        const uint64_t hw0 = c->hw_first + (item - c->item_begin) * c->tile_hw;
        const uint64_t hw_stop = min(hw0 + c->tile_hw, hw_end);
        const uint32_t n = c->n_inputs, n_instr = c->n_instr;
        const FES_CONST Instr* prog = as_const(c->prog);

        // The bound found by other waves is read once per work item: a device-scope load at
        // the start of every pass is a full memory round trip per pass.
        const uint64_t best_now =
            kSim ? ~0ull : uniform64(__hip_atomic_load(best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        const uint64_t W = L.sim_words;
        for (uint64_t base = hw0; base < hw_stop; base += 64u * K) {
            if (32u * base >= best_now) break;  // nothing at or above here can lower best
            V zero;
#pragma unroll
            for (int j = 0; j < K; ++j) zero.w[j] = 0u;
            *(V*)(col) = zero;
            if constexpr (kSim) {
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const uint64_t w = base + (uint64_t)(j * 64) + lane;
                    if (w < W) L.sim_sig[w] = 0u;
                }
            }
            for (uint32_t i = 0; i < n; ++i) {
                V x;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const uint64_t w = base + (uint64_t)(j * 64) + lane;
                    if constexpr (kSim) {
                        x.w[j] = w < W ? L.sim_pi[(size_t)i * W + w] : 0u;
                        if (w < W) L.sim_sig[(size_t)(1 + i) * W + w] = x.w[j];
                    } else {
                        x.w[j] = pi_word(i, w);
                    }
                }
                *(V*)(col + (size_t)(1 + i) * kRowWords) = x;
            }
            V m = zero;
            for (uint32_t t = 0; t < n_instr; t += B) {
                Instr ins[B];
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    ins[u].a = prog[t + u].a;
                    ins[u].b = prog[t + u].b;
                    ins[u].d = prog[t + u].d;
                    ins[u].flags = prog[t + u].flags;
                }
                V a[B], b[B];
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    a[u] = *(const V*)(col + (size_t)(ins[u].a & kRowMask) * kRowWords);
                    b[u] = *(const V*)(col + (size_t)(ins[u].b & kRowMask) * kRowWords);
                }
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const uint32_t ca = 0u - (ins[u].a >> 31), cb = 0u - (ins[u].b >> 31);
                    V r;
                    if constexpr (kSim) {
#pragma unroll
                        for (int j = 0; j < K; ++j) r.w[j] = (a[u].w[j] ^ ca) & (b[u].w[j] ^ cb);
                    } else {
                        // XOR instructions (three fused ANDs): the all-ones mask selects x ^ y.
                        // One v_bitop3 over (x, y, mask); table bit 4x + 2y + m is m ? x ^ y : x & y.
                        const uint32_t xm = 0u - ((ins[u].flags >> 2) & 1u);
#pragma unroll
                        for (int j = 0; j < K; ++j) {
                            const uint32_t x = a[u].w[j] ^ ca, y = b[u].w[j] ^ cb;
                            r.w[j] = __builtin_amdgcn_bitop3_b32(x, y, xm, 0x68);
                        }
                    }
                    *(V*)(col + (size_t)ins[u].d * kRowWords) = r;
                    if constexpr (kSim) {
                        if (ins[u].flags) {
#pragma unroll
                            for (int j = 0; j < K; ++j) {
                                const uint64_t w = base + (uint64_t)(j * 64) + lane;
                                if (w < W) L.sim_sig[(size_t)ins[u].flags * W + w] = r.w[j];
                            }
                        }
                    } else if (ins[u].flags & (kOutPos | kOutNeg)) {
                        const uint32_t op = 0u - (ins[u].flags & kOutPos), on = 0u - ((ins[u].flags >> 1) & 1u);
#pragma unroll
                        for (int j = 0; j < K; ++j) m.w[j] |= (r.w[j] & op) | (~r.w[j] & on);
                    }
                }
            }
            if constexpr (kSim) continue;
            // Lowest failing pattern of this pass: first sub-word j with a nonzero lane, then
            // its lowest lane l, then the lowest set bit of that lane's word.
            uint64_t p = ~0ull;
#pragma unroll
            for (int j = K - 1; j >= 0; --j) {
                const uint64_t hw = base + (uint64_t)(j * 64) + lane;
                const uint32_t mj = (hw >= hw_begin && hw < hw_end) ? m.w[j] : 0u;
                const uint64_t bal = __ballot(mj != 0u);
                const uint32_t l = bal ? (uint32_t)__builtin_ctzll(bal) : 0u;
                const uint32_t ml = __builtin_amdgcn_readlane(mj, l);
                if (bal) p = 32ull * (base + (uint64_t)(j * 64) + l) + (uint32_t)__builtin_ctz(ml);
            }
            if (p != ~0ull) {
                atomicMin(best, (unsigned long long)p);
                break;
            }
        }
    }
}

template <int K, int B, bool kLds, bool kSim = false>
hipError_t launch_one(const InterpLaunch& L, int grid, int block, hipStream_t stream) {
    const size_t lds = kLds ? interp_lds_bytes(L.rows_max, K, block / 64) : 0;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&es_interp_kernel<K, B, kLds, kSim>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((es_interp_kernel<K, B, kLds, kSim>), dim3(grid), dim3(block), lds, stream, L);
    return hipGetLastError();
}

template <int K, int B>
hipError_t launch_kb(const InterpLaunch& L, bool lds, int grid, int block, hipStream_t s) {
    return lds ? launch_one<K, B, true>(L, grid, block, s) : launch_one<K, B, false>(L, grid, block, s);
}

template <int K, int B>
hipError_t launch_sim_kb(const InterpLaunch& L, bool lds, int grid, int block, hipStream_t s) {
    return lds ? launch_one<K, B, true, true>(L, grid, block, s) : launch_one<K, B, false, true>(L, grid, block, s);
}

template <int K>
hipError_t launch_k(const InterpLaunch& L, int B, bool lds, int grid, int block, hipStream_t s) {
    switch (B) {
        case 1: return launch_kb<K, 1>(L, lds, grid, block, s);
        case 4: return launch_kb<K, 4>(L, lds, grid, block, s);
        case 8: return launch_kb<K, 8>(L, lds, grid, block, s);
        case 16: return launch_kb<K, 16>(L, lds, grid, block, s);
        default: return hipErrorInvalidValue;
    }
}

// ---- register tier ------------------------------------------------------------------------
//
// The value file of a wave in its own VGPRs instead of LDS.  With files in LDS a CU holds about
// 160 KB / (rows x 256 B) waves, about one per SIMD for the usual cones, and one wave issues at
// most one instruction every few cycles, so the interpreter runs at the issue rate of a single
// wave per SIMD.  The VGPR file is 512 KB per CU: the same cones fit two to four waves per SIMD.
//
// Row r of the file is v[kFileBase + r]; rows are read and written through gfx950's GPR index
// mode (s_set_gpr_idx_on / _idx / _off: the low 8 bits of an SGPR offset the register number of
// the indexed operand), so the file needs no address arithmetic.  The index is taken from the
// operand and destination words themselves: only their low 8 bits count, so a row with its
// complement flag (or the bundle's output mark) in bit 31 indexes the right register.  Bundles
// of four gates keep the stream's read-all-then-write-all semantics: the eight operands go to
// v16..v23, complemented by the instruction that reads them, then each result is selected and
// written to its row by one instruction.  The stream is the register tier's own encoding
// (encode_regs_stream: complement and XOR masks precomputed, one output mark per bundle), so a
// gate costs three VALU instructions and three index moves.  It comes in by
// scalar loads, one bundle (112 bytes) ahead into a second set of SGPRs; with no LDS operations
// in the pass, the scalar wait counter tracks only those loads.
//
// One pass (2,048 patterns: 64 lanes x 32) is one asm statement.  It owns v16..v(kFileBase+R-1),
// s36..s99 and m0.  Inputs: the stream, the bundle count, n, the pass's first half-word index
// (bits 6 and up give inputs 11 and up) and the lane words of inputs 5..10.  Output: the lane's
// miter word.
constexpr int kFileBase = 24;

// Eight operand reads of a bundle through the SRC0 index, each with its complement mask applied
// by the reading instruction itself: v16 = a0 ^ ca0, v17 = b0 ^ cb0, ..., v23 = b3 ^ cb3.  Index
// mode is left on (SRC0): the next s_set_gpr_idx_on replaces index and mode, and code that
// runs other VALU instructions first switches it off.
#define FES_RG_READS(A0, B0, A1, B1, A2, B2, A3, B3, CA0, CB0, CA1, CB1, CA2, CB2, CA3, CB3) \
    "s_set_gpr_idx_on " A0 ", gpr_idx(SRC0)\n"                                                \
    "v_xor_b32_e64 v16, v24, " CA0 "\n"                                                        \
    "s_set_gpr_idx_idx " B0 "\n"                                                               \
    "v_xor_b32_e64 v17, v24, " CB0 "\n"                                                        \
    "s_set_gpr_idx_idx " A1 "\n"                                                               \
    "v_xor_b32_e64 v18, v24, " CA1 "\n"                                                        \
    "s_set_gpr_idx_idx " B1 "\n"                                                               \
    "v_xor_b32_e64 v19, v24, " CB1 "\n"                                                        \
    "s_set_gpr_idx_idx " A2 "\n"                                                               \
    "v_xor_b32_e64 v20, v24, " CA2 "\n"                                                        \
    "s_set_gpr_idx_idx " B2 "\n"                                                               \
    "v_xor_b32_e64 v21, v24, " CB2 "\n"                                                        \
    "s_set_gpr_idx_idx " A3 "\n"                                                               \
    "v_xor_b32_e64 v22, v24, " CA3 "\n"                                                        \
    "s_set_gpr_idx_idx " B3 "\n"                                                               \
    "v_xor_b32_e64 v23, v24, " CB3 "\n"
// The gate's select over (XOR mask, a, b): a ^ b where the mask is set, a & b elsewhere (table
// 0x68), written straight into the destination row through the DST index.  The mask is an SGPR,
// so no source of the select is a VGPR the index applies to.  Index mode is left on (DST): only
// scalar instructions follow until the next bundle's reads (the pass switches it off at its end).
#define FES_RG_COMPUTE_WRITES(D0, D1, D2, D3, X0, X1, X2, X3)          \
    "s_set_gpr_idx_on " D0 ", gpr_idx(DST)\n"                         \
    "v_bitop3_b32 v24, " X0 ", v16, v17 bitop3:0x68\n"                 \
    "s_set_gpr_idx_idx " D1 "\n"                                       \
    "v_bitop3_b32 v24, " X1 ", v18, v19 bitop3:0x68\n"                 \
    "s_set_gpr_idx_idx " D2 "\n"                                       \
    "v_bitop3_b32 v24, " X2 ", v20, v21 bitop3:0x68\n"                 \
    "s_set_gpr_idx_idx " D3 "\n"                                       \
    "v_bitop3_b32 v24, " X3 ", v22, v23 bitop3:0x68\n"
// Bundles that hold an output: the select into TA first, then the output test, then the write.
#define FES_RG_GATE(TA, TB, XM) "v_bitop3_b32 " TA ", " XM ", " TA ", " TB " bitop3:0x68\n"
// Output accumulation of one gate of a marked bundle (result TA, scratch TB, flags F).
#define FES_RG_OUT(TA, TB, F, LBL)                                 \
    "s_and_b32 s93, " F ", 3\n"                                     \
    "s_cbranch_scc0 " LBL "_%=\n"                                   \
    "s_bfe_i32 s92, " F ", 0x10000\n"                               \
    "s_bfe_i32 s93, " F ", 0x10001\n"                               \
    "v_mov_b32 " TB ", s93\n"                                       \
    "v_bitop3_b32 " TB ", " TA ", s92, " TB " bitop3:0xca\n"        \
    "v_or_b32 %[m], %[m], " TB "\n"                                 \
    LBL "_%=:\n"
#define FES_RG_WRITES(D0, D1, D2, D3)          \
    "s_set_gpr_idx_on " D0 ", gpr_idx(DST)\n" \
    "v_mov_b32 v24, v16\n"                     \
    "s_set_gpr_idx_idx " D1 "\n"               \
    "v_mov_b32 v24, v18\n"                     \
    "s_set_gpr_idx_idx " D2 "\n"               \
    "v_mov_b32 v24, v20\n"                     \
    "s_set_gpr_idx_idx " D3 "\n"               \
    "v_mov_b32 v24, v22\n"                     \
    "s_set_gpr_idx_off\n"
// One bundle from the 28 SGPRs of a buffer (words a0..a3, b0..b3, d0..d3, ca, cb, xm, fl).  A
// bundle with its output mark (bit 31 of d0) branches to its out-of-line copy (FES_RG_MARKED),
// which returns to the label after it.
#define FES_RG_BUNDLE(a0, a1, a2, a3, b0, b1, b2, b3, d0, d1, d2, d3, ca0, ca1, ca2, ca3, cb0, cb1, cb2, cb3, x0, x1, \
                      x2, x3, f0, f1, f2, f3, P)                                                                     \
    FES_RG_READS(a0, b0, a1, b1, a2, b2, a3, b3, ca0, cb0, ca1, cb1, ca2, cb2, ca3, cb3)                               \
    "s_bitcmp1_b32 " d0 ", 31\n"                                                                                       \
    "s_cbranch_scc1 fes_rg" P "_marked_%=\n"                                                                           \
    FES_RG_COMPUTE_WRITES(d0, d1, d2, d3, x0, x1, x2, x3)                                                              \
    "fes_rg" P "_back_%=:\n"
#define FES_RG_MARKED(a0, a1, a2, a3, b0, b1, b2, b3, d0, d1, d2, d3, ca0, ca1, ca2, ca3, cb0, cb1, cb2, cb3, x0, x1, \
                      x2, x3, f0, f1, f2, f3, P)                                                                     \
    "fes_rg" P "_marked_%=:\n"                                                                                         \
    "s_set_gpr_idx_off\n"                                                                                              \
    FES_RG_GATE("v16", "v17", x0) FES_RG_GATE("v18", "v19", x1) FES_RG_GATE("v20", "v21", x2)                          \
    FES_RG_GATE("v22", "v23", x3)                                                                                      \
    FES_RG_OUT("v16", "v17", f0, "fes_rg" P "_o0") FES_RG_OUT("v18", "v19", f1, "fes_rg" P "_o1")                        \
    FES_RG_OUT("v20", "v21", f2, "fes_rg" P "_o2") FES_RG_OUT("v22", "v23", f3, "fes_rg" P "_o3")                        \
    FES_RG_WRITES(d0, d1, d2, d3)                                                                                      \
    "s_branch fes_rg" P "_back_%=\n"
// Buffer A: s36..s63, buffer B: s64..s91 (one bundle each, kRegsBundleWords = 28 words).
#define FES_RG_REGS_A(M)                                                                                    \
    M("s36", "s37", "s38", "s39", "s40", "s41", "s42", "s43", "s44", "s45", "s46", "s47", "s48", "s49", "s50", \
      "s51", "s52", "s53", "s54", "s55", "s56", "s57", "s58", "s59", "s60", "s61", "s62", "s63", "a")
#define FES_RG_REGS_B(M)                                                                                    \
    M("s64", "s65", "s66", "s67", "s68", "s69", "s70", "s71", "s72", "s73", "s74", "s75", "s76", "s77", "s78", \
      "s79", "s80", "s81", "s82", "s83", "s84", "s85", "s86", "s87", "s88", "s89", "s90", "s91", "b")
#define FES_RG_BUF_A FES_RG_REGS_A(FES_RG_BUNDLE)
#define FES_RG_BUF_B FES_RG_REGS_B(FES_RG_BUNDLE)
// Bundle k of the pair at s[94:95] (k = 0, 1 or 2: 112-byte bundles) into buffer A or B.
#define FES_RG_LOAD_A(O16, O8, O4)                  \
    "s_load_dwordx16 s[36:51], s[94:95], " O16 "\n" \
    "s_load_dwordx8 s[52:59], s[94:95], " O8 "\n"   \
    "s_load_dwordx4 s[60:63], s[94:95], " O4 "\n"
#define FES_RG_LOAD_B(O16, O8, O4)                  \
    "s_load_dwordx16 s[64:79], s[94:95], " O16 "\n" \
    "s_load_dwordx8 s[80:87], s[94:95], " O8 "\n"   \
    "s_load_dwordx4 s[88:91], s[94:95], " O4 "\n"

#define FES_RG_INPUT(I, ROW, VAL)            \
    "s_cmp_eq_u32 %[n], " #I "\n"            \
    "s_cbranch_scc1 fes_rg_in_done_%=\n"     \
    "v_mov_b32 " ROW ", " VAL "\n"

// Registers: s92, s93 scratch; s[94:95] stream pointer (advanced by two bundles per loop
// iteration: buffer A runs the bundle at the pointer, B the next); s96 bundles left after the
// current one (the loop ends when subtracting one borrows); s97 input index; s[98:99] a shifted
// copy of the pass index.  Every bundle's successor is loaded while it runs, so the last one
// loads the stream's padding bundle; the pass waits for that load before it ends, since the
// compiler takes the clobbered SGPRs as free once the statement is over (a load still in flight
// then overwrote the compiler's own values: correct answers, tens of times slower).
#define FES_RG_PASS_ASM                                                                                   \
    "v_mov_b32 v24, 0\n"                                                                                  \
    FES_RG_INPUT(0, "v25", "0xaaaaaaaa") FES_RG_INPUT(1, "v26", "0xcccccccc")                              \
    FES_RG_INPUT(2, "v27", "0xf0f0f0f0") FES_RG_INPUT(3, "v28", "0xff00ff00")                              \
    FES_RG_INPUT(4, "v29", "0xffff0000") FES_RG_INPUT(5, "v30", "%[x5]") FES_RG_INPUT(6, "v31", "%[x6]")    \
    FES_RG_INPUT(7, "v32", "%[x7]") FES_RG_INPUT(8, "v33", "%[x8]") FES_RG_INPUT(9, "v34", "%[x9]")         \
    FES_RG_INPUT(10, "v35", "%[x10]")                                                                      \
    "s_cmp_eq_u32 %[n], 11\n"                                                                             \
    "s_cbranch_scc1 fes_rg_in_done_%=\n"                                                                  \
    "s_mov_b32 s97, 11\n"                                                                                 \
    "fes_rg_in_loop_%=:\n"                                                                                \
    "s_sub_u32 s96, s97, 5\n"                                                                             \
    "s_lshr_b64 s[98:99], %[base], s96\n"                                                                 \
    "s_and_b32 s98, s98, 1\n"                                                                             \
    "s_sub_u32 s98, 0, s98\n"                                                                             \
    "s_add_u32 s99, s97, 1\n"                                                                             \
    "s_set_gpr_idx_on s99, gpr_idx(DST)\n"                                                                \
    "v_mov_b32 v24, s98\n"                                                                                \
    "s_set_gpr_idx_off\n"                                                                                 \
    "s_add_u32 s97, s97, 1\n"                                                                             \
    "s_cmp_lt_u32 s97, %[n]\n"                                                                            \
    "s_cbranch_scc1 fes_rg_in_loop_%=\n"                                                                  \
    "fes_rg_in_done_%=:\n"                                                                                \
    "v_mov_b32 %[m], 0\n"                                                                                 \
    "s_mov_b64 s[94:95], %[prog]\n"                                                                       \
    "s_sub_u32 s96, %[nb], 1\n"                                                                           \
    FES_RG_LOAD_A("0x0", "0x40", "0x60")                                                                  \
    "fes_rg_loop_%=:\n"                                                                                   \
    "s_waitcnt lgkmcnt(0)\n"                                                                              \
    FES_RG_LOAD_B("0x70", "0xb0", "0xd0")                                                                 \
    FES_RG_BUF_A                                                                                          \
    "s_sub_u32 s96, s96, 1\n"                                                                             \
    "s_cbranch_scc1 fes_rg_end_%=\n"                                                                      \
    "s_waitcnt lgkmcnt(0)\n"                                                                              \
    FES_RG_LOAD_A("0xe0", "0x120", "0x140")                                                               \
    FES_RG_BUF_B                                                                                          \
    "s_add_u32 s94, s94, 224\n"                                                                           \
    "s_addc_u32 s95, s95, 0\n"                                                                            \
    "s_sub_u32 s96, s96, 1\n"                                                                             \
    "s_cbranch_scc0 fes_rg_loop_%=\n"                                                                     \
    "fes_rg_end_%=:\n"                                                                                    \
    "s_waitcnt lgkmcnt(0)\n"                                                                              \
    "s_set_gpr_idx_off\n"                                                                                 \
    "s_branch fes_rg_exit_%=\n"                                                                           \
    FES_RG_REGS_A(FES_RG_MARKED) FES_RG_REGS_B(FES_RG_MARKED)                                             \
    "fes_rg_exit_%=:\n"

#define FES_RG_SCLOB                                                                                      \
    "m0", "scc", "s36", "s37", "s38", "s39", "s40", "s41", "s42", "s43", "s44", "s45", "s46", "s47", "s48",  \
        "s49", "s50", "s51", "s52", "s53", "s54", "s55", "s56", "s57", "s58", "s59", "s60", "s61", "s62",   \
        "s63", "s64", "s65", "s66", "s67", "s68", "s69", "s70", "s71", "s72", "s73", "s74", "s75", "s76",   \
        "s77", "s78", "s79", "s80", "s81", "s82", "s83", "s84", "s85", "s86", "s87", "s88", "s89", "s90",   \
        "s91", "s92", "s93", "s94", "s95", "s96", "s97", "s98", "s99"
#define FES_V10(d) "v" #d "0", "v" #d "1", "v" #d "2", "v" #d "3", "v" #d "4", "v" #d "5", "v" #d "6", \
                   "v" #d "7", "v" #d "8", "v" #d "9"
// v16..v127 (file rows 0..103)
#define FES_RG_VCLOB_104                                                                                  \
    "v16", "v17", "v18", "v19", FES_V10(2), FES_V10(3), FES_V10(4), FES_V10(5), FES_V10(6), FES_V10(7),     \
        FES_V10(8), FES_V10(9), FES_V10(10), FES_V10(11), "v120", "v121", "v122", "v123", "v124", "v125",   \
        "v126", "v127"
// v16..v167 (file rows 0..143)
#define FES_RG_VCLOB_144                                                                                  \
    FES_RG_VCLOB_104, "v128", "v129", FES_V10(13), FES_V10(14), FES_V10(15), "v160", "v161", "v162", "v163", \
        "v164", "v165", "v166", "v167"
// v16..v255 (file rows 0..231)
#define FES_RG_VCLOB_232                                                                                  \
    FES_RG_VCLOB_144, "v168", "v169", FES_V10(17), FES_V10(18), FES_V10(19), FES_V10(20), FES_V10(21),     \
        FES_V10(22), FES_V10(23), FES_V10(24), "v250", "v251", "v252", "v253", "v254", "v255"

template <int R>
__device__ __forceinline__ uint32_t regs_pass(const Instr* prog, uint32_t nb, uint32_t n, uint64_t base,
                                              uint32_t x5, uint32_t x6, uint32_t x7, uint32_t x8, uint32_t x9,
                                              uint32_t x10) {
    uint32_t m;
#define FES_RG_OPERANDS                                                                                   \
    : [m] "=&v"(m)                                                                                        \
    : [prog] "s"(prog), [nb] "s"(nb), [n] "s"(n), [base] "s"(base), [x5] "v"(x5), [x6] "v"(x6),            \
      [x7] "v"(x7), [x8] "v"(x8), [x9] "v"(x9), [x10] "v"(x10)
    if constexpr (R == 104) {
        asm volatile(FES_RG_PASS_ASM FES_RG_OPERANDS : FES_RG_SCLOB, FES_RG_VCLOB_104);
    } else if constexpr (R == 144) {
        asm volatile(FES_RG_PASS_ASM FES_RG_OPERANDS : FES_RG_SCLOB, FES_RG_VCLOB_144);
    } else {
        asm volatile(FES_RG_PASS_ASM FES_RG_OPERANDS : FES_RG_SCLOB, FES_RG_VCLOB_232);
    }
#undef FES_RG_OPERANDS
    return m;
}

// One wave per workgroup; waves_per_eu pins the occupancy the file size allows.
template <int R, int kWaves>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kWaves, kWaves)))
es_interp_regs_kernel(InterpLaunch L) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t x5 = 0u - (lane & 1u), x6 = 0u - ((lane >> 1) & 1u), x7 = 0u - ((lane >> 2) & 1u);
    const uint32_t x8 = 0u - ((lane >> 3) & 1u), x9 = 0u - ((lane >> 4) & 1u), x10 = 0u - ((lane >> 5) & 1u);
    const uint32_t wave_gid = blockIdx.x;
    const uint32_t waves = gridDim.x;
    const uint32_t nclaim = waves < kClaimCounters ? waves : kClaimCounters;
    const uint32_t claim = __builtin_amdgcn_readfirstlane(wave_gid % nclaim);
    unsigned long long* const counter = &L.ctl->next_item[claim * kClaimStride];
    for (;;) {
        const uint64_t k = uniform64(atomicAdd(counter, lane == 0 ? 1ull : 0ull));
        const uint64_t item = claim + k * nclaim;
        if (item >= L.total_items) break;
        if (L.cancel && __builtin_amdgcn_readfirstlane(
                            __hip_atomic_load(L.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)))
            break;
        const FES_CONST ConeDesc* cones = as_const(L.cones);
        uint32_t lo = 0, hi = L.num_cones - 1;
        while (lo < hi) {
            uint32_t mid = (lo + hi + 1) >> 1;
            if (cones[mid].item_begin <= item) lo = mid; else hi = mid - 1;
        }
        const FES_CONST ConeDesc* c = cones + lo;
        unsigned long long* best = &L.best[c->best_index];
        const uint64_t hw_begin = c->hw_begin, hw_end = c->hw_end;
        const uint64_t hw0 = c->hw_first + (item - c->item_begin) * c->tile_hw;
        const uint64_t hw_stop = min(hw0 + c->tile_hw, hw_end);
        const uint32_t n = __builtin_amdgcn_readfirstlane(c->n_inputs);
        const uint32_t nb = __builtin_amdgcn_readfirstlane(c->n_instr / 4u);
        const Instr* prog = c->prog;
        const uint64_t best_now = uniform64(__hip_atomic_load(best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        for (uint64_t base = hw0; base < hw_stop; base += 64u) {
            if (32u * base >= best_now) break;
            const uint32_t mw = nb ? regs_pass<R>(prog, nb, n, base, x5, x6, x7, x8, x9, x10) : 0u;
            const uint64_t hw = base + lane;
            const uint32_t mj = (hw >= hw_begin && hw < hw_end) ? mw : 0u;
            const uint64_t bal = __ballot(mj != 0u);
            if (bal) {
                const uint32_t l = (uint32_t)__builtin_ctzll(bal);
                const uint32_t ml = __builtin_amdgcn_readlane(mj, l);
                atomicMin(best, 32ull * (base + l) + (uint32_t)__builtin_ctz(ml));
                break;
            }
        }
    }
}

template <int R, int kWaves>
hipError_t launch_regs(const InterpLaunch& L, int grid, hipStream_t stream) {
    hipLaunchKernelGGL((es_interp_regs_kernel<R, kWaves>), dim3(grid), dim3(64), 0, stream, L);
    return hipGetLastError();
}

// ---- register tier, simulation mode --------------------------------------------------------
//
// The logic simulation that opens a sweeping flow (Section 2.3, step 1) with the value file in
// VGPRs: every variable's word is stored to its signature row, so the kernel is bound by HBM
// writes rather than by instruction issue.  One pass covers 64 caller words (one per lane).
// The stream (encode_sim_regs_stream) has the register tier's 28-word bundles with the XOR
// masks and output flags replaced by the absolute address of each gate's signature row (two
// words per gate; gates that define no variable point at a dummy row); it is built per call,
// since the addresses depend on the signature buffer and its row length.  A pass: row 0 (zero)
// and the n input rows are written to the file and stored, then per bundle the eight operand
// reads with their complements, four ANDs, four indexed writes and four row stores.  Lanes past
// the last word are masked off for the whole pass (EXEC), so they neither compute nor store.
// The stores are non-temporal: the signature matrix is far larger than the caches and is read
// back by a later kernel (16x16 miter at 2^18 words: 1.87 ms with ordinary stores, 1.45 ms).
#define FES_RS_BUNDLE(a0, a1, a2, a3, b0, b1, b2, b3, d0, d1, d2, d3, ca0, ca1, ca2, ca3, cb0, cb1, cb2, cb3, P0, P1, \
                      P2, P3)                                                                                        \
    FES_RG_READS(a0, b0, a1, b1, a2, b2, a3, b3, ca0, cb0, ca1, cb1, ca2, cb2, ca3, cb3)                               \
    "s_set_gpr_idx_off\n"                                                                                              \
    "v_and_b32 v16, v16, v17\n"                                                                                        \
    "v_and_b32 v18, v18, v19\n"                                                                                        \
    "v_and_b32 v20, v20, v21\n"                                                                                        \
    "v_and_b32 v22, v22, v23\n"                                                                                        \
    FES_RG_WRITES(d0, d1, d2, d3)                                                                                      \
    "global_store_dword %[off], v16, " P0 " nt\n"                                                                         \
    "global_store_dword %[off], v18, " P1 " nt\n"                                                                         \
    "global_store_dword %[off], v20, " P2 " nt\n"                                                                         \
    "global_store_dword %[off], v22, " P3 " nt\n"
#define FES_RS_BUF_A                                                                                           \
    FES_RS_BUNDLE("s36", "s37", "s38", "s39", "s40", "s41", "s42", "s43", "s44", "s45", "s46", "s47", "s48", "s49", \
                  "s50", "s51", "s52", "s53", "s54", "s55", "s[56:57]", "s[58:59]", "s[60:61]", "s[62:63]")
#define FES_RS_BUF_B                                                                                           \
    FES_RS_BUNDLE("s64", "s65", "s66", "s67", "s68", "s69", "s70", "s71", "s72", "s73", "s74", "s75", "s76", "s77", \
                  "s78", "s79", "s80", "s81", "s82", "s83", "s[84:85]", "s[86:87]", "s[88:89]", "s[90:91]")

// Registers: s[92:93] address of the next input's signature row; s[94:95] stream pointer; s96
// bundles left after the current one; s[98:99] address of the next input's caller row.  The
// input loads share one wait (vmcnt also counts the stores still in flight); the last stream
// prefetch is waited for before the statement ends.
// Input i (n <= 63) is loaded straight into its file row v(25 + i) and stored to its signature
// row: all loads of a pass are issued before one wait.
#define FES_RS_LD(I, V)                              \
    "s_cmp_eq_u32 %[n], " #I "\n"                    \
    "s_cbranch_scc1 fes_rs_ld_done_%=\n"              \
    "global_load_dword " V ", %[off], s[98:99]\n"     \
    "s_add_u32 s98, s98, %[wb_lo]\n"                 \
    "s_addc_u32 s99, s99, %[wb_hi]\n"
#define FES_RS_ST(I, V)                              \
    "s_cmp_eq_u32 %[n], " #I "\n"                    \
    "s_cbranch_scc1 fes_rs_st_done_%=\n"              \
    "global_store_dword %[off], " V ", s[92:93] nt\n" \
    "s_add_u32 s92, s92, %[wb_lo]\n"                 \
    "s_addc_u32 s93, s93, %[wb_hi]\n"
#define FES_RS_LOADS \
    FES_RS_LD(0, "v25") FES_RS_LD(1, "v26") FES_RS_LD(2, "v27") FES_RS_LD(3, "v28") \
    FES_RS_LD(4, "v29") FES_RS_LD(5, "v30") FES_RS_LD(6, "v31") FES_RS_LD(7, "v32") \
    FES_RS_LD(8, "v33") FES_RS_LD(9, "v34") FES_RS_LD(10, "v35") FES_RS_LD(11, "v36") \
    FES_RS_LD(12, "v37") FES_RS_LD(13, "v38") FES_RS_LD(14, "v39") FES_RS_LD(15, "v40") \
    FES_RS_LD(16, "v41") FES_RS_LD(17, "v42") FES_RS_LD(18, "v43") FES_RS_LD(19, "v44") \
    FES_RS_LD(20, "v45") FES_RS_LD(21, "v46") FES_RS_LD(22, "v47") FES_RS_LD(23, "v48") \
    FES_RS_LD(24, "v49") FES_RS_LD(25, "v50") FES_RS_LD(26, "v51") FES_RS_LD(27, "v52") \
    FES_RS_LD(28, "v53") FES_RS_LD(29, "v54") FES_RS_LD(30, "v55") FES_RS_LD(31, "v56") \
    FES_RS_LD(32, "v57") FES_RS_LD(33, "v58") FES_RS_LD(34, "v59") FES_RS_LD(35, "v60") \
    FES_RS_LD(36, "v61") FES_RS_LD(37, "v62") FES_RS_LD(38, "v63") FES_RS_LD(39, "v64") \
    FES_RS_LD(40, "v65") FES_RS_LD(41, "v66") FES_RS_LD(42, "v67") FES_RS_LD(43, "v68") \
    FES_RS_LD(44, "v69") FES_RS_LD(45, "v70") FES_RS_LD(46, "v71") FES_RS_LD(47, "v72") \
    FES_RS_LD(48, "v73") FES_RS_LD(49, "v74") FES_RS_LD(50, "v75") FES_RS_LD(51, "v76") \
    FES_RS_LD(52, "v77") FES_RS_LD(53, "v78") FES_RS_LD(54, "v79") FES_RS_LD(55, "v80") \
    FES_RS_LD(56, "v81") FES_RS_LD(57, "v82") FES_RS_LD(58, "v83") FES_RS_LD(59, "v84") \
    FES_RS_LD(60, "v85") FES_RS_LD(61, "v86") FES_RS_LD(62, "v87") \
    ""
#define FES_RS_STORES \
    FES_RS_ST(0, "v25") FES_RS_ST(1, "v26") FES_RS_ST(2, "v27") FES_RS_ST(3, "v28") \
    FES_RS_ST(4, "v29") FES_RS_ST(5, "v30") FES_RS_ST(6, "v31") FES_RS_ST(7, "v32") \
    FES_RS_ST(8, "v33") FES_RS_ST(9, "v34") FES_RS_ST(10, "v35") FES_RS_ST(11, "v36") \
    FES_RS_ST(12, "v37") FES_RS_ST(13, "v38") FES_RS_ST(14, "v39") FES_RS_ST(15, "v40") \
    FES_RS_ST(16, "v41") FES_RS_ST(17, "v42") FES_RS_ST(18, "v43") FES_RS_ST(19, "v44") \
    FES_RS_ST(20, "v45") FES_RS_ST(21, "v46") FES_RS_ST(22, "v47") FES_RS_ST(23, "v48") \
    FES_RS_ST(24, "v49") FES_RS_ST(25, "v50") FES_RS_ST(26, "v51") FES_RS_ST(27, "v52") \
    FES_RS_ST(28, "v53") FES_RS_ST(29, "v54") FES_RS_ST(30, "v55") FES_RS_ST(31, "v56") \
    FES_RS_ST(32, "v57") FES_RS_ST(33, "v58") FES_RS_ST(34, "v59") FES_RS_ST(35, "v60") \
    FES_RS_ST(36, "v61") FES_RS_ST(37, "v62") FES_RS_ST(38, "v63") FES_RS_ST(39, "v64") \
    FES_RS_ST(40, "v65") FES_RS_ST(41, "v66") FES_RS_ST(42, "v67") FES_RS_ST(43, "v68") \
    FES_RS_ST(44, "v69") FES_RS_ST(45, "v70") FES_RS_ST(46, "v71") FES_RS_ST(47, "v72") \
    FES_RS_ST(48, "v73") FES_RS_ST(49, "v74") FES_RS_ST(50, "v75") FES_RS_ST(51, "v76") \
    FES_RS_ST(52, "v77") FES_RS_ST(53, "v78") FES_RS_ST(54, "v79") FES_RS_ST(55, "v80") \
    FES_RS_ST(56, "v81") FES_RS_ST(57, "v82") FES_RS_ST(58, "v83") FES_RS_ST(59, "v84") \
    FES_RS_ST(60, "v85") FES_RS_ST(61, "v86") FES_RS_ST(62, "v87") \
    ""

#define FES_RS_PASS_ASM                                                                                   \
    "v_mov_b32 v24, 0\n"                                                                                  \
    "global_store_dword %[off], v24, %[sig] nt\n"                                                         \
    "s_mov_b64 s[98:99], %[pi]\n"                                                                         \
    FES_RS_LOADS                                                                                          \
    "fes_rs_ld_done_%=:\n"                                                                                \
    "s_waitcnt vmcnt(0)\n"                                                                                \
    "s_add_u32 s92, %[sig_lo], %[wb_lo]\n"                                                                \
    "s_addc_u32 s93, %[sig_hi], %[wb_hi]\n"                                                               \
    FES_RS_STORES                                                                                         \
    "fes_rs_st_done_%=:\n"                                                                                \
    "s_mov_b64 s[94:95], %[prog]\n"                                                                       \
    "s_sub_u32 s96, %[nb], 1\n"                                                                           \
    FES_RG_LOAD_A("0x0", "0x40", "0x60")                                                                  \
    "fes_rs_loop_%=:\n"                                                                                   \
    "s_waitcnt lgkmcnt(0)\n"                                                                              \
    FES_RG_LOAD_B("0x70", "0xb0", "0xd0")                                                                 \
    FES_RS_BUF_A                                                                                          \
    "s_sub_u32 s96, s96, 1\n"                                                                             \
    "s_cbranch_scc1 fes_rs_end_%=\n"                                                                      \
    "s_waitcnt lgkmcnt(0)\n"                                                                              \
    FES_RG_LOAD_A("0xe0", "0x120", "0x140")                                                               \
    FES_RS_BUF_B                                                                                          \
    "s_add_u32 s94, s94, 224\n"                                                                           \
    "s_addc_u32 s95, s95, 0\n"                                                                            \
    "s_sub_u32 s96, s96, 1\n"                                                                             \
    "s_cbranch_scc0 fes_rs_loop_%=\n"                                                                     \
    "fes_rs_end_%=:\n"                                                                                    \
    "s_waitcnt lgkmcnt(0)\n"

template <int R>
__device__ __forceinline__ void sim_regs_pass(const uint32_t* prog, uint32_t nb, uint32_t n, const uint32_t* pi,
                                              uint32_t* sig, uint32_t sig_lo, uint32_t sig_hi, uint32_t wb_lo,
                                              uint32_t wb_hi, uint32_t off) {
#define FES_RS_OPERANDS                                                                                   \
    :                                                                                                     \
    : [prog] "s"(prog), [nb] "s"(nb), [n] "s"(n), [pi] "s"(pi), [sig] "s"(sig), [sig_lo] "s"(sig_lo),      \
      [sig_hi] "s"(sig_hi), [wb_lo] "s"(wb_lo), [wb_hi] "s"(wb_hi), [off] "v"(off)
    if constexpr (R == 104) {
        asm volatile(FES_RS_PASS_ASM FES_RS_OPERANDS : "memory", FES_RG_SCLOB, FES_RG_VCLOB_104);
    } else if constexpr (R == 144) {
        asm volatile(FES_RS_PASS_ASM FES_RS_OPERANDS : "memory", FES_RG_SCLOB, FES_RG_VCLOB_144);
    } else {
        asm volatile(FES_RS_PASS_ASM FES_RS_OPERANDS : "memory", FES_RG_SCLOB, FES_RG_VCLOB_232);
    }
#undef FES_RS_OPERANDS
}

template <int R, int kWaves>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kWaves, kWaves)))
es_sim_regs_kernel(InterpLaunch L) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t waves = gridDim.x;
    const uint32_t nclaim = waves < kClaimCounters ? waves : kClaimCounters;
    const uint32_t claim = __builtin_amdgcn_readfirstlane(blockIdx.x % nclaim);
    unsigned long long* const counter = &L.ctl->next_item[claim * kClaimStride];
    const FES_CONST ConeDesc* c = as_const(L.cones);
    const uint32_t n = __builtin_amdgcn_readfirstlane(c->n_inputs);
    const uint32_t nb = __builtin_amdgcn_readfirstlane(c->n_instr / 4u);
    const uint32_t* prog = (const uint32_t*)c->prog;
    const uint64_t W = L.sim_words, tile = c->tile_hw;
    const uint64_t wb = W * 4u;
    const uint64_t sig = (uint64_t)L.sim_sig;
    for (;;) {
        const uint64_t k = uniform64(atomicAdd(counter, lane == 0 ? 1ull : 0ull));
        const uint64_t item = claim + k * nclaim;
        if (item >= L.total_items) break;
        const uint64_t hw0 = item * tile, hw_stop = min(hw0 + tile, W);
        for (uint64_t base = hw0; base < hw_stop; base += 64u) {
            const uint64_t w = base + lane;
            if (w < W)
                sim_regs_pass<R>(prog, nb, n, L.sim_pi, L.sim_sig, (uint32_t)sig, (uint32_t)(sig >> 32), (uint32_t)wb,
                                 (uint32_t)(wb >> 32), (uint32_t)(w * 4u));
        }
    }
}

template <int R, int kWaves>
hipError_t launch_sim_regs_t(const InterpLaunch& L, int grid, hipStream_t stream) {
    hipLaunchKernelGGL((es_sim_regs_kernel<R, kWaves>), dim3(grid), dim3(64), 0, stream, L);
    return hipGetLastError();
}

}  // namespace

int interp_regs_rows(uint32_t rows, int* waves_per_simd) {
    int w = 0, r = 0;
    if (rows <= 104) { r = 104; w = 4; }
    else if (rows <= 144) { r = 144; w = 3; }
    else if (rows <= 232) { r = 232; w = 2; }
    if (waves_per_simd) *waves_per_simd = w;
    return r;
}

hipError_t launch_interp_regs(const InterpLaunch& L, int regs, int grid, hipStream_t stream) {
    if (L.num_cones == 0 || grid <= 0 || L.rows_max > (uint32_t)regs) return hipErrorInvalidValue;
    switch (regs) {
        case 104: return launch_regs<104, 4>(L, grid, stream);
        case 144: return launch_regs<144, 3>(L, grid, stream);
        case 232: return launch_regs<232, 2>(L, grid, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sim_regs(const InterpLaunch& L, int regs, int grid, hipStream_t stream) {
    if (L.num_cones != 1 || !L.sim_sig || grid <= 0 || L.rows_max > (uint32_t)regs) return hipErrorInvalidValue;
    if (L.sim_words == 0 || L.sim_words > (1ull << 30)) return hipErrorInvalidValue;  // 32-bit byte offsets
    switch (regs) {
        case 104: return launch_sim_regs_t<104, 4>(L, grid, stream);
        case 144: return launch_sim_regs_t<144, 3>(L, grid, stream);
        case 232: return launch_sim_regs_t<232, 2>(L, grid, stream);
        default: return hipErrorInvalidValue;
    }
}

size_t interp_lds_bytes(uint32_t rows, int K, int waves_per_block) {
    return (size_t)waves_per_block * rows * 64u * (size_t)K * sizeof(uint32_t);
}

hipError_t launch_interp_sim(const InterpLaunch& L, int K, int B, bool lds, int grid, int block, hipStream_t stream) {
    if (L.num_cones != 1 || !L.sim_sig || grid <= 0 || block <= 0 || block % 64) return hipErrorInvalidValue;
    if (B == 8) {
        switch (K) {
            case 1: return launch_sim_kb<1, 8>(L, lds, grid, block, stream);
            case 2: return launch_sim_kb<2, 8>(L, lds, grid, block, stream);
            case 4: return launch_sim_kb<4, 8>(L, lds, grid, block, stream);
            default: return hipErrorInvalidValue;
        }
    }
    if (B == 16) {
        switch (K) {
            case 1: return launch_sim_kb<1, 16>(L, lds, grid, block, stream);
            case 2: return launch_sim_kb<2, 16>(L, lds, grid, block, stream);
            default: return hipErrorInvalidValue;  // K = 4 with 16-gate bundles spills registers
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_interp(const InterpLaunch& L, int K, int B, bool lds, int grid, int block, hipStream_t stream) {
    if (L.num_cones == 0 || grid <= 0 || block <= 0 || block % 64) return hipErrorInvalidValue;
    switch (K) {
        case 1: return launch_k<1>(L, B, lds, grid, block, stream);
        case 2: return launch_k<2>(L, B, lds, grid, block, stream);
        case 4: return launch_k<4>(L, B, lds, grid, block, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fes
