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

}  // namespace

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
