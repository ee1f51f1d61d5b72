// Issue-rate probe of the integer VALU on gfx950: the measured side of the roofline the
// specialized kernel is held against.  The specialized kernel is a straight-line stream of
// v_bitop3_b32 (one three-input LUT per instruction) whose operands are VGPRs, SGPRs
// (wave-uniform inputs) or constants, so the probe runs that instruction in three operand
// forms, each as 16 independent chains of 4 registers (v0..v63; a result is read 16
// instructions later) in one asm block per wave, 256 instructions per loop iteration with one
// scalar decrement and branch:
//   variant 0: v_bitop3_b32 with three VGPR sources, in three different register banks
//              (bank = register number mod 4);
//   variant 1: v_bitop3_b32 with two VGPR sources and one SGPR source;
//   variant 2: v_xor_b32 (two VGPR sources).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <string>

#include "runtime.hpp"

// 16 chains x 4 steps per round, 4 rounds per loop iteration.
constexpr int kInstrPerIter = 16 * 4 * 4;

#define FES_V(n) "v" #n
#define FES_B3(d, a, b, c) "v_bitop3_b32 " FES_V(d) ", " FES_V(a) ", " FES_V(b) ", " FES_V(c) " bitop3:0x96\n"
#define FES_B3S(d, a, b) "v_bitop3_b32 " FES_V(d) ", " FES_V(a) ", " FES_V(b) ", %[u] bitop3:0x96\n"
#define FES_X2(d, a, b) "v_xor_b32 " FES_V(d) ", " FES_V(a) ", " FES_V(b) "\n"
// step j of a chain whose registers are r0..r3 writes r_j from the chain's other registers
#define FES_V0_STEP0(r0, r1, r2, r3) FES_B3(r0, r1, r2, r3)
#define FES_V0_STEP1(r0, r1, r2, r3) FES_B3(r1, r0, r2, r3)
#define FES_V0_STEP2(r0, r1, r2, r3) FES_B3(r2, r0, r1, r3)
#define FES_V0_STEP3(r0, r1, r2, r3) FES_B3(r3, r0, r1, r2)
#define FES_V1_STEP0(r0, r1, r2, r3) FES_B3S(r0, r1, r2)
#define FES_V1_STEP1(r0, r1, r2, r3) FES_B3S(r1, r2, r3)
#define FES_V1_STEP2(r0, r1, r2, r3) FES_B3S(r2, r3, r0)
#define FES_V1_STEP3(r0, r1, r2, r3) FES_B3S(r3, r0, r1)
#define FES_V2_STEP0(r0, r1, r2, r3) FES_X2(r0, r1, r2)
#define FES_V2_STEP1(r0, r1, r2, r3) FES_X2(r1, r2, r3)
#define FES_V2_STEP2(r0, r1, r2, r3) FES_X2(r2, r3, r0)
#define FES_V2_STEP3(r0, r1, r2, r3) FES_X2(r3, r0, r1)
#define FES_ALL_CHAINS(S)                                                                             \
    S(0, 1, 2, 3) S(4, 5, 6, 7) S(8, 9, 10, 11) S(12, 13, 14, 15) S(16, 17, 18, 19) S(20, 21, 22, 23)  \
    S(24, 25, 26, 27) S(28, 29, 30, 31) S(32, 33, 34, 35) S(36, 37, 38, 39) S(40, 41, 42, 43)          \
    S(44, 45, 46, 47) S(48, 49, 50, 51) S(52, 53, 54, 55) S(56, 57, 58, 59) S(60, 61, 62, 63)
#define FES_ROUND(V)                       \
    FES_ALL_CHAINS(FES_##V##_STEP0)        \
    FES_ALL_CHAINS(FES_##V##_STEP1)        \
    FES_ALL_CHAINS(FES_##V##_STEP2)        \
    FES_ALL_CHAINS(FES_##V##_STEP3)
#define FES_INIT1(r) "v_xor_b32 " FES_V(r) ", " #r ", %[seed]\n"
#define FES_INIT4(a, b, c, d) FES_INIT1(a) FES_INIT1(b) FES_INIT1(c) FES_INIT1(d)
#define FES_FOLD1(r) "v_xor_b32 %[acc], %[acc], " FES_V(r) "\n"
#define FES_FOLD4(a, b, c, d) FES_FOLD1(a) FES_FOLD1(b) FES_FOLD1(c) FES_FOLD1(d)
#define FES_PROBE_ASM(V)                                                                                          \
    asm volatile(FES_ALL_CHAINS(FES_INIT4) "s_mov_b32 %[cnt], %[iters]\n"                                        \
                 "fes_probe_loop_%=:\n" FES_ROUND(V) FES_ROUND(V) FES_ROUND(V) FES_ROUND(V)                      \
                 "s_sub_u32 %[cnt], %[cnt], 1\n"                                                                  \
                 "s_cmp_lg_u32 %[cnt], 0\n"                                                                       \
                 "s_cbranch_scc1 fes_probe_loop_%=\n" FES_ALL_CHAINS(FES_FOLD4)                                   \
                 : [acc] "+v"(acc), [cnt] "=&s"(cnt)                                                              \
                 : [iters] "s"(iters), [seed] "v"(seed), [u] "s"(uniform)                                         \
                 : "scc", "v0", "v1", "v2", "v3", "v4", "v5", "v6", "v7", "v8", "v9", "v10", "v11", "v12", "v13",   \
                   "v14", "v15", "v16", "v17", "v18", "v19", "v20", "v21", "v22", "v23", "v24", "v25", "v26", "v27", \
                   "v28", "v29", "v30", "v31", "v32", "v33", "v34", "v35", "v36", "v37", "v38", "v39", "v40", "v41", \
                   "v42", "v43", "v44", "v45", "v46", "v47", "v48", "v49", "v50", "v51", "v52", "v53", "v54", "v55", \
                   "v56", "v57", "v58", "v59", "v60", "v61", "v62", "v63")

namespace fes {

template <int kVariant>
__global__ void __launch_bounds__(256) valu_probe_kernel(uint32_t iters, uint32_t* out) {
    uint32_t acc = 0, cnt;
    const uint32_t seed = threadIdx.x * 0x9E3779B9u + blockIdx.x;
    const uint32_t uniform = __builtin_amdgcn_readfirstlane(blockIdx.x * 0x85EBCA6Bu);
    if constexpr (kVariant == 0) {
        FES_PROBE_ASM(V0);
    } else if constexpr (kVariant == 1) {
        FES_PROBE_ASM(V1);
    } else {
        FES_PROBE_ASM(V2);
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace fes

namespace fes {

// Runs probe `variant` with `waves_per_simd` workgroups of four waves per CU (one wave per SIMD
// each); returns wave64 VALU instructions per second of the loop (init and fold excluded).
double valu_probe(Device& dev, uint32_t variant, uint32_t waves_per_simd, uint32_t iters, hipStream_t stream,
                  double* ms_out) {
    if (variant > 2) throw Error{kErrInvalid, "variant must be 0, 1 or 2"};
    if (waves_per_simd < 1 || waves_per_simd > 8) throw Error{kErrInvalid, "waves_per_simd must be 1..8"};
    if (iters < 1) throw Error{kErrInvalid, "iters must be positive"};
    const int cus = dev.prop.multiProcessorCount;
    const int grid = cus * (int)waves_per_simd;
    const int block = 256;
    Buffer buf = dev.acquire((size_t)grid * block * 4, 0);
    struct Releaser {
        Device& d;
        Buffer b;
        ~Releaser() { d.release(b); }
    } rel{dev, buf};
    ScopedEvent e0, e1;
    FES_HIP(hipEventRecord(e0.e, stream));
    uint32_t* out = (uint32_t*)buf.dev;
    if (variant == 0) hipLaunchKernelGGL(valu_probe_kernel<0>, dim3(grid), dim3(block), 0, stream, iters, out);
    else if (variant == 1) hipLaunchKernelGGL(valu_probe_kernel<1>, dim3(grid), dim3(block), 0, stream, iters, out);
    else hipLaunchKernelGGL(valu_probe_kernel<2>, dim3(grid), dim3(block), 0, stream, iters, out);
    FES_HIP(hipGetLastError());
    FES_HIP(hipEventRecord(e1.e, stream));
    FES_HIP(hipStreamSynchronize(stream));
    float ms = 0;
    FES_HIP(hipEventElapsedTime(&ms, e0.e, e1.e));
    if (ms_out) *ms_out = ms;
    const double instr = (double)grid * (block / 64) * (double)iters * kInstrPerIter;
    return ms > 0 ? instr / (ms / 1e3) : 0.0;
}

}  // namespace fes
