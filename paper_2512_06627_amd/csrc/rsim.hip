// Signature hashing for random-pattern simulation (gfx950).
//
// A sweeping flow proposes potentially equivalent node pairs from simulation
// signatures (paper, Section 2.3, step 1); a node and its complement are the
// same candidate, so each row is normalised to start with a 0 before it is
// hashed.  Row r of the signature matrix is hashed as
//     sum over words k of word'_k * (fmix32(k) | 1)   (mod 2^64)
// with word' = word XOR (all ones if bit 0 of word 0 is 1), fmix32 the
// MurmurHash3 32-bit finaliser (keys use k mod 2^32), and each product the
// exact 64-bit product of two 32-bit values.  The sum is order-free, so each
// lane accumulates its own words and one wave reduction finishes the row.
// The row's number of ones (before normalisation) is summed alongside; the
// paper's stability and entropy features (Section 3.2) derive from it.
//
// Work decomposition: one wave per row, rows taken grid-stride.  Each lane
// reads words lane, lane+64, ... (every wave load is 256 contiguous bytes);
// four independent loads are in flight per lane per iteration.  The kernel is
// bound by HBM reads: about 12 vector instructions per 64 words against 256
// bytes of traffic.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fes {
namespace {

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

__global__ void __launch_bounds__(256) signature_hash_kernel(const uint32_t* __restrict__ sig, uint64_t rows,
                                                             uint64_t W, uint64_t* __restrict__ hash,
                                                             uint64_t* __restrict__ ones) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t r = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < rows; r += waves) {
        const uint32_t* row = sig + r * W;
        const uint32_t flip = 0u - (__builtin_amdgcn_readfirstlane(row[0]) & 1u);
        uint64_t acc = 0, cnt = 0;
        uint64_t k = lane;
        for (; k + 192 < W; k += 256) {
            uint32_t w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) w[u] = row[k + 64 * u];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc += (uint64_t)(w[u] ^ flip) * (uint64_t)(fmix32((uint32_t)(k + 64 * u)) | 1u);
                cnt += (uint32_t)__builtin_popcount(w[u]);
            }
        }
        for (; k < W; k += 64) {
            const uint32_t w = row[k];
            acc += (uint64_t)(w ^ flip) * (uint64_t)(fmix32((uint32_t)k) | 1u);
            cnt += (uint32_t)__builtin_popcount(w);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            acc += __shfl_xor(acc, off, 64);
            cnt += __shfl_xor(cnt, off, 64);
        }
        if (lane == 0) {
            hash[r] = acc;
            ones[r] = cnt;
        }
    }
}

}  // namespace

hipError_t launch_signature_hash(const uint32_t* sig, uint64_t rows, uint64_t words, uint64_t* hash,
                                 uint64_t* ones, int grid, hipStream_t stream) {
    if (!sig || !hash || !ones || rows == 0 || words == 0 || grid <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(signature_hash_kernel, dim3(grid), dim3(256), 0, stream, sig, rows, words, hash, ones);
    return hipGetLastError();
}

}  // namespace fes
