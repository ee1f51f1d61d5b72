// Exact simulation without device allocation, for callers that cannot allocate (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The interpreter kernel (value files in LDS) runs exactly as for a plain check; only the
// memory it is handed differs.  Its control block (claim counters), the best-so-far value,
// the cone descriptor and a copy of the circuit's instruction stream live in one file-scope
// device array of fixed size instead of pooled hipMalloc buffers.  The array's device
// address is looked up once per device at the library's device set-up; host code only ever
// uses that address.  Every call on a device shares the device's one array, so calls are
// serialised per device by a host lock, and each call rewrites everything it reads: the
// control block is uploaded zeroed together with best and the descriptor, and the stream is
// uploaded after them, all in stream order before the launch.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>

#include "runtime.hpp"

namespace fes {
namespace {

constexpr size_t kScratchBytes = FASTLEC_NOALLOC_SCRATCH_BYTES;

// Control block, best value, descriptor and instruction stream of fastlec_es_check_noalloc.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// Layout of the scratch array.
constexpr size_t kBestOff = sizeof(LaunchCtl);
constexpr size_t kDescOff = (kBestOff + 8 + 63) & ~size_t(63);
constexpr size_t kProgOff = (kDescOff + sizeof(ConeDesc) + 255) & ~size_t(255);
static_assert(kProgOff < kScratchBytes, "scratch holds the control block and descriptor");

// Host staging of everything before the stream (about 2.4 KB).
struct alignas(256) Head {
    uint8_t bytes[kProgOff];
};

}  // namespace

void noalloc_setup(Device& dev) {
    // The caller (device set-up) has made dev.ordinal the current device.
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        dev.noalloc_scratch = nullptr;  // the no-allocation entry point then reports the error
        trace("device %d: no address for the no-allocation scratch (%s)", dev.ordinal, hipGetErrorString(e));
        return;
    }
    dev.noalloc_scratch = p;
}

uint64_t noalloc_check(Device& dev, Circuit& c, const fastlec_es_options& o, const HwRange& r, hipStream_t stream,
                       double* ms) {
    if (!dev.noalloc_scratch) throw Error{kErrDevice, "no-allocation scratch array has no device address"};
    // The schedule of a plain check, then the size limit of its stream, then the tier: value
    // files in VGPRs or LDS only.
    std::vector<Circuit*> one{&c};
    const Schedule sch = default_schedule(dev, one, &o);
    const Plan& p = c.plan_for((uint32_t)sch.B);
    // the register tier runs its own encoding of the stream, the other tiers the plan's
    const void* prog_src = sch.regs ? (const void*)c.regs_stream().data() : (const void*)p.prog.data();
    const size_t prog_bytes = sch.regs ? c.regs_stream().size() * sizeof(uint32_t) : p.prog.size() * sizeof(Instr);
    if (kProgOff + prog_bytes > kScratchBytes)
        throw Error{kErrInvalid, "instruction stream of " + std::to_string(p.prog.size()) + " instructions (" +
                                     std::to_string(prog_bytes) + " bytes) exceeds the no-allocation scratch (" +
                                     std::to_string(kScratchBytes - kProgOff) + " bytes)"};
    if (!sch.lds && !sch.regs)
        throw Error{kErrInvalid, "value file does not fit in LDS with this schedule; the no-allocation entry point "
                                 "has no device-memory value files"};
    std::lock_guard<std::mutex> g(dev.noalloc_mu);
    uint8_t* base = (uint8_t*)dev.noalloc_scratch;
    Head head;
    std::memset(head.bytes, 0, sizeof(head.bytes));
    uint64_t best = ~0ull;
    std::memcpy(head.bytes + kBestOff, &best, 8);
    Schedule s = sch;
    if (o.tile_words) s.tile_hw = 2ull * o.tile_words;
    ConeDesc d;
    const uint64_t items = fill_desc(p, (const Instr*)(base + kProgOff), r, 0, s, 0, d);
    std::memcpy(head.bytes + kDescOff, &d, sizeof(d));

    InterpLaunch L;
    L.cones = (const ConeDesc*)(base + kDescOff);
    L.num_cones = 1;
    L.rows_max = p.rows;
    L.total_items = items;
    L.ctl = (LaunchCtl*)base;
    L.best = (unsigned long long*)(base + kBestOff);
    L.hbm_rows = nullptr;
    L.cancel = nullptr;
    trace("noalloc launch: %llu items, K=%d B=%d grid=%d block=%d rows=%u", (unsigned long long)items, s.K, s.B,
          s.grid, s.block, p.rows);
    const auto t0 = std::chrono::steady_clock::now();
    FES_HIP(hipMemcpyAsync(base, head.bytes, sizeof(head.bytes), hipMemcpyHostToDevice, stream));
    if (prog_bytes)
        FES_HIP(hipMemcpyAsync(base + kProgOff, prog_src, prog_bytes, hipMemcpyHostToDevice, stream));
    FES_HIP(launch_schedule(L, s, stream));
    FES_HIP(hipMemcpyAsync(&best, base + kBestOff, 8, hipMemcpyDeviceToHost, stream));
    FES_HIP(hipStreamSynchronize(stream));
    if (ms) *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return best;
}

}  // namespace fes
