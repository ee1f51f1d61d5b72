// A host-only stand-in for the GPU, for running the library's host code under ThreadSanitizer
// on a machine without one.  Test infrastructure only: it is linked into the sanitizer drivers
// in this directory, never into the library.
//
// It provides the HIP runtime calls the host code makes (one device; memory from the C heap;
// copies and launches run synchronously on the calling thread; events read a host clock) and the
// library's kernel entry points, evaluated on the CPU from the same descriptors and instruction
// streams the GPU kernels read:
//   * the interpreter (16-byte instructions in bundles of B, or the register tier's 28-word
//     bundles: all reads of a bundle, then all writes), over each cone's work items in order,
//     lowering best[] to the lowest failing pattern;
//   * the specialized kernel, as the circuit's LUT program (eval_lut_program), "compiled" by a
//     short sleep so the server's compile thread overlaps its step loop.
// Entry points the race drivers do not reach (simulation, hashing, batch graphs, the
// no-allocation check, the issue-rate probe) throw.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "kernels.hpp"
#include "runtime.hpp"

namespace {

struct FakeEvent {
    std::chrono::steady_clock::time_point t;
};

thread_local int g_device = 0;  // the current device is per host thread, as in HIP

uint32_t pi_word(uint32_t i, uint64_t hw) {
    static const uint32_t kc[5] = {0xAAAAAAAAu, 0xCCCCCCCCu, 0xF0F0F0F0u, 0xFF00FF00u, 0xFFFF0000u};
    return i < 5 ? kc[i] : 0u - (uint32_t)((hw >> (i - 5)) & 1u);
}

// Miter word of one half-word from a 16-byte-instruction stream in bundles of B.
uint32_t eval_instrs(const fes::ConeDesc& c, uint32_t B, uint64_t hw, std::vector<uint32_t>& rows) {
    rows.assign(std::max<uint32_t>(c.rows, 1), 0u);
    for (uint32_t i = 0; i < c.n_inputs; ++i) rows[1 + i] = pi_word(i, hw);
    uint32_t m = 0;
    std::vector<uint32_t> val(B);
    for (uint32_t t = 0; t < c.n_instr; t += B) {
        for (uint32_t u = 0; u < B; ++u) {
            const fes::Instr& ins = c.prog[t + u];
            const uint32_t a = rows[ins.a & fes::kRowMask] ^ (0u - (ins.a >> 31));
            const uint32_t b = rows[ins.b & fes::kRowMask] ^ (0u - (ins.b >> 31));
            val[u] = (ins.flags & fes::kXor) ? a ^ b : a & b;
        }
        for (uint32_t u = 0; u < B; ++u) {
            const fes::Instr& ins = c.prog[t + u];
            rows[ins.d] = val[u];
            if (ins.flags & fes::kOutPos) m |= val[u];
            if (ins.flags & fes::kOutNeg) m |= ~val[u];
        }
    }
    return m;
}

// The same from the register tier's encoded stream (row = low 8 bits; masks in the stream).
uint32_t eval_regs(const fes::ConeDesc& c, uint64_t hw, std::vector<uint32_t>& rows) {
    rows.assign(256, 0u);
    for (uint32_t i = 0; i < c.n_inputs; ++i) rows[1 + i] = pi_word(i, hw);
    const uint32_t* s = (const uint32_t*)c.prog;
    uint32_t m = 0;
    for (uint32_t b = 0; b < c.n_instr / 4; ++b) {
        const uint32_t* w = s + (size_t)b * fes::kRegsBundleWords;
        uint32_t val[4];
        for (int u = 0; u < 4; ++u) {
            const uint32_t x = rows[w[u] & 0xFFu] ^ w[12 + u], y = rows[w[4 + u] & 0xFFu] ^ w[16 + u];
            val[u] = (w[20 + u] & (x ^ y)) | (~w[20 + u] & x & y);
        }
        const bool marked = (w[8] >> 31) != 0;
        for (int u = 0; u < 4; ++u) {
            rows[w[8 + u] & 0xFFu] = val[u];
            if (marked && (w[24 + u] & fes::kOutPos)) m |= val[u];
            if (marked && (w[24 + u] & fes::kOutNeg)) m |= ~val[u];
        }
    }
    return m;
}

// Every cone's work items in ascending order, as the kernels' claims would take them.
template <class Eval>
void run_cones(const fes::InterpLaunch& L, Eval eval) {
    std::vector<uint32_t> rows;
    for (uint32_t k = 0; k < L.num_cones; ++k) {
        const fes::ConeDesc& c = L.cones[k];
        unsigned long long& best = L.best[c.best_index];
        bool found = false;
        for (uint64_t item = c.item_begin; item < c.item_end && !found; ++item) {
            const uint64_t hw0 = c.hw_first + (item - c.item_begin) * c.tile_hw;
            const uint64_t hw_stop = std::min(hw0 + c.tile_hw, c.hw_end);
            for (uint64_t hw = std::max(hw0, c.hw_begin); hw < hw_stop; ++hw) {
                if (32ull * hw >= best) {
                    found = true;
                    break;
                }
                const uint32_t m = eval(c, hw, rows);
                if (m) {
                    best = std::min<unsigned long long>(best, 32ull * hw + (unsigned)__builtin_ctz(m));
                    found = true;
                    break;
                }
            }
        }
    }
}

struct FakeJit {
    fes::Circuit* c = nullptr;
};
std::mutex g_jit_mu;
std::map<std::pair<uint64_t, int>, std::shared_ptr<fes::JitKernel>> g_jit;  // (circuit uid, waves) -> kernel
std::map<const fes::JitKernel*, fes::Circuit*> g_jit_circuit;

std::shared_ptr<fes::JitKernel> fake_compile(fes::Circuit& c, int waves) {
    {
        std::lock_guard<std::mutex> g(g_jit_mu);
        auto it = g_jit.find({c.uid, waves});
        if (it != g_jit.end()) return it->second;
    }
    (void)c.lut_program();
    std::this_thread::sleep_for(std::chrono::milliseconds(3));  // the compile
    auto k = std::make_shared<fes::JitKernel>();
    k->waves_per_eu = k->waves_used = waves;
    k->code = std::make_shared<fes::CodeObject>();
    std::lock_guard<std::mutex> g(g_jit_mu);
    auto& slot = g_jit[{c.uid, waves}];
    if (!slot) {
        slot = k;
        g_jit_circuit[k.get()] = &c;
    }
    return slot;
}

}  // namespace

extern "C" {

hipError_t hipGetDeviceCount(int* n) {
    *n = 1;
    return hipSuccess;
}
hipError_t hipSetDevice(int d) {
    g_device = d;
    return d == 0 ? hipSuccess : hipErrorInvalidDevice;
}
hipError_t hipGetDevice(int* d) {
    *d = g_device;
    return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600* p, int) {
    std::memset(p, 0, sizeof(*p));
    std::strcpy(p->name, "host stand-in");
    std::strcpy(p->gcnArchName, "gfx950");
    p->multiProcessorCount = 4;
    p->maxSharedMemoryPerMultiProcessor = 160 * 1024;
    p->sharedMemPerBlock = 64 * 1024;
    p->warpSize = 64;
    p->maxThreadsPerBlock = 1024;
    p->totalGlobalMem = size_t(16) << 30;
    p->clockRate = 2400000;
    return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "host stand-in error"; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
    static int dummy[64];
    static std::atomic<int> next{0};
    *s = (hipStream_t)&dummy[next.fetch_add(1) % 64];
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipMalloc(void** p, size_t n) {
    *p = std::calloc(1, std::max<size_t>(n, 1));
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
    std::free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) {
    *p = std::calloc(1, std::max<size_t>(n, 1));
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
    if (n) std::memmove(d, s, n);
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
    *e = (hipEvent_t) new FakeEvent();
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    delete (FakeEvent*)e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    ((FakeEvent*)e)->t = std::chrono::steady_clock::now();
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    *ms = std::chrono::duration<float, std::milli>(((FakeEvent*)b)->t - ((FakeEvent*)a)->t).count();
    return hipSuccess;
}

}  // extern "C"

namespace fes {

int interp_regs_rows(uint32_t rows, int* waves_per_simd) {
    int w = 0, r = 0;
    if (rows <= 104) { r = 104; w = 4; }
    else if (rows <= 144) { r = 144; w = 3; }
    else if (rows <= 232) { r = 232; w = 2; }
    if (waves_per_simd) *waves_per_simd = w;
    return r;
}
size_t interp_lds_bytes(uint32_t rows, int K, int waves_per_block) {
    return (size_t)waves_per_block * rows * 64u * (size_t)K * sizeof(uint32_t);
}
hipError_t launch_interp(const InterpLaunch& L, int, int B, bool, int, int, hipStream_t) {
    run_cones(L, [B](const ConeDesc& c, uint64_t hw, std::vector<uint32_t>& rows) {
        return eval_instrs(c, (uint32_t)B, hw, rows);
    });
    return hipSuccess;
}
hipError_t launch_interp_regs(const InterpLaunch& L, int regs, int, hipStream_t) {
    if (L.rows_max > (uint32_t)regs) return hipErrorInvalidValue;
    run_cones(L, eval_regs);
    return hipSuccess;
}
hipError_t launch_interp_sim(const InterpLaunch&, int, int, bool, int, int, hipStream_t) {
    throw Error{kErrDevice, "host stand-in: no simulation"};
}
hipError_t launch_sim_regs(const InterpLaunch&, int, int, hipStream_t) {
    throw Error{kErrDevice, "host stand-in: no simulation"};
}
hipError_t launch_signature_hash(const uint32_t*, uint64_t, uint64_t, uint64_t*, uint64_t*, int, hipStream_t) {
    throw Error{kErrDevice, "host stand-in: no hashing"};
}
void noalloc_setup(Device& dev) { dev.noalloc_scratch = nullptr; }
uint64_t noalloc_check(Device&, Circuit&, const fastlec_es_options&, const HwRange&, hipStream_t, double*) {
    throw Error{kErrDevice, "host stand-in: no no-allocation check"};
}
double valu_probe(Device&, uint32_t, uint32_t, uint32_t, hipStream_t, double*) {
    throw Error{kErrDevice, "host stand-in: no probe"};
}
// Batches: the default schedule instead of timed candidates, and the grouped launch as one
// interpreter run over the group's cones (evaluated on the host like any launch here).
Schedule autotune(Device& dev, const std::vector<Circuit*>& cs, const std::vector<HwRange>&, hipStream_t, bool) {
    return default_schedule(dev, cs, nullptr);
}
void run_batch_graph(Device& dev, const std::vector<Circuit*>& cs, const std::vector<HwRange>& rs, const Schedule& sch,
                     hipStream_t stream, std::vector<uint64_t>& best, double* ms) {
    run_interp(dev, cs, rs, sch, stream, nullptr, best, ms);
}

int specialized_waves_per_eu() { return 3; }
int specialized_scalar_policy() { return 0; }
std::string jit_source(const LutProgram&, int, int, int* waves_used) {
    if (waves_used) *waves_used = 3;
    return std::string();
}
std::shared_ptr<JitKernel> jit_kernel(Circuit& c, int waves_per_eu, double* compile_ms) {
    if (compile_ms) *compile_ms = 3.0;
    return fake_compile(c, waves_per_eu);
}
// Three compile threads in the server, as with helper processes.
int compile_helpers() { return 3; }

std::vector<std::shared_ptr<JitKernel>> jit_kernels(const std::vector<Circuit*>& cs, int waves_per_eu,
                                                    std::vector<double>* compile_ms, CompileSplit) {
    std::vector<std::shared_ptr<JitKernel>> out;
    for (Circuit* c : cs) out.push_back(fake_compile(*c, waves_per_eu));
    if (compile_ms) compile_ms->assign(cs.size(), 3.0);
    return out;
}
std::shared_ptr<JitKernel> jit_ready(Circuit& c, int waves_per_eu) {
    std::lock_guard<std::mutex> g(g_jit_mu);
    auto it = g_jit.find({c.uid, waves_per_eu});
    return it == g_jit.end() ? nullptr : it->second;
}
JitLaunchPlan jit_prepare(Device&, JitKernel& k, const HwRange& r, uint64_t) {
    JitLaunchPlan lp;
    {
        std::lock_guard<std::mutex> g(g_jit_mu);
        lp.fn = (hipFunction_t)g_jit_circuit.at(&k);
    }
    lp.hw_begin = r.begin;
    lp.hw_end = r.end;
    return lp;
}
void jit_enqueue(const JitLaunchPlan& lp, uint64_t*, uint64_t* best, const int*, hipStream_t) {
    Circuit& c = *(Circuit*)lp.fn;
    const LutProgram& prog = c.lut_program();
    for (uint64_t hw = lp.hw_begin; hw < lp.hw_end; ++hw) {
        if (32ull * hw >= *best) return;
        const uint32_t m = eval_lut_program(prog, hw);
        if (m) {
            *best = std::min<uint64_t>(*best, 32ull * hw + (unsigned)__builtin_ctz(m));
            return;
        }
    }
}
void run_jit(Device&, Circuit& c, JitKernel&, const HwRange& r, uint64_t, hipStream_t, const int*, uint64_t* best,
             double* kernel_ms, DevMem) {
    const LutProgram& prog = c.lut_program();
    uint64_t b = ~0ull;
    for (uint64_t hw = r.begin; hw < r.end; ++hw) {
        const uint32_t m = eval_lut_program(prog, hw);
        if (m) {
            b = 32ull * hw + (unsigned)__builtin_ctz(m);
            break;
        }
    }
    *best = b;
    if (kernel_ms) *kernel_ms = 0;
}

CodeObject::~CodeObject() = default;
hipModule_t CodeObject::module(int) { return nullptr; }

}  // namespace fes
