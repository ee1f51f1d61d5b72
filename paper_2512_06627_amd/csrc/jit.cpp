// Specialized exact-simulation kernel: the circuit becomes straight-line code.
//
// The paper keeps the compiled instruction stream in the constant cache and
// each thread's bit-vector registers in shared memory, and finds the kernel
// bound by memory traffic (Section 3.3).  On gfx950 the circuit itself is
// compiled into the kernel: every planner slot is a 32-bit register variable,
// so a gate is one VALU operation on register operands (v_and_b32, v_bfi_b32
// or v_bitop3_b32 for complemented fanins) and no node value ever leaves the
// register file.  Primary inputs come from the pattern index: inputs 0..4 are
// constants inside a 32-bit word, inputs 5..10 are lane bits, inputs 11.. are
// bits of the wave's base index and so live in SGPRs, where gates whose
// fanins are all wave-uniform run on the scalar unit.
//
// The source is compiled once per circuit with hipRTC for gfx950 and cached.
#include <hip/hiprtc.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <sstream>

#include "runtime.hpp"

namespace fes {
namespace {

uint64_t fnv1a(const std::string& s) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

std::string ref_name(const LutRef& r) {
    switch (r.kind) {
        case LutRef::Word: return "w" + std::to_string(r.index);
        case LutRef::Input: return "x" + std::to_string(r.index);
        case LutRef::Uniform: return "su" + std::to_string(r.index);
        default: return "vr" + std::to_string(r.index);
    }
}

bool is_scalar(const LutRef& r) {
    return r.kind == LutRef::Word || r.kind == LutRef::Uniform || (r.kind == LutRef::Input && r.index >= 11);
}

}  // namespace

std::string jit_source(const LutProgram& lp, int waves_per_eu, int block) {
    std::ostringstream o;
    const uint32_t n = lp.num_inputs;
    o << "// exact simulation, " << n << " inputs: " << lp.lut_steps << " LUT steps, " << lp.scalar_steps
      << " scalar steps, " << lp.absorbed_gates << " gates absorbed into LUTs, " << lp.folded_gates << " folded\n";
    o << "typedef unsigned int u32;\ntypedef unsigned long long u64;\n";
    o << "extern \"C\" __global__ void __launch_bounds__(" << block << ") __attribute__((amdgpu_waves_per_eu("
      << waves_per_eu << ", " << waves_per_eu << ")))\n";
    o << "fes_es_kernel(u64 hw_begin, u64 hw_end, u64 hw_first, u64 tile_hw, u64 total_items,\n"
         "              u64* __restrict__ next_item, u64* __restrict__ best, const int* __restrict__ cancel) {\n";
    o << "  const u32 lane = threadIdx.x & 63u;\n";
    for (uint32_t i = 5; i < n && i < 11; ++i)
        o << "  const u32 x" << i << " = 0u - ((lane >> " << (i - 5) << ") & 1u);\n";
    for (uint32_t i = 0; i < lp.words.size(); ++i) {
        char buf[64];
        std::snprintf(buf, sizeof buf, "  const u32 w%u = 0x%08Xu;\n", i, lp.words[i]);
        o << buf;
    }
    // Control flow stays wave-uniform: every lane takes part in the claim (lane 0 adds 1, the
    // others 0) and in the atomicMin (all lanes hold the same value), so no branch depends on
    // the lane and every loop exit is a scalar branch.
    o << "  for (;;) {\n"
         "    const u64 claimed = atomicAdd(next_item, lane == 0u ? 1ull : 0ull);\n"
         "    const u64 item = ((u64)__builtin_amdgcn_readfirstlane((u32)(claimed >> 32)) << 32) |\n"
         "                     __builtin_amdgcn_readfirstlane((u32)claimed);\n"
         "    if (item >= total_items) break;\n"
         "    if (cancel && __builtin_amdgcn_readfirstlane(__hip_atomic_load(cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))) break;\n"
         "    const u64 hw0 = hw_first + item * tile_hw;\n"
         "    const u64 hw_stop = hw0 + tile_hw < hw_end ? hw0 + tile_hw : hw_end;\n"
         "    for (u64 base = hw0; base < hw_stop; base += 64) {\n"
         "      const u64 b_raw = __hip_atomic_load(best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);\n"
         "      const u64 best_now = ((u64)__builtin_amdgcn_readfirstlane((u32)(b_raw >> 32)) << 32) |\n"
         "                           __builtin_amdgcn_readfirstlane((u32)b_raw);\n"
         "      if (32ull * base >= best_now) break;\n";
    for (uint32_t i = 11; i < n; ++i)
        o << "      const u32 x" << i << " = 0u - (u32)((base >> " << (i - 5) << ") & 1ull);\n";
    o << "      u32 m = 0u;\n";
    // Every gate is an inline-asm instruction whose function the planner fixed, so the
    // compiler allocates registers and schedules but never rewrites the logic.  VALU
    // operands: at most one scalar (SGPR) source per instruction; others go through VGPRs.
    char buf[256];
    // Runs of consecutive scalar steps are emitted as one asm block (the compiler pads every
    // asm block with a wait state, so one block per gate would double the scalar issue count).
    // Block outputs are early-clobber: they never share a register with a block input.
    auto flush_scalar = [&](const std::vector<const LutStep*>& run) {
        if (run.empty()) return;
        std::vector<std::string> outs, ins;
        auto in_index = [&](const std::string& name) -> std::string {
            for (size_t i = 0; i < outs.size(); ++i)
                if (outs[i] == name) return "%" + std::to_string(i);
            for (size_t i = 0; i < ins.size(); ++i)
                if (ins[i] == name) return "%" + std::to_string(outs.size() + i);
            return "";
        };
        for (const LutStep* st : run) outs.push_back("su" + std::to_string(st->dst));
        for (const LutStep* st : run)
            for (int j = 0; j < 2; ++j) {
                const std::string nm = ref_name(st->leaf[j]);
                if (in_index(nm).empty()) ins.push_back(nm);
            }
        std::string text;
        for (const LutStep* st : run) {
            const bool na = st->table & 1, nb = (st->table >> 1) & 1;
            std::string a = in_index(ref_name(st->leaf[0])), b = in_index(ref_name(st->leaf[1]));
            const char* opname = "s_and_b32";
            if (na && nb) opname = "s_nor_b32";
            else if (nb) opname = "s_andn2_b32";
            else if (na) { opname = "s_andn2_b32"; std::swap(a, b); }
            text += std::string(text.empty() ? "" : "\\n\\t") + opname + " " + in_index("su" + std::to_string(st->dst)) + ", " + a + ", " + b;
        }
        o << "      u32";
        for (size_t i = 0; i < outs.size(); ++i) o << (i ? ", " : " ") << outs[i];
        o << ";\n      asm(\"" << text << "\" : ";
        for (size_t i = 0; i < outs.size(); ++i) o << (i ? ", " : "") << "\"=&s\"(" << outs[i] << ")";
        o << " : ";
        for (size_t i = 0; i < ins.size(); ++i) o << (i ? ", " : "") << "\"s\"(" << ins[i] << ")";
        o << " : \"scc\");\n";
    };
    std::vector<const LutStep*> run;
    auto run_operands = [&](const LutStep& st) {  // operand count if st joined the run
        std::vector<std::string> names;
        for (const LutStep* r : run) names.push_back("su" + std::to_string(r->dst));
        names.push_back("su" + std::to_string(st.dst));
        auto add = [&](const std::string& nm) {
            if (std::find(names.begin(), names.end(), nm) == names.end()) names.push_back(nm);
        };
        for (const LutStep* r : run) { add(ref_name(r->leaf[0])); add(ref_name(r->leaf[1])); }
        add(ref_name(st.leaf[0]));
        add(ref_name(st.leaf[1]));
        return names.size();
    };
    for (const LutStep& st : lp.steps) {
        if (st.op == LutStep::ScalarAnd) {
            if (!run.empty() && run_operands(st) > 30) {
                flush_scalar(run);
                run.clear();
            }
            run.push_back(&st);
            continue;
        }
        flush_scalar(run);
        run.clear();
        if (st.op == LutStep::Lut) {
            const uint32_t k = st.nleaves;
            const char* fmt = k == 3 ? "%%1, %%2, %%3" : k == 2 ? "%%1, %%2, %%2" : "%%1, %%1, %%1";
            char ops[32];
            std::snprintf(ops, sizeof ops, fmt);
            bool used_s = false;
            std::string cons;
            for (uint32_t j = 0; j < k; ++j) {
                const bool sc = is_scalar(st.leaf[j]) && !used_s;
                used_s |= sc;
                cons += std::string(j ? ", " : "") + (sc ? "\"s\"(" : "\"v\"(") + ref_name(st.leaf[j]) + ")";
            }
            std::snprintf(buf, sizeof buf, "      u32 vr%u; asm(\"v_bitop3_b32 %%0, %s bitop3:0x%02x\" : \"=v\"(vr%u) : %s);\n",
                          st.dst, ops, st.table, st.dst, cons.c_str());
            o << buf;
        } else {
            // m = m | (x ^ neg): table over (m, x, x)
            uint8_t table = 0;
            for (uint32_t idx = 0; idx < 8; ++idx) {
                const uint32_t mm = (idx >> 2) & 1u, x = (idx >> 1) & 1u;
                if (mm | (x ^ (st.out_neg ? 1u : 0u))) table |= (uint8_t)(1u << idx);
            }
            const std::string x = ref_name(st.leaf[0]);
            std::snprintf(buf, sizeof buf, "      asm(\"v_bitop3_b32 %%0, %%1, %%2, %%2 bitop3:0x%02x\" : \"=v\"(m) : \"v\"(m), \"%s\"(%s));\n",
                          table, is_scalar(st.leaf[0]) ? "s" : "v", x.c_str());
            o << buf;
        }
    }
    flush_scalar(run);
    o << "      const u64 hw = base + lane;\n"
         "      m = (hw >= hw_begin && hw < hw_end) ? m : 0u;\n"
         "      const u64 bal = __ballot(m != 0u);\n"
         "      if (bal) {\n"
         "        const u32 l = (u32)__builtin_ctzll(bal);\n"
         "        const u32 ml = __builtin_amdgcn_readlane(m, l);\n"
         "        atomicMin(best, 32ull * (base + l) + (u32)__builtin_ctz(ml));\n"
         "        break;\n"
         "      }\n"
         "    }\n"
         "  }\n"
         "}\n";
    return o.str();
}

namespace {

void rtc_check(hiprtcResult r, const char* what) {
    if (r != HIPRTC_SUCCESS) throw Error{kErrDevice, std::string(what) + ": " + hiprtcGetErrorString(r)};
}

std::vector<char> compile(const std::string& src, double* ms) {
    const double t0 = now_ms();
    hiprtcProgram prog;
    rtc_check(hiprtcCreateProgram(&prog, src.c_str(), "fes_es_kernel.hip", 0, nullptr, nullptr), "hiprtcCreateProgram");
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops"};
    hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        throw Error{kErrDevice, "hipRTC compile failed: " + log.substr(0, 2000)};
    }
    size_t size = 0;
    rtc_check(hiprtcGetCodeSize(prog, &size), "hiprtcGetCodeSize");
    std::vector<char> code(size);
    rtc_check(hiprtcGetCode(prog, code.data()), "hiprtcGetCode");
    hiprtcDestroyProgram(&prog);
    if (ms) *ms = now_ms() - t0;
    return code;
}

// Process-wide code-object cache keyed by source hash (circuits with identical plans share it).
std::mutex g_cache_mu;
std::map<uint64_t, std::vector<char>>& code_cache() {
    static std::map<uint64_t, std::vector<char>> m;
    return m;
}

}  // namespace

std::shared_ptr<JitKernel> jit_kernel(Circuit& c, int waves_per_eu, double* compile_ms) {
    if (compile_ms) *compile_ms = 0;
    std::shared_ptr<JitKernel> k;
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.jit.find(waves_per_eu);
        if (it != c.jit.end()) return it->second;
        k = std::make_shared<JitKernel>();
        k->waves_per_eu = waves_per_eu;
        k->block = 256;
        c.jit[waves_per_eu] = k;
    }
    std::lock_guard<std::mutex> g(k->mu);
    if (!k->code.empty()) return k;
    k->source = jit_source(c.lut_program(), waves_per_eu, k->block);
    k->hash = fnv1a(k->source);
    {
        std::lock_guard<std::mutex> cg(g_cache_mu);
        auto it = code_cache().find(k->hash);
        if (it != code_cache().end()) k->code = it->second;
    }
    if (k->code.empty()) {
        trace("specialized: compiling %zu bytes of source", k->source.size());
        try {
            k->code = compile(k->source, &k->compile_ms);
        } catch (...) {
            std::lock_guard<std::mutex> cg(c.mu);
            c.jit.erase(waves_per_eu);
            throw;
        }
        if (compile_ms) *compile_ms = k->compile_ms;
        trace("specialized: compiled in %.0f ms, %zu bytes of code", k->compile_ms, k->code.size());
        std::lock_guard<std::mutex> cg(g_cache_mu);
        code_cache()[k->hash] = k->code;
    }
    return k;
}

void run_jit(Device& dev, Circuit& c, JitKernel& k, const HwRange& r, uint64_t tile_hw, hipStream_t stream,
             const int* cancel, uint64_t* best_out, double* kernel_ms) {
    (void)c;
    hipFunction_t fn;
    int blocks_per_cu;
    {
        std::lock_guard<std::mutex> g(k.mu);
        auto it = k.per_device.find(dev.ordinal);
        if (it == k.per_device.end()) {
            hipModule_t mod;
            trace("specialized: loading module on device %d", dev.ordinal);
            FES_HIP(hipModuleLoadData(&mod, k.code.data()));
            FES_HIP(hipModuleGetFunction(&fn, mod, "fes_es_kernel"));
            int b = 0;
            FES_HIP(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, k.block, 0));
            k.per_device[dev.ordinal] = {mod, fn};
            k.blocks_per_cu[dev.ordinal] = std::max(1, b);
        }
        fn = k.per_device[dev.ordinal].second;
        blocks_per_cu = k.blocks_per_cu[dev.ordinal];
    }
    const int grid = dev.prop.multiProcessorCount * blocks_per_cu;
    const uint64_t waves = (uint64_t)grid * (k.block / 64);
    uint64_t hw_first = r.begin / 64 * 64;
    const uint64_t span = r.end - hw_first;
    uint64_t tile = tile_hw;
    if (!tile) {
        uint64_t target = span / std::max<uint64_t>(1, waves * 16);
        tile = 64;
        while (tile < target && tile < 64ull * 64) tile *= 2;
    }
    tile = (tile + 63) / 64 * 64;
    uint64_t total_items = (span + tile - 1) / tile;

    Buffer buf = dev.acquire(4096);
    struct Releaser {
        Device& d;
        Buffer b;
        ~Releaser() { d.release(b); }
    } rel{dev, buf};
    uint64_t* host = (uint64_t*)buf.host;
    std::memset(host, 0, 128);
    host[8] = ~0ull;  // best at byte offset 64, the counter at 0
    uint8_t* devp = (uint8_t*)buf.dev;
    uint64_t* next_item = (uint64_t*)devp;
    uint64_t* best = (uint64_t*)(devp + 64);
    uint64_t hw_begin = r.begin, hw_end = r.end;
    void* args[] = {&hw_begin, &hw_end, &hw_first, &tile, &total_items, &next_item, &best, &cancel};
    hipEvent_t e0, e1;
    FES_HIP(hipEventCreate(&e0));
    FES_HIP(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{e0, e1};
    trace("specialized launch: grid=%d block=%d items=%llu tile=%llu", grid, k.block,
          (unsigned long long)total_items, (unsigned long long)tile);
    FES_HIP(hipMemcpyAsync(devp, host, 128, hipMemcpyHostToDevice, stream));
    FES_HIP(hipEventRecord(e0, stream));
    FES_HIP(hipModuleLaunchKernel(fn, grid, 1, 1, k.block, 1, 1, 0, stream, args, nullptr));
    FES_HIP(hipEventRecord(e1, stream));
    FES_HIP(hipMemcpyAsync(host + 8, best, 8, hipMemcpyDeviceToHost, stream));
    FES_HIP(hipStreamSynchronize(stream));
    trace("specialized done");
    float ms = 0;
    FES_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (kernel_ms) *kernel_ms = ms;
    *best_out = host[8];
}

}  // namespace fes
