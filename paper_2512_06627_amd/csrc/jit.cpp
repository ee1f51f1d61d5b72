// Specialized exact-simulation kernel: the circuit becomes straight-line code.
//
// The paper keeps the compiled instruction stream in the constant cache and each
// thread's bit-vector registers in shared memory, and finds the kernel bound by memory
// traffic (Section 3.3).  On gfx950 the circuit itself is compiled into the kernel: the
// planner's LUT program (lut.cpp) becomes one inline-asm block per 2,048-pattern pass with
// planner-assigned registers (emit_block.cpp), so a LUT of up to three inputs is one
// v_bitop3_b32 and node values stay in registers (or, for very wide cones, LDS spill
// slots).  Primary inputs come from the pattern index: inputs 0..4 are constants inside a
// 32-bit word, inputs 5..10 are lane bits, inputs 11.. are bits of the wave's base index
// (SGPR operands).  Around the block, plain HIP claims tiles, prefetches the early-exit
// bound and reports the lowest failing pattern.  When no block fits, every gate becomes
// its own asm statement and the compiler allocates registers.
//
// The source is compiled once per circuit with hipRTC for gfx950 and cached.
#include <hip/hiprtc.h>

#include <dlfcn.h>
#include <spawn.h>
#include <sys/wait.h>
#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <chrono>
#include <condition_variable>
#include <csignal>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <iterator>
#include <mutex>
#include <sstream>
#include <thread>

#include "rtc_options.hpp"
#include "runtime.hpp"

extern char** environ;

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

std::string jit_source(const LutProgram& lp, int waves_per_eu, int block, int* waves_used) {
    std::ostringstream o;
    const uint32_t n = lp.num_inputs;
    // One asm block per pass when it fits: at the requested occupancy, else at two waves per
    // SIMD (a wide cone's live values need up to 256 VGPRs); otherwise one asm statement per
    // gate with the compiler's register allocation.  The compiler keeps its own values
    // (claims, bounds, pointers, lane masks, words, the ballot) in the registers the block
    // leaves alone: about 24 VGPRs and 30 SGPRs.
    std::string block_body;
    BlockStats bs;
    int waves = waves_per_eu;
    int lds_slots = 0;
    if (specialized_emit_mode() == 1) {
        // Attempts: (waves, LDS spill slots per wave).  LDS holds 160 KB per CU, shared by
        // 4 x waves waves; a slot is 256 bytes; ds offsets reach 255 slots.
        std::vector<std::pair<int, int>> tries = {{waves_per_eu, 0}};
        if (waves_per_eu > 2) tries.push_back({2, 0});
        for (int w : {std::min(waves_per_eu, 2), 1}) tries.push_back({w, std::min(255, 163840 / (4 * w) / 256)});
        const int cap = specialized_vgpr_cap();
        for (auto& tr : tries) {
            int vgpr_budget = std::min(256, 512 / tr.first / 8 * 8) - 24;
            if (cap > 0) vgpr_budget = std::min(vgpr_budget, cap);
            if (emit_block_body(lp, vgpr_budget, 64, 0, 20, specialized_latency_slots(), specialized_bank_aware() != 0,
                                tr.second, &block_body, &bs)) {
                waves = tr.first;
                lds_slots = bs.lds_slots;
                break;
            }
            block_body.clear();
        }
    }
    if (waves_used) *waves_used = waves;
    // One pass of 64 half-words (2,048 patterns) per loop iteration.
    o << "// exact simulation, " << n << " inputs: " << lp.lut_steps << " LUT steps, " << lp.scalar_steps
      << " scalar steps, " << lp.absorbed_gates << " gates absorbed into LUTs, " << lp.folded_gates << " folded, "
      << 1 << " passes per iteration\n";
    o << "typedef unsigned int u32;\ntypedef unsigned long long u64;\n";
    o << "extern \"C\" __global__ void __launch_bounds__(" << block << ") __attribute__((amdgpu_waves_per_eu("
      << waves << ", " << waves << ")))\n";
    o << "fes_es_kernel(u64 hw_begin, u64 hw_end, u64 hw_first, u64 tile_hw, u64 total_items,\n"
         "              u64* __restrict__ next_item, u64* __restrict__ best, const int* __restrict__ cancel) {\n";
    o << "  const u32 lane = threadIdx.x & 63u;\n";
    for (uint32_t i = 5; i < n && i < 11; ++i)
        o << "  const u32 x" << i << " = 0u - ((lane >> " << (i - 5) << ") & 1u);\n";
    char buf[320];
    for (uint32_t i = 0; i < lp.words.size(); ++i) {
        std::snprintf(buf, sizeof buf, "  const u32 w%u = 0x%08Xu;\n", i, lp.words[i]);
        o << buf;
    }
    if (lds_slots) {  // per-wave spill area of the asm block: slot s of lane l at [s * 64 + l]
        o << "  __shared__ u32 fes_spill[" << (block / 64) * lds_slots * 64 << "];\n"
          << "  const u32 spill_addr = (u32)(unsigned long)(__attribute__((address_space(3))) u32*)(fes_spill + (threadIdx.x >> 6) * "
          << lds_slots * 64 << "u + lane);\n";
    }
    // Control flow stays wave-uniform: every lane takes part in the claim (lane 0 adds 1, the
    // others 0) and in the atomicMin (all lanes hold the same value), so no branch depends on
    // the lane and every loop exit is a scalar branch.
    // Claims are spread over several counters on separate 128-byte lines (counter s hands out
    // items s, s + C, s + 2C, ...), so short work items are not serialised at one atomic.
    // A grid with fewer waves than counters uses one counter per wave, so every counter in use
    // has a wave and every item is claimed.
    o << "  const u32 waves = gridDim.x * (blockDim.x >> 6);\n"
         "  const u32 nclaim = waves < " << kClaimCounters << "u ? waves : " << kClaimCounters << "u;\n"
         "  const u32 claim = __builtin_amdgcn_readfirstlane((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % nclaim);\n"
         "  u64* const counter = next_item + claim * " << kClaimStride << "u;\n"
         "  for (;;) {\n"
         "    const u64 claimed = atomicAdd(counter, lane == 0u ? 1ull : 0ull);\n"
         "    const u64 k = ((u64)__builtin_amdgcn_readfirstlane((u32)(claimed >> 32)) << 32) |\n"
         "                  __builtin_amdgcn_readfirstlane((u32)claimed);\n"
         "    const u64 item = claim + k * nclaim;\n"
         "    if (item >= total_items) break;\n"
         "    if (cancel && __builtin_amdgcn_readfirstlane(__hip_atomic_load(cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM))) break;\n"
         "    const u64 hw0 = hw_first + item * tile_hw;\n"
         "    const u64 hw_stop = hw0 + tile_hw < hw_end ? hw0 + tile_hw : hw_end;\n"
         "    const u64 b_first = __hip_atomic_load(best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);\n"
         "    const u64 best_seen = ((u64)__builtin_amdgcn_readfirstlane((u32)(b_first >> 32)) << 32) |\n"
         "                    __builtin_amdgcn_readfirstlane((u32)b_first);\n"
         "    // passes of this tile that start below the bound (pattern 32*base < best_seen)\n"
         "    const u64 bound_hw = best_seen / 32u + ((best_seen & 31u) ? 1u : 0u);\n"
         "    const u64 stop = hw_stop < bound_hw ? hw_stop : bound_hw;\n"
         "    const u32 npass = stop > hw0 ? (u32)((stop - hw0 + 63u) / 64u) : 0u;\n"
         "    for (u32 t = 0; t < npass; ++t) {\n"
         "      const u64 base = hw0 + 64ull * t;\n";
    // The bound found by other waves is read once per tile (up to 64 passes): a device-scope
    // load each pass cost 15% (16x16 miter) to 37% (MAC8) of the kernel time, and after a
    // failure is found a wave finishes at most its current tile.  The pass loop runs on a
    // 32-bit counter (gfx9 has no scalar 64-bit ordered compare, so 64-bit loop tests became
    // vector compares).  Only the range's first and last pass can hold half-words outside it
    // (hw_first is hw_begin rounded down to a pass), so the range mask is applied inside the
    // branch taken when some lane fails: a failure outside the range is dropped there.
    if (specialized_emit_mode() == 1) {
        if (block_body.empty())
            o << "      // one asm block would need " << bs.vgprs << " VGPRs (" << bs.vgprs_min_live
              << " in the pressure-aware order) and " << bs.sgprs << " SGPRs\n";
        else
            o << "      // one asm block: " << bs.vgprs << " VGPRs, " << bs.sgprs << " SGPRs, " << bs.valu
              << " VALU and " << bs.salu << " SALU instructions, " << bs.copies << " scalar-operand copies, " << bs.spills
              << " values moved to VGPRs, " << waves << " waves per SIMD"
              << (lds_slots ? ", " + std::to_string(bs.lds_ops) + " LDS spill operations in " + std::to_string(lds_slots) + " slots" : std::string())
              << "\n";
    }
    if (!block_body.empty()) {
        o << "      const u32 base_lo = (u32)base, base_hi = (u32)(base >> 32);\n" << block_body;
    } else {
    for (uint32_t i = 11; i < n; ++i)
        o << "      const u32 x" << i << " = 0u - (u32)((base >> " << (i - 5) << ") & 1ull);\n";
    o << "      u32 m0 = 0u;\n";
    // Every gate is an inline-asm instruction whose function the planner fixed, so the
    // compiler allocates registers and schedules but never rewrites the logic.  VALU
    // operands: at most one scalar (SGPR) source per instruction; others go through VGPRs.
    auto scalar_name = [&](const LutRef& r) { return ref_name(r); };  // a scalar-step operand
    auto pass_name = [&](const LutRef& r, int q) {                     // a LUT operand
        if (r.kind == LutRef::Varying) return "vr" + std::to_string(r.index) + "_" + std::to_string(q);
        return ref_name(r);
    };
    // Runs of consecutive scalar steps are emitted as one asm block (the compiler pads every
    // asm block with a wait state, so one block per gate would double the scalar issue count).
    // Block outputs are early-clobber: they never share a register with a block input.
    std::vector<const LutStep*> run;
    auto flush_scalar = [&]() {
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
                const std::string nm = scalar_name(st->leaf[j]);
                if (in_index(nm).empty()) ins.push_back(nm);
            }
        const char* sfx = "_b32";
        std::string text;
        for (const LutStep* st : run) {
            const bool na = st->table & 1, nb = (st->table >> 1) & 1;
            std::string a = in_index(scalar_name(st->leaf[0])), b = in_index(scalar_name(st->leaf[1]));
            std::string opname = "s_and";
            if (na && nb) opname = "s_nor";
            else if (nb) opname = "s_andn2";
            else if (na) { opname = "s_andn2"; std::swap(a, b); }
            text += std::string(text.empty() ? "" : "\\n\\t") + opname + sfx + " " +
                    in_index("su" + std::to_string(st->dst)) + ", " + a + ", " + b;
        }
        o << "      u32";
        for (size_t i = 0; i < outs.size(); ++i) o << (i ? ", " : " ") << outs[i];
        o << ";\n      asm(\"" << text << "\" : ";
        for (size_t i = 0; i < outs.size(); ++i) o << (i ? ", " : "") << "\"=&s\"(" << outs[i] << ")";
        o << " : ";
        for (size_t i = 0; i < ins.size(); ++i) o << (i ? ", " : "") << "\"s\"(" << ins[i] << ")";
        o << " : \"scc\");\n";
        run.clear();
    };
    auto run_operands = [&](const LutStep& st) {  // operand count if st joined the run
        std::vector<std::string> names;
        for (const LutStep* r : run) names.push_back("su" + std::to_string(r->dst));
        names.push_back("su" + std::to_string(st.dst));
        auto add = [&](const std::string& nm) {
            if (std::find(names.begin(), names.end(), nm) == names.end()) names.push_back(nm);
        };
        for (const LutStep* r : run) { add(scalar_name(r->leaf[0])); add(scalar_name(r->leaf[1])); }
        add(scalar_name(st.leaf[0]));
        add(scalar_name(st.leaf[1]));
        return names.size();
    };
    for (const LutStep& st : lp.steps) {
        if (st.op == LutStep::ScalarAnd) {
            if (!run.empty() && run_operands(st) > 30) flush_scalar();
            run.push_back(&st);
            continue;
        }
        flush_scalar();
        {
            const int q = 0;
            if (st.op == LutStep::Lut) {
                const uint32_t k = st.nleaves;
                const char* ops = k == 3 ? "%1, %2, %3" : k == 2 ? "%1, %2, %2" : "%1, %1, %1";
                bool used_s = false;
                std::string cons;
                for (uint32_t j = 0; j < k; ++j) {
                    const bool sc = is_scalar(st.leaf[j]) && !used_s;
                    used_s |= sc;
                    cons += std::string(j ? ", " : "") + (sc ? "\"s\"(" : "\"v\"(") + pass_name(st.leaf[j], q) + ")";
                }
                std::snprintf(buf, sizeof buf, "      u32 vr%u_%d; asm(\"v_bitop3_b32 %%0, %s bitop3:0x%02x\" : \"=v\"(vr%u_%d) : %s);\n",
                              st.dst, q, ops, st.table, st.dst, q, cons.c_str());
                o << buf;
            } else {
                // m = m | (x ^ neg): table over (m, x, x)
                uint8_t table = 0;
                for (uint32_t idx = 0; idx < 8; ++idx) {
                    const uint32_t mm = (idx >> 2) & 1u, x = (idx >> 1) & 1u;
                    if (mm | (x ^ (st.out_neg ? 1u : 0u))) table |= (uint8_t)(1u << idx);
                }
                std::snprintf(buf, sizeof buf, "      asm(\"v_bitop3_b32 %%0, %%1, %%2, %%2 bitop3:0x%02x\" : \"=v\"(m%d) : \"v\"(m%d), \"%s\"(%s));\n",
                              table, q, q, is_scalar(st.leaf[0]) ? "s" : "v", pass_name(st.leaf[0], q).c_str());
                o << buf;
            }
        }
    }
    flush_scalar();
    }
    // Lowest failing pattern of this pass: the lowest lane, then its lowest bit; all of it
    // under a wave-uniform branch on the ballot.
    o << "      u64 bal = __ballot(m0 != 0u);\n"
         "      if (bal) {\n"
         "        u64 b = base;\n"
         "        asm volatile(\"\" : \"+s\"(b));  // keeps the loop from carrying the edge offsets\n"
         "        const u32 lo = b < hw_begin ? (u32)(hw_begin - b) : 0u;\n"
         "        const u64 left = hw_end - b;\n"
         "        bal &= (~0ull << lo) & (left >= 64u ? ~0ull : (1ull << left) - 1u);\n"
         "        if (bal) {\n"
         "          const u32 l = (u32)__builtin_ctzll(bal);\n"
         "          const u32 ml = __builtin_amdgcn_readlane(m0, l);\n"
         "          atomicMin(best, 32ull * (base + l) + (u32)__builtin_ctz(ml));\n"
         "          break;\n"
         "        }\n"
         "      }\n";
    o << "    }\n"
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
    hiprtcResult r = hiprtcCompileProgram(prog, kRtcOptionCount, const_cast<const char**>(kRtcOptions));
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

// Compile helper processes (the fastlec_es_rtc program next to this library): hipRTC serializes
// compiles inside one process, so the programs of a grouped compile run side by side in child
// processes.  FASTLEC_ES_RTC_PROCS sets how many at once (default: half the host threads, at most
// 8; 0 compiles in this process).
std::string helper_path() {
    static const std::string path = [] {
        Dl_info info;
        if (!dladdr((void*)&helper_path, &info) || !info.dli_fname) return std::string();
        std::string lib = info.dli_fname;
        const size_t slash = lib.rfind('/');
        const std::string exe = (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/fastlec_es_rtc";
        return access(exe.c_str(), X_OK) == 0 ? exe : std::string();
    }();
    return path;
}

int helper_procs() {
    static const int n = [] {
        const char* v = std::getenv("FASTLEC_ES_RTC_PROCS");
        if (v && *v) return std::max(0, std::min(32, std::atoi(v)));
        return (int)std::min<unsigned>(8, std::max(1u, std::thread::hardware_concurrency() / 2));
    }();
    return helper_path().empty() ? 0 : n;
}

// Helper processes running at once in this process, over all callers (the server's compile
// threads and batch calls share the limit helper_procs()).
std::mutex g_helper_mu;
std::condition_variable g_helper_cv;
int g_helpers_running = 0;

// Seconds a helper may run before it is killed and its program compiled in this process
// (FASTLEC_ES_RTC_TIMEOUT_S, default 300).
double helper_timeout_s() {
    static const double t = [] {
        const char* v = std::getenv("FASTLEC_ES_RTC_TIMEOUT_S");
        const double x = v && *v ? std::atof(v) : 0.0;
        return x > 0 ? x : 300.0;
    }();
    return t;
}

// Compiles srcs[i] into codes[i] in helper processes, at most `procs` of them running at once
// in the whole process; returns false for any program whose helper failed, timed out or could
// not start (the caller compiles that one in this process).  The helper writes its code object
// under a temporary name and renames it when complete, so a code object that exists is whole.
// Children start with only stdin, stdout and stderr open: they hold none of the host program's
// files (GPU device nodes included).
std::vector<uint8_t> compile_in_helpers(const std::vector<std::string>& srcs, std::vector<std::vector<char>>& codes,
                                        int procs) {
    std::vector<uint8_t> ok(srcs.size(), 0);
    const char* tmp = std::getenv("TMPDIR");
    std::string dir = std::string(tmp && *tmp ? tmp : "/tmp") + "/fes_rtc_XXXXXX";
    if (!mkdtemp(&dir[0])) return ok;
    const std::string exe = helper_path();
    auto file = [&](size_t i, const char* ext) { return dir + "/p" + std::to_string(i) + ext; };
    posix_spawn_file_actions_t fa;
    posix_spawn_file_actions_init(&fa);
    posix_spawn_file_actions_addclosefrom_np(&fa, 3);
    struct Child {
        pid_t pid;
        size_t i;
        double deadline;
    };
    std::vector<Child> running;
    size_t next = 0;
    auto collect = [&](const Child& c, bool exited_ok) {
        if (exited_ok) {
            std::ifstream in(file(c.i, ".co"), std::ios::binary);
            if (in) codes[c.i].assign(std::istreambuf_iterator<char>(in), std::istreambuf_iterator<char>());
            ok[c.i] = !codes[c.i].empty();
        }
        std::lock_guard<std::mutex> g(g_helper_mu);
        --g_helpers_running;
        g_helper_cv.notify_all();
    };
    while (next < srcs.size() || !running.empty()) {
        // Start helpers while the process-wide limit allows; wait for a slot only when none of
        // this call's helpers is running (their completion frees slots too).
        while (next < srcs.size()) {
            {
                std::unique_lock<std::mutex> g(g_helper_mu);
                if (running.empty())
                    g_helper_cv.wait(g, [&] { return g_helpers_running < procs; });
                if (g_helpers_running >= procs) break;
                ++g_helpers_running;
            }
            const size_t i = next++;
            std::ofstream(file(i, ".hip"), std::ios::binary) << srcs[i];
            const std::string a1 = file(i, ".hip"), a2 = file(i, ".co");
            char* argv[] = {const_cast<char*>(exe.c_str()), const_cast<char*>(a1.c_str()), const_cast<char*>(a2.c_str()),
                            nullptr};
            pid_t pid = 0;
            if (posix_spawn(&pid, exe.c_str(), &fa, nullptr, argv, environ) == 0) {
                running.push_back({pid, i, now_ms() + 1000.0 * helper_timeout_s()});
            } else {
                std::lock_guard<std::mutex> g(g_helper_mu);
                --g_helpers_running;
                g_helper_cv.notify_all();
            }
        }
        // Reap this call's helpers by their own pids (never waitpid(-1): children of the host
        // program are not ours to reap).
        bool progressed = false;
        for (size_t r = 0; r < running.size();) {
            int status = 0;
            const pid_t w = waitpid(running[r].pid, &status, WNOHANG);
            bool done = false, good = false;
            if (w == running[r].pid) {
                done = true;
                good = WIFEXITED(status) && WEXITSTATUS(status) == 0;
            } else if (w < 0 && errno != EINTR) {
                // Reaped elsewhere (a host program that ignores SIGCHLD): the renamed code object
                // tells whether the helper finished.
                done = true;
                good = access(file(running[r].i, ".co").c_str(), R_OK) == 0;
            } else if (w == 0 && now_ms() > running[r].deadline) {
                trace("specialized: helper for program %zu timed out; killing it", running[r].i);
                kill(running[r].pid, SIGKILL);
                while (waitpid(running[r].pid, &status, 0) < 0 && errno == EINTR) {
                }
                done = true;
            }
            if (done) {
                collect(running[r], good);
                running.erase(running.begin() + (long)r);
                progressed = true;
            } else {
                ++r;
            }
        }
        if (!progressed && !running.empty()) std::this_thread::sleep_for(std::chrono::milliseconds(1));
    }
    posix_spawn_file_actions_destroy(&fa);
    for (size_t i = 0; i < srcs.size(); ++i) {
        std::remove(file(i, ".hip").c_str());
        std::remove(file(i, ".co").c_str());
        std::remove((file(i, ".co") + ".part").c_str());
    }
    rmdir(dir.c_str());
    return ok;
}

// Compiles every program; wall-clock milliseconds of the whole set in *ms.  Several programs
// compile in helper processes side by side; a lone program compiles in this process unless
// `alone_in_helper` (a caller that runs several compiles at once: compiles in this process
// would serialize).
std::vector<std::vector<char>> compile_programs(const std::vector<std::string>& srcs, double* ms,
                                                bool alone_in_helper) {
    const double t0 = now_ms();
    std::vector<std::vector<char>> codes(srcs.size());
    std::vector<uint8_t> ok(srcs.size(), 0);
    const int procs = helper_procs();
    if (procs > 0 && (srcs.size() > 1 || alone_in_helper)) ok = compile_in_helpers(srcs, codes, procs);
    for (size_t i = 0; i < srcs.size(); ++i)
        if (!ok[i]) {
            if (procs > 0 && (srcs.size() > 1 || alone_in_helper))
                trace("specialized: helper failed on program %zu; compiling it in this process", i);
            codes[i] = compile(srcs[i], nullptr);
        }
    if (ms) *ms = now_ms() - t0;
    return codes;
}

// Process-wide code-object cache keyed by the hash of a kernel's own source (circuits with
// identical plans share it): the code object's bytes and the kernel's entry point in them.
struct CachedCode {
    std::shared_ptr<const std::vector<char>> bytes;
    std::string name;
};
std::mutex g_cache_mu;
std::map<uint64_t, CachedCode>& code_cache() {
    static std::map<uint64_t, CachedCode> m;
    return m;
}

bool from_cache(JitKernel& k) {
    std::lock_guard<std::mutex> cg(g_cache_mu);
    auto it = code_cache().find(k.hash);
    if (it == code_cache().end()) return false;
    k.code = std::make_shared<CodeObject>();
    k.code->bytes = it->second.bytes;
    k.name = it->second.name;
    return true;
}

// The kernel's source with its entry point renamed (several kernels in one program).
std::string renamed(const std::string& src, const std::string& name) {
    const std::string from = "\nfes_es_kernel(";
    const size_t at = src.find(from);
    if (at == std::string::npos) throw Error{kErrInvalid, "specialized source without its entry point"};
    return src.substr(0, at) + "\n" + name + "(" + src.substr(at + from.size());
}

}  // namespace

namespace {
int env_int(const char* name, int dflt, int lo, int hi) {
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    const int x = std::atoi(v);
    return x < lo || x > hi ? dflt : x;
}
}  // namespace

int specialized_latency_slots() { return env_int("FASTLEC_ES_JIT_DIST", 1, 1, 64); }
int specialized_vgpr_cap() { return env_int("FASTLEC_ES_JIT_VGPR_CAP", 0, 0, 256); }
int specialized_bank_aware() { return env_int("FASTLEC_ES_JIT_BANKS", 1, 0, 1); }
int specialized_emit_mode() { return env_int("FASTLEC_ES_JIT_EMIT", 1, 0, 1); }
int specialized_waves_per_eu() { return env_int("FASTLEC_ES_JIT_WAVES", 3, 1, 8); }
int specialized_scalar_policy() { return env_int("FASTLEC_ES_JIT_SCALAR", 2, 0, 2); }
int specialized_block() {
    const int b = env_int("FASTLEC_ES_JIT_BLOCK", 256, 64, 1024);
    return b % 64 ? 256 : b;
}

std::shared_ptr<JitKernel> jit_ready(Circuit& c, int waves_per_eu) {
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.jit.find(waves_per_eu);
    if (it == c.jit.end()) return nullptr;
    std::unique_lock<std::mutex> gk(it->second->mu, std::try_to_lock);
    if (!gk.owns_lock()) return nullptr;
    return it->second->code ? it->second : nullptr;
}

std::shared_ptr<JitKernel> jit_kernel(Circuit& c, int waves_per_eu, double* compile_ms) {
    if (compile_ms) *compile_ms = 0;
    std::shared_ptr<JitKernel> k;
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.jit.find(waves_per_eu);
        if (it != c.jit.end()) return it->second;
        k = std::make_shared<JitKernel>();
        k->waves_per_eu = waves_per_eu;
        k->block = specialized_block();
        c.jit[waves_per_eu] = k;
    }
    std::lock_guard<std::mutex> g(k->mu);
    if (k->code) return k;
    k->source = jit_source(c.lut_program(), waves_per_eu, k->block, &k->waves_used);
    k->hash = fnv1a(k->source);
    if (!from_cache(*k)) {
        trace("specialized: compiling %zu bytes of source", k->source.size());
        auto obj = std::make_shared<CodeObject>();
        try {
            obj->bytes = std::make_shared<const std::vector<char>>(compile(k->source, &k->compile_ms));
        } catch (...) {
            std::lock_guard<std::mutex> cg(c.mu);
            c.jit.erase(waves_per_eu);
            throw;
        }
        k->code = obj;
        k->name = "fes_es_kernel";
        if (compile_ms) *compile_ms = k->compile_ms;
        trace("specialized: compiled in %.0f ms, %zu bytes of code", k->compile_ms, obj->bytes->size());
        std::lock_guard<std::mutex> cg(g_cache_mu);
        code_cache()[k->hash] = {obj->bytes, k->name};
    }
    return k;
}

int compile_helpers() { return helper_procs(); }

std::vector<std::shared_ptr<JitKernel>> jit_kernels(const std::vector<Circuit*>& cs, int waves_per_eu,
                                                    std::vector<double>* compile_ms, CompileSplit split) {
    const size_t m = cs.size();
    std::vector<std::shared_ptr<JitKernel>> ks(m);
    if (compile_ms) compile_ms->assign(m, 0.0);
    // Each circuit's kernel object; their locks are taken in circuit order (uids never repeat),
    // so two callers with overlapping circuit sets cannot deadlock.
    std::vector<size_t> order(m);
    for (size_t i = 0; i < m; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cs[a]->uid < cs[b]->uid; });
    std::vector<std::unique_lock<std::mutex>> locks;
    std::vector<size_t> pending, need_source;
    for (size_t i : order) {
        Circuit& c = *cs[i];
        {
            std::lock_guard<std::mutex> g(c.mu);
            auto it = c.jit.find(waves_per_eu);
            if (it == c.jit.end()) {
                auto k = std::make_shared<JitKernel>();
                k->waves_per_eu = waves_per_eu;
                k->block = specialized_block();
                it = c.jit.emplace(waves_per_eu, k).first;
            }
            ks[i] = it->second;
        }
        bool dup = false;
        for (auto& l : locks) dup |= l.mutex() == &ks[i]->mu;
        if (dup) continue;  // the same circuit twice
        locks.emplace_back(ks[i]->mu);
        if (!ks[i]->code) need_source.push_back(i);
    }
    // LUT mapping and kernel source of each circuit on host threads in parallel (each kernel
    // object is locked above and written by one thread), then the code cache, in circuit order.
    parallel_for(need_source.size(), [&](size_t t) {
        JitKernel& k = *ks[need_source[t]];
        k.source = jit_source(cs[need_source[t]]->lut_program(), waves_per_eu, k.block, &k.waves_used);
        k.hash = fnv1a(k.source);
    });
    for (size_t i : need_source)
        if (!from_cache(*ks[i])) pending.push_back(i);
    // Programs of at most 64 kernels, each under its own entry-point name.  With compile helper
    // processes a group of 4 or more kernels is spread over as many programs as run at once
    // (every program pays hipRTC's fixed cost, but they overlap; on a 16-core host 16 kernels
    // took 0.34-0.39 s as one program and 0.16-0.17 s as eight, 4 kernels 0.18-0.19 s against
    // 0.14-0.15 s); fewer stay one program in this process, which saves a helper's start-up.
    // CompileSplit::kEach gives every kernel a program of its own, in a helper even when alone.
    if (pending.empty()) return ks;
    const size_t procs = (size_t)std::max(1, helper_procs());
    const bool each = split == CompileSplit::kEach;
    const size_t programs =
        each ? pending.size() : pending.size() >= 4 ? std::min(procs, pending.size()) : 1;
    size_t per = std::min<size_t>(64, (pending.size() + programs - 1) / programs);
    std::vector<std::pair<size_t, size_t>> parts;
    std::vector<std::string> srcs;
    size_t bytes = 0;
    for (size_t p0 = 0; p0 < pending.size(); p0 += per) {
        const size_t p1 = std::min(pending.size(), p0 + per);
        std::string src;
        for (size_t t = p0; t < p1; ++t) {
            JitKernel& k = *ks[pending[t]];
            k.name = "fes_es_kernel_" + std::to_string(t - p0);
            src += renamed(k.source, k.name);
            bytes += k.source.size();
        }
        parts.push_back({p0, p1});
        srcs.push_back(std::move(src));
    }
    double ms = 0;
    std::vector<std::vector<char>> codes;
    try {
        trace("specialized: compiling %zu kernels as %zu programs (%zu bytes of source, %d helper processes)",
              pending.size(), srcs.size(), bytes, helper_procs());
        codes = compile_programs(srcs, &ms, each);
    } catch (...) {
        for (size_t t = 0; t < pending.size(); ++t) {
            Circuit& c = *cs[pending[t]];
            std::lock_guard<std::mutex> g(c.mu);
            c.jit.erase(waves_per_eu);
        }
        throw;
    }
    trace("specialized: compiled %zu kernels in %.0f ms", pending.size(), ms);
    std::lock_guard<std::mutex> cg(g_cache_mu);
    for (size_t q = 0; q < parts.size(); ++q) {
        auto obj = std::make_shared<CodeObject>();
        obj->bytes = std::make_shared<const std::vector<char>>(std::move(codes[q]));
        for (size_t t = parts[q].first; t < parts[q].second; ++t) {
            JitKernel& k = *ks[pending[t]];
            k.code = obj;
            k.compile_ms = ms / (double)pending.size();
            if (compile_ms) (*compile_ms)[pending[t]] = k.compile_ms;
            code_cache()[k.hash] = {obj->bytes, k.name};
        }
    }
    return ks;
}

hipModule_t CodeObject::module(int device) {
    std::lock_guard<std::mutex> g(mu);
    auto it = modules.find(device);
    if (it != modules.end()) return it->second;
    hipModule_t mod;
    trace("specialized: loading a code object of %zu bytes on device %d", bytes->size(), device);
    FES_HIP(hipModuleLoadData(&mod, bytes->data()));
    modules[device] = mod;
    return mod;
}

CodeObject::~CodeObject() {
    for (auto& dm : modules) {
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess && hipSetDevice(dm.first) == hipSuccess) {
            (void)hipModuleUnload(dm.second);
            (void)hipSetDevice(cur);
        }
    }
}

JitLaunchPlan jit_prepare(Device& dev, JitKernel& k, const HwRange& r, uint64_t tile_hw) {
    JitLaunchPlan lp;
    int blocks_per_cu;
    {
        std::lock_guard<std::mutex> g(k.mu);
        auto it = k.per_device.find(dev.ordinal);
        if (it == k.per_device.end()) {
            hipFunction_t fn;
            FES_HIP(hipModuleGetFunction(&fn, k.code->module(dev.ordinal), k.name.c_str()));
            int b = 0;
            FES_HIP(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, k.block, 0));
            // The persistent grid holds the targeted waves per SIMD (a workgroup of `block`
            // threads puts block/256 waves on each of the CU's four SIMDs), never more: the
            // register count decides whether one more wave would fit, and at four waves per
            // SIMD the 16x16 kernel runs a third slower than at three.
            const int target = std::max(1, k.waves_used * 4 * 64 / k.block);
            k.per_device[dev.ordinal] = fn;
            k.blocks_per_cu[dev.ordinal] = std::max(1, std::min(b, target));
            if (trace_on()) {
                int regs = 0, spill = 0;
                (void)hipFuncGetAttribute(&regs, HIP_FUNC_ATTRIBUTE_NUM_REGS, fn);
                (void)hipFuncGetAttribute(&spill, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, fn);
                trace("specialized kernel %s loaded: %d registers per lane, %d bytes of scratch, "
                      "%d workgroups of %d per CU possible, %d used",
                      k.name.c_str(), regs, spill, b, k.block, k.blocks_per_cu[dev.ordinal]);
            }
        }
        lp.fn = k.per_device[dev.ordinal];
        blocks_per_cu = k.blocks_per_cu[dev.ordinal];
    }
    lp.grid = dev.prop.multiProcessorCount * blocks_per_cu;
    lp.block = k.block;
    const uint64_t waves = (uint64_t)lp.grid * (k.block / 64);
    const uint64_t step = 64;  // half-words per loop iteration (one pass)
    lp.hw_begin = r.begin;
    lp.hw_end = r.end;
    lp.hw_first = r.begin / step * step;
    const uint64_t span = r.end - lp.hw_first;
    uint64_t tile = tile_hw;
    if (!tile) {
        uint64_t target = span / std::max<uint64_t>(1, waves * 16);
        tile = step;
        while (tile < target && tile < 64ull * 64) tile *= 2;
    }
    lp.tile = (tile + step - 1) / step * step;
    lp.total_items = (span + lp.tile - 1) / lp.tile;
    return lp;
}

void jit_enqueue(const JitLaunchPlan& lp, uint64_t* next_item, uint64_t* best, const int* cancel, hipStream_t stream) {
    uint64_t hw_begin = lp.hw_begin, hw_end = lp.hw_end, hw_first = lp.hw_first, tile = lp.tile,
             total_items = lp.total_items;
    void* args[] = {&hw_begin, &hw_end, &hw_first, &tile, &total_items, &next_item, &best, &cancel};
    trace("specialized launch: grid=%d block=%d items=%llu tile=%llu", lp.grid, lp.block,
          (unsigned long long)lp.total_items, (unsigned long long)lp.tile);
    FES_HIP(hipModuleLaunchKernel(lp.fn, lp.grid, 1, 1, lp.block, 1, 1, 0, stream, args, nullptr));
}

void run_jit(Device& dev, Circuit& c, JitKernel& k, const HwRange& r, uint64_t tile_hw, hipStream_t stream,
             const int* cancel, uint64_t* best_out, double* kernel_ms, DevMem mem) {
    (void)c;
    const JitLaunchPlan lp = jit_prepare(dev, k, r, tile_hw);
    if (mem.ptr) check_dev_mem(mem, kClaimBytes + 8);
    Buffer buf = dev.acquire(mem.ptr ? 0 : 4096, 4096);
    struct Releaser {
        Device& d;
        Buffer b;
        ~Releaser() { d.release(b); }
    } rel{dev, buf};
    static_assert(kClaimBytes + 8 <= 4096, "claim counters and best fit the buffer");
    uint64_t* host = (uint64_t*)buf.host;
    std::memset(host, 0, kClaimBytes);
    uint64_t* hbest = host + kClaimBytes / 8;
    *hbest = ~0ull;  // the claim counters at 0, best right after them
    uint8_t* devp = (uint8_t*)(mem.ptr ? mem.ptr : buf.dev);
    uint64_t* next_item = (uint64_t*)devp;
    uint64_t* best = (uint64_t*)(devp + kClaimBytes);
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
    FES_HIP(hipMemcpyAsync(devp, host, kClaimBytes + 8, hipMemcpyHostToDevice, stream));
    FES_HIP(hipEventRecord(e0, stream));
    jit_enqueue(lp, next_item, best, cancel, stream);
    FES_HIP(hipEventRecord(e1, stream));
    FES_HIP(hipMemcpyAsync(hbest, best, 8, hipMemcpyDeviceToHost, stream));
    FES_HIP(hipStreamSynchronize(stream));
    trace("specialized done");
    float ms = 0;
    FES_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (kernel_ms) *kernel_ms = ms;
    *best_out = *hbest;
}

}  // namespace fes
