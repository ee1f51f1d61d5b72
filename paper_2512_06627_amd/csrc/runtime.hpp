// Host runtime: circuits, per-device state, schedules and launches.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fastlec_es.h"
#include "aig.hpp"
#include "kernels.hpp"
#include "model.hpp"
#include "plan.hpp"

namespace fes {

[[noreturn]] void throw_hip(hipError_t e, const char* what);
#define FES_HIP(call)                                  \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) ::fes::throw_hip(e_, #call); \
    } while (0)

// A HIP event owned by a scope (destroyed on every exit path, errors included).
struct ScopedEvent {
    hipEvent_t e = nullptr;
    ScopedEvent() { FES_HIP(hipEventCreate(&e)); }
    ~ScopedEvent() {
        if (e) (void)hipEventDestroy(e);
    }
    ScopedEvent(const ScopedEvent&) = delete;
    ScopedEvent& operator=(const ScopedEvent&) = delete;
};

double now_ms();

// Opt-in trace of host phases to stderr (environment FASTLEC_ES_TRACE=1).
bool trace_on();
void trace(const char* fmt, ...);

// A straight-line kernel compiled for one circuit (hipRTC code object) and its
// per-device module handles.
// A compiled code object (one or more specialized kernels) and its module on each device it was
// loaded on; the modules are unloaded when the last kernel that uses the object goes away.
struct CodeObject {
    std::shared_ptr<const std::vector<char>> bytes;
    std::mutex mu;
    std::map<int, hipModule_t> modules;
    hipModule_t module(int device);  // loads on first use; the device must be current
    ~CodeObject();
};

struct JitKernel {
    std::string source;                // the kernel's own source (entry point fes_es_kernel)
    std::string name = "fes_es_kernel";  // entry point in the code object
    std::shared_ptr<CodeObject> code;  // set once compiled
    uint64_t hash = 0;
    int waves_per_eu = 2;  // requested occupancy (the cache key)
    int waves_used = 2;    // occupancy the source was built for (the launch grid follows it)
    int block = 256;
    double compile_ms = 0;
    std::mutex mu;
    std::map<int, hipFunction_t> per_device;
    std::map<int, int> blocks_per_cu;
};

struct Circuit {
    uint64_t uid = 0;  // unique per loaded circuit in this process (never reused)
    Aig aig;
    Plan plan1;  // sequential plan (specialized kernel, info)
    Aig fused;   // copy with three-AND XORs fused (interpreter plans of bundles > 1)
    uint32_t fused_xors = 0;  // XOR gates of `fused` in the output cone (each replaces three ANDs)
    // Gate instructions of a bundled interpreter stream (runtime model's gate count).
    uint32_t interp_gates() const {
        const uint32_t g = plan1.num_gate_instrs - 2u * fused_xors;
        return g ? g : 1u;
    }
    double plan_ms = 0;
    std::mutex mu;
    std::map<uint32_t, std::unique_ptr<Plan>> bundled;                  // bundle size -> plan
    std::map<std::pair<int, uint32_t>, Instr*> dev_prog;                  // (device, bundle) -> stream
    std::map<int, std::shared_ptr<JitKernel>> jit;                       // waves_per_eu -> kernel
    std::unique_ptr<LutProgram> lut;                                      // specialized-kernel program
    std::map<uint32_t, std::unique_ptr<Plan>> sim;                        // bundle -> simulation plan
    std::map<std::pair<int, uint32_t>, Instr*> dev_sim_prog;              // (device, bundle) -> stream
    ~Circuit();
    const LutProgram& lut_program();
    // Value-file rows of the interpreter's stream in bundles of 4 (the runtime model's tier).
    uint32_t interp_rows() { return plan_for(4).rows; }
    // The register tier's stream: the plan in bundles of 4, each bundle kRegsBundleWords words
    // (operand and destination words, complement and XOR masks, output flags; see
    // encode_regs_stream; one bundle of zero padding at the end).  Host copy and per-device
    // copies, built on first use.
    const std::vector<uint32_t>& regs_stream();
    const uint32_t* device_regs_stream(int device, hipStream_t s);
    std::vector<uint32_t> regs_host;
    std::map<int, uint32_t*> dev_regs;
    // LUT steps of the specialized program if it is built, else the model's estimate (never
    // builds it).
    uint32_t lut_steps_known();
    const Plan& plan_for(uint32_t bundle);
    const Instr* device_prog(int device, uint32_t bundle, hipStream_t s);
    // Simulation covers every AND gate: the plan is made for the outputs plus every gate
    // that feeds nothing, in bundles of `bundle`; each gate instruction's flags hold its variable.
    const Plan& sim_plan(uint32_t bundle);
    const Instr* device_sim_prog(int device, uint32_t bundle, hipStream_t s);
};

// Device buffers handed out per call (thread-safe pool).  Only the first host_bytes of a
// buffer are staged through the host (control block, best values, descriptors); device-only
// parts such as value files have no pinned host copy.
struct Buffer {
    void* dev = nullptr;
    void* host = nullptr;   // pinned, host_bytes (null when host_bytes is 0)
    size_t bytes = 0;       // device bytes
    size_t host_bytes = 0;
};

struct Device {
    int ordinal = 0;
    hipDeviceProp_t prop{};
    hipStream_t stream = nullptr;          // library stream
    hipStream_t capture_stream = nullptr;  // used only to record hipGraphs
    std::mutex mu;
    std::vector<Buffer> free_bufs;
    size_t pool_device_bytes = 0, pool_pinned_bytes = 0;  // held by the pool (in use or free)
    Buffer acquire(size_t bytes) { return acquire(bytes, bytes); }
    Buffer acquire(size_t dev_bytes, size_t host_bytes);
    void release(Buffer b);
    // Device address of the no-allocation entry point's static scratch array on this device
    // (looked up once, at set-up, with this device current).
    void* noalloc_scratch = nullptr;
    std::mutex noalloc_mu;  // one no-allocation check at a time per device
};
Device& device(int ordinal);

// Set-up of the static scratch array for this device (its address on the device).
void noalloc_setup(Device& dev);

// Interpreter schedule: K half-words per lane, bundle B, workgroup size, tile size, tier.
struct Schedule {
    int K = 2;
    int B = 8;
    int block = 256;
    uint64_t tile_hw = 0;  // 0 = derived
    bool lds = true;
    int grid = 0;          // 0 = derived (persistent: fill the chip)
    int regs = 0;          // register tier: value-file rows in VGPRs (K 1, B 4, one wave per workgroup)
};
// Launch the interpreter kernel a schedule names (register, LDS or device-memory tier).
hipError_t launch_schedule(const InterpLaunch& L, const Schedule& sch, hipStream_t stream);
// Register-tier schedule for value files of `rows` rows; false when none holds them or the
// tier is switched off (FASTLEC_ES_INTERP_REGS=0).
bool make_schedule_regs(Device& dev, uint32_t rows, Schedule& out);
bool regs_tier_enabled();
// Waves per CU of device-memory-tier launches (FASTLEC_ES_HBM_WAVES, default 8).
int hbm_waves_per_cu();
// Runs f(0) .. f(n-1) on up to 16 host threads (the caller's included) and returns when all are
// done; the first exception thrown is rethrown.  For per-circuit host work (LUT mapping, kernel
// source) over many circuits.
void parallel_for(size_t n, const std::function<void(size_t)>& f);

struct CheckOut {
    uint64_t best = ~0ull;
    double kernel_ms = 0;
    double compile_ms = 0;
};

// Range of a check in half-words (32 patterns).
struct HwRange {
    uint64_t begin, end;
};
HwRange range_of(uint32_t n, uint64_t begin_word, uint64_t end_word);

// Exact simulation of range r of circuit c on the interpreter with value files in LDS, using
// only the device's static scratch array (no device or pinned allocation).  Returns the
// lowest failing pattern (~0 when none); *ms = host time of launch and wait.
uint64_t noalloc_check(Device& dev, Circuit& c, const fastlec_es_options& o, const HwRange& r, hipStream_t stream,
                       double* ms);

// Descriptors of an interpreter launch, written to `out` in longest-processing-time order
// (most gate evaluations first); cone i reports into best[best_index[i]].  Returns the
// launch's total number of work items.
uint64_t build_descs(Device& dev, const std::vector<Circuit*>& cs, const std::vector<HwRange>& ranges,
                     const std::vector<uint32_t>& best_index, const Schedule& sch, hipStream_t stream,
                     ConeDesc* out);
// One descriptor: cone plan p with its device stream prog over range r, work items numbered
// from item_begin (tile size from the schedule unless sch.tile_hw fixes it).  Returns the
// next free item number.
uint64_t fill_desc(const Plan& p, const Instr* prog, const HwRange& r, uint32_t best_index, const Schedule& sch,
                   uint64_t item_begin, ConeDesc& d);
uint32_t rows_for(const std::vector<Circuit*>& cs, int B);

// Caller-owned device memory that replaces a launch's library buffer (fastlec_es_options
// dev_scratch); null = the library's pool.
struct DevMem {
    void* ptr = nullptr;
    size_t bytes = 0;
};
// Checks that caller memory of `m.bytes` can hold `need` bytes (alignment and size).
void check_dev_mem(const DevMem& m, size_t need);

// One interpreter launch over several cones (k = 1 for a plain check).
void run_interp(Device& dev, const std::vector<Circuit*>& cs, const std::vector<HwRange>& ranges,
                const Schedule& sch, hipStream_t stream, const int* cancel, std::vector<uint64_t>& best,
                double* kernel_ms, DevMem mem = DevMem{});

// space_hw: half-words the launch will cover (0 = not known: device-memory files only when
// neither registers nor LDS hold them).
Schedule default_schedule(Device& dev, const std::vector<Circuit*>& cs, const fastlec_es_options* o,
                          uint64_t space_hw = 0);
// The server's rule: bundles of B, the option's K (default 2) and workgroup (default 256),
// shrinking the workgroup and then K only until one workgroup's value files fit in LDS.
Schedule shrink_schedule(Device& dev, const std::vector<Circuit*>& cs, const fastlec_es_options* o, int B);
// Schedule for fixed K (half-words per lane), B (bundle) and workgroup size; lds = prefer LDS
// value files.  Returns false when that combination does not fit (LDS too small).
bool make_schedule(Device& dev, const std::vector<Circuit*>& cs, int K, int B, int block, bool lds, Schedule& out);
bool make_schedule_rows(Device& dev, uint32_t rows, int K, int B, int block, bool lds, Schedule& out);


// Sub-miter of candidate pair (target, class_of[target]) by virtual sweeping, as ASCII AIGER;
// inputs (if not null) receives the original input index of each sub-miter input.
std::string submiter_aag(const Aig& g, const uint32_t* class_of, const uint8_t* polarity, uint64_t rows,
                         uint32_t target, std::vector<uint32_t>* inputs);

// Issue-rate probe (variant 0: v_bitop3_b32 on three VGPRs, 1: on two VGPRs and an SGPR,
// 2: v_xor_b32), `waves_per_simd` waves per SIMD; returns wave64 VALU instructions per second
// (kernel time in *ms).
double valu_probe(Device& dev, uint32_t variant, uint32_t waves_per_simd, uint32_t iters, hipStream_t stream,
                  double* ms);

// Random-pattern simulation: value of every variable on `words` columns of input words
// (pi: n rows, sig: max_var + 1 rows, both row-major on the device).
void run_sim(Device& dev, Circuit& c, const uint32_t* pi, uint64_t words, uint32_t* sig,
             const fastlec_es_options* o, hipStream_t stream, double* kernel_ms);
// Fastest interpreter schedule for this set of cones, measured on a bounded prefix of each
// cone's range and cached per device and batch shape.
Schedule autotune(Device& dev, const std::vector<Circuit*>& cs, const std::vector<HwRange>& ranges, hipStream_t stream,
                  bool hbm);
// One persistent interpreter launch over whole spaces, captured once as a hipGraph
// (descriptor upload, kernel, result readback) and replayed for identical batches.
void run_batch_graph(Device& dev, const std::vector<Circuit*>& cs, const std::vector<HwRange>& ranges,
                     const Schedule& sch, hipStream_t stream, std::vector<uint64_t>& best, double* ms);

// Specialized kernel.  Occupancy target (waves per SIMD) and workgroup size default to the
// tuned values; FASTLEC_ES_JIT_WAVES and FASTLEC_ES_JIT_BLOCK override them.
int specialized_waves_per_eu();
int specialized_block();
int specialized_scalar_policy();  // FASTLEC_ES_JIT_SCALAR: 0 all, 1 pure uniform only, 2 none
std::shared_ptr<JitKernel> jit_kernel(Circuit& c, int waves_per_eu, double* compile_ms);
// How jit_kernels splits kernels into hipRTC programs.  kGroup: a group of 4 or more kernels
// is spread over the compile helper processes (as many programs as helpers run at once), fewer
// form one program compiled in this process.  kEach: every kernel is a program of its own,
// compiled in a helper process even when alone, so that several callers' compiles overlap.
enum class CompileSplit { kGroup, kEach };
// Number of compile helper processes run at once (FASTLEC_ES_RTC_PROCS, default min(8, half the
// host threads)); 0 when the helper program is missing: compiles then run in this process, and
// hipRTC serializes them.
int compile_helpers();
// The specialized kernels of several circuits, compiled as hipRTC programs of one or more
// kernels (each under its own name): hipRTC's fixed cost, about 0.1 s per program, is paid once
// per program instead of once per circuit, and programs compile side by side in helper
// processes.  Kernels already compiled or cached are reused.  compile_ms (if not null) receives
// each circuit's share of the compile time (0 for reused kernels).
std::vector<std::shared_ptr<JitKernel>> jit_kernels(const std::vector<Circuit*>& cs, int waves_per_eu,
                                                    std::vector<double>* compile_ms,
                                                    CompileSplit split = CompileSplit::kGroup);
// The circuit's specialized kernel if it is already compiled, else null.  Never compiles and
// never waits: a kernel whose compile is in progress counts as not ready.
std::shared_ptr<JitKernel> jit_ready(Circuit& c, int waves_per_eu);
void run_jit(Device& dev, Circuit& c, JitKernel& k, const HwRange& r, uint64_t tile_hw, hipStream_t stream,
             const int* cancel, uint64_t* best, double* kernel_ms, DevMem mem = DevMem{});
// The same launch in two parts, for callers that keep `best` and the claim counter in their
// own device memory (the server): the grid and tiling of range r, then the launch alone.
// *next_item must be zero when the kernel starts.
struct JitLaunchPlan {
    hipFunction_t fn = nullptr;
    int grid = 0, block = 0;
    uint64_t hw_begin = 0, hw_end = 0, hw_first = 0, tile = 0, total_items = 0;
};
JitLaunchPlan jit_prepare(Device& dev, JitKernel& k, const HwRange& r, uint64_t tile_hw);
void jit_enqueue(const JitLaunchPlan& lp, uint64_t* next_item, uint64_t* best, const int* cancel, hipStream_t stream);
std::string jit_source(const LutProgram& lp, int waves_per_eu, int block, int* waves_used = nullptr);

// The per-pass body as one asm statement with planner-assigned registers (v0.., s<sgpr_base>..).
// Returns false, with the register counts in stats, when it needs more than the limits.
struct BlockStats {
    int vgprs = 0, sgprs = 0, word_operands = 0;
    uint32_t valu = 0, salu = 0, copies = 0, spills = 0;
    bool min_live_order = false;  // the program order did not fit; a pressure-aware order did
    int vgprs_min_live = 0;       // VGPRs of the pressure-aware order when neither fits
    uint32_t lds_ops = 0;         // spill writes and read-backs
    int lds_slots = 0;            // LDS slots used per wave
};
// dist: slots between a VALU result and its first reader that the scheduler aims for.
// bank_aware: place a LUT result in a VGPR bank other than its first reader's other operands.
// lds_slots > 0: vector values beyond vgpr_limit may live in that many per-wave LDS slots
// (256 bytes each); the block then reads the asm operand spill_addr (the lane's byte address
// of slot 0 in the wave's area).
bool emit_block_body(const LutProgram& lp, int vgpr_limit, int sgpr_limit, int sgpr_base, int word_operand_limit,
                     int dist, bool bank_aware, int lds_slots, std::string* code, BlockStats* stats);
int specialized_bank_aware();     // FASTLEC_ES_JIT_BANKS
int specialized_vgpr_cap();       // FASTLEC_ES_JIT_VGPR_CAP: lower VGPR limit of the asm block (tests)
int specialized_latency_slots();  // FASTLEC_ES_JIT_DIST
int specialized_emit_mode();  // FASTLEC_ES_JIT_EMIT: 1 one asm block per pass, 0 one asm statement per gate

}  // namespace fes

// Opaque handle type of the C ABI.
struct fastlec_es_circuit {
    fes::Circuit c;
};
