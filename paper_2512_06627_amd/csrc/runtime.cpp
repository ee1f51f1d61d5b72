#include "runtime.hpp"

#include <algorithm>
#include <atomic>
#include <exception>
#include <thread>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>

namespace fes {

[[noreturn]] void throw_hip(hipError_t e, const char* what) {
    throw Error{kErrDevice, std::string(what) + ": " + hipGetErrorString(e)};
}

bool trace_on() {
    static const bool on = [] {
        const char* v = std::getenv("FASTLEC_ES_TRACE");
        return v && *v && *v != '0';
    }();
    return on;
}

void trace(const char* fmt, ...) {
    if (!trace_on()) return;
    va_list ap;
    va_start(ap, fmt);
    std::fprintf(stderr, "[fastlec_es %.1f ms] ", now_ms());
    std::vfprintf(stderr, fmt, ap);
    std::fputc('\n', stderr);
    std::fflush(stderr);
    va_end(ap);
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ---- circuits --------------------------------------------------------------

Circuit::~Circuit() {
    for (auto& kv : dev_sim_prog) {
        if (!kv.second) continue;
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess && hipSetDevice(kv.first.first) == hipSuccess) {
            (void)hipFree(kv.second);
            (void)hipSetDevice(cur);
        }
    }
    for (auto& kv : dev_regs) {
        if (!kv.second) continue;
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess && hipSetDevice(kv.first) == hipSuccess) {
            (void)hipFree(kv.second);
            (void)hipSetDevice(cur);
        }
    }
    for (auto& kv : dev_prog) {
        if (!kv.second) continue;
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess && hipSetDevice(kv.first.first) == hipSuccess) {
            (void)hipFree(kv.second);
            (void)hipSetDevice(cur);
        }
    }
    // Specialized kernels unload their modules when their code object goes (CodeObject).
}

const Plan& Circuit::plan_for(uint32_t bundle) {
    if (bundle <= 1) return plan1;
    std::lock_guard<std::mutex> g(mu);
    auto it = bundled.find(bundle);
    if (it == bundled.end()) it = bundled.emplace(bundle, std::make_unique<Plan>(make_plan(fused, Order::Auto, bundle))).first;
    return *it->second;
}

uint32_t Circuit::lut_steps_known() {
    std::lock_guard<std::mutex> g(mu);
    return lut ? lut->lut_steps : model_lut_steps_estimate(plan1.num_ands_tfi);
}

const LutProgram& Circuit::lut_program() {
    std::lock_guard<std::mutex> g(mu);
    if (!lut) lut = std::make_unique<LutProgram>(make_lut_program(aig, plan1, specialized_scalar_policy()));
    return *lut;
}

const Instr* Circuit::device_prog(int dev, uint32_t bundle, hipStream_t s) {
    const Plan& p = plan_for(bundle);
    std::lock_guard<std::mutex> g(mu);
    auto key = std::make_pair(dev, bundle);
    auto it = dev_prog.find(key);
    if (it != dev_prog.end()) return it->second;
    Instr* d = nullptr;
    FES_HIP(hipMalloc(&d, std::max<size_t>(p.prog.size(), 1) * sizeof(Instr)));
    if (!p.prog.empty()) {
        FES_HIP(hipMemcpyAsync(d, p.prog.data(), p.prog.size() * sizeof(Instr), hipMemcpyHostToDevice, s));
        FES_HIP(hipStreamSynchronize(s));
    }
    dev_prog[key] = d;
    return d;
}

void encode_regs_stream(const Plan& p, std::vector<uint32_t>& out) {
    if (p.bundle != 4 || p.prog.size() % 4) throw Error{kErrInvalid, "register-tier stream needs bundles of 4"};
    // One zero bundle of padding after the last: the kernel loads the bundle after the current
    // one unconditionally.
    out.assign((p.prog.size() / 4 + 1) * kRegsBundleWords, 0u);
    for (size_t b = 0; b < p.prog.size() / 4; ++b) {
        uint32_t* w = out.data() + b * kRegsBundleWords;
        bool any_out = false;
        for (int u = 0; u < 4; ++u) {
            const Instr& ins = p.prog[b * 4 + u];
            w[u] = ins.a;
            w[4 + u] = ins.b;
            w[8 + u] = ins.d;
            w[12 + u] = (ins.a & kCompl) ? ~0u : 0u;
            w[16 + u] = (ins.b & kCompl) ? ~0u : 0u;
            w[20 + u] = (ins.flags & kXor) ? ~0u : 0u;
            w[24 + u] = ins.flags & (kOutPos | kOutNeg);
            any_out = any_out || (ins.flags & (kOutPos | kOutNeg));
        }
        if (any_out) w[8] |= 0x80000000u;
    }
}

void encode_sim_regs_stream(const Plan& p, const uint32_t* sig, uint64_t words, const uint32_t* dummy,
                            std::vector<uint32_t>& out) {
    if (p.bundle != 4 || p.prog.size() % 4) throw Error{kErrInvalid, "register-tier stream needs bundles of 4"};
    out.assign((p.prog.size() / 4 + 1) * kRegsBundleWords, 0u);
    for (size_t b = 0; b < p.prog.size() / 4; ++b) {
        uint32_t* w = out.data() + b * kRegsBundleWords;
        for (int u = 0; u < 4; ++u) {
            const size_t t = b * 4 + u;
            const Instr& ins = p.prog[t];
            w[u] = ins.a;
            w[4 + u] = ins.b;
            w[8 + u] = ins.d;
            w[12 + u] = (ins.a & kCompl) ? ~0u : 0u;
            w[16 + u] = (ins.b & kCompl) ? ~0u : 0u;
            // variable defined by the instruction (gates only): its signature row, else the dummy row
            const uint64_t addr = p.instr_gate[t] == UINT32_MAX
                                      ? (uint64_t)dummy
                                      : (uint64_t)(sig + (uint64_t)(p.num_inputs + 1 + p.instr_gate[t]) * words);
            w[20 + 2 * u] = (uint32_t)addr;
            w[21 + 2 * u] = (uint32_t)(addr >> 32);
        }
    }
}

const std::vector<uint32_t>& Circuit::regs_stream() {
    const Plan& p = plan_for(4);
    std::lock_guard<std::mutex> g(mu);
    if (regs_host.empty() && !p.prog.empty()) encode_regs_stream(p, regs_host);
    return regs_host;
}

const uint32_t* Circuit::device_regs_stream(int dev, hipStream_t s) {
    const std::vector<uint32_t>& h = regs_stream();
    std::lock_guard<std::mutex> g(mu);
    auto it = dev_regs.find(dev);
    if (it != dev_regs.end()) return it->second;
    uint32_t* d = nullptr;
    FES_HIP(hipMalloc(&d, std::max<size_t>(h.size(), 1) * sizeof(uint32_t)));
    if (!h.empty()) {
        FES_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
        FES_HIP(hipStreamSynchronize(s));
    }
    dev_regs[dev] = d;
    return d;
}

const Plan& Circuit::sim_plan(uint32_t bundle) {
    std::lock_guard<std::mutex> g(mu);
    std::unique_ptr<Plan>& sim = this->sim[bundle];  // bundle 4 (register tier), 8 or 16
    if (!sim) {
        Aig all = aig;
        std::vector<uint8_t> read(all.max_var() + 1, 0);
        for (uint32_t k = 0; k < all.num_ands(); ++k) read[all.and_r0[k] >> 1] = read[all.and_r1[k] >> 1] = 1;
        for (uint32_t o : all.outputs) read[o >> 1] = 1;
        for (uint32_t k = 0; k < all.num_ands(); ++k)
            if (!read[all.num_inputs + 1 + k]) all.outputs.push_back(2 * (all.num_inputs + 1 + k));
        sim = std::make_unique<Plan>(make_plan(all, Order::Auto, bundle));
        if (sim->num_ands_tfi != aig.num_ands()) throw Error{kErrInvalid, "simulation plan misses gates"};
        const std::string err = validate_plan(all, *sim);
        if (!err.empty()) throw Error{kErrInvalid, "simulation plan: " + err};
    }
    return *sim;
}

const Instr* Circuit::device_sim_prog(int dev, uint32_t bundle, hipStream_t s) {
    const Plan& p = sim_plan(bundle);
    std::lock_guard<std::mutex> g(mu);
    auto it = dev_sim_prog.find({dev, bundle});
    if (it != dev_sim_prog.end()) return it->second;
    std::vector<Instr> prog = p.prog;
    for (size_t t = 0; t < prog.size(); ++t)
        prog[t].flags = p.instr_gate[t] == UINT32_MAX ? 0u : p.num_inputs + 1 + p.instr_gate[t];
    Instr* d = nullptr;
    FES_HIP(hipMalloc(&d, std::max<size_t>(prog.size(), 1) * sizeof(Instr)));
    if (!prog.empty()) {
        FES_HIP(hipMemcpyAsync(d, prog.data(), prog.size() * sizeof(Instr), hipMemcpyHostToDevice, s));
        FES_HIP(hipStreamSynchronize(s));
    }
    dev_sim_prog[{dev, bundle}] = d;
    return d;
}

// ---- devices ----------------------------------------------------------------

Buffer Device::acquire(size_t dev_bytes, size_t host_bytes) {
    dev_bytes = (dev_bytes + 4095) & ~size_t(4095);
    host_bytes = (host_bytes + 4095) & ~size_t(4095);
    {
        std::lock_guard<std::mutex> g(mu);
        size_t best = SIZE_MAX;
        for (size_t i = 0; i < free_bufs.size(); ++i) {
            const Buffer& f = free_bufs[i];
            if (f.bytes >= dev_bytes && f.host_bytes >= host_bytes &&
                (best == SIZE_MAX || f.bytes + f.host_bytes < free_bufs[best].bytes + free_bufs[best].host_bytes))
                best = i;
        }
        if (best != SIZE_MAX) {
            Buffer b = free_bufs[best];
            free_bufs.erase(free_bufs.begin() + best);
            return b;
        }
    }
    Buffer b;
    b.bytes = dev_bytes;
    b.host_bytes = host_bytes;
    if (dev_bytes && hipMalloc(&b.dev, dev_bytes) != hipSuccess) throw Error{kErrNoMem, "device allocation failed"};
    if (host_bytes && hipHostMalloc(&b.host, host_bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(b.dev);
        throw Error{kErrNoMem, "pinned host allocation failed"};
    }
    std::lock_guard<std::mutex> g(mu);
    pool_device_bytes += dev_bytes;
    pool_pinned_bytes += host_bytes;
    return b;
}

void Device::release(Buffer b) {
    std::lock_guard<std::mutex> g(mu);
    free_bufs.push_back(b);
}

Device& device(int ordinal) {
    static std::mutex mu;
    static std::map<int, std::unique_ptr<Device>> devs;
    std::lock_guard<std::mutex> g(mu);
    auto it = devs.find(ordinal);
    if (it != devs.end()) {
        FES_HIP(hipSetDevice(ordinal));
        return *it->second;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) throw Error{kErrDevice, "no HIP device"};
    if (ordinal < 0 || ordinal >= count) throw Error{kErrInvalid, "device ordinal out of range"};
    trace("device %d: first use, %d devices", ordinal, count);
    auto d = std::make_unique<Device>();
    d->ordinal = ordinal;
    FES_HIP(hipSetDevice(ordinal));
    FES_HIP(hipGetDeviceProperties(&d->prop, ordinal));
    if (std::strncmp(d->prop.gcnArchName, "gfx950", 6) != 0)
        throw Error{kErrDevice, std::string("built for gfx950, device is ") + d->prop.gcnArchName};
    FES_HIP(hipStreamCreateWithFlags(&d->stream, hipStreamNonBlocking));
    FES_HIP(hipStreamCreateWithFlags(&d->capture_stream, hipStreamNonBlocking));
    noalloc_setup(*d);
    trace("device %d: %s, %d CUs, LDS %zu per block / %zu per CU", ordinal, d->prop.gcnArchName,
          d->prop.multiProcessorCount, (size_t)d->prop.sharedMemPerBlock, (size_t)d->prop.maxSharedMemoryPerMultiProcessor);
    Device& ref = *d;
    devs[ordinal] = std::move(d);
    return ref;
}

HwRange range_of(uint32_t n, uint64_t begin_word, uint64_t end_word) {
    const uint64_t words = n >= 6 ? (1ull << (n - 6)) : 1ull;
    const uint64_t halfs = n >= 5 ? (1ull << (n - 5)) : 1ull;
    if (begin_word == 0 && end_word == 0) end_word = words;
    if (begin_word >= end_word || end_word > words) throw Error{kErrInvalid, "word range empty or beyond 2^(n-6) words"};
    return HwRange{std::min(2 * begin_word, halfs), std::min(2 * end_word, halfs)};
}

// ---- interpreter launches ------------------------------------------------------

namespace {

struct Layout {
    size_t best_off, desc_off, files_off, total;
};

Layout layout(size_t k, size_t file_bytes) {
    Layout l;
    l.best_off = sizeof(LaunchCtl);
    l.desc_off = (l.best_off + 8 * k + 63) & ~size_t(63);
    l.files_off = (l.desc_off + sizeof(ConeDesc) * k + 255) & ~size_t(255);
    l.total = l.files_off + file_bytes;
    return l;
}

int max_waves_per_cu(const Device&) { return 32; }

}  // namespace

void parallel_for(size_t n, const std::function<void(size_t)>& f) {
    if (n == 0) return;
    const size_t hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t workers = std::min<size_t>({n, hw, 16});
    if (workers == 1) {
        for (size_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<size_t> next{0};
    std::mutex emu;
    std::exception_ptr first;
    auto run = [&] {
        for (size_t i; (i = next.fetch_add(1)) < n;) {
            try {
                f(i);
            } catch (...) {
                std::lock_guard<std::mutex> g(emu);
                if (!first) first = std::current_exception();
            }
        }
    };
    std::vector<std::thread> th;
    for (size_t t = 1; t < workers; ++t) th.emplace_back(run);
    run();
    for (auto& t : th) t.join();
    if (first) std::rethrow_exception(first);
}

bool regs_tier_enabled() {
    static const bool on = [] {
        const char* v = std::getenv("FASTLEC_ES_INTERP_REGS");
        return !(v && std::atoi(v) == 0);
    }();
    return on;
}

bool make_schedule_regs(Device& dev, uint32_t rows, Schedule& s) {
    int waves = 0;
    const int regs = interp_regs_rows(rows, &waves);
    if (!regs || !regs_tier_enabled()) return false;
    s = Schedule{};
    s.K = 1;
    s.B = 4;
    s.block = 64;
    s.lds = false;
    s.regs = regs;
    s.grid = dev.prop.multiProcessorCount * 4 * waves;  // `waves` one-wave workgroups per SIMD
    return true;
}

hipError_t launch_schedule(const InterpLaunch& L, const Schedule& sch, hipStream_t stream) {
    if (sch.regs) return launch_interp_regs(L, sch.regs, sch.grid, stream);
    return launch_interp(L, sch.K, sch.B, sch.lds, sch.grid, sch.block, stream);
}

bool make_schedule(Device& dev, const std::vector<Circuit*>& cs, int K, int B, int block, bool lds, Schedule& s) {
    return make_schedule_rows(dev, rows_for(cs, B), K, B, block, lds, s);
}

bool make_schedule_rows(Device& dev, uint32_t rows, int K, int B, int block, bool lds, Schedule& s) {
    s = Schedule{};
    s.K = K;
    s.B = B;
    s.block = block;
    s.lds = lds;
    const size_t lds_cu = dev.prop.maxSharedMemoryPerMultiProcessor ? dev.prop.maxSharedMemoryPerMultiProcessor : 65536;
    const size_t lds_blk = dev.prop.sharedMemPerBlock ? dev.prop.sharedMemPerBlock : 65536;
    const int waves_per_block = block / 64;
    if (lds && interp_lds_bytes(rows, K, waves_per_block) > lds_blk) return false;
    int blocks_per_cu;
    if (lds) {
        blocks_per_cu = (int)(lds_cu / interp_lds_bytes(rows, K, waves_per_block));
        blocks_per_cu = std::max(1, std::min(blocks_per_cu, max_waves_per_cu(dev) / waves_per_block));
    } else {
        blocks_per_cu = std::max(1, hbm_waves_per_cu() / waves_per_block);
    }
    s.grid = dev.prop.multiProcessorCount * blocks_per_cu;
    return true;
}

int hbm_waves_per_cu() {
    static const int w = [] {
        const char* v = std::getenv("FASTLEC_ES_HBM_WAVES");
        const int x = v ? std::atoi(v) : 0;
        return x >= 1 && x <= 32 ? x : 8;  // 8 measured best of 8/16/24/32 on files of 268-529 rows
    }();
    return w;
}

Schedule default_schedule(Device& dev, const std::vector<Circuit*>& cs, const fastlec_es_options* o,
                          uint64_t space_hw) {
    const bool fix_k = o && o->words_per_thread, fix_block = o && o->wg_size;
    const int K0 = fix_k ? (int)o->words_per_thread : 2;
    const int block0 = fix_block ? (int)o->wg_size : 256;
    const bool hbm = o && o->kernel == FASTLEC_KERNEL_INTERP_HBM;
    if (K0 != 1 && K0 != 2 && K0 != 4) throw Error{kErrInvalid, "words_per_thread must be 1, 2 or 4"};
    if (block0 < 64 || block0 > 1024 || block0 % 64) throw Error{kErrInvalid, "wg_size must be a multiple of 64 in [64, 1024]"};
    Schedule s;
    // Value files in VGPRs when they fit and the caller fixes no other schedule: two to four
    // waves per SIMD instead of the one that LDS files allow.
    if (!hbm && !fix_k && !fix_block && make_schedule_regs(dev, rows_for(cs, 4), s)) return s;
    if (!hbm) {
        // Value files in LDS: the interpreter is latency-bound, so take the words per lane and
        // workgroup size that keep the most pattern words in flight per CU (waves x K), with
        // bundles of 16 gates (8 with four words per lane, which spills registers).  Small
        // workgroups pack LDS more finely: 164 rows at one word per lane fit three one-wave
        // workgroups per CU but one two-wave workgroup.
        bool have = false;
        int best = -1;
        for (int K : fix_k ? std::vector<int>{K0} : std::vector<int>{1, 2})
            for (int block : fix_block ? std::vector<int>{block0} : std::vector<int>{256, 128, 64}) {
                Schedule t;
                if (!make_schedule(dev, cs, K, K <= 2 ? 16 : 8, block, true, t)) continue;
                const int score = t.grid / std::max(1, dev.prop.multiProcessorCount) * (block / 64) * K;
                if (!have || score > best || (score == best && K == s.K)) {  // ties: smaller workgroup
                    have = true;
                    best = score;
                    s = t;
                }
            }
        // Files too large for the register tier hold at most two waves per CU in LDS (61 KB and
        // more per wave).  When the space has at least one pass for every wave of a
        // device-memory launch (one word per lane, one-wave workgroups), that tier is faster
        // (1.8-3.9x on files of 268-417 rows at 2^22-2^26 half-words); on smaller spaces the
        // lower latency of LDS wins (1.3-1.5x at 2^11-2^15 half-words).
        if (have && best < 4 && !fix_k && !fix_block && space_hw) {
            Schedule h;
            if (make_schedule(dev, cs, 1, 8, 64, false, h) && space_hw / 64 >= (uint64_t)h.grid) return h;
        }
        if (have) return s;
    }
    // Value files in device memory.
    make_schedule(dev, cs, K0, 8, block0, false, s);
    return s;
}

Schedule shrink_schedule(Device& dev, const std::vector<Circuit*>& cs, const fastlec_es_options* o, int B) {
    int K = (o && o->words_per_thread) ? (int)o->words_per_thread : 2;
    int block = (o && o->wg_size) ? (int)o->wg_size : 256;
    bool lds = !(o && o->kernel == FASTLEC_KERNEL_INTERP_HBM);
    if (K != 1 && K != 2 && K != 4) throw Error{kErrInvalid, "words_per_thread must be 1, 2 or 4"};
    if (block < 64 || block > 1024 || block % 64) throw Error{kErrInvalid, "wg_size must be a multiple of 64 in [64, 1024]"};
    Schedule s;
    while (lds && !make_schedule(dev, cs, K, B, block, true, s)) {
        if (!(o && o->wg_size) && block > 64) block /= 2;
        else if (!(o && o->words_per_thread) && K > 1) K /= 2;
        else lds = false;
    }
    if (!lds) make_schedule(dev, cs, K, B, block, false, s);
    return s;
}

uint32_t rows_for(const std::vector<Circuit*>& cs, int B) {
    uint32_t rows = 0;
    for (Circuit* c : cs) rows = std::max(rows, c->plan_for(B).rows);
    return rows;
}

uint64_t build_descs(Device& dev, const std::vector<Circuit*>& cs, const std::vector<HwRange>& ranges,
                     const std::vector<uint32_t>& best_index, const Schedule& sch, hipStream_t stream,
                     ConeDesc* out) {
    const size_t k = cs.size();
    // Longest-processing-time order by the runtime model's interpreter time: the longest cones
    // get the lowest item numbers, so they start first and the short ones fill the tail.
    std::vector<size_t> order(k);
    std::iota(order.begin(), order.end(), 0);
    std::vector<double> cost(k);
    for (size_t i = 0; i < k; ++i)
        cost[i] = lpt_cost_ms(cs[i]->interp_gates(), cs[i]->interp_rows(),
                              32.0 * (double)(ranges[i].end - ranges[i].begin));
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    uint64_t item = 0;
    for (size_t t = 0; t < k; ++t) {
        size_t i = order[t];
        Circuit* c = cs[i];
        const Instr* prog = sch.regs ? (const Instr*)c->device_regs_stream(dev.ordinal, stream)
                                     : c->device_prog(dev.ordinal, sch.B, stream);
        item = fill_desc(c->plan_for(sch.B), prog, ranges[i], best_index[i], sch, item, out[t]);
    }
    return item;
}

uint64_t fill_desc(const Plan& p, const Instr* prog, const HwRange& r, uint32_t best_index, const Schedule& sch,
                   uint64_t item_begin, ConeDesc& d) {
    const uint32_t pass_hw = 64u * (uint32_t)sch.K;
    const size_t waves = (size_t)sch.grid * (sch.block / 64);
    d.prog = prog;
    d.n_instr = (uint32_t)p.prog.size();
    d.n_inputs = p.num_inputs;
    d.rows = p.rows;
    d.best_index = best_index;
    d.hw_begin = r.begin;
    d.hw_end = r.end;
    d.hw_first = r.begin / pass_hw * pass_hw;
    const uint64_t span = d.hw_end - d.hw_first;
    uint64_t tile = sch.tile_hw;
    if (!tile) {  // about 16 work items per wave over the launch, within [1, 64] passes
        const uint64_t target = span / std::max<uint64_t>(1, waves * 16);
        tile = pass_hw;
        while (tile < target && tile < 64ull * pass_hw) tile *= 2;
    }
    tile = (tile + pass_hw - 1) / pass_hw * pass_hw;
    d.tile_hw = tile;
    d.item_begin = item_begin;
    d.item_end = item_begin + (span + tile - 1) / tile;
    return d.item_end;
}

void check_dev_mem(const DevMem& m, size_t need) {
    if ((uintptr_t)m.ptr % 256)
        throw Error{kErrInvalid, "dev_scratch must be 256-byte aligned"};
    if (m.bytes < need)
        throw Error{kErrInvalid, "dev_scratch holds " + std::to_string(m.bytes) + " bytes; this check needs " +
                                     std::to_string(need)};
}

void run_interp(Device& dev, const std::vector<Circuit*>& cs, const std::vector<HwRange>& ranges, const Schedule& sch,
                hipStream_t stream, const int* cancel, std::vector<uint64_t>& best, double* kernel_ms, DevMem mem) {
    const size_t k = cs.size();
    const uint32_t rows_max = rows_for(cs, sch.B);
    const size_t waves = (size_t)sch.grid * (sch.block / 64);
    const size_t file_bytes = (sch.lds || sch.regs) ? 0 : waves * rows_max * 64ull * sch.K * 4ull;
    Layout lay = layout(k, file_bytes);
    if (mem.ptr) check_dev_mem(mem, lay.total);
    // With caller memory the pool only supplies the pinned staging of the control block.
    Buffer buf = dev.acquire(mem.ptr ? 0 : lay.total, lay.files_off);
    struct Releaser {
        Device& d;
        Buffer b;
        ~Releaser() { d.release(b); }
    } rel{dev, buf};

    uint8_t* host = (uint8_t*)buf.host;
    std::memset(host, 0, lay.files_off);
    uint64_t* hbest = (uint64_t*)(host + lay.best_off);
    for (size_t i = 0; i < k; ++i) hbest[i] = ~0ull;
    std::vector<uint32_t> idx(k);
    std::iota(idx.begin(), idx.end(), 0u);
    const uint64_t items = build_descs(dev, cs, ranges, idx, sch, stream, (ConeDesc*)(host + lay.desc_off));
    uint8_t* devp = (uint8_t*)(mem.ptr ? mem.ptr : buf.dev);
    InterpLaunch L;
    L.cones = (const ConeDesc*)(devp + lay.desc_off);
    L.num_cones = (uint32_t)k;
    L.rows_max = rows_max;
    L.total_items = items;
    L.ctl = (LaunchCtl*)devp;
    L.best = (unsigned long long*)(devp + lay.best_off);
    L.hbm_rows = (sch.lds || sch.regs) ? nullptr : (uint32_t*)(devp + lay.files_off);
    L.cancel = cancel;

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
    trace("interp launch: %zu cones, %llu items, K=%d B=%d %s grid=%d block=%d rows=%u", k,
          (unsigned long long)items, sch.K, sch.B, sch.regs ? "regs" : sch.lds ? "lds" : "hbm", sch.grid, sch.block,
          rows_max);
    FES_HIP(hipMemcpyAsync(devp, host, lay.files_off, hipMemcpyHostToDevice, stream));
    FES_HIP(hipEventRecord(e0, stream));
    FES_HIP(launch_schedule(L, sch, stream));
    FES_HIP(hipEventRecord(e1, stream));
    FES_HIP(hipMemcpyAsync(hbest, devp + lay.best_off, 8 * k, hipMemcpyDeviceToHost, stream));
    FES_HIP(hipStreamSynchronize(stream));
    trace("interp done");
    float ms = 0;
    FES_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (kernel_ms) *kernel_ms = ms;
    best.assign(hbest, hbest + k);
}

}  // namespace fes

namespace fes {

namespace {

// Simulation with the value file in VGPRs (register tier).  Returns false when the circuit's
// simulation plan does not fit that tier, or the call asks for another schedule.
bool run_sim_regs(Device& dev, Circuit& c, const uint32_t* pi, uint64_t words, uint32_t* sig,
                  const fastlec_es_options* o, hipStream_t stream, double* kernel_ms) {
    if (!regs_tier_enabled() || words > (1ull << 30)) return false;
    if (o && (o->kernel == FASTLEC_KERNEL_INTERP_HBM || o->words_per_thread || o->wg_size)) return false;
    const Plan& p = c.sim_plan(4);
    int waves_per_simd = 0;
    const int regs = interp_regs_rows(p.rows, &waves_per_simd);
    if (!regs || p.prog.empty()) return false;
    bool any_dummy = false;
    for (uint32_t g : p.instr_gate) any_dummy = any_dummy || g == UINT32_MAX;

    // One work item per pass of 64 words when passes are few, so the last round of claims is as
    // full as it can be; a grid no larger than the passes need.
    const uint64_t passes = (words + 63) / 64;
    const uint64_t cap = (uint64_t)dev.prop.multiProcessorCount * 4 * waves_per_simd;
    const uint64_t rounds = (passes + cap - 1) / cap;
    const uint64_t grid = (passes + rounds - 1) / rounds;
    uint64_t tile_passes = 1;
    if (o && o->tile_words) tile_passes = std::max<uint64_t>(1, (2ull * o->tile_words + 63) / 64);
    else
        while (tile_passes < 16 && passes / (tile_passes * 2) >= grid * 16) tile_passes *= 2;

    const size_t nbytes_stream = (p.prog.size() / 4 + 1) * kRegsBundleWords * sizeof(uint32_t);
    Layout lay = layout(1, 0);
    const size_t stream_off = lay.files_off;
    const size_t dummy_off = (stream_off + nbytes_stream + 255) & ~size_t(255);
    const size_t total = dummy_off + (any_dummy ? words * 4ull : 0);
    Buffer buf = dev.acquire(total, dummy_off);
    struct Releaser {
        Device& d;
        Buffer b;
        ~Releaser() { d.release(b); }
    } rel{dev, buf};
    uint8_t* host = (uint8_t*)buf.host;
    uint8_t* devp = (uint8_t*)buf.dev;
    std::memset(host, 0, lay.files_off);
    std::vector<uint32_t> st;
    encode_sim_regs_stream(p, sig, words, (const uint32_t*)(devp + dummy_off), st);
    std::memcpy(host + stream_off, st.data(), st.size() * sizeof(uint32_t));

    ConeDesc& d = *(ConeDesc*)(host + lay.desc_off);
    d.prog = (const Instr*)(devp + stream_off);
    d.n_instr = (uint32_t)p.prog.size();
    d.n_inputs = p.num_inputs;
    d.rows = p.rows;
    d.hw_begin = 0;
    d.hw_end = words;
    d.hw_first = 0;
    d.tile_hw = 64ull * tile_passes;
    d.item_begin = 0;
    d.item_end = (words + d.tile_hw - 1) / d.tile_hw;

    InterpLaunch L;
    L.cones = (const ConeDesc*)(devp + lay.desc_off);
    L.num_cones = 1;
    L.rows_max = p.rows;
    L.total_items = d.item_end;
    L.ctl = (LaunchCtl*)devp;
    L.best = (unsigned long long*)(devp + lay.best_off);
    L.hbm_rows = nullptr;
    L.cancel = nullptr;
    L.sim_pi = pi;
    L.sim_sig = sig;
    L.sim_words = words;

    ScopedEvent e0, e1;
    trace("sim launch (registers): %llu words, %llu items of %llu passes, file %d rows, grid=%llu",
          (unsigned long long)words, (unsigned long long)L.total_items, (unsigned long long)tile_passes, regs,
          (unsigned long long)grid);
    FES_HIP(hipMemcpyAsync(devp, host, dummy_off, hipMemcpyHostToDevice, stream));
    FES_HIP(hipEventRecord(e0.e, stream));
    FES_HIP(launch_sim_regs(L, regs, (int)grid, stream));
    FES_HIP(hipEventRecord(e1.e, stream));
    FES_HIP(hipStreamSynchronize(stream));
    float ms = 0;
    FES_HIP(hipEventElapsedTime(&ms, e0.e, e1.e));
    if (kernel_ms) *kernel_ms = ms;
    return true;
}

}  // namespace

void run_sim(Device& dev, Circuit& c, const uint32_t* pi, uint64_t words, uint32_t* sig,
             const fastlec_es_options* o, hipStream_t stream, double* kernel_ms) {
    if (run_sim_regs(dev, c, pi, words, sig, o, stream, kernel_ms)) return;
    // Bundles of 16 gates give each wave twice the independent LDS reads per wait (not with 4
    // words per lane, which spills registers).  Words per lane and workgroup size as for plain
    // checks: the most pattern words in flight per CU (16x16 miter, 2^18 words: 2.96 ms with
    // 8-gate bundles, two words per lane and the largest workgroup that fits; 2.30 ms with 16,
    // one and 64 threads).
    const bool fix_k = o && o->words_per_thread, fix_block = o && o->wg_size;
    const int K0 = fix_k ? (int)o->words_per_thread : 1;
    const int block0 = fix_block ? (int)o->wg_size : 256;
    if (K0 != 1 && K0 != 2 && K0 != 4) throw Error{kErrInvalid, "words_per_thread must be 1, 2 or 4"};
    if (block0 < 64 || block0 > 1024 || block0 % 64) throw Error{kErrInvalid, "wg_size must be a multiple of 64 in [64, 1024]"};
    const char* eb = std::getenv("FASTLEC_ES_SIM_BUNDLE");
    const uint32_t B = K0 == 4 || (eb && std::atoi(eb) == 8) ? 8u : 16u;
    const Plan& p = c.sim_plan(B);
    Schedule sch;
    bool have = false;
    if (!(o && o->kernel == FASTLEC_KERNEL_INTERP_HBM)) {
        int best = -1;
        for (int K : fix_k ? std::vector<int>{K0} : std::vector<int>{1, 2})
            for (int block : fix_block ? std::vector<int>{block0} : std::vector<int>{256, 128, 64}) {
                Schedule t;
                if (!make_schedule_rows(dev, p.rows, K, (int)B, block, true, t)) continue;
                const int score = t.grid / std::max(1, dev.prop.multiProcessorCount) * (block / 64) * K;
                // ties go to the smaller workgroup (one-wave workgroups measured best here)
                if (!have || score > best || (score == best && K == sch.K)) {
                    have = true;
                    best = score;
                    sch = t;
                }
            }
    }
    if (!have) make_schedule_rows(dev, p.rows, K0, (int)B, block0, false, sch);

    const size_t waves = (size_t)sch.grid * (sch.block / 64);
    const size_t file_bytes = sch.lds ? 0 : waves * p.rows * 64ull * sch.K * 4ull;
    Layout lay = layout(1, file_bytes);
    Buffer buf = dev.acquire(lay.total, lay.files_off);
    struct Releaser {
        Device& d;
        Buffer b;
        ~Releaser() { d.release(b); }
    } rel{dev, buf};
    uint8_t* host = (uint8_t*)buf.host;
    std::memset(host, 0, lay.files_off);
    *(uint64_t*)(host + lay.best_off) = ~0ull;

    ConeDesc& d = *(ConeDesc*)(host + lay.desc_off);
    const uint32_t pass_hw = 64u * (uint32_t)sch.K;
    d.prog = c.device_sim_prog(dev.ordinal, B, stream);
    d.n_instr = (uint32_t)p.prog.size();
    d.n_inputs = p.num_inputs;
    d.rows = p.rows;
    d.best_index = 0;
    d.hw_begin = 0;
    d.hw_end = words;
    d.hw_first = 0;
    uint64_t tile = o && o->tile_words ? 2ull * o->tile_words : 0;
    if (!tile) {  // about 16 work items per wave, within [1, 64] passes
        const uint64_t target = words / std::max<uint64_t>(1, waves * 16);
        tile = pass_hw;
        while (tile < target && tile < 64ull * pass_hw) tile *= 2;
    }
    d.tile_hw = (tile + pass_hw - 1) / pass_hw * pass_hw;
    d.item_begin = 0;
    d.item_end = (words + d.tile_hw - 1) / d.tile_hw;

    uint8_t* devp = (uint8_t*)buf.dev;
    InterpLaunch L;
    L.cones = (const ConeDesc*)(devp + lay.desc_off);
    L.num_cones = 1;
    L.rows_max = p.rows;
    L.total_items = d.item_end;
    L.ctl = (LaunchCtl*)devp;
    L.best = (unsigned long long*)(devp + lay.best_off);
    L.hbm_rows = sch.lds ? nullptr : (uint32_t*)(devp + lay.files_off);
    L.cancel = nullptr;
    L.sim_pi = pi;
    L.sim_sig = sig;
    L.sim_words = words;

    ScopedEvent e0, e1;
    trace("sim launch: %llu words, %llu items, K=%d %s grid=%d block=%d rows=%u", (unsigned long long)words,
          (unsigned long long)L.total_items, sch.K, sch.lds ? "lds" : "hbm", sch.grid, sch.block, p.rows);
    FES_HIP(hipMemcpyAsync(devp, host, lay.files_off, hipMemcpyHostToDevice, stream));
    FES_HIP(hipEventRecord(e0.e, stream));
    FES_HIP(launch_interp_sim(L, sch.K, (int)B, sch.lds, sch.grid, sch.block, stream));
    FES_HIP(hipEventRecord(e1.e, stream));
    FES_HIP(hipStreamSynchronize(stream));
    float ms = 0;
    FES_HIP(hipEventElapsedTime(&ms, e0.e, e1.e));
    if (kernel_ms) *kernel_ms = ms;
}

}  // namespace fes
