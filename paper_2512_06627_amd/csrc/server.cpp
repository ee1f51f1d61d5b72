// Continuous-batching exact-simulation server.
//
// Jobs are admitted by memory charge (peak live slots x words in flight x 8 B)
// against a budget, and every step is one interpreter launch over the next
// pattern slice of every job in flight (plus one launch per job on the specialized
// tier, below).  A job that arrives while others are on
// the device joins them at the next step; a job retires as soon as its answer
// is final, and its charge goes back to the budget.  Slices are sized so a
// step takes about FASTLEC_ES_SERVER_STEP_MS milliseconds (default 10), from a
// running estimate of the interpreter's node*pattern rate, and every job in
// flight gets the same amount of gate evaluations per step.
//
// Device-resident job table: best-so-far value per slot (written by the
// kernels' atomicMin, read back after each step, reset when a slot is reused)
// and the slot's descriptors, which the host refreshes each step with the
// job's next slice.
//
// Specialized tier: pattern spaces differ by many orders of magnitude (2^n), so a
// few large jobs carry most of the work.  A job whose remaining interpreter time is
// estimated well above the cost of compiling its specialized kernel is handed to the
// compile threads (one per compile helper process) while it keeps running on the
// interpreter; from the step after the kernel is ready, the job's slices run on the
// specialized kernel instead (same
// ascending slices, same best[] entry, so the answer cannot change).  Circuits
// submitted again reuse their compiled kernel at once.
#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <thread>

#include "runtime.hpp"

using namespace fes;

namespace {

struct Job {
    uint64_t ticket = 0;
    Circuit* c = nullptr;
    uint64_t charge = 0;
    HwRange range{0, 0};
    uint64_t cursor = 0;  // first half-word not yet simulated
    uint32_t slot = UINT32_MAX;
    double t_submit = 0, t_admit = 0;
    double kernel_ms = 0;
    bool done = false;
    int status = FASTLEC_OK;
    fastlec_es_result res{};
    bool compile_queued = false;     // handed to the compile threads
    bool compiling = false;          // a compile thread is using the circuit
    std::shared_ptr<JitKernel> jit;  // set when the specialized kernel is ready
};

uint64_t env_u64(const char* name, uint64_t dflt) {
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::strtoull(v, nullptr, 0);
}

// Interpreter configuration of the server's launches: half-words per lane (1), gates per bundle
// (16), and the LDS group's workgroup chosen for the most waves per CU (else shrunk only until
// it fits).  Measured on the serving mix at 0.7 load against 2 half-words, 8-gate bundles and
// shrinking: p50 1.8 vs 2.1 ms, p90 19 vs 26 ms, p99 37 vs 44 ms, the same capacity.
int server_k() {
    const char* v = std::getenv("FASTLEC_ES_SERVER_K");
    return v && std::atoi(v) == 2 ? 2 : 1;
}
int server_bundle() {
    const char* v = std::getenv("FASTLEC_ES_SERVER_BUNDLE");
    return v && std::atoi(v) == 8 ? 8 : 16;
}
bool server_occupancy() {
    const char* v = std::getenv("FASTLEC_ES_SERVER_OCCUPANCY");
    return !(v && std::atoi(v) == 0);
}
constexpr uint32_t kCapacity = 1024;

}  // namespace

struct fastlec_es_server {
    fastlec_es_options opts{};
    Device* dev = nullptr;
    hipStream_t stream = nullptr;
    uint64_t budget = 0, chunk_words = 1ull << 22;
    double step_ms_target = 10.0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<Job*> queue;
    std::vector<Job*> active;
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    fastlec_es_server_stats st{};
    std::string fatal;
    int fatal_code = 0;

    // device job table: [ctl lds][ctl hbm][best x capacity][desc lds x capacity][desc hbm x capacity]
    Buffer table;
    size_t off_best = 2 * sizeof(LaunchCtl), off_desc_lds = 0, off_desc_hbm = 0;
    Buffer files;  // value files of the device-memory tier
    std::vector<uint32_t> free_slots;
    double rate = 1e14;  // node*patterns per second, running estimate
    std::thread th;
    // specialized tier
    int jit_mode = 1;        // 0 off, 1 by estimate, 2 every job (test hook)
    double jit_rate = 2e15;  // node*patterns per second of the specialized kernel, estimate
    size_t off_ctl_jit = 0;  // per-slot claim counters of specialized launches
    std::deque<Job*> compile_queue;
    std::condition_variable cv_compile;
    std::vector<std::thread> compilers;
    void compile_loop();
    void plan_tiers(const std::vector<Job*>& act);

    uint64_t charge_of(const Circuit& c) const {
        const uint32_t n = c.plan1.num_inputs;
        const uint64_t words = n >= 6 ? (1ull << (n - 6)) : 1ull;
        return (uint64_t)std::max<uint32_t>(1, c.plan1.peak_slots) * std::min(words, chunk_words) * 8ull;
    }
    void loop();
    void step(const std::vector<Job*>& act);
    void finish(Job* j, double now);
};

void fastlec_es_server::compile_loop() {
    // With compile helper processes there is one compile thread per helper, and each takes one
    // job at a time: its kernel compiles alone in a helper as soon as a thread is free, so a
    // job never waits for the rest of a group (the threads' compiles overlap; in this process
    // they would serialize).  Without helpers one thread takes up to eight queued jobs and
    // compiles their kernels as one program, paying hipRTC's fixed cost (about 0.1 s) once.
    const bool helpers = compile_helpers() > 0;
    const size_t kGroup = helpers ? 1 : 8;
    for (;;) {
        std::vector<Job*> group;
        {
            std::unique_lock<std::mutex> g(mu);
            cv_compile.wait(g, [&] { return stop || !compile_queue.empty(); });
            if (stop) return;
            // Largest remaining work first: it gains the most from the specialized kernel.
            while (group.size() < kGroup && !compile_queue.empty()) {
                auto pick = compile_queue.end();
                double most = -1;
                for (auto it = compile_queue.begin(); it != compile_queue.end(); ++it) {
                    const double w = (double)(*it)->c->plan1.num_gate_instrs * (double)((*it)->range.end - (*it)->cursor);
                    if (!(*it)->done && w > most) {
                        most = w;
                        pick = it;
                    }
                }
                if (pick == compile_queue.end()) {  // only finished jobs are left
                    compile_queue.clear();
                    break;
                }
                Job* j = *pick;
                compile_queue.erase(pick);
                j->compiling = true;
                group.push_back(j);
            }
            if (group.empty()) continue;
        }
        std::vector<Circuit*> cs;
        for (Job* j : group) cs.push_back(j->c);
        std::vector<std::shared_ptr<JitKernel>> ks;
        try {
            ks = jit_kernels(cs, specialized_waves_per_eu(), nullptr,
                             helpers ? CompileSplit::kEach : CompileSplit::kGroup);
        } catch (...) {
            // one kernel that does not compile must not keep the others on the interpreter
            ks.assign(group.size(), nullptr);
            for (size_t t = 0; t < group.size(); ++t) {
                try {
                    ks[t] = jit_kernel(*cs[t], specialized_waves_per_eu(), nullptr);
                } catch (...) {
                    ks[t] = nullptr;  // the job stays on the interpreter
                }
            }
        }
        std::lock_guard<std::mutex> g(mu);
        for (size_t t = 0; t < group.size(); ++t) {
            Job* j = group[t];
            j->compiling = false;
            if (ks[t] && ks[t]->code && !j->done) j->jit = ks[t];
        }
        cv_done.notify_all();
    }
}

void fastlec_es_server::plan_tiers(const std::vector<Job*>& act) {
    if (jit_mode == 0) return;
    std::lock_guard<std::mutex> g(mu);
    // Jobs on the interpreter share each step's work equally, so one job's remaining time is
    // its remaining work over its share of the interpreter's rate.
    size_t sharing = 0;
    for (Job* j : act) sharing += j->jit ? 0 : 1;
    for (Job* j : act) {
        if (j->jit || j->compile_queued) continue;
        if (auto k = jit_ready(*j->c, specialized_waves_per_eu())) {
            j->jit = k;
            continue;
        }
        // The runtime model's rule: remaining interpreter time at this job's share against the
        // predicted compile time.  The LUT count is exact once the LUT program exists; it is
        // only built here (host time) when the remaining time could pay for a compile at all.
        TierJob tj;
        tj.interp_gates = j->c->interp_gates();
        tj.rows = j->c->interp_rows();
        tj.remaining_patterns = 32.0 * (double)(j->range.end - j->cursor);
        tj.lut_steps = 0;
        double remaining_ms = 0;
        server_wants_compile(tj, sharing, &remaining_ms, nullptr);
        bool want = false;
        if (remaining_ms > server_compile_threshold_ms()) {
            tj.lut_steps = j->c->lut_steps_known();
            want = server_wants_compile(tj, sharing, nullptr, nullptr);
        }
        if (jit_mode == 2 || want) {
            j->compile_queued = true;
            compile_queue.push_back(j);
            cv_compile.notify_one();
        }
    }
}

void fastlec_es_server::finish(Job* j, double now) {
    j->done = true;
    j->res.plan_ms = j->c->plan_ms;
    j->res.kernel_ms = j->kernel_ms;
    j->res.queued_ms = j->t_admit - j->t_submit;
    j->res.latency_ms = now - j->t_submit;
    st.completed++;
    st.charge_in_use_bytes -= j->charge;
    free_slots.push_back(j->slot);
}

void fastlec_es_server::step(const std::vector<Job*>& act) {
    const int kK = server_k(), kB = server_bundle();
    // Slices: equal gate-evaluation budget per job, at least 16 passes.
    const uint32_t pass_hw = 64u * kK;
    // Tier of every job for this step (a compile thread may set a kernel meanwhile).
    std::vector<std::shared_ptr<JitKernel>> jk(act.size());
    {
        std::lock_guard<std::mutex> g(mu);
        for (size_t t = 0; t < act.size(); ++t) jk[t] = act[t]->jit;
    }
    const double target_np = rate * step_ms_target / 1e3;
    size_t n_interp = 0;
    for (auto& k : jk) n_interp += k ? 0 : 1;
    const double per_job = target_np / (double)std::max<size_t>(1, n_interp);
    std::vector<Circuit*> lds_c, hbm_c;
    std::vector<HwRange> lds_r, hbm_r;
    std::vector<uint32_t> lds_i, hbm_i;
    const size_t lds_blk = dev->prop.sharedMemPerBlock ? dev->prop.sharedMemPerBlock : 65536;
    double step_np = 0;
    std::vector<HwRange> windows(act.size());
    std::vector<size_t> jit_jobs;
    for (size_t t = 0; t < act.size(); ++t) {
        Job* j = act[t];
        if (jk[t]) {  // specialized slice: about one step's worth at the kernel's rate
            const double per_hw = 32.0 * std::max<uint32_t>(1, j->c->plan1.num_gate_instrs);
            const uint64_t step_hw = 64;  // one pass of the specialized kernel
            uint64_t slice = (uint64_t)std::max(64.0 * (double)step_hw, std::floor(jit_rate * step_ms_target / 1e3 / per_hw));
            slice = (slice + step_hw - 1) / step_hw * step_hw;
            windows[t] = HwRange{j->cursor, std::min(j->range.end, j->cursor + slice)};
            jit_jobs.push_back(t);
            continue;
        }
        const Plan& p = j->c->plan_for(kB);
        const double per_hw = 32.0 * std::max<size_t>(1, p.prog.size());
        uint64_t slice = (uint64_t)std::max(16.0 * pass_hw, std::floor(per_job / per_hw));
        slice = (slice + pass_hw - 1) / pass_hw * pass_hw;
        HwRange w{j->cursor, std::min(j->range.end, j->cursor + slice)};
        windows[t] = w;
        step_np += per_hw * (double)(w.end - w.begin);
        // The first group runs in the register tier (or LDS when the caller fixes the schedule);
        // files too large for registers go to device memory, where more waves per CU fit.
        int regs_waves = 0;
        const bool fits = regs_tier_enabled() && !opts.wg_size && !opts.words_per_thread
                              ? interp_regs_rows(j->c->interp_rows(), &regs_waves) != 0
                              : interp_lds_bytes(p.rows, kK, 1) <= lds_blk;
        (fits ? lds_c : hbm_c).push_back(j->c);
        (fits ? lds_r : hbm_r).push_back(w);
        (fits ? lds_i : hbm_i).push_back(j->slot);
    }
    uint8_t* host = (uint8_t*)table.host;
    uint8_t* devp = (uint8_t*)table.dev;
    std::memset(host, 0, 2 * sizeof(LaunchCtl));
    struct Group {
        std::vector<Circuit*>* c;
        std::vector<HwRange>* r;
        std::vector<uint32_t>* i;
        size_t ctl_off, desc_off;
        bool lds;
        Schedule sch;
        uint64_t items = 0;
    };
    Group groups[2] = {{&lds_c, &lds_r, &lds_i, 0, off_desc_lds, true, {}}, {&hbm_c, &hbm_r, &hbm_i, sizeof(LaunchCtl), off_desc_hbm, false, {}}};
    for (Group& g : groups) {
        if (g.c->empty()) continue;
        fastlec_es_options o = opts;
        o.kernel = g.lds ? FASTLEC_KERNEL_INTERP : FASTLEC_KERNEL_INTERP_HBM;
        o.words_per_thread = kK;
        bool have = false;
        // Value files in VGPRs when every job of the group fits (bundles of 4).
        if (g.lds && !opts.wg_size && !opts.words_per_thread && make_schedule_regs(*dev, rows_for(*g.c, 4), g.sch))
            have = true;
        if (!have && g.lds && server_occupancy() && !opts.wg_size) {
            int best = -1;
            for (int block : {256, 128, 64}) {
                Schedule t;
                if (!make_schedule(*dev, *g.c, kK, kB, block, true, t)) continue;
                const int waves = t.grid / std::max(1, dev->prop.multiProcessorCount) * (block / 64);
                if (!have || waves > best) {
                    have = true;
                    best = waves;
                    g.sch = t;
                }
            }
        }
        if (!have) g.sch = shrink_schedule(*dev, *g.c, &o, kB);
        const bool files_needed = !g.sch.lds && !g.sch.regs;  // the register and LDS tiers hold their own
        if (files_needed) {
            // Value files in device memory: the grid is capped so that the server's device
            // memory (job table plus files) stays within the budget.
            const size_t per_block = (size_t)(g.sch.block / 64) * rows_for(*g.c, kB) * 64ull * g.sch.K * 4ull;
            const size_t room = budget > table.bytes + 4096 ? budget - table.bytes - 4096 : 0;  // 4 KiB rounding
            const size_t fit = room / per_block;
            if (fit < 1)
                throw Error{kErrNoMem, "the budget cannot hold one workgroup's value files in device memory"};
            g.sch.grid = (int)std::min<size_t>((size_t)g.sch.grid, fit);
        }
        g.items = build_descs(*dev, *g.c, *g.r, *g.i, g.sch, stream, (ConeDesc*)(host + g.desc_off));
        if (files_needed) {
            const size_t need = (size_t)g.sch.grid * (g.sch.block / 64) * rows_for(*g.c, kB) * 64ull * g.sch.K * 4ull;
            if (files.bytes < need) {  // device-only, exactly sized (not pooled), within the budget
                // files is read by stats callers under mu: swap it under the lock, allocate outside
                void* old = nullptr;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    old = files.dev;
                    files = Buffer{};
                }
                if (old) (void)hipFree(old);
                const size_t bytes = (need + 4095) & ~size_t(4095);
                void* fresh = nullptr;
                if (hipMalloc(&fresh, bytes) != hipSuccess)
                    throw Error{kErrNoMem, "device allocation of the server's value files failed"};
                std::lock_guard<std::mutex> lk(mu);
                files.dev = fresh;
                files.bytes = bytes;
            }
        }
    }
    // Upload the control words and this step's descriptors (best[] stays on the device).
    FES_HIP(hipMemcpyAsync(devp, host, 2 * sizeof(LaunchCtl), hipMemcpyHostToDevice, stream));
    for (Group& g : groups)
        if (!g.c->empty())
            FES_HIP(hipMemcpyAsync(devp + g.desc_off, host + g.desc_off, sizeof(ConeDesc) * g.c->size(),
                                   hipMemcpyHostToDevice, stream));
    ScopedEvent e0, e1, e2;
    FES_HIP(hipEventRecord(e0.e, stream));
    for (Group& g : groups) {
        if (g.c->empty()) continue;
        InterpLaunch L;
        L.cones = (const ConeDesc*)(devp + g.desc_off);
        L.num_cones = (uint32_t)g.c->size();
        L.rows_max = rows_for(*g.c, g.sch.B);
        L.total_items = g.items;
        L.ctl = (LaunchCtl*)(devp + g.ctl_off);
        L.best = (unsigned long long*)(devp + off_best);
        L.hbm_rows = (g.sch.lds || g.sch.regs) ? nullptr : (uint32_t*)files.dev;
        L.cancel = nullptr;
        FES_HIP(launch_schedule(L, g.sch, stream));
    }
    FES_HIP(hipEventRecord(e1.e, stream));
    // Specialized slices: own claim counter per slot (zeroed first), shared best[] entry.
    double jit_np = 0;
    if (!jit_jobs.empty()) {
        for (size_t t : jit_jobs) {
            Job* j = act[t];
            const size_t off = off_ctl_jit + kClaimBytes * j->slot;
            std::memset(host + off, 0, kClaimBytes);
            FES_HIP(hipMemcpyAsync(devp + off, host + off, kClaimBytes, hipMemcpyHostToDevice, stream));
            const JitLaunchPlan lp = jit_prepare(*dev, *jk[t], windows[t], 0);
            jit_enqueue(lp, (uint64_t*)(devp + off), (uint64_t*)(devp + off_best + 8ull * j->slot), nullptr, stream);
            jit_np += 32.0 * std::max<uint32_t>(1, j->c->plan1.num_gate_instrs) * (double)(windows[t].end - windows[t].begin);
        }
        FES_HIP(hipEventRecord(e2.e, stream));
    }
    FES_HIP(hipMemcpyAsync(host + off_best, devp + off_best, 8ull * kCapacity, hipMemcpyDeviceToHost, stream));
    FES_HIP(hipStreamSynchronize(stream));
    float ms = 0, jit_ms = 0;
    FES_HIP(hipEventElapsedTime(&ms, e0.e, e1.e));
    if (!jit_jobs.empty()) FES_HIP(hipEventElapsedTime(&jit_ms, e1.e, e2.e));
    if (n_interp && ms > 0.5f) rate = 0.7 * rate + 0.3 * (step_np / (ms / 1e3));
    if (jit_np > 0 && jit_ms > 0.5f) jit_rate = 0.7 * jit_rate + 0.3 * (jit_np / (jit_ms / 1e3));

    const uint64_t* best = (const uint64_t*)(host + off_best);
    const double now = now_ms();
    std::lock_guard<std::mutex> g(mu);
    st.steps++;
    st.busy_ms += ms + jit_ms;
    st.specialized_slices += jit_jobs.size();
    for (size_t t = 0; t < act.size(); ++t) {
        Job* j = act[t];
        j->kernel_ms += jk[t] ? jit_ms / (double)jit_jobs.size() : ms;
        const uint64_t b = best[j->slot];
        const uint32_t n = j->c->plan1.num_inputs;
        if (b != ~0ull) {
            j->res.verdict = FASTLEC_NONEQUIVALENT;
            j->res.cex = b;
            j->res.patterns_evaluated = b + 1;
            j->res.next_word = b / 64;
        } else {
            j->cursor = windows[t].end;
            if (j->cursor < j->range.end) continue;
            j->res.verdict = FASTLEC_EQUIVALENT;
            j->res.patterns_evaluated = n < 5 ? (1ull << n) : 32ull * (j->range.end - j->range.begin);
            j->res.next_word = n >= 6 ? (1ull << (n - 6)) : 1ull;
        }
        finish(j, now);
    }
    active.erase(std::remove_if(active.begin(), active.end(), [](Job* j) { return j->done; }), active.end());
    st.active = active.size();
    cv_done.notify_all();
}

void fastlec_es_server::loop() {
    try {
        FES_HIP(hipSetDevice(dev->ordinal));
        for (;;) {
            std::vector<Job*> act;
            std::vector<uint32_t> fresh;
            {
                std::unique_lock<std::mutex> g(mu);
                // Admission: first fit in arrival order, unless the oldest job has waited
                // more than two seconds, in which case nothing may pass it.
                const double now = now_ms();
                bool head_only = !queue.empty() && now - queue.front()->t_submit > 2000.0;
                for (auto it = queue.begin(); it != queue.end();) {
                    Job* j = *it;
                    if (st.charge_in_use_bytes + j->charge <= budget && !free_slots.empty()) {
                        j->slot = free_slots.back();
                        free_slots.pop_back();
                        j->t_admit = now;
                        // The model's ETA: the job's interpreter time alone, times the jobs that
                        // share the device with it at admission (itself included).
                        j->res.predicted_ms = model_interp_ms(j->c->interp_gates(), j->c->interp_rows(),
                                                              32.0 * (double)(j->range.end - j->range.begin)) *
                                              (double)(active.size() + 1);
                        st.charge_in_use_bytes += j->charge;
                        st.peak_charge_bytes = std::max(st.peak_charge_bytes, st.charge_in_use_bytes);
                        active.push_back(j);
                        fresh.push_back(j->slot);
                        it = queue.erase(it);
                    } else if (head_only) {
                        break;
                    } else {
                        ++it;
                    }
                }
                st.queued = queue.size();
                st.active = active.size();
                st.max_active = std::max<uint64_t>(st.max_active, active.size());
                if (active.empty()) {
                    if (stop) return;
                    cv_work.wait(g, [&] { return stop || !queue.empty(); });
                    if (stop && queue.empty()) return;
                    continue;
                }
                if (stop) return;
                act = active;
            }
            // Reset the best value of newly assigned slots on the device.
            uint64_t* hb = (uint64_t*)((uint8_t*)table.host + off_best);
            for (uint32_t s : fresh) {
                hb[s] = ~0ull;
                FES_HIP(hipMemcpyAsync((uint8_t*)table.dev + off_best + 8ull * s, &hb[s], 8, hipMemcpyHostToDevice, stream));
            }
            plan_tiers(act);
            step(act);
        }
    } catch (const Error& e) {
        std::lock_guard<std::mutex> g(mu);
        fatal = e.msg;
        fatal_code = e.code;
    } catch (const std::exception& e) {
        std::lock_guard<std::mutex> g(mu);
        fatal = e.what();
        fatal_code = FASTLEC_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> g(mu);
    const double now = now_ms();
    for (Job* j : active) {
        j->status = fatal_code;
        j->res.verdict = fatal_code;
        finish(j, now);
    }
    active.clear();
    for (Job* j : queue) {
        j->done = true;
        j->status = fatal_code;
        j->res.verdict = fatal_code;
    }
    queue.clear();
    cv_done.notify_all();
}

namespace {
thread_local std::string g_err;
}

extern "C" {

int fastlec_es_server_create(const fastlec_es_options* opts, size_t budget_bytes, fastlec_es_server** out) {
    if (!out || budget_bytes == 0) return FASTLEC_ERR_INVALID;
    *out = nullptr;
    try {
        auto s = std::make_unique<fastlec_es_server>();
        if (opts) s->opts = *opts;
        s->budget = budget_bytes;
        s->chunk_words = std::max<uint64_t>(1, env_u64("FASTLEC_ES_SERVER_CHUNK_WORDS", 1ull << 22));
        s->step_ms_target = (double)std::max<uint64_t>(1, env_u64("FASTLEC_ES_SERVER_STEP_MS", 10));
        // initial interpreter rate estimate (node*patterns/s) from which the first slices are sized
        if (const uint64_t r0 = env_u64("FASTLEC_ES_SERVER_RATE", 0)) s->rate = (double)r0;
        s->dev = &device(s->opts.device);
        s->stream = s->opts.hip_stream ? (hipStream_t)s->opts.hip_stream : s->dev->stream;
        s->jit_mode = (int)std::min<uint64_t>(2, env_u64("FASTLEC_ES_SERVER_JIT", 1));
        s->off_desc_lds = (s->off_best + 8ull * kCapacity + 255) & ~size_t(255);
        s->off_desc_hbm = s->off_desc_lds + sizeof(ConeDesc) * kCapacity;
        s->off_ctl_jit = (s->off_desc_hbm + sizeof(ConeDesc) * kCapacity + 255) & ~size_t(255);
        s->table = s->dev->acquire(s->off_ctl_jit + kClaimBytes * kCapacity);
        if (s->table.bytes >= budget_bytes) {
            s->dev->release(s->table);
            return FASTLEC_ERR_INVALID;  // the budget must exceed the job table
        }
        for (uint32_t i = kCapacity; i-- > 0;) s->free_slots.push_back(i);
        s->st.budget_bytes = budget_bytes;
        fastlec_es_server* raw = s.get();
        s->th = std::thread([raw] { raw->loop(); });
        for (int t = 0, n = std::max(1, compile_helpers()); t < n; ++t)
            s->compilers.emplace_back([raw] { raw->compile_loop(); });
        *out = s.release();
        return FASTLEC_OK;
    } catch (const Error& e) {
        return e.code;
    } catch (...) {
        return FASTLEC_ERR_DEVICE;
    }
}

int fastlec_es_server_submit(fastlec_es_server* s, const fastlec_es_circuit* c, uint64_t* ticket) {
    if (!s || !c || !ticket) return FASTLEC_ERR_INVALID;
    if (c->c.plan1.num_inputs > 63) return FASTLEC_ERR_UNSUPPORTED;
    auto j = std::make_unique<Job>();
    j->c = const_cast<Circuit*>(&c->c);
    j->charge = s->charge_of(j->c[0]);
    std::lock_guard<std::mutex> g(s->mu);
    if (s->fatal_code) return s->fatal_code;
    if (j->charge > s->budget) {
        s->st.rejected++;
        return FASTLEC_REJECTED;
    }
    j->range = range_of(j->c->plan1.num_inputs, 0, 0);
    j->cursor = j->range.begin;
    j->ticket = s->next_ticket++;
    j->t_submit = now_ms();
    *ticket = j->ticket;
    s->queue.push_back(j.get());
    s->jobs[j->ticket] = std::move(j);
    s->st.submitted++;
    s->st.queued = s->queue.size();
    s->cv_work.notify_one();
    return FASTLEC_OK;
}

int fastlec_es_server_poll(fastlec_es_server* s, uint64_t ticket, fastlec_es_result* out, int wait) {
    if (!s || !out) return FASTLEC_ERR_INVALID;
    std::unique_lock<std::mutex> g(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return FASTLEC_ERR_INVALID;
    Job* j = it->second.get();
    if (!j->done || j->compiling) {  // a compile in progress still reads the circuit
        if (!wait) return 0;
        s->cv_done.wait(g, [&] { return j->done && !j->compiling; });
    }
    *out = j->res;
    const int status = j->status;
    s->compile_queue.erase(std::remove(s->compile_queue.begin(), s->compile_queue.end(), j), s->compile_queue.end());
    s->jobs.erase(it);
    return status ? status : 1;
}

int fastlec_es_server_stats_get(fastlec_es_server* s, fastlec_es_server_stats* st) {
    if (!s || !st) return FASTLEC_ERR_INVALID;
    std::lock_guard<std::mutex> g(s->mu);
    *st = s->st;
    st->device_bytes = s->table.bytes + s->files.bytes;
    return FASTLEC_OK;
}

void fastlec_es_server_destroy(fastlec_es_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->cv_compile.notify_all();
    if (s->th.joinable()) s->th.join();
    for (auto& t : s->compilers)
        if (t.joinable()) t.join();
    if (s->table.dev) s->dev->release(s->table);
    if (s->files.dev) (void)hipFree(s->files.dev);
    delete s;
}

}  // extern "C"
