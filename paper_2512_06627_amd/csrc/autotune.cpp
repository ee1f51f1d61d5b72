// Interpreter schedule autotuner and hipGraph-captured batch launches.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "runtime.hpp"

namespace fes {
namespace {

struct TuneKey {
    int device;
    uint32_t rows_log2, cones_log2, work_log2;
    bool hbm;
    bool operator<(const TuneKey& o) const {
        return std::tie(device, rows_log2, cones_log2, work_log2, hbm) <
               std::tie(o.device, o.rows_log2, o.cones_log2, o.work_log2, o.hbm);
    }
};

uint32_t log2_bucket(double x) {
    uint32_t b = 0;
    while (x >= 2.0) {
        x /= 2.0;
        ++b;
    }
    return b;
}

std::mutex g_tune_mu;
std::map<TuneKey, Schedule>& tune_cache() {
    static std::map<TuneKey, Schedule> m;
    return m;
}

}  // namespace

Schedule autotune(Device& dev, const std::vector<Circuit*>& cs, const std::vector<HwRange>& ranges, hipStream_t stream,
                  bool hbm) {
    double work = 0;
    for (size_t i = 0; i < cs.size(); ++i)
        work += (double)cs[i]->plan1.num_gate_instrs * 32.0 * (double)(ranges[i].end - ranges[i].begin);
    TuneKey key{dev.ordinal, log2_bucket(rows_for(cs, 8)), log2_bucket((double)cs.size()), log2_bucket(work), hbm};
    {
        // A cached choice is re-fitted to this batch: the key buckets the value-file rows, and
        // within a bucket a larger cone may no longer fit the chosen workgroup in LDS.
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = tune_cache().find(key);
        if (it != tune_cache().end()) {
            Schedule s;
            if (it->second.regs ? make_schedule_regs(dev, rows_for(cs, 4), s)
                                : make_schedule(dev, cs, it->second.K, it->second.B, it->second.block, it->second.lds, s))
                return s;
            trace("autotune: cached K=%d B=%d block=%d does not fit this batch; re-tuning", it->second.K,
                  it->second.B, it->second.block);
        }
    }
    // Bounded sample: a prefix of every cone, about 2e11 gate evaluations in total.
    const double budget = 2e11;
    std::vector<HwRange> sample(ranges.size());
    double sample_work = 0;
    for (size_t i = 0; i < cs.size(); ++i) {
        const double per_hw = 32.0 * std::max<uint32_t>(1, cs[i]->plan1.num_gate_instrs);
        uint64_t hw = (uint64_t)std::max(512.0, budget / (double)cs.size() / per_hw);
        hw = std::min<uint64_t>(hw, ranges[i].end - ranges[i].begin);
        sample[i] = HwRange{ranges[i].begin, ranges[i].begin + hw};
        sample_work += per_hw * (double)hw;
    }
    std::vector<Schedule> cands;
    bool regs_fit = false;
    {
        Schedule rs;
        if (!hbm && make_schedule_regs(dev, rows_for(cs, 4), rs)) {
            cands.push_back(rs);
            regs_fit = true;
        }
    }
    for (int K : {1, 2, 4})
        for (int B : {4, 8, 16})
            for (int block : {64, 128, 256}) {
                if (B == 16 && K > 2) continue;  // 16 bundles of 4 words per lane spill registers
                Schedule s;
                if (make_schedule(dev, cs, K, B, block, !hbm, s)) cands.push_back(s);
            }
    // Files too large for the register tier: device-memory files with one or two words per lane
    // compete with the LDS candidates (LDS then holds at most two waves per CU).
    if (!hbm && !regs_fit)
        for (int K : {1, 2})
            for (int B : {8, 16})
                for (int block : {64, 128}) {
                    Schedule s;
                    if (make_schedule(dev, cs, K, B, block, false, s)) cands.push_back(s);
                }
    if (cands.empty()) {
        fastlec_es_options o{};
        o.kernel = hbm ? FASTLEC_KERNEL_INTERP_HBM : FASTLEC_KERNEL_INTERP;
        cands.push_back(default_schedule(dev, cs, &o));
    }
    Schedule best = cands[0];
    double best_rate = -1;
    std::vector<uint64_t> b;
    double ms = 0;
    // FASTLEC_ES_TUNE_FORCE="K,B,block" takes that candidate, when it fits, without timing
    // (a test hook for schedule-dependent paths).
    if (const char* f = std::getenv("FASTLEC_ES_TUNE_FORCE")) {
        int fk = 0, fb = 0, fw = 0;
        if (std::sscanf(f, "%d,%d,%d", &fk, &fb, &fw) == 3)
            for (const Schedule& s : cands)
                if (s.K == fk && s.B == fb && s.block == fw) {
                    std::lock_guard<std::mutex> g(g_tune_mu);
                    tune_cache()[key] = s;
                    return s;
                }
    }
    run_interp(dev, cs, sample, cands[0], stream, nullptr, b, &ms);  // uploads programs, warms caches
    for (const Schedule& s : cands) {
        run_interp(dev, cs, sample, s, stream, nullptr, b, &ms);
        const double rate = sample_work / std::max(1e-3, (double)ms);
        trace("autotune: K=%d B=%d block=%d grid=%d %s -> %.3f ms", s.K, s.B, s.block, s.grid,
              s.regs ? "regs" : s.lds ? "lds" : "hbm", ms);
        if (rate > best_rate) {
            best_rate = rate;
            best = s;
        }
    }
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_cache()[key] = best;
    return best;
}

namespace {

struct BatchGraph {
    std::vector<uint64_t> uids;
    Schedule sch;
    Buffer buf;
    size_t best_off = 0, total = 0;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    uint64_t last_use = 0;
};

std::map<int, bool> g_no_capture;  // devices on which recording a graph failed once

std::mutex g_graph_mu;
std::vector<std::unique_ptr<BatchGraph>>& graphs(int device) {
    static std::map<int, std::vector<std::unique_ptr<BatchGraph>>> m;
    return m[device];
}
uint64_t g_use_clock = 0;

}  // namespace

void run_batch_graph(Device& dev, const std::vector<Circuit*>& cs, const std::vector<HwRange>& ranges,
                     const Schedule& sch, hipStream_t stream, std::vector<uint64_t>& best, double* ms) {
    std::vector<uint64_t> uids;
    for (Circuit* c : cs) uids.push_back(c->uid);
    std::unique_lock<std::mutex> g(g_graph_mu);
    if (g_no_capture[dev.ordinal]) {
        g.unlock();
        run_interp(dev, cs, ranges, sch, stream, nullptr, best, ms);
        return;
    }
    auto& list = graphs(dev.ordinal);
    BatchGraph* bg = nullptr;
    for (auto& x : list)
        if (x->uids == uids && x->sch.K == sch.K && x->sch.B == sch.B && x->sch.block == sch.block &&
            x->sch.grid == sch.grid && x->sch.lds == sch.lds && x->sch.tile_hw == sch.tile_hw && x->sch.regs == sch.regs)
            bg = x.get();
    if (!bg) {
        if (list.size() >= 16) {  // evict the least recently used graph (a batch may hold several groups)
            auto it = std::min_element(list.begin(), list.end(),
                                       [](const auto& a, const auto& b) { return a->last_use < b->last_use; });
            BatchGraph* old = it->get();
            (void)hipGraphExecDestroy(old->exec);
            (void)hipGraphDestroy(old->graph);
            dev.release(old->buf);
            list.erase(it);
        }
        auto nb = std::make_unique<BatchGraph>();
        nb->uids = uids;
        nb->sch = sch;
        const size_t k = cs.size();
        const uint32_t rows_max = rows_for(cs, sch.B);
        const size_t waves = (size_t)sch.grid * (sch.block / 64);
        const size_t desc_off = (sizeof(LaunchCtl) + 8 * k + 63) & ~size_t(63);
        const size_t files_off = (desc_off + sizeof(ConeDesc) * k + 255) & ~size_t(255);
        const size_t file_bytes = (sch.lds || sch.regs) ? 0 : waves * rows_max * 64ull * sch.K * 4ull;
        nb->best_off = sizeof(LaunchCtl);
        nb->total = files_off + file_bytes;
        nb->buf = dev.acquire(nb->total, files_off);
        uint8_t* host = (uint8_t*)nb->buf.host;
        uint8_t* devp = (uint8_t*)nb->buf.dev;
        std::memset(host, 0, files_off);
        for (size_t i = 0; i < k; ++i) ((uint64_t*)(host + nb->best_off))[i] = ~0ull;
        std::vector<uint32_t> idx(k);
        std::iota(idx.begin(), idx.end(), 0u);
        const uint64_t items = build_descs(dev, cs, ranges, idx, sch, stream, (ConeDesc*)(host + desc_off));
        InterpLaunch L;
        L.cones = (const ConeDesc*)(devp + desc_off);
        L.num_cones = (uint32_t)k;
        L.rows_max = rows_max;
        L.total_items = items;
        L.ctl = (LaunchCtl*)devp;
        L.best = (unsigned long long*)(devp + nb->best_off);
        L.hbm_rows = (sch.lds || sch.regs) ? nullptr : (uint32_t*)(devp + files_off);
        L.cancel = nullptr;
        // Recorded on a stream used for nothing else (a null caller stream cannot be
        // captured); the graph is launched on the caller's stream.  The host staging area
        // (control block, best[], descriptors) stays intact for the graph's upload node.
        // Any failure ends the capture and switches this device to eager launches.
        (void)hipGetLastError();
        hipError_t e = hipStreamBeginCapture(dev.capture_stream, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) e = hipMemcpyAsync(devp, host, files_off, hipMemcpyHostToDevice, dev.capture_stream);
        if (e == hipSuccess) e = launch_schedule(L, sch, dev.capture_stream);
        hipGraph_t graph = nullptr;
        hipError_t e_end = hipStreamEndCapture(dev.capture_stream, &graph);
        if (e == hipSuccess) e = e_end;
        if (e == hipSuccess) e = hipGraphInstantiate(&nb->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            trace("graph capture failed (%s): eager launches from now on", hipGetErrorString(e));
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            dev.release(nb->buf);
            g_no_capture[dev.ordinal] = true;
            g.unlock();
            run_interp(dev, cs, ranges, sch, stream, nullptr, best, ms);
            return;
        }
        nb->graph = graph;
        bg = nb.get();
        list.push_back(std::move(nb));
    }
    bg->last_use = ++g_use_clock;
    const size_t k = cs.size();
    // Results are read back outside the graph into a small pooled buffer, so the graph's
    // upload source (the staging area) is never overwritten.
    Buffer res = dev.acquire(8 * k);
    struct Releaser {
        Device& d;
        Buffer b;
        ~Releaser() { d.release(b); }
    } rel{dev, res};
    ScopedEvent e0, e1;
    FES_HIP(hipEventRecord(e0.e, stream));
    FES_HIP(hipGraphLaunch(bg->exec, stream));
    FES_HIP(hipEventRecord(e1.e, stream));
    FES_HIP(hipMemcpyAsync(res.host, (uint8_t*)bg->buf.dev + bg->best_off, 8 * k, hipMemcpyDeviceToHost, stream));
    FES_HIP(hipStreamSynchronize(stream));
    float t = 0;
    if (hipEventElapsedTime(&t, e0.e, e1.e) != hipSuccess) t = 0;
    if (ms) *ms = t;
    best.assign((uint64_t*)res.host, (uint64_t*)res.host + k);
}

}  // namespace fes
