// C ABI of the exact-simulation library.  No exception crosses this boundary:
// every entry point catches, stores a thread-local message and returns a status.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <fstream>
#include <map>
#include <sstream>
#include <thread>
#include <unordered_map>

#include "runtime.hpp"

using namespace fes;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

template <class F>
int guarded(F&& f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const Error& e) {
        return fail(e.code, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(FASTLEC_ERR_NOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(FASTLEC_ERR_DEVICE, e.what());
    } catch (...) {
        return fail(FASTLEC_ERR_DEVICE, "unknown error");
    }
}

fastlec_es_options defaults() {
    fastlec_es_options o;
    std::memset(&o, 0, sizeof(o));
    return o;
}

uint64_t range_patterns(uint32_t n, const HwRange& r) {
    if (n < 5) return 1ull << n;  // one half-word holds the whole space
    return 32ull * (r.end - r.begin);
}

void fill_result(const Circuit& c, const HwRange& r, uint64_t best, fastlec_es_result* out) {
    const uint32_t n = c.plan1.num_inputs;
    out->reserved = 0;
    out->plan_ms = c.plan_ms;
    const uint64_t begin_p = n < 5 ? 0 : 32ull * r.begin;
    const uint64_t words = n >= 6 ? (1ull << (n - 6)) : 1ull;
    if (best == ~0ull) {
        out->verdict = FASTLEC_EQUIVALENT;
        out->cex = 0;
        out->patterns_evaluated = range_patterns(n, r);
        out->next_word = std::min(words, (r.end + 1) / 2);
    } else {
        out->verdict = FASTLEC_NONEQUIVALENT;
        out->cex = best;
        out->patterns_evaluated = best - begin_p + 1;
        out->next_word = best / 64;
    }
}

// Choose the kernel by the runtime model: a compiled specialized kernel when it is predicted
// faster; otherwise the specialized kernel only when its time plus the hipRTC compile, with a
// safety margin of 1.2 on the compile, beats the interpreter.  The paper guards its engine
// rules against prediction error with margins tuned within [0.5, 2] (Section 3.2); the
// compile model's largest error here is 4%.  The LUT program (needed for the specialized
// prediction) is only built when the interpreter's time could pay for a compile.
constexpr double kCompileMargin = 1.2;

// Specialized kernels in batches under AUTO (FASTLEC_ES_BATCH_JIT): 0 never, 1 by the runtime
// model (default), 2 every cone whose kernel already exists (a test hook).
int batch_jit_mode() {
    static const int m = [] {
        const char* e = std::getenv("FASTLEC_ES_BATCH_JIT");
        const int x = e && *e ? std::atoi(e) : 1;
        return x < 0 || x > 2 ? 1 : x;
    }();
    return m;
}

bool use_specialized(Circuit& c, const fastlec_es_options& o, const HwRange& r) {
    if (o.kernel == FASTLEC_KERNEL_SPECIALIZED) return true;
    if (o.kernel != FASTLEC_KERNEL_AUTO) return false;
    const double patterns = 32.0 * (double)(r.end - r.begin);
    const double t_interp = model_interp_ms(c.interp_gates(), c.interp_rows(), patterns);
    if (jit_ready(c, specialized_waves_per_eu()))
        return model_specialized_ms(c.lut_program().lut_steps, patterns) < t_interp;
    if (t_interp < kCompileMargin * model_compile_ms(0)) return false;
    const uint32_t luts = c.lut_program().lut_steps;
    return model_specialized_ms(luts, patterns) + kCompileMargin * model_compile_ms(luts) < t_interp;
}

void check_one(Circuit& c, const fastlec_es_options& o, fastlec_es_result* out) {
    if (o.kernel < FASTLEC_KERNEL_AUTO || o.kernel > FASTLEC_KERNEL_INTERP_HBM)
        throw Error{kErrInvalid, "unknown kernel"};
    Device& dev = device(o.device);
    hipStream_t stream = o.hip_stream ? (hipStream_t)o.hip_stream : dev.stream;
    HwRange full = range_of(c.plan1.num_inputs, o.begin_word, o.end_word);
    std::memset(out, 0, sizeof(*out));
    const bool spec = use_specialized(c, o, full);
    std::shared_ptr<JitKernel> jk;
    double compile_ms = 0;
    if (spec) jk = jit_kernel(c, specialized_waves_per_eu(), &compile_ms);
    Schedule sch;
    if (!spec) {
        std::vector<Circuit*> one{&c};
        sch = default_schedule(dev, one, &o, full.end - full.begin);
        if (o.tile_words) sch.tile_hw = 2ull * o.tile_words;
    }
    // Without a deadline or cancel flag the whole range is one launch.  With one, the range
    // runs as ascending chunks with the host checking between chunks.
    const bool chunked = o.deadline_s > 0 || o.cancel_flag;
    const double t_start = now_ms();
    uint64_t chunk = full.end - full.begin;
    if (chunked) chunk = std::max<uint64_t>(4096, (full.end - full.begin) / 256);
    double kernel_ms = 0;
    uint64_t best = ~0ull;
    uint64_t done_to = full.begin;
    int status = FASTLEC_OK;
    for (uint64_t lo = full.begin; lo < full.end && best == ~0ull; lo += chunk) {
        if (chunked) {
            if (o.cancel_flag && *o.cancel_flag) { status = FASTLEC_CANCELLED; break; }
            if (o.deadline_s > 0 && now_ms() - t_start >= o.deadline_s * 1e3) { status = FASTLEC_TIMEOUT; break; }
        }
        HwRange r{lo, std::min(full.end, lo + chunk)};
        double ms = 0;
        const DevMem mem{o.dev_scratch, o.dev_scratch ? o.dev_scratch_bytes : 0};
        if (spec) {
            run_jit(dev, c, *jk, r, o.tile_words ? 2ull * o.tile_words : 0, stream, nullptr, &best, &ms, mem);
        } else {
            std::vector<Circuit*> one{&c};
            std::vector<HwRange> rs{r};
            std::vector<uint64_t> b;
            run_interp(dev, one, rs, sch, stream, nullptr, b, &ms, mem);
            best = b[0];
        }
        kernel_ms += ms;
        done_to = r.end;
    }
    if (status != FASTLEC_OK) {
        out->verdict = status;
        out->patterns_evaluated = c.plan1.num_inputs < 5 ? 0 : 32ull * (done_to - full.begin);
        out->next_word = done_to / 2;
        out->plan_ms = c.plan_ms;
        out->kernel_ms = kernel_ms;
        out->compile_ms = compile_ms;
        throw Error{status, status == FASTLEC_CANCELLED ? "cancelled" : "deadline passed"};
    }
    fill_result(c, full, best, out);
    out->kernel_ms = kernel_ms;
    out->compile_ms = compile_ms;
    const double patterns = 32.0 * (double)(full.end - full.begin);
    out->predicted_ms = spec ? model_specialized_ms(c.lut_program().lut_steps, patterns)
                             : model_interp_ms(c.interp_gates(), c.interp_rows(), patterns);
}

}  // namespace

extern "C" {

void fastlec_es_options_init(fastlec_es_options* opts) {
    if (opts) *opts = defaults();
}

const char* fastlec_es_last_error(void) { return g_last_error.c_str(); }

int fastlec_es_load_aig(const void* bytes, size_t len, fastlec_es_circuit** out) {
    return guarded([&] {
        if (!out) throw Error{kErrInvalid, "null output handle"};
        *out = nullptr;
        static std::atomic<uint64_t> next_uid{1};
        auto h = std::make_unique<fastlec_es_circuit>();
        h->c.uid = next_uid++;
        h->c.aig = parse_aiger((const uint8_t*)bytes, len);
        const double t0 = now_ms();
        h->c.plan1 = make_plan(h->c.aig, Order::Auto, 1);
        h->c.fused = fuse_xors(h->c.aig);
        for (uint32_t k : h->c.plan1.order) h->c.fused_xors += h->c.fused.is_xor(k) ? 1u : 0u;
        h->c.plan_ms = now_ms() - t0;
        *out = h.release();
        return FASTLEC_OK;
    });
}

int fastlec_es_load_aig_file(const char* path, fastlec_es_circuit** out) {
    return guarded([&] {
        if (!path) throw Error{kErrInvalid, "null path"};
        std::ifstream f(path, std::ios::binary);
        if (!f) throw Error{kErrInvalid, std::string("cannot open ") + path};
        std::stringstream ss;
        ss << f.rdbuf();
        std::string s = ss.str();
        return fastlec_es_load_aig(s.data(), s.size(), out);
    });
}

int fastlec_es_info_get(const fastlec_es_circuit* c, fastlec_es_info* info) {
    return guarded([&] {
        if (!c || !info) throw Error{kErrInvalid, "null argument"};
        const Plan& p = c->c.plan1;
        info->num_pis = p.num_inputs;
        info->num_ands = p.num_ands_file;
        info->num_ands_tfi = p.num_ands_tfi;
        info->num_outputs = p.num_outputs;
        info->peak_live_slots = p.peak_slots;
        info->num_instrs = p.num_gate_instrs;
        info->levels = p.levels;
        info->num_xors = c->c.fused_xors;
        info->interp_rows = const_cast<Circuit&>(c->c).plan_for(4).rows;
        return FASTLEC_OK;
    });
}

int fastlec_es_check(const fastlec_es_circuit* c, const fastlec_es_options* opts, fastlec_es_result* out) {
    return guarded([&] {
        if (!c || !out) throw Error{kErrInvalid, "null argument"};
        fastlec_es_options o = opts ? *opts : defaults();
        check_one(const_cast<Circuit&>(c->c), o, out);
        return FASTLEC_OK;
    });
}

int fastlec_es_check_batch(const fastlec_es_circuit* const* cs, size_t k, const fastlec_es_options* opts,
                           fastlec_es_result* out) {
    if (cs && out) {
        // An entry's own error (a null handle) goes into that entry's verdict as a negative
        // status; the other entries are checked as one batch, and the call returns the first
        // entry's error once they are done.
        std::vector<size_t> valid;
        for (size_t i = 0; i < k; ++i)
            if (cs[i]) valid.push_back(i);
        if (valid.size() < k) {
            std::vector<const fastlec_es_circuit*> sub;
            for (size_t i : valid) sub.push_back(cs[i]);
            std::vector<fastlec_es_result> r(valid.size());
            if (!sub.empty()) {
                const int st = fastlec_es_check_batch(sub.data(), sub.size(), opts, r.data());
                if (st != FASTLEC_OK) return st;  // a failure of the whole call
            }
            for (size_t i = 0; i < k; ++i) {
                std::memset(&out[i], 0, sizeof(out[i]));
                out[i].verdict = FASTLEC_ERR_INVALID;
            }
            for (size_t t = 0; t < valid.size(); ++t) out[valid[t]] = r[t];
            size_t first = 0;
            while (cs[first]) ++first;
            return fail(FASTLEC_ERR_INVALID, "null circuit at batch entry " + std::to_string(first));
        }
    }
    return guarded([&] {
        if (!cs || !out) throw Error{kErrInvalid, "null argument"};
        if (k == 0) return FASTLEC_OK;
        fastlec_es_options o = opts ? *opts : defaults();
        Device& dev = device(o.device);
        hipStream_t stream = o.hip_stream ? (hipStream_t)o.hip_stream : dev.stream;
        std::vector<Circuit*> v;
        std::vector<HwRange> rs;
        for (size_t i = 0; i < k; ++i) {
            v.push_back(const_cast<Circuit*>(&cs[i]->c));
            rs.push_back(range_of(v.back()->plan1.num_inputs, 0, 0));
        }
        // Cones the runtime model gives to the specialized kernel (AUTO only) run as their own
        // launches; the rest share interpreter launches.  Their kernels compile together as
        // hipRTC programs side by side in helper processes, so a cone is a candidate when its
        // predicted saving beats its own part of the group's compile (kCompileMargin on its
        // per-kernel time over the helpers), and the candidates are taken when their summed
        // saving also covers the group's fixed cost (same margin).
        std::vector<size_t> spec;
        std::vector<uint8_t> is_spec(k, 0);
        if (o.kernel == FASTLEC_KERNEL_SPECIALIZED) {
            for (size_t i = 0; i < k; ++i) {
                is_spec[i] = 1;
                spec.push_back(i);
            }
        } else if (o.kernel == FASTLEC_KERNEL_AUTO && batch_jit_mode() == 2) {
            // Test hook: every cone whose kernel exists, whatever the model predicts.
            for (size_t i = 0; i < k; ++i)
                if (jit_ready(*v[i], specialized_waves_per_eu())) {
                    is_spec[i] = 1;
                    spec.push_back(i);
                }
            trace("batch: routing every cone whose kernel exists (%zu of %zu)", spec.size(), k);
        } else if (o.kernel == FASTLEC_KERNEL_AUTO && batch_jit_mode() == 1) {
            // First an optimistic bound (a LUT count below any cover measured) over the cones that
            // could pay for a compile share: when even that saving cannot pay for one program, only
            // cones whose kernels already exist are considered, and no LUT program is built.
            std::vector<size_t> cand;
            std::vector<double> tis;
            double optimistic = 0;
            const int helpers = compile_helpers();
            const double fixed_ms = model_group_compile_fixed_ms(helpers);
            for (size_t i = 0; i < k; ++i) {
                Circuit& c = *v[i];
                const double patterns = 32.0 * (double)(rs[i].end - rs[i].begin);
                const double ti = model_interp_ms(c.interp_gates(), c.interp_rows(), patterns);
                if (ti < kCompileMargin * model_group_compile_kernel_ms(0, helpers)) continue;  // cheap cone
                cand.push_back(i);
                tis.push_back(ti);
                const uint32_t lo = model_lut_steps_low(c.plan1.num_ands_tfi);
                const double ts = model_specialized_ms(lo, patterns);
                const double own = jit_ready(c, specialized_waves_per_eu()) ? 0.0
                                   : kCompileMargin * model_group_compile_kernel_ms(lo, helpers);
                if (ts + own < ti) optimistic += ti - ts - own;
            }
            const bool program_possible = optimistic >= kCompileMargin * fixed_ms;
            // The LUT programs the decision needs, mapped on host threads in parallel.
            std::vector<Circuit*> mapped;
            for (size_t i : cand)
                if (program_possible || jit_ready(*v[i], specialized_waves_per_eu())) mapped.push_back(v[i]);
            parallel_for(mapped.size(), [&](size_t t) { (void)mapped[t]->lut_program(); });
            double saving = 0;
            for (size_t ci = 0; ci < cand.size(); ++ci) {
                const size_t i = cand[ci];
                Circuit& c = *v[i];
                const double patterns = 32.0 * (double)(rs[i].end - rs[i].begin);
                const double ti = tis[ci];
                if (!program_possible && !jit_ready(c, specialized_waves_per_eu())) continue;
                const uint32_t luts = c.lut_program().lut_steps;
                const double ts = model_specialized_ms(luts, patterns);
                const double own = jit_ready(c, specialized_waves_per_eu()) ? 0.0
                                   : kCompileMargin * model_group_compile_kernel_ms(luts, helpers);
                if (ts + own < ti) {
                    is_spec[i] = 1;
                    spec.push_back(i);
                    saving += ti - ts - own;
                }
            }
            trace("batch: %zu candidate cones, %zu routed, predicted saving %.1f ms against a group compile "
                  "fixed cost of %.1f ms (%d helpers)",
                  cand.size(), spec.size(), saving, fixed_ms, helpers);
            if (saving < kCompileMargin * fixed_ms) {
                std::vector<size_t> kept;
                for (size_t i : spec) {  // not worth a program: only cones already compiled stay
                    if (jit_ready(*v[i], specialized_waves_per_eu())) kept.push_back(i);
                    else is_spec[i] = 0;
                }
                spec.swap(kept);
            }
        }
        // Compile the routed cones' kernels together, on a host thread while the interpreter
        // cones run on the device (compiles need no GPU).  Under AUTO a cone whose kernel does
        // not compile (the group is retried cone by cone first) runs on the interpreter
        // afterwards, as a launch of its own.  The thread only fills jk and cms; the guard
        // joins it on every path out of this call.
        std::vector<Circuit*> sc;
        for (size_t i : spec) sc.push_back(v[i]);
        std::vector<std::shared_ptr<JitKernel>> jk(spec.size());
        std::vector<double> cms(spec.size(), 0.0);
        std::exception_ptr compile_error;
        struct Joiner {
            std::thread t;
            ~Joiner() {
                if (t.joinable()) t.join();
            }
        } compile_job;
        const int spec_waves = specialized_waves_per_eu();
        const bool spec_forced = o.kernel == FASTLEC_KERNEL_SPECIALIZED;
        if (!sc.empty())
            compile_job.t = std::thread([&sc, &jk, &cms, &compile_error, spec_waves, spec_forced] {
                try {
                    try {
                        jk = jit_kernels(sc, spec_waves, &cms);
                    } catch (const Error& e) {
                        if (spec_forced) throw;
                        trace("batch: grouped compile failed (%s); compiling per cone", e.msg.c_str());
                        for (size_t j = 0; j < sc.size(); ++j) {
                            double ms = 0;
                            try {
                                jk[j] = jit_kernel(*sc[j], spec_waves, &ms);
                                cms[j] = ms;
                            } catch (const Error&) {
                                jk[j] = nullptr;  // back to the interpreter
                                cms[j] = 0;
                            }
                        }
                    }
                } catch (...) {
                    compile_error = std::current_exception();
                }
            });
        // Interpreter cones predicted to take at least a millisecond gain nothing from sharing
        // a launch (a launch costs tens of microseconds) and lose their own schedule to the
        // group's, which is sized for the group's largest cone: they run as their own launches.
        std::vector<size_t> alone;
        std::vector<uint8_t> is_alone(k, 0);
        if (!o.words_per_thread && !o.wg_size)
            for (size_t i = 0; i < k; ++i) {
                if (is_spec[i]) continue;
                Circuit& c = *v[i];
                const double patterns = 32.0 * (double)(rs[i].end - rs[i].begin);
                if (model_interp_ms(c.interp_gates(), c.interp_rows(), patterns) >= 1.0) {
                    is_alone[i] = 1;
                    alone.push_back(i);
                }
            }
        // Groups by value-file size: one launch sizes every wave's file for its largest cone,
        // so cones with few rows would otherwise run at the occupancy of the largest.  Rows
        // are bucketed by powers of two; each group gets its own schedule and recorded launch,
        // and the groups run back to back on the stream.
        // Cones whose files fit the register tier are grouped by its file size (104, 144, 232
        // rows: the waves per SIMD a launch gets), the others by powers of two of their rows.
        std::map<uint32_t, std::vector<size_t>> groups;
        for (size_t i = 0; i < k; ++i) {
            if (is_spec[i] || is_alone[i]) continue;
            const int t = regs_tier_enabled() ? model_interp_tier(v[i]->interp_rows()) : 3;
            if (t < 3) {
                groups[(uint32_t)t].push_back(i);
                continue;
            }
            uint32_t rows = v[i]->plan_for(8).rows, b = 0;
            while (rows > 1) {
                rows >>= 1;
                ++b;
            }
            groups[3 + b].push_back(i);
        }
        double total_ms = 0;
        for (auto& gi : groups) {
            std::vector<Circuit*> gv;
            std::vector<HwRange> gr;
            for (size_t i : gi.second) {
                gv.push_back(v[i]);
                gr.push_back(rs[i]);
            }
            // Schedule: the caller's fields when given, otherwise the autotuner's choice.
            Schedule sch;
            if (o.words_per_thread || o.wg_size) sch = default_schedule(dev, gv, &o);
            else sch = autotune(dev, gv, gr, stream, o.kernel == FASTLEC_KERNEL_INTERP_HBM);
            if (o.tile_words) sch.tile_hw = 2ull * o.tile_words;
            std::vector<uint64_t> best;
            double ms = 0;
            run_batch_graph(dev, gv, gr, sch, stream, best, &ms);
            total_ms += ms;
            for (size_t t = 0; t < gi.second.size(); ++t) {
                const size_t i = gi.second[t];
                std::memset(&out[i], 0, sizeof(out[i]));
                fill_result(*v[i], rs[i], best[t], &out[i]);
                out[i].predicted_ms = model_interp_ms(v[i]->interp_gates(), v[i]->interp_rows(),
                                                      32.0 * (double)(rs[i].end - rs[i].begin));
            }
        }
        for (size_t i = 0; i < k; ++i)
            if (!is_spec[i] && !is_alone[i]) out[i].kernel_ms = total_ms;
        auto run_alone = [&](size_t i) {
            std::vector<Circuit*> one{v[i]};
            std::vector<HwRange> r1{rs[i]};
            Schedule sch = default_schedule(dev, one, &o, rs[i].end - rs[i].begin);
            if (o.tile_words) sch.tile_hw = 2ull * o.tile_words;
            std::vector<uint64_t> best;
            double ms = 0;
            run_interp(dev, one, r1, sch, stream, nullptr, best, &ms);
            std::memset(&out[i], 0, sizeof(out[i]));
            fill_result(*v[i], rs[i], best[0], &out[i]);
            out[i].kernel_ms = ms;
            out[i].predicted_ms = model_interp_ms(v[i]->interp_gates(), v[i]->interp_rows(),
                                                  32.0 * (double)(rs[i].end - rs[i].begin));
        };
        for (size_t i : alone) run_alone(i);
        if (compile_job.t.joinable()) compile_job.t.join();
        if (compile_error) std::rethrow_exception(compile_error);
        if (!spec.empty()) {
            for (size_t j = 0; j < spec.size(); ++j) {
                const size_t i = spec[j];
                if (!jk[j]) {
                    run_alone(i);
                    continue;
                }
                uint64_t best = ~0ull;
                double ms = 0;
                run_jit(dev, *v[i], *jk[j], rs[i], o.tile_words ? 2ull * o.tile_words : 0, stream, nullptr, &best, &ms);
                std::memset(&out[i], 0, sizeof(out[i]));
                fill_result(*v[i], rs[i], best, &out[i]);
                out[i].kernel_ms = ms;
                out[i].compile_ms = cms[j];
                out[i].predicted_ms = model_specialized_ms(v[i]->lut_program().lut_steps,
                                                           32.0 * (double)(rs[i].end - rs[i].begin));
            }
        }
        return FASTLEC_OK;
    });
}

int fastlec_es_check_noalloc(const fastlec_es_circuit* c, const fastlec_es_options* opts, fastlec_es_result* out) {
    return guarded([&] {
        if (!c || !out) throw Error{kErrInvalid, "null argument"};
        fastlec_es_options o = opts ? *opts : defaults();
        if (o.kernel != FASTLEC_KERNEL_AUTO && o.kernel != FASTLEC_KERNEL_INTERP)
            throw Error{kErrInvalid, "the no-allocation entry point runs only the interpreter with LDS value files"};
        if (o.deadline_s > 0 || o.cancel_flag)
            throw Error{kErrInvalid, "the no-allocation entry point takes no deadline or cancel flag"};
        o.kernel = FASTLEC_KERNEL_INTERP;
        Circuit& cc = const_cast<Circuit&>(c->c);
        Device& dev = device(o.device);
        hipStream_t stream = o.hip_stream ? (hipStream_t)o.hip_stream : dev.stream;
        const HwRange r = range_of(cc.plan1.num_inputs, o.begin_word, o.end_word);
        std::memset(out, 0, sizeof(*out));
        double ms = 0;
        const uint64_t best = noalloc_check(dev, cc, o, r, stream, &ms);
        fill_result(cc, r, best, out);
        out->kernel_ms = ms;
        out->predicted_ms = model_interp_ms(cc.interp_gates(), cc.interp_rows(), 32.0 * (double)(r.end - r.begin));
        return FASTLEC_OK;
    });
}

void fastlec_es_free(fastlec_es_circuit* c) { delete c; }

// Compile the specialized kernel of a circuit without running it (no GPU needed).
// Writes the generated source's size and compile time; used to check the build path.
int fastlec_es_compile_specialized(const fastlec_es_circuit* c, int waves_per_eu, double* compile_ms,
                                   size_t* code_bytes) {
    return guarded([&] {
        if (!c) throw Error{kErrInvalid, "null circuit"};
        if (waves_per_eu < 1 || waves_per_eu > 8) throw Error{kErrInvalid, "waves_per_eu must be 1..8"};
        double ms = 0;
        auto k = jit_kernel(const_cast<Circuit&>(c->c), waves_per_eu, &ms);
        if (compile_ms) *compile_ms = ms;
        if (code_bytes) *code_bytes = k->code->bytes->size();
        return FASTLEC_OK;
    });
}

// Text of the specialized kernel source (for inspection); returns the length needed.
size_t fastlec_es_specialized_source(const fastlec_es_circuit* c, int waves_per_eu, char* buf, size_t len) {
    if (!c) return 0;
    std::string s = jit_source(const_cast<Circuit&>(c->c).lut_program(), waves_per_eu, 256);
    if (buf && len) {
        size_t m = std::min(len - 1, s.size());
        std::memcpy(buf, s.data(), m);
        buf[m] = 0;
    }
    return s.size() + 1;
}

// Host evaluation of the specialized kernel's LUT program, for validating the mapping without a GPU.
int fastlec_es_host_replay_specialized(const fastlec_es_circuit* c, uint64_t hw, uint64_t count, uint32_t* out) {
    return guarded([&] {
        if (!c || !out) throw Error{kErrInvalid, "null argument"};
        const LutProgram& lp = const_cast<Circuit&>(c->c).lut_program();
        for (uint64_t t = 0; t < count; ++t) out[t] = eval_lut_program(lp, hw + t);
        return FASTLEC_OK;
    });
}

// Replay of the register tier's encoded stream with that kernel's reading of it: row numbers
// are the low 8 bits of the operand and destination words, the complement and XOR masks are
// the stream's own words, and outputs count only in bundles whose mark bit is set.
void replay_regs_stream(Circuit& cc, uint64_t hw, uint64_t count, uint32_t* out) {
    const Plan& p = cc.plan_for(4);
    int waves = 0;
    if (!interp_regs_rows(p.rows, &waves)) throw Error{kErrInvalid, "value file does not fit the register tier"};
    const std::vector<uint32_t>& rs = cc.regs_stream();
    const size_t nb = p.prog.size() / 4;
    if (rs.size() != (nb + 1) * kRegsBundleWords) throw Error{kErrInvalid, "register stream size"};
    for (size_t k = nb * kRegsBundleWords; k < rs.size(); ++k)
        if (rs[k]) throw Error{kErrInvalid, "register stream padding is not zero"};
    static const uint32_t kc[5] = {0xAAAAAAAAu, 0xCCCCCCCCu, 0xF0F0F0F0u, 0xFF00FF00u, 0xFFFF0000u};
    std::vector<uint32_t> rows(256, 0);
    for (uint64_t t = 0; t < count; ++t) {
        const uint64_t h = hw + t;
        rows[0] = 0;
        for (uint32_t i = 0; i < p.num_inputs; ++i) rows[1 + i] = i < 5 ? kc[i] : 0u - (uint32_t)((h >> (i - 5)) & 1u);
        uint32_t m = 0;
        for (size_t b = 0; b < nb; ++b) {
            const uint32_t* w = rs.data() + b * kRegsBundleWords;
            uint32_t val[4];
            for (int u = 0; u < 4; ++u) {
                const uint32_t x = rows[w[u] & 0xFFu] ^ w[12 + u], y = rows[w[4 + u] & 0xFFu] ^ w[16 + u];
                val[u] = (w[20 + u] & (x ^ y)) | (~w[20 + u] & x & y);
            }
            const bool marked = (w[8] >> 31) != 0;
            for (int u = 0; u < 4; ++u) {
                rows[w[8 + u] & 0xFFu] = val[u];
                if (marked && (w[24 + u] & kOutPos)) m |= val[u];
                if (marked && (w[24 + u] & kOutNeg)) m |= ~val[u];
            }
        }
        out[t] = m;
    }
}

// Replay of the interpreter instruction stream on the host (bundle semantics: all reads of a
// bundle, then all writes), for validating plans without a GPU.  Returns the miter words of
// the 32-pattern half-words [hw, hw + count) in out.  Bundle 0 replays the register tier's
// encoded stream instead.
int fastlec_es_host_replay(const fastlec_es_circuit* c, uint32_t bundle, uint64_t hw, uint64_t count, uint32_t* out) {
    return guarded([&] {
        if (!c || !out) throw Error{kErrInvalid, "null argument"};
        Circuit& cc = const_cast<Circuit&>(c->c);
        if (bundle == 0) {
            replay_regs_stream(cc, hw, count, out);
            return FASTLEC_OK;
        }
        const Plan& p = cc.plan_for(bundle);
        std::string err = validate_plan(bundle <= 1 ? cc.aig : cc.fused, p);
        if (!err.empty()) throw Error{kErrInvalid, "invalid plan: " + err};
        std::vector<uint32_t> rows(p.rows, 0);
        for (uint64_t t = 0; t < count; ++t) {
            const uint64_t h = hw + t;
            static const uint32_t kc[5] = {0xAAAAAAAAu, 0xCCCCCCCCu, 0xF0F0F0F0u, 0xFF00FF00u, 0xFFFF0000u};
            rows[0] = 0;
            for (uint32_t i = 0; i < p.num_inputs; ++i)
                rows[1 + i] = i < 5 ? kc[i] : 0u - (uint32_t)((h >> (i - 5)) & 1u);
            uint32_t m = 0;
            for (size_t b0 = 0; b0 < p.prog.size(); b0 += p.bundle) {
                std::vector<uint32_t> val(p.bundle);
                for (uint32_t u = 0; u < p.bundle; ++u) {
                    const Instr& ins = p.prog[b0 + u];
                    uint32_t a = rows[ins.a & kRowMask] ^ (0u - (ins.a >> 31));
                    uint32_t b = rows[ins.b & kRowMask] ^ (0u - (ins.b >> 31));
                    val[u] = (ins.flags & kXor) ? a ^ b : a & b;
                }
                for (uint32_t u = 0; u < p.bundle; ++u) {
                    const Instr& ins = p.prog[b0 + u];
                    rows[ins.d] = val[u];
                    if (ins.flags & kOutPos) m |= val[u];
                    if (ins.flags & kOutNeg) m |= ~val[u];
                }
            }
            out[t] = m;
        }
        return FASTLEC_OK;
    });
}

int fastlec_es_simulate(const fastlec_es_circuit* c, const uint32_t* pi_words, uint64_t num_words, uint32_t* sig,
                        const fastlec_es_options* opts, double* kernel_ms) {
    return guarded([&] {
        if (!c || !sig || num_words == 0) throw Error{kErrInvalid, "null circuit or signature, or no words"};
        Circuit& cc = const_cast<Circuit&>(c->c);
        if (cc.aig.num_inputs && !pi_words) throw Error{kErrInvalid, "null input words"};
        fastlec_es_options o = opts ? *opts : defaults();
        Device& dev = device(o.device);
        hipStream_t stream = o.hip_stream ? (hipStream_t)o.hip_stream : dev.stream;
        run_sim(dev, cc, pi_words, num_words, sig, &o, stream, kernel_ms);
        return FASTLEC_OK;
    });
}

int fastlec_es_signature_hash(const uint32_t* sig, uint64_t rows, uint64_t num_words, uint64_t* hash, uint64_t* ones,
                              const fastlec_es_options* opts, double* kernel_ms) {
    return guarded([&] {
        if (!sig || !hash || !ones || rows == 0 || num_words == 0) throw Error{kErrInvalid, "null pointer or empty matrix"};
        fastlec_es_options o = opts ? *opts : defaults();
        Device& dev = device(o.device);
        hipStream_t stream = o.hip_stream ? (hipStream_t)o.hip_stream : dev.stream;
        // One wave per row; enough workgroups of four waves for eight per CU, fewer for few rows.
        const uint64_t want = (rows + 3) / 4;
        const int grid = (int)std::min<uint64_t>(want, (uint64_t)dev.prop.multiProcessorCount * 8);
        ScopedEvent e0, e1;
        FES_HIP(hipEventRecord(e0.e, stream));
        FES_HIP(launch_signature_hash(sig, rows, num_words, hash, ones, grid, stream));
        FES_HIP(hipEventRecord(e1.e, stream));
        FES_HIP(hipStreamSynchronize(stream));
        float ms = 0;
        FES_HIP(hipEventElapsedTime(&ms, e0.e, e1.e));
        if (kernel_ms) *kernel_ms = ms;
        return FASTLEC_OK;
    });
}

int fastlec_es_classes(const uint64_t* hash, uint64_t rows, uint32_t* class_of) {
    return guarded([&] {
        if (rows && (!hash || !class_of)) throw Error{kErrInvalid, "null pointer"};
        if (rows > UINT32_MAX) throw Error{kErrInvalid, "more than 2^32 - 1 rows"};
        std::unordered_map<uint64_t, uint32_t> first;
        first.reserve(rows);
        for (uint64_t r = 0; r < rows; ++r) class_of[r] = first.emplace(hash[r], (uint32_t)r).first->second;
        return FASTLEC_OK;
    });
}

int fastlec_es_submiter_aag(const fastlec_es_circuit* c, const uint32_t* class_of, const uint8_t* polarity,
                            uint64_t rows, uint32_t target, char* buf, size_t len, size_t* needed,
                            uint32_t* inputs, uint32_t* num_inputs) {
    return guarded([&] {
        if (!c || !class_of || !polarity) throw Error{kErrInvalid, "null argument"};
        std::vector<uint32_t> ins;
        const std::string text = submiter_aag(c->c.aig, class_of, polarity, rows, target, &ins);
        if (needed) *needed = text.size() + 1;
        if (num_inputs) *num_inputs = (uint32_t)ins.size();
        if (inputs) std::copy(ins.begin(), ins.end(), inputs);
        if (buf) {
            if (len < text.size() + 1) throw Error{kErrInvalid, "buffer too small"};
            std::memcpy(buf, text.c_str(), text.size() + 1);
        }
        return FASTLEC_OK;
    });
}

int fastlec_es_predict(const fastlec_es_circuit* c, uint64_t begin_word, uint64_t end_word, double* interp_ms,
                       double* specialized_ms, double* compile_ms) {
    return guarded([&] {
        if (!c) throw Error{kErrInvalid, "null circuit"};
        Circuit& cc = const_cast<Circuit&>(c->c);
        const HwRange r = range_of(cc.plan1.num_inputs, begin_word, end_word);
        const double patterns = 32.0 * (double)(r.end - r.begin);
        if (interp_ms)
            *interp_ms = model_interp_ms(cc.interp_gates(), cc.interp_rows(), patterns);
        if (specialized_ms || compile_ms) {
            const uint32_t luts = cc.lut_program().lut_steps;
            if (specialized_ms) *specialized_ms = model_specialized_ms(luts, patterns);
            if (compile_ms) *compile_ms = model_compile_ms(luts);
        }
        return FASTLEC_OK;
    });
}

int fastlec_es_memory_get(int dev_ordinal, uint64_t* device_bytes, uint64_t* pinned_bytes) {
    return guarded([&] {
        Device& dev = device(dev_ordinal);
        std::lock_guard<std::mutex> g(dev.mu);
        if (device_bytes) *device_bytes = dev.pool_device_bytes;
        if (pinned_bytes) *pinned_bytes = dev.pool_pinned_bytes;
        return FASTLEC_OK;
    });
}

int fastlec_es_valu_probe(int dev_ordinal, uint32_t variant, uint32_t waves_per_simd, uint32_t iters,
                          double* instr_per_s, double* kernel_ms) {
    return guarded([&] {
        Device& dev = device(dev_ordinal);
        const double r = valu_probe(dev, variant, waves_per_simd, iters, dev.stream, kernel_ms);
        if (instr_per_s) *instr_per_s = r;
        return FASTLEC_OK;
    });
}

int fastlec_es_compile_specialized_many(const fastlec_es_circuit* const* cs, size_t k, int waves_per_eu,
                                        double* compile_ms) {
    return guarded([&] {
        if (k && !cs) throw Error{kErrInvalid, "null argument"};
        if (waves_per_eu < 1 || waves_per_eu > 8) throw Error{kErrInvalid, "waves_per_eu must be 1..8"};
        std::vector<Circuit*> v;
        for (size_t i = 0; i < k; ++i) {
            if (!cs[i]) throw Error{kErrInvalid, "null circuit"};
            v.push_back(const_cast<Circuit*>(&cs[i]->c));
        }
        std::vector<double> ms;
        jit_kernels(v, waves_per_eu, &ms);
        double total = 0;
        for (double x : ms) total += x;
        if (compile_ms) *compile_ms = total;
        return FASTLEC_OK;
    });
}

}  // extern "C"
