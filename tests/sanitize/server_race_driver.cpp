// The serving loop's host scheduling under ThreadSanitizer.
//
// The server has three kinds of host threads: callers (submit, poll, stats), its step loop
// (admission, slices, retirement, device table) and its compile thread (specialized kernels for
// the jobs that carry most of the work).  This driver runs them against each other: several
// submitter threads, poller threads that take tickets from the submitters, a stats reader, and a
// second server destroyed while jobs and compiles are still in flight.  Every answer must equal
// the same circuit checked alone with fastlec_es_check.  In between, four threads run plain
// checks (each kernel choice) and predictions on the same handles at once, then two threads run
// batches of those handles and fresh ones (each kernel choice; with FASTLEC_ES_BATCH_JIT=2 AUTO
// routes the handles whose kernels exist to them, so each batch's compile thread runs beside its
// interpreter launches over the fresh handles).
//
// Built with -fsanitize=thread together with the library's host sources and fake_device.cpp
// (a host stand-in for the GPU: the HIP runtime finds no device in a process built with the
// thread sanitizer), so it runs without a GPU; a data race ends the run with the sanitizer's
// report and a non-zero status.  Linked with the library instead, it runs the same scenario on
// a GPU without the sanitizer.
//
// Usage: server_race_driver file.aig...   Prints "ok <jobs>" on success.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "fastlec_es.h"

namespace {

std::string read_file(const char* path) {
    std::ifstream f(path, std::ios::binary);
    std::stringstream ss;
    ss << f.rdbuf();
    return ss.str();
}

uint64_t answer(const fastlec_es_result& r) { return r.verdict == FASTLEC_NONEQUIVALENT ? r.cex : ~0ull; }

int fail(const char* what, int rc) {
    std::fprintf(stderr, "FAIL %s: %d %s\n", what, rc, fastlec_es_last_error());
    return 1;
}

}  // namespace

int main(int argc, char** argv) {
    std::vector<fastlec_es_circuit*> cs;
    for (int i = 1; i < argc; ++i) {
        const std::string s = read_file(argv[i]);
        fastlec_es_circuit* c = nullptr;
        const int rc = fastlec_es_load_aig(s.data(), s.size(), &c);
        if (rc) return fail(argv[i], rc);
        cs.push_back(c);
    }
    if (cs.empty()) return fail("no circuits", 0);
    fastlec_es_options o;
    fastlec_es_options_init(&o);
    std::vector<uint64_t> want(cs.size());
    for (size_t i = 0; i < cs.size(); ++i) {
        fastlec_es_result r;
        const int rc = fastlec_es_check(cs[i], &o, &r);
        if (rc) return fail("plain check", rc);
        want[i] = answer(r);
    }

    fastlec_es_server* srv = nullptr;
    int rc = fastlec_es_server_create(&o, size_t(64) << 30, &srv);
    if (rc) return fail("server create", rc);
    constexpr int kSubmitters = 4, kPollers = 2, kRounds = 3;
    std::mutex mu;
    std::vector<std::pair<uint64_t, size_t>> handed;  // tickets for the pollers
    std::atomic<int> submitters_left{kSubmitters};
    std::atomic<int> mismatches{0}, errors{0}, done{0};
    std::atomic<bool> stop_stats{false};
    auto check = [&](size_t i, const fastlec_es_result& r) {
        if (answer(r) != want[i]) mismatches.fetch_add(1);
        done.fetch_add(1);
    };
    std::vector<std::thread> th;
    for (int t = 0; t < kSubmitters; ++t)
        th.emplace_back([&, t] {
            std::vector<std::pair<uint64_t, size_t>> mine;
            for (int round = 0; round < kRounds; ++round)
                for (size_t k = 0; k < cs.size(); ++k) {
                    const size_t i = (k + (size_t)t) % cs.size();
                    uint64_t ticket = 0;
                    if (fastlec_es_server_submit(srv, cs[i], &ticket)) {
                        errors.fetch_add(1);
                        continue;
                    }
                    if ((k + (size_t)round) % 2) {
                        std::lock_guard<std::mutex> g(mu);
                        handed.emplace_back(ticket, i);
                    } else {
                        mine.emplace_back(ticket, i);
                    }
                }
            for (auto& [ticket, i] : mine) {
                fastlec_es_result r;
                if (fastlec_es_server_poll(srv, ticket, &r, 1) != 1) errors.fetch_add(1);
                else check(i, r);
            }
            submitters_left.fetch_sub(1);
        });
    for (int t = 0; t < kPollers; ++t)
        th.emplace_back([&] {
            for (;;) {
                std::pair<uint64_t, size_t> job;
                bool have = false;
                {
                    std::lock_guard<std::mutex> g(mu);
                    if (!handed.empty()) {
                        job = handed.back();
                        handed.pop_back();
                        have = true;
                    }
                }
                if (!have) {
                    if (submitters_left.load() == 0) {
                        std::lock_guard<std::mutex> g(mu);
                        if (handed.empty()) return;
                        continue;
                    }
                    std::this_thread::sleep_for(std::chrono::microseconds(200));
                    continue;
                }
                fastlec_es_result r;
                const int p = fastlec_es_server_poll(srv, job.first, &r, 0);  // not blocking: retry later
                if (p == 1) {
                    check(job.second, r);
                } else if (p == 0) {
                    std::lock_guard<std::mutex> g(mu);
                    handed.insert(handed.begin(), job);
                } else {
                    errors.fetch_add(1);
                }
            }
        });
    std::thread stats([&] {
        while (!stop_stats.load()) {
            fastlec_es_server_stats st;
            if (fastlec_es_server_stats_get(srv, &st) || st.completed > st.submitted) errors.fetch_add(1);
            std::this_thread::sleep_for(std::chrono::microseconds(500));
        }
    });
    for (auto& t : th) t.join();
    stop_stats.store(true);
    stats.join();
    fastlec_es_server_stats st;
    fastlec_es_server_stats_get(srv, &st);
    fastlec_es_server_destroy(srv);
    const int total = kSubmitters * kRounds * (int)cs.size();
    std::printf("server: %d jobs, %d done, %d mismatches, %d errors, %llu specialized slices, %llu steps\n", total,
                done.load(), mismatches.load(), errors.load(), (unsigned long long)st.specialized_slices,
                (unsigned long long)st.steps);
    if (done.load() != total || mismatches.load() || errors.load()) return fail("server answers", 0);

    // Plain checks of the same handles from several threads at once (the header allows it):
    // plan, stream and kernel caches, the device's buffer pool and the runtime model.
    std::atomic<int> plain_bad{0};
    std::vector<std::thread> pt;
    for (int t = 0; t < 4; ++t)
        pt.emplace_back([&, t] {
            for (int round = 0; round < 2; ++round)
                for (size_t k = 0; k < cs.size(); ++k) {
                    const size_t i = (k + (size_t)t) % cs.size();
                    fastlec_es_options po;
                    fastlec_es_options_init(&po);
                    po.kernel = (t + round) % 3 == 0 ? FASTLEC_KERNEL_AUTO
                                : (t + round) % 3 == 1 ? FASTLEC_KERNEL_INTERP : FASTLEC_KERNEL_SPECIALIZED;
                    fastlec_es_result r;
                    if (fastlec_es_check(cs[i], &po, &r) || answer(r) != want[i]) plain_bad.fetch_add(1);
                    double pi = 0, ps = 0, pc = 0;
                    if (fastlec_es_predict(cs[i], 0, 0, &pi, &ps, &pc)) plain_bad.fetch_add(1);
                }
        });
    for (auto& t : pt) t.join();
    std::printf("plain checks from 4 threads: %d wrong\n", plain_bad.load());
    if (plain_bad.load()) return fail("concurrent plain checks", 0);

    std::atomic<int> batch_bad{0};
    std::vector<std::thread> bt;
    for (int t = 0; t < 2; ++t)
        bt.emplace_back([&, t] {
            // The checked handles (kernels compiled above) and a fresh copy of each circuit.
            std::vector<fastlec_es_circuit*> mix;
            std::vector<uint64_t> mix_want;
            for (size_t i = 0; i < cs.size(); ++i) {
                const std::string s = read_file(argv[1 + i]);
                fastlec_es_circuit* c = nullptr;
                if (fastlec_es_load_aig(s.data(), s.size(), &c)) {
                    batch_bad.fetch_add(1);
                    return;
                }
                mix.push_back((i + (size_t)t) % 2 ? c : cs[i]);
                mix.push_back((i + (size_t)t) % 2 ? cs[i] : c);
                mix_want.push_back(want[i]);
                mix_want.push_back(want[i]);
            }
            for (int kern : {FASTLEC_KERNEL_AUTO, FASTLEC_KERNEL_INTERP, FASTLEC_KERNEL_SPECIALIZED}) {
                fastlec_es_options bo;
                fastlec_es_options_init(&bo);
                bo.kernel = kern;
                std::vector<fastlec_es_result> r(mix.size());
                if (fastlec_es_check_batch(mix.data(), mix.size(), &bo, r.data())) {
                    batch_bad.fetch_add(1);
                    continue;
                }
                for (size_t i = 0; i < mix.size(); ++i)
                    if (answer(r[i]) != mix_want[i]) batch_bad.fetch_add(1);
            }
            for (size_t i = 0; i < mix.size(); ++i)
                if (mix[i] != cs[i / 2]) fastlec_es_free(mix[i]);
        });
    for (auto& t : bt) t.join();
    std::printf("batches from 2 threads: %d wrong\n", batch_bad.load());
    if (batch_bad.load()) return fail("concurrent batches", 0);

    // Teardown with work in flight: jobs queued and running, compiles possibly under way.
    rc = fastlec_es_server_create(&o, size_t(64) << 30, &srv);
    if (rc) return fail("second server create", rc);
    for (int round = 0; round < 2; ++round)
        for (fastlec_es_circuit* c : cs) {
            uint64_t ticket = 0;
            if (fastlec_es_server_submit(srv, c, &ticket)) return fail("second server submit", 0);
        }
    std::this_thread::sleep_for(std::chrono::milliseconds(30));
    fastlec_es_server_destroy(srv);
    for (fastlec_es_circuit* c : cs) fastlec_es_free(c);
    std::printf("ok %d\n", total);
    return 0;
}
