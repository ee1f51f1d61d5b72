"""Write expected exact-simulation results of the named workloads, using only the oracle.

    python tests/golden/make_expected.py --resume PATH [NAME ...]

Each workload is scanned in ascending windows of ``threads << window_log2``
patterns; each window is one call of the oracle's multi-threaded scan, so the
first window holding a failure gives the lowest failing pattern.  Progress is
saved after every window in a resume file, and results go to expected.json as
soon as a workload finishes.  Every value written comes from
``oracle.Circuit``.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import miters  # noqa: E402
import oracle  # noqa: E402

DEFAULT = ["mult6_array_wallace", "mult6_array_wallace_f1", "mult12_array_booth",
           "mult12_array_booth_f1", "mult12_array_booth_f2", "mult12_array_booth_f3",
           "mult12_array_booth_f4", "mult16_array_booth_f1", "mult16_array_booth_f2",
           "mult16_array_booth_f3", "mult16_array_booth_f4", "mac8_fused_separate_f1",
           "mac8_fused_separate_f2", "mac8_fused_separate", "mult16_array_booth"]


def scan(name, threads, window_log2, resume_path, out_path):
    state = json.load(open(resume_path)) if os.path.exists(resume_path) else {}
    done = json.load(open(out_path)) if os.path.exists(out_path) else {}
    if name in done:
        return done[name]
    g = miters.workload(name)
    c = oracle.Circuit(g.to_aag())
    total = 1 << c.num_inputs
    st = state.get(name, {"next": 0, "simulated": 0, "seconds": 0.0})
    p = None
    last_print = 0.0
    while st["next"] < total and p is None:
        lo = st["next"]
        hi = min(total, lo + (threads << window_log2))
        t = time.time()
        p, ev = c.lowest_failure(lo, hi, threads=threads)
        st["seconds"] += time.time() - t
        st["simulated"] += ev
        st["next"] = hi
        state[name] = st
        if st["seconds"] - last_print > 60 or p is not None or hi == total:
            last_print = st["seconds"]
            json.dump(state, open(resume_path, "w"), indent=1)
            print(f"{name}: scanned to {hi:#x} of {total:#x}, p={p}, {st['seconds']:.0f}s", flush=True)
    res = {"num_inputs": c.num_inputs, "num_ands_in_cone": len(g.tfi_ands()),
           "lowest_failure": p, "patterns_simulated": st["simulated"],
           "oracle_seconds": round(st["seconds"], 1), "threads": threads}
    done = json.load(open(out_path)) if os.path.exists(out_path) else {}
    done[name] = res
    json.dump(done, open(out_path, "w"), indent=1, sort_keys=True)
    print("wrote", name, res, flush=True)
    return res


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*")
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    ap.add_argument("--window-log2", type=int, default=22)
    ap.add_argument("--resume", required=True,
                    help="file that keeps the scan position after every window (any writable path)")
    a = ap.parse_args()
    os.makedirs(os.path.dirname(os.path.abspath(a.resume)), exist_ok=True)
    for name in a.names or DEFAULT:
        scan(name, a.threads, a.window_log2, a.resume, os.path.join(HERE, "expected.json"))
