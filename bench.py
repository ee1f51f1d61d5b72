"""Benchmark: exact simulation of the 16x16 multiplier miter on one MI355X.

One step = one complete exact simulation of the miter of a 16x16 array
multiplier against a radix-4 Booth/Wallace multiplier (32 inputs, 2^32
patterns, every pattern simulated because the miter is equivalent), through
the C ABI (fastlec_es_check), on PyTorch's current stream.  The metric is AND
node * pattern evaluations per second: N (AND gates in the output cone) times
2^32 per step.

Prints one JSON line.  Besides the headline it reports the roofline of the
simulation kernel (integer VALU bound; achieved from the kernel's own HIP
event time) and the plain CPU oracle timed on a bounded sample on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Integer-VALU roofline of MI355X: 256 CUs * 64 lanes * 2.4 GHz int32 lane-ops per second;
# one lane-op evaluates one AND gate on 32 patterns.
CUS, LANES, CLOCK_HZ = 256, 64, 2.4e9
PEAK_LANE_OPS = CUS * LANES * CLOCK_HZ
PEAK_NODE_PATTERNS = PEAK_LANE_OPS * 32


def cpu_baseline(aag: bytes, num_ands: int, target_s: float = 12.0):
    """The oracle (one pattern at a time, all host cores) on an ascending prefix of the space."""
    import oracle
    c = oracle.Circuit(aag)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(threads, int(os.environ.get("OMP_NUM_THREADS", threads))))
    patterns = 1 << 14
    while True:
        t0 = time.perf_counter()
        p, ev = c.lowest_failure(0, patterns, threads=threads)
        dt = time.perf_counter() - t0
        if p is not None:
            raise RuntimeError("oracle found a failure in an equivalent miter")
        if dt >= target_s / 4 or patterns >= 1 << 30:
            break
        patterns = min(1 << 30, int(patterns * max(2.0, min(16.0, target_s / max(dt, 1e-3)))))
        patterns = 1 << (patterns.bit_length() - 1)
    return {"value": num_ands * ev / dt, "unit": "node*patterns/s", "cores": threads, "kind": "oracle",
            "sample": f"patterns [0, {patterns}) of the same miter, {dt:.1f} s on {threads} threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kernel", default="specialized")
    ap.add_argument("--workload", default="mult16_array_booth")
    ap.add_argument("--no-cpu", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only: exact simulation here is a single-GPU build "
              f"(--gpus {a.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch
    import miters
    import paper_2512_06627_amd as es

    torch.cuda.init()
    stream = torch.cuda.current_stream()
    g = miters.workload(a.workload)
    aig = g.to_aig()
    t0 = time.perf_counter()
    c = es.fastlec_es_load_aig(aig)
    load_ms = (time.perf_counter() - t0) * 1e3
    info = c.info()
    n, N = info["num_pis"], info["num_ands_tfi"]
    node_patterns = N * (1 << n)

    compile_ms = 0.0
    for _ in range(a.warmup):
        r = es.fastlec_es_check(c, stream=stream, kernel=a.kernel)
        compile_ms += r["compile_ms"]
        if r["verdict"] != es.FASTLEC_EQUIVALENT:
            raise RuntimeError(f"expected an equivalent miter, got {r}")

    kernel_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        r = es.fastlec_es_check(c, stream=stream, kernel=a.kernel)
        kernel_ms.append(r["kernel_ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for_each_ok = r["verdict"] == es.FASTLEC_EQUIVALENT and r["patterns_evaluated"] == 1 << n

    ms_per_step = elapsed * 1e3 / a.steps
    value = node_patterns * a.steps / elapsed
    k_ms = sorted(kernel_ms)[len(kernel_ms) // 2]
    achieved = node_patterns / (sum(kernel_ms) / len(kernel_ms) / 1e3)
    out = {
        "metric": "ES node*patterns/s (16x16 mult miter)",
        "value": value,
        "unit": "node*patterns/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: {n} inputs, 2^{n} patterns, {N} AND gates in cone, "
                               f"equivalent (all patterns simulated)",
                   "kernel": a.kernel, "peak_live_slots": info["peak_live_slots"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_NODE_PATTERNS,
                     "unit": "node*patterns/s", "frac": achieved / PEAK_NODE_PATTERNS, "traffic": None,
                     "kernel_ms_median": k_ms,
                     "note": "peak = 256 CU * 64 lanes * 2.4 GHz int32 lane-ops * 32 patterns per lane-op "
                             "(one lane-op per AND gate); achieved = N*2^n / mean kernel time (HIP events)"},
        "load_ms": load_ms,
        "compile_ms": compile_ms,
        "all_steps_equivalent": bool(for_each_ok),
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(g.to_aag(), N)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
