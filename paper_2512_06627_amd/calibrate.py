"""Measure exact-simulation times on this GPU and fit the library's runtime model.

The paper predicts ES time as linear in the gate count and exponential in the
input count, t = alpha * num_gates * 2^(num_PI - beta), with coefficients
fitted from measurements (Section 3.2, runtime prediction; alpha and beta
together are one rate, since alpha * 2^-beta is a single constant).  The
library's model (fastlec_es_predict) keeps that form per kernel and adds a
fixed launch cost:

* interpreter: t = t0 + N * max(2^n / R, L), N = gate instructions of its stream (AND gates
  of the cone, each fused three-AND XOR counted once), with one rate R per value-file tier
  (register tier files of at most 104, 144 and 232 rows, at four, three and two waves per SIMD;
  LDS or device memory above: the interpreter's rate follows the waves a SIMD holds); L is the
  time per gate of one wave's pass, the floor when the space has fewer passes than the chip has
  waves;
* specialized kernel: t = t0 + L * passes / R, L = LUT steps of its program,
  passes = 2^(n-11) (2,048 patterns per wave pass);
* hipRTC compile of the specialized kernel: t = c0 + c1 * L.

This script times plain checks of seeded layered cones and multiplier miters
with each kernel (kernel times from the library's HIP events; compile time as
the library reports it), fits the constants by least squares on relative
error, and prints one JSON object with the fitted constants, the data and the
fit's errors.  Run it on the GPU:  python -m paper_2512_06627_amd.calibrate
"""
import json
import sys

import numpy as np


def cones():
    import miters
    out = []
    for n in (16, 18, 20, 22, 24, 26, 28):
        for target in (300, 1000, 3000, 8000):
            if target * (1 << n) > 3e12:
                continue
            out.append((f"layered_n{n}_{target}", miters.layered_cone_miter(1000 + n * 7 + target, n, target)))
    for n, target in ((16, 14000), (16, 20000), (18, 20000), (20, 16000), (22, 12000), (24, 16000),
                      (26, 20000)):  # files above 232 rows, small and large spaces
        out.append((f"layered_n{n}_{target}", miters.layered_cone_miter(1000 + n * 7 + target, n, target)))
    for name in ("mult6_array_wallace", "mult12_array_booth", "mac8_fused_separate", "mult16_array_booth"):
        out.append((name, miters.workload(name)))
    return out


def lut_steps(es, c):
    src = es.fastlec_es_specialized_source(c, 3)
    head = [x for x in src.splitlines() if x.startswith("// exact simulation")][0]
    return int(head.split(": ")[1].split(" LUT")[0])


def measure(es, stream, reps=3):
    rows = []
    for name, g in cones():
        c = es.fastlec_es_load_aig(g.to_aig())
        info = c.info()
        rec = {"name": name, "n": info["num_pis"], "N": info["num_instrs"] - 2 * info["num_xors"],
               "rows": info["interp_rows"],
               "luts": lut_steps(es, c)}
        if rec["N"] * (1 << rec["n"]) <= 3e12:
            es.fastlec_es_check(c, stream=stream, kernel="interp")
            rec["interp_ms"] = float(np.median([es.fastlec_es_check(c, stream=stream, kernel="interp")["kernel_ms"]
                                                for _ in range(reps)]))
        r = es.fastlec_es_check(c, stream=stream, kernel="specialized")
        rec["compile_ms"] = r["compile_ms"]
        rec["specialized_ms"] = float(np.median([es.fastlec_es_check(c, stream=stream, kernel="specialized")["kernel_ms"]
                                                 for _ in range(reps)]))
        rows.append(rec)
        print(json.dumps(rec), file=sys.stderr, flush=True)
    return rows


def fit_linear(x, t):
    """t ~ a + b x, least squares on relative error (weights 1/t)."""
    x, t = np.asarray(x, float), np.asarray(t, float)
    A = np.stack([np.ones_like(x), x], axis=1) / t[:, None]
    (a, b), *_ = np.linalg.lstsq(A, np.ones_like(t), rcond=None)
    rel = (a + b * x) / t - 1
    return float(a), float(b), float(np.median(np.abs(rel))), float(np.max(np.abs(rel)))


TIER_ROWS = (104, 144, 232)  # register tier files; LDS or device memory above


def tier(rows):
    for t, r in enumerate(TIER_ROWS):
        if rows <= r:
            return t
    return len(TIER_ROWS)


def fit_interp(ri):
    """t ~ t0 + N max(2^n / R_tier, L): L by a search over a grid, t0 and the tier rates by least
    squares on relative error (a tier without data keeps no rate)."""
    t = np.array([r["interp_ms"] for r in ri])
    N = np.array([float(r["N"]) for r in ri])
    P = np.array([2.0 ** r["n"] for r in ri])
    tr = np.array([tier(r["rows"]) for r in ri])
    tiers = sorted(set(tr.tolist()))
    best = None
    for L in np.geomspace(1e-6, 1e-3, 61):  # ms per gate
        # for fixed L the model is linear in (t0, 1/R_tier) where N P / R exceeds N L; iterate
        # the split from "rate everywhere"
        use_rate = np.ones_like(t, dtype=bool)
        for _ in range(3):
            cols = [np.ones_like(t)] + [np.where(use_rate & (tr == k), N * P, 0) for k in tiers]
            A = np.stack(cols, axis=1)
            y = t - np.where(use_rate, 0, N * L)
            coef, *_ = np.linalg.lstsq(A / t[:, None], y / t, rcond=None)
            a = coef[0]
            b = np.zeros_like(t)
            for j, k in enumerate(tiers):
                b[tr == k] = coef[1 + j]
            use_rate = P * b > L
        pred = a + N * np.maximum(P * b, L)
        rel = pred / t - 1
        score = np.median(np.abs(rel)) + 0.25 * np.max(np.abs(rel))
        if best is None or score < best[0]:
            rates = {int(k): float(1e3 / coef[1 + j]) for j, k in enumerate(tiers)}
            best = (score, float(a), rates, float(L), float(np.median(np.abs(rel))), float(np.max(np.abs(rel))))
    return best[1:]


def fit(rows):
    ri = [r for r in rows if "interp_ms" in r]
    a_i, rates, L_i, med_i, max_i = fit_interp(ri)
    a_s, b_s, med_s, max_s = fit_linear([r["luts"] * 2.0 ** max(0, r["n"] - 11) for r in rows],
                                        [r["specialized_ms"] for r in rows])
    rc = [r for r in rows if r["compile_ms"] > 0]
    a_c, b_c, med_c, max_c = fit_linear([r["luts"] for r in rc], [r["compile_ms"] for r in rc])
    return {"interp_t0_ms": a_i, "interp_tier_rows": list(TIER_ROWS),
            "interp_gate_patterns_per_s_by_tier": rates,
            "interp_ms_per_gate_floor": L_i,
            "interp_median_rel_err": med_i, "interp_max_rel_err": max_i,
            "specialized_t0_ms": a_s, "specialized_lut_passes_per_s": 1e3 / b_s,
            "specialized_median_rel_err": med_s, "specialized_max_rel_err": max_s,
            "compile_c0_ms": a_c, "compile_ms_per_lut": b_c,
            "compile_median_rel_err": med_c, "compile_max_rel_err": max_c}


def main():
    import torch
    import paper_2512_06627_amd as es
    torch.cuda.init()
    rows = measure(es, torch.cuda.current_stream())
    print(json.dumps({"fit": fit(rows), "data": rows}))


if __name__ == "__main__":
    main()
