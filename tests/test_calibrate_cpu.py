"""The runtime-model fit (paper_2512_06627_amd/calibrate.py) recovers known constants.

Times are generated from the model's own form with chosen constants (interpreter: launch
cost, two rates split at ROWS_BREAK slots, a per-gate floor; specialized: launch cost and a
rate over LUT steps x passes; compile: fixed plus per-LUT cost) and perturbed by a seeded 3%
noise; the fit must return the constants within a few percent.  No GPU involved.
"""
import numpy as np

from paper_2512_06627_amd import calibrate


def synthetic(seed=7):
    rng = np.random.default_rng(seed)
    t0, r_lo, r_hi, floor = 0.02, 5e13, 3e13, 4e-5
    s0, s_rate, c0, c1 = 0.013, 6e11, 105.0, 0.0065
    rows = []
    for n in (12, 14, 16, 18, 20, 22, 24, 26, 28):
        for N in (300, 1000, 3000, 8000):
            slots = 40 + N // 60
            luts = N // 3
            P = 2.0 ** n
            ti = t0 + N * max(P / (r_hi if slots > calibrate.ROWS_BREAK else r_lo) * 1e3, floor)
            ts = s0 + luts * max(1.0, P / 2048.0) / s_rate * 1e3
            tc = c0 + c1 * luts
            noise = lambda: 1.0 + 0.03 * rng.standard_normal()
            rows.append({"name": f"n{n}_{N}", "n": n, "N": N, "rows": slots, "luts": luts,
                         "interp_ms": ti * noise(), "specialized_ms": ts * noise(), "compile_ms": tc * noise()})
    return rows, dict(t0=t0, r_lo=r_lo, r_hi=r_hi, floor=floor, s0=s0, s_rate=s_rate, c0=c0, c1=c1)


def test_fit_recovers_constants():
    rows, k = synthetic()
    f = calibrate.fit(rows)
    assert abs(f["interp_node_patterns_per_s"] / k["r_lo"] - 1) < 0.05
    assert abs(f["interp_node_patterns_per_s_above_break"] / k["r_hi"] - 1) < 0.05
    assert abs(f["interp_ms_per_gate_floor"] / k["floor"] - 1) < 0.15  # grid of 61 points per decade band
    assert abs(f["specialized_lut_passes_per_s"] / k["s_rate"] - 1) < 0.05
    assert abs(f["compile_c0_ms"] / k["c0"] - 1) < 0.05
    assert abs(f["compile_ms_per_lut"] / k["c1"] - 1) < 0.10
    assert f["interp_median_rel_err"] < 0.05 and f["specialized_median_rel_err"] < 0.05


def test_fit_linear_is_exact_without_noise():
    x = np.array([1.0, 2.0, 4.0, 8.0])
    a, b, med, mx = calibrate.fit_linear(x, 3.0 + 0.5 * x)
    assert abs(a - 3.0) < 1e-9 and abs(b - 0.5) < 1e-9 and mx < 1e-9
