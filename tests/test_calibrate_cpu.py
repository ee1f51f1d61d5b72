"""The runtime-model fit (paper_2512_06627_amd/calibrate.py) recovers known constants.

Times are generated from the model's own form with chosen constants (interpreter: launch
cost, one rate per value-file tier (register tier files of 104, 144, 232 rows, LDS above), a
per-gate floor; specialized: launch cost and a
rate over LUT steps x passes; compile: fixed plus per-LUT cost) and perturbed by a seeded 3%
noise; the fit must return the constants within a few percent.  No GPU involved.
"""
import numpy as np

from paper_2512_06627_amd import calibrate


def synthetic(seed=7):
    rng = np.random.default_rng(seed)
    t0, floor = 0.02, 4e-5
    rates = {0: 1.4e14, 1: 1.1e14, 2: 8e13, 3: 3e13}
    s0, s_rate, c0, c1 = 0.013, 6e11, 105.0, 0.0065
    rows = []
    for n in (12, 14, 16, 18, 20, 22, 24, 26, 28):
        for N in (300, 1000, 3000, 5000, 8000, 14000):  # value files of 46..320 rows: every tier
            slots = 40 + N // 50
            luts = N // 3
            P = 2.0 ** n
            ti = t0 + N * max(P / rates[calibrate.tier(slots)] * 1e3, floor)
            ts = s0 + luts * max(1.0, P / 2048.0) / s_rate * 1e3
            tc = c0 + c1 * luts
            noise = lambda: 1.0 + 0.03 * rng.standard_normal()
            rows.append({"name": f"n{n}_{N}", "n": n, "N": N, "rows": slots, "luts": luts,
                         "interp_ms": ti * noise(), "specialized_ms": ts * noise(), "compile_ms": tc * noise()})
    return rows, dict(t0=t0, rates=rates, floor=floor, s0=s0, s_rate=s_rate, c0=c0, c1=c1)


def test_fit_recovers_constants():
    rows, k = synthetic()
    f = calibrate.fit(rows)
    got = f["interp_gate_patterns_per_s_by_tier"]
    assert sorted(got) == sorted(k["rates"])  # every tier has data
    for t, r in k["rates"].items():
        assert abs(got[t] / r - 1) < 0.05, (t, got[t], r)
    assert abs(f["interp_ms_per_gate_floor"] / k["floor"] - 1) < 0.15  # grid of 61 points per decade band
    assert abs(f["specialized_lut_passes_per_s"] / k["s_rate"] - 1) < 0.05
    assert abs(f["compile_c0_ms"] / k["c0"] - 1) < 0.05
    assert abs(f["compile_ms_per_lut"] / k["c1"] - 1) < 0.10
    assert f["interp_median_rel_err"] < 0.05 and f["specialized_median_rel_err"] < 0.05


def test_fit_linear_is_exact_without_noise():
    x = np.array([1.0, 2.0, 4.0, 8.0])
    a, b, med, mx = calibrate.fit_linear(x, 3.0 + 0.5 * x)
    assert abs(a - 3.0) < 1e-9 and abs(b - 0.5) < 1e-9 and mx < 1e-9
