"""Planted mistakes in copies of the oracle must each break at least one pin.

Each mutant is the oracle source with one plausible slip applied as a text
substitution, compiled into a temporary library.  The pins below are the same
facts as in test_oracle_pins.py (closed-form products, hand-worked miters,
minterm circuits); a mutant that passes all of them would mean the pins
cannot see that kind of mistake.
"""
import json
import os
import subprocess

import numpy as np
import pytest

import miters
import oracle
from miters.miter import mult_circuit

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "es_oracle.c")

MUTANTS = {
    "drop_fanin_b_complement": ("uint8_t vb = (uint8_t)(val[b >> 1] ^ (b & 1u));",
                                "uint8_t vb = (uint8_t)(val[b >> 1]);"),
    "drop_fanin_a_complement": ("uint8_t va = (uint8_t)(val[a >> 1] ^ (a & 1u));",
                                "uint8_t va = (uint8_t)(val[a >> 1]);"),
    "reversed_input_bits": ("(uint8_t)((p >> i) & 1u)",
                            "(uint8_t)((p >> (g->num_inputs - 1u - i)) & 1u)"),
    "drop_output_complement": ("return (uint8_t)(val[lit >> 1] ^ (lit & 1u));",
                               "return (uint8_t)(val[lit >> 1]);"),
    "first_output_only": ("for (uint32_t j = 0; j < g->num_outputs; ++j) m |=",
                          "for (uint32_t j = 0; j < 1u && j < g->num_outputs; ++j) m |="),
    "or_instead_of_and": ("val[g->and_var[k]] = (uint8_t)(va & vb);",
                          "val[g->and_var[k]] = (uint8_t)(va | vb);"),
    "chunk_misses_last_pattern": ("jobs[t].hi = start + len;", "jobs[t].hi = start + len - (len > 1);"),
    "scan_skips_first_pattern": ("for (uint64_t p = job->lo; p < job->hi; ++p) {",
                                 "for (uint64_t p = job->lo + 1; p < job->hi; ++p) {"),
    "reports_chunk_start": ("while (p < cur && !atomic_compare_exchange_weak(job->best, &cur, p)) {",
                            "while (job->lo < cur && !atomic_compare_exchange_weak(job->best, &cur, job->lo)) {"),
    "file_order_not_topological": ("if (kind[fan[f]] != 3) continue;", "continue;"),
}


def _pins(lib):
    """Run the pin checks on one oracle build; return the names of the pins that fail."""
    failed = []
    hand = os.path.join(os.path.dirname(__file__), "golden")
    spec = json.load(open(os.path.join(hand, "hand_worked.json")))
    for name, s in spec.items():
        if name.startswith("_") or "error" in s:
            continue
        try:
            got = oracle.Circuit(open(os.path.join(hand, "hand", name), "rb").read(), lib).lowest_failure()[0]
        except oracle.OracleError:
            got = "error"
        if got != s["expect"]:
            failed.append("hand:" + name)
    for kind in ("array", "booth"):
        w = 4
        ps = np.arange(1 << (2 * w), dtype=np.uint64)
        out = oracle.Circuit(mult_circuit(kind, w).to_aag(), lib).outputs(ps)
        if not np.array_equal(out, (ps & np.uint64(15)) * (ps >> np.uint64(4))):
            failed.append("closed_form:" + kind)
    for n, targets in ((6, [63]), (8, [200, 17]), (16, [1 << 15, 12345, 54321])):
        got = oracle.Circuit(miters.minterm_miter(n, targets).to_aag(), lib).lowest_failure(threads=4)[0]
        if got != min(targets):
            failed.append(f"minterm:{n}")
    c = oracle.Circuit(miters.minterm_miter(20, [100, 5000, 70000]).to_aag(), lib)
    for threads in (1, 3):
        if c.lowest_failure(threads=threads)[0] != 100 or c.lowest_failure(101, threads=threads)[0] != 5000:
            failed.append(f"ranges:{threads}")
    return failed


def test_unmutated_oracle_passes_all_pins():
    assert _pins(oracle.lib()) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mutant = tmp_path / "es_oracle.c"
    mutant.write_text(src.replace(old, new))
    (tmp_path / "es_oracle.h").write_text(open(SRC[:-1] + "h").read())
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread", str(mutant), "-o", str(so)],
                   check=True)
    lib = oracle.load_library(str(so))
    assert _pins(lib), f"mutant {name} passed every pin"
