"""The specialized kernel's single-asm-block body, executed on the host against the oracle.

The block's text is exactly what runs on the GPU once the compiler has substituted its
operands (%0 the miter word, %1/%2 the base index, then lane masks and words).  A
per-lane model of the instructions it may contain (v_bitop3_b32, v_mov_b32,
s_and_b32, s_andn2_b32, s_nor_b32, s_bfe_i32, and the LDS spill pair ds_write_b32 /
ds_read_b32 with s_waitcnt) runs it for whole passes, and every lane's
miter word must equal the oracle's.  A register-allocation mistake (a value overwritten
while still live, a wrong operand, a lost complement) changes some lane's word.
"""
import re

import numpy as np
import pytest

import miters
import oracle
import paper_2512_06627_amd as es

M32 = np.uint64(0xFFFFFFFF)


@pytest.fixture(autouse=True, params=[("0", "6", "0", "0"), ("2", "1", "0", "0"), ("2", "6", "1", "0"),
                                      ("2", "1", "1", "24")],
                ids=["scalar-unit", "all-valu", "all-valu-spaced-banks", "all-valu-lds-spills"])
def block_emitter(monkeypatch, request):
    """Mappings and emitter options: wave-uniform gates on the scalar unit (policy 0) or all
    gates in VALU LUTs (policy 2); latency spacing; bank-aware VGPR choice; a 24-VGPR cap
    that forces values into LDS spill slots."""
    policy, dist, banks, cap = request.param
    monkeypatch.setenv("FASTLEC_ES_JIT_EMIT", "1")
    monkeypatch.setenv("FASTLEC_ES_JIT_SCALAR", policy)
    monkeypatch.setenv("FASTLEC_ES_JIT_DIST", dist)
    monkeypatch.setenv("FASTLEC_ES_JIT_BANKS", banks)
    monkeypatch.setenv("FASTLEC_ES_JIT_VGPR_CAP", cap)


def parse_block(src):
    """Instruction lines (one string literal each), input operands and word values."""
    start = src.index("asm volatile(\n") + len("asm volatile(\n")
    end = src.index('        : "=&v"(m0)')
    lines = []
    for t in src[start:end].splitlines():
        t = t.strip()
        assert t.startswith('"') and t.endswith('\\n\\t"'), t
        lines.append(t[1:-5])
    cons = src[end:].split("\n")[1]
    inputs = re.findall(r'"([sv])"\((\w+)\)', cons)
    words = {m.group(1): int(m.group(2), 16) for m in re.finditer(r"const u32 (w\d+) = 0x([0-9A-F]+)u;", src)}
    return lines, inputs, words


def run_block(lines, inputs, words, base):
    lane = np.arange(64, dtype=np.uint64)
    ops = {}
    for k, (kind, name) in enumerate(inputs):
        if name == "base_lo":
            ops[k + 1] = np.uint64(base & 0xFFFFFFFF)
        elif name == "base_hi":
            ops[k + 1] = np.uint64(base >> 32)
        elif name.startswith("x"):
            i = int(name[1:])
            ops[k + 1] = (np.uint64(0) - ((lane >> np.uint64(i - 5)) & np.uint64(1))) & M32
        elif name == "spill_addr":
            ops[k + 1] = np.uint64(0x4000) + lane * np.uint64(4)  # any wave base; lane-strided
        else:
            ops[k + 1] = np.uint64(words[name])
    v, s, lds = {}, {}, {}

    def val(tok):
        tok = tok.strip()
        if tok.startswith("%"):
            k = int(tok[1:])
            return v["m"] if k == 0 else ops[k]
        if tok[0] == "v":
            return v[int(tok[1:])]
        if tok[0] == "s":
            return s[int(tok[1:])]
        return np.uint64(int(tok, 0) & 0xFFFFFFFF)

    def put(tok, x, scalar):
        tok = tok.strip()
        x = np.asarray(x, dtype=np.uint64) & M32
        if tok == "%0":
            v["m"] = x
        elif scalar:
            assert tok[0] == "s" and x.ndim == 0
            s[int(tok[1:])] = x
        else:
            assert tok[0] == "v"
            v[int(tok[1:])] = np.broadcast_to(x, (64,)).copy()

    for ln in lines:
        op, rest = ln.split(None, 1)
        table = None
        if "bitop3:" in rest:
            rest, t = rest.split(" bitop3:")
            table = int(t, 0)
        a = [x.strip() for x in rest.split(",")]
        if op == "ds_write_b32":  # addr, data offset:N
            addr, rest2 = a[0], a[1].split()
            off = int(rest2[1].split(":")[1]) if len(rest2) > 1 else 0
            base = val(addr)
            data = np.broadcast_to(val(rest2[0]), (64,))
            for l in range(64):
                lds[int(base[l]) + off] = int(data[l])
            continue
        if op == "ds_read_b32":  # dst, addr offset:N
            dst, rest2 = a[0], a[1].split()
            off = int(rest2[1].split(":")[1]) if len(rest2) > 1 else 0
            base = val(rest2[0])
            put(dst, np.array([lds[int(base[l]) + off] for l in range(64)], dtype=np.uint64), False)
            continue
        if op == "s_waitcnt":
            continue
        if op == "v_bitop3_b32":
            assert sum(1 for x in a[1:] if x[0] == "s") <= 1 or len({x for x in a[1:] if x[0] == "s"}) == 1
            x, y, z = (np.broadcast_to(val(t), (64,)) for t in a[1:])
            r = np.zeros(64, dtype=np.uint64)
            for idx in range(8):
                if (table >> idx) & 1:
                    r |= (x if idx & 4 else ~x & M32) & (y if idx & 2 else ~y & M32) & (z if idx & 1 else ~z & M32)
            put(a[0], r, False)
        elif op == "v_mov_b32":
            put(a[0], val(a[1]), False)
        elif op == "s_and_b32":
            put(a[0], val(a[1]) & val(a[2]), True)
        elif op == "s_andn2_b32":
            put(a[0], val(a[1]) & ~val(a[2]), True)
        elif op == "s_nor_b32":
            put(a[0], ~(val(a[1]) | val(a[2])), True)
        elif op == "s_bfe_i32":
            ctl = int(a[2], 0)
            off, width = ctl & 31, (ctl >> 16) & 127
            assert width == 1
            bit = (int(val(a[1])) >> off) & 1
            put(a[0], np.uint64(0xFFFFFFFF if bit else 0), True)
        else:
            raise AssertionError("unexpected instruction " + op)
    return v["m"]


def check(g, bases, waves=2):
    c = es.fastlec_es_load_aig(g.to_aig())
    src = es.fastlec_es_specialized_source(c, waves)
    assert "one asm block" in src, "block emitter not used"
    lines, inputs, words = parse_block(src)
    o = oracle.Circuit(g.to_aag())
    n = g.num_inputs
    H = 1 << max(0, n - 5)
    for base in bases:
        m = run_block(lines, inputs, words, base)
        for l in range(64):
            hw = base + l
            if hw >= H:
                continue
            ps = np.array([32 * hw + j for j in range(32)], dtype=np.uint64)
            if n < 5:
                ps = ps % np.uint64(1 << n)
            want = int(sum(int(b) << j for j, b in enumerate(o.miter(ps))))
            assert int(m[l]) == want, (base, l)


def test_block_body_matches_oracle_on_workloads():
    rng = miters.SplitMix64(41)
    for name in ("mult6_array_wallace_f1", "mult12_array_booth_f2", "mac8_fused_separate_f1", "mult16_array_booth_f3"):
        g = miters.workload(name)
        P = 1 << (g.num_inputs - 11)
        check(g, [0, 64 * (P - 1)] + [64 * rng.below(P) for _ in range(3)])


@pytest.mark.parametrize("seed", range(4))
def test_block_body_matches_oracle_on_layered_cones(seed):
    rng = miters.SplitMix64(100 + seed)
    for i in range(3):
        n = rng.between(11, 18)
        g = miters.layered_cone_miter(900 + 10 * seed + i, n, rng.between(300, 2000),
                                      fault_seed=(i + 1 if i % 2 else None))
        P = 1 << (n - 11)
        check(g, sorted({0, 64 * (P - 1), 64 * rng.below(P)}))


def test_block_body_small_spaces():
    for n, t in ((6, [40]), (9, [300]), (11, [2047]), (13, [8000, 77])):
        check(miters.minterm_miter(n, t), [0] if n <= 11 else [0, 64])


def test_block_registers_stay_within_budget():
    c = es.fastlec_es_load_aig(miters.workload("mult16_array_booth").to_aig())
    src = es.fastlec_es_specialized_source(c, 2)
    m = re.search(r"one asm block: (\d+) VGPRs, (\d+) SGPRs", src)
    assert m and int(m.group(1)) <= 224 and int(m.group(2)) <= 64
