"""Miters and the named synthetic workloads.

A miter XORs paired primary outputs of two circuits over the same primary
inputs and ORs the results; the circuits are equivalent iff the miter output
is 0 for every input assignment (paper, Section 2.1).  Primary input i is bit
i of the pattern index p.
"""
from .aig import Aig, import_into
from .arith import (array_mult, wallace_mult, booth_wallace_mult, mac_fused,
                    mac_separate, full_adder, half_adder)
from .rng import SplitMix64

MULTIPLIERS = {
    "array": array_mult,
    "wallace": wallace_mult,
    "booth": booth_wallace_mult,
}


def circuit(num_inputs: int, build) -> Aig:
    """A standalone circuit: ``build(g)`` returns its output literals."""
    g = Aig(num_inputs)
    for o in build(g):
        g.add_output(o)
    return g


def mult_circuit(kind: str, w: int) -> Aig:
    """w x w unsigned multiplier; inputs a = 0..w-1, b = w..2w-1; 2w outputs."""
    f = MULTIPLIERS[kind]
    return circuit(2 * w, lambda g: f(g, g.inputs(0, w), g.inputs(w, w)))


def mac_circuit(kind: str, w: int) -> Aig:
    """a*b + c*d; inputs a, b, c, d of w bits each in that order; 2w+1 outputs."""
    f = {"fused": mac_fused, "separate": mac_separate}[kind]
    return circuit(4 * w, lambda g: f(g, g.inputs(0, w), g.inputs(w, w),
                                     g.inputs(2 * w, w), g.inputs(3 * w, w)))


def miter_of(a: Aig, b: Aig, or_outputs: bool = True) -> Aig:
    """Miter of two circuits with the same inputs and output count.

    With ``or_outputs`` the result has one output, the OR of the XORs of
    paired outputs; otherwise it keeps one XOR output per pair (a multi-output
    miter, equivalent iff every output is constant 0).
    """
    if a.num_inputs != b.num_inputs or len(a.outputs) != len(b.outputs):
        raise ValueError("miter needs circuits with matching inputs and outputs")
    g = Aig(a.num_inputs)
    oa = import_into(g, a)
    ob = import_into(g, b)
    diffs = [g.XOR(x, y) for x, y in zip(oa, ob)]
    if or_outputs:
        acc = 0
        for d in diffs:
            acc = g.OR(acc, d)
        g.add_output(acc)
    else:
        for d in diffs:
            g.add_output(d)
    return g


def inject_fault(c: Aig, seed: int) -> Aig:
    """Copy of ``c`` with one AND gate's fanin polarity flipped.

    The gate is drawn uniformly among the AND gates in the transitive fan-in
    of the outputs, and a seeded coin picks which of its two fanins flips.
    """
    rng = SplitMix64(seed)
    live = c.tfi_ands()
    if not live:
        raise ValueError("circuit has no AND gate to fault")
    gate = live[rng.below(len(live))]
    side = rng.bit()
    f = Aig(c.num_inputs)
    f.ands = list(c.ands)
    f.outputs = list(c.outputs)
    r0, r1 = f.ands[gate]
    f.ands[gate] = (r0 ^ 1, r1) if side == 0 else (r0, r1 ^ 1)
    f.fault = (gate, side)
    return f


def mult_pair(w: int, impl: str, fault_seed=None):
    """(reference array multiplier, implementation multiplier, possibly faulted)."""
    spec = mult_circuit("array", w)
    impl_c = mult_circuit(impl, w)
    if fault_seed is not None:
        impl_c = inject_fault(impl_c, fault_seed)
    return spec, impl_c


def mult_miter(w: int, impl: str = "booth", fault_seed=None) -> Aig:
    """Miter of a w x w array multiplier against ``impl`` ('wallace' or 'booth')."""
    spec, impl_c = mult_pair(w, impl, fault_seed)
    return miter_of(spec, impl_c)


def mac_miter(w: int, fault_seed=None) -> Aig:
    """Miter of a fused MAC tree against two array multipliers plus a ripple adder."""
    spec = mac_circuit("separate", w)
    impl = mac_circuit("fused", w)
    if fault_seed is not None:
        impl = inject_fault(impl, fault_seed)
    return miter_of(spec, impl)


def minterm_miter(n: int, targets) -> Aig:
    """Single-output circuit that is 1 exactly on the given patterns.

    Output = OR over t of the minterm AND_i (x_i if bit i of t else ~x_i), so
    the lowest counterexample is min(targets) and no other pattern fails.
    """
    g = Aig(n)
    acc = 0
    for t in targets:
        m = 1
        for i in range(n):
            m = g.AND(m, g.input(i) ^ (0 if (t >> i) & 1 else 1))
        acc = g.OR(acc, m)
    g.add_output(acc)
    return g


# ---- layered XOR-dense cones ---------------------------------------------

def _xor(g, enc, x, y):
    return (g.XOR, g.XOR_alt, g.XOR_andor)[enc % 3](x, y)


def _cell_fa(g, enc, x, y, z):
    """Full adder (sum, carry) in one of three structurally different encodings."""
    if enc == 0:
        return full_adder(g, x, y, z)
    if enc == 1:
        s = _xor(g, 1, x, _xor(g, 1, y, z))
        c = g.OR(g.OR(g.AND(x, y), g.AND(x, z)), g.AND(y, z))
        return s, c
    s = _xor(g, 2, _xor(g, 0, x, y), z)
    c = g.OR(g.AND(x, g.OR(y, z)), g.AND(y, z))
    return s, c


def _cell_ha(g, enc, x, y):
    if enc == 0:
        return half_adder(g, x, y)
    return _xor(g, enc, x, y), g.AND(x, y)


def layered_cone_pair(seed: int, n: int, target_ands: int, max_outputs: int = 16):
    """Two functionally identical XOR-dense layered circuits with different structure.

    Layer 0 holds every primary input with a random polarity.  Each new layer
    instantiates full-adder (3:2) and half-adder (2:2) cells on signals of the
    previous one or two layers; every signal of the previous layer feeds at
    least one cell, so all logic stays in the output cone.  Circuit A and
    circuit B share the netlist of cells but each cell uses a different
    encoding in B (alternative XOR forms, two majority forms, a re-associated
    three-input XOR), so the two are equivalent by construction without being
    structurally equal.  Layers are added until A holds about half the target
    AND count; the last layer is then compressed by full adders to at most
    ``max_outputs`` signals, which become the outputs.
    """
    rng = SplitMix64(seed)
    A, B = Aig(n), Aig(n)
    prev1 = []
    for i in range(n):
        pol = rng.bit()
        prev1.append((A.input(i) ^ pol, B.input(i) ^ pol))
    prev2 = []

    def make_cell(ins):
        enc_a = rng.below(3)
        enc_b = (enc_a + 1 + rng.below(2)) % 3
        if len(ins) == 3:
            oa = _cell_fa(A, enc_a, *[s[0] for s in ins])
            ob = _cell_fa(B, enc_b, *[s[1] for s in ins])
        else:
            oa = _cell_ha(A, enc_a, *[s[0] for s in ins])
            ob = _cell_ha(B, enc_b, *[s[1] for s in ins])
        return list(zip(oa, ob))

    def fresh(c, ins):
        return c not in ins and (c[0] ^ 1, c[1] ^ 1) not in ins

    half = max(1, target_ands // 2)
    while A.num_ands() < half:
        queue = list(prev1)
        rng.shuffle(queue)
        pool = prev1 + prev2
        nxt = []
        while queue:
            arity = 3 if rng.below(3) < 2 else 2
            ins = [queue.pop()]
            tries = 0
            while len(ins) < arity and tries < 16:
                tries += 1
                if queue and rng.bit() and fresh(queue[-1], ins):
                    ins.append(queue.pop())
                else:
                    cand = pool[rng.below(len(pool))]
                    if fresh(cand, ins):
                        ins.append(cand)
            if len(ins) < 2:
                nxt.append(ins[0])
                continue
            for o in make_cell(ins):
                pol = rng.bit()
                nxt.append((o[0] ^ pol, o[1] ^ pol))
        prev2, prev1 = prev1, nxt
    sigs = list(prev1)
    rng.shuffle(sigs)
    while len(sigs) > max_outputs:
        trio = sigs[:3]
        if len({t[0] >> 1 for t in trio}) < 3:
            sigs = sigs[1:] + sigs[:1]
            rng.shuffle(sigs)
            continue
        sigs = sigs[3:] + make_cell(trio)
    for sa, sb in sigs:
        A.add_output(sa)
        B.add_output(sb)
    return A, B


def layered_cone_miter(seed: int, n: int, target_ands: int, fault_seed=None) -> Aig:
    """Miter of a layered cone pair; ``fault_seed`` flips one fanin polarity in B."""
    A, B = layered_cone_pair(seed, n, target_ands)
    if fault_seed is not None:
        B = inject_fault(B, fault_seed)
    return miter_of(A, B)


def cone_batch(seed: int, count: int, faulty: int, n_range, size_range):
    """The batched-ES workload: ``count`` layered cone miters with n ~ U{n_range} inputs and
    about U[size_range] AND gates, exactly ``faulty`` of them (a seeded choice) with an
    injected fault.  Returns (miter, fault_seed or None) pairs; cone i uses generator seed
    ``seed * 100000 + i``."""
    rng = SplitMix64(seed)
    bad = set()
    while len(bad) < faulty:
        bad.add(rng.below(count))
    out = []
    for i in range(count):
        n, size = rng.between(*n_range), rng.between(*size_range)
        fault = rng.between(1, 1 << 20) if i in bad else None
        out.append((layered_cone_miter(seed * 100000 + i, n, size, fault_seed=fault), fault))
    return out


def serve_pool(rng: SplitMix64, seed: int, pool: int, n_range=(16, 34), size_range=(500, 20000)):
    """The serving workload's pool: ``pool`` layered cone miters, n ~ U{n_range}, about
    U[size_range] AND gates, each faulty with probability 1/10, drawn from ``rng`` (which the
    caller goes on to use for the arrival stream).  Returns (miter, fault_seed or None) pairs;
    cone i uses generator seed ``seed * 100000 + i``."""
    out = []
    for i in range(pool):
        n, size = rng.between(*n_range), rng.between(*size_range)
        fault = rng.between(1, 1 << 20) if rng.below(10) == 0 else None
        out.append((layered_cone_miter(seed * 100000 + i, n, size, fault_seed=fault), fault))
    return out


# ---- named workloads -------------------------------------------------------

def _mult_workload(w, impl, fault):
    return lambda: mult_miter(w, impl, fault)


WORKLOADS = {
    "mult6_array_wallace": _mult_workload(6, "wallace", None),
    "mult6_array_wallace_f1": _mult_workload(6, "wallace", 1),
    "mult12_array_booth": _mult_workload(12, "booth", None),
    **{f"mult12_array_booth_f{s}": _mult_workload(12, "booth", s) for s in (1, 2, 3, 4)},
    "mult16_array_booth": _mult_workload(16, "booth", None),
    **{f"mult16_array_booth_f{s}": _mult_workload(16, "booth", s) for s in (1, 2, 3, 4)},
    "mac8_fused_separate": lambda: mac_miter(8, None),
    **{f"mac8_fused_separate_f{s}": (lambda s=s: mac_miter(8, s)) for s in (1, 2)},
}


def workload(name: str) -> Aig:
    """Build a named workload miter (deterministic)."""
    return WORKLOADS[name]()
